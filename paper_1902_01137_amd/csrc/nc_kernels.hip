// nc_kernels.hip -- HIP kernels for gfx950: grid build, ordered crossing,
// null-collision transmissivity and the persistent backward path tracer.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "nc_internal.hpp"

namespace nc {

// ===========================================================================
// Grid build (Section 3.1.1; criterion of Section 4.2; Appendix C indexing)
// ===========================================================================

__device__ inline bool merge_criterion(float kmin, float kmax, double k_gas, double dz_node, double tau, int crit)
{
    // evaluated in FP64; the library is built without FMA contraction, so
    // this rounds as (kmax + k_gas) * dz_node (or (kmax - kmin) * dz_node)
    const double s = crit == 0 ? (double)kmax + k_gas : (double)kmax - (double)kmin;
    return s * dz_node < tau;
}

__device__ inline float2 encode_node(float kmin, float kmax, bool merged)
{
    const uint32_t b = (__float_as_uint(kmin) & 0x7fffffffu) | (merged ? 0x80000000u : 0u);
    return make_float2(__uint_as_float(b), kmax);
}

// Level 1 straight from the field: each node reduces its (up to) 2x2x2
// cells and validates them (finite, >= 0).
__global__ void build_level1_kernel(const float *__restrict__ kc, int nx, int ny, int nz, float2 *__restrict__ out,
                                    int d0, int d1, int d2, double k_gas, double dz_node, double tau, int crit,
                                    unsigned int *bad)
{
    const long long total = (long long)d0 * d1 * d2;
    bool flag = false;
    for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < total;
         id += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(id % d0);
        const int j = (int)((id / d0) % d1);
        const int m = (int)(id / ((long long)d0 * d1));
        float lo = INFINITY, hi = -INFINITY;
        for (int dm = 0; dm < 2; ++dm) {
            const int z = 2 * m + dm;
            if (z >= nz) break;
            for (int dj = 0; dj < 2; ++dj) {
                const int y = 2 * j + dj;
                if (y >= ny) break;
                const float *row = kc + ((size_t)z * ny + y) * nx;
                for (int di = 0; di < 2; ++di) {
                    const int x = 2 * i + di;
                    if (x >= nx) break;
                    const float v = row[x];
                    if (!(v >= 0.0f) || isinf(v)) flag = true;
                    lo = fminf(lo, v);
                    hi = fmaxf(hi, v);
                }
            }
        }
        out[id] = encode_node(lo, hi, merge_criterion(lo, hi, k_gas, dz_node, tau, crit));
    }
    if (flag) atomicOr(bad, 1u);
}

// Level l >= 2 from level l-1: min and max of the (up to) 8 children.
__global__ void build_level_kernel(const float2 *__restrict__ child, int c0, int c1, int c2, float2 *__restrict__ out,
                                   int d0, int d1, int d2, double k_gas, double dz_node, double tau, int crit)
{
    const long long total = (long long)d0 * d1 * d2;
    for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < total;
         id += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(id % d0);
        const int j = (int)((id / d0) % d1);
        const int m = (int)(id / ((long long)d0 * d1));
        float lo = INFINITY, hi = -INFINITY;
        for (int dm = 0; dm < 2; ++dm) {
            const int z = 2 * m + dm;
            if (z >= c2) break;
            for (int dj = 0; dj < 2; ++dj) {
                const int y = 2 * j + dj;
                if (y >= c1) break;
                for (int di = 0; di < 2; ++di) {
                    const int x = 2 * i + di;
                    if (x >= c0) break;
                    const float2 v = child[((size_t)z * c1 + y) * c0 + x];
                    lo = fminf(lo, node_kmin(v));
                    hi = fmaxf(hi, v.y);
                }
            }
        }
        out[id] = encode_node(lo, hi, merge_criterion(lo, hi, k_gas, dz_node, tau, crit));
    }
}

__global__ void export_level_kernel(const float2 *__restrict__ nodes, long long total, float *kmin, float *kmax,
                                    uint8_t *mg)
{
    for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < total;
         id += (long long)gridDim.x * blockDim.x) {
        const float2 v = nodes[id];
        if (kmin) kmin[id] = node_kmin(v);
        if (kmax) kmax[id] = v.y;
        if (mg) mg[id] = node_merged(v) ? 1 : 0;
    }
}

__global__ void leaf_level_kernel(GridView g, uint8_t *out)
{
    const long long total = (long long)g.n[0] * g.n[1] * g.n[2];
    for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < total;
         id += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(id % g.n[0]);
        const int y = (int)((id / g.n[0]) % g.n[1]);
        const int z = (int)(id / ((long long)g.n[0] * g.n[1]));
        int lev = 0;
        for (int l = g.L; l >= 1; --l) {
            const int d0 = level_dim(g.n[0], l), d1 = level_dim(g.n[1], l);
            const float2 v = g.nodes[g.off[l] + ((z >> l) * d1 + (y >> l)) * d0 + (x >> l)];
            if (node_merged(v)) { lev = l; break; }
        }
        out[id] = (uint8_t)lev;
    }
}

static int blocks_for(long long n, int block, int cap = 65536)
{
    long long b = (n + block - 1) / block;
    return (int)std::max<long long>(1, std::min<long long>(b, cap));
}

hipError_t launch_build(const nc_ctx *ctx, nc_grid *g, const float *d_kc, unsigned int *d_bad)
{
    const int block = 256;
    for (int l = 1; l <= g->L; ++l) {
        const int d0 = level_dim(g->n[0], l), d1 = level_dim(g->n[1], l), d2 = level_dim(g->n[2], l);
        const long long total = (long long)d0 * d1 * d2;
        const double dz_node = g->h[2] * (double)(1 << l);
        float2 *out = g->d_nodes + g->off[l];
        if (l == 1) {
            hipLaunchKernelGGL(build_level1_kernel, dim3(blocks_for(total, block)), dim3(block), 0, ctx->stream, d_kc,
                               g->n[0], g->n[1], g->n[2], out, d0, d1, d2, g->params.k_gas, dz_node,
                               g->params.tau_tilde, g->params.criterion, d_bad);
        } else {
            const int c0 = level_dim(g->n[0], l - 1), c1 = level_dim(g->n[1], l - 1), c2 = level_dim(g->n[2], l - 1);
            hipLaunchKernelGGL(build_level_kernel, dim3(blocks_for(total, block)), dim3(block), 0, ctx->stream,
                               (const float2 *)(g->d_nodes + g->off[l - 1]), c0, c1, c2, out, d0, d1, d2,
                               g->params.k_gas, dz_node, g->params.tau_tilde, g->params.criterion);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_export(const nc_ctx *ctx, const nc_grid *g, int l, float *kmin, float *kmax, uint8_t *mg)
{
    const long long total = (long long)level_dim(g->n[0], l) * level_dim(g->n[1], l) * level_dim(g->n[2], l);
    hipLaunchKernelGGL(export_level_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, ctx->stream,
                       (const float2 *)(g->d_nodes + g->off[l]), total, kmin, kmax, mg);
    return hipGetLastError();
}

hipError_t launch_leaf_levels(const nc_ctx *ctx, const nc_grid *g, uint8_t *out)
{
    GridView gv = grid_view(g, nullptr);
    const long long total = (long long)g->n[0] * g->n[1] * g->n[2];
    hipLaunchKernelGGL(leaf_level_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, ctx->stream, gv, out);
    return hipGetLastError();
}

// ===========================================================================
// Ordered crossing (Section 3.1.3): the voxel sequence of each ray.
// ===========================================================================
__global__ void trace_leaves_kernel(GridView g, const float *__restrict__ rays, int n, int maxv, int *leaf, float *tt,
                                    int *count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    NodeSrc ns{g.nodes, nullptr, g.off, g.L + 1, 0, g.n[0], g.n[1]};
    uint32_t reads = 0;
    Ray r;
    float o[3] = {rays[6 * i], rays[6 * i + 1], rays[6 * i + 2]};
    float d[3] = {rays[6 * i + 3], rays[6 * i + 4], rays[6 * i + 5]};
    int k = 0;
    if (ray_setup(g, r, o, d, 0.0f)) {
        find_leaf(g, ns, r, g.L, 1.0f, reads);
        for (;;) {
            if (r.texit > r.t) {
                if (k < maxv) {
                    const size_t b = (size_t)i * maxv + k;
                    const int l = r.lev;
                    leaf[4 * b + 0] = l;
                    leaf[4 * b + 1] = r.c[0] >> l;
                    leaf[4 * b + 2] = r.c[1] >> l;
                    leaf[4 * b + 3] = r.c[2] >> l;
                    tt[2 * b + 0] = r.t;
                    tt[2 * b + 1] = r.texit;
                }
                ++k;
            }
            if (!next_leaf(g, ns, r, 1.0f, reads)) break;
        }
    }
    count[i] = k;
}

hipError_t launch_trace_leaves(const nc_ctx *ctx, const nc_grid *g, const float *rays, int n, int maxv, int *leaf,
                               float *t, int *count)
{
    GridView gv = grid_view(g, nullptr);
    hipLaunchKernelGGL(trace_leaves_kernel, dim3((n + 127) / 128), dim3(128), 0, ctx->stream, gv, rays, n, maxv, leaf,
                       t, count);
    return hipGetLastError();
}

// ===========================================================================
// Direct transmissivity (Section 2.3): Bernoulli paths, t = 1 if the ray
// leaves the box before a real collision.
// ===========================================================================
struct TransArgs {
    GridView g;
    const float *rays;
    int n;
    int spp;
    int spi;
    long long items;
    uint64_t seed, sample_offset;
    float mscale;
    double *sum, *sumsq;
    nc_counters *counters;
    int lds_first, lds_nodes;
};

__global__ __launch_bounds__(256) void transmittance_kernel(TransArgs A)
{
    extern __shared__ float2 s_nodes[];
    __shared__ int s_off[NC_MAX_LEVELS + 2];
    stage_levels(A.g, A.lds_first, A.lds_nodes, s_nodes, s_off);
    const NodeSrc ns{A.g.nodes, s_nodes, s_off, A.lds_first, s_off[A.lds_first <= A.g.L ? A.lds_first : 0],
                     A.g.n[0], A.g.n[1]};
    Counters cnt = {};
    for (long long w = blockIdx.x * (long long)blockDim.x + threadIdx.x; w < A.items;
         w += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(w % A.n);
        const int blk = (int)(w / A.n);
        const int s0 = blk * A.spi, s1 = min(s0 + A.spi, A.spp);
        const float o[3] = {A.rays[6 * i], A.rays[6 * i + 1], A.rays[6 * i + 2]};
        const float d[3] = {A.rays[6 * i + 3], A.rays[6 * i + 4], A.rays[6 * i + 5]};
        double acc = 0.0;
        int hint = A.g.L;
        for (int s = s0; s < s1; ++s) {
            Rng rng;
            rng.init((uint32_t)i, (uint32_t)(A.sample_offset + s), 1u, A.seed);
            Ray r;
            start_ray(A.g, ns, r, o, d, hint, A.mscale, cnt);
            float tau = rng.exp1();
            float kc_hit = 0.0f;
            int res;
            do {
                res = track_step(A.g, ns, r, tau, rng, A.mscale, true, kc_hit, cnt);
            } while (res == kContinue);
            if (res == kExit) acc += 1.0;
            ++cnt.paths;
            ++cnt.nee_rays;
        }
        unsafeAtomicAdd(A.sum + i, acc);
        unsafeAtomicAdd(A.sumsq + i, acc);   // t is 0 or 1
    }
    flush_counters(cnt, A.counters);
}

hipError_t launch_transmittance(const nc_ctx *ctx, const nc_grid *g, const float *d_kc, const OptView &op,
                                const float *rays, int n, const nc_sampling &s, double *sum, double *sumsq,
                                nc_counters *counters)
{
    Shape sh = choose_shape(ctx, g, 256);
    TransArgs A;
    A.g = grid_view(g, d_kc);
    A.rays = rays;
    A.n = n;
    A.spp = s.spp;
    A.spi = std::max(1, std::min(s.spp, 64));
    A.items = (long long)n * ((s.spp + A.spi - 1) / A.spi);
    A.seed = s.seed;
    A.sample_offset = s.sample_offset;
    A.mscale = op.mscale;
    A.sum = sum;
    A.sumsq = sumsq;
    A.counters = counters;
    A.lds_first = sh.lds_first;
    A.lds_nodes = sh.lds_nodes;
    const int wgs = (int)std::max<long long>(1, std::min<long long>((A.items + 255) / 256, (long long)sh.wgs));
    hipLaunchKernelGGL(transmittance_kernel, dim3(wgs), dim3(256), (size_t)sh.lds_nodes * sizeof(float2), ctx->stream,
                       A);
    return hipGetLastError();
}

// ===========================================================================
// Backward radiance with the local estimate of the sun (Section 4.1, Fig. 4a)
//
// Persistent kernel: each lane owns one (pixel, block of samples) item from a
// global queue and runs its paths one after the other.  A path is a small
// state machine over one traversal step: the path ray (PATH) or the sun ray
// of the current event (SHADOW) advance by one voxel or one tentative
// collision per loop trip, so all lanes of a wave execute the same traversal
// code whatever their state.  Idle lanes are refilled from the queue with a
// wave ballot and a prefix count (one atomic per wave refill).
// ===========================================================================
struct RenderArgs {
    GridView g;
    CamView cam;
    OptView op;
    uint64_t seed, sample_offset;
    int spp, spi;
    int tiles_x, tiles_y;
    unsigned long long items;
    double *sum, *sumsq;
    nc_counters *counters;
    unsigned long long *queue;
    int lds_first, lds_nodes;
};

enum LaneState { kIdle = 0, kPath = 1, kShadow = 2 };

__device__ inline void camera_ray(const CamView &c, int px, int py, float u1, float u2, float o[3], float d[3])
{
    if (c.type == 0) {
        const float sx = (2.0f * ((float)px + u1) / (float)c.W - 1.0f) * c.sx;
        const float sy = (1.0f - 2.0f * ((float)py + u2) / (float)c.H) * c.sy;
        float v[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o[a] = c.pos[a];
            v[a] = c.f[a] + sx * c.r[a] + sy * c.u[a];
        }
        const float inv = rsqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) d[a] = v[a] * inv;
    } else {
        const float sx = (((float)px + u1) / (float)c.W - 0.5f) * c.sx;
        const float sy = (0.5f - ((float)py + u2) / (float)c.H) * c.sy;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o[a] = c.pos[a] + sx * c.r[a] + sy * c.u[a];
            d[a] = c.f[a];
        }
    }
}

__device__ inline unsigned int lanes_below(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__global__ __launch_bounds__(256) void render_kernel(RenderArgs A)
{
    extern __shared__ float2 s_nodes[];
    __shared__ int s_off[NC_MAX_LEVELS + 2];
    stage_levels(A.g, A.lds_first, A.lds_nodes, s_nodes, s_off);
    const GridView &g = A.g;
    const NodeSrc ns{g.nodes, s_nodes, s_off, A.lds_first, s_off[A.lds_first <= g.L ? A.lds_first : 0], g.n[0],
                     g.n[1]};
    const int lane = __lane_id();
    const int tile_px = A.tiles_x * A.tiles_y * 64;
    const float sun[3] = {A.op.sun[0], A.op.sun[1], A.op.sun[2]};

    Counters cnt = {};
    int state = kIdle;
    bool exhausted = false;
    int pix = 0, s = 0, s_end = 0;
    double acc = 0.0, acc2 = 0.0;
    float Lp = 0.0f;
    Ray r;
    float tau = 0.0f;
    Rng rng;
    float ex[3] = {0, 0, 0};   // position of the current event
    float pd[3] = {0, 0, 0};   // path direction at the current event
    float w_nee = 0.0f;        // sun contribution of the current event if its sun ray gets through
    float p_cont = 0.0f;       // probability that the path goes on after the event
    bool ground_ev = false;
    int order = 0, segs = 0, hint = g.L;

    for (;;) {
        bool do_start = false;
        // ---- refill idle lanes (ballot + prefix count, one atomic per wave)
        const bool want = state == kIdle && !exhausted;
        const unsigned long long need = __ballot(want);
        if (need) {
            const int leader = __ffsll((unsigned long long)need) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(A.queue, (unsigned long long)__popcll(need));
            base = __shfl(base, leader);
            if (want) {
                const unsigned long long w = base + lanes_below(need);
                if (w >= A.items) {
                    exhausted = true;
                } else {
                    const int blk = (int)(w / (unsigned long long)tile_px);
                    const int rem = (int)(w % (unsigned long long)tile_px);
                    const int tile = rem >> 6, within = rem & 63;
                    const int px = (tile % A.tiles_x) * 8 + (within & 7);
                    const int py = (tile / A.tiles_x) * 8 + (within >> 3);
                    s = blk * A.spi;
                    s_end = min(s + A.spi, A.spp);
                    if (px < A.cam.W && py < A.cam.H && s < s_end) {
                        pix = py * A.cam.W + px;
                        acc = 0.0;
                        acc2 = 0.0;
                        do_start = true;
                        state = kPath;
                    }
                }
            }
        }
        if (__all(state == kIdle && exhausted)) break;

        bool do_cont = false, do_finish = false;
        if (state != kIdle && !do_start) {
            float kc_hit = 0.0f;
            const bool shadow = state == kShadow;
            const int res = track_step(g, ns, r, tau, rng, A.op.mscale, shadow, kc_hit, cnt);
            if (++segs >= A.op.max_segments && res == kContinue) {
                ++cnt.truncated;
                do_finish = true;
            } else if (res == kReal) {
                if (shadow) {
                    do_cont = true;                       // sun ray blocked
                } else {
                    // volume event: local estimate, then scatter or absorb
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        ex[a] = r.o[a] + r.t * r.d[a];
                        pd[a] = r.d[a];
                    }
                    const float kd = g.kscale * kc_hit;
                    const float ssa = A.op.ssa * kd / (kd + g.k_gas);
                    const float mu = pd[0] * sun[0] + pd[1] * sun[1] + pd[2] * sun[2];
                    w_nee = ssa * hg_phase(A.op.g, mu) * A.op.S;
                    p_cont = ssa;
                    ground_ev = false;
                    ++order;
                    hint = r.lev;
                    if (A.op.max_scatter >= 0 && order > A.op.max_scatter) {
                        do_finish = true;
                    } else if (w_nee > 0.0f) {
                        ++cnt.nee_rays;
                        start_ray(g, ns, r, ex, sun, hint, A.op.mscale, cnt);
                        tau = rng.exp1();
                        state = kShadow;
                    } else {
                        do_cont = true;
                    }
                }
            } else if (res == kExit) {
                if (shadow) {
                    Lp += w_nee;                          // sun ray got through
                    do_cont = true;
                } else if (r.d[2] < 0.0f) {
                    // ground hit: Lambertian local estimate
                    const float tg = -r.o[2] / r.d[2];
#pragma unroll
                    for (int a = 0; a < 3; ++a) pd[a] = r.d[a];
                    ex[0] = r.o[0] + tg * r.d[0];
                    ex[1] = r.o[1] + tg * r.d[1];
                    ex[2] = 0.0f;
                    w_nee = A.op.ground_w;
                    p_cont = A.op.rho;
                    ground_ev = true;
                    ++order;
                    if (A.op.max_scatter >= 0 && order > A.op.max_scatter) {
                        do_finish = true;
                    } else if (w_nee > 0.0f) {
                        ++cnt.nee_rays;
                        start_ray(g, ns, r, ex, sun, hint, A.op.mscale, cnt);
                        tau = rng.exp1();
                        state = kShadow;
                    } else {
                        do_cont = true;
                    }
                } else {
                    do_finish = true;                     // escaped upward
                }
            }
        }
        if (do_cont) {
            state = kPath;
            if (A.op.max_scatter >= 0 && order >= A.op.max_scatter) {
                do_finish = true;
            } else if (rng.u01() >= p_cont) {
                do_finish = true;                         // absorbed (volume) or not reflected (ground)
            } else {
                const float u1 = rng.u01(), u2 = rng.u01();
                float nd[3] = {pd[0], pd[1], pd[2]};
                if (ground_ev)
                    lambert(nd, u1, u2);
                else
                    turn(nd, hg_sample_mu(A.op.g, u1), u2);
                start_ray(g, ns, r, ex, nd, hint, A.op.mscale, cnt);
                tau = rng.exp1();
            }
        }
        if (do_finish) {
            ++cnt.paths;
            acc += (double)Lp;
            acc2 += (double)Lp * (double)Lp;
            if (++s < s_end) {
                do_start = true;
            } else {
                unsafeAtomicAdd(A.sum + pix, acc);
                unsafeAtomicAdd(A.sumsq + pix, acc2);
                state = kIdle;
            }
        }
        if (do_start) {
            rng.init((uint32_t)pix, (uint32_t)(A.sample_offset + (uint64_t)s), 0u, A.seed);
            const int px = pix % A.cam.W, py = pix / A.cam.W;
            const float u1 = rng.u01(), u2 = rng.u01();
            float o[3], d[3];
            camera_ray(A.cam, px, py, u1, u2, o, d);
            Lp = 0.0f;
            order = 0;
            segs = 0;
            hint = g.L;
            state = kPath;
            start_ray(g, ns, r, o, d, hint, A.op.mscale, cnt);
            tau = rng.exp1();
        }
    }
    flush_counters(cnt, A.counters);
}

__global__ void zero_u64_kernel(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

hipError_t launch_render(const nc_ctx *ctx, const nc_grid *g, const float *d_kc, const OptView &op, const CamView &cam,
                         const nc_sampling &s, double *sum, double *sumsq, nc_counters *counters)
{
    Shape sh = choose_shape(ctx, g, 256);
    RenderArgs A;
    A.g = grid_view(g, d_kc);
    A.cam = cam;
    A.op = op;
    A.seed = s.seed;
    A.sample_offset = s.sample_offset;
    A.spp = s.spp;
    A.spi = std::max(1, std::min(sh.spi, s.spp));
    A.tiles_x = (cam.W + 7) / 8;
    A.tiles_y = (cam.H + 7) / 8;
    const unsigned long long blocks = (unsigned long long)((s.spp + A.spi - 1) / A.spi);
    A.items = (unsigned long long)A.tiles_x * A.tiles_y * 64ull * blocks;
    A.sum = sum;
    A.sumsq = sumsq;
    A.counters = counters;
    A.queue = ctx->d_scratch;
    A.lds_first = sh.lds_first;
    A.lds_nodes = sh.lds_nodes;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, ctx->stream, ctx->d_scratch, 1);
    // persistent grid: as many workgroups as can be resident at once
    int resident = 0;
    if (ctx->launch.waves_per_cu <= 0 &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, render_kernel, sh.block,
                                                     (size_t)sh.lds_nodes * sizeof(float2)) == hipSuccess &&
        resident > 0)
        sh.wgs = ctx->num_cus * resident;
    const long long max_wgs = (long long)((A.items + sh.block - 1) / sh.block);
    const int wgs = (int)std::max<long long>(1, std::min<long long>(max_wgs, sh.wgs));
    hipLaunchKernelGGL(render_kernel, dim3(wgs), dim3(sh.block), (size_t)sh.lds_nodes * sizeof(float2), ctx->stream,
                       A);
    return hipGetLastError();
}

__global__ void philox_kernel(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const U4 r = philox4x32_10(U4{ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]}, key[2 * i], key[2 * i + 1]);
    out[4 * i] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
}

hipError_t launch_philox(const nc_ctx *ctx, const uint32_t *ctr, const uint32_t *key, uint32_t *out, int n)
{
    hipLaunchKernelGGL(philox_kernel, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, ctr, key, out, n);
    return hipGetLastError();
}

// ===========================================================================
// Host helpers
// ===========================================================================
GridView grid_view(const nc_grid *g, const float *d_kc)
{
    GridView v;
    for (int a = 0; a < 3; ++a) {
        v.n[a] = g->n[a];
        v.lo[a] = (float)g->lo[a];
        v.h[a] = (float)g->h[a];
        v.inv_h[a] = (float)(1.0 / g->h[a]);
    }
    v.L = g->L;
    v.k_gas = (float)g->params.k_gas;
    v.kscale = 1.0f;
    v.kc = d_kc;
    v.nodes = g->d_nodes;
    v.off = g->d_off;
    return v;
}

Shape choose_shape(const nc_ctx *ctx, const nc_grid *g, int block_default)
{
    Shape sh;
    sh.block = ctx->launch.block > 0 ? ctx->launch.block : block_default;
    sh.block = std::max(64, std::min(256, (sh.block / 64) * 64));
    const int waves = ctx->launch.waves_per_cu > 0 ? ctx->launch.waves_per_cu : 16;
    sh.wgs = std::max(1, ctx->num_cus * waves / (sh.block / 64));
    sh.spi = ctx->launch.samples_per_item > 0 ? ctx->launch.samples_per_item : 4;
    // LDS staging of the top levels: as many whole levels as fit the budget
    const size_t wgs_per_cu = std::max(1, waves / (sh.block / 64));
    size_t budget = std::min<size_t>(ctx->lds_per_cu / wgs_per_cu, 60 * 1024) - 1024;
    int first = g->L + 1;
    if (ctx->launch.lds_levels == 0 || g->L == 0) {
        first = g->L + 1;
    } else {
        const int want = ctx->launch.lds_levels > 0 ? ctx->launch.lds_levels : NC_MAX_LEVELS;
        for (int l = g->L; l >= 1 && g->L - l + 1 <= want; --l) {
            const size_t nodes = (size_t)(g->off[g->L + 1] - g->off[l]);
            if (nodes * sizeof(float2) > budget) break;
            first = l;
        }
    }
    sh.lds_first = first;
    sh.lds_nodes = first <= g->L ? g->off[g->L + 1] - g->off[first] : 0;
    return sh;
}

}  // namespace nc
