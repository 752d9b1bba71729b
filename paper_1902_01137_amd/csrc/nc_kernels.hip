// nc_kernels.hip -- HIP kernels for gfx950: grid build, ordered crossing,
// null-collision transmissivity and the persistent backward path tracer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "nc_internal.hpp"

namespace nc {

// ===========================================================================
// Grid build (Section 3.1.1; criterion of Section 4.2; Appendix B.3 indexing)
// ===========================================================================

__device__ inline bool merge_criterion(float kmin, float kmax, double k_gas, double dz_node, double tau, int crit)
{
    // evaluated in FP64; the library is built without FMA contraction, so
    // this rounds as (kmax + k_gas) * dz_node (or (kmax - kmin) * dz_node)
    const double s = crit == 0 ? (double)kmax + k_gas : (double)kmax - (double)kmin;
    return s * dz_node < tau;
}

// The layered grid (criterion 3): a node covering z cells za..zb is one voxel
// when it lies wholly below or above the cloudy layer zc[0]..zc[1] (the z
// range of the cells with k_c > 0), or when its level is <= flat_level.
struct LayerRule {
    const int *zc;     // device: cloudy layer's lowest and highest z index (null: not criterion 3)
    int flat_level;
};

__device__ inline bool node_merged_rule(float kmin, float kmax, double k_gas, double dz_node, double tau, int crit,
                                        const LayerRule &lr, int level, int za, int zb)
{
    if (lr.zc) return zb < lr.zc[0] || za > lr.zc[1] || level <= lr.flat_level;
    return merge_criterion(kmin, kmax, k_gas, dz_node, tau, crit);
}

// z extent of the cells with k_c > 0 (zc starts at {nz, -1})
__global__ void cloud_layer_kernel(const float *__restrict__ kc, long long n, int nxy, int *__restrict__ zc)
{
    int lo = 0x7fffffff, hi = -1;
    for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < n;
         id += (long long)gridDim.x * blockDim.x) {
        if (kc[id] > 0.0f) {
            const int z = (int)(id / nxy);
            lo = min(lo, z);
            hi = max(hi, z);
        }
    }
    if (hi >= 0) {
        atomicMin(zc, lo);
        atomicMax(zc + 1, hi);
    }
}

__global__ void set_cloud_layer_kernel(int *zc, int nz)
{
    if (threadIdx.x == 0) {
        zc[0] = nz;
        zc[1] = -1;
    }
}

__device__ inline float2 encode_node(float kmin, float kmax, bool merged)
{
    const uint32_t b = (__float_as_uint(kmin) & 0x7fffffffu) | (merged ? 0x80000000u : 0u);
    return make_float2(__uint_as_float(b), kmax);
}

// Level l >= 2 from level l-1: min and max of the (up to) 8 children.
__global__ void build_level_kernel(const float2 *__restrict__ child, int c0, int c1, int c2, float2 *__restrict__ out,
                                   int d0, int d1, int d2, double k_gas, double dz_node, double tau, int crit,
                                   LayerRule lr, int level, int nz)
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
        out[id] = encode_node(lo, hi, node_merged_rule(lo, hi, k_gas, dz_node, tau, crit, lr, level, m << level,
                                                       min((m + 1) << level, nz) - 1));
    }
}

// Waves (level-4 nodes along x) per workgroup of the fused pass.
constexpr int kBuildWaves = 16;

// Merge settings of the levels the fused pass builds (index 1..4).
struct LevelRules {
    double dz_node[5];
    double tau[5];
    int crit[5];
};

__device__ inline float2 level_node(float lo, float hi, double k_gas, const LevelRules &R, const LayerRule &lr, int l,
                                    int m, int nz, bool &merged)
{
    merged = node_merged_rule(lo, hi, k_gas, R.dz_node[l], R.tau[l], R.crit[l], lr, l, m << l,
                              min((m + 1) << l, nz) - 1);
    return encode_node(lo, hi, merged);
}

// Levels 1..4 and their bits of the ancestry mask in one pass over the field
// (the field is read once; each level is written once).  A wave owns one
// level-4 node (16^3 cells), a lane one level-2 node (4^3 cells, read as 16
// rows of 4 cells).  The lane reduces its 8 level-1 nodes and its level-2
// node in registers, level 3 over 8 lanes and level 4 over the wave by lane
// exchange.  Lane bits 0..2: the level-2 node's octant in its level-3 parent
// (x, y, z); bits 3..5: that parent's octant in its level-4 parent.  The
// waves of a workgroup are consecutive level-4 nodes along x, so a workgroup
// reads 16 kBuildWaves consecutive cells of each row it touches.  Cells
// outside the field take no part in any reduction; nodes outside their level
// are not written.  Levels above L are neither written nor set in the mask.  kVec: nx is a multiple of
// 4, so a row's 4 cells are one 16-byte load and a level-1 node pair (and its
// mask pair) one store.  Launch: (ceil(d4x / kBuildWaves), d4y, d4z) x
// 64 kBuildWaves threads.
template <bool kVec>
__global__ __launch_bounds__(64 * kBuildWaves) void build_fused_kernel(const float *__restrict__ kc, int nx, int ny, int nz,
                                                          float2 *__restrict__ nodes, int off1, int off2, int off3,
                                                          int off4, uint16_t *__restrict__ mask, int L, double k_gas,
                                                          LevelRules R, LayerRule lr, unsigned int *bad)
{
    const int lane = (int)(threadIdx.x & 63u);
    const int X4 = (int)blockIdx.x * kBuildWaves + (int)(threadIdx.x >> 6);
    if (X4 >= level_dim(nx, 4)) return;   // wave-uniform, and the kernel has no block barrier
    const int a2 = 4 * X4 + (lane & 1) + ((lane >> 2) & 2);
    const int b2 = 4 * (int)blockIdx.y + ((lane >> 1) & 1) + ((lane >> 3) & 2);
    const int c2 = 4 * (int)blockIdx.z + ((lane >> 2) & 1) + ((lane >> 4) & 2);
    const int x0 = 4 * a2, y0 = 4 * b2, z0 = 4 * c2;
    float lo1[8], hi1[8];   // level-1 nodes of the lane, index 4 ez + 2 ey + ex
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        lo1[k] = INFINITY;
        hi1[k] = -INFINITY;
    }
    // all 16 rows are loaded first, unconditionally, from clamped in-bounds
    // addresses (so they are in flight together); cells outside the field
    // then take the reductions' identities
    float v[16][4];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int y = min(y0 + (r & 3), ny - 1), z = min(z0 + (r >> 2), nz - 1);
        const float *row = kc + ((size_t)z * ny + y) * nx;
        if (kVec) {
            const float4 f = *reinterpret_cast<const float4 *>(row + min(x0, nx - 4));
            v[r][0] = f.x;
            v[r][1] = f.y;
            v[r][2] = f.z;
            v[r][3] = f.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[r][e] = row[min(x0 + e, nx - 1)];
        }
    }
    bool flag = false;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int dy = r & 3, dz = r >> 2;
        const bool row_in = (y0 + dy < ny) & (z0 + dz < nz);
        const int k0 = (dz >> 1) * 4 + (dy >> 1) * 2;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool in = row_in & (kVec ? x0 < nx : x0 + e < nx);
            const float c = v[r][e];
            flag |= in & !((c >= 0.0f) & (c < INFINITY));
            lo1[k0 + (e >> 1)] = fminf(lo1[k0 + (e >> 1)], in ? c : INFINITY);
            hi1[k0 + (e >> 1)] = fmaxf(hi1[k0 + (e >> 1)], in ? c : -INFINITY);
        }
    }
    // level 2 (the lane's node), 3 (8 lanes) and 4 (the wave)
    float lo = lo1[0], hi = hi1[0];
#pragma unroll
    for (int k = 1; k < 8; ++k) {
        lo = fminf(lo, lo1[k]);
        hi = fmaxf(hi, hi1[k]);
    }
    const float lo2 = lo, hi2 = hi;
#pragma unroll
    for (int s = 1; s < 8; s <<= 1) {
        lo = fminf(lo, __shfl_xor(lo, s));
        hi = fmaxf(hi, __shfl_xor(hi, s));
    }
    const float lo3 = lo, hi3 = hi;
#pragma unroll
    for (int s = 8; s < 64; s <<= 1) {
        lo = fminf(lo, __shfl_xor(lo, s));
        hi = fmaxf(hi, __shfl_xor(hi, s));
    }
    const float lo4 = lo, hi4 = hi;
    const unsigned long long any_bad = __ballot(flag);
    if (lane == 0 && any_bad) atomicOr(bad, 1u);

    bool mg2 = false, mg3 = false, mg4 = false;
    const float2 n2 = level_node(lo2, hi2, k_gas, R, lr, 2, c2, nz, mg2);
    const float2 n3 = level_node(lo3, hi3, k_gas, R, lr, 3, c2 >> 1, nz, mg3);
    const float2 n4 = level_node(lo4, hi4, k_gas, R, lr, 4, c2 >> 2, nz, mg4);
    const uint32_t up = (L >= 2 && mg2 ? 4u : 0u) | (L >= 3 && mg3 ? 8u : 0u) | (L >= 4 && mg4 ? 16u : 0u);

    const int d1x = level_dim(nx, 1), d1y = level_dim(ny, 1), d1z = level_dim(nz, 1);
#pragma unroll
    for (int ez = 0; ez < 2; ++ez) {
#pragma unroll
        for (int ey = 0; ey < 2; ++ey) {
            const int i1 = 2 * a2, j1 = 2 * b2 + ey, m1 = 2 * c2 + ez;
            if (j1 >= d1y || m1 >= d1z || i1 >= d1x) continue;
            const size_t at = ((size_t)m1 * d1y + j1) * d1x + i1;
            const int k0 = 4 * ez + 2 * ey;
            bool g0 = false, g1 = false;
            const float2 v0 = level_node(lo1[k0], hi1[k0], k_gas, R, lr, 1, m1, nz, g0);
            const float2 v1 = level_node(lo1[k0 + 1], hi1[k0 + 1], k_gas, R, lr, 1, m1, nz, g1);
            const uint32_t b0 = up | (g0 ? 2u : 0u), b1 = up | (g1 ? 2u : 0u);
            if (kVec) {
                // d1x is even: the pair is whole, 16-byte aligned in the nodes and 4-byte aligned in the mask
                *reinterpret_cast<float4 *>(nodes + off1 + at) = make_float4(v0.x, v0.y, v1.x, v1.y);
                *reinterpret_cast<uint32_t *>(mask + at) = b0 | (b1 << 16);
            } else {
                nodes[off1 + at] = v0;
                mask[at] = (uint16_t)b0;
                if (i1 + 1 < d1x) {
                    nodes[off1 + at + 1] = v1;
                    mask[at + 1] = (uint16_t)b1;
                }
            }
        }
    }
    if (L >= 2 && a2 < level_dim(nx, 2) && b2 < level_dim(ny, 2) && c2 < level_dim(nz, 2))
        nodes[off2 + ((size_t)c2 * level_dim(ny, 2) + b2) * level_dim(nx, 2) + a2] = n2;
    const int a3 = a2 >> 1, b3 = b2 >> 1, c3 = c2 >> 1;
    if (L >= 3 && (lane & 7) == 0 && a3 < level_dim(nx, 3) && b3 < level_dim(ny, 3) && c3 < level_dim(nz, 3))
        nodes[off3 + ((size_t)c3 * level_dim(ny, 3) + b3) * level_dim(nx, 3) + a3] = n3;
    if (L >= 4 && lane == 0 && X4 < level_dim(nx, 4) && (int)blockIdx.y < level_dim(ny, 4) &&
        (int)blockIdx.z < level_dim(nz, 4))
        nodes[off4 + ((size_t)blockIdx.z * level_dim(ny, 4) + blockIdx.y) * level_dim(nx, 4) + X4] = n4;
}

// Mask bits of levels first..L (the levels above the fused pass), OR-ed into
// every level-1 node's mask.  One thread per run of 8 level-1 nodes along x
// in 4 consecutive rows (y = 4q .. 4q+3): the runs lie inside one level-4
// node, so their ancestors from level 4 up are shared, and the 4 rows' loads
// are in flight together.
__global__ void mask_upper_kernel(const float2 *__restrict__ nodes, const int *__restrict__ off, int n0, int n1,
                                  int n2, int L, int first, uint16_t *__restrict__ mask)
{
    const int d0 = level_dim(n0, 1), d1 = level_dim(n1, 1), d2 = level_dim(n2, 1);
    const int runs = (d0 + 7) >> 3, quads = (d1 + 3) >> 2;
    const long long total = (long long)runs * quads * d2;
    for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < total;
         id += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(id % runs) * 8;
        const int j0 = (int)((id / runs) % quads) * 4;
        const int m = (int)(id / ((long long)runs * quads));
        uint32_t bits = 0;
        for (int l = first; l <= L; ++l) {
            const int e0 = level_dim(n0, l), e1 = level_dim(n1, l);
            const int sh = l - 1;
            if (node_merged(nodes[off[l] + ((m >> sh) * e1 + (j0 >> sh)) * e0 + (i >> sh)])) bits |= 1u << l;
        }
        if (!bits) continue;
        const int nj = min(4, d1 - j0);
        if ((d0 & 7) == 0) {
            // 8 masks a row, 16-byte aligned
            const uint32_t b2 = bits | (bits << 16);
            uint4 w[4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r < nj) w[r] = *reinterpret_cast<const uint4 *>(mask + ((size_t)m * d1 + j0 + r) * d0 + i);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (r >= nj) break;
                w[r].x |= b2;
                w[r].y |= b2;
                w[r].z |= b2;
                w[r].w |= b2;
                *reinterpret_cast<uint4 *>(mask + ((size_t)m * d1 + j0 + r) * d0 + i) = w[r];
            }
        } else {
            for (int r = 0; r < nj; ++r) {
                uint16_t *row = mask + ((size_t)m * d1 + j0 + r) * d0;
                for (int e = 0; e < 8 && i + e < d0; ++e) row[i + e] = (uint16_t)(row[i + e] | bits);
            }
        }
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

hipError_t launch_build(const nc_ctx *ctx, nc_grid *g, const float *d_kc, unsigned int *d_bad, int *d_zc)
{
    const int block = 256;
    LayerRule lr{nullptr, g->params.flat_level};
    if (g->params.criterion == 3) {
        const long long cells = (long long)g->n[0] * g->n[1] * g->n[2];
        hipLaunchKernelGGL(set_cloud_layer_kernel, dim3(1), dim3(64), 0, ctx->stream, d_zc, g->n[2]);
        hipLaunchKernelGGL(cloud_layer_kernel, dim3(blocks_for(cells, block, 4096)), dim3(block), 0, ctx->stream, d_kc,
                           cells, g->n[0] * g->n[1], d_zc);
        lr.zc = d_zc;
    }
    if (g->L < 1) return hipSuccess;
    // merge settings per level: the flat grid merges whole levels, as
    // criterion 0 against +inf (always true for finite k) or 0 (never true)
    auto rule = [&](int l, double &dz_node, double &tau, int &crit) {
        const bool flat = g->params.criterion == 2;
        dz_node = g->h[2] * (double)(1 << l);
        tau = flat ? (l <= g->params.flat_level ? INFINITY : 0.0) : g->params.tau_tilde;
        crit = flat ? 0 : g->params.criterion;
    };
    LevelRules R{};
    for (int l = 1; l <= 4; ++l) rule(l, R.dz_node[l], R.tau[l], R.crit[l]);
    const int n0 = g->n[0], n1 = g->n[1], n2 = g->n[2];
    const dim3 fgrid((level_dim(n0, 4) + kBuildWaves - 1) / kBuildWaves, level_dim(n1, 4), level_dim(n2, 4));
    const int lvl = std::min(g->L, 4);
    const int o2 = g->off[std::min(2, lvl)], o3 = g->off[std::min(3, lvl)], o4 = g->off[lvl];
    if (n0 % 4 == 0 && reinterpret_cast<uintptr_t>(d_kc) % 16 == 0)
        hipLaunchKernelGGL(build_fused_kernel<true>, fgrid, dim3(64 * kBuildWaves), 0, ctx->stream, d_kc, n0, n1, n2, g->d_nodes,
                           g->off[1], o2, o3, o4, g->d_mask, g->L, g->params.k_gas, R, lr, d_bad);
    else
        hipLaunchKernelGGL(build_fused_kernel<false>, fgrid, dim3(64 * kBuildWaves), 0, ctx->stream, d_kc, n0, n1, n2, g->d_nodes,
                           g->off[1], o2, o3, o4, g->d_mask, g->L, g->params.k_gas, R, lr, d_bad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the levels above: one launch each from the level below (small)
    for (int l = 5; l <= g->L; ++l) {
        const int d0 = level_dim(n0, l), d1 = level_dim(n1, l), d2 = level_dim(n2, l);
        const int c0 = level_dim(n0, l - 1), c1 = level_dim(n1, l - 1), c2 = level_dim(n2, l - 1);
        double dz_node = 0.0, tau = 0.0;
        int crit = 0;
        rule(l, dz_node, tau, crit);
        hipLaunchKernelGGL(build_level_kernel, dim3(blocks_for((long long)d0 * d1 * d2, block)), dim3(block), 0,
                           ctx->stream, (const float2 *)(g->d_nodes + g->off[l - 1]), c0, c1, c2,
                           g->d_nodes + g->off[l], d0, d1, d2, g->params.k_gas, dz_node, tau, crit, lr, l, n2);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (g->L >= 5) {
        const long long runs =
            (long long)((level_dim(n0, 1) + 7) / 8) * ((level_dim(n1, 1) + 3) / 4) * level_dim(n2, 1);
        hipLaunchKernelGGL(mask_upper_kernel, dim3(blocks_for(runs, block)), dim3(block), 0, ctx->stream,
                           (const float2 *)g->d_nodes, (const int *)g->d_off, n0, n1, n2, g->L, 5, g->d_mask);
        e = hipGetLastError();
    }
    return e;
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
        find_leaf(g, ns, r, 1.0f, reads);
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
    int est;                 // 0 delta, 1 ratio, 2 residual ratio tracking
    double *sum, *sumsq;
    nc_counters *counters;
    int lds_first, lds_nodes;
};

// Ratio (kctrl = 0) or residual ratio tracking (kctrl = the voxel minimum,
// collisions sampled with the residual majorant) of one ray to the box exit.
// The same estimators as the renderer's sun rays, as a plain loop.
__device__ inline float ratio_transmittance(const GridView &g, const NodeSrc &ns, Ray &r, Rng &rng, float mscale,
                                            bool resid, Counters &cnt)
{
    const float sun_rr = 0.1f;
    float T = 1.0f;
    auto kctrl = [&]() { return resid ? g.kscale * r.kmin + g.k_gas : 0.0f; };
    if (resid) r.khat = fmaxf(r.khat - kctrl(), 0.0f);
    float tau = rng.exp1();
    for (;;) {
        ++cnt.segments;
        const float ktau = r.khat * (r.texit - r.t);
        if (r.khat > 0.0f && tau < ktau) {
            const float t0 = r.t;
            r.t = fminf(r.t + tau / r.khat, r.texit);
            const float kc = kctrl();
            float kx = g.kscale * r.kmin + g.k_gas;
            if (r.lev != 0) {
                kx = g.kscale * g.kc[collision_cell(g, r, r.t)] + g.k_gas;
                ++cnt.gathers;
            }
            ++cnt.tentative;
            ++cnt.nulls;
            T *= __expf(-kc * (r.t - t0)) * fmaxf(0.0f, 1.0f - (kx - kc) / r.khat);
            if (T < sun_rr) T = rng.u01() * sun_rr < T ? sun_rr : 0.0f;
            if (T == 0.0f) return 0.0f;
            tau = rng.exp1();
        } else {
            if (resid) {
                T *= __expf(-kctrl() * (r.texit - r.t));
                if (T < sun_rr) T = rng.u01() * sun_rr < T ? sun_rr : 0.0f;
                if (T == 0.0f) return 0.0f;
            }
            tau -= ktau;
            uint32_t rd = 0;
            if (!next_leaf(g, ns, r, mscale, rd)) return T;
            cnt.node_reads += rd;
            ++cnt.leaf_visits;
            if (resid) r.khat = fmaxf(r.khat - kctrl(), 0.0f);
        }
    }
}

__global__ __launch_bounds__(256) void transmittance_kernel(TransArgs A)
{
    extern __shared__ __align__(16) float2 s_nodes[];
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
        double acc = 0.0, acc2 = 0.0;
        for (int s = s0; s < s1; ++s) {
            Rng rng;
            rng.init((uint32_t)i, (uint32_t)(A.sample_offset + s), 1u, A.seed);
            Ray r;
            start_ray(A.g, ns, r, o, d, A.mscale, cnt);
            float T;
            if (A.est == 0) {
                float tau = rng.exp1();
                float kc_hit = 0.0f;
                int res;
                do {
                    res = track_step(A.g, ns, r, tau, rng, A.mscale, true, kc_hit, cnt);
                } while (res == kContinue);
                T = res == kExit ? 1.0f : 0.0f;
            } else {
                T = ratio_transmittance(A.g, ns, r, rng, A.mscale, A.est == 2, cnt);
            }
            acc += T;
            acc2 += (double)T * T;
            ++cnt.paths;
            ++cnt.nee_rays;
        }
        unsafeAtomicAdd(A.sum + i, acc);
        unsafeAtomicAdd(A.sumsq + i, acc2);
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
    A.est = s.flags & NC_SUN_ESTIMATOR_MASK;
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


enum LaneState { kIdle = 0, kPath = 1, kShadow = 2 };
// Queue items a wave takes per global atomic: one per lane, so that the last
// chunks are short (paths differ a lot in cost and the launch ends with the
// slowest wave); 64 atomics per 64 x samples_per_item paths are cheap.
constexpr int kChunk = 64;
static_assert(kChunk >= 64, "a chunk must cover every lane of a wave that needs an item");

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

// Parameters of the renderer that only the sample, event and guide phases
// need (the launch record).  They live in device memory; each workgroup
// stages the ones its loop reads in LDS.
struct RenderRare {
    uint64_t seed, sample_offset;
    double *sum, *sumsq;
    const JobView *jobs;
    int n_jobs;
    int spp, spi;
    uint32_t stream_base;
    // guided mode: the queue sets (items of set k: [set_begin[k], set_begin[k + 1]),
    // 8 per-XCD queues of set_span[k] items) and each set's network
    unsigned long long set_begin[kMaxQueueSets + 1];
    unsigned long long set_span[kMaxQueueSets];
    unsigned long long *queue;      // 8 queue heads per queue set, 16 words apart
    int set_group[kMaxQueueSets];   // a workgroup starts on the last set k with set_group[k] <= blockIdx / 8
    GuideWeights gw[kMaxQueueSets];
    // the event phase's medium constants (read when an event runs)
    HGc hg;
    float ssa;
    int max_scatter;
};

// The fields of the launch record that the persistent loop reads, staged in
// LDS by each workgroup and read there where used (relaxed atomic LDS loads,
// which the compiler neither hoists out of the loop nor merges): no scalar
// registers are held for them across the loop.
struct RareShared {
    HGc hg;
    float ssa;
    int max_scatter;
    const JobView *jobs;
    double *sum, *sumsq;
    unsigned long long *queue;
    int n_jobs, spi, spp;
    unsigned long long set_begin[kMaxQueueSets + 1];
    unsigned long long set_span[kMaxQueueSets];
};

template <class T>
__device__ inline T lds_get(const T &x)
{
    return __hip_atomic_load(&x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ inline void stage_rare(const RenderRare &R, RareShared &S)
{
    S.hg = R.hg;
    S.ssa = R.ssa;
    S.max_scatter = R.max_scatter;
    S.jobs = R.jobs;
    S.sum = R.sum;
    S.sumsq = R.sumsq;
    S.queue = R.queue;
    S.n_jobs = R.n_jobs;
    S.spi = R.spi;
    S.spp = R.spp;
    for (int k = 0; k <= kMaxQueueSets; ++k) S.set_begin[k] = R.set_begin[k];
    for (int k = 0; k < kMaxQueueSets; ++k) S.set_span[k] = R.set_span[k];
}

struct RenderArgs {
    GridView g;
    OptView op;
    uint32_t key0, key1;        // Philox key (the seed)
    uint32_t sample_base;       // sample_offset (fits 32 bits)
    uint32_t stream_base;
    const RenderRare *rare;
    GuideWeights gw;            // guided mode: the first queue set's network
    float guide_frac;           // guided mode: probability of sampling the guide
    int guide_max_order;        // guided mode: last guided scattering order (0: all)
    CollectView col;            // collection mode: where vertices go
    int col_spp;                // collection mode: samples per pixel (path slot = pix * spp + sample)
    int guide_lds;              // byte offset of the per-wave guide scratch in dynamic LDS
    float gpos[3];              // network position input: (x - lo) * gpos - 1 spans [-1, 1] over the box
    nc_counters *counters;
    int n_sets;                 // guided mode: queue sets (described in the launch record)
    int lds_first, lds_nodes;
};

// Lane phases.  Each loop trip the wave runs the phase that the most lanes
// are waiting in (ballot counts); the other lanes wait.  Expensive code
// (events, ray starts, new samples) thus runs for many lanes at once instead
// of diverging inside every traversal step.
enum Phase { kPhCross = 0, kPhCollide = 1, kPhEvent = 2, kPhRay = 3, kPhSample = 4, kPhGuide = 5, kPhIdle = 6 };
constexpr int kGuideMaxWait = 8;   // trips a partial tile of guided lanes may wait for more
enum RenderMode { kPlain = 0, kGuided = 1, kCollect = 2 };
// ratio estimators: Russian roulette of a sun ray's estimate below this
// transmissivity (survivors carry it).  On the cumulus view 0.25 reaches a
// given image error soonest: 0.1 takes 1.6 % longer (more voxel crossings of
// nearly spent sun rays), 0.5 takes 5 % longer (more variance).
constexpr float kSunRoulette = 0.25f;
static_assert(kPhGuide == 5 && kPhIdle == 6, "six running phases, one counter slot each");

// After the optical thickness tau has been drawn or carried: a tentative
// collision inside the current voxel, or a move to the next voxel.
__device__ inline int voxel_phase(const Ray &r, float tau)
{
    return (r.khat > 0.0f && tau < r.khat * (r.texit - r.t)) ? kPhCollide : kPhCross;
}

// block-level event counters in LDS (same order as nc_counters)
enum BlockCounter {
    kCPaths = 0, kCSegments, kCTentative, kCNulls, kCReals, kCLeaf, kCGathers, kCReads, kCNee, kCTrunc,
    kCTrips0, kCLanes0 = kCTrips0 + 6, kCCycles0 = kCLanes0 + 6, kCDeep = kCCycles0 + 6,
    kNumBlockCounters = kCDeep + 1
};

__device__ inline void wave_count(unsigned long long *s_cnt, int k, bool pred)
{
    if (!s_cnt) return;   // no counters asked for
    const unsigned long long m = __ballot(pred);
    if (m && __lane_id() == 0) atomicAdd(s_cnt + k, (unsigned long long)__popcll(m));
}

__device__ inline void camera_ray_v(const CamView &c, int px, int py, float u1, float u2, float o[3],
                                    float d[3])
{
    const float W = (float)c.W, H = (float)c.H;
    if (c.type == 0) {
        const float sx = (2.0f * ((float)px + u1) / W - 1.0f) * c.sx;
        const float sy = (1.0f - 2.0f * ((float)py + u2) / H) * c.sy;
        float v[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o[a] = c.pos[a];
            v[a] = c.f[a] + sx * c.r[a] + sy * c.u[a];
        }
        const float inv = rsqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) d[a] = v[a] * inv;
    } else if (c.type == 1) {
        const float sx = (((float)px + u1) / W - 0.5f) * c.sx;
        const float sy = (0.5f - ((float)py + u2) / H) * c.sy;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o[a] = c.pos[a] + sx * c.r[a] + sy * c.u[a];
            d[a] = c.f[a];
        }
    } else {
        // horizontal sensor: px along +x, py along +y, looking up
        o[0] = c.pos[0] + (((float)px + u1) / W - 0.5f) * c.sx;
        o[1] = c.pos[1] + (((float)py + u2) / H - 0.5f) * c.sy;
        o[2] = c.pos[2];
        d[0] = 0.0f;
        d[1] = 0.0f;
        d[2] = 1.0f;
    }
}

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// The network in LDS.  Layer 1 (15 inputs padded to 16) keeps W [out][in]
// with rows padded to 20 bf16 and runs as 16x16x16 products.  Layers 2..4
// (K = 64) run as two 16x16x32 products per 16-row block: the B operand of
// k-block kb is the lane's own outputs of the previous layer's blocks 2 kb and
// 2 kb + 1, so slot (lane group q, element e) of k-block kb stands for neuron
// 16 (2 kb + e / 4) + 4 q + e % 4.  The weights are staged with their
// columns in that order (rows of 72 bf16: 16-byte aligned fragment reads that
// fall on distinct banks).  The last layer's 40 rows are also permuted, to 48:
// lane group q of a tile column receives lobes 2 q and 2 q + 1, five values
// each, in its first ten output slots (the last two are zero rows).
constexpr int kW1Stride = 20, kWStride = 72;
constexpr int kWOff[5] = {0, 64 * kW1Stride, 64 * kW1Stride + 64 * kWStride, 64 * kW1Stride + 2 * 64 * kWStride,
                          64 * kW1Stride + 2 * 64 * kWStride + 48 * kWStride};
constexpr int kBOff[4] = {0, 64, 128, 192};
constexpr int kGuideWeightBytes = kWOff[4] * 2 + 240 * 4;                   // 28864
// per wave: the tile's inputs ([16][16] bf16) and per-vertex floats ([16][8]:
// incoming direction, the four uniforms of the step)
constexpr int kGuideInBytes = 16 * 16 * 2;
constexpr int kGuideScratchPerWave = kGuideInBytes + 16 * 8 * 4;           // 1024
static_assert(kWOff[1] % 8 == 0 && kWOff[2] % 8 == 0 && kWOff[3] % 8 == 0 && kWOff[4] % 8 == 0,
              "16-byte aligned weight blocks");

// neuron k of a 64-wide layer -> its column in the K = 32 operand order
__device__ inline int k32_col(int k)
{
    const int blk = k >> 4, r = k & 15;
    return 32 * (blk >> 1) + 8 * (r >> 2) + 4 * (blk & 1) + (r & 3);
}

// permuted last-layer row m (0..47) -> network output index, or -1 (zero row)
__device__ inline int out_row_src(int m)
{
    const int q = (m & 15) >> 2, s = 4 * (m >> 4) + (m & 3);
    return s < 10 ? 5 * (2 * q + (s >= 5 ? 1 : 0)) + (s >= 5 ? s - 5 : s) : -1;
}

// Copy the packed network (W_pad [out_pad][in_pad] bf16 and fp32 biases per
// layer) into the LDS layout above; all threads of the block take part.
__device__ inline void stage_guide(const GuideWeights &W, short *wl, float *bl)
{
    for (int i = threadIdx.x; i < 64 * 16; i += blockDim.x) wl[(i >> 4) * kW1Stride + (i & 15)] = W.w[0][i];
    for (int l = 1; l < 3; ++l)
        for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x)
            wl[kWOff[l] + (i >> 6) * kWStride + k32_col(i & 63)] = W.w[l][i];
    for (int i = threadIdx.x; i < 48 * 64; i += blockDim.x) {
        const int m = i >> 6, k = i & 63, src = out_row_src(m);
        wl[kWOff[3] + m * kWStride + k32_col(k)] = src >= 0 ? W.w[3][src * 64 + k] : (short)0;
    }
    for (int i = threadIdx.x; i < 64; i += blockDim.x) {
        bl[kBOff[0] + i] = W.b[0][i];
        bl[kBOff[1] + i] = W.b[1][i];
        bl[kBOff[2] + i] = W.b[2][i];
        if (i < 48) {
            const int src = out_row_src(i);
            bl[kBOff[3] + i] = src >= 0 ? W.b[3][src] : 0.0f;
        }
    }
}

// bf16 of four floats (round to nearest even; v_cvt_pk_bf16_f32 on gfx950).
__device__ inline bf16x4 cvt_bf16x4(float a, float b, float c, float d)
{
    bf16x4 r;
    r[0] = __builtin_bit_cast(short, (__bf16)a);
    r[1] = __builtin_bit_cast(short, (__bf16)b);
    r[2] = __builtin_bit_cast(short, (__bf16)c);
    r[3] = __builtin_bit_cast(short, (__bf16)d);
    return r;
}

// A K = 64 layer for the 16 vertices of a tile is D = W X^T with the weights
// as the A operand (rows = output neurons) and the activations as the B
// operand (columns = vertices).  Lane l receives
// out[vertex l % 16][16 nt + 4 (l / 16) + i] of block nt: the next layer's B slots.
// The ReLU acts on the rounded values as a signed 16-bit max with zero: a
// negative bf16 has its sign bit set, so it reads as a negative integer and
// becomes +0, while a positive one is unchanged; that is bf16(max(x, 0)) bit
// for bit up to the sign of a zero.  One packed instruction per pair, where
// fmaxf on the floats takes two per value (it first quiets a possible
// signalling NaN).
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 b16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ inline s16x2 relu_bf16x2(float a, float b)
{
    const s16x2 v = __builtin_bit_cast(s16x2, __builtin_convertvector(f32x2{a, b}, b16x2));
    return __builtin_elementwise_max(v, s16x2{0, 0});
}
__device__ inline bf16x4 relu_bf16x4(f32x4 c)
{
    return __builtin_shufflevector(relu_bf16x2(c[0], c[1]), relu_bf16x2(c[2], c[3]), 0, 1, 2, 3);
}

// Two 16-row blocks nt0, nt0 + 1 of a K = 64 layer.  Each weight fragment is
// read from LDS where its product needs it: reading all four ahead overlapped
// their latencies but held 16 more registers, which kept the guided renderer
// at 3 waves per SIMD (at 4 the other waves hide the latency).
__device__ inline void guide_pair32(const short *w, const float *b, int nt0, bf16x8 x0, bf16x8 x1, int n, int kq,
                                    f32x4 &c0, f32x4 &c1)
{
    const short *r0 = w + (nt0 * 16 + n) * kWStride + 8 * kq;
    const short *r1 = r0 + 16 * kWStride;
    // the bias is the accumulator's starting value
    c0 = mfma32(*reinterpret_cast<const bf16x8 *>(r0 + 32), x1,
                mfma32(*reinterpret_cast<const bf16x8 *>(r0), x0,
                       *reinterpret_cast<const f32x4 *>(b + nt0 * 16 + 4 * kq)));
    c1 = mfma32(*reinterpret_cast<const bf16x8 *>(r1 + 32), x1,
                mfma32(*reinterpret_cast<const bf16x8 *>(r1), x0,
                       *reinterpret_cast<const f32x4 *>(b + (nt0 + 1) * 16 + 4 * kq)));
}

__device__ inline void guide_hidden32(const short *w, const float *b, const bf16x4 *x, bf16x4 *y, int n, int kq)
{
    const bf16x8 x0 = __builtin_shufflevector(x[0], x[1], 0, 1, 2, 3, 4, 5, 6, 7);
    const bf16x8 x1 = __builtin_shufflevector(x[2], x[3], 0, 1, 2, 3, 4, 5, 6, 7);
    f32x4 c0, c1;
    guide_pair32(w, b, 0, x0, x1, n, kq, c0, c1);
    y[0] = relu_bf16x4(c0);
    y[1] = relu_bf16x4(c1);
    guide_pair32(w, b, 2, x0, x1, n, kq, c0, c1);
    y[2] = relu_bf16x4(c0);
    y[3] = relu_bf16x4(c1);
}

// The network on one tile of 16 vertices held by one wave.  in: the tile's
// [16][16] bf16 inputs (row = vertex, the 15 network inputs then a zero).  On return
// z[4 nt + i] (bf16-rounded) is permuted output row 16 nt + 4 (lane / 16) + i
// of vertex lane % 16: z[0..4] and z[5..9] are lobes 2 (lane / 16) and
// 2 (lane / 16) + 1 (logit, unnormalised mean, log kappa).
__device__ inline void guide_tile_forward(const short *wl, const float *bl, const short *in, int lane, float z[12])
{
    const int n = lane & 15, kq = lane >> 4;
    bf16x4 h[4], y[4];
    const bf16x4 x0 = *reinterpret_cast<const bf16x4 *>(in + n * 16 + 4 * kq);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
        y[nt] = relu_bf16x4(mfma16(*reinterpret_cast<const bf16x4 *>(wl + (nt * 16 + n) * kW1Stride + 4 * kq), x0,
                                   *reinterpret_cast<const f32x4 *>(bl + kBOff[0] + nt * 16 + 4 * kq)));
    guide_hidden32(wl + kWOff[1], bl + kBOff[1], y, h, n, kq);
    guide_hidden32(wl + kWOff[2], bl + kBOff[2], h, y, n, kq);
    const bf16x8 y0 = __builtin_shufflevector(y[0], y[1], 0, 1, 2, 3, 4, 5, 6, 7);
    const bf16x8 y1 = __builtin_shufflevector(y[2], y[3], 0, 1, 2, 3, 4, 5, 6, 7);
    f32x4 c0, c1;
    guide_pair32(wl + kWOff[3], bl + kBOff[3], 0, y0, y1, n, kq, c0, c1);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        z[i] = from_bf16(to_bf16(c0[i]));
        z[4 + i] = from_bf16(to_bf16(c1[i]));
    }
    // rows 32..47: slots 8..11 (the last two are zero rows)
    const short *row = wl + kWOff[3] + (32 + n) * kWStride + 8 * kq;
    const bf16x8 wa0 = *reinterpret_cast<const bf16x8 *>(row), wa1 = *reinterpret_cast<const bf16x8 *>(row + 32);
    const f32x4 b2 = *reinterpret_cast<const f32x4 *>(bl + kBOff[3] + 32 + 4 * kq);
    const f32x4 c2 = mfma32(wa1, y1, mfma32(wa0, y0, b2));
#pragma unroll
    for (int i = 0; i < 4; ++i) z[8 + i] = from_bf16(to_bf16(c2[i]));
}

// Guided scattering (one-sample MIS): with probability c the new direction
// comes from the network's vMF mixture, otherwise from HG; the path weight is
// multiplied by p_HG / (c q + (1 - c) p_HG).  The step runs where the last
// product leaves the outputs: the four lanes n, n + 16, n + 32, n + 48 of
// tile column n hold two lobes each (z from guide_tile_forward).  The lobe
// sums, the choice of lobe and the mixture density are shared across the four
// lanes; all four end with the same direction and factor.  slot: the
// column's floats (incoming direction, u_sel, u_lobe, u1, u2).  The whole
// wave calls it.
struct GuidedStep {
    float d[3];   // new direction
    float w;      // weight factor p / (c q + (1 - c) p)
    float q, p;   // mixture and HG densities at d
};

// The value lane l ^ 16 (or l ^ 32) holds, by the gfx950 row swaps: of the
// pair the swap returns, one is the lane's own value, the other its partner's
// (equal bits make the choice immaterial).
__device__ inline float lane_xor16(float v)
{
    const uint32_t u = __float_as_uint(v);
    const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    return __uint_as_float(r[0] == u ? r[1] : r[0]);
}

__device__ inline float lane_xor32(float v)
{
    const uint32_t u = __float_as_uint(v);
    const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    return __uint_as_float(r[0] == u ? r[1] : r[0]);
}

// Sum and maximum of the lane's value and that of lane l ^ 16 (l ^ 32): the
// swap returns both values, in the same order in the two lanes of a pair.
__device__ inline float lane_sum16(float v)
{
    const uint32_t u = __float_as_uint(v);
    const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ inline float lane_sum32(float v)
{
    const uint32_t u = __float_as_uint(v);
    const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ inline float lane_max16(float v)
{
    const uint32_t u = __float_as_uint(v);
    const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    return fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
}

__device__ inline float lane_max32(float v)
{
    const uint32_t u = __float_as_uint(v);
    const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    return fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
}

template <bool kTab>
__device__ inline GuidedStep guided_turn_tile(const float z[12], const float *slot, float c, const HGc &g,
                                              const PhaseView &tab, int kq)
{
    const float amax = lane_max32(lane_max16(fmaxf(z[0], z[5])));
    const float e0 = __expf(z[0] - amax), e1 = __expf(z[5] - amax);
    // the four group sums in lobe order, accumulated the same way in all four lanes
    const float loc = e0 + e1, loc16 = lane_xor16(loc);
    const float lev = (kq & 1) ? loc16 : loc, lod = (kq & 1) ? loc : loc16;   // groups 2 (kq / 2) and 2 (kq / 2) + 1
    const float xev = lane_xor32(lev), xod = lane_xor32(lod);
    const bool lowh = kq < 2;
    const float l0 = lowh ? lev : xev, l1 = lowh ? lod : xod, l2 = lowh ? xev : lev, l3 = lowh ? xod : lod;
    const float c1 = l0, c2 = c1 + l1, c3 = c2 + l2, psum = c3 + l3;
    const float pd[3] = {slot[0], slot[1], slot[2]};
    const float u_sel = slot[3], u_lobe = slot[4], u1 = slot[5], u2 = slot[6];
    const bool mix = u_sel < c;
    // the lobe: the first whose cumulative weight exceeds u_lobe * sum
    const float target = u_lobe * psum;
    const int qs = (target >= c1 ? 1 : 0) + (target >= c2 ? 1 : 0) + (target >= c3 ? 1 : 0);
    // both candidates in every lane, without branches, so that their
    // dependent chains interleave: the vMF draw from this lane's lobe that
    // the choice would fall on (used only in lane group qs) and the HG draw
    const float lo = kq == 0 ? 0.0f : kq == 1 ? c1 : kq == 2 ? c2 : c3;
    const bool second = target >= lo + e0;
    // per lobe of this lane: the reciprocal length of its mean, kappa and
    // exp(-2 kappa), shared by the draw and the mixture density
    float il[2], kl[2], el[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const float m0 = z[5 * h + 1], m1 = z[5 * h + 2], m2 = z[5 * h + 3];
        il[h] = rsqrtf(fmaxf(m0 * m0 + m1 * m1 + m2 * m2, 1e-24f));
        kl[h] = __expf(fminf(fmaxf(z[5 * h + 4], kLogKappaMin), kLogKappaMax));
        el[h] = __expf(-2.0f * kl[h]);
    }
    const float inv = second ? il[1] : il[0], kap = second ? kl[1] : kl[0];
    // the stable vMF cosine inversion (Jakob 2012)
    const float t = fminf(1.0f, fmaxf(-1.0f, 1.0f + __logf(u1 + (1.0f - u1) * (second ? el[1] : el[0])) *
                                                       __builtin_amdgcn_rcpf(kap)));
    const float sp = __builtin_amdgcn_sinf(u2), cp = __builtin_amdgcn_cosf(u2);   // the azimuth of both candidates
    float v[3] = {(second ? z[6] : z[1]) * inv, (second ? z[7] : z[2]) * inv, (second ? z[8] : z[3]) * inv};
    turn_sc(v, t, sp, cp);
    float hgd[3] = {pd[0], pd[1], pd[2]};
    turn_sc(hgd, kTab ? phase_sample_mu(g, tab, u1) : hg_sample_mu(g, u1), sp, cp);
    GuidedStep o;
    // the chosen lobe's direction from lane group qs of the column
    const int rel = qs ^ kq;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float v16 = lane_xor16(v[a]), v32 = lane_xor32(v[a]), v48 = lane_xor32(v16);
        const float vs = rel == 0 ? v[a] : rel == 1 ? v16 : rel == 2 ? v32 : v48;
        o.d[a] = mix ? vs : hgd[a];
    }
    // mixture density at the new direction: two lobes per lane, then the column sum
    float qp = 0.0f;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const float m0 = z[5 * h + 1], m1 = z[5 * h + 2], m2 = z[5 * h + 3];
        const float cw = (m0 * o.d[0] + m1 * o.d[1] + m2 * o.d[2]) * il[h];
        // kappa >= e^-3, so 1 - exp(-2 kappa) >= 0.095 keeps its relative precision
        const float norm = kl[h] * __builtin_amdgcn_rcpf(2.0f * kPi * (1.0f - el[h]));
        qp += (h == 0 ? e0 : e1) * norm * __expf(kl[h] * (cw - 1.0f));
    }
    qp = lane_sum32(lane_sum16(qp));   // the same sum in every lane of the column
    o.q = qp * __builtin_amdgcn_rcpf(psum);
    const float mu_o = pd[0] * o.d[0] + pd[1] * o.d[1] + pd[2] * o.d[2];
    o.p = kTab ? phase_eval(g, tab, mu_o) : hg_phase(g, mu_o);
    o.w = o.p * __builtin_amdgcn_rcpf(c * o.q + (1.0f - c) * o.p);
    return o;
}

// A direction drawn uniformly in the solar disc's cone about s (cosine
// uniform on [cos alpha, 1], azimuth 2 pi u2).
__device__ inline void cone_dir(const float s[3], float cos_a, float u1, float u2, float w[3])
{
    w[0] = s[0];
    w[1] = s[1];
    w[2] = s[2];
    turn(w, 1.0f - u1 * (1.0f - cos_a), u2);
}

// The number that picks the lobe: given u_sel < c, u_sel / c is uniform on
// [0, 1) and independent of the branch taken (unused otherwise).
__device__ inline float lobe_uniform(float u_sel, float c)
{
    return fminf(u_sel * __builtin_amdgcn_rcpf(c), 0.99999994f);
}

// A tile row's network inputs as bf16 (the 15 from the vertex's 7 values,
// then a zero) in two 16-byte stores.
__device__ inline void put_guide_inputs(short *row, const float x[7])
{
    bf16x8 a, b;
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = to_bf16(guide_feature(x, k));
#pragma unroll
    for (int k = 0; k < 7; ++k) b[k] = to_bf16(guide_feature(x, 8 + k));
    b[7] = 0;
    reinterpret_cast<bf16x8 *>(row)[0] = a;
    reinterpret_cast<bf16x8 *>(row)[1] = b;
}

// The renderer's guided scattering step on given vertices (one wave per 64):
// in rows of 8 floats (the vertex's 7 values; the incoming direction is
// values 3..5), u rows of 4 uniforms, out rows of 8 floats (new direction,
// weight factor, q, p_HG, 0, 0).
__global__ __launch_bounds__(64) void guide_sample_kernel(GuideWeights W, const float *__restrict__ in,
                                                          const float *__restrict__ u, float c, HGc g, int n,
                                                          float *__restrict__ out)
{
    __shared__ __align__(16) short wl[kWOff[4]];
    __shared__ __align__(16) float bl[240];
    __shared__ __align__(16) char tile[kGuideScratchPerWave];
    stage_guide(W, wl, bl);
    __syncthreads();
    short *tin = reinterpret_cast<short *>(tile);
    float *tf = reinterpret_cast<float *>(tile + kGuideInBytes);
    const int lane = threadIdx.x, col = lane & 15, kq = lane >> 4;
    for (int base = blockIdx.x * 64; base < n; base += gridDim.x * 64) {
        for (int t = 0; t < 4; ++t) {
            const int r = base + 16 * t + col;
            const bool valid = r < n;
            if (kq == 0) {
                float x[7];
                for (int k = 0; k < 7; ++k) x[k] = valid ? in[(size_t)r * 8 + k] : 0.0f;
                if (!valid) x[5] = 1.0f;
                put_guide_inputs(tin + col * 16, x);
                float *f = tf + col * 8;
                f[0] = x[3];
                f[1] = x[4];
                f[2] = x[5];
                const float u_sel = valid ? u[(size_t)r * 4] : 0.5f;
                f[3] = u_sel;
                f[4] = lobe_uniform(u_sel, c);
                f[5] = valid ? u[(size_t)r * 4 + 2] : 0.5f;
                f[6] = valid ? u[(size_t)r * 4 + 3] : 0.5f;
                f[7] = 0.0f;
            }
            wave_sync();
            float z[12];
            guide_tile_forward(wl, bl, tin, lane, z);
            const GuidedStep st = guided_turn_tile<false>(z, tf + col * 8, c, g, PhaseView{nullptr, nullptr, nullptr, 0}, kq);
            if (kq == 0 && valid) {
                float *o = out + (size_t)r * 8;
                o[0] = st.d[0];
                o[1] = st.d[1];
                o[2] = st.d[2];
                o[3] = st.w;
                o[4] = st.q;
                o[5] = st.p;
                o[6] = 0.0f;
                o[7] = 0.0f;
            }
            wave_sync();
        }
    }
}

// The tabulated phase function's sampler and value on given uniforms.
__global__ void phase_sample_kernel(PhaseView t, const float *__restrict__ u, int n, float *__restrict__ out)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float m = tab_sample(t, u[i]);
        out[2 * i] = m;
        out[2 * i + 1] = tab_phase(t, m);
    }
}

hipError_t launch_phase_sample(const nc_ctx *ctx, const PhaseView &t, const float *u, int n, float *out)
{
    hipLaunchKernelGGL(phase_sample_kernel, dim3(std::max(1, std::min((n + 255) / 256, 4096))), dim3(256), 0,
                       ctx->stream, t, u, n, out);
    return hipGetLastError();
}

hipError_t launch_guide_sample(const nc_ctx *ctx, const nc_guide *gd, const float *in, const float *u, float c,
                               float g, int n, float *out)
{
    const int blocks = std::max(1, std::min((n + 63) / 64, 4096));
    hipLaunchKernelGGL(guide_sample_kernel, dim3(blocks), dim3(64), 0, ctx->stream, guide_weights(gd), in, u, c,
                       make_hg(g), n, out);
    return hipGetLastError();
}

// kSets: the guided batch with more than one network (queue set); a
// workgroup whose set has drained moves to another.  Compiled only where a
// launch has several sets: the loop around the tracing loop keeps many more
// values live (the single-view guided kernel without it has 14 % fewer vector
// instructions in its code, keeps its scalars in scalar registers and renders
// 10 % faster).
template <int kWavesPerEU, int kMode, int kSun, bool kExt, bool kSets = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWavesPerEU))) void render_kernel(RenderArgs A)
{
    static_assert(!kSets || kMode == kGuided, "queue sets are for guided batches");
    extern __shared__ __align__(16) float2 s_nodes[];
    __shared__ int s_off[NC_MAX_LEVELS + 2];
    __shared__ unsigned long long s_cnt[kNumBlockCounters];
    __shared__ int s_next_set;
    __shared__ RareShared s_rare;
    for (int i = threadIdx.x; i < kNumBlockCounters; i += blockDim.x) s_cnt[i] = 0ull;
    if (threadIdx.x == 0) stage_rare(*A.rare, s_rare);   // visible after the barrier in stage_levels
    int cur = 0;   // workgroup-uniform: the queue set (and network) this workgroup serves
    if (kMode == kGuided) {
        const int grp = (int)(blockIdx.x >> 3);
        if (kSets)
            for (int k = 1; k < A.n_sets; ++k)
                if (grp >= A.rare->set_group[k]) cur = k;
        char *gb = reinterpret_cast<char *>(s_nodes) + A.guide_lds;
        if (cur == 0) {
            stage_guide(A.gw, reinterpret_cast<short *>(gb), reinterpret_cast<float *>(gb + kWOff[4] * 2));
        } else {
            const GuideWeights W = A.rare->gw[cur];
            stage_guide(W, reinterpret_cast<short *>(gb), reinterpret_cast<float *>(gb + kWOff[4] * 2));
        }
    }
    stage_levels(A.g, A.lds_first, A.lds_nodes, s_nodes, s_off);   // ends with a block barrier
    const GridView &g = A.g;
    const NodeSrc ns{g.nodes, s_nodes, s_off, A.lds_first, s_off[A.lds_first <= g.L ? A.lds_first : 0], g.n[0],
                     g.n[1]};
    // launch-record fields, read from LDS at each use
#define NC_R(f) lds_get(s_rare.f)
    const int lane = __lane_id();
    // statistics (ballots, LDS atomics, clock reads) only when counters are asked for
    const bool stats = A.counters != nullptr;
    unsigned long long *const cnt = stats ? s_cnt : nullptr;
    int job = 0;                           // the lane's current view x sun
    float sun[3] = {0.0f, 0.0f, 1.0f};     // that job's sun direction (its irradiance is applied at the flush)

    int phase = kPhSample;
    bool shadow = false;       // the current ray is a sun ray
    bool have_item = false;    // the lane holds a queue item with samples left
    bool traced = false;       // a path has been traced since the last sample phase
    int res = kContinue;       // outcome of the last step (for the event phase)
    float kc_hit = 0.0f;       // k_c at the last real collision of a path ray
    float &t_sun = kc_hit;     // during a sun ray (ratio estimators): its transmissivity estimate so far
    int pix = 0, s = 0, s_end = 0;
    float acc = 0.0f, acc2 = 0.0f;
    float Lp = 0.0f;
    Ray r;                     // at an event, r.o holds the event position (origin of the next ray)
    float tau = 0.0f;
    RngBuf rng;
    rng.reset();
    float pd[3] = {0, 0, 0};   // path direction / direction of the next path ray
    float w_nee = 0.0f;        // sun contribution of the current event if its sun ray gets through
    float p_cont = 0.0f;       // probability that the path goes on after the event
    bool ground_ev = false;
    int order = 0, segs = 0;
    float beta = 1.0f;                   // path weight (guided mode)
    float kev = 0.0f;                    // extinction at the current event (guided and collection modes)
    float kg = g.k_gas;                  // the path's gas extinction: a k-distribution point (kExt)
    // kExt: the extended medium (a k-distribution, a tabulated phase function,
    // the solar disc); the other variants have none of them in their code, so
    // neither a register for a per-path gas extinction nor the table's search
    auto path_kg = [&]() { return kExt ? kg : g.k_gas; };
    unsigned long long chunk_base = 0;   // wave-uniform: the wave's chunk of queue items
    int chunk_left = 0;
    bool queue_done = false;
    int q_seen = 0;                      // wave-uniform: queues found drained (its XCD's first)
    int guide_wait = 0;                  // wave-uniform: trips that lanes have waited for the network
    uint32_t tried = 0;                  // workgroup-uniform: queue sets this workgroup has served

    // the current queue set's items and queues, read where used (the plain
    // and collection kernels have one set)
#define NC_SET_LO() NC_R(set_begin[cur])
#define NC_SET_HI() NC_R(set_begin[cur + 1])
#define NC_SET_SPAN() NC_R(set_span[cur])
#define NC_SET_QUEUE() (NC_R(queue) + 128 * cur)
    for (;;) {   // one queue set at a time (a single pass unless guides differ across jobs)
    for (;;) {
        // lane counts per phase (scalar: 32-bit popcounts of the ballots); a
        // crossing step and a ray start run in the same trip (the step phase)
        const int n_step = (int)__builtin_amdgcn_readfirstlane(
            __popcll(__ballot((phase == kPhCross) | (phase == kPhRay))));
        const int n_coll = (int)__builtin_amdgcn_readfirstlane(__popcll(__ballot(phase == kPhCollide)));
        const int n_event = (int)__builtin_amdgcn_readfirstlane(__popcll(__ballot(phase == kPhEvent)));
        const int n_sample = (int)__builtin_amdgcn_readfirstlane(__popcll(__ballot(phase == kPhSample)));
        const int n_guide =
            kMode == kGuided ? (int)__builtin_amdgcn_readfirstlane(__popcll(__ballot(phase == kPhGuide))) : 0;
        const int n_other = n_step + n_coll + n_event + n_sample;
        if (n_other + n_guide == 0) break;
        int run = kPhCross, best = n_step;
        if (n_coll >= best) { run = kPhCollide; best = n_coll; }
        if (n_event >= best) { run = kPhEvent; best = n_event; }
        if (n_sample > best) { run = kPhSample; best = n_sample; }
        if (kMode == kGuided && n_guide > 0) {
            // lanes waiting for the network run as full tiles of 16, once two
            // tiles' worth wait (the phase's set-up is then shared by at least
            // two tiles: 2 % faster on the cumulus view than at one tile, while
            // waiting for three or four costs more lane time than it saves); a
            // partial tile only when nothing else is left or the wait grows long
            const bool flush = n_other == 0 || guide_wait >= kGuideMaxWait;
            if (n_guide >= 32 || flush) {
                run = kPhGuide;
                best = flush ? n_guide : (n_guide & ~15);
                guide_wait = 0;
            } else {
                ++guide_wait;
            }
        }
        if (stats && lane == 0) {
            atomicAdd(s_cnt + kCTrips0 + run, 1ull);
            atomicAdd(s_cnt + kCLanes0 + run, (unsigned long long)best);
        }
        const long long t_trip = stats ? wall_clock64() : 0;

        if (run == kPhCross) {
            // ---- a step of the ordered crossing: lanes crossing into the next
            // voxel (carrying the optical thickness) and lanes starting a ray
            // (from an event point along pd or towards the sun, or from the
            // camera) share the location of the voxel (ancestry mask, node)
            // and its exit face
            const bool crossing = phase == kPhCross, starting = phase == kPhRay;
            const bool resid = crossing && shadow && kSun == 2;
            bool locate = false, leaf = false, hit = false, trunc = false;
            if (resid) t_sun *= __expf(-(g.kscale * r.kmin + path_kg()) * (r.texit - r.t));
            // one random number at most: the Russian roulette of a small residual
            // estimate, or the optical thickness of a new ray
            const bool roul = resid && t_sun < kSunRoulette;
            if (roul || starting)
                rng.need(1, (uint32_t)pix, A.sample_base + (uint32_t)s, A.stream_base + (uint32_t)job, A.key0, A.key1);
            if (roul) t_sun = rng.take() * kSunRoulette < t_sun ? kSunRoulette : 0.0f;
            if (crossing) {
                tau -= r.khat * (r.texit - r.t);
                if (resid && t_sun == 0.0f) {
                    res = kReal;                    // the estimate is zero: the sun ray ends here
                    phase = kPhEvent;
                } else if (!step_cell(g, r)) {
                    res = kExit;
                    phase = kPhEvent;
                } else {
                    locate = true;
                }
            } else if (starting) {
                const float o[3] = {r.o[0], r.o[1], r.o[2]};
                const float rd[3] = {shadow ? sun[0] : pd[0], shadow ? sun[1] : pd[1], shadow ? sun[2] : pd[2]};
                if (ray_setup(g, r, o, rd, 0.0f)) {
                    hit = true;
                    // the start voxel is located afresh: keeping the event's voxel
                    // per lane to skip this lookup cost six registers through the
                    // whole loop, which cost more than the lookups
                    locate = true;
                } else {
                    // misses the box: the next step finds the ray outside
                    r.t = r.tend = r.texit = 0.0f;
                    r.khat = 0.0f;
                    r.kmin = 0.0f;
                    r.lev = g.L;
                }
            }
            if (locate) {
                uint32_t nr = 0;   // (counted by ballot below when statistics are on)
                locate_voxel(g, ns, r, A.op.mscale, nr);
            }
            if (locate) leaf_exit(g, r);
            if (crossing && locate) {
                leaf = true;
                if (resid) r.khat = fmaxf(r.khat - (g.kscale * r.kmin + path_kg()), 0.0f);
                phase = voxel_phase(r, tau);
                if (++segs >= A.op.max_segments) {
                    trunc = true;
                    phase = kPhSample;      // stop the path
                }
            }
            if (starting) {
                if (kSun != 0 && shadow) {
                    t_sun = 1.0f;
                    if (kSun == 2) r.khat = fmaxf(r.khat - (g.kscale * r.kmin + path_kg()), 0.0f);
                }
                tau = rng.take_exp1();
                phase = voxel_phase(r, tau);
            }
            if (stats) {
                // memory reads of a voxel lookup: the cell, the ancestry mask, and the
                // node when its level is not staged in LDS
                wave_count(cnt, kCReads, locate);
                if (g.L >= 1) wave_count(cnt, kCReads, locate);
                wave_count(cnt, kCReads, locate && r.lev >= 1 && r.lev < ns.lds_first);
                wave_count(cnt, kCSegments, crossing);
                wave_count(cnt, kCLeaf, leaf || hit);
                wave_count(cnt, kCDeep, (leaf || hit) && r.lev < ns.lds_first);
                wave_count(cnt, kCTrunc, trunc);
                wave_count(cnt, kCNee, starting && shadow);
            }
        } else if (run == kPhCollide) {
            // ---- tentative collision in the current voxel: real or null
            const bool active = phase == kPhCollide;
            bool real = false, gathered = false, trunc = false;
            if (active && shadow && kSun != 0) {
                // ratio tracking (control 0) or residual ratio tracking (control
                // = the voxel minimum; r.khat then holds the residual majorant):
                // every tentative collision scales the estimate t_sun by
                // 1 - (k - k_ctrl) / khat, the control part by exp(-k_ctrl dt)
                rng.need(2, (uint32_t)pix, A.sample_base + (uint32_t)s, A.stream_base + (uint32_t)job, A.key0, A.key1);
                const float t0 = r.t;
                r.t = fminf(r.t + tau * __builtin_amdgcn_rcpf(r.khat), r.texit);
                const float kmin = g.kscale * r.kmin + path_kg();
                const float kctrl = kSun == 2 ? kmin : 0.0f;
                float kx = kmin;                // a level-0 voxel is one cell: k is known
                if (r.lev != 0) {
                    kx = g.kscale * g.kc[collision_cell(g, r, r.t)] + path_kg();
                    gathered = true;
                }
                t_sun *= __expf(-kctrl * (r.t - t0)) * fmaxf(0.0f, 1.0f - (kx - kctrl) * __builtin_amdgcn_rcpf(r.khat));
                const float u = rng.take();
                if (t_sun < kSunRoulette) {     // Russian roulette on small estimates
                    if (u * kSunRoulette < t_sun)
                        t_sun = kSunRoulette;
                    else
                        t_sun = 0.0f;
                }
                if (t_sun == 0.0f) {
                    res = kReal;
                    phase = kPhEvent;
                    real = true;
                } else {
                    tau = rng.take_exp1();
                    phase = voxel_phase(r, tau);
                    if (++segs >= A.op.max_segments) {
                        trunc = true;
                        phase = kPhSample;
                    }
                }
            } else if (active) {
                rng.need(2, (uint32_t)pix, A.sample_base + (uint32_t)s, A.stream_base + (uint32_t)job, A.key0, A.key1);
                r.t = fminf(r.t + tau * __builtin_amdgcn_rcpf(r.khat), r.texit);
                const float thr = rng.take() * r.khat;
                if (shadow && thr < g.kscale * r.kmin + path_kg()) {
                    real = true;                // below the voxel's minimum: real without reading k
                } else {
                    if (r.lev == 0) {
                        kc_hit = r.kmin;        // a level-0 voxel is one cell: k is known
                    } else {
                        kc_hit = g.kc[collision_cell(g, r, r.t)];
                            gathered = true;
                    }
                    real = thr < g.kscale * kc_hit + path_kg();
                }
                if (real) {
                    res = kReal;
                    phase = kPhEvent;
                } else {
                    tau = rng.take_exp1();
                    phase = voxel_phase(r, tau);
                    if (++segs >= A.op.max_segments) {
                        trunc = true;
                        phase = kPhSample;
                    }
                }
            }
            if (stats) {
                wave_count(cnt, kCSegments, active);
                wave_count(cnt, kCTentative, active);
                wave_count(cnt, kCReals, real);
                wave_count(cnt, kCNulls, active && !real);
                wave_count(cnt, kCGathers, gathered);
                wave_count(cnt, kCTrunc, trunc);
            }
        } else if (run == kPhEvent) {
            if (phase == kPhEvent) {
                const HGc hg{NC_R(hg.a), NC_R(hg.b), NC_R(hg.c), NC_R(hg.e), NC_R(hg.d), NC_R(hg.r2g)};
                const int max_scatter = NC_R(max_scatter);
                // three numbers cover an event (absorption, then two for the new
                // direction); a guided step takes absorption plus three
                rng.need(kMode == kGuided ? 4 : 3, (uint32_t)pix, A.sample_base + (uint32_t)s,
                         A.stream_base + (uint32_t)job, A.key0, A.key1);
                bool cont = false;               // go on to the scatter / reflect decision
                if (shadow) {
                    if (res == kExit) Lp += beta * w_nee * (kSun != 0 ? t_sun : 1.0f);   // the sun ray got through
                    cont = true;
                } else if (res == kReal) {
                    // volume event: local estimate of the sun, then scatter or absorb
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        pd[a] = r.d[a];
                        r.o[a] = r.o[a] + r.t * r.d[a];
                    }
                    const float kd = g.kscale * kc_hit;
                    kev = kd + path_kg();
                    const float ssa = NC_R(ssa) * kd * __builtin_amdgcn_rcpf(kd + path_kg());
                    float gain = 1.0f;
                    if (kExt && A.op.cone) {
                        // solar disc: the local estimate's direction drawn in its cone
                        const JobView &J = NC_R(jobs)[job];
                        const float s0[3] = {J.sun[0], J.sun[1], J.sun[2]};
                        const float c1 = rng.take(), c2 = rng.take();
                        float w[3];
                        cone_dir(s0, A.op.cone_cos, c1, c2, w);
                        sun[0] = w[0];
                        sun[1] = w[1];
                        sun[2] = w[2];
                        gain = A.op.cone_gain;
                    }
                    const float mu = pd[0] * sun[0] + pd[1] * sun[1] + pd[2] * sun[2];
                    w_nee = ssa * (kExt ? phase_eval(hg, A.op.tab, mu) : hg_phase(hg, mu)) * gain;
                    p_cont = ssa;
                    ground_ev = false;
                    ++order;
                    if (max_scatter >= 0 && order > max_scatter) {
                        phase = kPhSample;
                    } else if (w_nee > 0.0f) {
                        shadow = true;
                        phase = kPhRay;
                    } else {
                        cont = true;
                    }
                } else if (r.d[2] < 0.0f) {
                    // ground hit: Lambertian local estimate
                    const float tg = -r.o[2] * __builtin_amdgcn_rcpf(r.d[2]);
#pragma unroll
                    for (int a = 0; a < 3; ++a) pd[a] = r.d[a];
                    r.o[0] = r.o[0] + tg * r.d[0];
                    r.o[1] = r.o[1] + tg * r.d[1];
                    r.o[2] = 0.0f;
                    const float rho = NC_R(jobs)[job].rho;
                    float gain = 1.0f;
                    if (kExt && A.op.cone) {
                        const JobView &J = NC_R(jobs)[job];
                        const float s0[3] = {J.sun[0], J.sun[1], J.sun[2]};
                        const float c1 = rng.take(), c2 = rng.take();
                        float w[3];
                        cone_dir(s0, A.op.cone_cos, c1, c2, w);
                        sun[0] = w[0];
                        sun[1] = w[1];
                        sun[2] = w[2];
                        gain = A.op.cone_gain;
                    }
                    w_nee = rho * (1.0f / kPi) * sun[2] * gain;   // <= 0 (no sun ray) when the direction is below the horizon
                    p_cont = rho;
                    ground_ev = true;
                    ++order;
                    if (max_scatter >= 0 && order > max_scatter) {
                        phase = kPhSample;
                    } else if (w_nee > 0.0f) {
                        shadow = true;
                        phase = kPhRay;
                    } else {
                        cont = true;
                    }
                } else {
                    // escaped upward: a camera ray that met nothing may look into the solar disc
                    if (kExt && A.op.cone && order == 0 && !ground_ev) {
                        const JobView &J = NC_R(jobs)[job];
                        if (r.d[0] * J.sun[0] + r.d[1] * J.sun[1] + r.d[2] * J.sun[2] >= A.op.cone_cos)
                            Lp += beta * A.op.cone_L;
                    }
                    phase = kPhSample;
                }
                if (cont) {
                    shadow = false;
                    // (the disc's draw may have left too few numbers for the scattering)
                    if (kExt && A.op.cone)
                        rng.need(kMode == kGuided ? 4 : 3, (uint32_t)pix, A.sample_base + (uint32_t)s,
                                 A.stream_base + (uint32_t)job, A.key0, A.key1);
                    if (max_scatter >= 0 && order >= max_scatter) {
                        phase = kPhSample;
                    } else if (rng.take() >= p_cont) {
                        phase = kPhSample;       // absorbed (volume) or not reflected (ground)
                    } else if (kMode == kGuided && !ground_ev &&
                               (A.guide_max_order == 0 || order <= A.guide_max_order)) {
                        phase = kPhGuide;        // the network proposes the new direction (a later trip)
                    } else {
                        const float u1 = rng.take(), u2 = rng.take();
                        const float win[3] = {pd[0], pd[1], pd[2]};
                        if (ground_ev)
                            lambert(pd, u1, u2);
                        else
                            turn(pd, kExt ? phase_sample_mu(hg, A.op.tab, u1) : hg_sample_mu(hg, u1), u2);
                        phase = kPhRay;
                        if (kMode == kCollect && !ground_ev) {
                            // training record: vertex, incoming and outgoing directions, radiance so far
                            const unsigned long long k = atomicAdd(A.col.count, 1ull);
                            if (k < A.col.cap) {
                                float *q = A.col.records + k * kGuideRecord;
#pragma unroll
                                for (int a = 0; a < 3; ++a) {
                                    q[a] = (r.o[a] - g.lo[a]) * A.gpos[a] - 1.0f;
                                    q[3 + a] = win[a];
                                    q[7 + a] = pd[a];
                                }
                                q[6] = __logf(1.0f + kev);
                                q[10] = Lp;
                                q[11] = __uint_as_float((uint32_t)(pix * A.col_spp + s));
                            }
                        }
                    }
                }
            }
        } else if (kMode == kGuided && run == kPhGuide) {
            // ---- guided scattering: network inference on the matrix cores,
            // then the MIS step in the same layout.  The first `best` waiting
            // lanes (by rank) are packed into tiles of 16.
            const bool waiting = phase == kPhGuide;
            const unsigned long long want = __ballot(waiting);
            const int rank = __popcll(want & ((1ull << lane) - 1ull));
            const bool active = waiting && rank < best;
            extern __shared__ __align__(16) float2 s_dyn[];
            char *gb = reinterpret_cast<char *>(s_dyn) + A.guide_lds;
            const short *wl = reinterpret_cast<const short *>(gb);
            const float *bl = reinterpret_cast<const float *>(gb + kWOff[4] * 2);
            char *wt = gb + kGuideWeightBytes + (threadIdx.x >> 6) * kGuideScratchPerWave;
            short *tin = reinterpret_cast<short *>(wt);
            float *tf = reinterpret_cast<float *>(wt + kGuideInBytes);
            const int ntiles = (best + 15) >> 4;
            const int row = rank & 15, col = lane & 15, kq = lane >> 4;
            for (int t = 0; t < ntiles; ++t) {
                const bool owner = active && (rank >> 4) == t;
                if (owner) {
                    float x[7];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        x[a] = (r.o[a] - g.lo[a]) * A.gpos[a] - 1.0f;
                        x[3 + a] = pd[a];
                    }
                    x[6] = __logf(1.0f + kev);
                    put_guide_inputs(tin + row * 16, x);
                    // the event trip left three numbers for this step
                    float *f = tf + row * 8;
                    const float u_sel = rng.take();
                    f[0] = pd[0];
                    f[1] = pd[1];
                    f[2] = pd[2];
                    f[3] = u_sel;
                    f[4] = lobe_uniform(u_sel, A.guide_frac);
                    f[5] = rng.take();   // u1
                    f[6] = rng.take();   // u2
                }
                wave_sync();
                float z[12];
                guide_tile_forward(wl, bl, tin, lane, z);
                const GuidedStep st = guided_turn_tile<kExt>(z, tf + col * 8, A.guide_frac,
                                                                HGc{NC_R(hg.a), NC_R(hg.b), NC_R(hg.c), NC_R(hg.e),
                                                                    NC_R(hg.d), NC_R(hg.r2g)},
                                                                A.op.tab, kq);
                // each owner takes its column's result
                const int src = owner ? row : lane;
                const float d0 = __shfl(st.d[0], src), d1 = __shfl(st.d[1], src), d2 = __shfl(st.d[2], src);
                const float wf = __shfl(st.w, src);
                if (owner) {
                    pd[0] = d0;
                    pd[1] = d1;
                    pd[2] = d2;
                    beta *= wf;
                    phase = kPhRay;
                }
                wave_sync();
            }
        } else {
            // ---- finish the lane's path, then start its next sample or item
            bool need_item = false;
            if (phase == kPhSample) {
                if (have_item) {
                    if (traced) {
                        if (kMode == kCollect) A.col.final_L[(size_t)pix * A.col_spp + s] = Lp;
                        acc += Lp;
                        acc2 += Lp * Lp;
                        ++s;
                    }
                    if (s >= s_end) {
                        const unsigned long long q = NC_R(jobs)[job].out_off + (unsigned long long)pix;
                        const double S = (double)NC_R(jobs)[job].S;   // radiances are in units of the sun irradiance
                        unsafeAtomicAdd(NC_R(sum) + q, S * (double)acc);
                        unsafeAtomicAdd(NC_R(sumsq) + q, S * S * (double)acc2);
                        have_item = false;
                        need_item = true;
                    }
                } else {
                    need_item = true;
                }
            }
            const bool finished = phase == kPhSample && traced;
            if (stats) wave_count(cnt, kCPaths, finished);
            if (phase == kPhSample) traced = false;   // only lanes in this phase: others are mid-path
            // queue refill in uniform control flow: ballot + prefix count over
            // the wave's chunk, one global atomic per kChunk items
            const unsigned long long need = __ballot(need_item);
            if (need) {
                const int n_need = __popcll(need);
                const int rank = (int)lanes_below(need);
                const int take_new = n_need - chunk_left;
                unsigned long long nb = NC_SET_HI();
                if (take_new > 0 && !queue_done) {
                    const int leader = __ffsll((unsigned long long)need) - 1;
                    if (lane == leader) {
                        // workgroups are dealt to the 8 XCDs in turn (blockIdx mod 8);
                        // queue q holds the q-th eighth of the set's items, so each XCD's
                        // L2 serves its own band of the image; a drained queue sends the
                        // wave on to the next one
                        for (;;) {
                            const int q = (int)((blockIdx.x + (unsigned)q_seen) & 7u);
                            const unsigned long long lo = NC_SET_LO() + (unsigned long long)q * NC_SET_SPAN();
                            const unsigned long long hi = lo + NC_SET_SPAN() < NC_SET_HI() ? lo + NC_SET_SPAN() : NC_SET_HI();
                            const unsigned long long b = lo + atomicAdd(NC_SET_QUEUE() + 16 * q, (unsigned long long)kChunk);
                            if (b < hi) { nb = b; break; }
                            if (++q_seen == 8) { nb = NC_SET_HI(); break; }
                        }
                    }
                    nb = __shfl(nb, leader);
                    q_seen = __shfl(q_seen, leader);
                    if (nb >= NC_SET_HI()) queue_done = true;
                }
                if (need_item) {
                    const unsigned long long w = rank < chunk_left ? chunk_base + (unsigned long long)rank
                                                                   : nb + (unsigned long long)(rank - chunk_left);
                    if (w >= NC_SET_HI()) {
                        phase = kPhIdle;
                    } else {
                        // the job holding item w: last job whose first item is <= w
                        int lo = 0, hi = NC_R(n_jobs) - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (NC_R(jobs)[mid].item_begin <= w)
                                lo = mid;
                            else
                                hi = mid - 1;
                        }
                        job = lo;
                        const JobView &J = NC_R(jobs)[job];
                        const int tx = J.tiles_x, spi = NC_R(spi), spp = NC_R(spp);
                        const int W = J.cam.W, H = J.cam.H;
                        // a job has fewer than 2^32 items (checked at launch): 32-bit divisions
                        const uint32_t lw = (uint32_t)(w - J.item_begin);
                        // items run tile by tile, each tile's sample blocks together: the
                        // waves in flight share a narrow band of the image, so their paths
                        // share the caches (sample block major: 6 % slower on the cumulus view)
                        const uint32_t nblk = (uint32_t)((spp + spi - 1) / spi);
                        const uint32_t per_tile = nblk * 64u;
                        const uint32_t tile_u = lw / per_tile;
                        const int tile = (int)tile_u;
                        const int rem = (int)(lw - tile_u * per_tile);
                        const int blk = rem >> 6, within = rem & 63;
                        const int trow = (int)((uint32_t)tile / (uint32_t)tx);
                        const int px = (tile - trow * tx) * 8 + (within & 7);
                        const int py = trow * 8 + (within >> 3);
                        s = blk * spi;
                        s_end = min(s + spi, spp);
                        if (px < W && py < H && s < s_end) {
                            pix = py * W + px;
                            acc = 0.0f;
                            acc2 = 0.0f;
                            have_item = true;
                        }
                    }
                }
                if (take_new > 0) {
                    chunk_base = nb + (unsigned long long)take_new;
                    chunk_left = kChunk - take_new;
                } else {
                    chunk_base += (unsigned long long)n_need;
                    chunk_left -= n_need;
                }
            }
            if (phase == kPhSample && have_item) {
                rng.reset();
                const JobView &J = NC_R(jobs)[job];
                const int W = J.cam.W;
                const int py = pix / W, px = pix - py * W;
                rng.need(kExt && A.op.kd_n ? 3 : 2, (uint32_t)pix, A.sample_base + (uint32_t)s, A.stream_base + (uint32_t)job, A.key0,
                         A.key1);
                if (kExt && A.op.kd_n) {
                    // spectral integration: the path's quadrature point (Section 4.1)
                    // (unrolled over the table, so that its entries stay scalar kernel arguments)
                    const float uk = rng.take();
                    kg = A.op.kd_k[0];
#pragma unroll
                    for (int q = 1; q < NC_KDIST_MAX; ++q)
                        if (q < A.op.kd_n && uk >= A.op.kd_cdf[q - 1]) kg = A.op.kd_k[q];
                }
                const float u1 = rng.take(), u2 = rng.take();
                float o[3];
                camera_ray_v(J.cam, px, py, u1, u2, o, pd);
                sun[0] = J.sun[0];
                sun[1] = J.sun[1];
                sun[2] = J.sun[2];
                ground_ev = false;
#pragma unroll
                for (int a = 0; a < 3; ++a) r.o[a] = o[a];
                Lp = 0.0f;
                beta = 1.0f;
                order = 0;
                segs = 0;
                shadow = false;
                traced = true;
                phase = kPhRay;
                if (J.cam.type == 2) {
                    // irradiance sensor: first the sun's direct beam (a sun ray of
                    // weight 1), then, as after a ground reflection that always
                    // happens, a cosine-distributed upward path of weight pi / mu_sun
                    beta = kPi / sun[2];
                    float gain = 1.0f;
                    if (kExt && A.op.cone) {
                        // the direct beam along a direction drawn in the disc's cone
                        const float s0[3] = {sun[0], sun[1], sun[2]};
                        rng.need(2, (uint32_t)pix, A.sample_base + (uint32_t)s, A.stream_base + (uint32_t)job, A.key0,
                                 A.key1);
                        const float c1 = rng.take(), c2 = rng.take();
                        float w[3];
                        cone_dir(s0, A.op.cone_cos, c1, c2, w);
                        sun[0] = w[0];
                        sun[1] = w[1];
                        sun[2] = w[2];
                        gain = A.op.cone_gain;
                    }
                    w_nee = sun[2] * (1.0f / kPi) * gain;
                    p_cont = 1.0f;
                    ground_ev = true;
                    shadow = true;
                }
            }
        }
        if (stats && lane == 0) atomicAdd(s_cnt + kCCycles0 + run, (unsigned long long)(wall_clock64() - t_trip));
    }
    if (!kSets || A.n_sets == 1) break;
    // every lane of this wave is idle: once all waves of the workgroup are, serve
    // a queue set (network) that still has work, if any
    tried |= 1u << cur;
    __syncthreads();
    if (threadIdx.x == 0) {
        int nxt = -1;
        for (int k = 0; k < A.n_sets && nxt < 0; ++k) {
            if ((tried >> k) & 1u) continue;
            const unsigned long long lo = NC_R(set_begin[k]), hi = NC_R(set_begin[k + 1]), span = NC_R(set_span[k]);
            for (int q = 0; q < 8; ++q) {
                const unsigned long long qlo = lo + (unsigned long long)q * span;
                if (qlo >= hi) break;
                const unsigned long long head =
                    __hip_atomic_load(NC_R(queue) + 128 * k + 16 * q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (qlo + head < hi) { nxt = k; break; }
            }
        }
        s_next_set = nxt;
    }
    __syncthreads();
    const int nxt = __builtin_amdgcn_readfirstlane(s_next_set);   // workgroup-uniform
    if (nxt < 0) break;
    cur = nxt;
    {
        char *gb = reinterpret_cast<char *>(s_nodes) + A.guide_lds;
        const GuideWeights W = A.rare->gw[cur];
        stage_guide(W, reinterpret_cast<short *>(gb), reinterpret_cast<float *>(gb + kWOff[4] * 2));
    }
    __syncthreads();
    phase = kPhSample;
    have_item = false;
    traced = false;
    chunk_left = 0;
    queue_done = false;
    q_seen = 0;
    guide_wait = 0;
    }   // queue sets
#undef NC_SET_LO
#undef NC_SET_HI
#undef NC_SET_SPAN
#undef NC_SET_QUEUE
#undef NC_R
    // the block's counters to global memory
    __syncthreads();
    if (A.counters && threadIdx.x == 0) {
        unsigned long long *o = reinterpret_cast<unsigned long long *>(A.counters);
        const unsigned long long v[10] = {s_cnt[kCPaths], s_cnt[kCSegments], s_cnt[kCTentative], s_cnt[kCNulls],
                                          s_cnt[kCReals], s_cnt[kCLeaf], s_cnt[kCGathers],
                                          s_cnt[kCReads], s_cnt[kCNee], s_cnt[kCTrunc]};
        for (int k = 0; k < 10; ++k)
            if (v[k]) atomicAdd(o + k, v[k]);
        unsigned long long *sch = reinterpret_cast<unsigned long long *>(A.counters->sched);
        for (int k = 0; k < 18; ++k)
            if (s_cnt[kCTrips0 + k]) atomicAdd(sch + k, s_cnt[kCTrips0 + k]);
        if (s_cnt[kCDeep]) atomicAdd(sch + 18, s_cnt[kCDeep]);
    }
}

__global__ void zero_u64_kernel(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void collect_finish_kernel(CollectView cv)
{
    const unsigned long long n = *cv.count < cv.cap ? *cv.count : cv.cap;
    for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x) {
        float *q = cv.records + i * kGuideRecord;
        const uint32_t slot = __float_as_uint(q[11]);
        // radiance the path gathered after this vertex: its final value minus what it held here
        q[10] = fmaxf(cv.final_L[slot] - q[10], 0.0f);
    }
}

hipError_t launch_collect_finish(const nc_ctx *ctx, const CollectView &cv)
{
    hipLaunchKernelGGL(collect_finish_kernel, dim3(512), dim3(256), 0, ctx->stream, cv);
    return hipGetLastError();
}

hipError_t launch_render(const nc_ctx *ctx, const nc_grid *g, const float *d_kc, const OptView &op,
                         const JobView *jobs_host, int n_jobs, const nc_sampling &s, double *sum, double *sumsq,
                         nc_counters *counters, const RenderScratch &scr, const nc_guide *const *guides,
                         const CollectView *collect)
{
    const int mode = guides ? kGuided : collect ? kCollect : kPlain;
    const int block0 = ctx->launch.block > 0 ? std::max(64, std::min(256, (ctx->launch.block / 64) * 64)) : 256;
    const size_t guide_bytes =
        mode == kGuided ? (size_t)kGuideWeightBytes + (size_t)(block0 / 64) * kGuideScratchPerWave : 0;
    Shape sh = choose_shape(ctx, g, 256, guide_bytes, 0);
    RenderRare rare;
    rare.seed = s.seed;
    rare.sample_offset = s.sample_offset;
    rare.spp = s.spp;
    rare.spi = std::max(1, std::min(sh.spi, s.spp));
    {
        // the kernel decodes a job's items in 32 bits: take more samples per
        // item when a job would otherwise have 2^32 items or more
        unsigned long long tiles64 = 0;
        for (int j = 0; j < n_jobs; ++j)
            tiles64 = std::max(tiles64, (unsigned long long)((jobs_host[j].cam.W + 7) / 8) *
                                            (unsigned long long)((jobs_host[j].cam.H + 7) / 8) * 64ull);
        const unsigned long long max_blocks = 0xffffffffull / std::max(tiles64, 1ull);
        if ((unsigned long long)((s.spp + rare.spi - 1) / rare.spi) > max_blocks)
            rare.spi = (int)std::min<unsigned long long>((unsigned long long)s.spp,
                                                         ((unsigned long long)s.spp + max_blocks - 1) / max_blocks);
    }
    rare.sum = sum;
    rare.sumsq = sumsq;
    rare.jobs = scr.jobs;
    rare.n_jobs = n_jobs;
    rare.stream_base = s.stream;
    const unsigned long long blocks = (unsigned long long)((s.spp + rare.spi - 1) / rare.spi);
    // queue items of each job: tiles of 8x8 pixels times sample blocks
    std::vector<JobView> jobs(jobs_host, jobs_host + n_jobs);
    unsigned long long items = 0;
    for (int j = 0; j < n_jobs; ++j) {
        jobs[j].tiles_x = (jobs[j].cam.W + 7) / 8;
        jobs[j].tiles_y = (jobs[j].cam.H + 7) / 8;
        jobs[j].item_begin = items;
        items += (unsigned long long)jobs[j].tiles_x * jobs[j].tiles_y * 64ull * blocks;   // < 2^32 per job
    }
    // queue sets: one per run of consecutive jobs sharing a guide (one set otherwise)
    int n_sets = 0;
    int set_first_job[kMaxQueueSets + 1];
    for (int j = 0; j < n_jobs; ++j) {
        if (j == 0 || (guides && guides[j] != guides[j - 1])) {
            if (n_sets == kMaxQueueSets || n_sets >= scr.max_sets) return hipErrorInvalidValue;
            set_first_job[n_sets++] = j;
        }
    }
    set_first_job[n_sets] = n_jobs;
    RenderArgs A;
    A.g = grid_view(g, d_kc);
    A.op = op;
    A.rare = reinterpret_cast<const RenderRare *>(scr.rare);
    A.key0 = (uint32_t)s.seed;
    A.key1 = (uint32_t)(s.seed >> 32);
    A.sample_base = (uint32_t)s.sample_offset;
    A.stream_base = s.stream;
    A.counters = counters;
    rare.queue = scr.queue;
    A.n_sets = n_sets;
    for (int k = 0; k <= n_sets; ++k)
        rare.set_begin[k] = set_first_job[k] < n_jobs ? jobs[set_first_job[k]].item_begin : items;
    for (int k = 0; k < n_sets; ++k) {
        const unsigned long long n = rare.set_begin[k + 1] - rare.set_begin[k];
        rare.set_span[k] = ((n + 8 * kChunk - 1) / (8 * kChunk)) * kChunk;
        rare.set_group[k] = 0;
    }
    A.lds_first = sh.lds_first;
    A.lds_nodes = sh.lds_nodes;
    const size_t node_bytes = ((size_t)sh.lds_nodes * sizeof(float2) + 15) & ~(size_t)15;
    A.guide_lds = (int)node_bytes;
    for (int a = 0; a < 3; ++a) A.gpos[a] = (float)(2.0 / ((double)g->n[a] * g->h[a]));
    A.guide_frac = s.guide_frac;
    A.guide_max_order = (int)std::min<uint32_t>(s.guide_max_order, 1u << 30);
    A.col_spp = s.spp;
    for (int k = 0; k < kMaxQueueSets; ++k) rare.gw[k] = GuideWeights{};
    A.col = CollectView{};
    if (guides)
        for (int k = 0; k < n_sets; ++k) rare.gw[k] = guide_weights(guides[set_first_job[k]]);
    A.gw = rare.gw[0];
    if (collect) A.col = *collect;
    rare.hg = op.hg;
    rare.ssa = op.ssa;
    rare.max_scatter = op.max_scatter;
    static_assert(sizeof(RenderRare) <= kRareBytes &&
                      kRareBytes <= (kScratchErr - kScratchRare) * sizeof(unsigned long long),
                  "scratch too small for the renderer parameters");
    // register budget: waves per SIMD the kernel is compiled for (3..6)
    // (default 4, a cap of 128 registers: the plain and collection kernels
    // take 80-95, so the occupancy query then gives them 5-6 waves per SIMD;
    // the guided ones fill the 128 with a few spilled)
    const int wpe = ctx->launch.waves_per_cu > 0 ? std::max(3, std::min(6, ctx->launch.waves_per_cu / 4)) : 4;
    // kernel variant: mode, sun-ray estimator, register budget (waves per SIMD)
    const int est = s.flags & NC_SUN_ESTIMATOR_MASK;
    const void *fn = nullptr;
    if (op.kd_n > 0 || op.tab.n > 0 || op.cone) {
        // the extended medium (k-distribution, phase table, solar disc): its own kernel variants
        if (mode == kGuided && n_sets > 1)
            fn = est == 0 ? (const void *)render_kernel<4, kGuided, 0, true, true>
                 : est == 1 ? (const void *)render_kernel<4, kGuided, 1, true, true>
                            : (const void *)render_kernel<4, kGuided, 2, true, true>;
        else if (mode == kGuided)
            fn = est == 0 ? (const void *)render_kernel<4, kGuided, 0, true>
                 : est == 1 ? (const void *)render_kernel<4, kGuided, 1, true>
                            : (const void *)render_kernel<4, kGuided, 2, true>;
        else if (mode == kCollect)
            fn = est == 0 ? (const void *)render_kernel<4, kCollect, 0, true>
                 : est == 1 ? (const void *)render_kernel<4, kCollect, 1, true>
                            : (const void *)render_kernel<4, kCollect, 2, true>;
        else
            fn = est == 0 ? (const void *)render_kernel<4, kPlain, 0, true>
                 : est == 1 ? (const void *)render_kernel<4, kPlain, 1, true>
                            : (const void *)render_kernel<4, kPlain, 2, true>;
    } else if (mode == kGuided && n_sets > 1) {
        fn = est == 0 ? (const void *)render_kernel<4, kGuided, 0, false, true>
             : est == 1 ? (const void *)render_kernel<4, kGuided, 1, false, true>
                        : (const void *)render_kernel<4, kGuided, 2, false, true>;
    } else if (mode == kGuided) {
        fn = est == 0 ? (const void *)render_kernel<4, kGuided, 0, false>
             : est == 1 ? (const void *)render_kernel<4, kGuided, 1, false>
                        : (const void *)render_kernel<4, kGuided, 2, false>;
    } else if (mode == kCollect) {
        fn = est == 0 ? (const void *)render_kernel<4, kCollect, 0, false>
             : est == 1 ? (const void *)render_kernel<4, kCollect, 1, false>
                        : (const void *)render_kernel<4, kCollect, 2, false>;
    } else if (est == 0) {
        fn = wpe == 3   ? (const void *)render_kernel<3, kPlain, 0, false>
             : wpe == 4 ? (const void *)render_kernel<4, kPlain, 0, false>
             : wpe == 5 ? (const void *)render_kernel<5, kPlain, 0, false>
                        : (const void *)render_kernel<6, kPlain, 0, false>;
    } else if (est == 1) {
        fn = wpe == 3 ? (const void *)render_kernel<3, kPlain, 1, false> : (const void *)render_kernel<4, kPlain, 1, false>;
    } else {
        fn = wpe == 3 ? (const void *)render_kernel<3, kPlain, 2, false> : (const void *)render_kernel<4, kPlain, 2, false>;
    }
    int resident = 0;
    const size_t lds = node_bytes + guide_bytes;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, fn, sh.block, lds) == hipSuccess && resident > 0)
        sh.wgs = ctx->num_cus * resident;
    const long long max_wgs = (long long)((items + sh.block - 1) / sh.block);
    const int wgs = (int)std::max<long long>(1, std::min<long long>(max_wgs, sh.wgs));
    if (n_sets > 1) {
        // each set's first workgroups: groups of 8 (one per XCD) in proportion
        // to its items, at least one group each when there are enough
        const long long groups = std::max<long long>(1, (wgs + 7) / 8);
        long long acc = 0;
        for (int k = 0; k < n_sets; ++k) {
            rare.set_group[k] = (int)std::min<long long>(groups - 1, std::max<long long>(
                k == 0 ? 0 : rare.set_group[k - 1] + (groups >= n_sets ? 1 : 0),
                (long long)((double)acc / (double)std::max(items, 1ull) * (double)groups)));
            acc += rare.set_begin[k + 1] - rare.set_begin[k];
        }
    }
    hipError_t e = hipMemcpyAsync(scr.jobs, jobs.data(), sizeof(JobView) * (size_t)n_jobs, hipMemcpyHostToDevice,
                                  ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(scr.rare, &rare, sizeof(rare), hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(2 * n_sets), dim3(64), 0, ctx->stream, scr.queue, 128 * n_sets);
    if (collect) hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, ctx->stream, collect->count, 1);
    void *args[] = {&A};
    return hipLaunchKernel(fn, dim3(wgs), dim3(sh.block), args, lds, ctx->stream);
}

// Error of an image estimate over b x b pixel blocks (b = 1: per pixel):
// acc[0] += block mean radiance, acc[1] += squared standard error of the
// block mean, acc[2] += 1 per block.  A ragged edge block averages the
// pixels it has.
__global__ void image_err_kernel(const double *sum, const double *sumsq, int W, int H, int n, int b, double *acc)
{
    const int bw = (W + b - 1) / b, bh = (H + b - 1) / b;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double m = 0.0, e = 0.0, c = 0.0;
    if (i < bw * bh) {
        const int bx = i % bw, by = i / bw;
        const int x1 = min(W, (bx + 1) * b), y1 = min(H, (by + 1) * b);
        int cnt = 0;
        for (int y = by * b; y < y1; ++y)
            for (int x = bx * b; x < x1; ++x) {
                const double mp = sum[(size_t)y * W + x] / n;
                const double var = fmax(sumsq[(size_t)y * W + x] / n - mp * mp, 0.0) * n / (n > 1 ? n - 1 : 1);
                m += mp;
                e += var / n;
                ++cnt;
            }
        m /= cnt;
        e /= (double)cnt * cnt;
        c = 1.0;
    }
    for (int off = 32; off > 0; off >>= 1) {
        m += __shfl_xor(m, off);
        e += __shfl_xor(e, off);
        c += __shfl_xor(c, off);
    }
    if (__lane_id() == 0 && c > 0.0) {
        atomicAdd(acc, m);
        atomicAdd(acc + 1, e);
        atomicAdd(acc + 2, c);
    }
}

hipError_t launch_image_err(const nc_ctx *ctx, const double *sum, const double *sumsq, int W, int H, int n, int b,
                            double *out3)
{
    double *acc = reinterpret_cast<double *>(ctx->d_scratch + kScratchErr);
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, ctx->stream,
                       reinterpret_cast<unsigned long long *>(acc), 3);
    const int units = ((W + b - 1) / b) * ((H + b - 1) / b);
    hipLaunchKernelGGL(image_err_kernel, dim3((units + 255) / 256), dim3(256), 0, ctx->stream, sum, sumsq, W, H, n, b,
                       acc);
    hipError_t e = hipMemcpyAsync(out3, acc, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    return e;
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
        v.hi[a] = (float)g->n[a] * v.h[a] + v.lo[a];   // float arithmetic, no contraction: as face_t rounds it
    }
    v.L = g->L;
    v.k_gas = (float)g->params.k_gas;
    v.kscale = 1.0f;
    v.kc = d_kc;
    v.nodes = g->d_nodes;
    v.off = g->d_off;
    v.mask = g->d_mask;
    return v;
}

Shape choose_shape(const nc_ctx *ctx, const nc_grid *g, int block_default, size_t reserve, int waves_default)
{
    Shape sh;
    sh.block = ctx->launch.block > 0 ? ctx->launch.block : block_default;
    sh.block = std::max(64, std::min(256, (sh.block / 64) * 64));
    const int waves = ctx->launch.waves_per_cu > 0 ? ctx->launch.waves_per_cu : waves_default > 0 ? waves_default : 16;
    sh.wgs = std::max(1, ctx->num_cus * waves / (sh.block / 64));
    // one sample per queue item: the lanes of a wave trace neighbouring pixels
    // of an 8x8 tile at the same sample index, and a lane's next item is its
    // next pixel (6 % faster than 4 samples a pixel on the cumulus view)
    sh.spi = ctx->launch.samples_per_item > 0 ? ctx->launch.samples_per_item : 1;
    // LDS staging of the top levels: as many whole levels as fit the budget
    const size_t wgs_per_cu = std::max(1, waves / (sh.block / 64));
    const size_t cap = std::min<size_t>(ctx->lds_per_cu / wgs_per_cu, 60 * 1024);
    const size_t budget = cap > 1024 + reserve ? cap - 1024 - reserve : 0;
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
