// nc_flux.hip -- forward photons: ground transmissivity under the field and
// its parametric sensitivities (Section 5.1), with the derivative-path
// (adjoint) replay.
//
// The sun lights the top of the box uniformly; photons start at a uniform
// point of the top face going along -omega_sun, are tracked by delta
// tracking in the grid's piecewise-constant majorant with analog absorption
// and HG scattering, and arrive at the ground, where an arrival inside the
// box's footprint is tallied in its ground pixel before a Lambertian
// reflection (probability rho) or absorption.
//
// Sensitivities follow the derivative of the integral formulation (Eq. 3):
// with k = s k_c + k_g and a majorant held fixed, every tentative collision
// multiplies the path density by k/k_hat (real) or 1 - k/k_hat (null), so a
// path carries the score
//   sigma_s = sum_real k_c/k - sum_null k_c/(k_hat - k) + sum_scatter k_g/(s k)
// (the last term is d ln ssa(x)/ds), every HG scattering of cosine mu adds
//   sigma_g += d ln p(mu)/dg = -2g/(1-g^2) - 3(g-mu)/(1+g^2-2g mu),
// and every scattering adds d ln ssa(x)/d alpha = -1/(1 - alpha) to the
// score of the droplets' absorptivity alpha = 1 - ssa (the sensitivity the
// paper computes in Section 5.1).  Absorbed photons arrive nowhere, so the
// absorption events need no term.
// The derivative of a tally is the mean of (tally) x sigma.  The adjoint
// replay re-runs the same photons (same counter-based random numbers) and
// accumulates grad[pixel] x sigma at each arrival.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "nc_internal.hpp"

namespace nc {

struct FluxArgs {
    GridView g;
    OptView op;
    int px_nx, px_ny;
    float x0, y0, Lx, Ly, ztop;
    unsigned long long n_photons;
    uint64_t seed, offset;
    double *tally;          // [9][px_ny][px_nx] (forward) or NULL
    double *glob;           // [4] (forward) or NULL
    const double *grad;     // [px_ny][px_nx] (adjoint) or NULL
    double *out;            // [3] (adjoint) or NULL
    double norm;            // factor of every arrival: 1, or px_nx px_ny / n_photons (normalised output)
    nc_counters *counters;
    int lds_first, lds_nodes;
};

__device__ inline float hg_dlng(float g, float mu)
{
    return -2.0f * g / (1.0f - g * g) - 3.0f * (g - mu) / (1.0f + g * g - 2.0f * g * mu);
}

// A delta-tracking step that also accumulates the scale score.
__device__ inline int track_step_scored(const GridView &g, const NodeSrc &ns, Ray &r, float &tau, Rng &rng,
                                        float mscale, float &kc_hit, float &sig_s, Counters &cnt)
{
    ++cnt.segments;
    const float ktau = r.khat * (r.texit - r.t);
    if (r.khat > 0.0f && tau < ktau) {
        r.t = fminf(r.t + tau / r.khat, r.texit);
        ++cnt.tentative;
        const float thr = rng.u01() * r.khat;
        if (r.lev == 0) {
            kc_hit = r.kmin;
        } else {
            kc_hit = g.kc[collision_cell(g, r, r.t)];
            ++cnt.gathers;
        }
        const float k = g.kscale * kc_hit + g.k_gas;
        if (thr < k) {
            sig_s += kc_hit / k;
            ++cnt.reals;
            return kReal;
        }
        sig_s -= kc_hit / (r.khat - k);
        ++cnt.nulls;
        tau = rng.exp1();
        return kContinue;
    }
    tau -= ktau;
    if (!next_leaf(g, ns, r, mscale, cnt.node_reads)) return kExit;
    ++cnt.leaf_visits;
    return kContinue;
}

template <bool kAdjoint>
__global__ __launch_bounds__(256) void flux_kernel(FluxArgs A)
{
    extern __shared__ float2 s_nodes[];
    __shared__ int s_off[NC_MAX_LEVELS + 2];
    stage_levels(A.g, A.lds_first, A.lds_nodes, s_nodes, s_off);
    const GridView &g = A.g;
    const NodeSrc ns{g.nodes, s_nodes, s_off, A.lds_first, s_off[A.lds_first <= g.L ? A.lds_first : 0], g.n[0],
                     g.n[1]};
    const float sun[3] = {A.op.sun[0], A.op.sun[1], A.op.sun[2]};
    const size_t np = (size_t)A.px_nx * A.px_ny;
    Counters cnt = {};
    uint32_t up = 0, gin = 0, gout = 0, vabs = 0;
    double adj_s = 0.0, adj_g = 0.0, adj_a = 0.0;
    const float dln_alpha = A.op.ssa > 0.0f ? -1.0f / A.op.ssa : 0.0f;

    for (unsigned long long p = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; p < A.n_photons;
         p += (unsigned long long)gridDim.x * blockDim.x) {
        const unsigned long long id = A.offset + p;
        Rng rng;
        rng.init((uint32_t)id, (uint32_t)(id >> 32), 2u, A.seed);
        float o[3] = {A.x0 + rng.u01() * A.Lx, A.y0 + rng.u01() * A.Ly, A.ztop};
        float d[3] = {-sun[0], -sun[1], -sun[2]};
        float sig_s = 0.0f, sig_g = 0.0f, sig_a = 0.0f;
        bool scattered = false;
        int segs = 0;
        Ray r;
        start_ray(g, ns, r, o, d, A.op.mscale, cnt);
        float tau = rng.exp1();
        for (;;) {
            float kc_hit = 0.0f;
            const int res = track_step_scored(g, ns, r, tau, rng, A.op.mscale, kc_hit, sig_s, cnt);
            if (++segs >= A.op.max_segments && res == kContinue) {
                ++cnt.truncated;
                break;
            }
            if (res == kContinue) continue;
            if (res == kReal) {
                float x[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) x[a] = r.o[a] + r.t * r.d[a];
                const float kd = g.kscale * kc_hit;
                const float k = kd + g.k_gas;
                const float ssa = A.op.ssa * kd / k;
                if (rng.u01() >= ssa) {
                    ++vabs;
                    break;
                }
                if (g.k_gas > 0.0f) sig_s += g.k_gas / (g.kscale * k);
                sig_a += dln_alpha;
                const float mu = hg_sample_mu(A.op.hg, rng.u01());
                sig_g += hg_dlng(A.op.g, mu);
                float nd[3] = {r.d[0], r.d[1], r.d[2]};
                turn(nd, mu, rng.u01());
                const VoxelCache vc = voxel_of(r);
                start_ray_cached(g, ns, r, x, nd, vc, A.op.mscale, cnt);
                tau = rng.exp1();
                scattered = true;
            } else if (r.d[2] < 0.0f) {
                const float tg = -r.o[2] / r.d[2];
                float x[3] = {r.o[0] + tg * r.d[0], r.o[1] + tg * r.d[1], 0.0f};
                const float fx = (x[0] - A.x0) / A.Lx, fy = (x[1] - A.y0) / A.Ly;
                const bool inside = fx >= 0.0f && fx < 1.0f && fy >= 0.0f && fy < 1.0f;
                if (inside) {
                    const int i = min((int)(fx * (float)A.px_nx), A.px_nx - 1);
                    const int j = min((int)(fy * (float)A.px_ny), A.px_ny - 1);
                    const size_t q = (size_t)j * A.px_nx + i;
                    if (kAdjoint) {
                        const double w = A.grad[q] * A.norm;
                        adj_s += w * (double)sig_s;
                        adj_g += w * (double)sig_g;
                        adj_a += w * (double)sig_a;
                    } else {
                        const double f = A.norm, f2 = f * f;
                        unsafeAtomicAdd(A.tally + q, f);
                        unsafeAtomicAdd(A.tally + np + q, f2);
                        if (!scattered) unsafeAtomicAdd(A.tally + 2 * np + q, f);
                        unsafeAtomicAdd(A.tally + 3 * np + q, f * (double)sig_s);
                        unsafeAtomicAdd(A.tally + 4 * np + q, f2 * (double)sig_s * (double)sig_s);
                        unsafeAtomicAdd(A.tally + 5 * np + q, f * (double)sig_g);
                        unsafeAtomicAdd(A.tally + 6 * np + q, f2 * (double)sig_g * (double)sig_g);
                        unsafeAtomicAdd(A.tally + 7 * np + q, f * (double)sig_a);
                        unsafeAtomicAdd(A.tally + 8 * np + q, f2 * (double)sig_a * (double)sig_a);
                    }
                }
                if (rng.u01() >= A.op.rho) {
                    if (inside) ++gin; else ++gout;
                    break;
                }
                float nd[3];
                const float u1 = rng.u01(), u2 = rng.u01();
                lambert(nd, u1, u2);
                start_ray(g, ns, r, x, nd, A.op.mscale, cnt);
                tau = rng.exp1();
                scattered = true;
            } else {
                ++up;
                break;
            }
        }
        ++cnt.paths;
    }
    flush_counters(cnt, A.counters);
    if (kAdjoint) {
        double s = adj_s, t = adj_g, u = adj_a;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            s += __shfl_xor(s, off);
            t += __shfl_xor(t, off);
            u += __shfl_xor(u, off);
        }
        if (__lane_id() == 0) {
            unsafeAtomicAdd(A.out, s);
            unsafeAtomicAdd(A.out + 1, t);
            unsafeAtomicAdd(A.out + 2, u);
        }
    } else {
        const unsigned long long a = wave_sum(up), b = wave_sum(gin), c = wave_sum(gout), e = wave_sum(vabs);
        if (__lane_id() == 0) {
            if (a) unsafeAtomicAdd(A.glob, (double)a);
            if (b) unsafeAtomicAdd(A.glob + 1, (double)b);
            if (c) unsafeAtomicAdd(A.glob + 2, (double)c);
            if (e) unsafeAtomicAdd(A.glob + 3, (double)e);
        }
    }
}

hipError_t launch_flux(const nc_ctx *ctx, const nc_grid *g, const float *d_kc, const OptView &op, float kscale,
                       int px_nx, int px_ny, unsigned long long n_photons, const nc_sampling &s, double *tally,
                       double *glob, const double *grad, double *out, nc_counters *counters)
{
    Shape sh = choose_shape(ctx, g, 256);
    FluxArgs A;
    A.g = grid_view(g, d_kc);
    A.g.kscale = kscale;
    A.op = op;
    A.px_nx = px_nx;
    A.px_ny = px_ny;
    A.x0 = (float)g->lo[0];
    A.y0 = (float)g->lo[1];
    A.Lx = (float)(g->n[0] * g->h[0]);
    A.Ly = (float)(g->n[1] * g->h[1]);
    A.ztop = (float)(g->lo[2] + g->n[2] * g->h[2]);
    A.n_photons = n_photons;
    A.seed = s.seed;
    A.offset = s.sample_offset;
    A.tally = tally;
    A.glob = glob;
    A.grad = grad;
    A.out = out;
    A.norm = (s.flags & NC_FLUX_NORMALISE) ? (double)px_nx * (double)px_ny / (double)n_photons : 1.0;
    A.counters = counters;
    A.lds_first = sh.lds_first;
    A.lds_nodes = sh.lds_nodes;
    const size_t lds = (size_t)sh.lds_nodes * sizeof(float2);
    const unsigned long long blocks = (n_photons + 255) / 256;
    const int wgs = (int)std::max<unsigned long long>(1, std::min<unsigned long long>(blocks, (unsigned long long)sh.wgs));
    if (grad)
        hipLaunchKernelGGL(flux_kernel<true>, dim3(wgs), dim3(256), lds, ctx->stream, A);
    else
        hipLaunchKernelGGL(flux_kernel<false>, dim3(wgs), dim3(256), lds, ctx->stream, A);
    return hipGetLastError();
}

}  // namespace nc
