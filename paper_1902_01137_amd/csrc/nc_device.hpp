// nc_device.hpp -- device building blocks of the null-collision tracer (gfx950).
//
// Counter-based random numbers, ordered crossing of the hierarchical
// majorant grid, collision sampling with null/real rejection, and the
// scattering laws.  Everything here is FP32 except the merge criterion of the
// grid build (FP64).  The whole library is compiled with -ffp-contract=off so
// that every expression below rounds exactly as written: the traversal relies
// on each face parameter being the same function of the face index wherever
// it is evaluated.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "nctrace.h"

namespace nc {

constexpr float kPi = 3.14159265358979f;
constexpr float kInv4Pi = 0.0795774715459477f;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// multiplies mixed with the key, the key bumped by Weyl constants.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64-bit product per multiplier (a single v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// The same with a key that is uniform over the wave (a kernel argument): the
// empty asm makes the key a fresh scalar at every call, so the round keys are
// formed by scalar adds inside the rounds instead of being hoisted out of
// the tracing loop as 18 loop invariants that take scalar registers from the
// loop (and are spilled).  Never call it with a key that differs across lanes.
__device__ inline U4 philox4x32_10_uk(U4 c, uint32_t k0, uint32_t k1)
{
    k0 = __builtin_amdgcn_readfirstlane(k0);   // uniform by contract: scalar registers
    k1 = __builtin_amdgcn_readfirstlane(k1);
    asm volatile("" : "+s"(k0), "+s"(k1));
    return philox4x32_10(c, k0, k1);
}

// A path's random stream: counter = (a, b, draw, stream), key = seed.  Each
// Philox call yields four uniforms, consumed in order.
struct Rng {
    uint32_t a, b, stream, draw;
    uint32_t k0, k1;
    uint32_t q0, q1, q2, q3;
    int left;

    __device__ void init(uint32_t a_, uint32_t b_, uint32_t stream_, uint64_t seed)
    {
        a = a_;
        b = b_;
        stream = stream_;
        draw = 0;
        k0 = (uint32_t)seed;
        k1 = (uint32_t)(seed >> 32);
        left = 0;
    }
    // uniform in [0, 1) with 24 random bits
    __device__ float u01()
    {
        if (left == 0) {
            U4 r = philox4x32_10_uk(U4{a, b, draw, stream}, k0, k1);
            ++draw;
            q0 = r.x; q1 = r.y; q2 = r.z; q3 = r.w;
            left = 4;
        }
        const uint32_t v = q0;
        q0 = q1; q1 = q2; q2 = q3;
        --left;
        return (float)(v >> 8) * 5.9604644775390625e-08f;
    }
    // optical thickness ~ Exp(1)
    __device__ float exp1() { return -__logf(1.0f - u01()); }

    // Batched draws: need(k) makes sure k uniforms are buffered (a fresh
    // Philox block replaces a buffer holding fewer), take() consumes one
    // without a check.  One refill site per caller keeps the Philox rounds
    // out of divergent branches.
    __device__ void need(int k)
    {
        if (left < k) {
            U4 r = philox4x32_10_uk(U4{a, b, draw, stream}, k0, k1);
            ++draw;
            q0 = r.x; q1 = r.y; q2 = r.z; q3 = r.w;
            left = 4;
        }
    }
    __device__ float take()
    {
        const uint32_t v = q0;
        q0 = q1; q1 = q2; q2 = q3;
        --left;
        return (float)(v >> 8) * 5.9604644775390625e-08f;
    }
    __device__ float take_exp1() { return -__logf(1.0f - take()); }
};

// The same stream with its counter words supplied by the caller at each
// refill (the renderer rebuilds them from its pixel, sample and job), so a
// lane keeps only the draw index and the four buffered words.
struct RngBuf {
    uint32_t draw;
    uint32_t q0, q1, q2, q3;
    int left;

    __device__ void reset()
    {
        draw = 0;
        left = 0;
    }
    __device__ void need(int k, uint32_t a, uint32_t b, uint32_t stream, uint32_t k0, uint32_t k1)
    {
        if (left < k) {
            U4 r = philox4x32_10_uk(U4{a, b, draw, stream}, k0, k1);
            ++draw;
            q0 = r.x; q1 = r.y; q2 = r.z; q3 = r.w;
            left = 4;
        }
    }
    __device__ float take()
    {
        const uint32_t v = q0;
        q0 = q1; q1 = q2; q2 = q3;
        --left;
        return (float)(v >> 8) * 5.9604644775390625e-08f;
    }
    __device__ float take_exp1() { return -__logf(1.0f - take()); }
};

// ---------------------------------------------------------------------------
// Grid as seen by the kernels.
// Nodes of levels 1..L are stored level after level, each level [z][y][x]
// with ceil(n/2^l) nodes per axis; a node is float2(kmin_c, kmax_c) with the
// merged flag in the sign bit of kmin_c (k_c >= 0, so the bit is free).
// ---------------------------------------------------------------------------
struct GridView {
    int n[3];
    int L;
    float lo[3];
    float h[3];
    float inv_h[3];
    float hi[3];         // the box's far faces, (float)n h + lo rounded as the crossing rounds a face position
    float k_gas;
    float kscale;        // droplet extinction is kscale * kc (the grid holds kc's min and max)
    const float *kc;
    const float2 *nodes;
    const int *off;      // device array: node offset of level l at index l, off[L+1] = total
    const uint16_t *mask;  // per level-1 node [z][y][x]: bit l (1..L) set if the level-l ancestor is merged
};

__host__ __device__ inline int level_dim(int n, int l) { return (n + (1 << l) - 1) >> l; }

__host__ __device__ inline bool node_merged(float2 v) { return (__builtin_bit_cast(uint32_t, v.x) >> 31) != 0; }
__host__ __device__ inline float node_kmin(float2 v)
{
    return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v.x) & 0x7fffffffu);
}

// Node access with the top levels (l >= lds_first) staged in LDS.
struct NodeSrc {
    const float2 *glob;
    const float2 *lds;   // nodes of levels lds_first..L, same order
    const int *off;      // per-level offsets (LDS copy)
    int lds_first;
    int lds_base;        // off[lds_first]
    int n0, n1;
};

__host__ __device__ inline float2 fetch_node(const NodeSrc &s, int l, int c0, int c1, int c2, uint32_t &gcount)
{
    const int d0 = level_dim(s.n0, l), d1 = level_dim(s.n1, l);
    const int idx = s.off[l] + ((c2 >> l) * d1 + (c1 >> l)) * d0 + (c0 >> l);
    if (l >= s.lds_first) return s.lds[idx - s.lds_base];
    ++gcount;
    return s.glob[idx];
}

// ---------------------------------------------------------------------------
// Ray state for the ordered crossing of the grid (Section 3.1.3).
//
// Face j of axis a lies at lo[a] + j h[a]; the ray meets it at
//   tf(a, j) = ((float)j * h[a] + lo[a] - o[a]) * inv[a],
// monotone in j.  A voxel's exit parameter is the smallest tf over its faces
// (clipped to the box), and every axis whose face attains it is stepped
// across exactly; the other axes keep a cell inside the voxel's slab (the
// floor of the position, clamped).  Only the voxel matters to the walk, the
// exit axes always move forward and no axis steps back across a voxel face,
// so the walk visits each voxel at most once and ends after at most
// nx + ny + nz voxels.
//
// The crossing functions are compiled for the host as well (a bit-exact
// FP32 twin for testing the walk on every ray): they use only IEEE
// operations that round the same on both sides (no approximate reciprocal;
// the library is built without FP contraction).
// ---------------------------------------------------------------------------
struct Ray {
    float o[3], d[3], inv[3];
    float t, tend;       // current parameter, exit from the box
    int c[3];            // current cell
    int lev;             // current voxel: level and node indices (c >> lev)
    float khat;          // voxel majorant m (kscale kmax_c + k_gas)
    float kmin;          // voxel minimum of k_c (for a level-0 voxel: k_c of the cell)
    float texit;         // voxel exit parameter
    int xmask;           // axes whose voxel face is met at texit (bit a)
};

__host__ __device__ inline float face_t(const GridView &g, const Ray &r, int a, int j)
{
    return ((float)j * g.h[a] + g.lo[a] - r.o[a]) * r.inv[a];
}

// Clip o + t d (t >= tmin) to the box; false if it misses.
__host__ __device__ inline bool ray_setup(const GridView &g, Ray &r, const float o[3], const float d[3], float tmin)
{
    float tin = tmin, tout = INFINITY;
    bool miss = false;
    float tlo[3], thi[3];
    // per axis, as selects (lanes that disagree would run both sides of a branch)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.o[a] = o[a];
        r.d[a] = d[a];
        const bool flat = d[a] == 0.0f;   // parallel to the axis' faces: inside their slab or a miss
        r.inv[a] = flat ? INFINITY : 1.0f / d[a];   // correctly rounded (the host twin divides alike)
        // (both faces straight from the grid view, not through face_t: the
        // compiler cannot fold 0 h, and the hoisted per-axis values held through a
        // persistent loop cost registers)
        const float b0 = g.lo[a], b1 = g.hi[a];
        miss = miss || (flat && (o[a] < b0 || o[a] > b1));
        const float t0 = (b0 - r.o[a]) * r.inv[a], t1 = (b1 - r.o[a]) * r.inv[a];
        tlo[a] = t0 > t1 ? t1 : t0;
        thi[a] = t0 > t1 ? t0 : t1;
        tin = flat ? tin : fmaxf(tin, tlo[a]);
        tout = flat ? tout : fminf(tout, thi[a]);
    }
    if (miss || !(tin < tout)) return false;
    r.t = tin;
    r.tend = tout;
    // starting cell: exact on the axis through whose face the ray enters the
    // box, the floor of the position (clamped) on the others; only the voxel
    // matters for the walk, and the walk never steps back across a face
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int j = (int)floorf((o[a] + tin * d[a] - g.lo[a]) * g.inv_h[a]);
        j = j < 0 ? 0 : (j > g.n[a] - 1 ? g.n[a] - 1 : j);
        const bool entered = tin > tmin && tlo[a] == tin;   // entered through this axis' face
        j = (entered && d[a] > 0.0f) ? 0 : j;
        j = (entered && d[a] < 0.0f) ? g.n[a] - 1 : j;
        r.c[a] = j;
    }
    return true;
}

__host__ __device__ inline void leaf_exit(const GridView &g, Ray &r);

// Voxel of the current cell: its coarsest merged ancestor (the cell itself
// when no ancestor is merged), with its majorant and minimum.  The ancestry
// mask of the cell's level-1 node gives the level in one read (highest set
// bit); the cell's own value is read at the same time, so a level-0 voxel
// costs one round trip to memory and a coarser one at most two (none when
// its level is staged in LDS).
__host__ __device__ inline void locate_voxel(const GridView &g, const NodeSrc &ns, Ray &r, float mscale,
                                             uint32_t &node_reads)
{
    float kmin, kmax;
    int l = 0;
    // cell indices are >= 0; the row index fits 32 bits (n1, n2 <= 2^15)
    const uint32_t row = (uint32_t)r.c[2] * (uint32_t)g.n[1] + (uint32_t)r.c[1];
    const uint64_t cell = (uint64_t)row * (uint32_t)g.n[0] + (uint32_t)r.c[0];
    const float kcell = g.kc[cell];
    ++node_reads;
    if (g.L >= 1) {
        const int d0 = level_dim(g.n[0], 1), d1 = level_dim(g.n[1], 1);
        const uint32_t mrow = (uint32_t)(r.c[2] >> 1) * (uint32_t)d1 + (uint32_t)(r.c[1] >> 1);
        const uint32_t m = g.mask[(uint64_t)mrow * (uint32_t)d0 + (uint32_t)(r.c[0] >> 1)];
        ++node_reads;
        l = m ? 31 - __builtin_clz(m) : 0;
    }
    if (l == 0) {
        kmin = kmax = kcell;
    } else {
        const float2 nd = fetch_node(ns, l, r.c[0], r.c[1], r.c[2], node_reads);
        kmin = node_kmin(nd);
        kmax = nd.y;
    }
    r.lev = l;
    r.khat = mscale * (g.kscale * kmax + g.k_gas);
    r.kmin = kmin;
}

__host__ __device__ inline void find_leaf(const GridView &g, const NodeSrc &ns, Ray &r, float mscale,
                                          uint32_t &node_reads)
{
    locate_voxel(g, ns, r, mscale, node_reads);
    leaf_exit(g, r);
}

// Exit parameter of the current voxel (its faces clipped to the field).
__host__ __device__ inline void leaf_exit(const GridView &g, Ray &r)
{
    const int l = r.lev;
    float te = r.tend;
    float tf[3];
    // per axis: the face the ray leaves the voxel through, if it lies inside
    // the field (the box faces are tend); selects, not branches: lanes that
    // disagree would run both sides anyway
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int i = r.c[a] >> l;
        const bool pos = r.d[a] > 0.0f;
        const int j = pos ? min((i + 1) << l, g.n[a]) : (i << l);
        const bool inner = pos ? j < g.n[a] : ((r.d[a] < 0.0f) & (j > 0));
        const float t = face_t(g, r, a, j);
        tf[a] = inner ? t : INFINITY;
        te = fminf(te, tf[a]);
    }
    r.xmask = (tf[0] == te ? 1 : 0) | (tf[1] == te ? 2 : 0) | (tf[2] == te ? 4 : 0);
    r.texit = te < r.t ? r.t : te;
}

// Cross the current voxel's exit face: the ray moves to its exit parameter
// and its cell to the first one past the face (false when the ray leaves the
// box).  The voxel there is not located.
__host__ __device__ inline bool step_cell(const GridView &g, Ray &r)
{
    r.t = r.texit;
    if (!(r.t < r.tend)) return false;
    const int l = r.lev;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int vlo = (r.c[a] >> l) << l;
        const int vhi = min(vlo + (1 << l), g.n[a]) - 1;
        const int across = r.d[a] > 0.0f ? vhi + 1 : vlo - 1;    // across the exit face
        int j = (int)floorf((r.o[a] + r.t * r.d[a] - g.lo[a]) * g.inv_h[a]);
        j = j < vlo ? vlo : (j > vhi ? vhi : j);                  // still inside the voxel's slab
        const int nc = (r.xmask & (1 << a)) ? across : j;
        r.c[a] = r.d[a] == 0.0f ? r.c[a] : nc;
    }
    return true;
}

// Move to the voxel after the current one; false when the ray leaves the box.
__host__ __device__ inline bool next_leaf(const GridView &g, const NodeSrc &ns, Ray &r, float mscale,
                                          uint32_t &node_reads)
{
    if (!step_cell(g, r)) return false;
    find_leaf(g, ns, r, mscale, node_reads);
    return true;
}

// Cell holding the point at parameter t, kept inside the current voxel so
// that the gathered k never exceeds the voxel's majorant.
__device__ inline size_t collision_cell(const GridView &g, const Ray &r, float t)
{
    const int l = r.lev;
    int cc[3];
    // (a level-0 voxel clamps to its own cell)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int base = (r.c[a] >> l) << l;
        const int top = min(base + (1 << l), g.n[a]) - 1;
        int j = (int)floorf((r.o[a] + t * r.d[a] - g.lo[a]) * g.inv_h[a]);
        cc[a] = j < base ? base : (j > top ? top : j);
    }
    const uint32_t row = (uint32_t)cc[2] * (uint32_t)g.n[1] + (uint32_t)cc[1];
    return (size_t)((uint64_t)row * (uint32_t)g.n[0] + (uint32_t)cc[0]);
}

// ---------------------------------------------------------------------------
// Scattering
// ---------------------------------------------------------------------------
// (reciprocals by v_rcp/v_rsq: a relative error of ~1e-7 in a Monte Carlo
// weight is far below the statistical error)
//
// The constants of one asymmetry g are formed once on the host and reach the
// kernels as arguments (scalar registers), so that no vector register holds
// them through the persistent loop.
struct HGc {
    float a;     // 1 + g^2
    float b;     // 2 g
    float c;     // (1 - g^2) / (4 pi)
    float e;     // 1 - g^2
    float d;     // 1 - g
    float r2g;   // 1 / (2 g); 0 when |g| < 1e-4 (then the cosine is uniform)
};

inline HGc make_hg(double g)
{
    HGc h;
    h.a = (float)(1.0 + g * g);
    h.b = (float)(2.0 * g);
    h.c = (float)((1.0 - g * g) / (4.0 * 3.14159265358979323846));
    h.e = (float)(1.0 - g * g);
    h.d = (float)(1.0 - g);
    h.r2g = std::fabs(g) < 1e-4 ? 0.0f : (float)(1.0 / (2.0 * g));
    return h;
}

__device__ inline float hg_phase(const HGc &h, float mu)
{
    const float den = h.a - h.b * mu;
    return h.c * __builtin_amdgcn_rsqf(den) * __builtin_amdgcn_rcpf(den);
}

// Inverse-CDF sample of the HG cosine.
__device__ inline float hg_sample_mu(const HGc &h, float xi)
{
    if (h.r2g == 0.0f) return 2.0f * xi - 1.0f;
    const float s = h.e * __builtin_amdgcn_rcpf(h.d + h.b * xi);
    const float mu = (h.a - s * s) * h.r2g;
    return fminf(1.0f, fmaxf(-1.0f, mu));
}

// A tabulated phase function: values p at cosines mu (n nodes, -1 .. 1),
// linear in between, normalised per steradian; cdf[i] = 2 pi times its
// integral up to mu[i].
struct PhaseView {
    const float *mu, *p, *cdf;
    int n;
};

// the node interval [mu[i], mu[i+1]] holding x of a sorted array (i in 0..n-2)
__device__ inline int tab_interval(const float *a, int n, float x)
{
    int lo = 0, hi = n - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ inline float tab_phase(const PhaseView &t, float m)
{
    const int i = tab_interval(t.mu, t.n, m);
    const float f = (m - t.mu[i]) * __builtin_amdgcn_rcpf(t.mu[i + 1] - t.mu[i]);
    return t.p[i] + f * (t.p[i + 1] - t.p[i]);
}

// Inverse CDF: in the interval holding xi the CDF is 2 pi (p_i x + s x^2 / 2)
// above cdf[i], x = m - mu[i], s the slope; x is the positive root, in the
// form without cancellation.
__device__ inline float tab_sample(const PhaseView &t, float xi)
{
    const int i = tab_interval(t.cdf, t.n, xi);
    const float m0 = t.mu[i], dm = t.mu[i + 1] - m0, p0 = t.p[i];
    const float s = (t.p[i + 1] - p0) * __builtin_amdgcn_rcpf(dm);
    const float r = fmaxf(xi - t.cdf[i], 0.0f) * (1.0f / (2.0f * kPi));
    const float den = p0 + sqrtf(fmaxf(p0 * p0 + 2.0f * s * r, 0.0f));
    const float x = den > 0.0f ? 2.0f * r * __builtin_amdgcn_rcpf(den) : 0.0f;
    return fminf(m0 + fminf(x, dm), 1.0f);
}

// The medium's phase function: the table when there is one, else HG.
__device__ inline float phase_eval(const HGc &h, const PhaseView &t, float mu)
{
    return t.n ? tab_phase(t, mu) : hg_phase(h, mu);
}

__device__ inline float phase_sample_mu(const HGc &h, const PhaseView &t, float xi)
{
    return t.n ? tab_sample(t, xi) : hg_sample_mu(h, xi);
}

// Orthonormal basis around unit n (Duff et al., "Building an orthonormal
// basis, revisited", JCGT 2017), then the direction at cosine mu, azimuth
// 2 pi u about n.
// (sp, cp: sine and cosine of the azimuth; the final normalisation absorbs the
// rounding of the basis.)
__device__ inline void turn_sc(float d[3], float mu, float sp, float cp)
{
    const float sgn = copysignf(1.0f, d[2]);
    const float a = -__builtin_amdgcn_rcpf(sgn + d[2]);
    const float b = d[0] * d[1] * a;
    const float b1[3] = {1.0f + sgn * d[0] * d[0] * a, sgn * b, -sgn * d[0]};
    const float b2[3] = {b, sgn + d[1] * d[1] * a, -d[1]};
    const float st = __builtin_amdgcn_sqrtf(fmaxf(0.0f, 1.0f - mu * mu));
    float n[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) n[k] = mu * d[k] + st * (cp * b1[k] + sp * b2[k]);
    const float inv = rsqrtf(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = n[k] * inv;
}

__device__ inline void turn(float d[3], float mu, float u)
{
    turn_sc(d, mu, __builtin_amdgcn_sinf(u), __builtin_amdgcn_cosf(u));   // sin, cos of 2 pi u
}

// Cosine-weighted direction about +z (Lambertian reflection).
__device__ inline void lambert(float d[3], float u1, float u2)
{
    const float sp = __builtin_amdgcn_sinf(u2), cp = __builtin_amdgcn_cosf(u2);   // sin, cos of 2 pi u2
    const float r = __builtin_amdgcn_sqrtf(u1);
    d[0] = r * cp;
    d[1] = r * sp;
    d[2] = __builtin_amdgcn_sqrtf(fmaxf(0.0f, 1.0f - u1));
}

// ---------------------------------------------------------------------------
// Per-lane event counters, reduced once per wave at the end of a launch.
// ---------------------------------------------------------------------------
struct Counters {
    uint32_t paths, segments, tentative, nulls, reals, leaf_visits, gathers, node_reads, nee_rays, truncated;
};

__device__ inline unsigned long long wave_sum(uint32_t v)
{
    unsigned long long s = v;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    return s;
}

__device__ inline void flush_counters(const Counters &c, nc_counters *out)
{
    if (!out) return;
    const unsigned long long v[10] = {wave_sum(c.paths), wave_sum(c.segments), wave_sum(c.tentative),
                                      wave_sum(c.nulls), wave_sum(c.reals), wave_sum(c.leaf_visits),
                                      wave_sum(c.gathers), wave_sum(c.node_reads), wave_sum(c.nee_rays),
                                      wave_sum(c.truncated)};
    if (__lane_id() == 0) {
        unsigned long long *o = reinterpret_cast<unsigned long long *>(out);
#pragma unroll
        for (int k = 0; k < 10; ++k)
            if (v[k]) atomicAdd(o + k, v[k]);
    }
}

// ===========================================================================
// One step of null-collision tracking in the piecewise-constant majorant
// (Section 2.3 and Eq. 2, with the optical thickness tau carried from voxel
// to voxel): either a tentative collision inside the current voxel, tested
// against the true k gathered from the field, or a move to the next voxel.
// ===========================================================================
enum StepResult { kContinue = 0, kReal = 1, kExit = 2 };

// Step outcome flags (for wave-level event counting).
enum StepFlags : uint32_t { kFTentative = 1, kFReal = 2, kFNull = 4, kFGather = 8, kFLeaf = 16 };

// One step; `reads` counts global grid/field reads, `flags` what happened.
__device__ inline int track_step_f(const GridView &g, const NodeSrc &ns, Ray &r, float &tau, Rng &rng, float mscale,
                                   bool shadow, float &kc_hit, uint32_t &reads, uint32_t &flags)
{
    const float ktau = r.khat * (r.texit - r.t);
    if (r.khat > 0.0f && tau < ktau) {
        r.t = fminf(r.t + tau / r.khat, r.texit);
        const float thr = rng.u01() * r.khat;
        bool real;
        flags = kFTentative;
        if (shadow && thr < g.kscale * r.kmin + g.k_gas) {
            real = true;                      // below the voxel's minimum: real without reading k
        } else if (r.lev == 0) {
            kc_hit = r.kmin;                  // a level-0 voxel is one cell: k is known
            real = thr < g.kscale * kc_hit + g.k_gas;
        } else {
            kc_hit = g.kc[collision_cell(g, r, r.t)];
            ++reads;
            flags |= kFGather;
            real = thr < g.kscale * kc_hit + g.k_gas;
        }
        if (real) {
            flags |= kFReal;
            return kReal;
        }
        flags |= kFNull;
        tau = rng.exp1();
        return kContinue;
    }
    tau -= ktau;
    flags = 0;
    if (!next_leaf(g, ns, r, mscale, reads)) return kExit;
    flags = kFLeaf;
    return kContinue;
}

__device__ inline int track_step(const GridView &g, const NodeSrc &ns, Ray &r, float &tau, Rng &rng, float mscale,
                                 bool shadow, float &kc_hit, Counters &cnt)
{
    uint32_t flags = 0, rd = 0;
    ++cnt.segments;
    const int res = track_step_f(g, ns, r, tau, rng, mscale, shadow, kc_hit, rd, flags);
    cnt.node_reads += rd - ((flags & kFGather) ? 1u : 0u);
    cnt.tentative += (flags & kFTentative) ? 1 : 0;
    cnt.reals += (flags & kFReal) ? 1 : 0;
    cnt.nulls += (flags & kFNull) ? 1 : 0;
    cnt.gathers += (flags & kFGather) ? 1 : 0;
    cnt.leaf_visits += (flags & kFLeaf) ? 1 : 0;
    return res;
}

// Start a ray; a ray that misses the box is set up to exit on its first step.
__device__ inline void start_ray(const GridView &g, const NodeSrc &ns, Ray &r, const float o[3], const float d[3],
                                 float mscale, Counters &cnt)
{
    if (ray_setup(g, r, o, d, 0.0f)) {
        find_leaf(g, ns, r, mscale, cnt.node_reads);
        ++cnt.leaf_visits;
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            r.o[a] = o[a];
            r.d[a] = d[a];
        }
        r.t = r.tend = r.texit = 0.0f;
        r.khat = 0.0f;
        r.kmin = 0.0f;
        r.lev = g.L;
    }
}

// The voxel a ray was in when it stopped at an event; a new ray leaving the
// event point starts in the same voxel unless rounding put its origin in a
// neighbouring cell, which the check below detects.
struct VoxelCache {
    int lev, i0, i1, i2;
    float khat, kmin;
};

__device__ inline VoxelCache voxel_of(const Ray &r)
{
    return VoxelCache{r.lev, r.c[0] >> r.lev, r.c[1] >> r.lev, r.c[2] >> r.lev, r.khat, r.kmin};
}

__device__ inline void start_ray_cached(const GridView &g, const NodeSrc &ns, Ray &r, const float o[3],
                                        const float d[3], const VoxelCache &vc, float mscale, Counters &cnt)
{
    if (ray_setup(g, r, o, d, 0.0f)) {
        if ((r.c[0] >> vc.lev) == vc.i0 && (r.c[1] >> vc.lev) == vc.i1 && (r.c[2] >> vc.lev) == vc.i2) {
            r.lev = vc.lev;
            r.khat = vc.khat;
            r.kmin = vc.kmin;
            leaf_exit(g, r);
        } else {
            find_leaf(g, ns, r, mscale, cnt.node_reads);
        }
        ++cnt.leaf_visits;
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            r.o[a] = o[a];
            r.d[a] = d[a];
        }
        r.t = r.tend = r.texit = 0.0f;
        r.khat = 0.0f;
        r.kmin = 0.0f;
        r.lev = vc.lev;
    }
}

__device__ inline void stage_levels(const GridView &g, int lds_first, int lds_nodes, float2 *s_nodes, int *s_off)
{
    for (int i = threadIdx.x; i < NC_MAX_LEVELS + 2; i += blockDim.x) s_off[i] = i <= g.L + 1 ? g.off[i] : 0;
    if (lds_nodes > 0) {
        const int base = g.off[lds_first];
        for (int i = threadIdx.x; i < lds_nodes; i += blockDim.x) s_nodes[i] = g.nodes[base + i];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Matrix-core fragments.  For v_mfma_f32_16x16x16_bf16, lane l (0..63) holds
//   A[m][k] for m = l % 16, k = 4 (l / 16) + i  (i = 0..3),
//   B[k][n] for n = l % 16, k = 4 (l / 16) + i,
//   D[m][n] for n = l % 16, m = 4 (l / 16) + i.
// ---------------------------------------------------------------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline short to_bf16(float x)
{
    // round to nearest even (v_cvt_pk_bf16_f32 on gfx950; the same bits as
    // adding 0x7fff plus the kept low bit, for every finite x)
    return __builtin_bit_cast(short, (__bf16)x);
}

__device__ inline float from_bf16(short h) { return __uint_as_float(((uint32_t)(uint16_t)h) << 16); }

__device__ inline f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// v_mfma_f32_16x16x32_bf16 (gfx950): as above with eight k values per lane,
// A[m][k] and B[k][n] from lane group l / 16 and element e alike, and the same
// D layout.  Callers only rely on A and B pairing lane group and element the
// same way (the order of k within a product is free).
typedef short bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c)
{
    typedef __bf16 bf16v8 __attribute__((ext_vector_type(8)));
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16v8, a), __builtin_bit_cast(bf16v8, b), c, 0,
                                                   0, 0);
}

}  // namespace nc
