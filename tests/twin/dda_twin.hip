// dda_twin.hip -- the GPU path's ordered crossing of the grid, compiled for
// the host (test tooling, not the oracle).
//
// The crossing functions of nc_device.hpp are __host__ __device__ and use
// only IEEE float operations (no approximate reciprocal, no contraction), so
// this host build walks every ray exactly as the GPU does, degenerate rays
// included.  The tests compare the GPU's crossing with this twin on every ray
// and the twin with the oracle on the rays the oracle does not flag.
//
// The grid is rebuilt here from the library's exported levels in the layout
// the kernels read: float2 nodes (kmin_c with the merged flag in its sign
// bit, kmax_c) level after level, per-level offsets, and one ancestry mask
// per level-1 node (bit l: the level-l ancestor is merged).
#include <stdint.h>

#include <vector>

#include "nc_device.hpp"

using nc::GridView;
using nc::NodeSrc;
using nc::Ray;

extern "C" int twin_trace(int nx, int ny, int nz, double x0, double y0, double z0, double dx, double dy, double dz,
                          int L, const float *kmin, const float *kmax, const uint8_t *merged, const float *kc,
                          const float *rays, int n, int maxv, int *leaf, float *tt, int *count)
{
    if (L < 0 || L > NC_MAX_LEVELS - 1 || n < 0 || maxv < 0) return -1;
    const int dims[3] = {nx, ny, nz};
    std::vector<int> off(NC_MAX_LEVELS + 2, 0);
    long long total = 0;
    for (int l = 1; l <= L; ++l) {
        off[l] = (int)total;
        total += (long long)nc::level_dim(nx, l) * nc::level_dim(ny, l) * nc::level_dim(nz, l);
    }
    off[L + 1] = (int)total;
    std::vector<float2> nodes((size_t)total);
    for (long long i = 0; i < total; ++i) {
        const uint32_t bits = __builtin_bit_cast(uint32_t, kmin[i]) | (merged[i] ? 0x80000000u : 0u);
        nodes[i] = make_float2(__builtin_bit_cast(float, bits), kmax[i]);
    }
    std::vector<uint16_t> mask;
    if (L >= 1) {
        const int d0 = nc::level_dim(nx, 1), d1 = nc::level_dim(ny, 1), d2 = nc::level_dim(nz, 1);
        mask.assign((size_t)d0 * d1 * d2, 0);
        for (int k = 0; k < d2; ++k)
            for (int j = 0; j < d1; ++j)
                for (int i = 0; i < d0; ++i) {
                    uint16_t m = 0;
                    for (int l = 1; l <= L; ++l) {
                        const int s = l - 1;   // level-l ancestor of the level-1 node (i, j, k)
                        const int e0 = nc::level_dim(nx, l), e1 = nc::level_dim(ny, l);
                        const long long q = off[l] + ((long long)(k >> s) * e1 + (j >> s)) * e0 + (i >> s);
                        if (merged[q]) m |= (uint16_t)(1u << l);
                    }
                    mask[((size_t)k * d1 + j) * d0 + i] = m;
                }
    }
    GridView g;
    const double lo[3] = {x0, y0, z0}, h[3] = {dx, dy, dz};
    for (int a = 0; a < 3; ++a) {
        g.n[a] = dims[a];
        g.lo[a] = (float)lo[a];
        g.h[a] = (float)h[a];
        g.inv_h[a] = (float)(1.0 / h[a]);
        g.hi[a] = (float)dims[a] * g.h[a] + g.lo[a];
    }
    g.L = L;
    g.k_gas = 0.0f;
    g.kscale = 1.0f;
    g.kc = kc;
    g.nodes = nodes.data();
    g.off = off.data();
    g.mask = mask.empty() ? nullptr : mask.data();
    const NodeSrc ns{nodes.data(), nullptr, off.data(), L + 1, 0, nx, ny};
    for (int i = 0; i < n; ++i) {
        uint32_t reads = 0;
        Ray r;
        const float o[3] = {rays[6 * i], rays[6 * i + 1], rays[6 * i + 2]};
        const float d[3] = {rays[6 * i + 3], rays[6 * i + 4], rays[6 * i + 5]};
        int k = 0;
        if (nc::ray_setup(g, r, o, d, 0.0f)) {
            nc::find_leaf(g, ns, r, 1.0f, reads);
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
                if (!nc::next_leaf(g, ns, r, 1.0f, reads)) break;
            }
        }
        count[i] = k;
    }
    return 0;
}
