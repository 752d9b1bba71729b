/*
 * oracle.c -- serial FP64 reference implementation of null-collision Monte
 * Carlo path tracing through a hierarchical min/max extinction grid
 * (Villefranque et al., "Path-tracing Monte Carlo library for 3D radiative
 * transfer in highly resolved cloudy atmospheres", JAMES 2019).
 *
 * TEST INFRASTRUCTURE.  This file is the checker, not the product: only the
 * test-suite, the smoke entry point and the CPU-baseline leg of the benchmark
 * load it.  It shares no code, header, table or constant with the HIP path.
 * It is deliberately plain and slow: every function walks the definition it
 * cites, in double precision, one path at a time.
 *
 * Scene model (both implementations are written against the same statement
 * of the problem, nothing else):
 *   - box B = [x0, x0+nx dx] x [y0, y0+ny dy] x [z0, z0+nz dz] (km) holding a
 *     cell field k_c >= 0 (km^-1), plus a uniform absorbing gas k_g inside B;
 *     k = k_c + k_g; vacuum outside B;
 *   - single-scattering albedo ssa(x) = ssa_c k_c / k (the gas only absorbs);
 *   - Henyey-Greenstein phase function of asymmetry g;
 *   - Lambertian ground z = 0 of albedo rho (infinite plane, below B);
 *   - directional sun of zenith theta, azimuth phi (from +X towards +Y),
 *     irradiance S normal to the beam.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define ORC_MAXL 24

/* ========================================================================
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11).  Each round multiplies two counter words by
 * fixed odd constants, splits the 64-bit products into halves and mixes
 * them with the other words and the key; the key is bumped by two Weyl
 * constants between rounds.
 * ======================================================================== */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    int r;
    for (r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The oracle's own random stream: Philox blocks keyed by a 64-bit seed,
 * counter = (stream id low, stream id high, block index, 0), converted to
 * 53-bit doubles in [0,1) from pairs of words. */
typedef struct {
    uint32_t key[2];
    uint64_t id;
    uint32_t block;
    uint32_t buf[4];
    int pos;
} orc_rng;

static void rng_init(orc_rng *r, uint64_t seed, uint64_t id)
{
    r->key[0] = (uint32_t)seed;
    r->key[1] = (uint32_t)(seed >> 32);
    r->id = id;
    r->block = 0;
    r->pos = 4;
}

static double rng_u01(orc_rng *r)
{
    uint32_t a, b;
    if (r->pos > 2) {
        uint32_t ctr[4];
        ctr[0] = (uint32_t)r->id;
        ctr[1] = (uint32_t)(r->id >> 32);
        ctr[2] = r->block++;
        ctr[3] = 0x6f726163u; /* 'orac': keeps the oracle's counters apart */
        orc_philox4x32_10(ctr, r->key, r->buf);
        r->pos = 0;
    }
    a = r->buf[r->pos] >> 5;      /* 27 bits */
    b = r->buf[r->pos + 1] >> 6;  /* 26 bits */
    r->pos += 2;
    return ((double)a * 67108864.0 + (double)b) * (1.0 / 9007199254740992.0);
}

/* ========================================================================
 * Scene records (the oracle's own)
 * ======================================================================== */
typedef struct {
    int32_t nx, ny, nz, pad_;
    double x0, y0, z0, dx, dy, dz;
    double k_gas;
    const float *kc;   /* [nz][ny][nx] */
    double kscale;     /* the medium's droplet extinction is kscale * kc (the grid is built on kc) */
} orc_field;

typedef struct {
    double ssa, g, rho, sun_zenith_deg, sun_azimuth_deg, S, majorant_scale;
    int32_t max_scatter, max_segments;
    double sun_half_angle_deg;   /* angular radius of the solar disc; 0: directional sun */
    int32_t tab_n, tab_pad_;     /* tabulated phase function (n >= 2 nodes) instead of HG; 0: HG */
    const double *tab_mu;        /* node cosines, -1 = mu_0 < ... < mu_{n-1} = 1 */
    const double *tab_p;         /* phase function at the nodes (any positive scale) */
    int32_t kd_n, kd_pad_;       /* k-distribution: n quadrature points (0: the field's k_gas alone) */
    const double *kd_w;          /* their weights (any positive scale) */
    const double *kd_k;          /* their gas extinction, km^-1 */
} orc_optics;

typedef struct {
    int32_t type, width, height, pad_;
    double pos[3], target[3], up[3];
    double fov_y_deg, ortho_w, ortho_h;
} orc_camera;

static void field_arrays(const orc_field *f, int n[3], double lo[3], double h[3])
{
    n[0] = f->nx; n[1] = f->ny; n[2] = f->nz;
    lo[0] = f->x0; lo[1] = f->y0; lo[2] = f->z0;
    h[0] = f->dx; h[1] = f->dy; h[2] = f->dz;
}

static double cell_kc(const orc_field *f, int i, int j, int m)
{
    return (double)f->kc[((size_t)m * f->ny + j) * f->nx + i];
}

/* droplet extinction of a cell as the transport sees it */
static double cell_kd(const orc_field *f, int i, int j, int m)
{
    return f->kscale * cell_kc(f, i, j, m);
}

/* ========================================================================
 * Grid build (Section 3.1.1 "Construction"; Section 4.2 merge criterion;
 * Appendix B.3 power-of-two intermediate grid).
 *
 * Level 0 is the cell field.  A level-l node (i,j,m) covers the cells
 * [i 2^l, min((i+1) 2^l, n)) along each axis, which is the node indexing of
 * an octree over the field padded to the next power of two, with the padding
 * left out.  It stores the minimum and maximum of k_c over the cells it
 * covers.  The node is "merged" (one voxel of the acceleration grid) iff the
 * optical-depth criterion holds:
 *   criterion 0: (kmax_c + k_g) * dz 2^l  <  tau_tilde
 *   criterion 1: (kmax_c - kmin_c) * dz 2^l < tau_tilde
 *   criterion 2: l <= flat_level (no test on the field: a flat grid of
 *                supercells of 2^flat_level cells, the single-level majorant
 *                grid the paper sets against its hierarchy, Sections 2.4 and 3)
 *   criterion 3: the node lies wholly above or below the cloudy layer, or
 *                l <= flat_level: the layered grid the paper cites as the
 *                step before its hierarchy (Section 3.1.1: the cloudy layer
 *                split from the clear layers above and below it, each with
 *                its own fixed resolution).  The cloudy layer is the range of
 *                z indices holding a cell with k_c > 0; clear layers get the
 *                coarsest nodes that stay clear, the cloudy layer supercells
 *                of 2^flat_level cells
 * evaluated in double precision.  All are monotone (a merged node has merged
 * children), so the bottom-up merging of groups of 2^3 children gives the
 * same voxels as taking, for each cell, its coarsest ancestor that passes the
 * criterion; that ancestor's level is the cell's leaf level (0: the cell
 * itself).  tau_tilde = 0 never merges (Section 4.2).
 * ======================================================================== */
typedef struct {
    int L;
    int dim[ORC_MAXL + 1][3];
    float *kmin[ORC_MAXL + 1];
    float *kmax[ORC_MAXL + 1];
    unsigned char *merged[ORC_MAXL + 1];
    unsigned char *leaf;
    int n[3];
} orc_grid;

void orc_grid_free(orc_grid *g)
{
    int l;
    if (!g) return;
    for (l = 0; l <= ORC_MAXL; ++l) {
        free(g->kmin[l]);
        free(g->kmax[l]);
        free(g->merged[l]);
    }
    free(g->leaf);
    free(g);
}

orc_grid *orc_grid_build(const orc_field *f, double tau_tilde, int criterion, int flat_level)
{
    orc_grid *g = (orc_grid *)calloc(1, sizeof(orc_grid));
    int nmax, l;
    if (!g) return NULL;
    g->n[0] = f->nx; g->n[1] = f->ny; g->n[2] = f->nz;
    nmax = f->nx;
    if (f->ny > nmax) nmax = f->ny;
    if (f->nz > nmax) nmax = f->nz;
    g->L = 0;
    while ((1 << g->L) < nmax) g->L++;
    /* criterion 3: z extent [zc_lo, zc_hi] of the cells with k_c > 0 (empty if none) */
    int zc_lo = f->nz, zc_hi = -1;
    if (criterion == 3) {
        int ci, cj, cm;
        for (cm = 0; cm < f->nz; ++cm)
            for (cj = 0; cj < f->ny; ++cj)
                for (ci = 0; ci < f->nx; ++ci)
                    if (cell_kc(f, ci, cj, cm) > 0.0) {
                        if (cm < zc_lo) zc_lo = cm;
                        if (cm > zc_hi) zc_hi = cm;
                    }
    }
    for (l = 1; l <= g->L; ++l) {
        int a, i, j, m;
        size_t nn;
        for (a = 0; a < 3; ++a) g->dim[l][a] = (g->n[a] + (1 << l) - 1) >> l;
        nn = (size_t)g->dim[l][0] * g->dim[l][1] * g->dim[l][2];
        g->kmin[l] = (float *)malloc(nn * sizeof(float));
        g->kmax[l] = (float *)malloc(nn * sizeof(float));
        g->merged[l] = (unsigned char *)malloc(nn);
        for (m = 0; m < g->dim[l][2]; ++m)
            for (j = 0; j < g->dim[l][1]; ++j)
                for (i = 0; i < g->dim[l][0]; ++i) {
                    int ia = i << l, ib = (i + 1) << l;
                    int ja = j << l, jb = (j + 1) << l;
                    int ma = m << l, mb = (m + 1) << l;
                    int ci, cj, cm;
                    double lo = INFINITY, hi = -INFINITY, crit, dz_node;
                    size_t id = ((size_t)m * g->dim[l][1] + j) * g->dim[l][0] + i;
                    if (ib > f->nx) ib = f->nx;
                    if (jb > f->ny) jb = f->ny;
                    if (mb > f->nz) mb = f->nz;
                    for (cm = ma; cm < mb; ++cm)
                        for (cj = ja; cj < jb; ++cj)
                            for (ci = ia; ci < ib; ++ci) {
                                double v = cell_kc(f, ci, cj, cm);
                                if (v < lo) lo = v;
                                if (v > hi) hi = v;
                            }
                    g->kmin[l][id] = (float)lo;  /* exact: values are floats */
                    g->kmax[l][id] = (float)hi;
                    dz_node = f->dz * (double)(1 << l);
                    if (criterion == 2) {
                        g->merged[l][id] = (unsigned char)(l <= flat_level);
                        continue;
                    }
                    if (criterion == 3) {
                        /* cells ma .. mb-1 in z: clear if wholly below or above the cloudy layer */
                        const int clear = (mb - 1 < zc_lo) || (ma > zc_hi);
                        g->merged[l][id] = (unsigned char)(clear || l <= flat_level);
                        continue;
                    }
                    if (criterion == 0) {
                        volatile double s = hi + f->k_gas;
                        crit = s * dz_node;
                    } else {
                        volatile double s = hi - lo;
                        crit = s * dz_node;
                    }
                    g->merged[l][id] = (unsigned char)(crit < tau_tilde);
                }
    }
    g->leaf = (unsigned char *)malloc((size_t)f->nx * f->ny * f->nz);
    {
        int i, j, m;
        for (m = 0; m < f->nz; ++m)
            for (j = 0; j < f->ny; ++j)
                for (i = 0; i < f->nx; ++i) {
                    int lev = 0;
                    for (l = g->L; l >= 1; --l) {
                        size_t id = ((size_t)(m >> l) * g->dim[l][1] + (j >> l)) * g->dim[l][0] + (i >> l);
                        if (g->merged[l][id]) { lev = l; break; }
                    }
                    g->leaf[((size_t)m * f->ny + j) * f->nx + i] = (unsigned char)lev;
                }
    }
    return g;
}

int orc_grid_levels(const orc_grid *g) { return g->L; }

void orc_grid_level_dims(const orc_grid *g, int l, int32_t out[3])
{
    out[0] = g->dim[l][0]; out[1] = g->dim[l][1]; out[2] = g->dim[l][2];
}

void orc_grid_export(const orc_grid *g, int l, float *kmin, float *kmax, uint8_t *merged)
{
    size_t nn = (size_t)g->dim[l][0] * g->dim[l][1] * g->dim[l][2];
    memcpy(kmin, g->kmin[l], nn * sizeof(float));
    memcpy(kmax, g->kmax[l], nn * sizeof(float));
    memcpy(merged, g->merged[l], nn);
}

void orc_grid_leaf_levels(const orc_grid *g, uint8_t *out)
{
    memcpy(out, g->leaf, (size_t)g->n[0] * g->n[1] * g->n[2]);
}

/* Majorant of the leaf holding cell (i,j,m), before the k_g and scale terms:
 * kmax_c of the coarsest merged ancestor, or k_c itself for a level-0 leaf. */
static double leaf_kmax_c(const orc_field *f, const orc_grid *g, int i, int j, int m, int *lev_out, int id_out[3])
{
    int lev = g->leaf[((size_t)m * f->ny + j) * f->nx + i];
    if (lev_out) *lev_out = lev;
    if (id_out) { id_out[0] = i >> lev; id_out[1] = j >> lev; id_out[2] = m >> lev; }
    if (lev == 0) return cell_kc(f, i, j, m);
    return (double)g->kmax[lev][((size_t)(m >> lev) * g->dim[lev][1] + (j >> lev)) * g->dim[lev][0] + (i >> lev)];
}

/* ========================================================================
 * Ray / box geometry
 * ======================================================================== */
/* Clip the ray o + t d, t >= tmin0, to B.  Returns 1 and [ta,tb] if the
 * clipped segment has positive length. */
static int clip_box(const orc_field *f, const double o[3], const double d[3], double tmin0,
                    double *ta, double *tb)
{
    int n[3], a;
    double lo[3], h[3], t0 = tmin0, t1 = INFINITY;
    field_arrays(f, n, lo, h);
    for (a = 0; a < 3; ++a) {
        double blo = lo[a], bhi = lo[a] + n[a] * h[a];
        if (d[a] == 0.0) {
            if (o[a] < blo || o[a] > bhi) return 0;
        } else {
            double u = (blo - o[a]) / d[a], v = (bhi - o[a]) / d[a];
            if (u > v) { double w = u; u = v; v = w; }
            if (u > t0) t0 = u;
            if (v < t1) t1 = v;
        }
    }
    if (!(t0 < t1)) return 0;
    *ta = t0;
    *tb = t1;
    return 1;
}

/* ========================================================================
 * Ordered crossing of the grid (Section 3.1.3): the sequence of leaves a ray
 * passes through, with the parameter interval spent in each.
 *
 * Written from the definition rather than as a traversal: all cell faces the
 * ray crosses inside B are listed and sorted; in each interval between
 * consecutive crossings the cell is found from the interval's midpoint and
 * mapped to its leaf; consecutive intervals in the same leaf are joined.
 *
 * The result is "degenerate" when floating-point rounding in any other
 * implementation could change it: two crossings along different axes closer
 * than eps (along the ray) next to a change of leaf or at the box boundary,
 * an origin inside B within eps of a face, an axis-parallel ray within eps of
 * a face plane, or a ray that grazes B within eps.
 * ======================================================================== */
typedef struct { double t; int axis; } orc_event;

static int cmp_event(const void *a, const void *b)
{
    double ta = ((const orc_event *)a)->t, tb = ((const orc_event *)b)->t;
    return (ta > tb) - (ta < tb);
}

int orc_leaf_sequence(const orc_field *f, const orc_grid *g, const double ray[6], double eps,
                      int32_t maxv, int32_t *leaf, double *tout, int32_t *degenerate)
{
    int n[3], a, ne = 0, nint, i, count = 0, deg = 0;
    double lo[3], h[3], o[3], d[3], ta, tb;
    orc_event *ev;
    double *pts;
    int32_t (*ids)[4];
    field_arrays(f, n, lo, h);
    for (a = 0; a < 3; ++a) { o[a] = ray[a]; d[a] = ray[3 + a]; }
    *degenerate = 0;

    /* grazing / near-miss test: slab intersection length with t unrestricted below 0 */
    {
        double t0 = -INFINITY, t1 = INFINITY;
        int inside_par = 1;
        for (a = 0; a < 3; ++a) {
            double blo = lo[a], bhi = lo[a] + n[a] * h[a];
            if (d[a] == 0.0) {
                if (o[a] < blo - eps || o[a] > bhi + eps) inside_par = 0;
                else if (fabs(o[a] - blo) < eps || fabs(o[a] - bhi) < eps) deg = 1;
            } else {
                double u = (blo - o[a]) / d[a], v = (bhi - o[a]) / d[a];
                if (u > v) { double w = u; u = v; v = w; }
                if (u > t0) t0 = u;
                if (v < t1) t1 = v;
            }
        }
        if (inside_par && t1 > 0.0 && fabs(t1 - t0) < eps) deg = 1;
        if (inside_par && fabs(t1) < eps) deg = 1;
    }
    if (!clip_box(f, o, d, 0.0, &ta, &tb)) { *degenerate = deg; return 0; }

    /* axis-parallel rays running along an interior face plane */
    for (a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            int k;
            for (k = 0; k <= n[a]; ++k)
                if (fabs(lo[a] + k * h[a] - o[a]) < eps) deg = 1;
        }
    }

    ev = (orc_event *)malloc(sizeof(orc_event) * (size_t)(n[0] + n[1] + n[2] + 8));
    for (a = 0; a < 3; ++a) {
        int k;
        if (d[a] == 0.0) continue;
        for (k = 0; k <= n[a]; ++k) {
            double t = (lo[a] + k * h[a] - o[a]) / d[a];
            if (t > ta - 2 * eps && t < tb + 2 * eps) {
                ev[ne].t = t;
                ev[ne].axis = a;
                ne++;
            }
        }
    }
    qsort(ev, (size_t)ne, sizeof(orc_event), cmp_event);

    /* interval end points strictly inside (ta, tb) */
    pts = (double *)malloc(sizeof(double) * (size_t)(ne + 2));
    nint = 0;
    pts[nint++] = ta;
    for (i = 0; i < ne; ++i)
        if (ev[i].t > ta && ev[i].t < tb) pts[nint++] = ev[i].t;
    pts[nint++] = tb;
    ids = (int32_t(*)[4])malloc(sizeof(int32_t) * 4 * (size_t)nint);

    for (i = 0; i + 1 < nint; ++i) {
        double t0 = pts[i], t1 = pts[i + 1], tm, c[3];
        int ci[3], lev;
        if (!(t1 > t0)) { ids[i][0] = -2; continue; }
        tm = 0.5 * (t0 + t1);
        for (a = 0; a < 3; ++a) {
            c[a] = floor((o[a] + tm * d[a] - lo[a]) / h[a]);
            if (c[a] < 0) c[a] = 0;
            if (c[a] > n[a] - 1) c[a] = n[a] - 1;
            ci[a] = (int)c[a];
        }
        lev = g->leaf[((size_t)ci[2] * n[1] + ci[1]) * n[0] + ci[0]];
        ids[i][0] = lev;
        ids[i][1] = ci[0] >> lev;
        ids[i][2] = ci[1] >> lev;
        ids[i][3] = ci[2] >> lev;
        if (count > 0 && memcmp(leaf + 4 * (count - 1), ids[i], 4 * sizeof(int32_t)) == 0) {
            tout[2 * (count - 1) + 1] = t1;
        } else {
            if (count < maxv) {
                memcpy(leaf + 4 * count, ids[i], 4 * sizeof(int32_t));
                tout[2 * count] = t0;
                tout[2 * count + 1] = t1;
            }
            count++;
            if (count > maxv) count = maxv + 1;  /* saturate: caller sees overflow */
        }
    }

    /* near-coincident crossings at leaf changes or at the box boundary */
    if (ta < eps && ta == 0.0) {
        /* origin inside B: any face within eps of the origin */
        for (i = 0; i < ne; ++i)
            if (fabs(ev[i].t) < eps) deg = 1;
    }
    for (i = 0; i + 1 < ne; ++i) {
        if (ev[i].axis != ev[i + 1].axis && ev[i + 1].t - ev[i].t < eps) {
            /* leaf ids just before ev[i] and just after ev[i+1] */
            double tb0 = ev[i].t, tb1 = ev[i + 1].t;
            int k, same = 1, first = 1;
            int32_t ref[4] = {0, 0, 0, 0};
            int touches_box = (tb0 <= ta + eps) || (tb1 >= tb - eps);
            for (k = 0; k + 1 < nint; ++k) {
                if (ids[k][0] == -2) continue;
                if (pts[k + 1] < tb0 - eps || pts[k] > tb1 + eps) continue;
                if (first) { memcpy(ref, ids[k], sizeof(ref)); first = 0; }
                else if (memcmp(ref, ids[k], sizeof(ref)) != 0) same = 0;
            }
            if (!same || touches_box) deg = 1;
        }
    }
    free(ids);
    free(pts);
    free(ev);
    *degenerate = deg;
    return count;
}

/* ========================================================================
 * Cell walker: the cells a ray crosses inside B, in order (used by regular
 * tracking, Fig. 2a, and by the cell-by-cell form of hierarchical delta
 * tracking below).
 * ======================================================================== */
typedef struct {
    const orc_field *f;
    double o[3], d[3];
    double t, tend;
    int idx[3], n[3];
    double lo[3], h[3];
} walker;

static int walker_init(walker *w, const orc_field *f, const double o[3], const double d[3], double tstart)
{
    double ta, tb, p;
    int a;
    w->f = f;
    field_arrays(f, w->n, w->lo, w->h);
    for (a = 0; a < 3; ++a) { w->o[a] = o[a]; w->d[a] = d[a]; }
    if (!clip_box(f, o, d, tstart, &ta, &tb)) return 0;
    w->t = ta;
    w->tend = tb;
    /* the cell containing the point just after ta */
    for (a = 0; a < 3; ++a) {
        double tm = ta + 1e-9 * (tb - ta);
        p = floor((o[a] + tm * d[a] - w->lo[a]) / w->h[a]);
        if (p < 0) p = 0;
        if (p > w->n[a] - 1) p = w->n[a] - 1;
        w->idx[a] = (int)p;
    }
    return 1;
}

/* Current cell's exit parameter (clipped to the box exit). */
static double walker_exit(const walker *w, int *axis)
{
    double te = w->tend;
    int a;
    *axis = -1;
    for (a = 0; a < 3; ++a) {
        double face, t;
        if (w->d[a] == 0.0) continue;
        face = w->lo[a] + (w->d[a] > 0 ? (w->idx[a] + 1) : w->idx[a]) * w->h[a];
        t = (face - w->o[a]) / w->d[a];
        if (t < te) { te = t; *axis = a; }
    }
    if (te < w->t) te = w->t;
    return te;
}

/* Step into the next cell; returns 0 when the ray leaves B. */
static int walker_advance(walker *w, double te, int axis)
{
    int a;
    w->t = te;
    if (axis < 0) return 0;
    /* every axis whose face is crossed at (numerically) the same parameter */
    for (a = 0; a < 3; ++a) {
        double face, t;
        if (w->d[a] == 0.0) continue;
        face = w->lo[a] + (w->d[a] > 0 ? (w->idx[a] + 1) : w->idx[a]) * w->h[a];
        t = (face - w->o[a]) / w->d[a];
        if (a == axis || t <= te) {
            w->idx[a] += (w->d[a] > 0) ? 1 : -1;
            if (w->idx[a] < 0 || w->idx[a] >= w->n[a]) return 0;
        }
    }
    return w->t < w->tend;
}

static double walker_k(const walker *w)
{
    return cell_kd(w->f, w->idx[0], w->idx[1], w->idx[2]) + w->f->k_gas;
}

/* Optical depth of k along the ray from t0 to t1 (t1 = INFINITY: to the box
 * exit), summed exactly cell by cell (path tracking, Fig. 2a).  Stops early
 * once tau exceeds tau_cap (pass INFINITY for none). */
double orc_optical_depth_ray(const orc_field *f, const double o[3], const double d[3], double t0, double t1,
                             double tau_cap)
{
    walker w;
    double tau = 0.0;
    if (!walker_init(&w, f, o, d, t0)) return 0.0;
    for (;;) {
        int axis;
        double te = walker_exit(&w, &axis), a = w.t, b = te;
        if (b > t1) b = t1;
        if (b > a) tau += walker_k(&w) * (b - a);
        if (te >= t1 || tau > tau_cap) break;
        if (!walker_advance(&w, te, axis)) break;
    }
    return tau;
}

double orc_optical_depth(const orc_field *f, const double ray[6], double t1)
{
    return orc_optical_depth_ray(f, ray, ray + 3, 0.0, t1, INFINITY);
}

/* Free path by regular tracking: the parameter where the optical depth from
 * tstart reaches tau_s, or returns 0 if the ray leaves B first. */
static int regular_free_path(const orc_field *f, const double o[3], const double d[3], double tstart,
                             double tau_s, double *tcoll, double *kc_at)
{
    walker w;
    if (!walker_init(&w, f, o, d, tstart)) return 0;
    for (;;) {
        int axis;
        double te = walker_exit(&w, &axis), k = walker_k(&w), len = te - w.t;
        if (len > 0 && tau_s < k * len) {
            *tcoll = w.t + tau_s / k;
            *kc_at = cell_kd(f, w.idx[0], w.idx[1], w.idx[2]);
            return 1;
        }
        if (len > 0) tau_s -= k * len;
        if (!walker_advance(&w, te, axis)) return 0;
    }
}

/* ========================================================================
 * Null-collision direct transmissivity (Section 2.3, the five-step algorithm
 * and its integral counterpart, Eq. 2).
 *
 * A path from x0 along omega: sample the optical thickness tau_s ~ Exp(1) in
 * the majorant field; if the ray leaves the volume first the path has t = 1;
 * otherwise at the collision point the collision is true with probability
 * k/k_hat (t = 0) and null otherwise, in which case the walk restarts from
 * the collision point.  The oracle offers three majorant fields:
 *   mode 1: one homogeneous majorant m (max k_c + k_g) over B (Fig. 2b);
 *   mode 2: the piecewise-constant majorant of the acceleration grid,
 *           m (kmax_c(leaf) + k_g) in each leaf (Fig. 2c), with the free path
 *           carried from leaf to leaf;
 *   mode 0: no sampling: the exact exp(-tau).
 * counters (modes 1 and 2, may be NULL): [0] tentative collisions, [1] null
 * collisions, [2] leaf visits, summed over all samples; counters_sq (may be
 * NULL): the sums of their per-sample squares (for standard errors).
 * ======================================================================== */
static double field_max_kc(const orc_field *f)
{
    size_t i, n = (size_t)f->nx * f->ny * f->nz;
    double m = 0.0;
    for (i = 0; i < n; ++i)
        if ((double)f->kc[i] > m) m = (double)f->kc[i];
    return f->kscale * m;
}

static double kc_at_point(const orc_field *f, const double x[3])
{
    int n[3], a, c[3];
    double lo[3], h[3];
    field_arrays(f, n, lo, h);
    for (a = 0; a < 3; ++a) {
        double p = floor((x[a] - lo[a]) / h[a]);
        if (p < 0) p = 0;
        if (p > n[a] - 1) p = n[a] - 1;
        c[a] = (int)p;
    }
    return cell_kd(f, c[0], c[1], c[2]);
}

/* Delta tracking with one homogeneous majorant khat over B. */
static int delta_global(const orc_field *f, double khat, const double o[3], const double d[3], orc_rng *r,
                        uint64_t *cnt)
{
    double ta, tb, t;
    if (!clip_box(f, o, d, 0.0, &ta, &tb)) return 1;
    if (khat <= 0.0) return 1;
    t = ta;
    for (;;) {
        double x[3], k;
        t += -log(1.0 - rng_u01(r)) / khat;
        if (!(t < tb)) return 1;
        x[0] = o[0] + t * d[0]; x[1] = o[1] + t * d[1]; x[2] = o[2] + t * d[2];
        k = kc_at_point(f, x) + f->k_gas;
        if (cnt) cnt[0]++;
        if (rng_u01(r) * khat < k) return 0;
        if (cnt) cnt[1]++;
    }
}

/* Delta tracking in the grid's piecewise-constant majorant, written cell by
 * cell: inside one leaf the majorant is constant, so consuming the leaf one
 * cell at a time with the remaining optical thickness carried over is the
 * same walk as consuming it at once.  Returns 1 at the first real collision
 * (its parameter and the droplet extinction there in *tc, *kd) and 0 when
 * the ray leaves B.  cnt (may be NULL): [0] tentative collisions, [1] nulls,
 * [2] leaves entered. */
static int delta_hier_walk(const orc_field *f, const orc_grid *g, double m, const double o[3], const double d[3],
                           orc_rng *r, uint64_t *cnt, double *tc, double *kd)
{
    walker w;
    double tau_s;
    int prev[4] = {-1, -1, -1, -1};
    if (!walker_init(&w, f, o, d, 0.0)) return 0;
    tau_s = -log(1.0 - rng_u01(r));
    for (;;) {
        int axis, lev, id[3];
        double te = walker_exit(&w, &axis);
        double kmc = leaf_kmax_c(f, g, w.idx[0], w.idx[1], w.idx[2], &lev, id);
        double khat = m * (f->kscale * kmc + f->k_gas);
        if (lev != prev[0] || id[0] != prev[1] || id[1] != prev[2] || id[2] != prev[3]) {
            if (cnt) cnt[2]++;
            prev[0] = lev; prev[1] = id[0]; prev[2] = id[1]; prev[3] = id[2];
        }
        while (te > w.t && khat > 0.0 && tau_s < khat * (te - w.t)) {
            double k;
            w.t += tau_s / khat;
            k = walker_k(&w);
            if (cnt) cnt[0]++;
            if (rng_u01(r) * khat < k) {
                if (tc) *tc = w.t;
                if (kd) *kd = cell_kd(f, w.idx[0], w.idx[1], w.idx[2]);
                return 1;
            }
            if (cnt) cnt[1]++;
            tau_s = -log(1.0 - rng_u01(r));
        }
        if (te > w.t) tau_s -= khat * (te - w.t);
        if (!walker_advance(&w, te, axis)) return 0;
    }
}

/* The 0/1 transmissivity estimate of delta tracking: 1 iff no real collision. */
static int delta_hier(const orc_field *f, const orc_grid *g, double m, const double o[3], const double d[3],
                      orc_rng *r, uint64_t *cnt)
{
    return !delta_hier_walk(f, g, m, o, d, r, cnt, NULL, NULL);
}

void orc_transmittance(const orc_field *f, const orc_grid *g, int mode, double majorant_scale,
                       const double *rays, int32_t n, int32_t nsamples, uint64_t seed,
                       double *mean, double *se, uint64_t *counters, double *counters_sq)
{
    int i, s, k;
    double kglob = majorant_scale * (field_max_kc(f) + f->k_gas);
    for (i = 0; i < n; ++i) {
        const double *o = rays + 6 * i, *d = rays + 6 * i + 3;
        if (mode == 0) {
            mean[i] = exp(-orc_optical_depth_ray(f, o, d, 0.0, INFINITY, INFINITY));
            se[i] = 0.0;
            continue;
        }
        {
            double sum = 0.0;
            for (s = 0; s < nsamples; ++s) {
                orc_rng r;
                uint64_t pc[3] = {0, 0, 0};
                int t;
                rng_init(&r, seed, ((uint64_t)i << 24) + (uint64_t)s);
                if (mode == 1) t = delta_global(f, kglob, o, d, &r, pc);
                else t = delta_hier(f, g, majorant_scale, o, d, &r, pc);
                sum += t;
                for (k = 0; k < 3; ++k) {
                    if (counters) counters[k] += pc[k];
                    if (counters_sq) counters_sq[k] += (double)pc[k] * (double)pc[k];
                }
            }
            mean[i] = sum / nsamples;
            /* the estimator is Bernoulli: its variance is p(1-p) */
            se[i] = sqrt(mean[i] * (1.0 - mean[i]) / (nsamples > 1 ? nsamples - 1 : 1));
        }
    }
}

/* ========================================================================
 * Scattering functions
 * ======================================================================== */
/* Henyey-Greenstein phase function per steradian, mu = cosine of the angle
 * between incident and scattered propagation directions. */
double orc_hg_phase(double g, double mu)
{
    double den = 1.0 + g * g - 2.0 * g * mu;
    return (1.0 - g * g) / (4.0 * ORC_PI * den * sqrt(den));
}

/* Inverse-CDF sample of the HG cosine. */
double orc_hg_sample_mu(double g, double xi)
{
    if (fabs(g) < 1e-6) return 2.0 * xi - 1.0;  /* the g -> 0 limit of the inverse below */
    {
        double s = (1.0 - g * g) / (1.0 - g + 2.0 * g * xi);
        double mu = (1.0 + g * g - s * s) / (2.0 * g);
        if (mu > 1.0) mu = 1.0;
        if (mu < -1.0) mu = -1.0;
        return mu;
    }
}

/* A tabulated phase function (Section 4.1 takes the droplets' phase
 * function from Mie tables): values p_i at cosines mu_i, linear in mu between
 * nodes, scaled so that 2 pi times its integral over [-1, 1] is 1 (per
 * steradian).  tab_scale returns that scale. */
static double tab_scale(const double *mu, const double *p, int n)
{
    double a = 0.0;
    int i;
    for (i = 0; i + 1 < n; ++i) a += 0.5 * (p[i] + p[i + 1]) * (mu[i + 1] - mu[i]);
    return 1.0 / (2.0 * ORC_PI * a);
}

double orc_tab_phase(const double *mu, const double *p, int32_t n, double m)
{
    int i = 0;
    double t;
    while (i + 2 < n && mu[i + 1] <= m) ++i;      /* the node interval holding m */
    t = (m - mu[i]) / (mu[i + 1] - mu[i]);
    return ((1.0 - t) * p[i] + t * p[i + 1]) * tab_scale(mu, p, n);
}

/* Inverse CDF: the cosine m with 2 pi int_{-1}^{m} p = xi, by bisection on
 * the exact (piecewise quadratic) CDF. */
double orc_tab_sample(const double *mu, const double *p, int32_t n, double xi)
{
    double c = tab_scale(mu, p, n), acc = 0.0, lo, hi, base;
    int i = 0, it;
    for (;;) {
        double seg = 2.0 * ORC_PI * c * 0.5 * (p[i] + p[i + 1]) * (mu[i + 1] - mu[i]);
        if (xi < acc + seg || i + 2 >= n) break;
        acc += seg;
        ++i;
    }
    base = acc;
    lo = mu[i];
    hi = mu[i + 1];
    for (it = 0; it < 64; ++it) {
        double m = 0.5 * (lo + hi), x = m - mu[i];
        double pm = p[i] + (p[i + 1] - p[i]) * x / (mu[i + 1] - mu[i]);
        double F = base + 2.0 * ORC_PI * c * 0.5 * (p[i] + pm) * x;
        if (F < xi) lo = m; else hi = m;
    }
    return 0.5 * (lo + hi);
}

static double phase_eval(const orc_optics *op, double mu)
{
    return op->tab_n >= 2 ? orc_tab_phase(op->tab_mu, op->tab_p, op->tab_n, mu) : orc_hg_phase(op->g, mu);
}

static double phase_sample(const orc_optics *op, double xi)
{
    return op->tab_n >= 2 ? orc_tab_sample(op->tab_mu, op->tab_p, op->tab_n, xi) : orc_hg_sample_mu(op->g, xi);
}

static void normalize3(double v[3])
{
    double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n; v[1] /= n; v[2] /= n;
}

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Direction at polar cosine mu and azimuth phi about axis w.  The frame is
 * built from the coordinate axis least aligned with w. */
static void rotate_about(const double w[3], double mu, double phi, double out[3])
{
    double a[3] = {0, 0, 0}, u[3], v[3], s;
    int k = 0;
    if (fabs(w[1]) < fabs(w[k])) k = 1;
    if (fabs(w[2]) < fabs(w[k])) k = 2;
    a[k] = 1.0;
    cross3(w, a, u);
    normalize3(u);
    cross3(w, u, v);
    s = sqrt(fmax(0.0, 1.0 - mu * mu));
    out[0] = mu * w[0] + s * (cos(phi) * u[0] + sin(phi) * v[0]);
    out[1] = mu * w[1] + s * (cos(phi) * u[1] + sin(phi) * v[1]);
    out[2] = mu * w[2] + s * (cos(phi) * u[2] + sin(phi) * v[2]);
    normalize3(out);
}

static void sun_dir(const orc_optics *op, double s[3])
{
    double t = op->sun_zenith_deg * ORC_PI / 180.0, p = op->sun_azimuth_deg * ORC_PI / 180.0;
    s[0] = sin(t) * cos(p);
    s[1] = sin(t) * sin(p);
    s[2] = cos(t);
}

/* The sun as a disc of angular radius alpha about s with uniform radiance
 * L_s, its irradiance through a plane normal to s being S = L_s pi sin^2
 * alpha (the sun model of Appendix A's "solar cone"; alpha = 0 is the
 * directional sun).  The local estimate draws its direction uniformly over
 * the cone (solid angle 2 pi (1 - cos alpha)), so the estimate of an event
 * carries S times cone_gain = 2 pi (1 - cos alpha) / (pi sin^2 alpha) =
 * 2 / (1 + cos alpha). */
static double cone_gain(const orc_optics *op)
{
    return 2.0 / (1.0 + cos(op->sun_half_angle_deg * ORC_PI / 180.0));
}

static void sun_sample(const orc_optics *op, const double s[3], orc_rng *r, double w[3])
{
    double ca, mu, phi;
    if (op->sun_half_angle_deg <= 0.0) {     /* directional sun: no draw */
        w[0] = s[0]; w[1] = s[1]; w[2] = s[2];
        return;
    }
    ca = cos(op->sun_half_angle_deg * ORC_PI / 180.0);
    mu = 1.0 - rng_u01(r) * (1.0 - ca);     /* uniform over the cap's solid angle */
    phi = 2.0 * ORC_PI * rng_u01(r);
    rotate_about(s, mu, phi, w);
}

/* radiance of the disc seen along d (units of S): S / (pi sin^2 alpha) inside it */
static double sun_seen(const orc_optics *op, const double s[3], const double d[3])
{
    double a = op->sun_half_angle_deg * ORC_PI / 180.0;
    if (a <= 0.0) return 0.0;
    return (d[0] * s[0] + d[1] * s[1] + d[2] * s[2] >= cos(a)) ? op->S / (ORC_PI * sin(a) * sin(a)) : 0.0;
}

/* ========================================================================
 * Camera (Section 4.1 and Table 3): pinhole with a vertical field of view,
 * or orthographic; row 0 is the top of the image; the direction is sampled
 * uniformly over the pixel's footprint on the image plane.
 * ======================================================================== */
static void camera_ray(const orc_camera *c, int px, int py, double u1, double u2, double o[3], double d[3])
{
    double f[3], r[3], u[3];
    int a;
    for (a = 0; a < 3; ++a) f[a] = c->target[a] - c->pos[a];
    normalize3(f);
    cross3(f, c->up, r);
    normalize3(r);
    cross3(r, f, u);
    if (c->type == 0) {
        double th = tan(0.5 * c->fov_y_deg * ORC_PI / 180.0);
        double aspect = (double)c->width / (double)c->height;
        double sx = (2.0 * (px + u1) / c->width - 1.0) * th * aspect;
        double sy = (1.0 - 2.0 * (py + u2) / c->height) * th;
        for (a = 0; a < 3; ++a) { o[a] = c->pos[a]; d[a] = f[a] + sx * r[a] + sy * u[a]; }
        normalize3(d);
    } else if (c->type == 2) {
        /* horizontal sensor: pixel (px, py) of an ortho_w x ortho_h rectangle
         * centred at pos, px along +x, py along +y; looks up */
        o[0] = c->pos[0] + ((px + u1) / c->width - 0.5) * c->ortho_w;
        o[1] = c->pos[1] + ((py + u2) / c->height - 0.5) * c->ortho_h;
        o[2] = c->pos[2];
        d[0] = 0.0; d[1] = 0.0; d[2] = 1.0;
    } else {
        double sx = ((px + u1) / c->width - 0.5) * c->ortho_w;
        double sy = (0.5 - (py + u2) / c->height) * c->ortho_h;
        for (a = 0; a < 3; ++a) { o[a] = c->pos[a] + sx * r[a] + sy * u[a]; d[a] = f[a]; }
    }
}

void orc_camera_ray(const orc_camera *c, int px, int py, double u1, double u2, double *ray6)
{
    camera_ray(c, px, py, u1, u2, ray6, ray6 + 3);
}

/* ========================================================================
 * Backward radiance with the local estimate of the sun (Section 4.1, Fig. 4a).
 *
 * From the camera the path is tracked through the medium until it escapes
 * or is absorbed.  At every real collision and every ground hit the direct
 * sun is added: transmissivity from the event towards the sun, times the
 * probability density of scattering (or reflecting) the solar beam into the
 * tracked direction.  The volume collision is absorbing with probability
 * 1 - ssa(x) (analog absorption); the ground terminates with probability
 * 1 - rho; otherwise a new direction is drawn from the HG phase function or
 * the Lambertian (cosine) law.  Paths escaping upward contribute nothing
 * more, except a camera ray that escapes without any event inside the
 * solar disc (Section 4.1's direct sun; the scattered paths' sun is counted
 * by the local estimates only).  With a solar disc the local estimate's
 * direction is drawn uniformly in its cone (sun_sample).
 *
 * The oracle finds the next collision by path tracking (regular tracking,
 * an exact free path in the true field) and evaluates the sun's
 * transmissivity exactly as exp(-tau); both have the same expectation as the
 * null-collision estimators they check.  Contributions whose sun
 * transmissivity is below exp(-200) are dropped.
 *
 * A camera of type 2 is a horizontal sensor of the downward irradiance E
 * at its plane, reported as S times the transmissivity E / (S mu_sun): per
 * path, S times the sun's direct transmissivity to the point (with a disc:
 * along a direction w drawn in the cone, times cone_gain w_z / mu_sun), plus
 * pi / mu_sun times the radiance of a path started from the point in a
 * cosine-distributed upward direction (the cosine density is mu / pi, so
 * pi L estimates the diffuse irradiance).
 *
 * Per pixel: sum and sum of squares of the per-path radiance (units of S,
 * per steradian), over `spp` paths.  `pixels` lists the pixel indices
 * (row-major, row 0 top) to estimate; sum/sumsq are indexed like it.
 * counters: [0] real volume collisions, [1] ground hits, [2] paths.
 * ======================================================================== */
static double sun_transmissivity(const orc_field *f, const double x[3], const double s[3])
{
    double tau = orc_optical_depth_ray(f, x, s, 0.0, INFINITY, 200.0);
    return tau > 200.0 ? 0.0 : exp(-tau);
}

/* How a path's rays meet the medium.  g == NULL: path tracking (exact free
 * paths) and the exact sun transmissivity, as above.  g != NULL: the
 * null-collision algorithm of Section 2.3 in the grid's piecewise-constant
 * majorant m (kmax_c + k_g) for the free paths and for the sun rays (a sun
 * ray then reports 0 or 1), with the path's tentative collisions, nulls and
 * leaves entered counted in cnt. */
typedef struct {
    const orc_grid *g;
    double m;
    uint64_t cnt[3];
} orc_tracker;

/* Sun contribution `weight` times the transmissivity towards the sun along w;
 * no sun ray is traced for a zero weight. */
static double local_estimate(const orc_field *f, orc_tracker *tk, const double x[3], const double w[3], double weight,
                             orc_rng *r)
{
    if (!(weight > 0.0)) return 0.0;
    if (tk->g) return delta_hier(f, tk->g, tk->m, x, w, r, tk->cnt) ? weight : 0.0;
    return weight * sun_transmissivity(f, x, w);
}

static double radiance_path(const orc_field *f, const orc_optics *op, const double s[3], double o_in[3],
                            double d_in[3], int primary, orc_rng *r, uint64_t *cnt, orc_tracker *tk)
{
    double o[3], d[3], L = 0.0, gain = cone_gain(op);
    int order = 0, a, segs = 0;
    for (a = 0; a < 3; ++a) { o[a] = o_in[a]; d[a] = d_in[a]; }
    for (;;) {
        double tc, kc;
        int hit;
        if (tk->g) {
            if (++segs > op->max_segments) break;
            hit = delta_hier_walk(f, tk->g, tk->m, o, d, r, tk->cnt, &tc, &kc);
        } else {
            double tau_s = -log(1.0 - rng_u01(r));
            if (++segs > op->max_segments) break;
            hit = regular_free_path(f, o, d, 0.0, tau_s, &tc, &kc);
        }
        if (hit) {
            double x[3], k = kc + f->k_gas, ssa = op->ssa * kc / k, mu_sun, nd[3];
            for (a = 0; a < 3; ++a) x[a] = o[a] + tc * d[a];
            if (cnt) cnt[0]++;
            order++;
            if (op->max_scatter >= 0 && order > op->max_scatter) break;
            {
                double w[3];
                sun_sample(op, s, r, w);
                mu_sun = d[0] * w[0] + d[1] * w[1] + d[2] * w[2];
                L += local_estimate(f, tk, x, w, ssa * phase_eval(op, mu_sun) * op->S * gain, r);
            }
            if (op->max_scatter >= 0 && order >= op->max_scatter) break;
            if (rng_u01(r) >= ssa) break;
            {
                double mu = phase_sample(op, rng_u01(r));
                double phi = 2.0 * ORC_PI * rng_u01(r);
                rotate_about(d, mu, phi, nd);
            }
            for (a = 0; a < 3; ++a) { o[a] = x[a]; d[a] = nd[a]; }
        } else if (d[2] < 0.0) {
            double tg = -o[2] / d[2], x[3], nd[3];
            for (a = 0; a < 3; ++a) x[a] = o[a] + tg * d[a];
            x[2] = 0.0;
            if (cnt) cnt[1]++;
            order++;
            if (op->max_scatter >= 0 && order > op->max_scatter) break;
            {
                double w[3];
                sun_sample(op, s, r, w);
                if (w[2] > 0.0) L += local_estimate(f, tk, x, w, (op->rho / ORC_PI) * op->S * gain * w[2], r);
            }
            if (op->max_scatter >= 0 && order >= op->max_scatter) break;
            if (rng_u01(r) >= op->rho) break;
            {
                double u1 = rng_u01(r), u2 = rng_u01(r);
                double rr = sqrt(u1), phi = 2.0 * ORC_PI * u2;
                nd[0] = rr * cos(phi);
                nd[1] = rr * sin(phi);
                nd[2] = sqrt(fmax(0.0, 1.0 - u1));
            }
            for (a = 0; a < 3; ++a) { o[a] = x[a]; d[a] = nd[a]; }
        } else {
            /* escaped upward; a camera ray that met nothing may look into the sun's disc */
            if (primary && order == 0) L += sun_seen(op, s, d);
            break;
        }
    }
    return L;
}

/* Spectral integration by a k-distribution (Section 4.1: a quadrature point
 * of the band is sampled per path): point i with probability w_i / sum w,
 * whose gas extinction replaces the field's for the whole path.  The
 * estimate's expectation is sum_i w_i L(k_gas,i) / sum w. */
static double kd_pick(const orc_optics *op, double u)
{
    double tot = 0.0, acc = 0.0;
    int i;
    for (i = 0; i < op->kd_n; ++i) tot += op->kd_w[i];
    for (i = 0; i < op->kd_n - 1; ++i) {
        acc += op->kd_w[i];
        if (u * tot < acc) return op->kd_k[i];
    }
    return op->kd_k[op->kd_n - 1];
}

static void render_pixels(const orc_field *f, const orc_optics *op, const orc_camera *cam, int32_t spp,
                          uint64_t seed, const int32_t *pixels, int32_t npix, double *sum, double *sumsq,
                          uint64_t *counters, const orc_grid *g, double *path_stats)
{
    double s[3];
    int i, k, c;
    sun_dir(op, s);
    for (i = 0; i < npix; ++i) {
        int p = pixels[i], px = p % cam->width, py = p / cam->width;
        double acc = 0.0, acc2 = 0.0;
        for (k = 0; k < spp; ++k) {
            orc_rng r;
            double o[3], d[3], L;
            orc_field fk = *f;      /* the path's medium (its gas extinction under a k-distribution) */
            orc_tracker tk = {g, op->majorant_scale, {0, 0, 0}};
            rng_init(&r, seed, ((uint64_t)p << 24) + (uint64_t)k);
            if (op->kd_n > 0) fk.k_gas = kd_pick(op, rng_u01(&r));
            {
                double u1 = rng_u01(&r), u2 = rng_u01(&r);
                camera_ray(cam, px, py, u1, u2, o, d);
            }
            if (cam->type == 2) {
                double w[3];
                sun_sample(op, s, &r, w);
                L = (s[2] > 0.0 && w[2] > 0.0)
                        ? local_estimate(&fk, &tk, o, w, op->S * cone_gain(op) * (w[2] / s[2]), &r)
                        : 0.0;
                if (op->max_scatter != 0 && s[2] > 0.0) {
                    double v1 = rng_u01(&r), v2 = rng_u01(&r), rr = sqrt(v1), phi = 2.0 * ORC_PI * v2;
                    d[0] = rr * cos(phi);
                    d[1] = rr * sin(phi);
                    d[2] = sqrt(fmax(0.0, 1.0 - v1));
                    L += ORC_PI / s[2] * radiance_path(&fk, op, s, o, d, 0, &r, counters, &tk);
                }
            } else {
                L = radiance_path(&fk, op, s, o, d, 1, &r, counters, &tk);
            }
            if (counters) counters[2]++;
            if (path_stats)
                for (c = 0; c < 3; ++c) {
                    path_stats[c] += (double)tk.cnt[c];
                    path_stats[3 + c] += (double)tk.cnt[c] * (double)tk.cnt[c];
                }
            acc += L;
            acc2 += L * L;
        }
        sum[i] = acc;
        sumsq[i] = acc2;
    }
}

void orc_render(const orc_field *f, const orc_optics *op, const orc_camera *cam, int32_t spp, uint64_t seed,
                const int32_t *pixels, int32_t npix, double *sum, double *sumsq, uint64_t *counters)
{
    render_pixels(f, op, cam, spp, seed, pixels, npix, sum, sumsq, counters, NULL, NULL);
}

/* The same estimate with every ray tracked by the null-collision algorithm
 * in the grid's majorant op->majorant_scale (kmax_c + k_g) (O4b: free paths
 * and delta-tracked sun rays, leaf by leaf), for the expected event counts of
 * the GPU renderer with delta-tracked sun rays.  path_stats[6]: sums over
 * paths of the path's tentative collisions, null collisions and leaves
 * entered (all its rays), then the sums of their squares. */
void orc_render_tracked(const orc_field *f, const orc_grid *g, const orc_optics *op, const orc_camera *cam,
                        int32_t spp, uint64_t seed, const int32_t *pixels, int32_t npix, double *sum, double *sumsq,
                        uint64_t *counters, double *path_stats)
{
    render_pixels(f, op, cam, spp, seed, pixels, npix, sum, sumsq, counters, g, path_stats);
}

/* ========================================================================
 * Forward photons and the ground transmissivity under a cloud, with its
 * parametric sensitivities (Section 5.1; the derivative of the integral
 * formulation, Eq. 3, generalised from the direct transmissivity to paths
 * with scattering).
 *
 * The sun lights the top of the box uniformly: photons start at a uniform
 * point of the top face going along -omega_sun.  They are tracked with
 * analog absorption (probability 1 - ssa(x)) and HG scattering; at the
 * ground an arrival inside the box's footprint is tallied in its ground
 * pixel (px_nx x px_ny pixels over the footprint, pixel (i, j) = index
 * j px_nx + i, i along x), then the photon is reflected with probability
 * rho (Lambertian) or stops.  Every photon ends in exactly one of: escape
 * upward, absorption by the ground inside / outside the footprint,
 * absorption in the volume.
 *
 * Per arrival the tallies receive 1 (transmissivity; "direct" if the photon
 * was never scattered or reflected) and the accumulated scores
 *   sigma_s = sum over tentative collisions of d ln(probability)/d s, with
 *             k = s k_c + k_g and a majorant that does not depend on s:
 *             real: k_c / k;  null: -k_c / (k_hat - k);  and, at each
 *             scattering, d ln ssa(x) / d s = k_g / (s k),
 *   sigma_g = sum over HG scatterings of d ln p(mu) / d g,
 *   sigma_a = sum over scatterings of d ln ssa(x) / d alpha = -1 / (1 - alpha)
 *             for the droplets' absorptivity alpha = 1 - ssa (the
 *             sensitivity of Section 5.1; an absorbed photon arrives
 *             nowhere, so absorption events need no term),
 * so that the derivative estimates are the means of (arrival) x sigma.
 * The scores need the tentative collisions of null-collision tracking
 * (mode 2: the grid's majorant m (s kmax_c + k_g)); mode 0 tracks with exact
 * free paths and reports the transmissivity only.
 *
 * tally[9][px_ny][px_nx]: T sum, T sum of squares, direct-T sum,
 *   dT/ds sum, dT/ds sum of squares, dT/dg sum, dT/dg sum of squares,
 *   dT/dalpha sum, dT/dalpha sum of squares
 *   (per-arrival values; the caller scales by A_top / (N a_pixel)).
 * glob[4]: up-escapes, ground absorptions in / out of the footprint,
 *   volume absorptions.
 * ======================================================================== */
double orc_hg_dlng(double g, double mu)
{
    return -2.0 * g / (1.0 - g * g) - 3.0 * (g - mu) / (1.0 + g * g - 2.0 * g * mu);
}

/* Next real collision by hierarchical delta tracking, accumulating the
 * scale score of every tentative collision into *sig_s. */
static int delta_hier_scored(const orc_field *f, const orc_grid *g, double m, const double o[3], const double d[3],
                             orc_rng *r, double *tcoll, double *kd_at, double *sig_s)
{
    walker w;
    double tau_s;
    if (!walker_init(&w, f, o, d, 0.0)) return 0;
    tau_s = -log(1.0 - rng_u01(r));
    for (;;) {
        int axis;
        double te = walker_exit(&w, &axis);
        double khat = m * (f->kscale * leaf_kmax_c(f, g, w.idx[0], w.idx[1], w.idx[2], NULL, NULL) + f->k_gas);
        while (te > w.t && khat > 0.0 && tau_s < khat * (te - w.t)) {
            double kc, k;
            w.t += tau_s / khat;
            kc = cell_kc(f, w.idx[0], w.idx[1], w.idx[2]);
            k = f->kscale * kc + f->k_gas;
            if (rng_u01(r) * khat < k) {
                *sig_s += kc / k;
                *tcoll = w.t;
                *kd_at = f->kscale * kc;
                return 1;
            }
            *sig_s -= kc / (khat - k);
            tau_s = -log(1.0 - rng_u01(r));
        }
        if (te > w.t) tau_s -= khat * (te - w.t);
        if (!walker_advance(&w, te, axis)) return 0;
    }
}

typedef struct { int pix; int direct; double ss, sg, sa; } orc_arrival;

/* One photon; returns the number of arrivals stored (at most cap). */
static int photon_walk(const orc_field *f, const orc_grid *g, const orc_optics *op, int mode, orc_rng *r,
                       int px_nx, int px_ny, orc_arrival *arr, int cap, double *glob)
{
    double s[3], o[3], d[3], sig_s = 0.0, sig_g = 0.0, sig_a = 0.0;
    double Lx = f->nx * f->dx, Ly = f->ny * f->dy;
    int a, scattered = 0, n = 0, segs = 0;
    sun_dir(op, s);
    o[0] = f->x0 + rng_u01(r) * Lx;
    o[1] = f->y0 + rng_u01(r) * Ly;
    o[2] = f->z0 + f->nz * f->dz;
    for (a = 0; a < 3; ++a) d[a] = -s[a];
    for (;;) {
        double tc = 0.0, kd = 0.0;
        int hit;
        if (++segs > op->max_segments) return n;
        if (mode == 0)
            hit = regular_free_path(f, o, d, 0.0, -log(1.0 - rng_u01(r)), &tc, &kd);
        else
            hit = delta_hier_scored(f, g, op->majorant_scale, o, d, r, &tc, &kd, &sig_s);
        if (hit) {
            double k = kd + f->k_gas, ssa = op->ssa * kd / k, nd[3];
            for (a = 0; a < 3; ++a) o[a] = o[a] + tc * d[a];
            if (rng_u01(r) >= ssa) { glob[3] += 1.0; return n; }
            if (f->k_gas > 0.0) sig_s += f->k_gas / (f->kscale * k);
            /* survival has probability (1 - alpha) k_d / k: d ln / d alpha = -1 / (1 - alpha) */
            sig_a -= 1.0 / op->ssa;
            {
                double mu = orc_hg_sample_mu(op->g, rng_u01(r));
                double phi = 2.0 * ORC_PI * rng_u01(r);
                rotate_about(d, mu, phi, nd);
                sig_g += orc_hg_dlng(op->g, mu);
            }
            for (a = 0; a < 3; ++a) d[a] = nd[a];
            scattered = 1;
        } else if (d[2] < 0.0) {
            double tg = -o[2] / d[2], x[3];
            int inside;
            for (a = 0; a < 3; ++a) x[a] = o[a] + tg * d[a];
            x[2] = 0.0;
            inside = x[0] >= f->x0 && x[0] < f->x0 + Lx && x[1] >= f->y0 && x[1] < f->y0 + Ly;
            if (inside) {
                int i = (int)floor((x[0] - f->x0) / Lx * px_nx), j = (int)floor((x[1] - f->y0) / Ly * px_ny);
                if (i > px_nx - 1) i = px_nx - 1;
                if (j > px_ny - 1) j = px_ny - 1;
                if (n < cap) {
                    arr[n].pix = j * px_nx + i;
                    arr[n].direct = !scattered;
                    arr[n].ss = sig_s;
                    arr[n].sg = sig_g;
                    arr[n].sa = sig_a;
                    n++;
                }
            }
            if (rng_u01(r) >= op->rho) { glob[inside ? 1 : 2] += 1.0; return n; }
            {
                double u1 = rng_u01(r), u2 = rng_u01(r), rr = sqrt(u1), phi = 2.0 * ORC_PI * u2;
                d[0] = rr * cos(phi);
                d[1] = rr * sin(phi);
                d[2] = sqrt(fmax(0.0, 1.0 - u1));
            }
            for (a = 0; a < 3; ++a) o[a] = x[a];
            scattered = 1;
        } else {
            glob[0] += 1.0;
            return n;
        }
    }
}

#define ORC_MAX_ARRIVALS 4096

void orc_flux(const orc_field *f, const orc_grid *g, const orc_optics *op, int32_t mode, int32_t px_nx,
              int32_t px_ny, int64_t n_photons, uint64_t seed, uint64_t photon_offset, double *tally, double *glob)
{
    size_t np = (size_t)px_nx * px_ny;
    int64_t p;
    orc_arrival *arr = (orc_arrival *)malloc(sizeof(orc_arrival) * ORC_MAX_ARRIVALS);
    for (p = 0; p < n_photons; ++p) {
        orc_rng r;
        int n, i;
        rng_init(&r, seed, (uint64_t)(photon_offset + p));
        n = photon_walk(f, g, op, mode, &r, px_nx, px_ny, arr, ORC_MAX_ARRIVALS, glob);
        for (i = 0; i < n; ++i) {
            size_t q = (size_t)arr[i].pix;
            tally[0 * np + q] += 1.0;
            tally[1 * np + q] += 1.0;
            tally[2 * np + q] += arr[i].direct;
            tally[3 * np + q] += arr[i].ss;
            tally[4 * np + q] += arr[i].ss * arr[i].ss;
            tally[5 * np + q] += arr[i].sg;
            tally[6 * np + q] += arr[i].sg * arr[i].sg;
            tally[7 * np + q] += arr[i].sa;
            tally[8 * np + q] += arr[i].sa * arr[i].sa;
        }
    }
    free(arr);
}

/* Central finite differences with common random numbers: each photon is
 * traced twice with identical random streams and exact free paths (path
 * tracking), at parameter + h and - h (which = 0: extinction scale s,
 * which = 1: asymmetry g, which = 2: droplet absorptivity alpha = 1 - ssa).  With exact free-path inversion and inverse-CDF
 * HG sampling the trajectories move continuously with the parameter.
 * out[2][px_ny][px_nx]: sum and sum of squares over photons of the
 * per-photon quotient (arrivals(+h) - arrivals(-h)) / (2h) in each pixel;
 * tot[2]: the same for the quotient summed over all pixels. */
void orc_flux_fd(const orc_field *f_in, const orc_optics *op_in, int32_t which, double h, int32_t px_nx,
                 int32_t px_ny, int64_t n_photons, uint64_t seed, uint64_t photon_offset, double *out, double *tot)
{
    size_t np = (size_t)px_nx * px_ny;
    int64_t p;
    orc_arrival *ap = (orc_arrival *)malloc(sizeof(orc_arrival) * ORC_MAX_ARRIVALS);
    orc_arrival *am = (orc_arrival *)malloc(sizeof(orc_arrival) * ORC_MAX_ARRIVALS);
    double glob[4];
    for (p = 0; p < n_photons; ++p) {
        orc_field fp = *f_in, fm = *f_in;
        orc_optics opp = *op_in, opm = *op_in;
        orc_rng r;
        int np_, nm_, i, j;
        if (which == 0) { fp.kscale += h; fm.kscale -= h; }
        else if (which == 1) { opp.g += h; opm.g -= h; }
        else { opp.ssa -= h; opm.ssa += h; }
        rng_init(&r, seed, (uint64_t)(photon_offset + p));
        np_ = photon_walk(&fp, NULL, &opp, 0, &r, px_nx, px_ny, ap, ORC_MAX_ARRIVALS, glob);
        rng_init(&r, seed, (uint64_t)(photon_offset + p));
        nm_ = photon_walk(&fm, NULL, &opm, 0, &r, px_nx, px_ny, am, ORC_MAX_ARRIVALS, glob);
        if (tot) {
            double q = (np_ - nm_) / (2.0 * h);
            tot[0] += q;
            tot[1] += q * q;
        }
        /* net arrival difference per pixel touched by this photon */
        for (i = 0; i < np_ + nm_; ++i) {
            int pix = i < np_ ? ap[i].pix : am[i - np_].pix, seen = 0, cnt = 0;
            for (j = 0; j < i; ++j)
                if ((j < np_ ? ap[j].pix : am[j - np_].pix) == pix) { seen = 1; break; }
            if (seen) continue;
            for (j = 0; j < np_; ++j) cnt += ap[j].pix == pix;
            for (j = 0; j < nm_; ++j) cnt -= am[j].pix == pix;
            if (cnt != 0) {
                double q = cnt / (2.0 * h);
                out[pix] += q;
                out[np + pix] += q * q;
            }
        }
    }
    free(ap);
    free(am);
}
