/*
 * nctrace.h -- C ABI of the null-collision path tracer for MI355X (gfx950).
 *
 * The library implements the method of Villefranque et al. (JAMES 2019,
 * "Path-tracing Monte Carlo library for 3D radiative transfer in highly
 * resolved cloudy atmospheres"): a hierarchical grid of per-node minimum and
 * maximum extinction is built over a voxel field (Section 3.1), and
 * radiances, transmissivities and fluxes are estimated by null-collision
 * (maximum cross-section) path sampling through it (Sections 2.3 and 4.1).
 *
 * Conventions for every entry point
 *   - Lengths are km, extinction coefficients km^-1, angles degrees.
 *   - A field is a contiguous float32 array [nz][ny][nx] (x fastest) of the
 *     condensed-phase extinction k_c >= 0; a uniform gas k_gas (pure
 *     absorber) is added inside the field's box.  Outside the box is vacuum;
 *     the ground is the plane z = 0 (the box must satisfy z0 >= 0).
 *   - Pointers named d_* are caller-owned DEVICE buffers on the context's
 *     device; the library never frees them.  Structs are passed as host
 *     pointers and are read during the call only.
 *   - Handles (nc_ctx, nc_grid) are library-owned; release them with the
 *     matching destroy call.
 *   - Calls enqueue work on the context's stream and return; results are
 *     valid once that stream is synchronised.  nc_grid_build synchronises
 *     (it reads back the field-validation flag).
 *   - Every call returns an nc_status.  Arguments are validated before any
 *     work is enqueued; on error nothing is written to the outputs and
 *     nc_last_error() describes the problem.  Calls never abort the process.
 *   - Determinism: the same seed, sample offset and inputs reproduce every
 *     path exactly (counter-based Philox4x32-10 random numbers); FP64
 *     accumulations may differ in the last bits through atomic ordering.
 *   - A context owns a small device scratch area (work-queue head, launch
 *     parameters): calls on one context must not overlap in time on
 *     different streams.  Use one context per stream for concurrent work.
 */
#ifndef NCTRACE_H
#define NCTRACE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NC_ABI_VERSION 1u
#define NC_MAX_LEVELS 24

typedef int32_t nc_status;
#define NC_OK 0
#define NC_ERR_INVALID_ARG 1   /* null pointer, bad size, bad enum */
#define NC_ERR_RANGE 2         /* NaN/Inf/negative extinction, g outside (-1,1), albedo outside [0,1], ... */
#define NC_ERR_OOM 3           /* device allocation failed */
#define NC_ERR_DEVICE 4        /* no usable device, or a HIP runtime error */
#define NC_ERR_UNSUPPORTED 5
#define NC_ERR_STATE 6         /* grid built for another field shape */

typedef struct nc_ctx nc_ctx;
typedef struct nc_grid nc_grid;
typedef struct nc_phase nc_phase;

/* Voxel field geometry: box [x0, x0+nx dx] x [y0, y0+ny dy] x [z0, z0+nz dz]. */
typedef struct {
    int32_t nx, ny, nz, pad_;
    double x0, y0, z0, dx, dy, dz;
} nc_field_desc;

/* Merge rule of the acceleration grid (Section 3.1.1, criterion of Section 4.2).
 * A node of level l (2^l cells per side, clipped to the field) is one voxel of
 * the grid when its optical-depth criterion, evaluated in double precision, is
 *   criterion 0: (kmax_c + k_gas) * dz * 2^l < tau_tilde    (default)
 *   criterion 1: (kmax_c - kmin_c) * dz * 2^l < tau_tilde
 *   criterion 2: l <= flat_level, whatever the field: the flat, single-level
 *                majorant grid of 2^flat_level-cell supercells that the
 *                hierarchy is compared with (Sections 2.4, 3); tau_tilde unused
 *   criterion 3: the node lies wholly below or above the cloudy layer (the z
 *                range of the cells with k_c > 0), or l <= flat_level: the
 *                layered grid of Section 3.1.1's comparison (clear layers
 *                split from the cloudy one, a resolution for each); clear
 *                layers take the coarsest nodes that stay clear, the cloudy
 *                layer 2^flat_level-cell supercells; tau_tilde unused
 * tau_tilde = 0 keeps the raw resolution; tau_tilde = +inf gives one voxel. */
typedef struct {
    double tau_tilde;
    double k_gas;
    int32_t criterion;
    int32_t flat_level;     /* criteria 2 and 3, 0..NC_MAX_LEVELS */
} nc_grid_params;

/* Medium, ground and sun.  ssa is the droplets' single-scattering albedo
 * (the local albedo is ssa k_c / (k_c + k_gas)); g the Henyey-Greenstein
 * asymmetry; ground_albedo the Lambertian reflectivity of z = 0; the sun is
 * directional, azimuth measured from +X towards +Y, irradiance normal to the
 * beam sun_irradiance.  The null-collision majorant of a voxel is
 * majorant_scale * (kmax_c + k_gas), majorant_scale >= 1.  max_scatter >= 0
 * limits the number of scattering/reflection events whose sun contribution
 * is counted (-1: unlimited); max_segments caps tracking steps per path
 * (paths reaching it are stopped and counted as truncated).
 * sun_half_angle_deg > 0 makes the sun a disc of that angular radius (the
 * solar cone of Section 4.1) with uniform radiance S / (pi sin^2 alpha), S =
 * sun_irradiance through a plane normal to its centre: local estimates go
 * along a direction drawn uniformly in the cone (weight 2 / (1 + cos alpha)),
 * and a camera ray that escapes without any event inside the disc sees it;
 * 0 is the directional sun; [0, 90) degrees, and for a sensor (camera type 2)
 * zenith + half angle < 90.  nc_flux and nc_flux_adjoint take the directional
 * sun only (NC_ERR_UNSUPPORTED otherwise).
 * phase: a tabulated phase function (nc_phase_create) that replaces HG(g) in
 * the renderers (local estimates, scattering, the guided step's MIS weight
 * and its phase-function candidate); NULL = HG.  It must live on the
 * context's device; nc_flux and nc_flux_adjoint take HG only.
 * kdist: a k-distribution (host struct, read at the call): the renderers draw
 * one quadrature point per path (Section 4.1), whose gas extinction replaces
 * the grid's k_gas along the whole path; the grid's majorant stays the
 * grid's, so every point's k_gas must be <= the grid's k_gas (one grid shared
 * by all points; NC_ERR_RANGE otherwise).  NULL = the grid's k_gas.  Not
 * taken by nc_transmittance, nc_flux, nc_flux_adjoint (NC_ERR_UNSUPPORTED). */
#define NC_KDIST_MAX 16
typedef struct {
    int32_t n;                     /* 1 .. NC_KDIST_MAX points */
    int32_t pad_;
    double w[NC_KDIST_MAX];        /* weights >= 0, normalised by the library */
    double k_gas[NC_KDIST_MAX];    /* gas extinction per point, km^-1, >= 0 */
} nc_kdist;
typedef struct {
    double ssa, g, ground_albedo;
    double sun_zenith_deg, sun_azimuth_deg, sun_irradiance;
    double majorant_scale;
    int32_t max_scatter;
    int32_t max_segments;
    double sun_half_angle_deg;
    const nc_phase *phase;
    const nc_kdist *kdist;
} nc_optics;

/* Camera (Section 4.1, Table 3): type 0 pinhole with vertical field of view
 * fov_y_deg, type 1 orthographic of extent ortho_w x ortho_h; forward =
 * target - pos, right = forward x up, row 0 is the top of the image, pixel
 * (i, j) is index j*width + i; directions are sampled uniformly over the
 * pixel's footprint on the image plane.
 * Type 2 is a horizontal irradiance sensor (the ground pixels of the
 * flux estimate, Section 5.1, traced backwards): an ortho_w x ortho_h
 * rectangle centred at pos in the plane z = pos[2], pixel (i, j) with i
 * along +x and j along +y (as nc_flux's ground pixels); target and up are
 * ignored.  A sensor path adds the sun's direct transmissivity to a uniform
 * point of the pixel and pi / cos(theta_sun) times the radiance of a path
 * leaving it in a cosine-distributed upward direction, so its expectation is
 * the downward irradiance over sun_irradiance * cos(theta_sun) (the
 * transmissivity) times sun_irradiance.  It needs the sun above the horizon
 * (NC_ERR_RANGE otherwise). */
typedef struct {
    int32_t type;
    int32_t width, height;
    int32_t pad_;
    double pos[3], target[3], up[3];
    double fov_y_deg, ortho_w, ortho_h;
} nc_camera;

/* Estimators of the sun's transmissivity in the local estimate (bits 0-1
 * of nc_sampling.flags).  Section 4.1 evaluates the direct sun with
 * decomposition tracking (Novak et al. 2014; Kutz et al. 2017):
 *   NC_SUN_DELTA     null-collision (delta) tracking: 0 or 1 per sun ray;
 *   NC_SUN_RATIO     ratio tracking: the product of 1 - k/k_hat over the
 *                    tentative collisions to the box exit;
 *   NC_SUN_RESIDUAL  residual ratio tracking with each voxel's minimum
 *                    extinction as the control: exp(-integral of k_min)
 *                    times the product of 1 - (k - k_min)/(k_hat - k_min)
 *                    over collisions sampled with the residual majorant.
 * The ratio estimators play Russian roulette below a transmissivity of 0.1.
 * All three have the same expectation. */
#define NC_SUN_DELTA 0
#define NC_SUN_RATIO 1
#define NC_SUN_RESIDUAL 2
#define NC_SUN_ESTIMATOR_MASK 3
/* nc_flux and nc_flux_adjoint (bit 2 of nc_sampling.flags): apply the
 * estimator's normalisation px_nx * px_ny / n_photons (ground flux over the
 * flux through the top face, per unit area) inside the kernels, so that the
 * tallies are the transmissivity map and its derivatives and the adjoint
 * output is dL/ds, dL/dg, dL/dalpha (see nc_flux). */
#define NC_FLUX_NORMALISE 4

/* Sampling: seed keys the random streams; sample s of pixel p of job j uses
 * the Philox counter (p, sample_offset + s, draw, stream + j), so a run with
 * sample_offset = n continues one that took n samples per pixel, and runs
 * with different `stream` values are independent.  guide_frac and
 * guide_max_order concern nc_render_guided only: the probability of drawing
 * from the guide at a scattering, and the last scattering order that is
 * guided (0: every order; the weights of guided events multiply along a
 * path, so guiding only the first orders bounds their spread). */
typedef struct {
    uint64_t seed;
    uint64_t sample_offset;
    int32_t spp;
    int32_t flags;
    double guide_frac;
    uint32_t stream;
    uint32_t guide_max_order;
} nc_sampling;

/* Per-call event counters (summed over all paths of the call). */
typedef struct {
    uint64_t paths;          /* paths completed */
    uint64_t segments;       /* tracking steps: voxel visits + tentative collisions */
    uint64_t tentative;      /* tentative collisions sampled in the majorant field */
    uint64_t nulls;          /* rejected (null) collisions */
    uint64_t reals;          /* accepted collisions (path and sun rays) */
    uint64_t leaf_visits;    /* acceleration-grid voxels entered */
    uint64_t gathers;        /* raw field reads for the null/real test */
    uint64_t node_reads;     /* grid node reads from global memory */
    uint64_t nee_rays;       /* sun rays traced */
    uint64_t truncated;      /* paths stopped at max_segments */
    uint64_t sched[24];      /* renderer scheduling, per phase (step = voxel crossings and ray
                                starts, collision, event, (unused), sample, guide network):
                                [0..5] wave trips, [6..11] active lanes summed over the trips,
                                [12..17] wave wall-clock ticks spent in the phase; [18] voxels
                                entered whose level is not staged in LDS (the
                                method's grid reads from memory: leaf_visits less those served
                                from LDS); [19..23] unused */
} nc_counters;

/* A tabulated phase function (Section 4.1 takes the droplets' phase function
 * from Mie tables): values h_p[i] >= 0 at cosines h_mu[i] (host arrays, n >= 2,
 * h_mu[0] = -1 < ... < h_mu[n-1] = 1), linear in the cosine between nodes,
 * scaled by the library so that 2 pi times its integral is 1 (per
 * steradian).  Sampling inverts its piecewise-quadratic CDF.  The object holds
 * device copies (float32 cosines, values and CDF at the nodes) and may be
 * shared by any number of nc_optics on its device.  NC_ERR_RANGE for a bad
 * table. */
nc_status nc_phase_create(nc_ctx *ctx, const double *h_mu, const double *h_p, int32_t n, nc_phase **out);
void nc_phase_destroy(nc_phase *phase);
/* The phase function's sampler and value on the GPU (for testing): for n
 * uniforms d_u in [0,1), d_out[2i] = the sampled cosine, d_out[2i+1] = the
 * phase function at it (per steradian).  Device float arrays. */
nc_status nc_phase_sample(nc_ctx *ctx, const nc_phase *phase, const float *d_u, int32_t n, float *d_out);

/* Library ABI version (NC_ABI_VERSION). */
uint32_t nc_abi_version(void);

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  NC_ERR_DEVICE if the device
 * is missing. */
nc_status nc_ctx_create(int32_t device, void *hip_stream, nc_ctx **out);
nc_status nc_ctx_set_stream(nc_ctx *ctx, void *hip_stream);
void nc_ctx_destroy(nc_ctx *ctx);
/* Text of the last error on this context (or of the last failed
 * nc_ctx_create when ctx is NULL).  Valid until the next call. */
const char *nc_last_error(const nc_ctx *ctx);

/* Build the acceleration grid over d_kc (Section 3.1.1; Appendix B.3's
 * power-of-two octree, with nodes wholly outside the field left out).
 * Level 0 is the field itself; level l (1..L, L = ceil(log2 max(nx,ny,nz)))
 * has ceil(n/2^l) nodes per axis, each holding the min and max of k_c over
 * the cells it covers.  A cell's voxel is its coarsest ancestor that passes
 * the merge criterion (the cell itself if none does).  The field is checked
 * (finite and >= 0: else NC_ERR_RANGE).  The grid keeps no reference to
 * d_kc; estimators take the field again and check its shape. */
nc_status nc_grid_build(nc_ctx *ctx, const float *d_kc, const nc_field_desc *desc, const nc_grid_params *params,
                        nc_grid **out);
/* Rebuild `grid` in place over the field d_kc, which has the shape the grid
 * was built for (same levels, criterion and parameters; Section 3.1.1): for
 * a field that changes between renders (a time series, a new extinction
 * scale) without a new allocation.  Synchronises like nc_grid_build.  On
 * NC_ERR_RANGE (NaN, Inf or negative extinction) the grid's contents are
 * unspecified until a rebuild over a valid field succeeds. */
nc_status nc_grid_rebuild(nc_ctx *ctx, nc_grid *grid, const float *d_kc);
void nc_grid_destroy(nc_grid *grid);
/* Number of levels L above the cells, and the node counts of level l. */
nc_status nc_grid_info(const nc_grid *grid, int32_t *levels, int32_t level, int32_t dims_out[3]);
/* Copy level l (1..L) to caller buffers of dims[2]*dims[1]*dims[0] entries:
 * kmin_c, kmax_c (float32) and the merged flag (uint8, 1 = voxel of the grid
 * or inside one).  Any output pointer may be NULL. */
nc_status nc_grid_export(nc_ctx *ctx, const nc_grid *grid, int32_t level, float *d_kmin, float *d_kmax,
                         uint8_t *d_merged);
/* The ancestry mask the crossing reads (Section 3.1.3's descent from the
 * coarsest merged ancestor): one uint16 per level-1 node, [z][y][x] over
 * level 1's node counts, bit l (1..L) set if the node's level-l ancestor
 * (itself for l = 1) is merged.  d_mask: device, caller-owned.  A grid with
 * L = 0 has none (NC_ERR_INVALID_ARG). */
nc_status nc_grid_export_mask(nc_ctx *ctx, const nc_grid *grid, uint16_t *d_mask);
/* Per-cell voxel level (uint8 [nz][ny][nx]). */
nc_status nc_grid_leaf_levels(nc_ctx *ctx, const nc_grid *grid, uint8_t *d_leaf_level);

/* Ordered crossing of the grid (Section 3.1.3): for each of n rays
 * (d_rays: n x 6 float32, origin then unit direction) the voxels met inside
 * the box, in order: d_leaf[n][max_visits][4] = (level, ix, iy, iz) of the
 * voxel at that level, d_t[n][max_visits][2] = entry and exit parameters.
 * d_count[n] = number of voxels (may exceed max_visits; only max_visits are
 * written). */
nc_status nc_trace_leaves(nc_ctx *ctx, const nc_grid *grid, const float *d_rays, int32_t n, int32_t max_visits,
                          int32_t *d_leaf, float *d_t, int32_t *d_count);

/* Direct transmissivity by the null-collision algorithm of Section 2.3
 * (Eq. 2): for each ray, sampling->spp paths in the grid's piecewise-constant
 * majorant, each returning 0 or 1 (NC_SUN_DELTA) or a ratio-tracking
 * estimate (NC_SUN_RATIO, NC_SUN_RESIDUAL: bits 0-1 of sampling->flags);
 * d_sum[n], d_sumsq[n] (float64) receive the sum and sum of squares of the
 * path estimates.  The ground is not intersected (rays are cast through the
 * field's box only). */
nc_status nc_transmittance(nc_ctx *ctx, const nc_grid *grid, const float *d_kc, const nc_optics *optics,
                           const float *d_rays, int32_t n, const nc_sampling *sampling, double *d_sum,
                           double *d_sumsq, nc_counters *d_counters);

/* Radiance image by the backward algorithm with the local estimate of the
 * sun (Section 4.1, Fig. 4a): per pixel, spp paths from the camera; at each
 * real collision and ground hit the sun's transmissivity (null-collision
 * shadow ray) times the phase function (or Lambertian BRDF) is added; the
 * path then scatters (HG), reflects (cosine law) or is absorbed.  Output:
 * d_sum, d_sumsq [height*width] float64 sum and sum of squares of the path
 * radiances (units of sun_irradiance per steradian), ADDED to the buffers
 * (zero them first).  d_counters (device, may be NULL) is added to. */
nc_status nc_render(nc_ctx *ctx, const nc_grid *grid, const float *d_kc, const nc_optics *optics,
                    const nc_camera *camera, const nc_sampling *sampling, double *d_sum, double *d_sumsq,
                    nc_counters *d_counters);

/* Ground transmissivity under the field by forward photons, with its
 * sensitivities to the extinction scale s and to the HG asymmetry g
 * (Section 5.1; derivative of the integral formulation, Eq. 3).
 *
 * The sun (optics) lights the top face of the box uniformly: n_photons
 * photons start at uniform points of the top face going along -omega_sun,
 * photon i using random stream sampling->sample_offset + i.  The medium's
 * droplet extinction is extinction_scale * k_c; photons are tracked by
 * null-collision tracking in the grid's majorant
 * majorant_scale * (extinction_scale * kmax_c + k_gas) with analog
 * absorption and HG scattering; at the ground (z = 0) an arrival inside the
 * box footprint is tallied in ground pixel (i, j) of a px_nx x px_ny grid
 * over the footprint (i along x, index j*px_nx + i), then the photon is
 * reflected (Lambertian, probability ground_albedo) or stops.
 *
 * Each arrival adds, in pixel order [k][px_ny][px_nx] of d_tally (float64,
 * 9 x px_ny x px_nx, ADDED to the buffer):
 *   k=0: 1, k=1: 1 (sum of squares), k=2: 1 if the photon was never
 *   scattered or reflected (direct), k=3: sigma_s, k=4: sigma_s^2,
 *   k=5: sigma_g, k=6: sigma_g^2, k=7: sigma_a, k=8: sigma_a^2,
 * where sigma_s and sigma_g are the path's accumulated scores: real
 * collision + k_c/k, null collision - k_c/(k_hat - k), scattering
 * + k_gas/(s k); HG scattering of cosine mu + d ln p(mu)/dg; sigma_a, the
 * score of the droplets' absorptivity alpha = 1 - ssa (Section 5.1's
 * sensitivity), adds -1/(1 - alpha) per scattering.  The
 * transmissivity of pixel p is T_p = tally[0][p] * px_nx*px_ny / n_photons
 * (ground flux over the flux through the top, per unit area), and
 * dT_p/ds, dT_p/dg, dT_p/dalpha are tally[3][p], tally[5][p], tally[7][p]
 * times the same factor.  With NC_FLUX_NORMALISE in sampling->flags each
 * arrival adds f = px_nx*px_ny / n_photons times the values above (f^2 times
 * the squares), so that tally[0] = T_p, tally[2] = its direct part, and
 * tally[3], tally[5], tally[7] = dT_p/ds, dT_p/dg, dT_p/dalpha.
 * d_global[4] (float64, added): photons escaping upward, absorbed by the
 * ground inside / outside the footprint, absorbed in the volume; they sum to
 * n_photons. */
nc_status nc_flux(nc_ctx *ctx, const nc_grid *grid, const float *d_kc, const nc_optics *optics,
                  double extinction_scale, int32_t px_nx, int32_t px_ny, uint64_t n_photons,
                  const nc_sampling *sampling, double *d_tally, double *d_global, nc_counters *d_counters);

/* Derivative-path replay of nc_flux: the same photons (same sampling and
 * n_photons) are traced again and, at every arrival in pixel p, d_grad[p]
 * times the path's scores is accumulated: d_out[0] += sum grad[p] sigma_s,
 * d_out[1] += sum grad[p] sigma_g, d_out[2] += sum grad[p] sigma_a
 * (float64).  Multiplied by px_nx*px_ny / n_photons this is dL/ds, dL/dg
 * and dL/dalpha for L = sum_p grad[p] T_p; with NC_FLUX_NORMALISE in
 * sampling->flags the kernel applies that factor (d_out receives dL/ds,
 * dL/dg, dL/dalpha).
 * d_grad is float64 [px_ny][px_nx]. */
nc_status nc_flux_adjoint(nc_ctx *ctx, const nc_grid *grid, const float *d_kc, const nc_optics *optics,
                          double extinction_scale, int32_t px_nx, int32_t px_ny, uint64_t n_photons,
                          const nc_sampling *sampling, const double *d_grad, double *d_out);

/* ---------------------------------------------------------------------------
 * Learned proposal for scattering directions (path guiding).  An MLP
 * 15 -> 64 -> 64 -> 64 -> 40 (ReLU) maps a scattering vertex to a mixture of
 * 8 von Mises-Fisher lobes over the outgoing direction.  A vertex is 7
 * values: the position normalised to [-1, 1]^3 over the field's box, the
 * incoming direction, and ln(1 + k / 1 km^-1) at the vertex; the network's
 * 15 inputs are those 7, then sin and cos of 8 pi x, 8 pi y, 16 pi x and
 * 16 pi y of the normalised position.  Output j*5 + {0,1,2,3,4}:
 * lobe logit, unnormalised mean direction (3), log concentration (clamped to
 * [-3, 8]).  Products run in bf16 on the matrix cores with fp32
 * accumulation; master weights and Adam moments are fp32.  Parameters are
 * flat fp32, layer by layer: W [out][in] row-major, then b [out] (11944).
 * A training record is 12 floats: vertex values (7), outgoing direction (3),
 * weight (1), unused (1); the loss is -sum w ln q(w_out) / sum w.
 * ------------------------------------------------------------------------- */
typedef struct nc_guide nc_guide;
#define NC_GUIDE_PARAMS 11944
#define NC_GUIDE_RECORD 12

/* New network with He-uniform weights from `seed` and zero biases. */
nc_status nc_guide_create(nc_ctx *ctx, uint64_t seed, nc_guide **out);
void nc_guide_destroy(nc_guide *guide);
/* Copy the fp32 parameters to / from a device buffer of NC_GUIDE_PARAMS floats. */
nc_status nc_guide_get_params(nc_ctx *ctx, const nc_guide *guide, float *d_params);
nc_status nc_guide_set_params(nc_ctx *ctx, nc_guide *guide, const float *d_params);
/* Raw network outputs for n inputs (rows of `stride` floats, inputs first):
 * d_out is n x 48 floats (the 40 outputs, then padding). */
nc_status nc_guide_forward(nc_ctx *ctx, const nc_guide *guide, const float *d_in, int32_t n, int32_t stride,
                           float *d_out);
/* One Adam step (lr) on the loss of n records; d_loss (may be NULL) receives
 * [sum of -w ln q, sum of w] as float64. */
nc_status nc_guide_train_step(nc_ctx *ctx, nc_guide *guide, const float *d_records, int32_t n, float lr,
                              double *d_loss);
/* Gradient of the loss of n records (NC_GUIDE_PARAMS floats), no update. */
nc_status nc_guide_gradient(nc_ctx *ctx, nc_guide *guide, const float *d_records, int32_t n, float *d_grad,
                            double *d_loss);

/* Guided radiance image: nc_render, except that at a volume scattering
 * event the new direction is drawn with probability c =
 * sampling->guide_frac from the guide's vMF mixture q and otherwise from the
 * HG phase function p, and the path weight is multiplied by
 * p / (c q + (1 - c) p) (one-sample multiple importance sampling with the
 * balance heuristic, Veach 1997).  The estimate is unbiased for any network;
 * its variance depends on how closely q follows the light arriving at the
 * vertex.  Ground reflections keep the cosine law.  The network runs inside
 * the tracer (bf16 matrix cores, 16 vertices per product tile).  guide_frac
 * outside [0, 1] is NC_ERR_INVALID_ARG. */
nc_status nc_render_guided(nc_ctx *ctx, const nc_grid *grid, const float *d_kc, const nc_optics *optics,
                           const nc_camera *camera, const nc_sampling *sampling, const nc_guide *guide,
                           double *d_sum, double *d_sumsq, nc_counters *d_counters);

/* The guided scattering step of nc_render_guided on n given vertices (for
 * testing and inspection): the network on the matrix cores, then with
 * probability guide_frac a direction from the vMF mixture q, else from HG(g)
 * about the incoming direction.  d_in: n rows of 8 floats (the vertex's 7
 * values, of which 3..5 are the incoming direction; one unused); d_u: n rows
 * of 4 uniforms in [0,1): u0 picks the branch (mixture if u0 < guide_frac) and
 * then u0 / guide_frac the lobe, u1 is ignored, u2 and u3 give the cosine and
 * the azimuth (the renderer draws three numbers per step); d_out: n rows of 8
 * floats: new direction (3), weight factor p / (c q + (1 - c) p), q and p at
 * the new direction, 2 zeros.  All device float arrays. */
nc_status nc_guide_sample(nc_ctx *ctx, const nc_guide *guide, const float *d_in, const float *d_u, int32_t n,
                          float guide_frac, float g, float *d_out);

/* Progressive rendering to a target relative standard error.  Rounds of
 * nc_render (guide NULL) or nc_render_guided add samples with consecutive
 * sample offsets (the union of the rounds is one render of spp_done samples)
 * until eps <= target_rel_err or max_spp samples per pixel are done.
 * eps = sqrt(mean over units of SE_u^2) / mean over units of L_u, where a
 * unit is a block x block pixel block (block = 1: one pixel), L_u the block's
 * mean radiance and SE_u its standard error.  Each round after the first asks
 * for the samples the 1/sqrt(n) law predicts are missing (+5 %), at most
 * doubling the total.  The stream is synchronised after every round (the
 * error is read back).  d_sum/d_sumsq must start at zero. */
typedef struct {
    double target_rel_err;  /* e.g. 0.01 */
    int32_t first_spp;      /* samples per pixel of the first round (>= 2) */
    int32_t max_spp;        /* cap on the total */
    int32_t block;          /* pixel block side of the error estimate (>= 1) */
    int32_t pad_;
} nc_progressive;
typedef struct {
    int32_t spp_done;       /* samples per pixel taken */
    int32_t rounds;
    double rel_err;         /* eps after the last round */
    double mean;            /* mean radiance over the units */
    double seconds;         /* host wall time of all rounds */
} nc_progress_report;
nc_status nc_render_progressive(nc_ctx *ctx, const nc_grid *grid, const float *d_kc, const nc_optics *optics,
                                const nc_camera *camera, const nc_sampling *sampling, const nc_guide *guide,
                                const nc_progressive *plan, double *d_sum, double *d_sumsq, nc_counters *d_counters,
                                nc_progress_report *report);

/* Device random-read rate (not part of the method: the measured ceiling
 * of the tracers' roofline).  threads x loads independent 4-byte reads at
 * hashed addresses in d_buf[0 .. n_words) (n_words a power of two <= 2^32,
 * device float array; pick it larger than the last-level cache to measure
 * HBM); d_out receives one float per thread.  The second of two launches is
 * timed on the ctx stream (synchronised); *loads_per_s = reads per second. */
nc_status nc_gather_rate(nc_ctx *ctx, const float *d_buf, uint64_t n_words, int32_t threads, int32_t loads,
                         float *d_out, double *loads_per_s);

/* Training vertices for the guide: renders exactly as nc_render (same paths,
 * same d_sum/d_sumsq) and, at every volume scattering event after which the
 * path goes on, writes one NC_GUIDE_RECORD: the guide inputs at the vertex
 * (7), the sampled outgoing direction (3), as weight the radiance the path
 * gathered after the vertex (its final radiance minus what it held once the
 * vertex's own sun estimate was added), and in [11] the path's slot
 * (pixel * spp + sample) as uint32 bits.  d_records: device, capacity x 12
 * floats; *d_count (device uint64, overwritten) receives the number of
 * events, which may exceed capacity (the records past capacity are dropped,
 * in no defined order).  d_path_L: device scratch of width * height * spp
 * floats (per-path radiance), width * height * spp < 2^32. */
nc_status nc_collect_vertices(nc_ctx *ctx, const nc_grid *grid, const float *d_kc, const nc_optics *optics,
                              const nc_camera *camera, const nc_sampling *sampling, float *d_records,
                              uint64_t capacity, unsigned long long *d_count, float *d_path_L, double *d_sum,
                              double *d_sumsq, nc_counters *d_counters);

/* Counter-based random numbers (Salmon et al., SC'11): out[i] =
 * Philox4x32-10(counter = d_ctr[4i..4i+3], key = d_key[2i..2i+1]) for i < n.
 * All buffers are uint32 device arrays.  The path tracers draw their random
 * numbers from this generator; the entry point exposes it for testing. */
nc_status nc_philox4x32_10(nc_ctx *ctx, const uint32_t *d_ctr, const uint32_t *d_key, uint32_t *d_out, int32_t n);

/* Many views and suns in one persistent launch: job j renders camera cams[j]
 * under optics[j] into d_sum/d_sumsq starting at element out_offsets[j]
 * (host array; image j occupies cams[j].height * cams[j].width elements).
 * The medium's parameters (ssa, g, majorant_scale, max_scatter,
 * max_segments, the sun's half angle, the phase table, the k-distribution's
 * points) must be equal across jobs; the sun's direction and irradiance and
 * the ground albedo may differ.  Queue items of all jobs are
 * drawn from one work queue, so views of uneven size balance across the
 * GPU.  Random streams: job j uses stream sampling->stream + j. */
nc_status nc_render_batch(nc_ctx *ctx, const nc_grid *grid, const float *d_kc, int32_t n_jobs, const nc_camera *cams,
                          const nc_optics *optics, const uint64_t *out_offsets, const nc_sampling *sampling,
                          double *d_sum, double *d_sumsq, nc_counters *d_counters);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * nc_render_batch without any device allocation.  Its job table, launch
 * record and work-queue heads live in a fixed array inside the library
 * (NC_NOALLOC_MAX_JOBS job records, about 125 KB), one copy per GPU, held
 * until the process ends; its address on a device is resolved when the
 * first context is created there.  n_jobs above NC_NOALLOC_MAX_JOBS is
 * NC_ERR_INVALID_ARG.  Every call on a GPU uses that GPU's one array and
 * rewrites all of it that the launch reads (the queue heads are cleared by
 * a kernel), so a call never depends on an earlier one, but calls that
 * overlap in time on one GPU (any context, any stream) race and must not be
 * made.  Otherwise as nc_render_batch: same arguments, same images. */
#define NC_NOALLOC_MAX_JOBS 1024
nc_status nc_render_batch_noalloc(nc_ctx *ctx, const nc_grid *grid, const float *d_kc, int32_t n_jobs,
                                  const nc_camera *cams, const nc_optics *optics, const uint64_t *out_offsets,
                                  const nc_sampling *sampling, double *d_sum, double *d_sumsq,
                                  nc_counters *d_counters);

/* nc_render_batch with guided scattering (nc_render_guided) in every job,
 * job j guided by guides[j] (host array of n_jobs handles).  The network's
 * inputs do not include the sun, so a guide is trained for one sun and the
 * jobs of each sun take theirs, all in one persistent launch.  Jobs that
 * share a guide must be consecutive, in at most NC_BATCH_MAX_GUIDES runs
 * (NC_ERR_INVALID_ARG otherwise).  Each run's queue items form their own
 * work queues; a workgroup holds one run's network in LDS and takes work from
 * its queues, and once they are drained and its waves are idle it loads the
 * network of a run that still has work. */
#define NC_BATCH_MAX_GUIDES 8
nc_status nc_render_batch_guided(nc_ctx *ctx, const nc_grid *grid, const float *d_kc, int32_t n_jobs,
                                 const nc_camera *cams, const nc_optics *optics, const uint64_t *out_offsets,
                                 const nc_sampling *sampling, const nc_guide *const *guides, double *d_sum,
                                 double *d_sumsq, nc_counters *d_counters);

/* Launch-shape knobs of the path-tracing kernels (0 = library default). */
typedef struct {
    int32_t block;          /* threads per workgroup (multiple of 64, at most 256) */
    int32_t waves_per_cu;   /* resident waves per CU the persistent grid is sized for */
    int32_t samples_per_item; /* samples of one pixel taken by one lane per queue item */
    int32_t lds_levels;     /* top grid levels staged in LDS (-1: as many as fit) */
} nc_launch;
nc_status nc_set_launch(nc_ctx *ctx, const nc_launch *launch);
nc_status nc_get_launch(const nc_ctx *ctx, nc_launch *launch);

/* Autotuner: renders the given view with a few spp under candidate launch
 * shapes (samples per queue item, workgroup size, register budget, LDS-staged
 * levels), timing each with HIP events on the context's stream, and leaves
 * the fastest in the context (nc_get_launch reads it back).  d_sum/d_sumsq
 * are scratch images of the camera's size (overwritten).  *best_ms receives
 * the fastest time (may be NULL).  Synchronises the stream. */
nc_status nc_autotune_render(nc_ctx *ctx, const nc_grid *grid, const float *d_kc, const nc_optics *optics,
                             const nc_camera *camera, const nc_sampling *sampling, double *d_sum, double *d_sumsq,
                             double *best_ms);

/* The same autotuner on a batched launch (nc_render_batch with these jobs):
 * d_sum/d_sumsq are scratch buffers of the batch's outputs (overwritten).
 * The chosen shape stays in the context for the following launches. */
nc_status nc_autotune_batch(nc_ctx *ctx, const nc_grid *grid, const float *d_kc, int32_t n_jobs,
                            const nc_camera *cams, const nc_optics *optics, const uint64_t *out_offsets,
                            const nc_sampling *sampling, double *d_sum, double *d_sumsq, double *best_ms);

#ifdef __cplusplus
}
#endif

#endif /* NCTRACE_H */
