// nc_internal.hpp -- host-side objects of the library and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "nc_device.hpp"
#include "nctrace.h"

struct nc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    unsigned long long *d_scratch = nullptr;   // work-queue heads and flags (kScratchWords words)
    nc_launch launch{};
    void *d_jobs = nullptr;        // device job table of batched renders
    size_t jobs_cap = 0;
    int num_cus = 256;
    size_t lds_per_cu = 160 * 1024;
};

struct nc_phase {
    int device = 0;
    int n = 0;
    float *d_mu = nullptr, *d_p = nullptr, *d_cdf = nullptr;   // nodes, values per steradian, CDF at the nodes
};

struct nc_grid {
    int device = 0;
    int n[3] = {0, 0, 0};
    double lo[3] = {0, 0, 0}, h[3] = {0, 0, 0};
    nc_grid_params params{};
    int L = 0;
    int off[NC_MAX_LEVELS + 2] = {};
    size_t total_nodes = 0;
    float2 *d_nodes = nullptr;
    int *d_off = nullptr;
    uint16_t *d_mask = nullptr;   // per level-1 node: bit l set if its level-l ancestor is merged
};

namespace nc {
constexpr int kGuideRaw = 7;    // a vertex's inputs: position in [-1, 1]^3, incoming direction, ln(1 + k)
constexpr int kGuideIn = 15;    // the network's: those 7, then 8 features of the horizontal position

// Network input k (0..14) from a vertex's 7 values x: x[k] for k < 7, then
// sin and cos of 8 pi x, 8 pi y, 16 pi x, 16 pi y (a fixed Fourier encoding
// of the position; v_sin / v_cos take revolutions).
__device__ inline float guide_feature(const float *x, int k)
{
    if (k < kGuideRaw) return x[k];
    const int j = k - kGuideRaw;
    const float v = x[(j >> 1) & 1] * (j < 4 ? 4.0f : 8.0f);
    return (j & 1) ? __builtin_amdgcn_cosf(v) : __builtin_amdgcn_sinf(v);
}
constexpr int kGuideWidth = 64;
constexpr int kGuideLayers = 4;
constexpr int kGuideLobes = 8;
constexpr int kGuideOut = 5 * kGuideLobes;
constexpr int kGuideParams = kGuideIn * 64 + 64 + 2 * (64 * 64 + 64) + 64 * 40 + 40;   // 11944
constexpr int kGuideRecord = 12;   // floats per training record
constexpr float kLogKappaMin = -3.0f, kLogKappaMax = 8.0f;
}  // namespace nc

struct nc_guide {
    int device = 0;
    float *d_params = nullptr;                 // fp32 master weights (flat, layer by layer: W [out][in], b [out])
    float *d_m = nullptr, *d_v = nullptr;      // Adam moments
    float *d_grad = nullptr;                   // gradient of the last step
    double *d_acc = nullptr;                   // [loss sum, weight sum] of the last step
    short *d_w[4] = {};                        // bf16 padded weights [out_pad][in_pad]
    short *d_wt[4] = {};                       // and transposed
    float *d_bias[4] = {};                     // fp32 padded biases
    float *d_scratch = nullptr;                // training activations
    int scratch_cap = 0;
    long long step = 0;
};

namespace nc {

constexpr int kMaxQueueSets = NC_BATCH_MAX_GUIDES;   // work-queue sets of one launch (one per guide)
constexpr int kScratchWords = 256 + 128 * kMaxQueueSets;   // [1] validation flag, [2] cloudy layer, [8..] launch
                                                           // parameters, [256..] queue heads
constexpr int kScratchRare = 8;
constexpr int kScratchErr = 240;     // [240..242] image error accumulators (float64)
constexpr int kScratchQueues = 256;  // [256 + 16 (8 set + q)] head of work queue q (q < 8) of a queue set,
                                     // one per 128-byte line

// Camera, optics and launch records as the kernels see them (FP32).
struct CamView {
    int type, W, H;
    float pos[3], f[3], r[3], u[3];
    float sx, sy;        // pinhole: tan(fov/2)*aspect, tan(fov/2); ortho: width, height
};

struct OptView {
    float ssa, g, rho, S, mscale;
    HGc hg;              // the phase function's constants
    PhaseView tab;       // a tabulated phase function (tab.n == 0: HG)
    int kd_n;            // k-distribution points (0: the grid's gas extinction for every path)
    float kd_cdf[NC_KDIST_MAX];   // cumulative normalised weights
    float kd_k[NC_KDIST_MAX];     // gas extinction per point
    int cone;            // the sun is a disc (else directional)
    float cone_cos;      // cos of its angular radius
    float cone_gain;     // 2 / (1 + cos alpha): a local estimate's weight for a direction drawn in the cone
    float cone_L;        // its radiance per unit irradiance, 1 / (pi sin^2 alpha)
    float sun[3];
    float ground_w;      // rho / pi * S * cos(theta_sun): ground local estimate before transmissivity
    int max_scatter, max_segments;
};

// bf16 weights of the guide network as the kernels read them.
struct GuideWeights {
    const short *w[4];    // W_pad [out_pad][in_pad]
    const short *wt[4];   // W_pad transposed [in_pad][out_pad]
    const float *b[4];    // bias [out_pad]
};
GuideWeights guide_weights(const nc_guide *gd);

// Vertex collection: where the renderer writes training records.
struct CollectView {
    float *records;                   // cap x 12 floats
    unsigned long long cap;
    unsigned long long *count;        // records attempted (may exceed cap)
    float *final_L;                   // per path (pix * spp + sample): the path's radiance
};

// One job of a batched render: a view and its sun (device memory).
struct JobView {
    CamView cam;
    float sun[3];
    float S, rho;
    int tiles_x, tiles_y;
    int pad_;
    unsigned long long item_begin;   // first queue item of the job (set by the launcher)
    unsigned long long out_off;      // first output element of the job's image
};

struct Shape {
    int block;
    int wgs;
    int spi;             // samples per queue item
    int lds_first;       // first grid level staged in LDS (L+1: none)
    int lds_nodes;
};

GridView grid_view(const nc_grid *g, const float *d_kc);
Shape choose_shape(const nc_ctx *ctx, const nc_grid *g, int block_default, size_t reserve = 0, int waves_default = 0);

hipError_t launch_build(const nc_ctx *ctx, nc_grid *g, const float *d_kc, unsigned int *d_bad, int *d_zc);
hipError_t launch_phase_sample(const nc_ctx *ctx, const PhaseView &t, const float *u, int n, float *out);
hipError_t launch_export(const nc_ctx *ctx, const nc_grid *g, int level, float *kmin, float *kmax, uint8_t *mg);
hipError_t launch_leaf_levels(const nc_ctx *ctx, const nc_grid *g, uint8_t *out);
hipError_t launch_trace_leaves(const nc_ctx *ctx, const nc_grid *g, const float *rays, int n, int maxv, int *leaf,
                               float *t, int *count);
hipError_t launch_transmittance(const nc_ctx *ctx, const nc_grid *g, const float *d_kc, const OptView &op,
                                const float *rays, int n, const nc_sampling &s, double *sum, double *sumsq,
                                nc_counters *counters);
hipError_t launch_flux(const nc_ctx *ctx, const nc_grid *g, const float *d_kc, const OptView &op, float kscale,
                       int px_nx, int px_ny, unsigned long long n_photons, const nc_sampling &s, double *tally,
                       double *glob, const double *grad, double *out, nc_counters *counters);
hipError_t guide_pack(const nc_ctx *ctx, nc_guide *gd);
hipError_t guide_forward(const nc_ctx *ctx, const nc_guide *gd, const float *X, int n, int rec_stride, float *Z,
                         float *H0, float *H1, float *H2);
hipError_t guide_train_step(const nc_ctx *ctx, nc_guide *gd, const float *rec, int n, int rec_stride, float lr,
                            double *d_loss, bool apply);
hipError_t launch_philox(const nc_ctx *ctx, const uint32_t *ctr, const uint32_t *key, uint32_t *out, int n);
// Device memory a render launch writes before it starts: the job table, the
// launch record (the renderer's rarely used parameters, at most kRareBytes)
// and the 8 work-queue heads (128 words, 16 apart, zeroed by a kernel at each
// launch).  Either the context's buffers or the no-allocation scratch.
constexpr size_t kRareBytes = 1536;
struct RenderScratch {
    JobView *jobs;
    unsigned long long *rare;
    unsigned long long *queue;   // 128 words per queue set
    int max_sets;                // queue sets it holds
};
hipError_t launch_render(const nc_ctx *ctx, const nc_grid *g, const float *d_kc, const OptView &op,
                         const JobView *jobs, int n_jobs, const nc_sampling &s, double *sum, double *sumsq,
                         nc_counters *counters, const RenderScratch &scr, const nc_guide *const *guides = nullptr,
                         const CollectView *collect = nullptr);
// The no-allocation scratch (nc_noalloc.hip): a file-scope device array of
// kNoallocMaxJobs job records plus a launch record and queue heads, one copy
// per GPU.  noalloc_init_device resolves its address on the current device
// (once per device, at context creation); noalloc_render_scratch returns the
// views into it (jobs == nullptr if the device was never initialised).
constexpr int kNoallocMaxJobs = NC_NOALLOC_MAX_JOBS;
hipError_t noalloc_init_device(int device);
RenderScratch noalloc_render_scratch(int device);
hipError_t launch_collect_finish(const nc_ctx *ctx, const CollectView &cv);
hipError_t launch_guide_sample(const nc_ctx *ctx, const nc_guide *gd, const float *in, const float *u, float c,
                               float g, int n, float *out);
hipError_t launch_gather_rate(const nc_ctx *ctx, const float *buf, uint32_t mask, int threads, int loads,
                              uint32_t seed, float *out);
// Block-mean error statistics of an image estimate (synchronises the stream):
// out3 = [sum of block means, sum of squared block standard errors, blocks].
hipError_t launch_image_err(const nc_ctx *ctx, const double *sum, const double *sumsq, int W, int H, int n, int b,
                            double *out3);

}  // namespace nc
