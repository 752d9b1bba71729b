// nc_api.hip -- host side of the C ABI: contexts, validation, grid storage,
// and the estimator entry points.  See include/nctrace.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <vector>

#include "nc_internal.hpp"

namespace {

thread_local std::string g_create_err;

nc_status fail(nc_ctx *ctx, nc_status st, const std::string &msg)
{
    if (ctx)
        ctx->err = msg;
    else
        g_create_err = msg;
    return st;
}

nc_status hip_fail(nc_ctx *ctx, hipError_t e, const char *where)
{
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(ctx, e == hipErrorOutOfMemory ? NC_ERR_OOM : NC_ERR_DEVICE, m);
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

nc_status check_desc(nc_ctx *ctx, const nc_field_desc *d)
{
    if (!d) return fail(ctx, NC_ERR_INVALID_ARG, "field descriptor is NULL");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(ctx, NC_ERR_INVALID_ARG, "field dimensions must be >= 1");
    if ((long long)d->nx * d->ny * d->nz > (1ll << 33))
        return fail(ctx, NC_ERR_INVALID_ARG, "field larger than 2^33 cells");
    if (!finite_pos(d->dx) || !finite_pos(d->dy) || !finite_pos(d->dz))
        return fail(ctx, NC_ERR_RANGE, "cell sizes must be finite and > 0");
    if (!std::isfinite(d->x0) || !std::isfinite(d->y0) || !std::isfinite(d->z0))
        return fail(ctx, NC_ERR_RANGE, "box origin must be finite");
    if (d->z0 < 0.0) return fail(ctx, NC_ERR_RANGE, "box must lie above the ground (z0 >= 0)");
    return NC_OK;
}

nc_status check_optics(nc_ctx *ctx, const nc_optics *o)
{
    if (!o) return fail(ctx, NC_ERR_INVALID_ARG, "optics is NULL");
    if (!(o->ssa >= 0.0 && o->ssa <= 1.0)) return fail(ctx, NC_ERR_RANGE, "ssa must be in [0,1]");
    if (!(o->g > -1.0 && o->g < 1.0)) return fail(ctx, NC_ERR_RANGE, "g must be in (-1,1)");
    if (!(o->ground_albedo >= 0.0 && o->ground_albedo <= 1.0))
        return fail(ctx, NC_ERR_RANGE, "ground albedo must be in [0,1]");
    if (!std::isfinite(o->sun_zenith_deg) || !std::isfinite(o->sun_azimuth_deg) || !(o->sun_zenith_deg >= 0.0) ||
        !(o->sun_zenith_deg < 90.0))
        return fail(ctx, NC_ERR_RANGE, "sun zenith must be in [0,90) degrees");
    if (!(o->sun_irradiance >= 0.0) || !std::isfinite(o->sun_irradiance))
        return fail(ctx, NC_ERR_RANGE, "sun irradiance must be finite and >= 0");
    if (!(o->majorant_scale >= 1.0) || !std::isfinite(o->majorant_scale))
        return fail(ctx, NC_ERR_RANGE, "majorant_scale must be finite and >= 1");
    if (o->max_segments < 1) return fail(ctx, NC_ERR_INVALID_ARG, "max_segments must be >= 1");
    if (!(o->sun_half_angle_deg >= 0.0 && o->sun_half_angle_deg < 90.0))
        return fail(ctx, NC_ERR_RANGE, "sun half angle must be in [0,90) degrees");
    if (o->phase && o->phase->device != ctx->device)
        return fail(ctx, NC_ERR_INVALID_ARG, "phase table lives on another device");
    if (o->kdist) {
        const nc_kdist &k = *o->kdist;
        if (k.n < 1 || k.n > NC_KDIST_MAX) return fail(ctx, NC_ERR_INVALID_ARG, "k-distribution needs 1 .. 16 points");
        double tot = 0.0;
        for (int i = 0; i < k.n; ++i) {
            if (!std::isfinite(k.w[i]) || !(k.w[i] >= 0.0) || !std::isfinite(k.k_gas[i]) || !(k.k_gas[i] >= 0.0))
                return fail(ctx, NC_ERR_RANGE, "k-distribution weights and extinctions must be finite, >= 0");
            tot += k.w[i];
        }
        if (!(tot > 0.0)) return fail(ctx, NC_ERR_RANGE, "k-distribution weights sum to 0");
    }
    return NC_OK;
}

// two k-distributions with the same points (or both absent)
bool same_kdist(const nc_kdist *a, const nc_kdist *b)
{
    if (!a || !b) return a == b;
    if (a->n != b->n) return false;
    for (int i = 0; i < a->n; ++i)
        if (a->w[i] != b->w[i] || a->k_gas[i] != b->k_gas[i]) return false;
    return true;
}

// every k-distribution point within the shared grid's majorant
nc_status check_kdist_grid(nc_ctx *ctx, const nc_optics *o, const nc_grid *g)
{
    if (!o->kdist) return NC_OK;
    for (int i = 0; i < o->kdist->n; ++i)
        if (o->kdist->k_gas[i] > g->params.k_gas)
            return fail(ctx, NC_ERR_RANGE, "a k-distribution point's k_gas exceeds the grid's (its majorant)");
    return NC_OK;
}

// an irradiance sensor needs the whole sun above the horizon
bool sensor_sun_ok(const nc_optics *o)
{
    return o->sun_zenith_deg + o->sun_half_angle_deg < 90.0;
}

nc_status check_grid(nc_ctx *ctx, const nc_grid *g)
{
    if (!g) return fail(ctx, NC_ERR_INVALID_ARG, "grid is NULL");
    if (g->device != ctx->device) return fail(ctx, NC_ERR_STATE, "grid lives on another device");
    return NC_OK;
}

nc::OptView make_opt(const nc_optics *o, double k_gas)
{
    (void)k_gas;
    nc::OptView v;
    const double th = o->sun_zenith_deg * M_PI / 180.0, ph = o->sun_azimuth_deg * M_PI / 180.0;
    v.ssa = (float)o->ssa;
    v.g = (float)o->g;
    v.hg = nc::make_hg(o->g);
    v.tab = nc::PhaseView{nullptr, nullptr, nullptr, 0};
    if (o->phase) v.tab = nc::PhaseView{o->phase->d_mu, o->phase->d_p, o->phase->d_cdf, o->phase->n};
    v.kd_n = 0;
    for (int i = 0; i < NC_KDIST_MAX; ++i) v.kd_cdf[i] = v.kd_k[i] = 0.0f;
    if (o->kdist) {
        double tot = 0.0, acc = 0.0;
        for (int i = 0; i < o->kdist->n; ++i) tot += o->kdist->w[i];
        v.kd_n = o->kdist->n;
        for (int i = 0; i < o->kdist->n; ++i) {
            acc += o->kdist->w[i];
            v.kd_cdf[i] = (float)(acc / tot);
            v.kd_k[i] = (float)o->kdist->k_gas[i];
        }
    }
    const double a = o->sun_half_angle_deg * M_PI / 180.0;
    v.cone = a > 0.0 ? 1 : 0;
    v.cone_cos = (float)std::cos(a);
    v.cone_gain = (float)(2.0 / (1.0 + std::cos(a)));
    v.cone_L = a > 0.0 ? (float)(1.0 / (M_PI * std::sin(a) * std::sin(a))) : 0.0f;
    v.rho = (float)o->ground_albedo;
    v.S = (float)o->sun_irradiance;
    v.mscale = (float)o->majorant_scale;
    v.sun[0] = (float)(std::sin(th) * std::cos(ph));
    v.sun[1] = (float)(std::sin(th) * std::sin(ph));
    v.sun[2] = (float)std::cos(th);
    v.ground_w = (float)(o->ground_albedo / M_PI * o->sun_irradiance * std::cos(th));
    v.max_scatter = o->max_scatter;
    v.max_segments = o->max_segments;
    return v;
}

void norm3(double v[3])
{
    const double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n;
    v[1] /= n;
    v[2] /= n;
}

void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

nc_status make_cam(nc_ctx *ctx, const nc_camera *c, nc::CamView &v)
{
    if (!c) return fail(ctx, NC_ERR_INVALID_ARG, "camera is NULL");
    if (c->type < 0 || c->type > 2) return fail(ctx, NC_ERR_INVALID_ARG, "camera type must be 0, 1 or 2");
    if (c->width < 1 || c->height < 1 || (long long)c->width * c->height > (1ll << 30))
        return fail(ctx, NC_ERR_INVALID_ARG, "bad image size");
    if (c->type == 2) {
        // horizontal sensor: only the position and the rectangle matter
        if (!(c->ortho_w > 0.0 && c->ortho_h > 0.0)) return fail(ctx, NC_ERR_RANGE, "sensor extent must be > 0");
        v.type = 2;
        v.W = c->width;
        v.H = c->height;
        for (int a = 0; a < 3; ++a) {
            v.pos[a] = (float)c->pos[a];
            v.f[a] = a == 2 ? 1.0f : 0.0f;
            v.r[a] = a == 0 ? 1.0f : 0.0f;
            v.u[a] = a == 1 ? 1.0f : 0.0f;
        }
        v.sx = (float)c->ortho_w;
        v.sy = (float)c->ortho_h;
        return NC_OK;
    }
    double f[3], r[3], u[3];
    for (int a = 0; a < 3; ++a) f[a] = c->target[a] - c->pos[a];
    const double fn = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(fn > 0.0) || !std::isfinite(fn)) return fail(ctx, NC_ERR_RANGE, "camera target equals position");
    norm3(f);
    cross3(f, c->up, r);
    const double rn = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(rn > 1e-12)) return fail(ctx, NC_ERR_RANGE, "camera up vector is parallel to the view direction");
    norm3(r);
    cross3(r, f, u);
    if (c->type == 0 && !(c->fov_y_deg > 0.0 && c->fov_y_deg < 180.0))
        return fail(ctx, NC_ERR_RANGE, "fov_y_deg must be in (0,180)");
    if (c->type == 1 && !(c->ortho_w > 0.0 && c->ortho_h > 0.0))
        return fail(ctx, NC_ERR_RANGE, "orthographic extent must be > 0");
    v.type = c->type;
    v.W = c->width;
    v.H = c->height;
    for (int a = 0; a < 3; ++a) {
        v.pos[a] = (float)c->pos[a];
        v.f[a] = (float)f[a];
        v.r[a] = (float)r[a];
        v.u[a] = (float)u[a];
    }
    if (c->type == 0) {
        const double t = std::tan(0.5 * c->fov_y_deg * M_PI / 180.0);
        v.sx = (float)(t * (double)c->width / (double)c->height);
        v.sy = (float)t;
    } else {
        v.sx = (float)c->ortho_w;
        v.sy = (float)c->ortho_h;
    }
    return NC_OK;
}

nc::JobView make_job(const nc::CamView &cam, const nc_optics *o, unsigned long long out_off)
{
    nc::JobView j{};
    const double th = o->sun_zenith_deg * M_PI / 180.0, ph = o->sun_azimuth_deg * M_PI / 180.0;
    j.cam = cam;
    j.sun[0] = (float)(std::sin(th) * std::cos(ph));
    j.sun[1] = (float)(std::sin(th) * std::sin(ph));
    j.sun[2] = (float)std::cos(th);
    j.S = (float)o->sun_irradiance;
    j.rho = (float)o->ground_albedo;
    j.out_off = out_off;
    return j;
}

hipError_t ensure_jobs(nc_ctx *ctx, size_t n)
{
    if (ctx->jobs_cap >= n) return hipSuccess;
    if (ctx->d_jobs) {
        hipError_t e = hipFree(ctx->d_jobs);
        ctx->d_jobs = nullptr;
        ctx->jobs_cap = 0;
        if (e != hipSuccess) return e;
    }
    const size_t cap = (n + 63) / 64 * 64;
    hipError_t e = hipMalloc(&ctx->d_jobs, cap * sizeof(nc::JobView));
    if (e == hipSuccess) ctx->jobs_cap = cap;
    return e;
}

// The context's buffers for a render launch (the job table must hold the jobs).
nc::RenderScratch ctx_render_scratch(const nc_ctx *ctx)
{
    return nc::RenderScratch{(nc::JobView *)ctx->d_jobs, ctx->d_scratch + nc::kScratchRare,
                             ctx->d_scratch + nc::kScratchQueues, nc::kMaxQueueSets};
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" {

uint32_t nc_abi_version(void) { return NC_ABI_VERSION; }

nc_status nc_ctx_create(int32_t device, void *hip_stream, nc_ctx **out)
{
    if (!out) return fail(nullptr, NC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) return fail(nullptr, NC_ERR_DEVICE, "no HIP device available");
    if (device < 0 || device >= count) return fail(nullptr, NC_ERR_DEVICE, "device index out of range");
    DeviceGuard guard(device);
    nc_ctx *ctx = new (std::nothrow) nc_ctx();
    if (!ctx) return fail(nullptr, NC_ERR_OOM, "host allocation failed");
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        ctx->num_cus = cus;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) == hipSuccess &&
        lds > 0)
        ctx->lds_per_cu = (size_t)lds;
    e = hipMalloc(&ctx->d_scratch, sizeof(unsigned long long) * nc::kScratchWords);
    if (e != hipSuccess) {
        delete ctx;
        return hip_fail(nullptr, e, "hipMalloc(scratch)");
    }
    // the no-allocation entry point's scratch: its address on this device, once
    e = nc::noalloc_init_device(device);
    if (e != hipSuccess) {
        (void)hipFree(ctx->d_scratch);
        delete ctx;
        return hip_fail(nullptr, e, "no-allocation scratch address");
    }
    *out = ctx;
    return NC_OK;
}

nc_status nc_ctx_set_stream(nc_ctx *ctx, void *hip_stream)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    ctx->stream = (hipStream_t)hip_stream;
    return NC_OK;
}

void nc_ctx_destroy(nc_ctx *ctx)
{
    if (!ctx) return;
    DeviceGuard guard(ctx->device);
    if (ctx->d_scratch) (void)hipFree(ctx->d_scratch);
    if (ctx->d_jobs) (void)hipFree(ctx->d_jobs);
    delete ctx;
}

const char *nc_last_error(const nc_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

nc_status nc_set_launch(nc_ctx *ctx, const nc_launch *launch)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    if (!launch) {
        ctx->launch = nc_launch{};
        return NC_OK;
    }
    if (launch->block < 0 || launch->block > 256 || (launch->block % 64) != 0)
        return fail(ctx, NC_ERR_INVALID_ARG, "block must be a multiple of 64 in [64,256] (or 0)");
    if (launch->waves_per_cu < 0 || launch->waves_per_cu > 32)
        return fail(ctx, NC_ERR_INVALID_ARG, "waves_per_cu must be in [0,32]");
    if (launch->samples_per_item < 0) return fail(ctx, NC_ERR_INVALID_ARG, "samples_per_item must be >= 0");
    if (launch->lds_levels < -1 || launch->lds_levels > NC_MAX_LEVELS)
        return fail(ctx, NC_ERR_INVALID_ARG, "lds_levels must be in [-1, NC_MAX_LEVELS]");
    ctx->launch = *launch;
    return NC_OK;
}

// Levels, ancestry masks and the field check over d_kc into g's memory;
// synchronises (reads the check's flag back).
static nc_status grid_fill(nc_ctx *ctx, nc_grid *g, const float *d_kc)
{
    unsigned int *d_bad = reinterpret_cast<unsigned int *>(ctx->d_scratch + 1);
    unsigned int h_bad = 0;
    hipError_t e = hipMemcpyAsync(d_bad, &h_bad, sizeof(unsigned int), hipMemcpyHostToDevice, ctx->stream);
    int *d_zc = reinterpret_cast<int *>(ctx->d_scratch + 2);
    if (e == hipSuccess) e = nc::launch_build(ctx, g, d_kc, d_bad, d_zc);
    if (e == hipSuccess && g->L == 0) {
        // a single cell: validate it on the host
        float v = 0.0f;
        e = hipMemcpyAsync(&v, d_kc, sizeof(float), hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e == hipSuccess && (!(v >= 0.0f) || std::isinf(v))) h_bad = 1;
    }
    if (e == hipSuccess && g->L > 0)
        e = hipMemcpyAsync(&h_bad, d_bad, sizeof(unsigned int), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "grid build");
    if (h_bad) return fail(ctx, NC_ERR_RANGE, "field holds NaN, Inf or negative extinction");
    return NC_OK;
}

nc_status nc_grid_build(nc_ctx *ctx, const float *d_kc, const nc_field_desc *desc, const nc_grid_params *params,
                        nc_grid **out)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    if (!out) return fail(ctx, NC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!d_kc) return fail(ctx, NC_ERR_INVALID_ARG, "field pointer is NULL");
    nc_status st = check_desc(ctx, desc);
    if (st != NC_OK) return st;
    if (!params) return fail(ctx, NC_ERR_INVALID_ARG, "grid params is NULL");
    if (!(params->tau_tilde >= 0.0)) return fail(ctx, NC_ERR_RANGE, "tau_tilde must be >= 0");
    if (!(params->k_gas >= 0.0) || !std::isfinite(params->k_gas))
        return fail(ctx, NC_ERR_RANGE, "k_gas must be finite and >= 0");
    if (params->criterion < 0 || params->criterion > 3)
        return fail(ctx, NC_ERR_INVALID_ARG, "criterion must be 0, 1, 2 or 3");
    if (params->criterion >= 2 && (params->flat_level < 0 || params->flat_level > NC_MAX_LEVELS))
        return fail(ctx, NC_ERR_INVALID_ARG, "flat_level must lie in [0, NC_MAX_LEVELS]");
    DeviceGuard guard(ctx->device);
    nc_grid *g = new (std::nothrow) nc_grid();
    if (!g) return fail(ctx, NC_ERR_OOM, "host allocation failed");
    g->device = ctx->device;
    g->n[0] = desc->nx;
    g->n[1] = desc->ny;
    g->n[2] = desc->nz;
    g->lo[0] = desc->x0;
    g->lo[1] = desc->y0;
    g->lo[2] = desc->z0;
    g->h[0] = desc->dx;
    g->h[1] = desc->dy;
    g->h[2] = desc->dz;
    g->params = *params;
    int nmax = std::max(desc->nx, std::max(desc->ny, desc->nz));
    int L = 0;
    while ((1 << L) < nmax) ++L;
    if (L > 15) {   // the per-node ancestry mask holds levels 1..15
        delete g;
        return fail(ctx, NC_ERR_INVALID_ARG, "field too large");
    }
    g->L = L;
    size_t total = 0;
    g->off[0] = 0;
    for (int l = 1; l <= L; ++l) {
        g->off[l] = (int)total;
        total += (size_t)nc::level_dim(g->n[0], l) * nc::level_dim(g->n[1], l) * nc::level_dim(g->n[2], l);
        if (total > (size_t)0x7fffffff) {
            delete g;
            return fail(ctx, NC_ERR_INVALID_ARG, "grid has more than 2^31 nodes");
        }
    }
    g->off[L + 1] = (int)total;
    for (int l = L + 2; l < NC_MAX_LEVELS + 2; ++l) g->off[l] = (int)total;
    g->total_nodes = total;
    hipError_t e = hipMalloc(&g->d_nodes, std::max<size_t>(total, 1) * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc(&g->d_off, sizeof(int) * (NC_MAX_LEVELS + 2));
    if (e == hipSuccess && L >= 1)
        e = hipMalloc(&g->d_mask, sizeof(uint16_t) * (size_t)nc::level_dim(desc->nx, 1) *
                                      nc::level_dim(desc->ny, 1) * nc::level_dim(desc->nz, 1));
    if (e != hipSuccess) {
        nc_grid_destroy(g);
        return hip_fail(ctx, e, "hipMalloc(grid)");
    }
    e = hipMemcpyAsync(g->d_off, g->off, sizeof(int) * (NC_MAX_LEVELS + 2), hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) {
        nc_grid_destroy(g);
        return hip_fail(ctx, e, "grid build");
    }
    st = grid_fill(ctx, g, d_kc);
    if (st != NC_OK) {
        nc_grid_destroy(g);
        return st;
    }
    *out = g;
    return NC_OK;
}

nc_status nc_grid_rebuild(nc_ctx *ctx, nc_grid *grid, const float *d_kc)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    if (!grid) return fail(ctx, NC_ERR_INVALID_ARG, "grid is NULL");
    if (!d_kc) return fail(ctx, NC_ERR_INVALID_ARG, "field pointer is NULL");
    if (grid->device != ctx->device) return fail(ctx, NC_ERR_INVALID_ARG, "grid and context are on different devices");
    DeviceGuard guard(ctx->device);
    return grid_fill(ctx, grid, d_kc);
}

nc_status nc_grid_export_mask(nc_ctx *ctx, const nc_grid *grid, uint16_t *d_mask)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    if (!grid) return fail(ctx, NC_ERR_INVALID_ARG, "grid is NULL");
    if (!d_mask) return fail(ctx, NC_ERR_INVALID_ARG, "mask pointer is NULL");
    if (grid->L < 1) return fail(ctx, NC_ERR_INVALID_ARG, "a one-cell grid has no level 1");
    DeviceGuard guard(ctx->device);
    const size_t n = (size_t)nc::level_dim(grid->n[0], 1) * nc::level_dim(grid->n[1], 1) * nc::level_dim(grid->n[2], 1);
    const hipError_t e = hipMemcpyAsync(d_mask, grid->d_mask, n * sizeof(uint16_t), hipMemcpyDeviceToDevice, ctx->stream);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "hipMemcpyAsync(mask)");
}

void nc_grid_destroy(nc_grid *g)
{
    if (!g) return;
    DeviceGuard guard(g->device);
    if (g->d_nodes) (void)hipFree(g->d_nodes);
    if (g->d_off) (void)hipFree(g->d_off);
    if (g->d_mask) (void)hipFree(g->d_mask);
    delete g;
}

nc_status nc_grid_info(const nc_grid *g, int32_t *levels, int32_t level, int32_t dims_out[3])
{
    if (!g) return fail(nullptr, NC_ERR_INVALID_ARG, "grid is NULL");
    if (levels) *levels = g->L;
    if (dims_out) {
        if (level < 0 || level > g->L) return fail(nullptr, NC_ERR_INVALID_ARG, "level out of range");
        for (int a = 0; a < 3; ++a) dims_out[a] = nc::level_dim(g->n[a], level);
    }
    return NC_OK;
}

nc_status nc_grid_export(nc_ctx *ctx, const nc_grid *g, int32_t level, float *d_kmin, float *d_kmax,
                         uint8_t *d_merged)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    nc_status st = check_grid(ctx, g);
    if (st != NC_OK) return st;
    if (level < 1 || level > g->L) return fail(ctx, NC_ERR_INVALID_ARG, "level must be in [1, L]");
    DeviceGuard guard(ctx->device);
    hipError_t e = nc::launch_export(ctx, g, level, d_kmin, d_kmax, d_merged);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "grid export");
}

nc_status nc_grid_leaf_levels(nc_ctx *ctx, const nc_grid *g, uint8_t *d_leaf_level)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    nc_status st = check_grid(ctx, g);
    if (st != NC_OK) return st;
    if (!d_leaf_level) return fail(ctx, NC_ERR_INVALID_ARG, "output is NULL");
    DeviceGuard guard(ctx->device);
    hipError_t e = nc::launch_leaf_levels(ctx, g, d_leaf_level);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "leaf levels");
}

nc_status nc_trace_leaves(nc_ctx *ctx, const nc_grid *g, const float *d_rays, int32_t n, int32_t max_visits,
                          int32_t *d_leaf, float *d_t, int32_t *d_count)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    nc_status st = check_grid(ctx, g);
    if (st != NC_OK) return st;
    if (n < 0 || max_visits < 0) return fail(ctx, NC_ERR_INVALID_ARG, "negative size");
    if (n == 0) return NC_OK;
    if (!d_rays || !d_count || (max_visits > 0 && (!d_leaf || !d_t)))
        return fail(ctx, NC_ERR_INVALID_ARG, "NULL buffer");
    DeviceGuard guard(ctx->device);
    hipError_t e = nc::launch_trace_leaves(ctx, g, d_rays, n, max_visits, d_leaf, d_t, d_count);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "trace leaves");
}

nc_status nc_transmittance(nc_ctx *ctx, const nc_grid *g, const float *d_kc, const nc_optics *optics,
                           const float *d_rays, int32_t n, const nc_sampling *s, double *d_sum, double *d_sumsq,
                           nc_counters *d_counters)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    nc_status st = check_grid(ctx, g);
    if (st != NC_OK) return st;
    if ((st = check_optics(ctx, optics)) != NC_OK) return st;
    if (optics->kdist) return fail(ctx, NC_ERR_UNSUPPORTED, "the transmittance kernel takes the grid's gas extinction");
    if (!s) return fail(ctx, NC_ERR_INVALID_ARG, "sampling is NULL");
    if (n < 0 || s->spp < 0) return fail(ctx, NC_ERR_INVALID_ARG, "negative size");
    if (n == 0 || s->spp == 0) return NC_OK;
    if ((s->flags & NC_SUN_ESTIMATOR_MASK) == 3) return fail(ctx, NC_ERR_INVALID_ARG, "unknown sun estimator");
    if (!d_kc || !d_rays || !d_sum || !d_sumsq) return fail(ctx, NC_ERR_INVALID_ARG, "NULL buffer");
    DeviceGuard guard(ctx->device);
    hipError_t e = nc::launch_transmittance(ctx, g, d_kc, make_opt(optics, g->params.k_gas), d_rays, n, *s, d_sum,
                                            d_sumsq, d_counters);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "transmittance");
}

static nc_status render_one(nc_ctx *ctx, const nc_grid *g, const float *d_kc, const nc_optics *optics,
                            const nc_camera *camera, const nc_sampling *s, double *d_sum, double *d_sumsq,
                            nc_counters *d_counters, const nc_guide *guide, const nc::CollectView *collect)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    nc_status st = check_grid(ctx, g);
    if (st != NC_OK) return st;
    if ((st = check_optics(ctx, optics)) != NC_OK) return st;
    if ((st = check_kdist_grid(ctx, optics, g)) != NC_OK) return st;
    nc::CamView cam;
    if ((st = make_cam(ctx, camera, cam)) != NC_OK) return st;
    if (!s) return fail(ctx, NC_ERR_INVALID_ARG, "sampling is NULL");
    if (s->spp < 0) return fail(ctx, NC_ERR_INVALID_ARG, "negative spp");
    if (s->spp == 0) return NC_OK;
    if (s->sample_offset + (uint64_t)s->spp > 0xffffffffull)
        return fail(ctx, NC_ERR_INVALID_ARG, "sample_offset + spp must fit in 32 bits");
    if (!d_kc || !d_sum || !d_sumsq) return fail(ctx, NC_ERR_INVALID_ARG, "NULL buffer");
    DeviceGuard guard(ctx->device);
    if (cam.type == 2 && !sensor_sun_ok(optics))
        return fail(ctx, NC_ERR_RANGE, "an irradiance sensor needs the sun above the horizon");
    if ((s->flags & NC_SUN_ESTIMATOR_MASK) == 3) return fail(ctx, NC_ERR_INVALID_ARG, "unknown sun estimator");
    if (guide && guide->device != ctx->device) return fail(ctx, NC_ERR_INVALID_ARG, "guide lives on another device");
    if (guide && !(s->guide_frac >= 0.0f && s->guide_frac <= 1.0f))
        return fail(ctx, NC_ERR_INVALID_ARG, "guide_frac must lie in [0, 1]");
    const nc::JobView job = make_job(cam, optics, 0);
    hipError_t e = ensure_jobs(ctx, 1);
    if (e == hipSuccess)
        e = nc::launch_render(ctx, g, d_kc, make_opt(optics, g->params.k_gas), &job, 1, *s, d_sum, d_sumsq,
                              d_counters, ctx_render_scratch(ctx), guide ? &guide : nullptr, collect);
    if (e == hipSuccess && collect) e = nc::launch_collect_finish(ctx, *collect);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "render");
}

nc_status nc_render(nc_ctx *ctx, const nc_grid *g, const float *d_kc, const nc_optics *optics, const nc_camera *camera,
                    const nc_sampling *s, double *d_sum, double *d_sumsq, nc_counters *d_counters)
{
    return render_one(ctx, g, d_kc, optics, camera, s, d_sum, d_sumsq, d_counters, nullptr, nullptr);
}

nc_status nc_render_guided(nc_ctx *ctx, const nc_grid *g, const float *d_kc, const nc_optics *optics,
                           const nc_camera *camera, const nc_sampling *s, const nc_guide *guide, double *d_sum,
                           double *d_sumsq, nc_counters *d_counters)
{
    if (!guide) return fail(ctx, NC_ERR_INVALID_ARG, "guide is NULL");
    return render_one(ctx, g, d_kc, optics, camera, s, d_sum, d_sumsq, d_counters, guide, nullptr);
}

nc_status nc_render_progressive(nc_ctx *ctx, const nc_grid *g, const float *d_kc, const nc_optics *optics,
                                const nc_camera *camera, const nc_sampling *s, const nc_guide *guide,
                                const nc_progressive *plan, double *d_sum, double *d_sumsq, nc_counters *d_counters,
                                nc_progress_report *report)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    if (!s || !plan || !report || !camera) return fail(ctx, NC_ERR_INVALID_ARG, "NULL argument");
    if (!(plan->target_rel_err > 0.0) || plan->first_spp < 2 || plan->max_spp < plan->first_spp || plan->block < 1)
        return fail(ctx, NC_ERR_INVALID_ARG, "need target_rel_err > 0, 2 <= first_spp <= max_spp, block >= 1");
    if (s->sample_offset + (uint64_t)plan->max_spp > 0xffffffffull)
        return fail(ctx, NC_ERR_INVALID_ARG, "sample_offset + max_spp must fit in 32 bits");
    *report = nc_progress_report{};
    DeviceGuard guard(ctx->device);
    const auto t0 = std::chrono::steady_clock::now();
    int done = 0, next = plan->first_spp;
    double err = INFINITY, mean = 0.0;
    while (next > 0) {
        nc_sampling r = *s;
        r.sample_offset = s->sample_offset + (uint64_t)done;
        r.spp = next;
        const nc_status st = guide ? nc_render_guided(ctx, g, d_kc, optics, camera, &r, guide, d_sum, d_sumsq, d_counters)
                                   : nc_render(ctx, g, d_kc, optics, camera, &r, d_sum, d_sumsq, d_counters);
        if (st != NC_OK) return st;
        done += next;
        double acc[3];
        const hipError_t e = nc::launch_image_err(ctx, d_sum, d_sumsq, camera->width, camera->height, done,
                                                  plan->block, acc);
        if (e != hipSuccess) return hip_fail(ctx, e, "progressive error estimate");
        mean = acc[0] / acc[2];
        err = mean > 0.0 ? std::sqrt(acc[1] / acc[2]) / mean : INFINITY;
        ++report->rounds;
        if (err <= plan->target_rel_err || done >= plan->max_spp) break;
        // the error falls as 1/sqrt(n): ask for the predicted remainder (5 % margin), at most doubling
        const double need = std::isfinite(err) ? done * ((err / plan->target_rel_err) * (err / plan->target_rel_err) - 1.0) * 1.05
                                               : (double)done;
        next = (int)std::min<double>({std::ceil(need), (double)done, (double)(plan->max_spp - done)});
        next = std::max(next, 1);
    }
    report->spp_done = done;
    report->rel_err = err;
    report->mean = mean;
    report->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return NC_OK;
}

nc_status nc_guide_sample(nc_ctx *ctx, const nc_guide *guide, const float *d_in, const float *d_u, int32_t n,
                          float guide_frac, float g, float *d_out)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    if (!guide || !d_in || !d_u || !d_out) return fail(ctx, NC_ERR_INVALID_ARG, "NULL argument");
    if (n < 0) return fail(ctx, NC_ERR_INVALID_ARG, "negative count");
    if (!(guide_frac >= 0.0f && guide_frac <= 1.0f)) return fail(ctx, NC_ERR_INVALID_ARG, "guide_frac must lie in [0, 1]");
    if (!(g > -1.0f && g < 1.0f)) return fail(ctx, NC_ERR_RANGE, "g must lie in (-1, 1)");
    if (n == 0) return NC_OK;
    DeviceGuard guard(ctx->device);
    const hipError_t e = nc::launch_guide_sample(ctx, guide, d_in, d_u, guide_frac, g, n, d_out);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "guide sample");
}

nc_status nc_phase_create(nc_ctx *ctx, const double *h_mu, const double *h_p, int32_t n, nc_phase **out)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    if (!out || !h_mu || !h_p) return fail(ctx, NC_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (n < 2 || n > (1 << 20)) return fail(ctx, NC_ERR_INVALID_ARG, "the table needs 2 .. 2^20 nodes");
    if (h_mu[0] != -1.0 || h_mu[n - 1] != 1.0) return fail(ctx, NC_ERR_RANGE, "the cosines must run from -1 to 1");
    double area = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(h_p[i]) || !(h_p[i] >= 0.0)) return fail(ctx, NC_ERR_RANGE, "phase values must be finite, >= 0");
        if (i > 0 && !(h_mu[i] > h_mu[i - 1])) return fail(ctx, NC_ERR_RANGE, "the cosines must increase");
        if (i > 0) area += 0.5 * (h_p[i] + h_p[i - 1]) * (h_mu[i] - h_mu[i - 1]);
    }
    if (!(area > 0.0) || !std::isfinite(area)) return fail(ctx, NC_ERR_RANGE, "the phase function integrates to 0");
    // per steradian, and the CDF at the nodes (in double, then float)
    const double c = 1.0 / (2.0 * M_PI * area);
    std::vector<float> mu(n), p(n), cdf(n);
    double acc = 0.0;
    for (int i = 0; i < n; ++i) {
        if (i > 0) acc += 2.0 * M_PI * c * 0.5 * (h_p[i] + h_p[i - 1]) * (h_mu[i] - h_mu[i - 1]);
        mu[i] = (float)h_mu[i];
        p[i] = (float)(c * h_p[i]);
        cdf[i] = (float)acc;
    }
    cdf[n - 1] = 1.0f;
    for (int i = 1; i < n; ++i)
        if (!(mu[i] > mu[i - 1])) return fail(ctx, NC_ERR_RANGE, "cosines closer than float32 resolves");
    DeviceGuard guard(ctx->device);
    nc_phase *ph = new (std::nothrow) nc_phase();
    if (!ph) return fail(ctx, NC_ERR_OOM, "host allocation failed");
    ph->device = ctx->device;
    ph->n = n;
    hipError_t e = hipMalloc(&ph->d_mu, sizeof(float) * n);
    if (e == hipSuccess) e = hipMalloc(&ph->d_p, sizeof(float) * n);
    if (e == hipSuccess) e = hipMalloc(&ph->d_cdf, sizeof(float) * n);
    if (e == hipSuccess) e = hipMemcpyAsync(ph->d_mu, mu.data(), sizeof(float) * n, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ph->d_p, p.data(), sizeof(float) * n, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ph->d_cdf, cdf.data(), sizeof(float) * n, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);   // the host vectors go out of scope
    if (e != hipSuccess) {
        nc_phase_destroy(ph);
        return hip_fail(ctx, e, "phase table");
    }
    *out = ph;
    return NC_OK;
}

void nc_phase_destroy(nc_phase *ph)
{
    if (!ph) return;
    DeviceGuard guard(ph->device);
    if (ph->d_mu) (void)hipFree(ph->d_mu);
    if (ph->d_p) (void)hipFree(ph->d_p);
    if (ph->d_cdf) (void)hipFree(ph->d_cdf);
    delete ph;
}

nc_status nc_phase_sample(nc_ctx *ctx, const nc_phase *ph, const float *d_u, int32_t n, float *d_out)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    if (!ph || !d_u || !d_out) return fail(ctx, NC_ERR_INVALID_ARG, "NULL argument");
    if (ph->device != ctx->device) return fail(ctx, NC_ERR_INVALID_ARG, "phase table lives on another device");
    if (n < 0) return fail(ctx, NC_ERR_INVALID_ARG, "negative count");
    if (n == 0) return NC_OK;
    DeviceGuard guard(ctx->device);
    const hipError_t e =
        nc::launch_phase_sample(ctx, nc::PhaseView{ph->d_mu, ph->d_p, ph->d_cdf, ph->n}, d_u, n, d_out);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "phase sample");
}

nc_status nc_gather_rate(nc_ctx *ctx, const float *d_buf, uint64_t n_words, int32_t threads, int32_t loads,
                         float *d_out, double *loads_per_s)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    if (!d_buf || !d_out || !loads_per_s) return fail(ctx, NC_ERR_INVALID_ARG, "NULL argument");
    if (n_words < 2 || n_words > (1ull << 32) || (n_words & (n_words - 1)) != 0)
        return fail(ctx, NC_ERR_INVALID_ARG, "n_words must be a power of two in [2, 2^32]");
    if (threads < 256 || threads % 256 != 0 || loads < 8 || loads % 8 != 0)
        return fail(ctx, NC_ERR_INVALID_ARG, "threads must be a multiple of 256, loads a multiple of 8");
    DeviceGuard guard(ctx->device);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const uint32_t mask = (uint32_t)(n_words - 1);
    if (e == hipSuccess) e = nc::launch_gather_rate(ctx, d_buf, mask, threads, loads, 1u, d_out);   // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
    if (e == hipSuccess) e = nc::launch_gather_rate(ctx, d_buf, mask, threads, loads, 2u, d_out);
    if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(ctx, e, "gather rate");
    *loads_per_s = (double)threads * loads / (ms * 1e-3);
    return NC_OK;
}

nc_status nc_collect_vertices(nc_ctx *ctx, const nc_grid *g, const float *d_kc, const nc_optics *optics,
                              const nc_camera *camera, const nc_sampling *s, float *d_records, uint64_t capacity,
                              unsigned long long *d_count, float *d_path_L, double *d_sum, double *d_sumsq,
                              nc_counters *d_counters)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    if (!camera || !s) return fail(ctx, NC_ERR_INVALID_ARG, "camera or sampling is NULL");
    if (!d_count || !d_path_L || (capacity > 0 && !d_records))
        return fail(ctx, NC_ERR_INVALID_ARG, "NULL collection buffer");
    const uint64_t slots = (uint64_t)(camera->width > 0 ? camera->width : 0) *
                           (uint64_t)(camera->height > 0 ? camera->height : 0) * (uint64_t)(s->spp > 0 ? s->spp : 0);
    if (slots > 0xffffffffull) return fail(ctx, NC_ERR_INVALID_ARG, "width * height * spp must fit in 32 bits");
    nc::CollectView cv;
    cv.records = d_records;
    cv.cap = capacity;
    cv.count = d_count;
    cv.final_L = d_path_L;
    if (s->spp == 0) {
        DeviceGuard guard(ctx->device);
        const hipError_t e = hipMemsetAsync(d_count, 0, sizeof(unsigned long long), ctx->stream);
        return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "collect");
    }
    return render_one(ctx, g, d_kc, optics, camera, s, d_sum, d_sumsq, d_counters, nullptr, &cv);
}

static nc_status render_batch_common(nc_ctx *ctx, const nc_grid *g, const float *d_kc, int32_t n_jobs,
                                     const nc_camera *cams, const nc_optics *optics, const uint64_t *out_offsets,
                                     const nc_sampling *s, const nc_guide *const *guides, double *d_sum,
                                     double *d_sumsq, nc_counters *d_counters, bool noalloc = false)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    nc_status st = check_grid(ctx, g);
    if (st != NC_OK) return st;
    if (n_jobs < 0) return fail(ctx, NC_ERR_INVALID_ARG, "negative job count");
    if (noalloc && n_jobs > nc::kNoallocMaxJobs)
        return fail(ctx, NC_ERR_INVALID_ARG, "nc_render_batch_noalloc takes at most NC_NOALLOC_MAX_JOBS jobs");
    if (!s) return fail(ctx, NC_ERR_INVALID_ARG, "sampling is NULL");
    if (s->spp < 0) return fail(ctx, NC_ERR_INVALID_ARG, "negative spp");
    if (n_jobs == 0 || s->spp == 0) return NC_OK;
    if ((s->flags & NC_SUN_ESTIMATOR_MASK) == 3) return fail(ctx, NC_ERR_INVALID_ARG, "unknown sun estimator");
    if (!cams || !optics || !out_offsets || !d_kc || !d_sum || !d_sumsq)
        return fail(ctx, NC_ERR_INVALID_ARG, "NULL buffer");
    if (s->sample_offset + (uint64_t)s->spp > 0xffffffffull)
        return fail(ctx, NC_ERR_INVALID_ARG, "sample_offset + spp must fit in 32 bits");
    std::vector<nc::JobView> jobs((size_t)n_jobs);
    for (int j = 0; j < n_jobs; ++j) {
        if ((st = check_optics(ctx, optics + j)) != NC_OK) return st;
        if ((st = check_kdist_grid(ctx, optics + j, g)) != NC_OK) return st;
        const nc_optics &a = optics[0], &b = optics[j];
        if (a.ssa != b.ssa || a.g != b.g || a.majorant_scale != b.majorant_scale || a.max_scatter != b.max_scatter ||
            a.max_segments != b.max_segments || a.sun_half_angle_deg != b.sun_half_angle_deg || a.phase != b.phase ||
            !same_kdist(a.kdist, b.kdist))
            return fail(ctx, NC_ERR_INVALID_ARG, "the medium's optics must be the same for every job");
        nc::CamView cam;
        if ((st = make_cam(ctx, cams + j, cam)) != NC_OK) return st;
        if (cam.type == 2 && !sensor_sun_ok(optics + j))
            return fail(ctx, NC_ERR_RANGE, "an irradiance sensor needs the sun above the horizon");
        jobs[j] = make_job(cam, optics + j, out_offsets[j]);
    }
    if (guides) {
        int runs = 0;
        for (int j = 0; j < n_jobs; ++j) {
            if (!guides[j]) return fail(ctx, NC_ERR_INVALID_ARG, "a job's guide is NULL");
            if (guides[j]->device != ctx->device) return fail(ctx, NC_ERR_INVALID_ARG, "guide lives on another device");
            if (j == 0 || guides[j] != guides[j - 1]) ++runs;
        }
        if (runs > NC_BATCH_MAX_GUIDES)
            return fail(ctx, NC_ERR_INVALID_ARG,
                        "jobs sharing a guide must be consecutive, in at most NC_BATCH_MAX_GUIDES runs");
        if (!(s->guide_frac >= 0.0f && s->guide_frac <= 1.0f))
            return fail(ctx, NC_ERR_INVALID_ARG, "guide_frac must lie in [0, 1]");
    }
    DeviceGuard guard(ctx->device);
    nc::RenderScratch scr;
    hipError_t e = hipSuccess;
    if (noalloc) {
        scr = nc::noalloc_render_scratch(ctx->device);
        if (!scr.jobs) return fail(ctx, NC_ERR_DEVICE, "no-allocation scratch not set up on this device");
    } else {
        e = ensure_jobs(ctx, (size_t)n_jobs);
        scr = ctx_render_scratch(ctx);
    }
    if (e == hipSuccess)
        e = nc::launch_render(ctx, g, d_kc, make_opt(optics, g->params.k_gas), jobs.data(), n_jobs, *s, d_sum,
                              d_sumsq, d_counters, scr, guides, nullptr);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "render batch");
}

nc_status nc_render_batch(nc_ctx *ctx, const nc_grid *g, const float *d_kc, int32_t n_jobs, const nc_camera *cams,
                          const nc_optics *optics, const uint64_t *out_offsets, const nc_sampling *s, double *d_sum,
                          double *d_sumsq, nc_counters *d_counters)
{
    return render_batch_common(ctx, g, d_kc, n_jobs, cams, optics, out_offsets, s, nullptr, d_sum, d_sumsq,
                               d_counters);
}

nc_status nc_render_batch_noalloc(nc_ctx *ctx, const nc_grid *g, const float *d_kc, int32_t n_jobs,
                                  const nc_camera *cams, const nc_optics *optics, const uint64_t *out_offsets,
                                  const nc_sampling *s, double *d_sum, double *d_sumsq, nc_counters *d_counters)
{
    return render_batch_common(ctx, g, d_kc, n_jobs, cams, optics, out_offsets, s, nullptr, d_sum, d_sumsq,
                               d_counters, true);
}

nc_status nc_render_batch_guided(nc_ctx *ctx, const nc_grid *g, const float *d_kc, int32_t n_jobs,
                                 const nc_camera *cams, const nc_optics *optics, const uint64_t *out_offsets,
                                 const nc_sampling *s, const nc_guide *const *guides, double *d_sum,
                                 double *d_sumsq, nc_counters *d_counters)
{
    if (!guides && n_jobs > 0) return fail(ctx, NC_ERR_INVALID_ARG, "guides is NULL");
    return render_batch_common(ctx, g, d_kc, n_jobs, cams, optics, out_offsets, s, guides, d_sum, d_sumsq,
                               d_counters);
}

nc_status nc_get_launch(const nc_ctx *ctx, nc_launch *launch)
{
    if (!ctx || !launch) return fail(nullptr, NC_ERR_INVALID_ARG, "NULL argument");
    *launch = ctx->launch;
    return NC_OK;
}

// Coordinate descent over the launch knobs (samples per queue item, workgroup
// size, resident waves per CU, i.e. the register budget, LDS-staged levels),
// starting from the library defaults; each candidate runs `render` twice on
// the context's stream (a warm-up, then a run timed with HIP events) after
// `clear` has zeroed its outputs.  Leaves the fastest knobs in the context.
static nc_status autotune(nc_ctx *ctx, const std::function<nc_status()> &clear,
                          const std::function<nc_status()> &render, double *best_ms)
{
    const int spis[] = {1, 2, 4, 8, 16};
    const int blocks[] = {64, 128, 256};
    const int waves[] = {12, 16};
    const int ldsl[] = {0, 2, -1};
    nc_launch cur{256, 16, 4, -1};   // the library defaults
    hipEvent_t e0 = nullptr, e1 = nullptr;
    DeviceGuard guard(ctx->device);
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he != hipSuccess) return hip_fail(ctx, he, "hipEventCreate");
    auto time_one = [&](const nc_launch &ln, float &ms) -> nc_status {
        ctx->launch = ln;
        nc_status r = clear();
        if (r == NC_OK) r = render();   // warm-up
        if (r != NC_OK) return r;
        (void)hipEventRecord(e0, ctx->stream);
        r = render();
        if (r != NC_OK) return r;
        (void)hipEventRecord(e1, ctx->stream);
        hipError_t e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "autotune timing");
    };
    float best = 0.0f;
    nc_status st = time_one(cur, best);
    for (int pass = 0; pass < 4 && st == NC_OK; ++pass) {
        const int n = pass == 0 ? 5 : pass == 1 ? 3 : pass == 2 ? 2 : 3;
        for (int k = 0; k < n && st == NC_OK; ++k) {
            nc_launch cand = cur;
            if (pass == 0) cand.samples_per_item = spis[k];
            if (pass == 1) cand.block = blocks[k];
            if (pass == 2) cand.waves_per_cu = waves[k];
            if (pass == 3) cand.lds_levels = ldsl[k];
            if (std::memcmp(&cand, &cur, sizeof(cand)) == 0) continue;
            float ms = 0.0f;
            st = time_one(cand, ms);
            if (st == NC_OK && ms < best) {
                best = ms;
                cur = cand;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->launch = cur;
    if (st != NC_OK) return st;
    if (best_ms) *best_ms = best;
    return NC_OK;
}

static nc_status clear_f64(nc_ctx *ctx, double *p, size_t n)
{
    const hipError_t e = hipMemsetAsync(p, 0, n * sizeof(double), ctx->stream);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "autotune clear");
}

nc_status nc_autotune_render(nc_ctx *ctx, const nc_grid *g, const float *d_kc, const nc_optics *optics,
                             const nc_camera *camera, const nc_sampling *s, double *d_sum, double *d_sumsq,
                             double *best_ms)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    if (!s || s->spp < 1) return fail(ctx, NC_ERR_INVALID_ARG, "autotuning needs spp >= 1");
    if (!camera || !d_sum || !d_sumsq) return fail(ctx, NC_ERR_INVALID_ARG, "NULL argument");
    const size_t npix = (size_t)std::max(1, camera->width) * std::max(1, camera->height);
    return autotune(
        ctx,
        [&]() {
            nc_status r = clear_f64(ctx, d_sum, npix);
            return r == NC_OK ? clear_f64(ctx, d_sumsq, npix) : r;
        },
        [&]() { return nc_render(ctx, g, d_kc, optics, camera, s, d_sum, d_sumsq, nullptr); }, best_ms);
}

nc_status nc_autotune_batch(nc_ctx *ctx, const nc_grid *g, const float *d_kc, int32_t n_jobs, const nc_camera *cams,
                            const nc_optics *optics, const uint64_t *out_offsets, const nc_sampling *s, double *d_sum,
                            double *d_sumsq, double *best_ms)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    if (!s || s->spp < 1) return fail(ctx, NC_ERR_INVALID_ARG, "autotuning needs spp >= 1");
    if (n_jobs < 1 || !cams || !out_offsets || !d_sum || !d_sumsq) return fail(ctx, NC_ERR_INVALID_ARG, "NULL argument");
    size_t total = 0;
    for (int j = 0; j < n_jobs; ++j)
        total = std::max<size_t>(total, out_offsets[j] + (size_t)std::max(0, cams[j].width) * std::max(0, cams[j].height));
    return autotune(
        ctx,
        [&]() {
            nc_status r = clear_f64(ctx, d_sum, total);
            return r == NC_OK ? clear_f64(ctx, d_sumsq, total) : r;
        },
        [&]() {
            return nc_render_batch(ctx, g, d_kc, n_jobs, cams, optics, out_offsets, s, d_sum, d_sumsq, nullptr);
        },
        best_ms);
}

static nc_status flux_common(nc_ctx *ctx, const nc_grid *g, const float *d_kc, const nc_optics *optics,
                             double scale, int32_t px_nx, int32_t px_ny, const nc_sampling *s)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    nc_status st = check_grid(ctx, g);
    if (st != NC_OK) return st;
    if ((st = check_optics(ctx, optics)) != NC_OK) return st;
    if (optics->sun_half_angle_deg != 0.0)
        return fail(ctx, NC_ERR_UNSUPPORTED, "forward photons take the directional sun only");
    if (optics->phase) return fail(ctx, NC_ERR_UNSUPPORTED, "forward photons take the HG phase function only");
    if (optics->kdist) return fail(ctx, NC_ERR_UNSUPPORTED, "forward photons take the grid's gas extinction only");
    if (!s) return fail(ctx, NC_ERR_INVALID_ARG, "sampling is NULL");
    if (!(scale > 0.0) || !std::isfinite(scale)) return fail(ctx, NC_ERR_RANGE, "extinction_scale must be > 0");
    if (px_nx < 1 || px_ny < 1 || (long long)px_nx * px_ny > (1ll << 28))
        return fail(ctx, NC_ERR_INVALID_ARG, "bad ground pixel grid");
    if (!d_kc) return fail(ctx, NC_ERR_INVALID_ARG, "field pointer is NULL");
    return NC_OK;
}

nc_status nc_flux(nc_ctx *ctx, const nc_grid *g, const float *d_kc, const nc_optics *optics, double extinction_scale,
                  int32_t px_nx, int32_t px_ny, uint64_t n_photons, const nc_sampling *s, double *d_tally,
                  double *d_global, nc_counters *d_counters)
{
    nc_status st = flux_common(ctx, g, d_kc, optics, extinction_scale, px_nx, px_ny, s);
    if (st != NC_OK) return st;
    if (!d_tally || !d_global) return fail(ctx, NC_ERR_INVALID_ARG, "NULL buffer");
    if (n_photons == 0) return NC_OK;
    DeviceGuard guard(ctx->device);
    hipError_t e = nc::launch_flux(ctx, g, d_kc, make_opt(optics, g->params.k_gas), (float)extinction_scale, px_nx,
                                   px_ny, n_photons, *s, d_tally, d_global, nullptr, nullptr, d_counters);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "flux");
}

nc_status nc_flux_adjoint(nc_ctx *ctx, const nc_grid *g, const float *d_kc, const nc_optics *optics,
                          double extinction_scale, int32_t px_nx, int32_t px_ny, uint64_t n_photons,
                          const nc_sampling *s, const double *d_grad, double *d_out)
{
    nc_status st = flux_common(ctx, g, d_kc, optics, extinction_scale, px_nx, px_ny, s);
    if (st != NC_OK) return st;
    if (!d_grad || !d_out) return fail(ctx, NC_ERR_INVALID_ARG, "NULL buffer");
    if (n_photons == 0) return NC_OK;
    DeviceGuard guard(ctx->device);
    hipError_t e = nc::launch_flux(ctx, g, d_kc, make_opt(optics, g->params.k_gas), (float)extinction_scale, px_nx,
                                   px_ny, n_photons, *s, nullptr, nullptr, d_grad, d_out, nullptr);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "flux adjoint");
}

nc_status nc_guide_create(nc_ctx *ctx, uint64_t seed, nc_guide **out)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    if (!out) return fail(ctx, NC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    DeviceGuard guard(ctx->device);
    nc_guide *gd = new (std::nothrow) nc_guide();
    if (!gd) return fail(ctx, NC_ERR_OOM, "host allocation failed");
    gd->device = ctx->device;
    const size_t np = nc::kGuideParams;
    hipError_t e = hipMalloc(&gd->d_params, np * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&gd->d_m, np * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&gd->d_v, np * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&gd->d_grad, np * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&gd->d_acc, 2 * sizeof(double));
    const int in_pad[4] = {16, 64, 64, 64}, out_pad[4] = {64, 64, 64, 48};
    for (int l = 0; l < 4 && e == hipSuccess; ++l) {
        e = hipMalloc(&gd->d_w[l], sizeof(short) * in_pad[l] * out_pad[l]);
        if (e == hipSuccess) e = hipMalloc(&gd->d_wt[l], sizeof(short) * in_pad[l] * out_pad[l]);
        if (e == hipSuccess) e = hipMalloc(&gd->d_bias[l], sizeof(float) * out_pad[l]);
    }
    if (e != hipSuccess) {
        nc_guide_destroy(gd);
        return hip_fail(ctx, e, "hipMalloc(guide)");
    }
    // He-uniform weights U(-sqrt(6/in), sqrt(6/in)) from a splitmix64 stream, zero biases
    std::vector<float> h(np, 0.0f), zero(np, 0.0f);
    uint64_t st = seed;
    auto next_u = [&st]() {
        uint64_t z = (st += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * (1.0 / 9007199254740992.0);
    };
    const int ins[4] = {nc::kGuideIn, 64, 64, 64}, outs[4] = {64, 64, 64, 40};
    size_t k = 0;
    for (int l = 0; l < 4; ++l) {
        const double lim = std::sqrt(6.0 / ins[l]);
        for (int i = 0; i < outs[l] * ins[l]; ++i) h[k++] = (float)((2.0 * next_u() - 1.0) * lim);
        k += outs[l];
    }
    e = hipMemcpyAsync(gd->d_params, h.data(), np * sizeof(float), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(gd->d_m, zero.data(), np * sizeof(float), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(gd->d_v, zero.data(), np * sizeof(float), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = nc::guide_pack(ctx, gd);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        nc_guide_destroy(gd);
        return hip_fail(ctx, e, "guide init");
    }
    *out = gd;
    return NC_OK;
}

void nc_guide_destroy(nc_guide *gd)
{
    if (!gd) return;
    DeviceGuard guard(gd->device);
    (void)hipFree(gd->d_params);
    (void)hipFree(gd->d_m);
    (void)hipFree(gd->d_v);
    (void)hipFree(gd->d_grad);
    (void)hipFree(gd->d_acc);
    for (int l = 0; l < 4; ++l) {
        (void)hipFree(gd->d_w[l]);
        (void)hipFree(gd->d_wt[l]);
        (void)hipFree(gd->d_bias[l]);
    }
    (void)hipFree(gd->d_scratch);
    delete gd;
}

static nc_status guide_check(nc_ctx *ctx, const nc_guide *gd)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    if (!gd) return fail(ctx, NC_ERR_INVALID_ARG, "guide is NULL");
    if (gd->device != ctx->device) return fail(ctx, NC_ERR_STATE, "guide lives on another device");
    return NC_OK;
}

nc_status nc_guide_get_params(nc_ctx *ctx, const nc_guide *gd, float *d_params)
{
    nc_status st = guide_check(ctx, gd);
    if (st != NC_OK) return st;
    if (!d_params) return fail(ctx, NC_ERR_INVALID_ARG, "NULL buffer");
    DeviceGuard guard(ctx->device);
    hipError_t e = hipMemcpyAsync(d_params, gd->d_params, sizeof(float) * nc::kGuideParams, hipMemcpyDeviceToDevice,
                                  ctx->stream);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "guide get params");
}

nc_status nc_guide_set_params(nc_ctx *ctx, nc_guide *gd, const float *d_params)
{
    nc_status st = guide_check(ctx, gd);
    if (st != NC_OK) return st;
    if (!d_params) return fail(ctx, NC_ERR_INVALID_ARG, "NULL buffer");
    DeviceGuard guard(ctx->device);
    hipError_t e = hipMemcpyAsync(gd->d_params, d_params, sizeof(float) * nc::kGuideParams, hipMemcpyDeviceToDevice,
                                  ctx->stream);
    if (e == hipSuccess) e = nc::guide_pack(ctx, gd);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "guide set params");
}

nc_status nc_guide_forward(nc_ctx *ctx, const nc_guide *gd, const float *d_in, int32_t n, int32_t stride,
                           float *d_out)
{
    nc_status st = guide_check(ctx, gd);
    if (st != NC_OK) return st;
    if (n < 0 || stride < nc::kGuideRaw) return fail(ctx, NC_ERR_INVALID_ARG, "bad size or stride");
    if (n == 0) return NC_OK;
    if (!d_in || !d_out) return fail(ctx, NC_ERR_INVALID_ARG, "NULL buffer");
    DeviceGuard guard(ctx->device);
    hipError_t e = nc::guide_forward(ctx, gd, d_in, n, stride, d_out, nullptr, nullptr, nullptr);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "guide forward");
}

nc_status nc_guide_train_step(nc_ctx *ctx, nc_guide *gd, const float *d_records, int32_t n, float lr, double *d_loss)
{
    nc_status st = guide_check(ctx, gd);
    if (st != NC_OK) return st;
    if (n < 1) return fail(ctx, NC_ERR_INVALID_ARG, "need at least one record");
    if (!d_records) return fail(ctx, NC_ERR_INVALID_ARG, "NULL buffer");
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return fail(ctx, NC_ERR_RANGE, "bad learning rate");
    DeviceGuard guard(ctx->device);
    hipError_t e = nc::guide_train_step(ctx, gd, d_records, n, nc::kGuideRecord, lr, d_loss, true);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "guide train step");
}

nc_status nc_guide_gradient(nc_ctx *ctx, nc_guide *gd, const float *d_records, int32_t n, float *d_grad,
                            double *d_loss)
{
    nc_status st = guide_check(ctx, gd);
    if (st != NC_OK) return st;
    if (n < 1) return fail(ctx, NC_ERR_INVALID_ARG, "need at least one record");
    if (!d_records || !d_grad) return fail(ctx, NC_ERR_INVALID_ARG, "NULL buffer");
    DeviceGuard guard(ctx->device);
    hipError_t e = nc::guide_train_step(ctx, gd, d_records, n, nc::kGuideRecord, 0.0f, d_loss, false);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_grad, gd->d_grad, sizeof(float) * nc::kGuideParams, hipMemcpyDeviceToDevice,
                           ctx->stream);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "guide gradient");
}

nc_status nc_philox4x32_10(nc_ctx *ctx, const uint32_t *d_ctr, const uint32_t *d_key, uint32_t *d_out, int32_t n)
{
    if (!ctx) return fail(nullptr, NC_ERR_INVALID_ARG, "ctx is NULL");
    if (n < 0) return fail(ctx, NC_ERR_INVALID_ARG, "negative size");
    if (n == 0) return NC_OK;
    if (!d_ctr || !d_key || !d_out) return fail(ctx, NC_ERR_INVALID_ARG, "NULL buffer");
    DeviceGuard guard(ctx->device);
    hipError_t e = nc::launch_philox(ctx, d_ctr, d_key, d_out, n);
    return e == hipSuccess ? NC_OK : hip_fail(ctx, e, "philox");
}

}  // extern "C"
