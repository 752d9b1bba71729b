"""Python binding of the C ABI (argument marshalling only).

Every estimator runs in the HIP kernels of libnctrace.so; PyTorch provides
device memory and the stream.  Names follow include/nctrace.h.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import asdict

import numpy as np

import torch

from . import _lib
from .inputs import Camera, FieldDesc, GridParams, Optics, Sampling


def _check(status, ctx_handle=None):
    if status != _lib.NC_OK:
        msg = _lib.load().nc_last_error(ctx_handle)
        raise _lib.NcError(status, msg.decode() if msg else "")


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _desc(d: FieldDesc):
    return _lib.FieldDesc(d.nx, d.ny, d.nz, 0, d.x0, d.y0, d.z0, d.dx, d.dy, d.dz)


class PhaseTable:
    """A tabulated phase function on the device (nc_phase_*): values p at
    cosines mu (-1 .. 1, increasing), linear in between, normalised by the
    library."""

    def __init__(self, ctx, mu, p):
        self.ctx = ctx
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        p = np.ascontiguousarray(p, dtype=np.float64)
        h = C.c_void_p()
        _check(_lib.load().nc_phase_create(ctx.handle, mu.ctypes.data, p.ctypes.data, len(mu), C.byref(h)), ctx.handle)
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _lib.load().nc_phase_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sample(self, u: torch.Tensor) -> torch.Tensor:
        """u (n,) float32 on the device -> (n, 2): sampled cosine, phase function there."""
        u = u.contiguous()
        out = torch.empty((u.numel(), 2), dtype=torch.float32, device=u.device)
        _check(_lib.load().nc_phase_sample(self.ctx.handle, self.handle, _ptr(u), u.numel(), _ptr(out)),
               self.ctx.handle)
        return out


# device copies of the tables that Optics.phase_table names, per context
_PHASE_CACHE = {}


def _phase_handle(o: Optics, ctx):
    tab = getattr(o, "phase_table", None)
    if tab is None:
        return None
    if isinstance(tab, PhaseTable):
        return tab.handle
    mu, p = tab
    key = (id(ctx), id(mu), id(p))
    hit = _PHASE_CACHE.get(key)
    if hit is None or hit[1] is not mu or hit[2] is not p:
        hit = (PhaseTable(ctx, mu, p), mu, p)
        _PHASE_CACHE[key] = hit
    return hit[0].handle


def _optics(o: Optics, ctx=None):
    ph = _phase_handle(o, ctx) if ctx is not None else None
    if getattr(o, "phase_table", None) is not None and ph is None:
        raise ValueError("a phase table needs the context")
    r = _lib.Optics(o.ssa, o.g, o.ground_albedo, o.sun_zenith_deg, o.sun_azimuth_deg, o.sun_irradiance,
                    o.majorant_scale, o.max_scatter, o.max_segments, o.sun_half_angle_deg, ph, None)
    kd = getattr(o, "kdist", None)
    if kd is not None:
        w, k = (np.asarray(a, dtype=np.float64).ravel() for a in kd)
        if len(w) != len(k) or not 1 <= len(w) <= _lib.KDIST_MAX:
            raise ValueError("a k-distribution needs 1 .. %d (weight, k_gas) pairs" % _lib.KDIST_MAX)
        rec = _lib.KDist()
        rec.n = len(w)
        for i in range(len(w)):
            rec.w[i] = w[i]
            rec.k_gas[i] = k[i]
        r._kdist = rec                      # kept alive with the optics record
        r.kdist = C.addressof(rec)
    return r


def _camera(c: Camera):
    cc = _lib.Camera()
    cc.type, cc.width, cc.height = c.type, c.width, c.height
    for i in range(3):
        cc.pos[i], cc.target[i], cc.up[i] = c.pos[i], c.target[i], c.up[i]
    cc.fov_y_deg, cc.ortho_w, cc.ortho_h = c.fov_y_deg, c.ortho_w, c.ortho_h
    return cc


def _sampling(s: Sampling):
    return _lib.Sampling(s.seed, s.sample_offset, s.spp, s.flags, s.guide_frac, s.stream, s.guide_max_order)


def counters_dict(t: torch.Tensor):
    v = t.cpu().numpy()
    return {k: int(v[i]) for i, k in enumerate(_lib.COUNTER_NAMES)}


class Context:
    """A library context on one device, enqueueing on torch's current stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        L = _lib.load()
        self.device = device
        s = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        st = L.nc_ctx_create(device, C.c_void_p(s.cuda_stream), C.byref(h))
        _check(st, None)
        self.handle = h
        self.stream = s

    def set_stream(self, stream: torch.cuda.Stream):
        _check(_lib.load().nc_ctx_set_stream(self.handle, C.c_void_p(stream.cuda_stream)), self.handle)
        self.stream = stream

    def set_launch(self, block=0, waves_per_cu=0, samples_per_item=0, lds_levels=-1):
        ln = _lib.Launch(block, waves_per_cu, samples_per_item, lds_levels)
        _check(_lib.load().nc_set_launch(self.handle, C.byref(ln)), self.handle)

    def get_launch(self):
        ln = _lib.Launch()
        _check(_lib.load().nc_get_launch(self.handle, C.byref(ln)), self.handle)
        return dict(block=ln.block, waves_per_cu=ln.waves_per_cu, samples_per_item=ln.samples_per_item,
                    lds_levels=ln.lds_levels)

    def close(self):
        if getattr(self, "handle", None):
            _lib.load().nc_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self):
        m = _lib.load().nc_last_error(self.handle)
        return m.decode() if m else ""


class Grid:
    """Hierarchical min/max extinction grid (library-owned device memory)."""

    def __init__(self, ctx: Context, kc: torch.Tensor, desc: FieldDesc, params: GridParams):
        assert kc.is_cuda and kc.dtype == torch.float32 and kc.is_contiguous()
        assert tuple(kc.shape) == (desc.nz, desc.ny, desc.nx)
        self.ctx, self.desc, self.params = ctx, desc, params
        h = C.c_void_p()
        d = _desc(desc)
        p = _lib.GridParams(params.tau_tilde, params.k_gas, params.criterion, params.flat_level)
        _check(_lib.load().nc_grid_build(ctx.handle, _ptr(kc), C.byref(d), C.byref(p), C.byref(h)), ctx.handle)
        self.handle = h
        lv = C.c_int32()
        _check(_lib.load().nc_grid_info(self.handle, C.byref(lv), 0, None))
        self.L = lv.value

    def close(self):
        if getattr(self, "handle", None):
            _lib.load().nc_grid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def rebuild(self, kc: torch.Tensor):
        """Rebuild in place over a field of the same shape."""
        assert kc.is_cuda and kc.dtype == torch.float32 and kc.is_contiguous()
        assert tuple(kc.shape) == (self.desc.nz, self.desc.ny, self.desc.nx)
        _check(_lib.load().nc_grid_rebuild(self.ctx.handle, self.handle, _ptr(kc)), self.ctx.handle)

    def mask(self):
        """Ancestry mask per level-1 node (int32 view of the uint16 bits)."""
        nx, ny, nz = self.level_dims(1)
        m = torch.empty((nz, ny, nx), dtype=torch.int16, device=torch.device("cuda", self.ctx.device))
        _check(_lib.load().nc_grid_export_mask(self.ctx.handle, self.handle, _ptr(m)), self.ctx.handle)
        return m.to(torch.int32) & 0xFFFF

    def level_dims(self, level):
        d = (C.c_int32 * 3)()
        _check(_lib.load().nc_grid_info(self.handle, None, level, C.cast(d, C.c_void_p)))
        return tuple(int(v) for v in d)   # (nx, ny, nz)

    def level(self, level):
        nx, ny, nz = self.level_dims(level)
        dev = torch.device("cuda", self.ctx.device)
        kmin = torch.empty((nz, ny, nx), dtype=torch.float32, device=dev)
        kmax = torch.empty_like(kmin)
        mg = torch.empty((nz, ny, nx), dtype=torch.uint8, device=dev)
        _check(_lib.load().nc_grid_export(self.ctx.handle, self.handle, level, _ptr(kmin), _ptr(kmax), _ptr(mg)),
               self.ctx.handle)
        return kmin, kmax, mg

    def leaf_levels(self):
        d = self.desc
        out = torch.empty((d.nz, d.ny, d.nx), dtype=torch.uint8, device=torch.device("cuda", self.ctx.device))
        _check(_lib.load().nc_grid_leaf_levels(self.ctx.handle, self.handle, _ptr(out)), self.ctx.handle)
        return out


def build_grid(ctx: Context, kc: torch.Tensor, desc: FieldDesc, params: GridParams) -> Grid:
    return Grid(ctx, kc, desc, params)


def trace_leaves(ctx: Context, grid: Grid, rays: torch.Tensor, max_visits: int):
    n = rays.shape[0]
    dev = rays.device
    leaf = torch.zeros((n, max_visits, 4), dtype=torch.int32, device=dev)
    t = torch.zeros((n, max_visits, 2), dtype=torch.float32, device=dev)
    cnt = torch.zeros(n, dtype=torch.int32, device=dev)
    _check(_lib.load().nc_trace_leaves(ctx.handle, grid.handle, _ptr(rays.contiguous()), n, max_visits, _ptr(leaf),
                                       _ptr(t), _ptr(cnt)), ctx.handle)
    return leaf, t, cnt


def new_counters(device):
    return torch.zeros(_lib.N_COUNTER_WORDS, dtype=torch.int64, device=device)


def transmittance(ctx: Context, grid: Grid, kc: torch.Tensor, optics: Optics, rays: torch.Tensor,
                  sampling: Sampling, counters: torch.Tensor | None = None):
    n = rays.shape[0]
    s = torch.zeros(n, dtype=torch.float64, device=rays.device)
    s2 = torch.zeros_like(s)
    o = _optics(optics, ctx)
    sm = _sampling(sampling)
    _check(_lib.load().nc_transmittance(ctx.handle, grid.handle, _ptr(kc), C.byref(o), _ptr(rays.contiguous()), n,
                                        C.byref(sm), _ptr(s), _ptr(s2), _ptr(counters)), ctx.handle)
    return s, s2


def render(ctx: Context, grid: Grid, kc: torch.Tensor, optics: Optics, camera: Camera, sampling: Sampling,
           out_sum: torch.Tensor | None = None, out_sumsq: torch.Tensor | None = None,
           counters: torch.Tensor | None = None):
    dev = kc.device
    if out_sum is None:
        out_sum = torch.zeros((camera.height, camera.width), dtype=torch.float64, device=dev)
    if out_sumsq is None:
        out_sumsq = torch.zeros((camera.height, camera.width), dtype=torch.float64, device=dev)
    o = _optics(optics, ctx)
    c = _camera(camera)
    sm = _sampling(sampling)
    _check(_lib.load().nc_render(ctx.handle, grid.handle, _ptr(kc), C.byref(o), C.byref(c), C.byref(sm),
                                 _ptr(out_sum), _ptr(out_sumsq), _ptr(counters)), ctx.handle)
    return out_sum, out_sumsq


def render_guided(ctx: Context, grid: Grid, kc: torch.Tensor, optics: Optics, camera: Camera, sampling: Sampling,
                  guide: "Guide", out_sum: torch.Tensor | None = None, out_sumsq: torch.Tensor | None = None,
                  counters: torch.Tensor | None = None):
    """Guided radiance image (nc_render_guided): one-sample MIS between the
    guide's vMF mixture (probability sampling.guide_frac) and HG."""
    dev = kc.device
    if out_sum is None:
        out_sum = torch.zeros((camera.height, camera.width), dtype=torch.float64, device=dev)
    if out_sumsq is None:
        out_sumsq = torch.zeros((camera.height, camera.width), dtype=torch.float64, device=dev)
    o = _optics(optics, ctx)
    c = _camera(camera)
    sm = _sampling(sampling)
    _check(_lib.load().nc_render_guided(ctx.handle, grid.handle, _ptr(kc), C.byref(o), C.byref(c), C.byref(sm),
                                        guide.handle, _ptr(out_sum), _ptr(out_sumsq), _ptr(counters)), ctx.handle)
    return out_sum, out_sumsq


def render_progressive(ctx: Context, grid: Grid, kc: torch.Tensor, optics: Optics, camera: Camera,
                       sampling: Sampling, target_rel_err: float = 0.01, first_spp: int = 16, max_spp: int = 1 << 20,
                       block: int = 1, guide: "Guide | None" = None, counters: torch.Tensor | None = None):
    """Render in rounds until the image's relative standard error reaches the
    target (nc_render_progressive).  Returns (sum, sumsq, report dict)."""
    dev = kc.device
    out_sum = torch.zeros((camera.height, camera.width), dtype=torch.float64, device=dev)
    out_sumsq = torch.zeros((camera.height, camera.width), dtype=torch.float64, device=dev)
    plan = _lib.Progressive(float(target_rel_err), int(first_spp), int(max_spp), int(block), 0)
    rep = _lib.ProgressReport()
    o = _optics(optics, ctx)
    c = _camera(camera)
    sm = _sampling(sampling)
    _check(_lib.load().nc_render_progressive(ctx.handle, grid.handle, _ptr(kc), C.byref(o), C.byref(c), C.byref(sm),
                                             guide.handle if guide is not None else None, C.byref(plan),
                                             _ptr(out_sum), _ptr(out_sumsq), _ptr(counters), C.byref(rep)),
           ctx.handle)
    return out_sum, out_sumsq, {k: getattr(rep, k) for k in ("spp_done", "rounds", "rel_err", "mean", "seconds")}


def gather_rate(ctx: Context, buf: torch.Tensor, threads: int = 1 << 20, loads: int = 64) -> float:
    """Random 4-byte reads per second over buf (float32, power-of-two length): nc_gather_rate."""
    out = torch.empty(threads, dtype=torch.float32, device=buf.device)
    r = C.c_double()
    _check(_lib.load().nc_gather_rate(ctx.handle, _ptr(buf), buf.numel(), int(threads), int(loads), _ptr(out),
                                      C.byref(r)), ctx.handle)
    return r.value


def collect_vertices(ctx: Context, grid: Grid, kc: torch.Tensor, optics: Optics, camera: Camera,
                     sampling: Sampling, capacity: int, counters: torch.Tensor | None = None):
    """Training vertices (nc_collect_vertices).  Returns (records (m, 12) with
    m = min(events, capacity), number of events, sum image, sum-of-squares image)."""
    dev = kc.device
    records = torch.empty((max(int(capacity), 1), _lib.GUIDE_RECORD), dtype=torch.float32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    path_L = torch.empty(max(camera.width * camera.height * sampling.spp, 1), dtype=torch.float32, device=dev)
    out_sum = torch.zeros((camera.height, camera.width), dtype=torch.float64, device=dev)
    out_sumsq = torch.zeros((camera.height, camera.width), dtype=torch.float64, device=dev)
    o = _optics(optics, ctx)
    c = _camera(camera)
    sm = _sampling(sampling)
    _check(_lib.load().nc_collect_vertices(ctx.handle, grid.handle, _ptr(kc), C.byref(o), C.byref(c), C.byref(sm),
                                           _ptr(records), int(capacity), _ptr(count), _ptr(path_L), _ptr(out_sum),
                                           _ptr(out_sumsq), _ptr(counters)), ctx.handle)
    n = int(count.item())
    return records[:min(n, int(capacity))], n, out_sum, out_sumsq


def philox4x32_10(ctx: Context, ctr: torch.Tensor, key: torch.Tensor) -> torch.Tensor:
    """ctr: (n, 4) int32 (bit patterns of uint32), key: (n, 2) int32 -> (n, 4) int32."""
    n = ctr.shape[0]
    out = torch.empty((n, 4), dtype=torch.int32, device=ctr.device)
    _check(_lib.load().nc_philox4x32_10(ctx.handle, _ptr(ctr.contiguous()), _ptr(key.contiguous()), _ptr(out), n),
           ctx.handle)
    return out


def flux(ctx: Context, grid: Grid, kc: torch.Tensor, optics: Optics, px: tuple, n_photons: int,
         sampling: Sampling, extinction_scale: float = 1.0, counters: torch.Tensor | None = None):
    """Forward photons (nc_flux): raw tallies [9, py, px] and terminal counts [4], float64 on the device."""
    nx, ny = px
    tally = torch.zeros((9, ny, nx), dtype=torch.float64, device=kc.device)
    glob = torch.zeros(4, dtype=torch.float64, device=kc.device)
    o = _optics(optics, ctx)
    sm = _sampling(sampling)
    _check(_lib.load().nc_flux(ctx.handle, grid.handle, _ptr(kc), C.byref(o), float(extinction_scale), nx, ny,
                               int(n_photons), C.byref(sm), _ptr(tally), _ptr(glob), _ptr(counters)), ctx.handle)
    return tally, glob


def flux_adjoint(ctx: Context, grid: Grid, kc: torch.Tensor, optics: Optics, px: tuple, n_photons: int,
                 sampling: Sampling, grad: torch.Tensor, extinction_scale: float = 1.0):
    """Derivative-path replay (nc_flux_adjoint): raw [sum grad*sigma_s, sum grad*sigma_g, sum grad*sigma_a]."""
    nx, ny = px
    assert tuple(grad.shape) == (ny, nx)
    out = torch.zeros(3, dtype=torch.float64, device=kc.device)
    g64 = grad.to(dtype=torch.float64).contiguous()
    o = _optics(optics, ctx)
    sm = _sampling(sampling)
    _check(_lib.load().nc_flux_adjoint(ctx.handle, grid.handle, _ptr(kc), C.byref(o), float(extinction_scale), nx, ny,
                                       int(n_photons), C.byref(sm), _ptr(g64), _ptr(out)), ctx.handle)
    return out


class TransmissionFn(torch.autograd.Function):
    """Ground transmissivity map T(s, g, alpha) with gradients through the adjoint kernel.

    s scales the droplet extinction, g is the HG asymmetry, alpha = 1 - ssa the
    droplets' absorptivity.  forward: photons traced by nc_flux with
    NC_FLUX_NORMALISE, whose first tally is T_p.  backward: nc_flux_adjoint
    (same flag) replays the same photons weighting each arrival by
    grad_T[p] and returns dL/ds, dL/dg and dL/dalpha for the same samples.
    This class only moves tensors: the kernels compute every number."""

    @staticmethod
    def forward(fctx, scale, g, alpha, lib_ctx, grid, kc, optics, px, n_photons, sampling):
        import dataclasses
        op = dataclasses.replace(optics, g=float(g), ssa=1.0 - float(alpha))
        smp = dataclasses.replace(sampling, flags=sampling.flags | _lib.NC_FLUX_NORMALISE)
        tally, _ = flux(lib_ctx, grid, kc, op, px, n_photons, smp, float(scale))
        fctx.args = (lib_ctx, grid, kc, op, px, n_photons, smp, float(scale))
        fctx.dev = scale.device if torch.is_tensor(scale) else kc.device
        return tally[0]

    @staticmethod
    def backward(fctx, grad_T):
        lib_ctx, grid, kc, op, px, n_photons, smp, s = fctx.args
        out = flux_adjoint(lib_ctx, grid, kc, op, px, n_photons, smp, grad_T, s)
        ds = out[0].to(fctx.dev)
        dg = out[1].to(fctx.dev)
        da = out[2].to(fctx.dev)
        return ds, dg, da, None, None, None, None, None, None, None


def render_batch(ctx: Context, grid: Grid, kc: torch.Tensor, jobs: list, sampling: Sampling,
                 counters: torch.Tensor | None = None, guide=None):
    """Render many (camera, optics) jobs in one persistent launch (nc_render_batch,
    or nc_render_batch_guided when guides are given: one Guide for every job,
    or a list with one per job, jobs sharing a guide consecutive).

    Returns (sum, sumsq, offsets): flat float64 buffers holding the images one
    after the other, and each image's first element."""
    n = len(jobs)
    cams = (_lib.Camera * n)(*[_camera(c) for c, _ in jobs])
    recs = [_optics(o, ctx) for _, o in jobs]   # (they keep any k-distribution records alive through the call)
    opts = (_lib.Optics * n)(*recs)
    offs, total = [], 0
    for c, _ in jobs:
        offs.append(total)
        total += c.width * c.height
    off_arr = (C.c_uint64 * n)(*offs)
    s = torch.zeros(total, dtype=torch.float64, device=kc.device)
    s2 = torch.zeros_like(s)
    sm = _sampling(sampling)
    if guide is None:
        _check(_lib.load().nc_render_batch(ctx.handle, grid.handle, _ptr(kc), n, C.cast(cams, C.c_void_p),
                                           C.cast(opts, C.c_void_p), C.cast(off_arr, C.c_void_p), C.byref(sm), _ptr(s),
                                           _ptr(s2), _ptr(counters)), ctx.handle)
    else:
        per_job = list(guide) if isinstance(guide, (list, tuple)) else [guide] * n
        if len(per_job) != n:
            raise ValueError("one guide per job")
        handles = (C.c_void_p * n)(*[gd.handle for gd in per_job])
        _check(_lib.load().nc_render_batch_guided(ctx.handle, grid.handle, _ptr(kc), n, C.cast(cams, C.c_void_p),
                                                  C.cast(opts, C.c_void_p), C.cast(off_arr, C.c_void_p), C.byref(sm),
                                                  C.cast(handles, C.c_void_p), _ptr(s), _ptr(s2), _ptr(counters)),
               ctx.handle)
    return s, s2, offs


def autotune_render(ctx: Context, grid: Grid, kc: torch.Tensor, optics: Optics, camera: Camera, sampling: Sampling):
    """Pick the fastest launch shape for this view (nc_autotune_render); returns (launch dict, best ms)."""
    s = torch.zeros((camera.height, camera.width), dtype=torch.float64, device=kc.device)
    s2 = torch.zeros_like(s)
    best = C.c_double()
    _check(_lib.load().nc_autotune_render(ctx.handle, grid.handle, _ptr(kc), C.byref(_optics(optics, ctx)),
                                          C.byref(_camera(camera)), C.byref(_sampling(sampling)), _ptr(s), _ptr(s2),
                                          C.byref(best)), ctx.handle)
    return ctx.get_launch(), best.value


def autotune_batch(ctx: Context, grid: Grid, kc: torch.Tensor, jobs: list, sampling: Sampling):
    """Pick the fastest launch shape for this batch (nc_autotune_batch); returns (launch dict, best ms)."""
    n = len(jobs)
    cams = (_lib.Camera * n)(*[_camera(c) for c, _ in jobs])
    recs = [_optics(o, ctx) for _, o in jobs]
    opts = (_lib.Optics * n)(*recs)
    offs, total = [], 0
    for c, _ in jobs:
        offs.append(total)
        total += c.width * c.height
    off_arr = (C.c_uint64 * n)(*offs)
    s = torch.zeros(max(total, 1), dtype=torch.float64, device=kc.device)
    s2 = torch.zeros_like(s)
    best = C.c_double()
    _check(_lib.load().nc_autotune_batch(ctx.handle, grid.handle, _ptr(kc), n, C.cast(cams, C.c_void_p),
                                         C.cast(opts, C.c_void_p), C.cast(off_arr, C.c_void_p),
                                         C.byref(_sampling(sampling)), _ptr(s), _ptr(s2), C.byref(best)), ctx.handle)
    return ctx.get_launch(), best.value


class Guide:
    """The learned proposal's network (nc_guide_*): bf16 MFMA forward/backward, fp32 Adam."""

    def __init__(self, ctx: Context, seed: int = 1):
        self.ctx = ctx
        h = C.c_void_p()
        _check(_lib.load().nc_guide_create(ctx.handle, int(seed), C.byref(h)), ctx.handle)
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _lib.load().nc_guide_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> torch.Tensor:
        p = torch.empty(_lib.GUIDE_PARAMS, dtype=torch.float32, device=torch.device("cuda", self.ctx.device))
        _check(_lib.load().nc_guide_get_params(self.ctx.handle, self.handle, _ptr(p)), self.ctx.handle)
        return p

    def set_params(self, p: torch.Tensor):
        p = p.to(dtype=torch.float32, device=torch.device("cuda", self.ctx.device)).contiguous()
        assert p.numel() == _lib.GUIDE_PARAMS
        _check(_lib.load().nc_guide_set_params(self.ctx.handle, self.handle, _ptr(p)), self.ctx.handle)

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        """x: (n, stride >= 7) float32 -> raw outputs (n, 40)."""
        x = x.contiguous()
        n, stride = x.shape
        out = torch.empty((n, 48), dtype=torch.float32, device=x.device)
        _check(_lib.load().nc_guide_forward(self.ctx.handle, self.handle, _ptr(x), n, stride, _ptr(out)),
               self.ctx.handle)
        return out[:, :40]

    def train_step(self, records: torch.Tensor, lr: float):
        """records: (n, 12) float32.  Returns a (2,) float64 tensor [sum -w ln q, sum w] (not synchronised)."""
        r = records.contiguous()
        loss = torch.zeros(2, dtype=torch.float64, device=r.device)
        _check(_lib.load().nc_guide_train_step(self.ctx.handle, self.handle, _ptr(r), r.shape[0], float(lr),
                                               _ptr(loss)), self.ctx.handle)
        return loss

    def sample(self, inputs: torch.Tensor, u: torch.Tensor, guide_frac: float, g: float) -> torch.Tensor:
        """The renderer's guided scattering step (nc_guide_sample): inputs (n, 8)
        float32, u (n, 4) -> (n, 8) [direction(3), weight factor, q, p, 0, 0]."""
        x = inputs.contiguous()
        uu = u.contiguous()
        out = torch.empty((x.shape[0], 8), dtype=torch.float32, device=x.device)
        _check(_lib.load().nc_guide_sample(self.ctx.handle, self.handle, _ptr(x), _ptr(uu), x.shape[0],
                                           float(guide_frac), float(g), _ptr(out)), self.ctx.handle)
        return out

    def gradient(self, records: torch.Tensor):
        r = records.contiguous()
        g = torch.empty(_lib.GUIDE_PARAMS, dtype=torch.float32, device=r.device)
        loss = torch.zeros(2, dtype=torch.float64, device=r.device)
        _check(_lib.load().nc_guide_gradient(self.ctx.handle, self.handle, _ptr(r), r.shape[0], _ptr(g), _ptr(loss)),
               self.ctx.handle)
        return g, loss
