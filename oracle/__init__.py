"""CPU oracle for null-collision path tracing (test infrastructure only).

This package is the checker: a serial FP64 C implementation (oracle.c) of
what the GPU path computes, written from the paper's definitions, with a
ctypes wrapper.  Only the tests, the smoke entry point and the benchmark's
CPU-baseline leg use it; the product path never imports it.  It shares no
code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (IEEE double, no contraction into FMA)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-Wall", "-Wno-unused-function",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Field(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("pad_", C.c_int32),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("k_gas", C.c_double), ("kc", C.POINTER(C.c_float)), ("kscale", C.c_double)]


class OpticsC(C.Structure):
    _fields_ = [("ssa", C.c_double), ("g", C.c_double), ("rho", C.c_double),
                ("sun_zenith_deg", C.c_double), ("sun_azimuth_deg", C.c_double),
                ("S", C.c_double), ("majorant_scale", C.c_double),
                ("max_scatter", C.c_int32), ("max_segments", C.c_int32), ("sun_half_angle_deg", C.c_double),
                ("tab_n", C.c_int32), ("tab_pad_", C.c_int32), ("tab_mu", C.c_void_p), ("tab_p", C.c_void_p),
                ("kd_n", C.c_int32), ("kd_pad_", C.c_int32), ("kd_w", C.c_void_p), ("kd_k", C.c_void_p)]


class CameraC(C.Structure):
    _fields_ = [("type", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("pad_", C.c_int32),
                ("pos", C.c_double * 3), ("target", C.c_double * 3), ("up", C.c_double * 3),
                ("fov_y_deg", C.c_double), ("ortho_w", C.c_double), ("ortho_h", C.c_double)]


_P = C.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        L.orc_philox4x32_10.argtypes = [_P, _P, _P]
        L.orc_grid_build.argtypes = [C.POINTER(Field), C.c_double, C.c_int, C.c_int]
        L.orc_grid_build.restype = _P
        L.orc_grid_free.argtypes = [_P]
        L.orc_grid_levels.argtypes = [_P]
        L.orc_grid_levels.restype = C.c_int
        L.orc_grid_level_dims.argtypes = [_P, C.c_int, _P]
        L.orc_grid_export.argtypes = [_P, C.c_int, _P, _P, _P]
        L.orc_grid_leaf_levels.argtypes = [_P, _P]
        L.orc_leaf_sequence.argtypes = [C.POINTER(Field), _P, _P, C.c_double, C.c_int32, _P, _P, _P]
        L.orc_leaf_sequence.restype = C.c_int
        L.orc_optical_depth.argtypes = [C.POINTER(Field), _P, C.c_double]
        L.orc_optical_depth.restype = C.c_double
        L.orc_transmittance.argtypes = [C.POINTER(Field), _P, C.c_int, C.c_double, _P, C.c_int32, C.c_int32,
                                        C.c_uint64, _P, _P, _P, _P]
        L.orc_hg_phase.argtypes = [C.c_double, C.c_double]
        L.orc_hg_phase.restype = C.c_double
        L.orc_hg_sample_mu.argtypes = [C.c_double, C.c_double]
        L.orc_hg_sample_mu.restype = C.c_double
        L.orc_tab_phase.argtypes = [_P, _P, C.c_int32, C.c_double]
        L.orc_tab_phase.restype = C.c_double
        L.orc_tab_sample.argtypes = [_P, _P, C.c_int32, C.c_double]
        L.orc_tab_sample.restype = C.c_double
        L.orc_camera_ray.argtypes = [C.POINTER(CameraC), C.c_int, C.c_int, C.c_double, C.c_double, _P]
        L.orc_render.argtypes = [C.POINTER(Field), C.POINTER(OpticsC), C.POINTER(CameraC), C.c_int32, C.c_uint64,
                                 _P, C.c_int32, _P, _P, _P]
        L.orc_render_tracked.argtypes = [C.POINTER(Field), _P, C.POINTER(OpticsC), C.POINTER(CameraC), C.c_int32,
                                         C.c_uint64, _P, C.c_int32, _P, _P, _P, _P]
        L.orc_hg_dlng.argtypes = [C.c_double, C.c_double]
        L.orc_hg_dlng.restype = C.c_double
        L.orc_flux.argtypes = [C.POINTER(Field), _P, C.POINTER(OpticsC), C.c_int32, C.c_int32, C.c_int32,
                               C.c_int64, C.c_uint64, C.c_uint64, _P, _P]
        L.orc_flux_fd.argtypes = [C.POINTER(Field), C.POINTER(OpticsC), C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                  C.c_int64, C.c_uint64, C.c_uint64, _P, _P]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def make_field(desc, kc: np.ndarray, k_gas: float = 0.0, kscale: float = 1.0):
    """Field record pointing at a contiguous float32 (nz, ny, nx) array (kept alive on the record)."""
    kc = np.ascontiguousarray(kc, dtype=np.float32)
    f = Field(desc.nx, desc.ny, desc.nz, 0, desc.x0, desc.y0, desc.z0, desc.dx, desc.dy, desc.dz, float(k_gas),
              kc.ctypes.data_as(C.POINTER(C.c_float)), float(kscale))
    f._keep = kc
    return f


def make_optics(op) -> OpticsC:
    """The optics record; a tabulated phase function (op.phase_table = (mu, p)) replaces HG."""
    o = OpticsC(op.ssa, op.g, op.ground_albedo, op.sun_zenith_deg, op.sun_azimuth_deg, op.sun_irradiance,
                op.majorant_scale, op.max_scatter, op.max_segments, getattr(op, "sun_half_angle_deg", 0.0))
    tab = getattr(op, "phase_table", None)
    if tab is not None:
        mu = np.ascontiguousarray(tab[0], dtype=np.float64)
        p = np.ascontiguousarray(tab[1], dtype=np.float64)
        o.tab_n = len(mu)
        o.tab_mu = mu.ctypes.data
        o.tab_p = p.ctypes.data
        o._keep = (mu, p)
    kd = getattr(op, "kdist", None)
    if kd is not None:
        w = np.ascontiguousarray(kd[0], dtype=np.float64)
        kk = np.ascontiguousarray(kd[1], dtype=np.float64)
        o.kd_n = len(w)
        o.kd_w = w.ctypes.data
        o.kd_k = kk.ctypes.data
        o._keep_kd = (w, kk)
    return o


def tab_phase(mu, p, m):
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    return lib().orc_tab_phase(_ptr(mu), _ptr(p), len(mu), float(m))


def tab_sample(mu, p, xi):
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    return lib().orc_tab_sample(_ptr(mu), _ptr(p), len(mu), float(xi))


def make_camera(cam) -> CameraC:
    c = CameraC()
    c.type, c.width, c.height = cam.type, cam.width, cam.height
    for i in range(3):
        c.pos[i], c.target[i], c.up[i] = cam.pos[i], cam.target[i], cam.up[i]
    c.fov_y_deg, c.ortho_w, c.ortho_h = cam.fov_y_deg, cam.ortho_w, cam.ortho_h
    return c


# ---------------------------------------------------------------------------
# Philox4x32-10
# ---------------------------------------------------------------------------

def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


# ---------------------------------------------------------------------------
# Grid
# ---------------------------------------------------------------------------

class OracleGrid:
    """Per-level (kmin_c, kmax_c, merged) arrays and the per-cell leaf-level map."""

    def __init__(self, desc, kc, tau_tilde=1.0, k_gas=0.0, criterion=0, flat_level=3):
        self.field = make_field(desc, kc, k_gas)
        self.handle = lib().orc_grid_build(C.byref(self.field), float(tau_tilde), int(criterion), int(flat_level))
        if not self.handle:
            raise MemoryError("oracle grid build failed")
        self.L = lib().orc_grid_levels(self.handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.orc_grid_free(h)
            self.handle = None

    def level_dims(self, l):
        d = np.zeros(3, dtype=np.int32)
        lib().orc_grid_level_dims(self.handle, l, _ptr(d))
        return tuple(int(v) for v in d)  # (nx, ny, nz) of the level

    def level(self, l):
        nx, ny, nz = self.level_dims(l)
        kmin = np.zeros((nz, ny, nx), np.float32)
        kmax = np.zeros((nz, ny, nx), np.float32)
        mg = np.zeros((nz, ny, nx), np.uint8)
        lib().orc_grid_export(self.handle, l, _ptr(kmin), _ptr(kmax), _ptr(mg))
        return kmin, kmax, mg

    def leaf_levels(self):
        f = self.field
        out = np.zeros((f.nz, f.ny, f.nx), np.uint8)
        lib().orc_grid_leaf_levels(self.handle, _ptr(out))
        return out

    def leaf_sequence(self, ray, eps, maxv=4096):
        r = np.asarray(ray, dtype=np.float64).copy()
        leaf = np.zeros((maxv, 4), np.int32)
        t = np.zeros((maxv, 2), np.float64)
        deg = np.zeros(1, np.int32)
        n = lib().orc_leaf_sequence(C.byref(self.field), self.handle, _ptr(r), float(eps), maxv,
                                    _ptr(leaf), _ptr(t), _ptr(deg))
        if n > maxv:
            raise ValueError("leaf sequence longer than maxv")
        return leaf[:n].copy(), t[:n].copy(), bool(deg[0])

    def transmittance(self, rays, nsamples, seed, mode=2, majorant_scale=1.0, with_sq=False):
        return transmittance(self.field, rays, nsamples, seed, mode, majorant_scale, grid=self, with_sq=with_sq)


# ---------------------------------------------------------------------------
# Estimators
# ---------------------------------------------------------------------------

def optical_depth(field: Field, ray, t1=np.inf):
    r = np.asarray(ray, dtype=np.float64).copy()
    return lib().orc_optical_depth(C.byref(field), _ptr(r), float(t1))


def transmittance(field: Field, rays, nsamples, seed, mode, majorant_scale=1.0, grid=None, with_sq=False):
    """Per-ray (mean, se, counters[tentative, null, leaf visits]) and, with
    with_sq, the sums of the counters' per-path squares."""
    rays = np.ascontiguousarray(rays, dtype=np.float64).reshape(-1, 6)
    n = rays.shape[0]
    mean = np.zeros(n)
    se = np.zeros(n)
    cnt = np.zeros(3, np.uint64)
    sq = np.zeros(3)
    lib().orc_transmittance(C.byref(field), grid.handle if grid is not None else None, int(mode),
                            float(majorant_scale), _ptr(rays), n, int(nsamples), int(seed),
                            _ptr(mean), _ptr(se), _ptr(cnt), _ptr(sq))
    return (mean, se, cnt, sq) if with_sq else (mean, se, cnt)


def hg_phase(g, mu):
    return lib().orc_hg_phase(float(g), float(mu))


def hg_sample_mu(g, xi):
    return lib().orc_hg_sample_mu(float(g), float(xi))


def camera_ray(cam, px, py, u1, u2):
    c = make_camera(cam)
    out = np.zeros(6)
    lib().orc_camera_ray(C.byref(c), px, py, float(u1), float(u2), _ptr(out))
    return out


def render(desc, kc, k_gas, optics, cam, spp, seed, pixels=None):
    """Backward radiance per pixel: (sum, sumsq, counters) over spp paths.

    counters: [real volume collisions, ground hits, paths]."""
    f = make_field(desc, kc, k_gas)
    op = make_optics(optics)
    c = make_camera(cam)
    if pixels is None:
        pixels = np.arange(cam.width * cam.height, dtype=np.int32)
    pixels = np.ascontiguousarray(pixels, dtype=np.int32)
    s = np.zeros(len(pixels))
    s2 = np.zeros(len(pixels))
    cnt = np.zeros(3, np.uint64)
    lib().orc_render(C.byref(f), C.byref(op), C.byref(c), int(spp), int(seed), _ptr(pixels), len(pixels),
                     _ptr(s), _ptr(s2), _ptr(cnt))
    return s, s2, cnt


def render_tracked(desc, kc, k_gas, optics, cam, spp, seed, grid, pixels=None):
    """Backward radiance with every ray null-collision tracked in `grid`'s
    majorant (an OracleGrid over the same kc and k_gas; the majorant scale is
    optics.majorant_scale) and delta-tracked sun rays: (sum, sumsq, stats)
    with stats[0:3] the sums over paths of the path's tentative collisions,
    nulls and leaves entered, stats[3:6] the sums of their squares."""
    f = make_field(desc, kc, k_gas)
    op = make_optics(optics)
    c = make_camera(cam)
    if pixels is None:
        pixels = np.arange(cam.width * cam.height, dtype=np.int32)
    pixels = np.ascontiguousarray(pixels, dtype=np.int32)
    s = np.zeros(len(pixels))
    s2 = np.zeros(len(pixels))
    cnt = np.zeros(3, np.uint64)
    st = np.zeros(6)
    lib().orc_render_tracked(C.byref(f), grid.handle, C.byref(op), C.byref(c), int(spp), int(seed), _ptr(pixels),
                             len(pixels), _ptr(s), _ptr(s2), _ptr(cnt), _ptr(st))
    return s, s2, st


def hg_dlng(g, mu):
    return lib().orc_hg_dlng(float(g), float(mu))


def flux(desc, kc, k_gas, optics, px, n_photons, seed, mode=0, kscale=1.0, grid=None, photon_offset=0):
    """Forward photons: (tally[7, py, px], glob[4]) as raw sums over arrivals.

    mode 0: exact free paths (transmissivity only); mode 2: delta tracking in
    `grid` (an OracleGrid over the same kc) with the scale and g scores."""
    f = make_field(desc, kc, k_gas, kscale)
    op = make_optics(optics)
    nx, ny = px
    tally = np.zeros((9, ny, nx))
    glob = np.zeros(4)
    lib().orc_flux(C.byref(f), grid.handle if grid is not None else None, C.byref(op), int(mode), nx, ny,
                   int(n_photons), int(seed), int(photon_offset), _ptr(tally), _ptr(glob))
    return tally, glob


def flux_fd(desc, kc, k_gas, optics, px, n_photons, seed, which, h=1e-3, kscale=1.0, photon_offset=0,
            with_total=False):
    """CRN central differences: out[2, py, px] = sum and sum of squares of the
    per-photon quotient; with_total also returns (sum, sumsq) of its sum over pixels."""
    f = make_field(desc, kc, k_gas, kscale)
    op = make_optics(optics)
    nx, ny = px
    out = np.zeros((2, ny, nx))
    tot = np.zeros(2)
    lib().orc_flux_fd(C.byref(f), C.byref(op), int(which), float(h), nx, ny, int(n_photons), int(seed),
                      int(photon_offset), _ptr(out), _ptr(tot))
    return (out, tot) if with_total else out


# ---------------------------------------------------------------------------
# Independent photon chunks in worker processes (the oracle itself stays
# serial; chunks use disjoint photon streams).
# ---------------------------------------------------------------------------

def _flux_chunk(args):
    kind, desc, kc, k_gas, optics, px, n, seed, off, extra = args
    if kind == "flux":
        mode, kscale, tau_tilde = extra
        grid = OracleGrid(desc, kc, tau_tilde=tau_tilde, k_gas=k_gas) if mode == 2 else None
        return flux(desc, kc, k_gas, optics, px, n, seed, mode=mode, kscale=kscale, grid=grid, photon_offset=off)
    which, h = extra
    return flux_fd(desc, kc, k_gas, optics, px, n, seed, which, h=h, photon_offset=off, with_total=True)


def _pool_map(jobs, workers):
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        return pool.map(_flux_chunk, jobs)


def parallel_flux(desc, kc, k_gas, optics, px, n_photons, seed, mode=0, kscale=1.0, tau_tilde=1.0, workers=8):
    step = -(-n_photons // workers)
    jobs = [("flux", desc, kc, k_gas, optics, px, min(step, n_photons - i * step), seed, i * step,
             (mode, kscale, tau_tilde)) for i in range(workers) if i * step < n_photons]
    res = _pool_map(jobs, workers)
    return sum(r[0] for r in res), sum(r[1] for r in res)


def parallel_flux_fd(desc, kc, k_gas, optics, px, n_photons, seed, which, h=1e-3, workers=8):
    step = -(-n_photons // workers)
    jobs = [("fd", desc, kc, k_gas, optics, px, min(step, n_photons - i * step), seed, i * step, (which, h))
            for i in range(workers) if i * step < n_photons]
    res = _pool_map(jobs, workers)
    return sum(r[0] for r in res), sum(r[1] for r in res)
