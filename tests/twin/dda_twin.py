"""Host build of the GPU path's ordered crossing (test tooling, not the oracle).

build() compiles dda_twin.hip for the host only (hipcc, no FP contraction, as
the library); trace() walks rays through a grid given by its exported levels
exactly as the GPU kernels do."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(os.path.dirname(_HERE))
_SRC = os.path.join(_HERE, "dda_twin.hip")
_LIB = os.path.join(_HERE, "libdda_twin.so")
_HDR = os.path.join(_ROOT, "paper_1902_01137_amd", "csrc", "nc_device.hpp")
_lib = None


def build(force: bool = True) -> str:
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in (_SRC, _HDR))
    if force or stale:
        tmp = _LIB + ".tmp"
        subprocess.check_call(["hipcc", "--offload-arch=gfx950", "--offload-host-only", "-O2", "-std=c++17", "-fPIC",
                               "-shared", "-ffp-contract=off", "-I" + os.path.join(_ROOT, "include"),
                               "-I" + os.path.dirname(_HDR), _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.twin_trace.argtypes = [C.c_int, C.c_int, C.c_int] + [C.c_double] * 6 + [C.c_int, P, P, P, P, P, C.c_int,
                                                                                   C.c_int, P, P, P]
        L.twin_trace.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def trace(desc, kc, levels, rays, maxv):
    """levels: list over l = 1..L of (kmin, kmax, merged) arrays [z][y][x] as
    exported by the library.  Returns (leaf[n, maxv, 4], t[n, maxv, 2], count[n])."""
    L = len(levels)
    kmin = np.ascontiguousarray(np.concatenate([lv[0].ravel() for lv in levels]) if L else np.zeros(0), np.float32)
    kmax = np.ascontiguousarray(np.concatenate([lv[1].ravel() for lv in levels]) if L else np.zeros(0), np.float32)
    mg = np.ascontiguousarray(np.concatenate([lv[2].ravel() for lv in levels]) if L else np.zeros(0), np.uint8)
    kc = np.ascontiguousarray(kc, np.float32)
    rays = np.ascontiguousarray(rays, np.float32)
    n = rays.shape[0]
    leaf = np.zeros((n, maxv, 4), np.int32)
    t = np.zeros((n, maxv, 2), np.float32)
    cnt = np.zeros(n, np.int32)
    rc = lib().twin_trace(desc.nx, desc.ny, desc.nz, desc.x0, desc.y0, desc.z0, desc.dx, desc.dy, desc.dz, L,
                          _p(kmin), _p(kmax), _p(mg), _p(kc), _p(rays), n, maxv, _p(leaf), _p(t), _p(cnt))
    if rc != 0:
        raise ValueError("twin_trace: bad arguments")
    return leaf, t, cnt
