"""ctypes mirror of include/nctrace.h and the loader of libnctrace.so.

The library is loaded from this package directory; there is no fallback:
if it is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnctrace.so")

NC_OK = 0
NC_ERR_INVALID_ARG = 1
NC_ERR_RANGE = 2
NC_ERR_OOM = 3
NC_ERR_DEVICE = 4
NC_ERR_UNSUPPORTED = 5
NC_ERR_STATE = 6
NC_MAX_LEVELS = 24

STATUS_NAMES = {0: "NC_OK", 1: "NC_ERR_INVALID_ARG", 2: "NC_ERR_RANGE", 3: "NC_ERR_OOM", 4: "NC_ERR_DEVICE",
                5: "NC_ERR_UNSUPPORTED", 6: "NC_ERR_STATE"}


class FieldDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("pad_", C.c_int32),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double)]


class GridParams(C.Structure):
    _fields_ = [("tau_tilde", C.c_double), ("k_gas", C.c_double), ("criterion", C.c_int32), ("flat_level", C.c_int32)]


KDIST_MAX = 16


class KDist(C.Structure):
    _fields_ = [("n", C.c_int32), ("pad_", C.c_int32), ("w", C.c_double * KDIST_MAX),
                ("k_gas", C.c_double * KDIST_MAX)]


class Optics(C.Structure):
    _fields_ = [("ssa", C.c_double), ("g", C.c_double), ("ground_albedo", C.c_double),
                ("sun_zenith_deg", C.c_double), ("sun_azimuth_deg", C.c_double), ("sun_irradiance", C.c_double),
                ("majorant_scale", C.c_double), ("max_scatter", C.c_int32), ("max_segments", C.c_int32),
                ("sun_half_angle_deg", C.c_double), ("phase", C.c_void_p), ("kdist", C.c_void_p)]


class Camera(C.Structure):
    _fields_ = [("type", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("pad_", C.c_int32),
                ("pos", C.c_double * 3), ("target", C.c_double * 3), ("up", C.c_double * 3),
                ("fov_y_deg", C.c_double), ("ortho_w", C.c_double), ("ortho_h", C.c_double)]


class Sampling(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("sample_offset", C.c_uint64), ("spp", C.c_int32), ("flags", C.c_int32),
                ("guide_frac", C.c_double), ("stream", C.c_uint32), ("guide_max_order", C.c_uint32)]


class Launch(C.Structure):
    _fields_ = [("block", C.c_int32), ("waves_per_cu", C.c_int32), ("samples_per_item", C.c_int32),
                ("lds_levels", C.c_int32)]


# scheduler slots per phase: "step" = voxel crossings and ray starts (one
# phase); slot 3 is unused (kept so that the layout of nc_counters holds)
PHASES = ("step", "collide", "event", "unused", "sample", "guide")
COUNTER_NAMES = ["paths", "segments", "tentative", "nulls", "reals", "leaf_visits", "gathers", "node_reads",
                 "nee_rays", "truncated"] + ["%s_%s" % (a, b) for a in ("trips", "lanes", "ticks")
                                              for b in PHASES] + ["deep_visits"] + ["sched_pad%d" % i for i in range(5)]
N_COUNTER_WORDS = 34
NC_SUN_DELTA, NC_SUN_RATIO, NC_SUN_RESIDUAL = 0, 1, 2
NC_FLUX_NORMALISE = 4
GUIDE_PARAMS = 11944
NOALLOC_MAX_JOBS = 1024
GUIDE_RECORD = 12

class Progressive(C.Structure):
    _fields_ = [("target_rel_err", C.c_double), ("first_spp", C.c_int32), ("max_spp", C.c_int32),
                ("block", C.c_int32), ("pad_", C.c_int32)]


class ProgressReport(C.Structure):
    _fields_ = [("spp_done", C.c_int32), ("rounds", C.c_int32), ("rel_err", C.c_double), ("mean", C.c_double),
                ("seconds", C.c_double)]


# (name, restype, argtypes)
_P = C.c_void_p
_SIGS = [
    ("nc_abi_version", C.c_uint32, []),
    ("nc_phase_create", C.c_int32, [_P, _P, _P, C.c_int32, C.POINTER(_P)]),
    ("nc_phase_destroy", None, [_P]),
    ("nc_phase_sample", C.c_int32, [_P, _P, _P, C.c_int32, _P]),
    ("nc_ctx_create", C.c_int32, [C.c_int32, _P, C.POINTER(_P)]),
    ("nc_ctx_set_stream", C.c_int32, [_P, _P]),
    ("nc_ctx_destroy", None, [_P]),
    ("nc_last_error", C.c_char_p, [_P]),
    ("nc_grid_build", C.c_int32, [_P, _P, C.POINTER(FieldDesc), C.POINTER(GridParams), C.POINTER(_P)]),
    ("nc_grid_destroy", None, [_P]),
    ("nc_grid_info", C.c_int32, [_P, C.POINTER(C.c_int32), C.c_int32, _P]),
    ("nc_grid_export", C.c_int32, [_P, _P, C.c_int32, _P, _P, _P]),
    ("nc_grid_leaf_levels", C.c_int32, [_P, _P, _P]),
    ("nc_grid_rebuild", C.c_int32, [_P, _P, _P]),
    ("nc_grid_export_mask", C.c_int32, [_P, _P, _P]),
    ("nc_trace_leaves", C.c_int32, [_P, _P, _P, C.c_int32, C.c_int32, _P, _P, _P]),
    ("nc_transmittance", C.c_int32, [_P, _P, _P, C.POINTER(Optics), _P, C.c_int32, C.POINTER(Sampling), _P, _P, _P]),
    ("nc_render", C.c_int32, [_P, _P, _P, C.POINTER(Optics), C.POINTER(Camera), C.POINTER(Sampling), _P, _P, _P]),
    ("nc_set_launch", C.c_int32, [_P, C.POINTER(Launch)]),
    ("nc_get_launch", C.c_int32, [_P, C.POINTER(Launch)]),
    ("nc_render_guided", C.c_int32, [_P, _P, _P, C.POINTER(Optics), C.POINTER(Camera), C.POINTER(Sampling), _P, _P,
                                     _P, _P]),
    ("nc_render_progressive", C.c_int32, [_P, _P, _P, C.POINTER(Optics), C.POINTER(Camera), C.POINTER(Sampling), _P,
                                          C.POINTER(Progressive), _P, _P, _P, C.POINTER(ProgressReport)]),
    ("nc_guide_sample", C.c_int32, [_P, _P, _P, _P, C.c_int32, C.c_float, C.c_float, _P]),
    ("nc_gather_rate", C.c_int32, [_P, _P, C.c_uint64, C.c_int32, C.c_int32, _P, C.POINTER(C.c_double)]),
    ("nc_collect_vertices", C.c_int32, [_P, _P, _P, C.POINTER(Optics), C.POINTER(Camera), C.POINTER(Sampling), _P,
                                        C.c_uint64, _P, _P, _P, _P, _P]),
    ("nc_render_batch_guided", C.c_int32, [_P, _P, _P, C.c_int32, _P, _P, _P, C.POINTER(Sampling), _P, _P, _P, _P]),
    ("nc_render_batch", C.c_int32, [_P, _P, _P, C.c_int32, _P, _P, _P, C.POINTER(Sampling), _P, _P, _P]),
    ("nc_render_batch_noalloc", C.c_int32, [_P, _P, _P, C.c_int32, _P, _P, _P, C.POINTER(Sampling), _P, _P, _P]),
    ("nc_autotune_render", C.c_int32, [_P, _P, _P, C.POINTER(Optics), C.POINTER(Camera), C.POINTER(Sampling), _P, _P,
                                       C.POINTER(C.c_double)]),
    ("nc_autotune_batch", C.c_int32, [_P, _P, _P, C.c_int32, _P, _P, _P, C.POINTER(Sampling), _P, _P,
                                      C.POINTER(C.c_double)]),
    ("nc_philox4x32_10", C.c_int32, [_P, _P, _P, _P, C.c_int32]),
    ("nc_guide_create", C.c_int32, [_P, C.c_uint64, C.POINTER(_P)]),
    ("nc_guide_destroy", None, [_P]),
    ("nc_guide_get_params", C.c_int32, [_P, _P, _P]),
    ("nc_guide_set_params", C.c_int32, [_P, _P, _P]),
    ("nc_guide_forward", C.c_int32, [_P, _P, _P, C.c_int32, C.c_int32, _P]),
    ("nc_guide_train_step", C.c_int32, [_P, _P, _P, C.c_int32, C.c_float, _P]),
    ("nc_guide_gradient", C.c_int32, [_P, _P, _P, C.c_int32, _P, _P]),
    ("nc_flux", C.c_int32, [_P, _P, _P, C.POINTER(Optics), C.c_double, C.c_int32, C.c_int32, C.c_uint64,
                            C.POINTER(Sampling), _P, _P, _P]),
    ("nc_flux_adjoint", C.c_int32, [_P, _P, _P, C.POINTER(Optics), C.c_double, C.c_int32, C.c_int32, C.c_uint64,
                                    C.POINTER(Sampling), _P, _P]),
]

EXPORTED = [s[0] for s in _SIGS]

_lib = None


def load():
    """Load libnctrace.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libnctrace.so is not built (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class NcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), msg))
        self.status = status
