"""nc_render_batch_noalloc (no device allocation: fixed library scratch)
against nc_render_batch, called through the C ABI: two calls in a row, the
second with fewer and smaller jobs, each image equal to the allocating
entry point's (the same paths; float64 sums up to atomic order); a job count
above the maximum is refused before any work."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_common import ctx, device_field
from paper_1902_01137_amd import _lib, api, inputs
from paper_1902_01137_amd.inputs import Camera, Optics, Sampling

pytestmark = pytest.mark.gpu


def _jobs(sc, sizes):
    (xa, xb), (ya, yb), _ = sc.desc.box
    cx, cy = (xa + xb) / 2, (ya + yb) / 2
    out = []
    for i, (w, h) in enumerate(sizes):
        a = np.deg2rad(50.0 * i)
        cam = Camera(type=0, pos=(cx + 5 * np.cos(a), cy + 5 * np.sin(a), 3.0), target=(cx, cy, 2.6), up=(0, 0, 1),
                     fov_y_deg=35.0, width=w, height=h)
        op = Optics(**{**vars(sc.optics), "sun_zenith_deg": 20.0 + 10 * i, "ground_albedo": 0.1 + 0.05 * i})
        out.append((cam, op))
    return out


def _call(name, c, g, kd, jobs, smp):
    """The entry point `name` through ctypes; returns (sum, sumsq, offsets, status)."""
    n = len(jobs)
    cams = (_lib.Camera * n)(*[api._camera(cam) for cam, _ in jobs])
    recs = [api._optics(op, c) for _, op in jobs]
    opts = (_lib.Optics * n)(*recs)
    offs, total = [], 0
    for cam, _ in jobs:
        offs.append(total)
        total += cam.width * cam.height
    off_arr = (C.c_uint64 * n)(*offs)
    s = torch.zeros(max(total, 1), dtype=torch.float64, device="cuda")
    s2 = torch.zeros_like(s)
    sm = api._sampling(smp)
    st = getattr(_lib.load(), name)(c.handle, g.handle, C.c_void_p(kd.data_ptr()), n, C.cast(cams, C.c_void_p),
                                    C.cast(opts, C.c_void_p), C.cast(off_arr, C.c_void_p), C.byref(sm),
                                    C.c_void_p(s.data_ptr()), C.c_void_p(s2.data_ptr()), None)
    return s, s2, offs, st


def test_noalloc_batch_matches_allocating_batch():
    sc = inputs.scene_small()
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    for sizes, smp in (([(48, 40), (17, 9), (64, 64), (33, 21), (8, 8), (50, 23)], Sampling(seed=71, spp=8, stream=3)),
                       ([(9, 5), (20, 12)], Sampling(seed=72, spp=4, stream=11))):
        jobs = _jobs(sc, sizes)
        a, a2, _, st_a = _call("nc_render_batch_noalloc", c, g, kd, jobs, smp)
        b, b2, _, st_b = _call("nc_render_batch", c, g, kd, jobs, smp)
        torch.cuda.synchronize()
        assert st_a == _lib.NC_OK and st_b == _lib.NC_OK
        assert float(a.sum()) > 0.0
        torch.testing.assert_close(a, b, rtol=1e-12, atol=1e-15)
        torch.testing.assert_close(a2, b2, rtol=1e-12, atol=1e-15)


def test_noalloc_batch_refuses_too_many_jobs():
    sc = inputs.scene_small()
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    jobs = _jobs(sc, [(2, 2)]) * (_lib.NOALLOC_MAX_JOBS + 1)
    s, _, _, st = _call("nc_render_batch_noalloc", c, g, kd, jobs, Sampling(seed=1, spp=1))
    torch.cuda.synchronize()
    assert st == _lib.NC_ERR_INVALID_ARG
    assert "NC_NOALLOC_MAX_JOBS" in _lib.load().nc_last_error(c.handle).decode()
    assert float(s.abs().sum()) == 0.0
