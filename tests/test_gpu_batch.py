"""Batched rendering: many views and suns of uneven image size in one
persistent launch must reproduce, image by image, the single-view renders
with the same random streams; the autotuner picks a launch shape that does
not change any result."""
import numpy as np
import pytest
import torch

from gpu_common import ctx, device_field
from paper_1902_01137_amd import api, inputs
from paper_1902_01137_amd.inputs import Camera, Optics, Sampling

pytestmark = pytest.mark.gpu


def _scene():
    sc = inputs.scene_small()
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    return sc, c, kd, g


def _jobs(sc):
    (xa, xb), (ya, yb), (za, zb) = sc.desc.box
    cx, cy = (xa + xb) / 2, (ya + yb) / 2
    jobs = []
    sizes = [(17, 9), (64, 64), (33, 40), (8, 8), (50, 23)]
    for i, (w, h) in enumerate(sizes):
        a = np.deg2rad(40.0 * i)
        cam = Camera(type=0, pos=(cx + 5 * np.cos(a), cy + 5 * np.sin(a), 3.0), target=(cx, cy, 2.6),
                     up=(0, 0, 1), fov_y_deg=35.0, width=w, height=h)
        op = Optics(**{**vars(sc.optics), "sun_zenith_deg": 15.0 + 12 * i, "sun_azimuth_deg": 30.0 * i,
                       "ground_albedo": 0.1 + 0.1 * i})
        jobs.append((cam, op))
    jobs.append((sc.camera, sc.optics))
    return jobs


def test_batch_equals_single_renders():
    sc, c, kd, g = _scene()
    jobs = _jobs(sc)
    smp = Sampling(seed=31, spp=12, stream=5)
    cnt = api.new_counters("cuda")
    s, s2, offs = api.render_batch(c, g, kd, jobs, smp, counters=cnt)
    torch.cuda.synchronize()
    total_px = sum(cam.width * cam.height for cam, _ in jobs)
    assert api.counters_dict(cnt)["paths"] == total_px * 12
    for j, (cam, op) in enumerate(jobs):
        one = Sampling(seed=31, spp=12, stream=5 + j)
        r, r2 = api.render(c, g, kd, op, cam, one)
        n = cam.width * cam.height
        torch.testing.assert_close(s[offs[j]:offs[j] + n], r.ravel(), rtol=1e-12, atol=1e-12)
        torch.testing.assert_close(s2[offs[j]:offs[j] + n], r2.ravel(), rtol=1e-12, atol=1e-12)


def test_batch_with_extended_medium_equals_single_renders():
    """A solar disc, a tabulated phase function and a k-distribution shared
    by all jobs (the extended-medium kernels): still image by image the
    single renders."""
    sc = inputs.scene_small()
    c = ctx()
    kd = device_field(sc.kc)
    kdist = (np.array([0.3, 0.5, 0.2]), np.array([0.0, 0.02, 0.05]))
    g = api.build_grid(c, kd, sc.desc, inputs.GridParams(sc.grid.tau_tilde, 0.05, sc.grid.criterion))
    tab = api.PhaseTable(c, *inputs.phase_table_tthg(n=61))
    ext = {"sun_half_angle_deg": 2.0, "phase_table": tab, "kdist": kdist}
    jobs = [(cam, Optics(**{**vars(op), **ext})) for cam, op in _jobs(sc)]
    smp = Sampling(seed=37, spp=6, stream=9)
    s, s2, offs = api.render_batch(c, g, kd, jobs, smp)
    torch.cuda.synchronize()
    for j, (cam, op) in enumerate(jobs):
        r, r2 = api.render(c, g, kd, op, cam, Sampling(seed=37, spp=6, stream=9 + j))
        n = cam.width * cam.height
        torch.testing.assert_close(s[offs[j]:offs[j] + n], r.ravel(), rtol=1e-12, atol=1e-12)
        torch.testing.assert_close(s2[offs[j]:offs[j] + n], r2.ravel(), rtol=1e-12, atol=1e-12)
    assert float(s.sum()) > 0.0


def test_batch_rejects_mixed_media():
    sc, c, kd, g = _scene()
    jobs = _jobs(sc)[:2]
    jobs[1] = (jobs[1][0], Optics(**{**vars(jobs[1][1]), "g": 0.5}))
    from paper_1902_01137_amd import _lib
    with pytest.raises(_lib.NcError) as e:
        api.render_batch(c, g, kd, jobs, Sampling(seed=1, spp=1))
    assert e.value.status == _lib.NC_ERR_INVALID_ARG


def test_autotune_keeps_results():
    sc, c, kd, g = _scene()
    smp = Sampling(seed=7, spp=8)
    c.set_launch()                       # library defaults
    ref, ref2 = api.render(c, g, kd, sc.optics, sc.camera, smp)
    launch, ms = api.autotune_render(c, g, kd, sc.optics, sc.camera, Sampling(seed=1, spp=4))
    assert ms > 0 and launch["samples_per_item"] in (1, 2, 4, 8, 16) and launch["block"] in (64, 128, 256)
    out, out2 = api.render(c, g, kd, sc.optics, sc.camera, smp)
    # every path is the same; only the grouping of samples into queue items
    # (whose partial sums are float32 before the float64 accumulation) changes
    torch.testing.assert_close(out, ref, rtol=1e-6, atol=1e-9)
    torch.testing.assert_close(out2, ref2, rtol=1e-6, atol=1e-9)
    c.set_launch()


def test_multiview_multisun_batch_cumulus():
    """The 48 views x 4 suns layout on a reduced cumulus field, image sides
    scaled by 1/8 (32..128 px): every job equals its single render."""
    sc = inputs.scene_cumulus(fine=(80, 256, 256), pool=2)
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    (xa, xb), (ya, yb), _ = sc.desc.box
    views = inputs.batch_views(centre=((xa + xb) / 2, (ya + yb) / 2), ring=5.0, base_side=32, side_step=16)
    jobs = [(cam, Optics(**{**vars(sc.optics), "sun_zenith_deg": sz})) for cam, sz in views]
    assert len(jobs) == 192
    smp = Sampling(seed=11, spp=2)
    s, s2, offs = api.render_batch(c, g, kd, jobs, smp)
    torch.cuda.synchronize()
    for j in (0, 5, 47, 48, 101, 191):
        cam, op = jobs[j]
        r, _ = api.render(c, g, kd, op, cam, Sampling(seed=11, spp=2, stream=j))
        n = cam.width * cam.height
        torch.testing.assert_close(s[offs[j]:offs[j] + n], r.ravel(), rtol=1e-12, atol=1e-12)


def test_guided_batch_equals_single_guided_renders():
    """One sun, several views of uneven size: the guided batch reproduces
    each job's single guided render bit for bit."""
    sc, c, kd, g = _scene()
    jobs = [(cam, Optics(**{**vars(op), "sun_zenith_deg": 30.0, "sun_azimuth_deg": 0.0})) for cam, op in _jobs(sc)]
    gd = api.Guide(c, seed=9)
    smp = Sampling(seed=41, spp=8, stream=3, guide_frac=0.5, guide_max_order=2)
    s, s2, offs = api.render_batch(c, g, kd, jobs, smp, guide=gd)
    torch.cuda.synchronize()
    for j, (cam, op) in enumerate(jobs):
        one = Sampling(seed=41, spp=8, stream=3 + j, guide_frac=0.5, guide_max_order=2)
        r, r2 = api.render_guided(c, g, kd, op, cam, one, gd)
        n = cam.width * cam.height
        torch.testing.assert_close(s[offs[j]:offs[j] + n], r.ravel(), rtol=1e-12, atol=1e-12)
        torch.testing.assert_close(s2[offs[j]:offs[j] + n], r2.ravel(), rtol=1e-12, atol=1e-12)


def test_guided_batch_with_a_guide_per_run_of_jobs():
    """Three networks over consecutive runs of jobs in one launch (each
    workgroup serves one run's queues, then moves to a run with work left):
    every job equals its single guided render with its own network."""
    sc, c, kd, g = _scene()
    jobs = _jobs(sc) * 2
    guides = [api.Guide(c, seed=s) for s in (9, 10, 11)]
    per_job = [guides[0]] * 3 + [guides[1]] * 5 + [guides[2]] * 4
    assert len(per_job) == len(jobs)
    smp = Sampling(seed=43, spp=6, stream=7, guide_frac=0.5, guide_max_order=0)
    s, s2, offs = api.render_batch(c, g, kd, jobs, smp, guide=per_job)
    torch.cuda.synchronize()
    for j, (cam, op) in enumerate(jobs):
        one = Sampling(seed=43, spp=6, stream=7 + j, guide_frac=0.5, guide_max_order=0)
        r, r2 = api.render_guided(c, g, kd, op, cam, one, per_job[j])
        n = cam.width * cam.height
        torch.testing.assert_close(s[offs[j]:offs[j] + n], r.ravel(), rtol=1e-12, atol=1e-12)
        torch.testing.assert_close(s2[offs[j]:offs[j] + n], r2.ravel(), rtol=1e-12, atol=1e-12)


def test_guided_batch_guide_runs_are_limited():
    from paper_1902_01137_amd import _lib
    sc, c, kd, g = _scene()
    jobs = _jobs(sc)[:2] * 5                       # 10 jobs
    a, b = api.Guide(c, seed=1), api.Guide(c, seed=2)
    with pytest.raises(_lib.NcError) as e:         # 10 alternating runs > NC_BATCH_MAX_GUIDES
        api.render_batch(c, g, kd, jobs, Sampling(seed=1, spp=1), guide=[a, b] * 5)
    assert e.value.status == _lib.NC_ERR_INVALID_ARG
    api.render_batch(c, g, kd, jobs, Sampling(seed=1, spp=1), guide=[a] * 5 + [b] * 5)
    torch.cuda.synchronize()


def test_autotune_batch_keeps_every_image():
    """nc_autotune_batch leaves a launch shape in the context; the batch
    rendered on it holds the same images (only the grouping of samples into
    float32 partial sums per queue item can change)."""
    sc, c, kd, g = _scene()
    jobs = _jobs(sc)
    smp = Sampling(seed=51, spp=8, stream=2)
    c.set_launch()
    ref, ref2, _ = api.render_batch(c, g, kd, jobs, smp)
    launch, ms = api.autotune_batch(c, g, kd, jobs, Sampling(seed=1, spp=2))
    assert ms > 0 and launch["samples_per_item"] in (1, 2, 4, 8, 16) and launch["block"] in (64, 128, 256)
    assert c.get_launch() == launch
    out, out2, _ = api.render_batch(c, g, kd, jobs, smp)
    torch.testing.assert_close(out, ref, rtol=1e-6, atol=1e-9)
    torch.testing.assert_close(out2, ref2, rtol=1e-6, atol=1e-9)
    c.set_launch()
