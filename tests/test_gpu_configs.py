"""Oracle parity of the refinement family's finest field and of the
many-view batch.

* 1024 x 1024 x 320 (12.5 m) cumulus field, the finest point of the
  coarse-graining sweep (Section 4.2, Fig. 5) and the only field larger than
  the last-level cache: its grid bit for bit against the oracle's, and its
  512 x 512 view at 32 samples per pixel (residual ratio tracking, as timed)
  on every 16th pixel against the oracle's image.
* The 48 views x 4 suns batch over the 512 x 512 x 160 field (Section 4.3's
  BOMEX-shaped domain): six jobs of one persistent launch, chosen across
  view sizes and suns, each against the oracle on a 32 x 32 pixel lattice;
  and the guided batch (a trained network per sun, every order guided) in
  one launch.

The acceptance rule takes z on blocks of pixels (4 x 4 lattice pixels, 512
paths a side), where it is near-Gaussian; at 32 paths a pixel a side that
missed a rare bright path has a low mean and a low standard error at once,
so single-pixel z is reported, not tested.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import ctx, device_field
from paper_1902_01137_amd import _lib, api, inputs
from paper_1902_01137_amd.inputs import Optics, Sampling
from stats import compare, mean_se

pytestmark = pytest.mark.gpu


def _lattice(W, H, n=32):
    """n x n pixels spread over a W x H image (centres of an n x n partition)."""
    xs = (np.arange(n) * W // n + W // (2 * n)).astype(np.int64)
    ys = (np.arange(n) * H // n + H // (2 * n)).astype(np.int64)
    yy, xx = np.meshgrid(ys, xs, indexing="ij")
    return (yy * W + xx).ravel().astype(np.int32)


def _blocks(m, se, n=32, b=4):
    mb = m.reshape(n // b, b, n // b, b).mean(axis=(1, 3)).ravel()
    sb = np.sqrt((se.reshape(n // b, b, n // b, b) ** 2).sum(axis=(1, 3))).ravel() / (b * b)
    return mb, sb


@pytest.fixture(scope="module")
def fine_field():
    return inputs.cumulus_field(pool=1)


def test_refinement_finest_grid_bit_exact(fine_field):
    desc, k = fine_field
    assert (desc.nx, desc.ny, desc.nz) == (1024, 1024, 320)
    c = ctx()
    kd = device_field(k)
    gp = inputs.GridParams(1.0, 0.05, 0)
    g = api.build_grid(c, kd, desc, gp)
    og = oracle.OracleGrid(desc, k, tau_tilde=gp.tau_tilde, k_gas=gp.k_gas)
    assert g.L == og.L == 10
    for l in range(1, g.L + 1):
        kmin, kmax, mg = (t.cpu().numpy() for t in g.level(l))
        okmin, okmax, omg = og.level(l)
        assert np.array_equal(kmin, okmin) and np.array_equal(kmax, okmax) and np.array_equal(mg, omg), l
    assert np.array_equal(g.leaf_levels().cpu().numpy(), og.leaf_levels())


def test_refinement_finest_view_vs_oracle(fine_field):
    sc = inputs.scene_cumulus(field=fine_field, width=512, height=512, spp=32)
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    spp = 32
    cnt = api.new_counters("cuda")
    s, s2 = api.render(c, g, kd, sc.optics, sc.camera,
                       Sampling(seed=inputs.SEED_GPU_BASE + 3, spp=spp, flags=_lib.NC_SUN_RESIDUAL), counters=cnt)
    torch.cuda.synchronize()
    assert api.counters_dict(cnt)["truncated"] == 0
    pix = _lattice(512, 512)
    gm, gse = mean_se(s.cpu().numpy().ravel()[pix], s2.cpu().numpy().ravel()[pix], spp)
    os_, os2, _ = oracle.render(sc.desc, sc.kc, sc.grid.k_gas, sc.optics, sc.camera, spp,
                                inputs.SEED_ORACLE_BASE + 3, pixels=pix)
    om, ose = mean_se(os_, os2, spp)
    res = compare(*_blocks(gm, gse), *_blocks(om, ose))
    assert res["ok"], str(res)
    print("finest view: per-pixel z (reported): %s" % compare(gm, gse, om, ose))


@pytest.fixture(scope="module")
def cumulus():
    return inputs.scene_cumulus()


# (view index on the ring, sun zenith): the smallest and largest views, every sun
_PICKED = ((0, 15.0), (6, 15.0), (13, 30.0), (20, 45.0), (34, 45.0), (47, 60.0))


def _batch_jobs(sc):
    views = inputs.batch_views()
    return [(cam, Optics(**{**vars(sc.optics), "sun_zenith_deg": sz})) for cam, sz in views], views


def _job_index(views, view, sun):
    per_sun = len(views) // 4
    suns = sorted({z for _, z in views})
    return suns.index(sun) * per_sun + view


def test_batch_jobs_vs_oracle(cumulus):
    sc = cumulus
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    jobs, views = _batch_jobs(sc)
    assert len(jobs) == 192
    spp = 32
    cnt = api.new_counters("cuda")
    s, s2, offs = api.render_batch(c, g, kd, jobs, Sampling(seed=inputs.SEED_GPU_BASE + 5, spp=spp,
                                                           flags=_lib.NC_SUN_RESIDUAL), counters=cnt)
    torch.cuda.synchronize()
    cd = api.counters_dict(cnt)
    assert cd["paths"] == sum(cam.width * cam.height for cam, _ in jobs) * spp and cd["truncated"] == 0
    S, S2 = s.cpu().numpy(), s2.cpu().numpy()
    sides = set()
    for view, sun in _PICKED:
        j = _job_index(views, view, sun)
        cam, op = jobs[j]
        assert views[j][1] == sun
        sides.add(cam.width)
        pix = _lattice(cam.width, cam.height)
        gm, gse = mean_se(S[offs[j] + pix], S2[offs[j] + pix], spp)
        os_, os2, _ = oracle.render(sc.desc, sc.kc, sc.grid.k_gas, op, cam, spp, inputs.SEED_ORACLE_BASE + 5 + j,
                                    pixels=pix)
        om, ose = mean_se(os_, os2, spp)
        res = compare(*_blocks(gm, gse), *_blocks(om, ose))
        assert res["ok"], str((j, res))
        print("job %d: per-pixel z (reported): %s" % (j, compare(gm, gse, om, ose)))
    assert min(sides) == 256 and max(sides) == 1024


def _train_guide(c, g, kd, sc, jobs, steps=3000):
    recs = []
    for cam, op in jobs:
        r, _, _, _ = api.collect_vertices(c, g, kd, op, cam, Sampling(seed=inputs.SEED_GPU_BASE + 7, spp=4,
                                                                      flags=_lib.NC_SUN_RESIDUAL),
                                          cam.width * cam.height * 4 * 16)
        recs.append(r)
    rec = torch.cat(recs)
    gd = api.Guide(c, seed=1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    for it in range(steps):
        idx = torch.randint(0, rec.shape[0], (16384,), device="cuda", generator=gen)
        gd.train_step(rec[idx], 3e-3 * (0.2 if it >= 0.8 * steps else 1.0))
    torch.cuda.synchronize()
    return gd


def test_guided_batch_jobs_vs_oracle(cumulus):
    """The whole 48 views x 4 suns batch guided in one launch, one network
    per sun (trained on vertices of 8 of its views, every scattering order
    guided, c = 0.5): four jobs, one per sun, against the oracle's plain
    estimate."""
    sc = cumulus
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    jobs, views = _batch_jobs(sc)
    suns = sorted({z for _, z in views})
    guides = {sz: _train_guide(c, g, kd, sc, [jobs[_job_index(views, v, sz)] for v in range(0, 48, 6)])
              for sz in suns}
    per_job = [guides[z] for _, z in views]
    spp = 32
    smp = Sampling(seed=inputs.SEED_GPU_BASE + 8, spp=spp, flags=_lib.NC_SUN_RESIDUAL, guide_frac=0.5,
                   guide_max_order=0)
    s, s2, offs = api.render_batch(c, g, kd, jobs, smp, guide=per_job)
    torch.cuda.synchronize()
    S, S2 = s.cpu().numpy(), s2.cpu().numpy()
    for v in (_job_index(views, 3, 15.0), _job_index(views, 20, 30.0), _job_index(views, 34, 45.0),
              _job_index(views, 41, 60.0)):
        cam, op = jobs[v]
        pix = _lattice(cam.width, cam.height)
        gm, gse = mean_se(S[offs[v] + pix], S2[offs[v] + pix], spp)
        os_, os2, _ = oracle.render(sc.desc, sc.kc, sc.grid.k_gas, op, cam, spp, inputs.SEED_ORACLE_BASE + 40 + v,
                                    pixels=pix)
        om, ose = mean_se(os_, os2, spp)
        res = compare(*_blocks(gm, gse), *_blocks(om, ose))
        assert res["ok"], str((v, res))
        print("view %d: per-pixel z (reported): %s" % (v, compare(gm, gse, om, ose)))
