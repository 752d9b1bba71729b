"""The guided estimator in the configuration the benchmark reports: a network
trained on the plain tracer's vertices (Adam with the benchmark's cosine
step-size decay, fewer steps), every scattering order guided, guide fraction
c = 0.5, residual ratio tracking of the sun rays.

Each guided event multiplies the path weight by p / (c q + (1 - c) p), a
factor in [0, 1 / (1 - c)] with mean 1; along a path of many events the
product is unbiased but skewed, so two things are checked:

* unbiasedness: the guided image (16 independent renders combined) against
  the oracle's plain image on 8x8-pixel blocks, where z is near-Gaussian (a
  single pixel's 64 paths per render do not make the skewed weight product
  Gaussian, so its z is reported, not tested);
* honest error bars: the spread of the 16 renders' block means against the
  standard errors each render reports (chi-square with 15 degrees of freedom
  per block, summed over blocks), and the spread of the renders' pixel means
  against the pixels' reported variances summed over the image (the quantity
  behind the image's relative standard error: a time to a target error
  computed from one render's standard errors must not be an underestimate).

Scenes: the small blob (nadir view) and a cumulus field at 50 m seen
obliquely (many scattering orders inside thick cloud).
"""
import math

import numpy as np
import pytest
import torch
from scipy import stats as sst

import oracle
from gpu_common import ctx, device_field
from paper_1902_01137_amd import _lib, api, inputs
from paper_1902_01137_amd.inputs import Sampling
from stats import block, compare, mean_se

pytestmark = pytest.mark.gpu

K = 16          # independent guided renders
SPP = 64        # samples per pixel of each


def _scene(name):
    if name == "blob":
        return inputs.scene_small()
    desc, k = inputs.cumulus_field(fine=(80, 256, 256), pool=2)
    sc = inputs.scene_cumulus(field=(desc, k), width=64, height=64, spp=SPP)
    (xa, xb), (ya, yb), _ = desc.box
    sc.camera = inputs.Camera(type=0, pos=(xa - 1.5, (ya + yb) / 2, 1.5), target=((xa + xb) / 2, (ya + yb) / 2, 0.75),
                              up=(0.0, 0.0, 1.0), fov_y_deg=50.0, width=64, height=64)
    return sc


@pytest.fixture(scope="module", params=["blob", "cumulus50m"])
def guided_runs(request):
    sc = _scene(request.param)
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    cam = sc.camera
    flags = _lib.NC_SUN_RESIDUAL
    rec, _, _, _ = api.collect_vertices(c, g, kd, sc.optics, cam, Sampling(seed=501, spp=64, flags=flags),
                                        cam.width * cam.height * 64 * 24)
    gd = api.Guide(c, seed=1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    steps = 4000
    for it in range(steps):
        idx = torch.randint(0, rec.shape[0], (65536,), device="cuda", generator=gen)
        gd.train_step(rec[idx], 3e-3 * max(0.01, 0.5 * (1.0 + math.cos(math.pi * it / steps))))
    del rec
    runs = []
    for k in range(K):
        smp = Sampling(seed=600 + k, spp=SPP, flags=flags, guide_frac=0.5, guide_max_order=0)
        s, s2 = api.render_guided(c, g, kd, sc.optics, cam, smp, gd)
        torch.cuda.synchronize()
        runs.append(mean_se(s.cpu().numpy().ravel(), s2.cpu().numpy().ravel(), SPP))
    ps, ps2 = api.render(c, g, kd, sc.optics, cam, Sampling(seed=700, spp=K * SPP, flags=flags))
    torch.cuda.synchronize()
    plain = mean_se(ps.cpu().numpy().ravel(), ps2.cpu().numpy().ravel(), K * SPP)
    return request.param, sc, runs, plain


def test_guided_bench_config_unbiased(guided_runs):
    name, sc, runs, plain = guided_runs
    cam = sc.camera
    gm = np.mean([m for m, _ in runs], axis=0)
    gse = np.sqrt(np.sum([e ** 2 for _, e in runs], axis=0)) / K
    spp_o = 128 if name == "blob" else 64
    os_, os2, _ = oracle.render(sc.desc, sc.kc, sc.grid.k_gas, sc.optics, cam, spp_o, inputs.SEED_ORACLE_BASE + 51)
    om, ose = mean_se(os_, os2, spp_o)
    shape = (cam.height, cam.width)
    res = compare(*block(gm, gse, shape), *block(om, ose, shape))
    assert res["ok"], (name, res)
    print("%s: per-pixel z (not tested): %s" % (name, compare(gm, gse, om, ose)))
    print("%s: plain per-pixel z at the same spp: %s" % (name, compare(plain[0], plain[1], om, ose)))
    # what the guide gains (reported; a guide trained this briefly can cost
    # variance in thick cloud, where its weights multiply over many events)
    ratio = float((gse ** 2).sum() / (plain[1] ** 2).sum())
    print("%s: variance ratio guided/plain %.3f" % (name, ratio))


def test_guided_bench_config_error_bars(guided_runs):
    """Block means of K independent renders: their sample variance against
    the mean of the standard errors the renders report.  Per block,
    (K - 1) var / se^2 ~ chi2(K - 1) if the reported errors are right; the
    sum over blocks must lie inside the central 99.9 % of chi2(B (K - 1)) and
    the blocks beyond the 99.73 % point must be as rare as Binomial allows."""
    name, sc, runs, _ = guided_runs
    shape = (sc.camera.height, sc.camera.width)
    bm, be = zip(*[block(m, e, shape) for m, e in runs])
    bm, be = np.array(bm), np.array(be)                 # (K, blocks)
    lit = (be > 0).all(axis=0)
    var = bm[:, lit].var(axis=0, ddof=1)
    se2 = (be[:, lit] ** 2).mean(axis=0)
    T = (K - 1) * var / se2
    dof = (K - 1) * int(lit.sum())
    lo, hi = sst.chi2.ppf([0.0005, 0.9995], dof)
    ratio = T.sum() / dof
    print("%s: spread / reported variance %.3f (%d blocks)" % (name, ratio, lit.sum()))
    assert lo <= T.sum() <= hi, (name, ratio, lo / dof, hi / dof)
    q = sst.chi2.ppf(0.9973, K - 1)
    k = int((T > q).sum())
    p = 1.0 - sst.binom.cdf(k - 1, len(T), 0.0027)
    assert p >= 1e-3, (name, k, len(T))


def test_guided_bench_config_pixel_error_bars(guided_runs):
    """Over the image, the sum of the pixels' variances across the K renders
    against the sum of the variances the renders report (the square of the
    image's relative standard error, up to the mean): their ratio must be 1
    within a bootstrap interval over 8x8-pixel blocks (99.9 %)."""
    name, sc, runs, _ = guided_runs
    H, W = sc.camera.height, sc.camera.width
    M = np.array([m for m, _ in runs])
    E2 = np.array([e ** 2 for _, e in runs])
    spread = M.var(axis=0, ddof=1).reshape(H // 8, 8, W // 8, 8).sum(axis=(1, 3)).ravel()
    reported = E2.mean(axis=0).reshape(H // 8, 8, W // 8, 8).sum(axis=(1, 3)).ravel()
    ratio = spread.sum() / reported.sum()
    rng = np.random.default_rng(7)
    idx = rng.integers(0, len(spread), (4000, len(spread)))
    boot = spread[idx].sum(axis=1) / reported[idx].sum(axis=1)
    lo, hi = np.quantile(boot, [0.0005, 0.9995])
    print("%s: pixel spread / reported variance %.3f (bootstrap %.3f .. %.3f)" % (name, ratio, lo, hi))
    assert lo <= 1.0 <= hi, (name, ratio, lo, hi)
