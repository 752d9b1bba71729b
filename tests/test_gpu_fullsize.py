"""Parity at the benchmark's full size: the 512x512x160 cumulus field (25 m)
seen by the 1024x1024 oblique camera at 64 samples per pixel, rendered by the
GPU with the benchmark's launch shape and both sun-ray estimators (residual
ratio tracking, the one the benchmark times, and delta tracking), against the
oracle on a strided subset of pixels; the event counts per path of the
delta-tracked render against the oracle's delta-tracked walk on randomly
drawn pixels; and the grid of that field, bit for bit."""
import math

import numpy as np
import pytest
import torch

import oracle
from gpu_common import ctx, device_field
from paper_1902_01137_amd import _lib, api, inputs
from paper_1902_01137_amd.inputs import Sampling
from stats import compare, mean_se

pytestmark = pytest.mark.gpu

# every 16th pixel in both directions, offset to avoid the image border
_YS, _XS = np.meshgrid(np.arange(8, 1024, 16), np.arange(8, 1024, 16), indexing="ij")
_PIX = (_YS * 1024 + _XS).ravel().astype(np.int32)


@pytest.fixture(scope="module")
def cumulus():
    return inputs.scene_cumulus()


@pytest.fixture(scope="module")
def oracle_pixels(cumulus):
    sc = cumulus
    os_, os2, _ = oracle.render(sc.desc, sc.kc, sc.grid.k_gas, sc.optics, sc.camera, sc.sampling.spp,
                                inputs.SEED_ORACLE_BASE + 2, pixels=_PIX)
    return mean_se(os_, os2, sc.sampling.spp)


def test_cumulus_grid_bit_exact(cumulus):
    sc = cumulus
    c = ctx()
    g = api.build_grid(c, device_field(sc.kc), sc.desc, sc.grid)
    og = oracle.OracleGrid(sc.desc, sc.kc, tau_tilde=sc.grid.tau_tilde, k_gas=sc.grid.k_gas)
    assert g.L == og.L == 9
    for l in range(1, g.L + 1):
        kmin, kmax, mg = (t.cpu().numpy() for t in g.level(l))
        okmin, okmax, omg = og.level(l)
        assert np.array_equal(kmin, okmin) and np.array_equal(kmax, okmax) and np.array_equal(mg, omg), l
    assert np.array_equal(g.leaf_levels().cpu().numpy(), og.leaf_levels())


def _lattice_blocks(m, se):
    """4x4 blocks of the 64x64 sampled-pixel lattice."""
    mb = m.reshape(16, 4, 16, 4).mean(axis=(1, 3)).ravel()
    sb = np.sqrt((se.reshape(16, 4, 16, 4) ** 2).sum(axis=(1, 3))).ravel() / 16
    return mb, sb


@pytest.mark.parametrize("est", [_lib.NC_SUN_RESIDUAL, _lib.NC_SUN_DELTA], ids=["residual", "delta"])
def test_cumulus_image_sampled_pixels(cumulus, oracle_pixels, est):
    sc = cumulus
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    spp = sc.sampling.spp
    cnt = api.new_counters("cuda")
    s, s2 = api.render(c, g, kd, sc.optics, sc.camera, Sampling(seed=sc.sampling.seed + est, spp=spp, flags=est),
                       counters=cnt)
    torch.cuda.synchronize()
    cd = api.counters_dict(cnt)
    assert cd["paths"] == 1024 * 1024 * spp and cd["truncated"] == 0
    gm, gse = mean_se(s.cpu().numpy().ravel()[_PIX], s2.cpu().numpy().ravel()[_PIX], spp)
    om, ose = oracle_pixels
    res = compare(*_lattice_blocks(gm, gse), *_lattice_blocks(om, ose))
    assert res["ok"], res
    res_px = compare(gm, gse, om, ose)
    assert res_px["ok"], res_px


def test_cumulus_counts_per_path_vs_oracle(cumulus):
    """Tentative collisions, nulls and voxels entered per path over the whole
    image (delta-tracked sun rays): the GPU's counters over all 67 M paths
    against the oracle's delta-tracked walk on 4096 pixels drawn uniformly
    (8 paths each), whose per-path spread gives the standard error."""
    sc = cumulus
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    spp = sc.sampling.spp
    cnt = api.new_counters("cuda")
    api.render(c, g, kd, sc.optics, sc.camera, Sampling(seed=sc.sampling.seed + 11, spp=spp, flags=_lib.NC_SUN_DELTA),
               counters=cnt)
    torch.cuda.synchronize()
    gc = api.counters_dict(cnt)
    n_g = 1024 * 1024 * spp
    og = oracle.OracleGrid(sc.desc, sc.kc, tau_tilde=sc.grid.tau_tilde, k_gas=sc.grid.k_gas)
    pix = np.random.default_rng(12).choice(1024 * 1024, 4096, replace=False).astype(np.int32)
    spp_o = 8
    _, _, st = oracle.render_tracked(sc.desc, sc.kc, sc.grid.k_gas, sc.optics, sc.camera, spp_o,
                                     inputs.SEED_ORACLE_BASE + 12, og, pixels=pix)
    n_o = len(pix) * spp_o
    for i, name in enumerate(("tentative", "nulls", "leaf_visits")):
        om = st[i] / n_o
        var = max(st[3 + i] / n_o - om * om, 0.0) * n_o / (n_o - 1)
        se = math.sqrt(var / n_g + var / n_o)
        z = (gc[name] / n_g - om) / se
        assert abs(z) < 3.0, (name, gc[name] / n_g, om, se)
