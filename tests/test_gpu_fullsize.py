"""Parity at the benchmark's full size: the 512x512x160 cumulus field (25 m)
seen by the 1024x1024 oblique camera at 64 samples per pixel, rendered by the
GPU exactly as the benchmark times it, against the oracle on a strided
subset of pixels; plus the grid of that field, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import ctx, device_field
from paper_1902_01137_amd import api, inputs
from paper_1902_01137_amd.inputs import Sampling
from stats import compare, mean_se

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cumulus():
    return inputs.scene_cumulus()


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


def test_cumulus_image_sampled_pixels(cumulus):
    sc = cumulus
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    spp = sc.sampling.spp
    cnt = api.new_counters("cuda")
    s, s2 = api.render(c, g, kd, sc.optics, sc.camera, Sampling(seed=sc.sampling.seed, spp=spp), counters=cnt)
    torch.cuda.synchronize()
    cd = api.counters_dict(cnt)
    assert cd["paths"] == 1024 * 1024 * spp and cd["truncated"] == 0
    W = sc.camera.width
    # every 16th pixel in both directions, offset to avoid the image border
    ys, xs = np.meshgrid(np.arange(8, 1024, 16), np.arange(8, 1024, 16), indexing="ij")
    pix = (ys * W + xs).ravel().astype(np.int32)
    gm, gse = mean_se(s.cpu().numpy().ravel()[pix], s2.cpu().numpy().ravel()[pix], spp)
    os_, os2, _ = oracle.render(sc.desc, sc.kc, sc.grid.k_gas, sc.optics, sc.camera, spp,
                                inputs.SEED_ORACLE_BASE + 2, pixels=pix)
    om, ose = mean_se(os_, os2, spp)
    # 4x4 blocks of the 64x64 sampled-pixel lattice
    gb = gm.reshape(16, 4, 16, 4).mean(axis=(1, 3)).ravel()
    gbs = np.sqrt((gse.reshape(16, 4, 16, 4) ** 2).sum(axis=(1, 3))).ravel() / 16
    ob = om.reshape(16, 4, 16, 4).mean(axis=(1, 3)).ravel()
    obs = np.sqrt((ose.reshape(16, 4, 16, 4) ** 2).sum(axis=(1, 3))).ravel() / 16
    res = compare(gb, gbs, ob, obs)
    assert res["ok"], res
    res_px = compare(gm, gse, om, ose)
    assert res_px["ok"], res_px
