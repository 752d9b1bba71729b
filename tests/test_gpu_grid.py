"""Grid build on the GPU against the oracle: every level's kmin, kmax and
merged flag and the per-cell voxel level must match bit for bit."""
import math

import numpy as np
import pytest
import torch

import oracle
from gpu_common import ctx, device_field
from paper_1902_01137_amd import _lib, api, inputs
from paper_1902_01137_amd.inputs import FieldDesc, GridParams

pytestmark = pytest.mark.gpu


def _compare(desc, k, tau, kg=0.0, crit=0, flat=3):
    c = ctx()
    kd = device_field(k)
    g = api.build_grid(c, kd, desc, GridParams(tau, kg, crit, flat))
    og = oracle.OracleGrid(desc, k, tau_tilde=tau, k_gas=kg, criterion=crit, flat_level=flat)
    assert g.L == og.L
    for l in range(1, g.L + 1):
        assert g.level_dims(l) == og.level_dims(l)
        kmin, kmax, mg = (t.cpu().numpy() for t in g.level(l))
        okmin, okmax, omg = og.level(l)
        assert np.array_equal(kmin, okmin), l
        assert np.array_equal(kmax, okmax), l
        assert np.array_equal(mg, omg), l
    assert np.array_equal(g.leaf_levels().cpu().numpy(), og.leaf_levels())
    return g


@pytest.mark.parametrize("tau", [0.0, 0.5, 1.0, 10.0, math.inf])
@pytest.mark.parametrize("crit", [0, 1])
def test_blob(tau, crit):
    desc, k = inputs.lognormal_blob()
    _compare(desc, k, tau, 0.01, crit)


@pytest.mark.parametrize("shape", [(7, 3, 5), (5, 9, 12), (1, 1, 6), (33, 17, 65), (1, 1, 1)])
def test_ragged(shape):
    rng = np.random.default_rng(sum(shape))
    k = (rng.random(shape) ** 8 * 60).astype(np.float32)
    nz, ny, nx = shape
    desc = FieldDesc(nx, ny, nz, 0, 0, 0, 0.05, 0.05, 0.05)
    for tau in (0.0, 0.3, 3.0):
        _compare(desc, k, tau, 0.02)


@pytest.mark.parametrize("flat", [0, 1, 3, 9])
def test_flat_supercells(flat):
    desc, k = inputs.lognormal_blob()
    g = _compare(desc, k, 0.0, 0.01, 2, flat)
    assert (g.leaf_levels().cpu().numpy() == min(flat, g.L)).all()
    rng = np.random.default_rng(flat)
    k2 = (rng.random((5, 9, 12)) ** 8 * 60).astype(np.float32)
    _compare(FieldDesc(12, 9, 5, 0, 0, 0, 0.05, 0.05, 0.05), k2, 0.0, 0.02, 2, flat)


@pytest.mark.parametrize("flat", [0, 1, 3])
def test_layered_grid(flat):
    """Criterion 3 (clear layers split from the cloudy layer): bit for bit
    against the oracle on the cumulus field (clear air above and below its
    cloud layer), on ragged fields with a random layer, on a field without
    cloud (one voxel) and on the blob (cloud in every layer)."""
    desc, k = inputs.cumulus_field(fine=(80, 256, 256), pool=2)
    _compare(desc, k, 0.0, 0.05, 3, flat)
    rng = np.random.default_rng(40 + flat)
    for shape, layer in (((33, 17, 65), (9, 20)), ((64, 8, 8), (0, 5)), ((20, 6, 10), (19, 19))):
        nz, ny, nx = shape
        k2 = np.zeros(shape, np.float32)
        z0, z1 = layer
        blob = (rng.random((z1 - z0 + 1, ny, nx)) ** 6 * 40).astype(np.float32)
        blob[rng.random(blob.shape) < 0.6] = 0.0
        blob[0, 0, 0], blob[-1, -1, -1] = 1.0, 3.0
        k2[z0:z1 + 1] = blob
        _compare(FieldDesc(nx, ny, nz, 0, 0, 0, 0.05, 0.05, 0.05), k2, 1.0, 0.02, 3, flat)
    g = _compare(FieldDesc(12, 9, 5, 0, 0, 0, 0.05, 0.05, 0.05), np.zeros((5, 9, 12), np.float32), 0.0, 0.02, 3, flat)
    assert (g.leaf_levels().cpu().numpy() == g.L).all()
    bd, bk = inputs.lognormal_blob()
    g = _compare(bd, bk, 0.0, 0.01, 3, flat)
    assert (g.leaf_levels().cpu().numpy() == min(flat, g.L)).all()


def test_cylinder_256():
    desc, k = inputs.cylinder_cumulus()
    _compare(desc, k, 1.0)


def test_cumulus_small():
    desc, k = inputs.cumulus_field(fine=(80, 256, 256), pool=2)
    for tau in (0.0, 1.0, 10.0):
        _compare(desc, k, tau, 0.05)


def test_invalid_fields():
    c = ctx()
    desc = FieldDesc(4, 4, 4, 0, 0, 0, 0.1, 0.1, 0.1)
    for bad in (np.nan, -1.0, np.inf):
        k = np.ones((4, 4, 4), np.float32)
        k[2, 1, 3] = bad
        with pytest.raises(_lib.NcError) as e:
            api.build_grid(c, device_field(k), desc, GridParams(1.0))
        assert e.value.status == _lib.NC_ERR_RANGE
    with pytest.raises(_lib.NcError) as e:
        api.build_grid(c, device_field(np.ones((4, 4, 4), np.float32)), desc, GridParams(-1.0))
    assert e.value.status == _lib.NC_ERR_RANGE
