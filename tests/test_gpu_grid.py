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
    if g.L >= 1:
        assert np.array_equal(g.mask().cpu().numpy(), _oracle_mask(og))
    return g


def _oracle_mask(og):
    """Ancestry bits per level-1 node from the oracle's merged flags: bit l
    set if the level-l ancestor (the node itself at l = 1) is merged."""
    d0, d1, d2 = og.level_dims(1)
    m, j, i = np.meshgrid(np.arange(d2), np.arange(d1), np.arange(d0), indexing="ij")
    bits = np.zeros((d2, d1, d0), np.int64)
    for l in range(1, og.L + 1):
        mg = og.level(l)[2]
        sh = l - 1
        bits |= mg[m >> sh, j >> sh, i >> sh].astype(np.int64) << l
    return bits


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


def test_row_aligned_and_misaligned_field():
    """A field whose rows are whole 16-byte groups (nx a multiple of 4), with
    ragged y and z over several 16^3 blocks: built from an aligned buffer and
    from one offset by a single float (read cell by cell), both against the
    oracle."""
    rng = np.random.default_rng(52)
    shape = (37, 45, 52)
    k = (rng.random(shape) ** 8 * 60).astype(np.float32)
    nz, ny, nx = shape
    desc = FieldDesc(nx, ny, nz, 0, 0, 0, 0.05, 0.05, 0.05)
    for tau in (0.0, 0.3, 3.0):
        _compare(desc, k, tau, 0.02)
    c = ctx()
    buf = torch.empty(k.size + 1, dtype=torch.float32, device="cuda")
    buf[1:] = torch.from_numpy(k.ravel()).cuda()
    kd = buf[1:].view(shape)
    assert kd.data_ptr() % 16 == 4
    g = api.build_grid(c, kd, desc, GridParams(0.3, 0.02, 0, 3))
    og = oracle.OracleGrid(desc, k, tau_tilde=0.3, k_gas=0.02)
    for l in range(1, g.L + 1):
        kmin, kmax, mg = (t.cpu().numpy() for t in g.level(l))
        assert all(np.array_equal(a, b) for a, b in zip((kmin, kmax, mg), og.level(l))), l
    assert np.array_equal(g.mask().cpu().numpy(), _oracle_mask(og))


def test_rebuild_in_place():
    """A grid rebuilt over a second field of its shape equals a fresh build
    over that field (every level and the mask); a rebuild over an invalid
    field is refused, and a later valid rebuild restores the grid."""
    desc, k = inputs.lognormal_blob()
    c = ctx()
    gp = GridParams(1.0, 0.01, 0, 3)
    g = api.build_grid(c, device_field(k), desc, gp)
    k2 = (k * 0.37)[::-1].copy()
    kd2 = device_field(k2)
    g.rebuild(kd2)
    f = api.build_grid(c, kd2, desc, gp)
    og = oracle.OracleGrid(desc, k2, tau_tilde=1.0, k_gas=0.01)
    for l in range(1, g.L + 1):
        a = [t.cpu().numpy() for t in g.level(l)]
        b = [t.cpu().numpy() for t in f.level(l)]
        assert all(np.array_equal(x, y) for x, y in zip(a, b)), l
        assert all(np.array_equal(x, y) for x, y in zip(a, og.level(l))), l
    assert np.array_equal(g.mask().cpu().numpy(), f.mask().cpu().numpy())
    bad = k2.copy()
    bad[3, 4, 5] = np.nan
    with pytest.raises(_lib.NcError) as e:
        g.rebuild(device_field(bad))
    assert e.value.status == _lib.NC_ERR_RANGE
    g.rebuild(kd2)
    assert np.array_equal(g.mask().cpu().numpy(), _oracle_mask(og))


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
