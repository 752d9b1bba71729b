"""Pins of the oracle's grid build (Section 3.1.1, merge criterion of Section 4.2).

Hand-computed partitions on tiny grids, the closed form for a uniform field,
the tau_tilde = 0 and tau_tilde = inf limits, and invariants checked by brute
force (numpy block reductions) on random fields.
"""
import math

import numpy as np
import pytest

from paper_1902_01137_amd.inputs import FieldDesc


def grid(orc, desc, k, tau, kg=0.0, crit=0):
    return orc.OracleGrid(desc, k, tau_tilde=tau, k_gas=kg, criterion=crit)


def test_2x2x2_strict_threshold(orc):
    k = (np.arange(1, 9, dtype=np.float32) / 8.0).reshape(2, 2, 2)   # 0.125 .. 1.0
    desc = FieldDesc(2, 2, 2, 0, 0, 0, 1.0, 1.0, 1.0)
    # level-1 root: kmax = 1.0, criterion value 1.0 * (1.0 * 2) = 2.0
    g = grid(orc, desc, k, 2.0)
    assert g.L == 1
    kmin, kmax, mg = g.level(1)
    assert kmin.item() == 0.125 and kmax.item() == 1.0 and mg.item() == 0   # 2.0 < 2.0 is false
    assert (g.leaf_levels() == 0).all()
    g = grid(orc, desc, k, 2.0000001)
    assert g.level(1)[2].item() == 1
    assert (g.leaf_levels() == 1).all()


def test_4x4x2_single_bright_cell(orc):
    # nx=4, ny=4, nz=2, dz=0.5; bright cell at x=3, y=0, z=1
    k = np.ones((2, 4, 4), np.float32)
    k[1, 0, 3] = 10.0
    desc = FieldDesc(4, 4, 2, 0, 0, 0, 0.5, 0.5, 0.5)
    g = grid(orc, desc, k, 5.0)
    assert g.L == 2
    assert g.level_dims(1) == (2, 2, 1) and g.level_dims(2) == (1, 1, 1)
    _, kmax1, mg1 = g.level(1)
    # level-1 nodes (x,y): (1,0) holds the bright cell; criterion kmax * 0.5 * 2
    assert kmax1[0].tolist() == [[1.0, 10.0], [1.0, 1.0]]
    assert mg1[0].tolist() == [[1, 0], [1, 1]]
    _, kmax2, mg2 = g.level(2)
    assert kmax2.item() == 10.0 and mg2.item() == 0          # 10 * 0.5 * 4 = 20
    expect = np.ones((2, 4, 4), np.uint8)
    expect[:, 0:2, 2:4] = 0
    assert (g.leaf_levels() == expect).all()
    g = grid(orc, desc, k, 25.0)
    assert (g.leaf_levels() == 2).all()


@pytest.mark.parametrize("kval,kg,tau,expect", [
    (0.5, 0.0, 1.0, 2),     # 0.5*0.25*2^l < 1  ->  l <= 2
    (0.5, 0.5, 1.0, 1),     # (0.5+0.5)*0.25*2^l < 1 -> l <= 1
    (0.5, 0.0, 0.0, 0),     # tau_tilde = 0: never merged
    (0.5, 0.0, math.inf, 3),  # tau_tilde = inf: the root
    (0.0, 0.0, 1e-30, 3),   # empty field: 0 < tiny merges everything
])
def test_uniform_field_closed_form(orc, kval, kg, tau, expect):
    k = np.full((8, 8, 8), kval, np.float32)
    desc = FieldDesc(8, 8, 8, 0, 0, 0, 0.25, 0.25, 0.25)
    g = grid(orc, desc, k, tau, kg)
    assert (g.leaf_levels() == expect).all()


def _check_invariants(orc, desc, k, tau, kg, crit):
    g = grid(orc, desc, k, tau, kg, crit)
    nz, ny, nx = k.shape
    assert g.L == max(0, math.ceil(math.log2(max(nx, ny, nz))))
    leaf = g.leaf_levels()
    cover = np.zeros(k.shape, np.int32)
    for l in range(1, g.L + 1):
        kmin, kmax, mg = g.level(l)
        f = 1 << l
        dims = g.level_dims(l)
        assert dims == (-(-nx // f), -(-ny // f), -(-nz // f))
        # brute-force block min / max with edge padding by +-inf
        pad = [(0, dims[2] * f - nz), (0, dims[1] * f - ny), (0, dims[0] * f - nx)]
        hi = np.pad(k, pad, constant_values=-np.inf).reshape(dims[2], f, dims[1], f, dims[0], f)
        lo = np.pad(k, pad, constant_values=np.inf).reshape(dims[2], f, dims[1], f, dims[0], f)
        assert np.array_equal(kmax, hi.max(axis=(1, 3, 5)))
        assert np.array_equal(kmin, lo.min(axis=(1, 3, 5)))
        dz = desc.dz * f
        crit_v = (kmax.astype(np.float64) + kg) * dz if crit == 0 else \
            (kmax.astype(np.float64) - kmin.astype(np.float64)) * dz
        assert np.array_equal(mg.astype(bool), crit_v < tau)
        # monotone: merged parent => merged children
        if l >= 2:
            _, _, mgc = g.level(l - 1)
            up = np.repeat(np.repeat(np.repeat(mg, 2, 0), 2, 1), 2, 2)[:mgc.shape[0], :mgc.shape[1], :mgc.shape[2]]
            assert not np.any(up.astype(bool) & ~mgc.astype(bool))
    # each cell's leaf: merged at its level, parent (if any) not merged
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for l in range(0, g.L + 1):
        sel = leaf == l
        if not sel.any():
            continue
        if l >= 1:
            _, _, mg = g.level(l)
            assert mg[zz[sel] >> l, yy[sel] >> l, xx[sel] >> l].all()
        if l < g.L:
            _, _, mgp = g.level(l + 1)
            assert not mgp[zz[sel] >> (l + 1), yy[sel] >> (l + 1), xx[sel] >> (l + 1)].any()
        cover[sel] += 1
    assert (cover == 1).all()   # leaves tile the cells exactly once
    return g


@pytest.mark.parametrize("shape", [(7, 3, 5), (16, 16, 16), (5, 9, 12), (1, 1, 6)])
@pytest.mark.parametrize("crit", [0, 1])
def test_random_field_invariants(orc, shape, crit):
    rng = np.random.default_rng(sum(shape) + crit)
    k = (rng.random(shape) ** 8 * 60).astype(np.float32)
    nz, ny, nx = shape
    desc = FieldDesc(nx, ny, nz, 0, 0, 0, 0.05, 0.05, 0.05)
    for tau in (0.0, 0.3, 1.0, 10.0, np.inf):
        _check_invariants(orc, desc, k, tau, 0.02, crit)


def test_single_cell_field(orc):
    k = np.full((1, 1, 1), 3.0, np.float32)
    g = grid(orc, FieldDesc(1, 1, 1, 0, 0, 0, 1, 1, 1), k, 10.0)
    assert g.L == 0 and (g.leaf_levels() == 0).all()


@pytest.mark.parametrize("shape,flat", [((16, 16, 16), 3), ((7, 3, 5), 1), ((5, 9, 12), 8), ((1, 1, 6), 0)])
def test_flat_supercell_grid(orc, shape, flat):
    """Criterion 2: every node of level <= flat_level is merged whatever the
    field, so every cell's voxel is its level-min(flat_level, L) ancestor,
    and the stored extrema are still the exact block extrema."""
    rng = np.random.default_rng(sum(shape) + flat)
    k = (rng.random(shape) ** 8 * 60).astype(np.float32)
    nz, ny, nx = shape
    desc = FieldDesc(nx, ny, nz, 0, 0, 0, 0.05, 0.05, 0.05)
    g = orc.OracleGrid(desc, k, tau_tilde=0.0, criterion=2, flat_level=flat)
    assert (g.leaf_levels() == min(flat, g.L)).all()
    for l in range(1, g.L + 1):
        kmin, kmax, mg = g.level(l)
        assert (mg == (l <= flat)).all()
        s = 1 << l
        dz_, dy_, dx_ = kmin.shape
        for m, j, i in [(0, 0, 0), (dz_ - 1, dy_ - 1, dx_ - 1), (dz_ // 2, dy_ // 2, dx_ // 2)]:
            blk = k[m * s:(m + 1) * s, j * s:(j + 1) * s, i * s:(i + 1) * s]
            assert kmin[m, j, i] == blk.min() and kmax[m, j, i] == blk.max()


def test_layered_grid_hand_case(orc):
    """Criterion 3 on a 4 x 4 x 16 field whose only cloud cells sit at z = 5
    and z = 9, supercells of 2 cells (flat_level 1) in the cloudy layer.
    Per z index, the voxel level follows from the node ranges by hand: z 0-3
    and 12-15 lie in clear level-2 nodes (z 0-3, 12-15) whose level-3 parents
    (z 0-7, 8-15) reach the cloud; z 4-11 have no clear level-2 ancestor and
    stop at level 1."""
    k = np.zeros((16, 4, 4), np.float32)
    k[5, 1, 2] = 30.0
    k[9, 3, 0] = 0.5
    desc = FieldDesc(4, 4, 16, 0, 0, 0, 0.05, 0.05, 0.05)
    g = orc.OracleGrid(desc, k, tau_tilde=0.0, k_gas=0.05, criterion=3, flat_level=1)
    leaf = g.leaf_levels()
    expect_z = [2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2]
    for z in range(16):
        assert (leaf[z] == expect_z[z]).all(), (z, leaf[z])


def _layered_leaf_by_definition(k, flat):
    """Brute force: for each cell, the coarsest level l whose node either has
    no cloud cell anywhere in its z range's layers or has l <= flat."""
    nz, ny, nx = k.shape
    cloudy_z = np.nonzero((k > 0).any(axis=(1, 2)))[0]
    L = max(int(math.ceil(math.log2(max(nx, ny, nz)))), 0)
    leaf = np.zeros(k.shape, np.int64)
    for z in range(nz):
        best = 0
        for l in range(1, L + 1):
            za, zb = (z >> l) << l, min(((z >> l) + 1) << l, nz) - 1
            clear = not np.any((cloudy_z >= za) & (cloudy_z <= zb))
            if clear or l <= flat:
                best = l
        leaf[z] = best
    return leaf


@pytest.mark.parametrize("shape,flat,layer", [((40, 24, 32), 2, (11, 23)), ((33, 17, 9), 0, (3, 3)),
                                              ((64, 8, 8), 3, (20, 47)), ((16, 16, 16), 1, None)])
def test_layered_grid_matches_definition(orc, shape, flat, layer):
    """Criterion 3 against a cell-by-cell restatement of its definition on
    ragged fields with a random cloud layer (or none: then one voxel)."""
    rng = np.random.default_rng(sum(shape) + flat)
    nz, ny, nx = shape
    k = np.zeros(shape, np.float32)
    if layer is not None:
        z0, z1 = layer
        blob = (rng.random((z1 - z0 + 1, ny, nx)) ** 6 * 40).astype(np.float32)
        blob[rng.random(blob.shape) < 0.7] = 0.0
        blob[0, 0, 0], blob[-1, -1, -1] = 1.0, 2.0        # the layer's bottom and top hold cloud
        k[z0:z1 + 1] = blob
    desc = FieldDesc(nx, ny, nz, 0, 0, 0, 0.025, 0.025, 0.025)
    g = orc.OracleGrid(desc, k, tau_tilde=1.0, k_gas=0.05, criterion=3, flat_level=flat)
    assert np.array_equal(g.leaf_levels(), _layered_leaf_by_definition(k, flat))
    if layer is None:
        assert (g.leaf_levels() == g.L).all()
