"""Pins of the oracle's ordered grid crossing (Section 3.1.3).

Brute-force marching with a step far below the cell size, closed-form
sequences for axis-parallel rays, and the chord-length identity.
"""
import numpy as np
import pytest

from paper_1902_01137_amd.inputs import FieldDesc, random_rays


def _field(seed=3, n=(8, 8, 8), cell=0.1):
    rng = np.random.default_rng(seed)
    nz, ny, nx = n
    k = (rng.random(n) ** 6 * 40).astype(np.float32)
    k[:, :, : nx // 2] *= 0.01     # a clear half that merges into coarse leaves
    return FieldDesc(nx, ny, nz, 0.2, -0.3, 1.0, cell, cell, cell), k


def _march(desc, leaf_map, ray, step):
    o = ray[:3].astype(np.float64)
    d = ray[3:].astype(np.float64)
    lo = np.array([desc.x0, desc.y0, desc.z0])
    h = np.array([desc.dx, desc.dy, desc.dz])
    n = np.array([desc.nx, desc.ny, desc.nz])
    hi = lo + n * h
    with np.errstate(divide="ignore", invalid="ignore"):
        t0 = (lo - o) / d
        t1 = (hi - o) / d
    tmin = np.where(d != 0, np.minimum(t0, t1), -np.inf)
    tmax = np.where(d != 0, np.maximum(t0, t1), np.inf)
    inside_par = np.all((d != 0) | ((o >= lo) & (o <= hi)))
    ta, tb = max(tmin.max(), 0.0), tmax.min()
    if not inside_par or not ta < tb:
        return []
    ts = np.arange(ta + step / 2, tb, step)
    p = o[None, :] + ts[:, None] * d[None, :]
    c = np.clip(np.floor((p - lo) / h).astype(np.int64), 0, n - 1)
    lev = leaf_map[c[:, 2], c[:, 1], c[:, 0]].astype(np.int64)
    ids = np.stack([lev, c[:, 0] >> lev, c[:, 1] >> lev, c[:, 2] >> lev], axis=1)
    change = np.ones(len(ids), bool)
    change[1:] = np.any(ids[1:] != ids[:-1], axis=1)
    return [tuple(int(v) for v in r) for r in ids[change]]


@pytest.mark.parametrize("tau", [0.0, 1.0, 5.0])
def test_leaf_sequence_vs_brute_force_marching(orc, tau):
    desc, k = _field()
    g = orc.OracleGrid(desc, k, tau_tilde=tau, k_gas=0.01)
    leaf_map = g.leaf_levels()
    rays = random_rays(desc, 120, seed=11)
    step = 2e-5
    checked = 0
    for r in rays:
        seq, t, deg = g.leaf_sequence(r, eps=1e-9)
        if deg or (len(seq) and np.min(t[:, 1] - t[:, 0]) < 50 * step):
            continue
        marched = _march(desc, leaf_map, r, step)
        assert [tuple(x) for x in seq.tolist()] == marched
        checked += 1
    assert checked > 60


def test_chord_length_identity(orc):
    desc, k = _field(seed=4)
    g = orc.OracleGrid(desc, k, tau_tilde=1.0)
    rays = random_rays(desc, 300, seed=12)
    (xa, xb), (ya, yb), (za, zb) = desc.box
    for r in rays:
        seq, t, deg = g.leaf_sequence(r, eps=1e-9)
        if len(seq) == 0:
            continue
        o, d = r[:3].astype(np.float64), r[3:].astype(np.float64)
        lo = np.array([xa, ya, za])
        hi = np.array([xb, yb, zb])
        with np.errstate(divide="ignore", invalid="ignore"):
            a = np.where(d != 0, np.minimum((lo - o) / d, (hi - o) / d), -np.inf)
            b = np.where(d != 0, np.maximum((lo - o) / d, (hi - o) / d), np.inf)
        chord = b.min() - max(a.max(), 0.0)
        assert np.isclose((t[:, 1] - t[:, 0]).sum(), chord, rtol=0, atol=1e-12)
        assert np.all(t[1:, 0] == t[:-1, 1])      # contiguous


def test_axis_parallel_closed_form(orc):
    # tau_tilde = 0: every cell is a leaf; a +x ray through cell row (j, m)
    desc, k = _field(seed=5)
    g = orc.OracleGrid(desc, k, tau_tilde=0.0)
    j, m = 3, 5
    y = desc.y0 + (j + 0.37) * desc.dy
    z = desc.z0 + (m + 0.61) * desc.dz
    ox = desc.x0 - 0.5
    seq, t, deg = g.leaf_sequence(np.array([ox, y, z, 1.0, 0.0, 0.0]), eps=1e-9)
    assert not deg
    assert seq.tolist() == [[0, i, j, m] for i in range(desc.nx)]
    edges = desc.x0 + np.arange(desc.nx + 1) * desc.dx - ox
    assert np.allclose(t[:, 0], edges[:-1], atol=1e-12) and np.allclose(t[:, 1], edges[1:], atol=1e-12)
    # same ray backwards from inside cell 4: cells 4..0
    seq, t, deg = g.leaf_sequence(np.array([desc.x0 + 4.5 * desc.dx, y, z, -1.0, 0.0, 0.0]), eps=1e-9)
    assert seq.tolist() == [[0, i, j, m] for i in range(4, -1, -1)]
    assert np.isclose(t[0, 1], 0.5 * desc.dx)


def test_merged_root_single_leaf(orc):
    desc, k = _field(seed=6)
    g = orc.OracleGrid(desc, k, tau_tilde=np.inf)
    for r in random_rays(desc, 50, seed=13):
        seq, t, deg = g.leaf_sequence(r, eps=1e-9)
        assert len(seq) <= 1
        if len(seq):
            assert seq.tolist() == [[3, 0, 0, 0]]


def test_missing_ray_and_degenerate_flags(orc):
    desc, k = _field(seed=7)
    g = orc.OracleGrid(desc, k, tau_tilde=0.0)
    (xa, xb), (ya, yb), (za, zb) = desc.box
    # pointing away from the box
    seq, t, deg = g.leaf_sequence(np.array([xa - 1, ya + 0.1, za + 0.1, -1, 0, 0]), eps=1e-9)
    assert len(seq) == 0
    # running exactly along an interior face plane
    seq, t, deg = g.leaf_sequence(np.array([xa - 1, ya + 2 * desc.dy, za + 0.05, 1, 0, 0]), eps=1e-9)
    assert deg
    # through an interior cell edge (two faces crossed at once)
    p = np.array([xa + 3 * desc.dx, ya + 3 * desc.dy, za + 0.35])
    d = np.array([1.0, 1.0, 0.0]) / np.sqrt(2)
    seq, t, deg = g.leaf_sequence(np.concatenate([p - 0.3 * d, d]), eps=1e-9)
    assert deg
