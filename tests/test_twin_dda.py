"""The GPU path's ordered crossing compiled for the host (FP32 twin) against
the oracle's FP64 crossing (Section 3.1.3), on the CPU: every ray the oracle
does not flag as degenerate must give the same voxel sequence, and every ray
must cover its chord inside the box without gap or overlap, each voxel once.
The GPU itself is compared with the twin on every ray in test_gpu_dda.py."""
import numpy as np
import pytest

from paper_1902_01137_amd import inputs
from paper_1902_01137_amd.inputs import FieldDesc
from twin import dda_twin


def _eps(desc):
    (xa, xb), (ya, yb), (za, zb) = desc.box
    scale = max(abs(xa), abs(xb), abs(ya), abs(yb), abs(za), abs(zb), xb - xa, yb - ya, zb - za) * 2.5
    return 64 * scale * 2.0 ** -23


def covers_chord(desc, ray, leaf, t, n):
    """Voxels in order along the ray, each entered where the last one was
    left, none twice; the first entered at the box entry, the last left at
    the box exit (float32 walk: equal up to the walk's own rounding)."""
    if n == 0:
        return True
    lv = [tuple(v) for v in leaf[:n]]
    if len(set(lv)) != n:
        return False
    if not np.all(t[1:n, 0] == t[:n - 1, 1]):
        return False
    if not np.all(t[:n, 1] > t[:n, 0]):
        return False
    o, d = ray[:3].astype(np.float64), ray[3:].astype(np.float64)
    (xa, xb), (ya, yb), (za, zb) = desc.box
    lo, hi = np.array([xa, ya, za]), np.array([xb, yb, zb])
    with np.errstate(divide="ignore", invalid="ignore"):
        ta = np.where(d != 0, (lo - o) / d, -np.inf)
        tb = np.where(d != 0, (hi - o) / d, np.inf)
    tin = max(0.0, np.minimum(ta, tb).max())
    tout = np.maximum(ta, tb).min()
    tol = 1e-5 * max(1.0, abs(tout))
    return abs(t[0, 0] - tin) <= tol and abs(t[n - 1, 1] - tout) <= tol


def _check(orc, desc, k, tau, rays, kg=0.0, maxv=2048):
    og = orc.OracleGrid(desc, k, tau_tilde=tau, k_gas=kg)
    levels = [og.level(l) for l in range(1, og.L + 1)]
    leaf, t, cnt = dda_twin.trace(desc, k, levels, rays, maxv)
    eps = _eps(desc)
    deg = 0
    for i, r in enumerate(rays):
        assert cnt[i] <= maxv
        assert covers_chord(desc, r, leaf[i], t[i], cnt[i]), i
        oseq, ot, odeg = og.leaf_sequence(r.astype(np.float64), eps, maxv=maxv)
        if odeg:
            deg += 1
            continue
        n = cnt[i]
        assert n == len(oseq), (i, n, len(oseq))
        assert np.array_equal(leaf[i, :n], oseq), i
        assert np.allclose(t[i, :n], ot, rtol=0, atol=4 * eps), i
    return deg


@pytest.mark.parametrize("tau", [0.0, 1.0, 10.0])
def test_twin_blob_random_rays(orc, tau):
    desc, k = inputs.lognormal_blob()
    rays = inputs.random_rays(desc, 3000, seed=31)
    deg = _check(orc, desc, k, tau, rays)
    assert deg <= 0.03 * len(rays), deg


def test_twin_ragged_grid_rays(orc):
    rng = np.random.default_rng(8)
    k = (rng.random((13, 21, 37)) ** 6 * 30).astype(np.float32)
    desc = FieldDesc(37, 21, 13, -1.3, 2.2, 0.4, 0.07, 0.11, 0.05)
    rays = inputs.random_rays(desc, 3000, seed=32)
    deg = _check(orc, desc, k, 0.7, rays, kg=0.01)
    assert deg <= 0.03 * len(rays), deg


def test_twin_axis_parallel_rays_through_faces(orc):
    """Rays along the axes lying exactly in cell-face planes (the oracle
    flags them; the twin must still cover the chord once)."""
    desc, k = inputs.lognormal_blob()
    og = orc.OracleGrid(desc, k, tau_tilde=1.0)
    levels = [og.level(l) for l in range(1, og.L + 1)]
    rays = []
    for a in range(3):
        for f in (4, 8, 16):
            o = np.array([desc.x0 + 1.55, desc.y0 + 1.45, desc.z0 + 1.65])
            b = (a + 1) % 3
            o[b] = (desc.x0, desc.y0, desc.z0)[b] + f * (desc.dx, desc.dy, desc.dz)[b]
            d = np.zeros(3)
            d[a] = 1.0
            o[a] = (desc.x0, desc.y0, desc.z0)[a] - 0.5
            rays.append(np.concatenate([o, d]))
    rays = np.array(rays, np.float32)
    leaf, t, cnt = dda_twin.trace(desc, k, levels, rays, 256)
    for i, r in enumerate(rays):
        assert cnt[i] > 0 and covers_chord(desc, r, leaf[i], t[i], cnt[i]), i
