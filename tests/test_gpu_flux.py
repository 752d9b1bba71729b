"""Forward photons and their sensitivities on the GPU (Section 5.1, Eq. 3):
energy conservation, Beer-Lambert and its derivative, the cylinder cumulus
against the oracle (transmissivity, score estimates and CRN finite
differences), and the adjoint replay / autograd path."""
import math
import os

import numpy as np
import pytest
import torch

import oracle
from gpu_common import ctx, device_field
from paper_1902_01137_amd import _lib, api, inputs
from paper_1902_01137_amd.inputs import GridParams, Optics, Sampling
from stats import compare, z_scalar

pytestmark = pytest.mark.gpu


def _setup(desc, k, tau_tilde=1.0, kg=0.0):
    c = ctx()
    kd = device_field(k)
    g = api.build_grid(c, kd, desc, GridParams(tau_tilde, kg, 0))
    return c, kd, g


def test_energy_conservation():
    desc, k = inputs.slab_field([4.0], 0.5, z0=0.2)
    c, kd, g = _setup(desc, k)
    n = 200000
    for ssa, rho in ((0.9, 0.3), (1.0, 1.0), (0.0, 0.5)):
        op = Optics(ssa=ssa, g=0.7, ground_albedo=rho, sun_zenith_deg=30.0)
        tally, glob = api.flux(c, g, kd, op, (1, 1), n, Sampling(seed=3))
        gl = glob.cpu().numpy()
        assert gl.sum() == n
        if ssa == 1.0:
            assert gl[3] == 0
        if ssa == 1.0 and rho == 1.0:
            assert gl[0] == n


@pytest.mark.parametrize("s", [1.0, 1.4])
def test_beer_lambert_and_scale_derivative(s):
    tau, th0 = 1.2, 40.0
    desc, k = inputs.slab_field([tau / 0.5], 0.5, z0=0.3)
    c, kd, g = _setup(desc, k)
    op = Optics(ssa=0.0, g=0.85, ground_albedo=0.0, sun_zenith_deg=th0, majorant_scale=2.0)
    n = 2_000_000
    tally, glob = api.flux(c, g, kd, op, (1, 1), n, Sampling(seed=4), extinction_scale=s)
    t = tally.cpu().numpy().reshape(9)
    mu0 = math.cos(math.radians(th0))
    exact = math.exp(-s * tau / mu0)
    T = t[0] / n
    assert abs(z_scalar(T, math.sqrt(exact * (1 - exact) / n), exact)) < 3.0
    d = t[3] / n
    se = math.sqrt(max(t[4] / n - d * d, 0) / n)
    assert abs(z_scalar(d, se, -(tau / mu0) * exact)) < 3.0
    assert t[5] == 0.0 and t[7] == 0.0 and t[2] == t[0]


def _cyl(n_photons_gpu=10_000_000):
    sc = inputs.scene_cylinder()
    c, kd, g = _setup(sc.desc, sc.kc, sc.grid.tau_tilde)
    cnt = api.new_counters("cuda")
    tally, glob = api.flux(c, g, kd, sc.optics, (100, 100), n_photons_gpu, Sampling(seed=1004), counters=cnt)
    torch.cuda.synchronize()
    return sc, c, kd, g, tally.cpu().numpy(), glob.cpu().numpy(), api.counters_dict(cnt)


def _maps(t, n, f):
    """mean and SE maps of tallies (sum, sumsq) scaled by f."""
    m = t[0] / n
    se = np.sqrt(np.maximum(t[1] / n - m * m, 0) / n)
    return m * f, se * f


def _blocks(m, se, b=10):
    H, W = m.shape
    mb = m.reshape(H // b, b, W // b, b).mean(axis=(1, 3)).ravel()
    sb = np.sqrt((se.reshape(H // b, b, W // b, b) ** 2).sum(axis=(1, 3))).ravel() / (b * b)
    return mb, sb


def test_cylinder_transmissivity_vs_oracle():
    N = 10_000_000
    sc, c, kd, g, t, glob, cnt = _cyl(N)
    assert glob.sum() == N and cnt["truncated"] == 0
    f = 100 * 100
    gm, gse = _maps(np.stack([t[0], t[1]]), N, f)
    No = 800_000
    ot, oglob = oracle.parallel_flux(sc.desc, sc.kc, 0.0, sc.optics, (100, 100), No, seed=inputs.SEED_ORACLE_BASE + 4)
    om, ose = _maps(np.stack([ot[0], ot[1]]), No, f)
    res = compare(*_blocks(gm, gse), *_blocks(om, ose))
    assert res["ok"], res
    # clear-sky pixels far from the cloud see the direct beam: T = 1 (no gas)
    assert abs(gm[:5, :5].mean() - 1.0) < 0.02


def test_cylinder_sensitivities_vs_oracle():
    """GPU score estimates of dT/ds, dT/dg and dT/dalpha against the oracle's
    score estimator and its common-random-number central differences."""
    N = 10_000_000
    sc, c, kd, g, t, glob, cnt = _cyl(N)
    f = 100 * 100
    ds_g, ds_gse = _maps(np.stack([t[3], t[4]]), N, f)
    dg_g, dg_gse = _maps(np.stack([t[5], t[6]]), N, f)
    da_g, da_gse = _maps(np.stack([t[7], t[8]]), N, f)
    No = 800_000
    ot, _ = oracle.parallel_flux(sc.desc, sc.kc, 0.0, sc.optics, (100, 100), No, seed=inputs.SEED_ORACLE_BASE + 14,
                                 mode=2, tau_tilde=1.0)
    ds_o, ds_ose = _maps(np.stack([ot[3], ot[4]]), No, f)
    dg_o, dg_ose = _maps(np.stack([ot[5], ot[6]]), No, f)
    da_o, da_ose = _maps(np.stack([ot[7], ot[8]]), No, f)
    for a, sa, b, sb in ((ds_g, ds_gse, ds_o, ds_ose), (dg_g, dg_gse, dg_o, dg_ose), (da_g, da_gse, da_o, da_ose)):
        res = compare(*_blocks(a, sa), *_blocks(b, sb))
        assert res["ok"], res
    # domain means against CRN finite differences of exactly-tracked photons
    Nf = 2_000_000
    # alpha = 1 - ssa = 0.001 here: its step stays below alpha so that ssa stays a probability
    for which, (a, sa), h in ((0, (ds_g, ds_gse), 1e-3), (1, (dg_g, dg_gse), 1e-3), (2, (da_g, da_gse), 5e-4)):
        _, tot = oracle.parallel_flux_fd(sc.desc, sc.kc, 0.0, sc.optics, (100, 100), Nf,
                                         seed=inputs.SEED_ORACLE_BASE + 24 + which, which=which, h=h)
        q = tot[0] / Nf        # per-photon quotient summed over pixels
        q2 = tot[1] / Nf
        se_fd = math.sqrt(max(q2 - q * q, 0) / Nf)
        gpu_mean = a.mean()                       # mean over pixels of dT_p/dpi
        gpu_se = math.sqrt((sa ** 2).sum()) / a.size
        fd_mean = q      # = (1/npix) sum_p dT_p/dpi, since T_p = arrivals_p * npix / N
        assert abs(fd_mean) > 2 * se_fd or abs(gpu_mean) < 3 * gpu_se
        z = (gpu_mean - fd_mean) / math.sqrt(gpu_se ** 2 + se_fd ** 2)
        assert abs(z) < 3, (which, gpu_mean, gpu_se, fd_mean, se_fd)


def test_cylinder_block_derivatives_vs_crn_fd():
    """dT/ds, dT/dg and dT/dalpha per 20x20-pixel ground block: the GPU's
    score estimates against the oracle's common-random-number central
    differences of exactly-tracked photons (h = 1e-3; 5e-4 for alpha, which
    is 1e-3 here), within 3 combined standard errors by the parity rule."""
    N = 10_000_000
    sc, c, kd, g, t, glob, cnt = _cyl(N)
    f = 100 * 100
    Nf = 6_000_000
    workers = min(16, os.cpu_count() or 1)
    for which, (ti, h) in enumerate(((3, 1e-3), (5, 1e-3), (7, 5e-4))):
        gm, gse = _maps(np.stack([t[ti], t[ti + 1]]), N, f)
        out, _ = oracle.parallel_flux_fd(sc.desc, sc.kc, 0.0, sc.optics, (100, 100), Nf,
                                         seed=inputs.SEED_ORACLE_BASE + 34 + which, which=which, h=h, workers=workers)
        om, ose = _maps(out, Nf, f)
        res = compare(*_blocks(gm, gse, 20), *_blocks(om, ose, 20))
        assert res["ok"], (which, res)


def test_normalised_flux_outputs():
    """NC_FLUX_NORMALISE: the kernels apply px_nx px_ny / n_photons to every
    arrival (its square to the squares) and to the adjoint's sums."""
    sc = inputs.scene_cylinder()
    c, kd, g = _setup(sc.desc, sc.kc)
    N = 1_000_000
    smp = Sampling(seed=79)
    smpn = Sampling(seed=79, flags=_lib.NC_FLUX_NORMALISE)
    raw, glob = api.flux(c, g, kd, sc.optics, (50, 40), N, smp)
    nrm, globn = api.flux(c, g, kd, sc.optics, (50, 40), N, smpn)
    f = 50 * 40 / N
    for k in range(9):
        fk = f * f if k in (1, 4, 6, 8) else f
        torch.testing.assert_close(nrm[k], raw[k] * fk, rtol=1e-9, atol=1e-12)
    torch.testing.assert_close(globn, glob, rtol=0, atol=0)
    grad = torch.from_numpy(np.random.default_rng(4).standard_normal((40, 50))).cuda()
    a = api.flux_adjoint(c, g, kd, sc.optics, (50, 40), N, smp, grad)
    b = api.flux_adjoint(c, g, kd, sc.optics, (50, 40), N, smpn, grad)
    torch.testing.assert_close(b, a * f, rtol=1e-9, atol=1e-12)


def test_adjoint_replays_forward_paths():
    sc = inputs.scene_cylinder()
    c, kd, g = _setup(sc.desc, sc.kc)
    N = 1_000_000
    smp = Sampling(seed=77)
    tally, _ = api.flux(c, g, kd, sc.optics, (100, 100), N, smp)
    rng = np.random.default_rng(3)
    grad = torch.from_numpy(rng.standard_normal((100, 100))).cuda()
    out = api.flux_adjoint(c, g, kd, sc.optics, (100, 100), N, smp, grad)
    t = tally.cpu().numpy()
    gr = grad.cpu().numpy()
    exp_s = (gr * t[3]).sum()
    exp_g = (gr * t[5]).sum()
    exp_a = (gr * t[7]).sum()
    o = out.cpu().numpy()
    assert o[0] == pytest.approx(exp_s, rel=1e-9, abs=1e-6)
    assert o[1] == pytest.approx(exp_g, rel=1e-9, abs=1e-6)
    assert o[2] == pytest.approx(exp_a, rel=1e-9, abs=1e-6)


def test_autograd_function():
    sc = inputs.scene_cylinder()
    c, kd, g = _setup(sc.desc, sc.kc)
    N = 1_000_000
    smp = Sampling(seed=78)
    s = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    gg = torch.tensor(0.85, dtype=torch.float64, requires_grad=True)
    aa = torch.tensor(1.0 - sc.optics.ssa, dtype=torch.float64, requires_grad=True)
    T = api.TransmissionFn.apply(s, gg, aa, c, g, kd, sc.optics, (100, 100), N, smp)
    w = torch.linspace(0, 1, 100 * 100, dtype=torch.float64, device="cuda").reshape(100, 100)
    L = (T * w).sum()
    L.backward()
    tally, _ = api.flux(c, g, kd, sc.optics, (100, 100), N, smp)
    t = tally.cpu().numpy()
    f = 100 * 100 / N
    wn = w.cpu().numpy()
    assert float(L.detach()) == pytest.approx((wn * t[0]).sum() * f, rel=1e-12)
    assert float(s.grad) == pytest.approx((wn * t[3]).sum() * f, rel=1e-9)
    assert float(gg.grad) == pytest.approx((wn * t[5]).sum() * f, rel=1e-9)
    assert float(aa.grad) == pytest.approx((wn * t[7]).sum() * f, rel=1e-9)
    assert float(aa.grad) < 0          # more absorption -> less transmission
    # more extinction -> less transmission under the cloud
    assert float(s.grad) < 0
