"""Pins of the oracle's forward-photon ground transmissivity and its
sensitivities (Section 5.1; Eq. 3 generalised to scattering paths):
energy conservation, Beer-Lambert, closed-form derivatives, and agreement of
the null-collision score estimator with common-random-number finite
differences of the plain transmissivity."""
import math

import numpy as np
import pytest

from paper_1902_01137_amd.inputs import Optics, slab_field


def _slab(tau, H=0.5, z0=0.3):
    return slab_field([tau / H], H, z0=z0)


def test_terminal_tallies_sum_to_n(orc):
    desc, k = _slab(2.0)
    for ssa, rho in ((0.9, 0.3), (1.0, 1.0), (0.0, 0.5)):
        op = Optics(ssa=ssa, g=0.7, ground_albedo=rho, sun_zenith_deg=30.0)
        n = 4000
        tally, glob = orc.flux(desc, k, 0.0, op, (1, 1), n, seed=3)
        assert glob.sum() == n
        if ssa == 1.0:
            assert glob[3] == 0.0            # no volume absorption
        if ssa == 1.0 and rho == 1.0:
            assert glob[0] == n              # everything escapes upward


@pytest.mark.parametrize("mode", [0, 2])
def test_beer_lambert_transmissivity(orc, mode):
    tau, th0, s = 1.2, 40.0, 1.3
    desc, k = _slab(tau)
    og = orc.OracleGrid(desc, k, tau_tilde=1.0) if mode == 2 else None
    op = Optics(ssa=0.0, g=0.85, ground_albedo=0.0, sun_zenith_deg=th0, majorant_scale=2.0)
    n = 60000
    tally, glob = orc.flux(desc, k, 0.0, op, (1, 1), n, seed=4, mode=mode, kscale=s, grid=og)
    mu0 = math.cos(math.radians(th0))
    exact = math.exp(-s * tau / mu0)
    T = tally[0].sum() / n
    assert abs(T - exact) < 3 * math.sqrt(exact * (1 - exact) / n)
    assert tally[2].sum() == tally[0].sum()          # all direct
    if mode == 2:
        # d/ds exp(-s tau / mu0) = -(tau/mu0) exp(-s tau/mu0)
        d = tally[3].sum() / n
        se = math.sqrt((tally[4].sum() / n - d * d) / n)
        exact_d = -(tau / mu0) * exact
        assert abs(d - exact_d) < 3 * se, (d, exact_d, se)
        assert tally[5].sum() == 0.0                 # no scattering: no g score


def test_fd_matches_closed_form_derivative(orc):
    tau, th0 = 1.2, 40.0
    desc, k = _slab(tau)
    op = Optics(ssa=0.0, g=0.85, ground_albedo=0.0, sun_zenith_deg=th0)
    n = 200000
    out = orc.flux_fd(desc, k, 0.0, op, (1, 1), n, seed=5, which=0, h=1e-2)
    d = out[0].sum() / n
    se = math.sqrt((out[1].sum() / n - d * d) / n)
    mu0 = math.cos(math.radians(th0))
    exact = -(tau / mu0) * math.exp(-tau / mu0)
    assert abs(d - exact) < 3 * se + 1e-3, (d, exact, se)


@pytest.mark.parametrize("which", [0, 1])
def test_score_estimator_matches_crn_fd(orc, which):
    """Scattering slab: the scores along delta-tracked paths and the finite
    differences of exactly-tracked paths estimate the same derivative."""
    tau = 2.0
    desc, k = _slab(tau)
    og = orc.OracleGrid(desc, k, tau_tilde=1.0)
    op = Optics(ssa=0.95, g=0.7, ground_albedo=0.0, sun_zenith_deg=20.0, majorant_scale=2.0)
    n = 100000
    tally, _ = orc.flux(desc, k, 0.0, op, (1, 1), n, seed=6, mode=2, grid=og)
    i = 3 if which == 0 else 5
    ds = tally[i].sum() / n
    se_s = math.sqrt(max(tally[i + 1].sum() / n - ds * ds, 0) / n)
    out = orc.flux_fd(desc, k, 0.0, op, (1, 1), 2 * n, seed=7, which=which, h=1e-3)
    dfd = out[0].sum() / (2 * n)
    se_fd = math.sqrt(max(out[1].sum() / (2 * n) - dfd * dfd, 0) / (2 * n))
    z = (ds - dfd) / math.sqrt(se_s ** 2 + se_fd ** 2)
    assert abs(z) < 3, (ds, se_s, dfd, se_fd)
    assert abs(ds) > 4 * se_s          # a real signal, not two zeros


def test_score_with_gas_matches_fd(orc):
    """With an absorbing gas the local albedo depends on the scale: its score
    term must be included for the estimators to agree."""
    tau = 1.5
    desc, k = _slab(tau)
    kg = 0.8
    og = orc.OracleGrid(desc, k, tau_tilde=1.0, k_gas=kg)
    op = Optics(ssa=1.0, g=0.5, ground_albedo=0.0, sun_zenith_deg=10.0, majorant_scale=2.0)
    n = 100000
    tally, _ = orc.flux(desc, k, kg, op, (1, 1), n, seed=8, mode=2, grid=og)
    ds = tally[3].sum() / n
    se_s = math.sqrt(max(tally[4].sum() / n - ds * ds, 0) / n)
    out = orc.flux_fd(desc, k, kg, op, (1, 1), 2 * n, seed=9, which=0, h=1e-3)
    dfd = out[0].sum() / (2 * n)
    se_fd = math.sqrt(max(out[1].sum() / (2 * n) - dfd * dfd, 0) / (2 * n))
    assert abs(ds - dfd) < 3 * math.sqrt(se_s ** 2 + se_fd ** 2), (ds, se_s, dfd, se_fd)


def test_hg_log_derivative(orc):
    for g in (0.1, 0.6, 0.85, -0.4):
        for mu in (-0.9, 0.0, 0.5, 0.99):
            h = 1e-6
            num = (math.log(orc.hg_phase(g + h, mu)) - math.log(orc.hg_phase(g - h, mu))) / (2 * h)
            assert orc.hg_dlng(g, mu) == pytest.approx(num, rel=1e-6, abs=1e-6)


def test_absorptivity_score_matches_crn_fd(orc):
    """Sensitivity to the droplets' absorptivity alpha = 1 - ssa (Section
    5.1): the score -1/(1 - alpha) per scattering along delta-tracked paths
    against central differences of exactly-tracked paths (the survival draw
    is shared, so the difference only counts the flipped decisions)."""
    tau = 2.0
    desc, k = _slab(tau)
    og = orc.OracleGrid(desc, k, tau_tilde=1.0)
    op = Optics(ssa=0.9, g=0.7, ground_albedo=0.0, sun_zenith_deg=20.0, majorant_scale=2.0)
    n = 100000
    tally, _ = orc.flux(desc, k, 0.0, op, (1, 1), n, seed=16, mode=2, grid=og)
    da = tally[7].sum() / n
    se_a = math.sqrt(max(tally[8].sum() / n - da * da, 0) / n)
    out = orc.flux_fd(desc, k, 0.0, op, (1, 1), 4 * n, seed=17, which=2, h=1e-2)
    dfd = out[0].sum() / (4 * n)
    se_fd = math.sqrt(max(out[1].sum() / (4 * n) - dfd * dfd, 0) / (4 * n))
    z = (da - dfd) / math.sqrt(se_a ** 2 + se_fd ** 2)
    assert abs(z) < 3, (da, se_a, dfd, se_fd)
    assert da < -4 * se_a               # more absorption, less transmission


def test_absorptivity_forward_scattering_closed_form(orc):
    """With an almost delta-forward phase function (g = 0.9999) photons keep
    their direction, so T = exp(-alpha tau / mu0) and
    dT/dalpha = -(tau / mu0) T (up to the tiny angular spread)."""
    tau, th0, alpha = 1.5, 30.0, 0.2
    desc, k = _slab(tau)
    og = orc.OracleGrid(desc, k, tau_tilde=1.0)
    op = Optics(ssa=1.0 - alpha, g=0.9999, ground_albedo=0.0, sun_zenith_deg=th0, majorant_scale=2.0)
    n = 100000
    tally, _ = orc.flux(desc, k, 0.0, op, (1, 1), n, seed=18, mode=2, grid=og)
    mu0 = math.cos(math.radians(th0))
    T_exact = math.exp(-alpha * tau / mu0)
    T = tally[0].sum() / n
    assert abs(T - T_exact) < 3 * math.sqrt(T_exact * (1 - T_exact) / n) + 1e-3
    da = tally[7].sum() / n
    se_a = math.sqrt(max(tally[8].sum() / n - da * da, 0) / n)
    d_exact = -(tau / mu0) * T_exact
    assert abs(da - d_exact) < 3 * se_a + 2e-3, (da, d_exact, se_a)
