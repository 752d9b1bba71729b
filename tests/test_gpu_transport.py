"""Null-collision estimators on the GPU: closed forms (Beer-Lambert, pure
absorber over a Lambertian ground, single scattering), majorant invariance,
counter expectations and image parity with the oracle."""
import math

import numpy as np
import pytest
import torch

import oracle
from gpu_common import ctx, device_field
from paper_1902_01137_amd import _lib, api, inputs
from paper_1902_01137_amd.inputs import Camera, GridParams, Optics, Sampling
from stats import block, compare, mean_se, vs_exact

pytestmark = pytest.mark.gpu


def _trans(desc, k, tau_tilde, kg, rays, spp, m=1.0, seed=77, counters=None):
    c = ctx()
    kd = device_field(k)
    g = api.build_grid(c, kd, desc, GridParams(tau_tilde, kg, 0))
    s, s2 = api.transmittance(c, g, kd, Optics(majorant_scale=m), torch.from_numpy(rays).cuda(),
                              Sampling(seed=seed, spp=spp), counters)
    torch.cuda.synchronize()
    return s.cpu().numpy() / spp


@pytest.mark.parametrize("tau_tilde", [0.0, 1.0, math.inf])
@pytest.mark.parametrize("m", [1.0, 2.0])
def test_beer_lambert_slab(tau_tilde, m):
    desc, k = inputs.slab_field([0.7, 2.5, 0.0, 1.2], 0.5)
    kg = 0.05
    mus = np.array([1.0, 0.8, 0.5, 0.3])
    rays = np.zeros((len(mus), 6), np.float32)
    rays[:, 2] = 2.0 + 0.25
    rays[:, 3] = np.sqrt(1 - mus ** 2)
    rays[:, 5] = -mus
    spp = 200000
    T = _trans(desc, k, tau_tilde, kg, rays, spp, m)
    tau = (0.7 + 2.5 + 0.0 + 1.2 + 4 * kg) * 0.5
    exact = np.exp(-tau / mus)
    se = np.sqrt(exact * (1 - exact) / spp)
    res = vs_exact(T, se, exact)
    assert res["ok"], res


def test_majorant_invariance_blob():
    desc, k = inputs.lognormal_blob()
    rays = inputs.random_rays(desc, 64, seed=41, inside_frac=0.6, axis_frac=0.0)
    exact, _, _ = oracle.transmittance(oracle.make_field(desc, k, 0.0), rays, 1, 0, mode=0)
    spp = 40000
    se = np.sqrt(np.maximum(exact * (1 - exact), 1e-5) / spp)
    for tt in (0.0, 1.0, 10.0, math.inf):
        for m in (1.0, 2.0, 10.0):
            T = _trans(desc, k, tt, 0.0, rays, spp, m)
            res = vs_exact(T, se, exact)
            assert res["ok"], (tt, m, res)


def count_z(g_total, n_g, o_total, o_sq, n_o):
    """z of the per-path mean of an event count, GPU against oracle; both
    sample the same distribution of paths, whose per-path variance the
    oracle's sum of squares estimates."""
    om = o_total / n_o
    var = max(o_sq / n_o - om * om, 0.0) * n_o / (n_o - 1)
    se = math.sqrt(var / n_g + var / n_o)
    d = g_total / n_g - om
    return d / se if se > 0 else (0.0 if d == 0 else math.inf)


def test_counter_expectations_match_oracle():
    """E[tentative], E[null] and E[voxel visits] per transmissivity path are
    properties of the algorithm: GPU and oracle must agree within 3 standard
    errors."""
    desc, k = inputs.lognormal_blob()
    rays = inputs.random_rays(desc, 16, seed=42, inside_frac=0.5, axis_frac=0.0)
    spp = 20000
    cnt = api.new_counters("cuda")
    _trans(desc, k, 1.0, 0.02, rays, spp, 2.0, counters=cnt)
    gc = api.counters_dict(cnt)
    og = oracle.OracleGrid(desc, k, tau_tilde=1.0, k_gas=0.02)
    _, _, oc, osq = og.transmittance(rays, spp, seed=5, mode=2, majorant_scale=2.0, with_sq=True)
    n = len(rays) * spp
    assert gc["paths"] == n
    for i, name in enumerate(("tentative", "nulls", "leaf_visits")):
        z = count_z(gc[name], n, float(oc[i]), float(osq[i]), n)
        assert abs(z) < 3.0, (name, gc[name] / n, oc[i] / n, z)


@pytest.mark.parametrize("m", [1.0, 2.0])
def test_render_counters_match_oracle(m):
    """The renderer with delta-tracked sun rays: tentative collisions, nulls
    and voxels entered per path (camera, scattered and sun rays together)
    against the oracle's delta-tracked render over the same grid, within 3
    standard errors; the image too."""
    sc = inputs.scene_small()
    op = Optics(**{**vars(sc.optics), "majorant_scale": m})
    spp_g, spp_o = 64, 16
    cnt = api.new_counters("cuda")
    s, s2 = _render(sc.desc, sc.kc, sc.grid.k_gas, sc.grid.tau_tilde, op, sc.camera, spp_g, seed=1031,
                    counters=cnt)
    gc = api.counters_dict(cnt)
    og = oracle.OracleGrid(sc.desc, sc.kc, tau_tilde=sc.grid.tau_tilde, k_gas=sc.grid.k_gas)
    os_, os2, st = oracle.render_tracked(sc.desc, sc.kc, sc.grid.k_gas, op, sc.camera, spp_o,
                                         inputs.SEED_ORACLE_BASE + 31, og)
    n_g, n_o = 64 * 64 * spp_g, 64 * 64 * spp_o
    assert gc["paths"] == n_g and gc["truncated"] == 0
    for i, name in enumerate(("tentative", "nulls", "leaf_visits")):
        z = count_z(gc[name], n_g, st[i], st[3 + i], n_o)
        assert abs(z) < 3.0, (name, gc[name] / n_g, st[i] / n_o, z)
    if m > 1.0:
        assert gc["nulls"] > 0
    gm, gse = mean_se(s, s2, spp_g)
    om, ose = mean_se(os_, os2, spp_o)
    res = compare(*block(gm, gse, (64, 64)), *block(om, ose, (64, 64)))
    assert res["ok"], res


def _render(desc, k, kg, tau_tilde, optics, cam, spp, seed=123, counters=None):
    c = ctx()
    kd = device_field(k)
    g = api.build_grid(c, kd, desc, GridParams(tau_tilde, kg, 0))
    s, s2 = api.render(c, g, kd, optics, cam, Sampling(seed=seed, spp=spp), counters=counters)
    torch.cuda.synchronize()
    return s.cpu().numpy().ravel(), s2.cpu().numpy().ravel()


def _slab_camera(mu, z_top, n=4):
    s = math.sqrt(1 - mu * mu)
    pos = (0.0, 0.0, z_top + 0.5)
    return Camera(type=1, pos=pos, target=(pos[0] + s, pos[1], pos[2] - mu), up=(0.0, 0.0, 1.0),
                  ortho_w=0.1, ortho_h=0.1, width=n, height=n)


@pytest.mark.parametrize("tau_tilde", [0.0, math.inf])
def test_pure_absorber_over_lambertian_ground(tau_tilde):
    tau, H, rho, mu, th0 = 0.8, 0.4, 0.3, 0.7, 40.0
    desc, k = inputs.slab_field([tau / H], H)
    op = Optics(ssa=0.0, g=0.85, ground_albedo=rho, sun_zenith_deg=th0, sun_azimuth_deg=25.0)
    spp = 50000
    s, s2 = _render(desc, k, 0.0, tau_tilde, op, _slab_camera(mu, H), spp)
    mu0 = math.cos(math.radians(th0))
    cst = rho / math.pi * mu0 * math.exp(-tau / mu0)
    p = math.exp(-tau / mu) * math.exp(-tau / mu0)   # delta-tracked sun ray: Bernoulli too
    exact = rho / math.pi * mu0 * math.exp(-tau / mu0) * math.exp(-tau / mu)
    se = rho / math.pi * mu0 * math.sqrt(p * (1 - p) / spp)
    m = s / spp
    res = vs_exact(m, se, exact)
    assert res["ok"], (res, cst)


def test_single_scattering_slab():
    tau, H, ssa, g, mu, th0, phi0 = 1.3, 0.5, 0.9, 0.6, 0.55, 35.0, 60.0
    desc, k = inputs.slab_field([tau / H], H)
    op = Optics(ssa=ssa, g=g, ground_albedo=0.0, sun_zenith_deg=th0, sun_azimuth_deg=phi0, max_scatter=1)
    spp = 100000
    s, s2 = _render(desc, k, 0.0, 1.0, op, _slab_camera(mu, H), spp)
    mu0 = math.cos(math.radians(th0))
    sv = np.array([math.sin(math.radians(th0)) * math.cos(math.radians(phi0)),
                   math.sin(math.radians(th0)) * math.sin(math.radians(phi0)), mu0])
    d = np.array([math.sqrt(1 - mu * mu), 0.0, -mu])
    cosT = float(d @ sv)
    p = (1 - g * g) / (4 * math.pi * (1 + g * g - 2 * g * cosT) ** 1.5)
    exact = ssa * p * mu0 / (mu0 + mu) * (1 - math.exp(-tau * (1 / mu0 + 1 / mu)))
    m, se = mean_se(s, s2, spp)
    res = vs_exact(m, se, exact)
    assert res["ok"], res


def test_small_cloud_image_vs_oracle():
    sc = inputs.scene_small()
    spp_g, spp_o = 256, 128
    cnt = api.new_counters("cuda")
    s, s2 = _render(sc.desc, sc.kc, sc.grid.k_gas, sc.grid.tau_tilde, sc.optics, sc.camera, spp_g, seed=1001,
                    counters=cnt)
    os_, os2, _ = oracle.render(sc.desc, sc.kc, sc.grid.k_gas, sc.optics, sc.camera, spp_o, inputs.SEED_ORACLE_BASE + 1)
    gm, gse = mean_se(s, s2, spp_g)
    om, ose = mean_se(os_, os2, spp_o)
    res = compare(*block(gm, gse, (64, 64)), *block(om, ose, (64, 64)))
    assert res["ok"], res
    res_px = compare(gm, gse, om, ose)
    assert res_px["ok"], res_px
    c = api.counters_dict(cnt)
    assert c["paths"] == 64 * 64 * spp_g and c["truncated"] == 0


def test_small_cloud_majorant_and_grid_invariance():
    sc = inputs.scene_small()
    spp = 128
    ref = _render(sc.desc, sc.kc, 0.0, 1.0, sc.optics, sc.camera, spp, seed=5)
    rm, rse = mean_se(*ref, spp)
    for tt, m in ((0.0, 1.0), (math.inf, 1.0), (10.0, 3.0)):
        op = inputs.Optics(**{**vars(sc.optics), "majorant_scale": m})
        s, s2 = _render(sc.desc, sc.kc, 0.0, tt, op, sc.camera, spp, seed=6 + int(m))
        gm, gse = mean_se(s, s2, spp)
        res = compare(*block(gm, gse, (64, 64)), *block(rm, rse, (64, 64)))
        assert res["ok"], (tt, m, res)


def test_small_cloud_flat_supercell_grid():
    """The flat grid of 8^3-cell supercells is a valid majorant: same image."""
    sc = inputs.scene_small()
    spp = 128
    rm, rse = mean_se(*_render(sc.desc, sc.kc, 0.0, 1.0, sc.optics, sc.camera, spp, seed=5), spp)
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, GridParams(0.0, 0.0, 2, 3))
    s, s2 = api.render(c, g, kd, sc.optics, sc.camera, Sampling(seed=61, spp=spp))
    torch.cuda.synchronize()
    gm, gse = mean_se(s.cpu().numpy().ravel(), s2.cpu().numpy().ravel(), spp)
    res = compare(*block(gm, gse, (64, 64)), *block(rm, rse, (64, 64)))
    assert res["ok"], res


def test_cumulus_layered_grid_image_equals_hierarchy():
    """The layered grid is a valid majorant: a small cumulus view rendered
    over it agrees with the same view over the hierarchical grid (whose
    images are checked against the oracle above) within 3 combined standard
    errors per 8x8 block."""
    desc, k = inputs.cumulus_field(fine=(80, 256, 256), pool=2)
    (xa, xb), (ya, yb), (za, zb) = desc.box
    cam = inputs.Camera(type=0, pos=(xa - 1.5, (ya + yb) / 2, 1.5), target=((xa + xb) / 2, (ya + yb) / 2, 0.75),
                        up=(0.0, 0.0, 1.0), fov_y_deg=50.0, width=64, height=64)
    op = inputs.Optics(ssa=0.999, g=0.86, ground_albedo=0.2, sun_zenith_deg=45.0, sun_azimuth_deg=0.0)
    c = ctx()
    kd = device_field(k)
    spp = 256
    out = {}
    for name, gp in (("hier", GridParams(1.0, 0.05, 0)), ("layered", GridParams(0.0, 0.05, 3, 1))):
        g = api.build_grid(c, kd, desc, gp)
        cnt = api.new_counters("cuda")
        s, s2 = api.render(c, g, kd, op, cam, Sampling(seed=71 if name == "hier" else 72, spp=spp), counters=cnt)
        torch.cuda.synchronize()
        out[name] = mean_se(s.cpu().numpy().ravel(), s2.cpu().numpy().ravel(), spp)
        assert api.counters_dict(cnt)["truncated"] == 0
    res = compare(*block(*out["layered"], (64, 64)), *block(*out["hier"], (64, 64)))
    assert res["ok"], res


def test_resume_with_sample_offset():
    sc = inputs.scene_small()
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    s_full, q_full = api.render(c, g, kd, sc.optics, sc.camera, Sampling(seed=9, spp=8))
    s_a, q_a = api.render(c, g, kd, sc.optics, sc.camera, Sampling(seed=9, spp=4))
    api.render(c, g, kd, sc.optics, sc.camera, Sampling(seed=9, spp=4, sample_offset=4), s_a, q_a)
    torch.cuda.synchronize()
    assert torch.allclose(s_full, s_a, rtol=1e-12, atol=1e-12)
    assert torch.allclose(q_full, q_a, rtol=1e-12, atol=1e-12)


def _sensor(desc, n, z=0.0):
    (xa, xb), (ya, yb), _ = desc.box
    c = ((xa + xb) / 2, (ya + yb) / 2, z)
    return Camera(type=2, pos=c, target=(c[0], c[1], z + 1.0), up=(0.0, 1.0, 0.0), ortho_w=xb - xa, ortho_h=yb - ya,
                  width=n, height=n)


def test_sensor_pure_absorber_slab():
    """Irradiance sensor under an absorbing slab: S times Bernoulli(exp(-tau/mu0))."""
    tau, H, th0 = 0.8, 0.4, 40.0
    desc, k = inputs.slab_field([tau / H], H)
    op = Optics(ssa=0.0, g=0.85, ground_albedo=0.5, sun_zenith_deg=th0, sun_azimuth_deg=10.0, sun_irradiance=2.0)
    cam = Camera(type=2, pos=(0.0, 0.0, 0.0), ortho_w=0.1, ortho_h=0.1, width=4, height=4)
    spp = 4096
    s, s2 = _render(desc, k, 0.0, 1.0, op, cam, spp, seed=71)
    p = math.exp(-tau / math.cos(math.radians(th0)))
    se = 2.0 * math.sqrt(p * (1 - p) / spp)
    res = vs_exact(s / spp, se, 2.0 * p)
    assert res["ok"], res
    assert np.allclose(s2, 2.0 * s)        # every path is 0 or S


def test_sensor_image_vs_oracle():
    sc = inputs.scene_small()
    cam = _sensor(sc.desc, 8)
    spp_g, spp_o = 16384, 4096
    s, s2 = _render(sc.desc, sc.kc, sc.grid.k_gas, 1.0, sc.optics, cam, spp_g, seed=72)
    os_, os2, _ = oracle.render(sc.desc, sc.kc, sc.grid.k_gas, sc.optics, cam, spp_o, inputs.SEED_ORACLE_BASE + 72)
    res = compare(*mean_se(s, s2, spp_g), *mean_se(os_, os2, spp_o))
    assert res["ok"], res


def test_sensor_reciprocity_with_forward_flux():
    """The cylinder cumulus (sun at zenith, black ground): backward sensor
    paths and forward photons (nc_flux) give the same ground transmissivity."""
    sc = inputs.scene_cylinder()
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    n, N, spp = 16, 1 << 23, 8192
    tally, glob = api.flux(c, g, kd, sc.optics, (n, n), N, Sampling(seed=73, spp=1))
    s, s2 = api.render(c, g, kd, sc.optics, _sensor(sc.desc, n), Sampling(seed=74, spp=spp))
    torch.cuda.synchronize()
    t = tally.cpu().numpy()
    Tf = t[0] * n * n / N
    sef = np.sqrt(np.maximum(t[1] * (n * n) ** 2 / N - Tf ** 2, 0) / (N - 1))
    mb, seb = mean_se(s.cpu().numpy().ravel(), s2.cpu().numpy().ravel(), spp)
    res = compare(mb, seb, Tf.ravel(), sef.ravel())
    assert res["ok"], res
    assert 0.05 < Tf.mean() < 1.0


# ---------------------------------------------------------------- sun-ray estimators (decomposition tracking)

def _trans_est(desc, k, tau_tilde, kg, rays, spp, m, est, seed=77):
    c = ctx()
    kd = device_field(k)
    g = api.build_grid(c, kd, desc, GridParams(tau_tilde, kg, 0))
    s, s2 = api.transmittance(c, g, kd, Optics(majorant_scale=m), torch.from_numpy(rays).cuda(),
                              Sampling(seed=seed, spp=spp, flags=est))
    torch.cuda.synchronize()
    return mean_se(s.cpu().numpy(), s2.cpu().numpy(), spp)


def _slab_rays():
    mus = np.array([1.0, 0.8, 0.5, 0.3])
    rays = np.zeros((len(mus), 6), np.float32)
    rays[:, 2] = 2.0 + 0.25
    rays[:, 3] = np.sqrt(1 - mus ** 2)
    rays[:, 5] = -mus
    return mus, rays


@pytest.mark.parametrize("est", [_lib.NC_SUN_RATIO, _lib.NC_SUN_RESIDUAL])
@pytest.mark.parametrize("tau_tilde,m", [(0.0, 1.0), (0.0, 2.0), (math.inf, 1.0), (1.0, 3.0)])
def test_ratio_estimators_beer_lambert(est, tau_tilde, m):
    desc, k = inputs.slab_field([0.7, 2.5, 0.0, 1.2], 0.5)
    kg = 0.05
    mus, rays = _slab_rays()
    spp = 100000
    mean, se = _trans_est(desc, k, tau_tilde, kg, rays, spp, m, est)
    tau = (0.7 + 2.5 + 0.0 + 1.2 + 4 * kg) * 0.5
    exact = np.exp(-tau / mus)
    # float32 optical depths: ~1e-6 relative, added to the statistical error
    res = vs_exact(mean, np.hypot(se, 1e-6 * exact), exact)
    assert res["ok"], res
    # below the Bernoulli spread of delta tracking
    assert np.all(se <= np.sqrt(exact * (1 - exact) / spp) * 1.02), (se, exact)


def test_residual_ratio_is_exact_in_homogeneous_voxels():
    """Each layer is one voxel whose minimum equals its maximum: with
    majorant scale 1 the residual majorant vanishes and every path returns
    exp(-tau) (up to float32 rounding), so the spread is nil."""
    desc, k = inputs.slab_field([0.3, 0.6, 0.0, 0.4], 0.5)
    mus, rays = _slab_rays()
    spp = 64
    mean, se = _trans_est(desc, k, 0.0, 0.05, rays, spp, 1.0, _lib.NC_SUN_RESIDUAL)
    exact = np.exp(-(0.3 + 0.6 + 0.4 + 4 * 0.05) * 0.5 / mus)
    # Russian roulette acts only below 0.1; these transmissivities are above it except the grazing ray
    sel = exact > 0.1
    assert np.allclose(mean[sel], exact[sel], rtol=2e-5)
    assert np.all(se[sel] < 1e-6)


@pytest.mark.parametrize("est", [_lib.NC_SUN_RATIO, _lib.NC_SUN_RESIDUAL])
def test_ratio_estimators_majorant_invariance_blob(est):
    desc, k = inputs.lognormal_blob()
    rays = inputs.random_rays(desc, 64, seed=43, inside_frac=0.6, axis_frac=0.0)
    exact, _, _ = oracle.transmittance(oracle.make_field(desc, k, 0.0), rays, 1, 0, mode=0)
    spp = 40000
    for tt in (0.0, 1.0, math.inf):
        for m in (1.0, 2.0):
            mean, se = _trans_est(desc, k, tt, 0.0, rays, spp, m, est)
            # rays through thick cloud may see no surviving sample (estimates
            # are 0 or >= the roulette threshold), so the spread gets the same
            # floor as the Bernoulli case; float32 optical depths add ~1e-6
            res = vs_exact(mean, np.hypot(np.maximum(se, np.sqrt(1e-5 / spp)), 1e-5 * exact), exact)
            assert res["ok"], (tt, m, res)


@pytest.mark.parametrize("est", [_lib.NC_SUN_RATIO, _lib.NC_SUN_RESIDUAL])
def test_small_cloud_image_ratio_estimators_vs_oracle(est):
    sc = inputs.scene_small()
    spp_g, spp_o = 256, 128
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    s, s2 = api.render(c, g, kd, sc.optics, sc.camera, Sampling(seed=1009 + est, spp=spp_g, flags=est))
    d, d2 = api.render(c, g, kd, sc.optics, sc.camera, Sampling(seed=1019, spp=spp_g))
    torch.cuda.synchronize()
    os_, os2, _ = oracle.render(sc.desc, sc.kc, sc.grid.k_gas, sc.optics, sc.camera, spp_o, inputs.SEED_ORACLE_BASE + 1)
    gm, gse = mean_se(s.cpu().numpy().ravel(), s2.cpu().numpy().ravel(), spp_g)
    om, ose = mean_se(os_, os2, spp_o)
    res = compare(*block(gm, gse, (64, 64)), *block(om, ose, (64, 64)))
    assert res["ok"], res
    dm, dse = mean_se(d.cpu().numpy().ravel(), d2.cpu().numpy().ravel(), spp_g)
    assert (gse ** 2).sum() < (dse ** 2).sum()      # the sun estimate is smoother than delta tracking


def test_unknown_sun_estimator_is_rejected():
    sc = inputs.scene_small()
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    with pytest.raises(_lib.NcError) as e:
        api.render(c, g, kd, sc.optics, sc.camera, Sampling(seed=1, spp=1, flags=3))
    assert e.value.status == _lib.NC_ERR_INVALID_ARG


# ---------------------------------------------------------------- the solar disc (Section 4.1's solar cone)

def _cone_mean(tau, alpha_deg):
    """E over w uniform in a cone of half-angle alpha about the zenith of
    gain w_z exp(-tau / w_z), gain = 2 / (1 + cos alpha) (cap quadrature)."""
    from scipy import integrate
    ca = math.cos(math.radians(alpha_deg))
    val, _ = integrate.quad(lambda m: m * math.exp(-tau / m), ca, 1.0, epsabs=1e-14, epsrel=1e-12)
    return 2.0 / (1.0 + ca) * val / (1.0 - ca)


@pytest.mark.parametrize("alpha", [0.265, 10.0, 30.0])
def test_disc_sun_over_lambertian_ground(alpha):
    """Pure absorber over a Lambertian ground, zenith sun disc: the ground's
    local estimate averages the cap integral (delta-tracked sun rays)."""
    tau, H, rho, mu = 0.8, 0.4, 0.3, 0.7
    desc, k = inputs.slab_field([tau / H], H)
    op = Optics(ssa=0.0, g=0.85, ground_albedo=rho, sun_zenith_deg=0.0, sun_half_angle_deg=alpha)
    spp = 50000
    s, s2 = _render(desc, k, 0.0, 1.0, op, _slab_camera(mu, H), spp, seed=77)
    exact = rho / math.pi * _cone_mean(tau, alpha) * math.exp(-tau / mu)
    m, se = mean_se(s, s2, spp)
    res = vs_exact(m, se, exact)
    assert res["ok"], res


def test_disc_sun_seen_by_the_camera():
    """Looking straight up at a zenith disc through a pure absorber:
    S / (pi sin^2 alpha) exp(-tau); looking 2 alpha away: nothing."""
    tau, H, alpha = 0.5, 0.4, 4.0
    desc, k = inputs.slab_field([tau / H], H)
    op = Optics(ssa=0.0, g=0.85, ground_albedo=0.0, sun_zenith_deg=0.0, sun_half_angle_deg=alpha, sun_irradiance=1.5)
    Ls = 1.5 / (math.pi * math.sin(math.radians(alpha)) ** 2)
    spp = 20000
    up = Camera(type=1, pos=(0.0, 0.0, -0.2), target=(0.0, 0.0, 1.0), up=(0.0, 1.0, 0.0), ortho_w=0.1, ortho_h=0.1,
                width=4, height=4)
    s, s2 = _render(desc, k, 0.0, 1.0, op, up, spp, seed=78)
    p = math.exp(-tau)
    se = Ls * math.sqrt(p * (1 - p) / spp)
    res = vs_exact(s / spp, se, Ls * p)
    assert res["ok"], res
    t = math.radians(2 * alpha)
    off = Camera(type=1, pos=(0.0, 0.0, -0.2), target=(math.sin(t), 0.0, -0.2 + math.cos(t)), up=(0.0, 1.0, 0.0),
                 ortho_w=0.1, ortho_h=0.1, width=4, height=4)
    s, _ = _render(desc, k, 0.0, 1.0, op, off, 512, seed=79)
    assert np.all(s == 0.0)


def test_disc_sun_sensor():
    """Irradiance sensor under a pure absorber, zenith disc: the direct
    term's mean is S times the cap integral."""
    tau, H, alpha = 0.8, 0.4, 20.0
    desc, k = inputs.slab_field([tau / H], H)
    op = Optics(ssa=0.0, g=0.85, ground_albedo=0.0, sun_zenith_deg=0.0, sun_half_angle_deg=alpha, sun_irradiance=2.0)
    cam = Camera(type=2, pos=(0.0, 0.0, 0.0), target=(0.0, 0.0, 1.0), up=(0.0, 1.0, 0.0), ortho_w=0.1, ortho_h=0.1,
                 width=4, height=4)
    spp = 20000
    s, s2 = _render(desc, k, 0.0, 1.0, op, cam, spp, seed=80)
    m, se = mean_se(s, s2, spp)
    exact = 2.0 * _cone_mean(tau, alpha)
    res = vs_exact(m, se, exact)
    assert res["ok"], res


def test_small_cloud_disc_sun_vs_oracle():
    """A 5-degree disc on the small cloud scene (nadir view: the disc enters
    through the local estimates at every event): GPU image against the
    oracle's."""
    sc = inputs.scene_small()
    op = Optics(**{**vars(sc.optics), "sun_half_angle_deg": 5.0})
    spp_g, spp_o = 256, 128
    s, s2 = _render(sc.desc, sc.kc, sc.grid.k_gas, sc.grid.tau_tilde, op, sc.camera, spp_g, seed=1011)
    os_, os2, _ = oracle.render(sc.desc, sc.kc, sc.grid.k_gas, op, sc.camera, spp_o, inputs.SEED_ORACLE_BASE + 11)
    gm, gse = mean_se(s, s2, spp_g)
    om, ose = mean_se(os_, os2, spp_o)
    res = compare(*block(gm, gse, (64, 64)), *block(om, ose, (64, 64)))
    assert res["ok"], res
    res_px = compare(gm, gse, om, ose)
    assert res_px["ok"], res_px


def test_disc_sun_argument_checks():
    sc = inputs.scene_small()
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    for bad in (-1.0, 90.0, float("nan")):
        op = Optics(**{**vars(sc.optics), "sun_half_angle_deg": bad})
        with pytest.raises(_lib.NcError) as e:
            api.render(c, g, kd, op, sc.camera, Sampling(seed=1, spp=1))
        assert e.value.status == _lib.NC_ERR_RANGE
    op = Optics(**{**vars(sc.optics), "sun_half_angle_deg": 1.0})
    with pytest.raises(_lib.NcError) as e:
        api.flux(c, g, kd, op, (4, 4), 1000, Sampling(seed=1, spp=1))
    assert e.value.status == _lib.NC_ERR_UNSUPPORTED
    sensor = Camera(type=2, pos=(0.0, 0.0, 0.0), target=(0.0, 0.0, 1.0), up=(0.0, 1.0, 0.0), ortho_w=0.1, ortho_h=0.1,
                    width=2, height=2)
    op = Optics(**{**vars(sc.optics), "sun_zenith_deg": 80.0, "sun_half_angle_deg": 15.0})
    with pytest.raises(_lib.NcError) as e:
        api.render(c, g, kd, op, sensor, Sampling(seed=1, spp=1))
    assert e.value.status == _lib.NC_ERR_RANGE


# ---------------------------------------------------------------- k-distribution (spectral quadrature)

def test_kdistribution_gas_slab_closed_form():
    """Gas-only slab over a Lambertian ground, 4 quadrature points drawn per
    path, one grid shared by all (built with the largest point's k_gas)."""
    H, rho, mu, th0 = 0.6, 0.4, 0.8, 30.0
    desc, k = inputs.slab_field([0.0], H)
    w = np.array([0.1, 0.4, 0.3, 0.2])
    kg = np.array([0.05, 0.4, 1.3, 3.0])
    op = Optics(ssa=0.5, g=0.85, ground_albedo=rho, sun_zenith_deg=th0, kdist=(w, kg))
    spp = 100000
    s, s2 = _render(desc, k, 3.0, 1.0, op, _slab_camera(mu, H), spp, seed=93)
    mu0 = math.cos(math.radians(th0))
    exact = float((w * rho / math.pi * mu0 * np.exp(-kg * H / mu0) * np.exp(-kg * H / mu)).sum())
    m, se = mean_se(s, s2, spp)
    res = vs_exact(m, se, exact)
    assert res["ok"], res


def test_small_cloud_kdistribution_vs_oracle():
    """The small cloud with an 8-point synthetic k-distribution of the gas
    (0.001 .. 1 km^-1): GPU image (shared grid at the largest k_gas) against
    the oracle's."""
    sc = inputs.scene_small()
    kd = inputs.kdist_synthetic()
    op = Optics(**{**vars(sc.optics), "kdist": kd})
    spp_g, spp_o = 256, 128
    s, s2 = _render(sc.desc, sc.kc, float(kd[1].max()), sc.grid.tau_tilde, op, sc.camera, spp_g, seed=1021)
    os_, os2, _ = oracle.render(sc.desc, sc.kc, 0.0, op, sc.camera, spp_o, inputs.SEED_ORACLE_BASE + 21)
    gm, gse = mean_se(s, s2, spp_g)
    om, ose = mean_se(os_, os2, spp_o)
    res = compare(*block(gm, gse, (64, 64)), *block(om, ose, (64, 64)))
    assert res["ok"], res
    res_px = compare(gm, gse, om, ose)
    assert res_px["ok"], res_px


def test_kdistribution_argument_checks():
    sc = inputs.scene_small()
    c = ctx()
    kd_ = device_field(sc.kc)
    g = api.build_grid(c, kd_, sc.desc, GridParams(1.0, 0.5, 0))
    ok = (np.array([0.5, 0.5]), np.array([0.1, 0.5]))
    api.render(c, g, kd_, Optics(**{**vars(sc.optics), "kdist": ok}), sc.camera, Sampling(seed=1, spp=1))
    for bad, status in (((np.array([0.5, 0.5]), np.array([0.1, 0.6])), _lib.NC_ERR_RANGE),    # above the grid's k_gas
                        ((np.array([0.0, 0.0]), np.array([0.1, 0.2])), _lib.NC_ERR_RANGE),
                        ((np.array([1.0, -1.0]), np.array([0.1, 0.2])), _lib.NC_ERR_RANGE)):
        with pytest.raises(_lib.NcError) as e:
            api.render(c, g, kd_, Optics(**{**vars(sc.optics), "kdist": bad}), sc.camera, Sampling(seed=1, spp=1))
        assert e.value.status == status
    op = Optics(**{**vars(sc.optics), "kdist": ok})
    with pytest.raises(_lib.NcError) as e:
        api.flux(c, g, kd_, op, (4, 4), 1000, Sampling(seed=1, spp=1))
    assert e.value.status == _lib.NC_ERR_UNSUPPORTED
