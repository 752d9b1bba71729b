"""The tabulated phase function on the GPU (Section 4.1's Mie tables, here
a synthetic two-term HG table): its sampler and values against the oracle's,
the single-scattering slab closed form, images against the oracle (plain and
guided), and argument checks."""
import math

import numpy as np
import pytest
import torch

import oracle
from gpu_common import ctx, device_field
from paper_1902_01137_amd import _lib, api, inputs
from paper_1902_01137_amd.inputs import Camera, GridParams, Optics, Sampling
from stats import block, compare, mean_se

pytestmark = pytest.mark.gpu


def test_sampler_and_values_match_the_oracle():
    c = ctx()
    mu, p = inputs.phase_table_tthg()
    tab = api.PhaseTable(c, mu, p)
    u = np.concatenate([np.linspace(0.0, 0.999999, 2001), np.random.default_rng(1).random(2000)]).astype(np.float32)
    out = tab.sample(torch.from_numpy(u).cuda()).cpu().numpy().astype(np.float64)
    ref_mu = np.array([oracle.tab_sample(mu, p, float(x)) for x in u])
    ref_p = np.array([oracle.tab_phase(mu, p, m) for m in out[:, 0]])
    assert np.all(np.abs(out[:, 0] - ref_mu) < 2e-4), np.max(np.abs(out[:, 0] - ref_mu))
    assert np.allclose(out[:, 1], ref_p, rtol=2e-4, atol=1e-7)
    assert np.all(out[:, 0] >= -1.0) and np.all(out[:, 0] <= 1.0)


def test_sampled_cosines_follow_the_table():
    """Kolmogorov-Smirnov distance of 2^20 sampled cosines to the table's CDF
    (computed on the host from the oracle's values)."""
    c = ctx()
    mu, p = inputs.phase_table_tthg(n=91)
    tab = api.PhaseTable(c, mu, p)
    n = 1 << 20
    u = torch.rand(n, device="cuda", generator=torch.Generator(device="cuda").manual_seed(3))
    m = np.sort(tab.sample(u)[:, 0].cpu().numpy().astype(np.float64))
    # exact CDF of the piecewise-linear table at the sampled points
    pn = np.array([oracle.tab_phase(mu, p, x) for x in mu])
    seg = 2 * np.pi * 0.5 * (pn[1:] + pn[:-1]) * np.diff(mu)
    cdf_nodes = np.concatenate([[0.0], np.cumsum(seg)])
    i = np.clip(np.searchsorted(mu, m, side="right") - 1, 0, len(mu) - 2)
    x = m - mu[i]
    slope = (pn[i + 1] - pn[i]) / (mu[i + 1] - mu[i])
    F = cdf_nodes[i] + 2 * np.pi * (pn[i] * x + 0.5 * slope * x * x)
    emp = (np.arange(n) + 0.5) / n
    assert np.max(np.abs(F - emp)) < 1.8 / math.sqrt(n)


def _slab_camera(mu, z_top, n=4):
    s = math.sqrt(1 - mu * mu)
    pos = (0.0, 0.0, z_top + 0.5)
    return Camera(type=1, pos=pos, target=(pos[0] + s, pos[1], pos[2] - mu), up=(0.0, 0.0, 1.0),
                  ortho_w=0.1, ortho_h=0.1, width=n, height=n)


def test_tabulated_single_scattering_slab():
    mu_t, p_t = inputs.phase_table_tthg()
    tau, H, ssa, mu, th0, phi0 = 1.3, 0.5, 0.9, 0.55, 35.0, 60.0
    desc, k = inputs.slab_field([tau / H], H)
    op = Optics(ssa=ssa, g=0.0, ground_albedo=0.0, sun_zenith_deg=th0, sun_azimuth_deg=phi0, max_scatter=1,
                phase_table=(mu_t, p_t))
    c = ctx()
    kd = device_field(k)
    g = api.build_grid(c, kd, desc, GridParams(1.0, 0.0, 0))
    spp = 100000
    s, s2 = api.render(c, g, kd, op, _slab_camera(mu, H), Sampling(seed=91, spp=spp))
    torch.cuda.synchronize()
    mu0 = math.cos(math.radians(th0))
    sv = np.array([math.sin(math.radians(th0)) * math.cos(math.radians(phi0)),
                   math.sin(math.radians(th0)) * math.sin(math.radians(phi0)), mu0])
    d = np.array([math.sqrt(1 - mu * mu), 0.0, -mu])
    pv = oracle.tab_phase(mu_t, p_t, float(d @ sv))
    exact = ssa * pv * mu0 / (mu0 + mu) * (1 - math.exp(-tau * (1 / mu0 + 1 / mu)))
    m, se = mean_se(s.cpu().numpy().ravel(), s2.cpu().numpy().ravel(), spp)
    assert np.all(np.abs(m - exact) < 4.5 * se + 1e-4 * exact), (m, exact, se)


@pytest.fixture(scope="module")
def tab_oracle_image():
    sc = inputs.scene_small()
    op = Optics(**{**vars(sc.optics), "phase_table": inputs.phase_table_tthg()})
    spp = 128
    s, s2, _ = oracle.render(sc.desc, sc.kc, sc.grid.k_gas, op, sc.camera, spp, inputs.SEED_ORACLE_BASE + 41)
    return op, mean_se(s, s2, spp)


def test_small_cloud_tabulated_vs_oracle(tab_oracle_image):
    op, (om, ose) = tab_oracle_image
    sc = inputs.scene_small()
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    spp = 256
    s, s2 = api.render(c, g, kd, op, sc.camera, Sampling(seed=4001, spp=spp))
    torch.cuda.synchronize()
    gm, gse = mean_se(s.cpu().numpy().ravel(), s2.cpu().numpy().ravel(), spp)
    res = compare(*block(gm, gse, (64, 64)), *block(om, ose, (64, 64)))
    assert res["ok"], res
    res = compare(gm, gse, om, ose)
    assert res["ok"], res


def test_guided_with_tabulated_phase_is_unbiased(tab_oracle_image):
    """The guided step mixes the network's lobes with the table (its sampler
    and its value in the MIS weight): unbiased against the oracle's plain
    image for a random network."""
    op, (om, ose) = tab_oracle_image
    sc = inputs.scene_small()
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    gd = api.Guide(c, seed=23)
    spp = 256
    s, s2 = api.render_guided(c, g, kd, op, sc.camera, Sampling(seed=4002, spp=spp, guide_frac=0.5, guide_max_order=1),
                              gd)
    torch.cuda.synchronize()
    gm, gse = mean_se(s.cpu().numpy().ravel(), s2.cpu().numpy().ravel(), spp)
    res = compare(*block(gm, gse, (64, 64)), *block(om, ose, (64, 64)))
    assert res["ok"], res


def test_phase_table_argument_checks():
    c = ctx()
    mu, p = inputs.phase_table_tthg(n=21)
    bad = [(mu[1:], p[1:]), (mu[::-1].copy(), p), (mu, -p), (mu, np.zeros_like(p)), (mu[:1], p[:1])]
    for bm, bp in bad:
        with pytest.raises(_lib.NcError) as e:
            api.PhaseTable(c, bm, bp)
        assert e.value.status in (_lib.NC_ERR_RANGE, _lib.NC_ERR_INVALID_ARG)
    sc = inputs.scene_small()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    op = Optics(**{**vars(sc.optics), "phase_table": (mu, p)})
    with pytest.raises(_lib.NcError) as e:
        api.flux(c, g, kd, op, (4, 4), 1000, Sampling(seed=1, spp=1))
    assert e.value.status == _lib.NC_ERR_UNSUPPORTED
