"""Pins of the guide oracle: bfloat16 rounding, the vMF density and sampler,
the mixture log-likelihood gradient and the MLP backward pass (finite
differences), the one-sample MIS weight (unbiasedness) and Adam's first step."""
import math

import numpy as np
import pytest
import torch

from oracle import guide as G


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(10000) * 10 ** rng.uniform(-8, 8, 10000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 65504.0, 1e-40]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(G.bf16_round(x), ref)
    assert G.bf16_round(np.float32(1.0 + 2 ** -8)) == 1.0              # tie to even
    assert G.bf16_round(np.float32(1.0 + 3 * 2 ** -8)) == 1.0 + 2 ** -6


@pytest.mark.parametrize("kappa", [0.05, 1.0, 20.0, 1000.0])
def test_vmf_normalised(kappa):
    # integrate over the cosine t with the azimuth done analytically (2 pi)
    t = np.linspace(-1, 1, 400001)
    mu = np.array([[0.0, 0.0, 1.0]])
    w = np.stack([np.sqrt(1 - t * t), np.zeros_like(t), t], axis=1)
    p = G.vmf_pdf(mu, np.array([kappa]), w)
    integral = np.trapezoid(2 * math.pi * p, t)
    assert integral == pytest.approx(1.0, rel=1e-5)


@pytest.mark.parametrize("kappa", [0.05, 3.0, 500.0])
def test_vmf_sampler_inverts_cosine_cdf(kappa):
    u1 = np.linspace(0.0005, 0.9995, 300)
    u2 = np.full_like(u1, 0.3)
    mu = np.tile(np.array([0.3, -0.4, np.sqrt(1 - 0.25)]), (len(u1), 1))
    d = G.vmf_sample(mu, np.full(len(u1), kappa), u1, u2)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-12)
    t = np.sum(d * mu, axis=1)
    # cosine density is proportional to exp(kappa t) on [-1, 1]; its CDF, written without overflow
    F = np.exp(kappa * (t - 1)) * -np.expm1(-kappa * (t + 1)) / -np.expm1(-2 * kappa)
    assert np.allclose(F, u1, atol=1e-9)


def test_output_gradient_finite_differences():
    rng = np.random.default_rng(2)
    n = 20
    out = rng.standard_normal((n, G.N_OUT))
    w_out = rng.standard_normal((n, 3))
    w_out /= np.linalg.norm(w_out, axis=1, keepdims=True)
    weight = rng.random(n)
    L, g = G.loss_and_grad_out(out, w_out, weight)
    h = 1e-6
    for k in rng.integers(0, n * G.N_OUT, 60):
        i, j = divmod(int(k), G.N_OUT)
        op, om = out.copy(), out.copy()
        op[i, j] += h
        om[i, j] -= h
        fd = (G.loss_and_grad_out(op, w_out, weight)[0] - G.loss_and_grad_out(om, w_out, weight)[0]) / (2 * h)
        assert g[i, j] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def test_parameter_gradient_finite_differences(monkeypatch):
    """The backward pass checked against central differences of the loss,
    with bf16 rounding switched off (it makes the loss piecewise constant)."""
    monkeypatch.setattr(G, "bf16_round", lambda x: np.asarray(x, dtype=np.float64))
    rng = np.random.default_rng(3)
    params = G.init_params(4).astype(np.float64) * 0.5
    n = 16
    X = rng.uniform(-1, 1, (n, G.N_RAW))
    w_out = rng.standard_normal((n, 3))
    w_out /= np.linalg.norm(w_out, axis=1, keepdims=True)
    weight = rng.random(n) + 0.1
    L, grad = G.loss_grad(params, X, w_out, weight)
    h = 1e-6
    for k in rng.integers(0, G.n_params(), 80):
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        fd = (G.loss_grad(pp, X, w_out, weight)[0] - G.loss_grad(pm, X, w_out, weight)[0]) / (2 * h)
        assert grad[k] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_parameter_count():
    # 15 x 64 + 64, 2 x (64 x 64 + 64), 64 x 40 + 40
    assert G.n_params() == 11944


def test_position_features():
    """The Fourier features against identities they must obey: unit circle
    per pair, the double angle between the two frequencies, periodicity of
    1/4 (8 pi) in x and y, and the raw inputs passed through."""
    rng = np.random.default_rng(9)
    X = rng.uniform(-1, 1, (500, G.N_RAW))
    F = G.features(X)
    assert F.shape == (500, 15) and np.array_equal(F[:, :7], X)
    for j in range(4):
        assert np.allclose(F[:, 7 + 2 * j] ** 2 + F[:, 8 + 2 * j] ** 2, 1.0)
    # sin 16 pi x = 2 sin 8 pi x cos 8 pi x, cos 16 pi y = cos^2 8 pi y - sin^2 8 pi y
    assert np.allclose(F[:, 11], 2 * F[:, 7] * F[:, 8])
    assert np.allclose(F[:, 14], F[:, 10] ** 2 - F[:, 9] ** 2)
    Xs = X.copy()
    Xs[:, 0] += 0.25
    Xs[:, 1] -= 0.25
    assert np.allclose(G.features(Xs)[:, 7:], F[:, 7:])
    # x = 1/16: 8 pi x = pi / 2
    Z = np.zeros((1, G.N_RAW))
    Z[0, 0] = 1.0 / 16.0
    assert np.allclose(G.features(Z)[0, 7:], [1, 0, 0, 1, 0, -1, 0, 1], atol=1e-12)


def test_mis_weight_is_unbiased():
    """E over the mixture proposal of weight * f equals E over HG of f."""
    rng = np.random.default_rng(5)
    g, c = 0.85, 0.5
    win = np.array([0.0, 0.0, 1.0])
    mu = np.array([0.6, 0.0, 0.8])
    kappa = 15.0
    f = lambda d: 1.0 + 3.0 * d[:, 0] ** 2 + d[:, 1]     # any bounded function of the direction

    def hg_pdf(cos):
        return (1 - g * g) / (4 * math.pi * (1 + g * g - 2 * g * cos) ** 1.5)

    def hg_sample(n):
        xi = rng.random(n)
        s = (1 - g * g) / (1 - g + 2 * g * xi)
        t = (1 + g * g - s * s) / (2 * g)
        ph = 2 * math.pi * rng.random(n)
        st = np.sqrt(np.maximum(0, 1 - t * t))
        return np.stack([st * np.cos(ph), st * np.sin(ph), t], axis=1)

    n = 400000
    ref = f(hg_sample(n)).mean()
    pick = rng.random(n) < c
    d = hg_sample(n)
    dv = G.vmf_sample(np.tile(mu, (n, 1)), np.full(n, kappa), rng.random(n), rng.random(n))
    d[pick] = dv[pick]
    p = hg_pdf(d @ win)
    q = G.vmf_pdf(mu[None, :], np.array([kappa]), d)
    est = G.mis_weight(p, q, c) * f(d)
    se = math.sqrt(est.var() / n + f(hg_sample(n)).var() / n)
    assert abs(est.mean() - ref) < 3 * se


def test_adam_first_step_is_signed_lr():
    p = np.array([1.0, -2.0, 3.0], dtype=np.float32)
    g = np.array([0.5, -1e-3, 2.0])
    out, m, v = G.adam_step(p, np.zeros(3), np.zeros(3), g, 1, 0.01)
    assert np.allclose(out, p - 0.01 * np.sign(g), atol=1e-6)
