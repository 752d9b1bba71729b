"""Oracle of the learned path-guiding proposal (test infrastructure only).

A small MLP maps a scattering vertex (normalised position, incoming
direction, log extinction) to a mixture of von Mises-Fisher lobes over the
outgoing direction.  At a volume scattering event the tracer picks, with
probability c, a direction from the mixture and otherwise from the phase
function (one-sample multiple importance sampling, balance heuristic), and
multiplies the path weight by p_HG / (c q + (1 - c) p_HG).  The network is
fitted to the tracer's own vertices by weighted maximum likelihood.

Everything here is plain numpy in float64 on inputs and weights first
rounded to bfloat16 (the precision the GPU kernels store them in).  This file
shares no code with the HIP path.

Network: 15 -> 64 -> 64 -> 64 -> 8*5, ReLU on the hidden layers.  Its 15
inputs are the vertex's 7 values (position scaled to [-1, 1]^3, incoming
direction, ln(1 + k)) followed by 8 features of the horizontal position,
sin and cos of 8 pi x, 8 pi y, 16 pi x and 16 pi y (a fixed Fourier
encoding, after Tancik et al. 2020, that lets a small MLP resolve the
kilometre-scale structure of a cloud field).  Output lobe j: (logit a_j,
m_j in R^3, log kappa_j); weights pi = softmax(a), mean direction
mu_j = m_j / |m_j|, concentration kappa_j = exp(clamp(s_j)).
"""
from __future__ import annotations

import math

import numpy as np

N_RAW, N_FEAT, WIDTH, DEPTH, N_LOBES = 7, 8, 64, 3, 8
N_IN = N_RAW + N_FEAT
N_OUT = 5 * N_LOBES
LOG_KAPPA_MIN, LOG_KAPPA_MAX = -3.0, 8.0


def bf16_round(x):
    """Round float32 values to bfloat16 (round to nearest even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    nan = np.isnan(a)
    out = np.where(nan, a, out)
    return out.astype(np.float64)


def layer_shapes():
    dims = [N_IN] + [WIDTH] * DEPTH + [N_OUT]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def n_params():
    return sum(o * i + o for o, i in layer_shapes())


def unpack(flat):
    """Flat parameter vector -> list of (W [out, in], b [out])."""
    flat = np.asarray(flat, dtype=np.float64)
    out, k = [], 0
    for o, i in layer_shapes():
        W = flat[k:k + o * i].reshape(o, i)
        k += o * i
        b = flat[k:k + o]
        k += o
        out.append((W, b))
    return out


def init_params(seed):
    """He-uniform weights, zero biases, float32 (the GPU's master copy is float32)."""
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in layer_shapes():
        lim = math.sqrt(6.0 / i)
        parts.append(rng.uniform(-lim, lim, size=o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def features(X):
    """The network's 15 inputs from the vertex's 7 (n, 7) -> (n, 15)."""
    X = np.asarray(X, dtype=np.float64)
    x, y = X[:, 0], X[:, 1]
    enc = [f(math.pi * k * v) for k in (8.0, 16.0) for v in (x, y) for f in (np.sin, np.cos)]
    return np.concatenate([X[:, :N_RAW], np.stack(enc, axis=1)], axis=1)


def forward(params, X):
    """MLP output (n, 40) and the per-layer pre-activations (for backward).

    X: the vertices' 7 inputs.  Weights and the network inputs are rounded to
    bfloat16, hidden activations too (the GPU feeds them to the next bf16
    product); arithmetic is float64."""
    layers = unpack(bf16_round(params))
    h = bf16_round(features(X))
    cache = [h]
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        if li < len(layers) - 1:
            h = bf16_round(np.maximum(z, 0.0))
            cache.append(h)
        else:
            h = z
    return h, cache


def lobes(out):
    """Mixture parameters from raw outputs: (pi [n,8], mu [n,8,3], kappa [n,8], |m| [n,8])."""
    o = out.reshape(-1, N_LOBES, 5)
    a = o[:, :, 0]
    a = a - a.max(axis=1, keepdims=True)
    pi = np.exp(a)
    pi /= pi.sum(axis=1, keepdims=True)
    m = o[:, :, 1:4]
    nm = np.linalg.norm(m, axis=2)
    mu = m / np.maximum(nm, 1e-12)[:, :, None]
    kappa = np.exp(np.clip(o[:, :, 4], LOG_KAPPA_MIN, LOG_KAPPA_MAX))
    return pi, mu, kappa, nm


def vmf_pdf(mu, kappa, w):
    """von Mises-Fisher density on the sphere, per steradian:
    kappa / (2 pi (1 - exp(-2 kappa))) exp(kappa (mu.w - 1))."""
    c = np.sum(mu * w, axis=-1)
    return kappa / (2.0 * math.pi * (-np.expm1(-2.0 * kappa))) * np.exp(kappa * (c - 1.0))


def mixture_pdf(out, w):
    pi, mu, kappa, _ = lobes(out)
    return np.sum(pi * vmf_pdf(mu, kappa, w[:, None, :]), axis=1)


def vmf_sample(mu, kappa, u1, u2):
    """Numerically stable inversion for the cosine (Jakob 2012,
    "Numerically stable sampling of the von Mises-Fisher distribution on
    S^2"): t = 1 + ln(u1 + (1 - u1) exp(-2 kappa)) / kappa, then an azimuth
    2 pi u2 about mu."""
    t = 1.0 + np.log(u1 + (1.0 - u1) * np.exp(-2.0 * kappa)) / kappa
    t = np.clip(t, -1.0, 1.0)
    s = np.sqrt(np.maximum(0.0, 1.0 - t * t))
    # any orthonormal frame about mu
    a = np.where(np.abs(mu[..., 0:1]) < 0.9, np.array([1.0, 0, 0]), np.array([0, 1.0, 0]))
    t1 = np.cross(mu, a)
    t1 /= np.linalg.norm(t1, axis=-1, keepdims=True)
    t2 = np.cross(mu, t1)
    phi = 2.0 * math.pi * u2
    return t[..., None] * mu + s[..., None] * (np.cos(phi)[..., None] * t1 + np.sin(phi)[..., None] * t2)


def mis_weight(p_hg, q, c):
    """One-sample balance-heuristic weight of a direction drawn from the
    mixture c q + (1 - c) p_HG, for an integrand proportional to p_HG."""
    return p_hg / (c * q + (1.0 - c) * p_hg)


def loss_and_grad_out(out, w_out, weight):
    """Weighted negative log-likelihood L = -sum_i w_i ln q_i / sum_i w_i and
    its gradient with respect to the raw network outputs (n, 40)."""
    pi, mu, kappa, nm = lobes(out)
    v = vmf_pdf(mu, kappa, w_out[:, None, :])
    q = np.sum(pi * v, axis=1)
    W = weight.sum()
    L = -np.sum(weight * np.log(q)) / W
    r = pi * v / q[:, None]                                   # responsibilities
    o = out.reshape(-1, N_LOBES, 5)
    g = np.zeros_like(o)
    g[:, :, 0] = r - pi                                       # d ln q / d a
    cosw = np.sum(mu * w_out[:, None, :], axis=2)
    # d ln v / d kappa = 1/kappa - 2 e^{-2k}/(1 - e^{-2k}) + (mu.w - 1); with kappa = exp(s)
    dlk = 1.0 / kappa - 2.0 * np.exp(-2.0 * kappa) / (-np.expm1(-2.0 * kappa)) + (cosw - 1.0)
    inside = (o[:, :, 4] > LOG_KAPPA_MIN) & (o[:, :, 4] < LOG_KAPPA_MAX)
    g[:, :, 4] = np.where(inside, r * dlk * kappa, 0.0)
    # d ln v / d m = kappa (w - (mu.w) mu) / |m|
    g[:, :, 1:4] = (r * kappa / np.maximum(nm, 1e-12))[:, :, None] * (w_out[:, None, :] - cosw[:, :, None] * mu)
    g = -(weight / W)[:, None, None] * g
    return L, g.reshape(-1, N_OUT)


def backward(params, cache, g_out):
    """Gradient of the loss with respect to the flat parameters (float64),
    given d L / d outputs; weights as used in the forward pass (bf16)."""
    layers = unpack(bf16_round(params))
    grads = []
    g = g_out
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        h = cache[li]
        grads.append((g.T @ h, g.sum(axis=0)))
        if li > 0:
            g = (g @ W) * (cache[li] > 0)
    grads.reverse()
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def loss_grad(params, X, w_out, weight):
    out, cache = forward(params, X)
    L, g = loss_and_grad_out(out, w_out, weight)
    return L, backward(params, cache, g)


def adam_step(params, m, v, grad, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba 2015) on the float32 master parameters."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return (params - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32), m, v
