"""Statistical comparison helpers for Monte Carlo parity tests."""
import math

import numpy as np
from scipy import stats


def mean_se(s, s2, n):
    """Per-element mean and standard error from sums over n samples."""
    m = np.asarray(s, dtype=np.float64) / n
    var = np.maximum(np.asarray(s2, dtype=np.float64) / n - m * m, 0.0) * n / max(n - 1, 1)
    return m, np.sqrt(var / n)


def block(mean, se, shape, b=8):
    """Average over b x b pixel blocks (pixels are independent)."""
    H, W = shape
    Hb, Wb = H // b, W // b
    m = mean.reshape(H, W)[:Hb * b, :Wb * b].reshape(Hb, b, Wb, b)
    e = se.reshape(H, W)[:Hb * b, :Wb * b].reshape(Hb, b, Wb, b)
    return m.mean(axis=(1, 3)).ravel(), np.sqrt((e ** 2).sum(axis=(1, 3))).ravel() / (b * b)


# Relative precision of the GPU's float32 path arithmetic: an estimate whose
# paths nearly all return the same value (a ground point lit through clear
# air) has a tiny standard error, and the float32 rounding of that value
# against the oracle's float64 must not count as a statistical excess.
F32_REL = 1e-5


def compare(ma, sa, mb, sb, zmax_global=3.0, p_min=1e-3):
    """Two-sample z-tests with independent errors.

    Passes if the number of |z| > 3 elements is consistent with
    Binomial(n, 0.0027) (p-value >= p_min) and the z of the overall mean is
    below zmax_global (the acceptance rule of the parity tests: 3 combined
    standard errors, p >= 1e-3).  Each element's error includes the float32
    rounding floor F32_REL of its value.  Returns a dict of diagnostics and
    the verdict."""
    ma, sa, mb, sb = (np.asarray(x, dtype=np.float64).ravel() for x in (ma, sa, mb, sb))
    floor = F32_REL * np.maximum(np.abs(ma), np.abs(mb))
    den = np.sqrt(sa ** 2 + sb ** 2 + floor ** 2)
    ok = den > 0
    z = np.zeros_like(ma)
    z[ok] = (ma[ok] - mb[ok]) / den[ok]
    # elements with no spread on either side (every path returned the same
    # value, e.g. a sky pixel or a ground point lit through vacuum) must agree
    # to the rounding of float32 path arithmetic
    exact_eq = (~ok) & (ma != mb)
    n = int(ok.sum())
    k = int((np.abs(z) > 3).sum())
    p = 1.0 - stats.binom.cdf(k - 1, n, 0.0027) if n else 1.0
    zg = (ma.mean() - mb.mean()) / math.sqrt((sa ** 2).sum() + (sb ** 2).sum()) * len(ma) if (sa ** 2).sum() + (
        sb ** 2).sum() > 0 else 0.0
    ex = np.abs(z) > 3
    rel = np.abs(ma - mb) / np.maximum(np.maximum(np.abs(ma), np.abs(mb)), 1e-300)
    res = dict(n=n, exceed=k, exceed_low=int((z < -3).sum()), exceed_high=int((z > 3).sum()), p=p, z_global=zg,
               zmax=float(np.abs(z).max()) if n else 0.0, bad_zero_se=int(exact_eq.sum()),
               exceed_rel_diff_max=float(rel[ex].max()) if ex.any() else 0.0,
               exceed_rel_se_min=float((np.sqrt(sa ** 2 + sb ** 2)[ex] / np.maximum(np.abs(ma), 1e-300)[ex]).min())
               if ex.any() else 0.0)
    res["ok"] = (p >= p_min) and abs(zg) < zmax_global and res["bad_zero_se"] == 0
    return res


def vs_exact(m, se, exact, zmax_global=3.0, p_min=1e-3):
    """compare() of estimates against exact values (zero standard error)."""
    m = np.asarray(m, dtype=np.float64).ravel()
    ex = np.broadcast_to(np.asarray(exact, dtype=np.float64).ravel() if np.ndim(exact) else exact, m.shape)
    se = np.broadcast_to(np.asarray(se, dtype=np.float64).ravel() if np.ndim(se) else se, m.shape)
    return compare(m, np.array(se, dtype=np.float64), np.array(ex, dtype=np.float64), np.zeros_like(m), zmax_global,
                   p_min)


def z_scalar(a, sa, b, sb=0.0):
    """z of one difference with independent errors."""
    den = math.sqrt(sa * sa + sb * sb)
    return (a - b) / den if den > 0 else (0.0 if a == b else math.inf)
