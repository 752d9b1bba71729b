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


def compare(ma, sa, mb, sb, zmax_global=4.0, p_min=1e-4):
    """Two-sample z-tests with independent errors.

    Passes if the number of |z| > 3 elements is consistent with
    Binomial(n, 0.0027) (p-value >= p_min) and the z of the overall mean is
    below zmax_global.  Returns a dict of diagnostics and the verdict."""
    ma, sa, mb, sb = (np.asarray(x, dtype=np.float64).ravel() for x in (ma, sa, mb, sb))
    den = np.sqrt(sa ** 2 + sb ** 2)
    ok = den > 0
    z = np.zeros_like(ma)
    z[ok] = (ma[ok] - mb[ok]) / den[ok]
    exact_eq = (~ok) & (ma != mb)
    n = int(ok.sum())
    k = int((np.abs(z) > 3).sum())
    p = 1.0 - stats.binom.cdf(k - 1, n, 0.0027) if n else 1.0
    zg = (ma.mean() - mb.mean()) / math.sqrt((sa ** 2).sum() + (sb ** 2).sum()) * len(ma) if (sa ** 2).sum() + (
        sb ** 2).sum() > 0 else 0.0
    res = dict(n=n, exceed=k, p=p, z_global=zg, zmax=float(np.abs(z).max()) if n else 0.0,
               bad_zero_se=int(exact_eq.sum()))
    res["ok"] = (p >= p_min) and abs(zg) < zmax_global and res["bad_zero_se"] == 0
    return res
