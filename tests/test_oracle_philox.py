"""Statistical checks of the counter-based generator (Philox4x32-10): the
GPU's generator is bit-exact with this one (test_gpu_philox), so these
properties hold for the tracer's random numbers too."""
import numpy as np
from scipy import stats


def _stream(orc, n, key=(0x1234, 0x9876), word=7):
    """n Philox blocks of consecutive counters (i, 0, word, 0) under one key."""
    out = np.zeros((n, 4), np.uint32)
    for i in range(n):
        out[i] = orc.philox4x32_10(np.array([i, 0, word, 0], np.uint32), np.array(key, np.uint32))
    return out.ravel()


def test_uniformity_chi_square(orc):
    x = _stream(orc, 1 << 14)                      # 65536 words
    u = (x >> 8).astype(np.float64) * 2.0 ** -24   # the tracer's uniform in [0, 1)
    counts, _ = np.histogram(u, bins=256, range=(0.0, 1.0))
    chi2, p = stats.chisquare(counts)
    assert p > 1e-3, (chi2, p)
    # every output bit is balanced
    bits = np.unpackbits(x.view(np.uint8)).reshape(-1, 32).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / np.sqrt(len(x)))


def test_serial_correlation(orc):
    x = _stream(orc, 1 << 14, word=11)
    u = (x >> 8).astype(np.float64) * 2.0 ** -24
    for lag in (1, 2, 3, 4, 5):
        r = np.corrcoef(u[:-lag], u[lag:])[0, 1]
        assert abs(r) < 5 / np.sqrt(len(u)), (lag, r)


def test_neighbouring_counters_and_keys_decorrelate(orc):
    a = _stream(orc, 1 << 12, key=(1, 0))
    b = _stream(orc, 1 << 12, key=(2, 0))
    c = _stream(orc, 1 << 12, key=(1, 0), word=8)
    for y in (b, c):
        ua = (a >> 8).astype(np.float64)
        uy = (y >> 8).astype(np.float64)
        assert abs(np.corrcoef(ua, uy)[0, 1]) < 5 / np.sqrt(len(ua))
        # about half the bits differ between streams
        diff = np.unpackbits((a ^ y).view(np.uint8)).mean()
        assert abs(diff - 0.5) < 0.01


def test_known_answer_vectors(orc):
    """The published known-answer vectors of Philox4x32-10 (tests/golden)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(v, 16) for v in r]
        ctr, key, want = np.array(w[0:4], np.uint32), np.array(w[4:6], np.uint32), np.array(w[6:10], np.uint32)
        assert np.array_equal(orc.philox4x32_10(ctr, key), want), r
