"""Philox4x32-10 on the GPU against the oracle's implementation (bit-exact)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import ctx
from paper_1902_01137_amd import api

pytestmark = pytest.mark.gpu


def test_philox_bit_exact():
    rng = np.random.default_rng(5)
    n = 4099
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    key[0] = 0
    ctr[1] = 0xffffffff
    key[1] = 0xffffffff
    c = ctx()
    out = api.philox4x32_10(c, torch.from_numpy(ctr.view(np.int32)).cuda(), torch.from_numpy(key.view(np.int32)).cuda())
    got = out.cpu().numpy().view(np.uint32)
    for i in range(n):
        assert np.array_equal(got[i], oracle.philox4x32_10(ctr[i], key[i])), i


def test_philox_known_answer_vectors():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = [[int(v, 16) for v in l.split()] for l in open(path) if l.strip() and not l.startswith("#")]
    ctr = np.array([r[0:4] for r in rows], np.uint32)
    key = np.array([r[4:6] for r in rows], np.uint32)
    want = np.array([r[6:10] for r in rows], np.uint32)
    out = api.philox4x32_10(ctx(), torch.from_numpy(ctr.view(np.int32)).cuda(), torch.from_numpy(key.view(np.int32)).cuda())
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want)
