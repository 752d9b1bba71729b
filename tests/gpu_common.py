"""Shared set-up for the GPU tests: one library context per session."""
import numpy as np
import pytest
import torch

from paper_1902_01137_amd import api


def device_field(kc):
    return torch.from_numpy(np.ascontiguousarray(kc, dtype=np.float32)).cuda()


_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        if not torch.cuda.is_available():
            pytest.skip("no GPU")
        _CTX = api.Context(0)
    return _CTX
