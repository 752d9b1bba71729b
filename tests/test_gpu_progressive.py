"""Progressive rendering to a target relative standard error: the rounds
form one render of spp_done samples, the reported error is the one the
buffers give, and the stopping rule meets the target."""
import numpy as np
import pytest
import torch

from gpu_common import ctx, device_field
from paper_1902_01137_amd import api, inputs
from paper_1902_01137_amd.inputs import Sampling

pytestmark = pytest.mark.gpu


def _eps(s, s2, n, b):
    H, W = s.shape
    m = s / n
    var = np.maximum(s2 / n - m * m, 0) * n / (n - 1)
    e = var / n
    ms, es = [], []
    for y in range(0, H, b):
        for x in range(0, W, b):
            mb = m[y:y + b, x:x + b]
            ms.append(mb.mean())
            es.append(e[y:y + b, x:x + b].sum() / mb.size ** 2)
    return np.sqrt(np.mean(es)) / np.mean(ms)


@pytest.mark.parametrize("block", [1, 8, 5])
def test_progressive_reaches_target_and_equals_one_render(block):
    sc = inputs.scene_small()
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    target = {1: 0.1, 5: 0.02, 8: 0.01}[block]
    s, s2, rep = api.render_progressive(c, g, kd, sc.optics, sc.camera, Sampling(seed=21, spp=0), target, first_spp=4,
                                        max_spp=4096, block=block)
    torch.cuda.synchronize()
    n = rep["spp_done"]
    assert rep["rel_err"] <= target and 4 <= n < 4096 and rep["rounds"] >= 1
    sn, s2n = s.cpu().numpy(), s2.cpu().numpy()
    assert rep["rel_err"] == pytest.approx(_eps(sn, s2n, n, block), rel=1e-9)
    # the union of the rounds is one render of n samples (partial sums group differently)
    r, r2 = api.render(c, g, kd, sc.optics, sc.camera, Sampling(seed=21, spp=n))
    torch.testing.assert_close(s, r, rtol=1e-6, atol=1e-9)
    torch.testing.assert_close(s2, r2, rtol=1e-6, atol=1e-9)


def test_progressive_stops_at_max_spp():
    sc = inputs.scene_small()
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    _, _, rep = api.render_progressive(c, g, kd, sc.optics, sc.camera, Sampling(seed=3, spp=0), 1e-6, first_spp=4,
                                       max_spp=40)
    assert rep["spp_done"] == 40 and rep["rel_err"] > 1e-6
