"""The oracle's chunked photon runs equal one serial run over the same photon streams."""
import numpy as np

import oracle
from paper_1902_01137_amd.inputs import Optics, slab_field


def test_parallel_chunks_equal_serial():
    desc, k = slab_field([3.0], 0.5, z0=0.2)
    op = Optics(ssa=0.9, g=0.7, ground_albedo=0.3, sun_zenith_deg=30.0)
    t1, g1 = oracle.flux(desc, k, 0.0, op, (4, 4), 3001, seed=11)
    t2, g2 = oracle.parallel_flux(desc, k, 0.0, op, (4, 4), 3001, seed=11, workers=3)
    assert np.allclose(t1, t2, rtol=1e-12, atol=1e-9) and np.array_equal(g1, g2)
    f1, tot1 = oracle.flux_fd(desc, k, 0.0, op, (4, 4), 2000, 12, 0, with_total=True)
    f2, tot2 = oracle.parallel_flux_fd(desc, k, 0.0, op, (4, 4), 2000, 12, 0, workers=2)
    assert np.allclose(f1, f2, rtol=1e-12, atol=1e-9) and np.allclose(tot1, tot2, rtol=1e-12, atol=1e-9)
