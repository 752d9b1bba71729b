"""Edge cases of the estimator entry points: empty work, one-pixel images,
cameras that miss the field, fields without extinction, axis-aligned rays,
the thinnest and the largest images, and argument errors."""
import math

import numpy as np
import pytest
import torch

from gpu_common import ctx, device_field
from paper_1902_01137_amd import _lib, api, inputs
from paper_1902_01137_amd.inputs import Camera, FieldDesc, GridParams, Optics, Sampling

pytestmark = pytest.mark.gpu


def _small():
    sc = inputs.scene_small()
    c = ctx()
    kd = device_field(sc.kc)
    g = api.build_grid(c, kd, sc.desc, sc.grid)
    return sc, c, kd, g


def test_zero_samples_leave_outputs_untouched():
    sc, c, kd, g = _small()
    s = torch.full((64, 64), 7.0, dtype=torch.float64, device="cuda")
    s2 = torch.full((64, 64), 9.0, dtype=torch.float64, device="cuda")
    api.render(c, g, kd, sc.optics, sc.camera, Sampling(seed=1, spp=0), s, s2)
    rays = torch.zeros((0, 6), dtype=torch.float32, device="cuda")
    t, t2 = api.transmittance(c, g, kd, Optics(), rays, Sampling(seed=1, spp=16))
    torch.cuda.synchronize()
    assert torch.all(s == 7.0) and torch.all(s2 == 9.0)
    assert t.numel() == 0 and t2.numel() == 0


@pytest.mark.parametrize("est", [0, 1, 2])
def test_one_pixel_and_thin_images(est):
    sc, c, kd, g = _small()
    for w, h in ((1, 1), (1, 37), (53, 1)):
        cam = Camera(**{**vars(sc.camera), "width": w, "height": h})
        cnt = api.new_counters("cuda")
        s, s2 = api.render(c, g, kd, sc.optics, cam, Sampling(seed=5, spp=33, flags=est), counters=cnt)
        torch.cuda.synchronize()
        assert api.counters_dict(cnt)["paths"] == w * h * 33
        assert torch.all(s >= 0) and torch.all(s2 >= 0) and torch.isfinite(s).all()


def test_camera_looking_away_sees_nothing():
    sc, c, kd, g = _small()
    (xa, xb), (ya, yb), (za, zb) = sc.desc.box
    cam = Camera(type=0, pos=(xa - 1.0, ya - 1.0, zb + 5.0), target=(xa - 10.0, ya - 10.0, zb + 20.0),
                 up=(0.0, 0.0, 1.0), fov_y_deg=20.0, width=16, height=16)
    s, s2 = api.render(c, g, kd, sc.optics, cam, Sampling(seed=3, spp=16))
    torch.cuda.synchronize()
    assert float(s.abs().sum()) == 0.0


def test_field_without_extinction_is_transparent():
    desc = FieldDesc(8, 8, 8, 0.0, 0.0, 1.0, 0.1, 0.1, 0.1)
    k = np.zeros((8, 8, 8), np.float32)
    c = ctx()
    kd = device_field(k)
    g = api.build_grid(c, kd, desc, GridParams(1.0, 0.0, 0))
    rays = inputs.random_rays(desc, 32, seed=4, inside_frac=0.5, axis_frac=0.5)
    for est in (0, 1, 2):
        t, t2 = api.transmittance(c, g, kd, Optics(), torch.from_numpy(rays).cuda(), Sampling(seed=2, spp=64, flags=est))
        torch.cuda.synchronize()
        assert torch.all(t == 64.0) and torch.all(t2 == 64.0)
    # a nadir sensor under the clear box sees the direct sun exactly (no gas, black ground)
    op = Optics(ssa=0.9, g=0.5, ground_albedo=0.0, sun_zenith_deg=20.0)
    cam = Camera(type=2, pos=(0.4, 0.4, 0.0), ortho_w=0.8, ortho_h=0.8, width=4, height=4)
    s, s2 = api.render(c, g, kd, op, cam, Sampling(seed=9, spp=16))
    torch.cuda.synchronize()
    assert torch.allclose(s, torch.full_like(s, 16.0))


def test_axis_aligned_rays_through_a_slab():
    """Rays along the axes (two direction components exactly zero) meet the
    closed form exp(-tau) of a layered slab."""
    desc, k = inputs.slab_field([0.4, 1.0, 0.2], 0.5)
    c = ctx()
    kd = device_field(k)
    g = api.build_grid(c, kd, desc, GridParams(1.0, 0.0, 0))
    rays = np.array([[0.0, 0.0, 2.0, 0.0, 0.0, -1.0], [0.0, 0.0, -0.5, 0.0, 0.0, 1.0]], np.float32)
    spp = 200000
    s, s2 = api.transmittance(c, g, kd, Optics(), torch.from_numpy(rays).cuda(), Sampling(seed=6, spp=spp))
    torch.cuda.synchronize()
    exact = math.exp(-(0.4 + 1.0 + 0.2) * 0.5)
    T = s.cpu().numpy() / spp
    assert np.all(np.abs(T - exact) < 4.5 * math.sqrt(exact * (1 - exact) / spp)), T


def test_large_image_paths_all_counted():
    """A 2048 x 2048 image with one sample: every pixel is traced once."""
    sc, c, kd, g = _small()
    cam = Camera(**{**vars(sc.camera), "width": 2048, "height": 2048})
    cnt = api.new_counters("cuda")
    s, s2 = api.render(c, g, kd, sc.optics, cam, Sampling(seed=8, spp=1), counters=cnt)
    torch.cuda.synchronize()
    assert api.counters_dict(cnt)["paths"] == 2048 * 2048
    assert torch.isfinite(s).all()


def test_argument_errors():
    sc, c, kd, g = _small()
    bad = [
        (Camera(**{**vars(sc.camera), "width": 0}), sc.optics, Sampling(seed=1, spp=1)),
        (Camera(**{**vars(sc.camera), "type": 7}), sc.optics, Sampling(seed=1, spp=1)),
        (sc.camera, Optics(**{**vars(sc.optics), "g": 1.0}), Sampling(seed=1, spp=1)),
        (sc.camera, Optics(**{**vars(sc.optics), "ssa": 1.5}), Sampling(seed=1, spp=1)),
        (sc.camera, Optics(**{**vars(sc.optics), "majorant_scale": 0.5}), Sampling(seed=1, spp=1)),
        (sc.camera, sc.optics, Sampling(seed=1, spp=-1)),
        (sc.camera, sc.optics, Sampling(seed=1, spp=4, sample_offset=(1 << 32) - 2)),
    ]
    for cam, op, smp in bad:
        with pytest.raises(_lib.NcError):
            api.render(c, g, kd, op, cam, smp)
    # an irradiance sensor needs the sun above the horizon
    cam = Camera(type=2, pos=(1.6, 1.6, 0.0), ortho_w=1.0, ortho_h=1.0, width=2, height=2)
    with pytest.raises(_lib.NcError) as e:
        api.render(c, g, kd, Optics(**{**vars(sc.optics), "sun_zenith_deg": 95.0}), cam, Sampling(seed=1, spp=1))
    assert e.value.status == _lib.NC_ERR_RANGE
