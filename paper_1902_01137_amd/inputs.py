"""Seeded synthetic inputs: voxel extinction fields, ray sets and scene descriptions.

This module is shared by the HIP path's tests/benchmarks and by the oracle's
tests.  It holds input recipes only (random fields, geometry, camera and sun
set-ups), none of the path-tracing arithmetic.  Every generator is seeded and
deterministic.

Units: lengths in km, extinction coefficients in km^-1, angles in degrees.
Fields are float32 arrays of shape (nz, ny, nx), x fastest.

The paper's own LES fields (Meso-NH congestus, BOMEX, ARMCu, FIRE) are not
available; the recipes below stand in for them with the same grid shapes
(512x512x160 at 25 m is BOMEX's shape, Section 4.3) and the same kind of
structure (broken boundary-layer cumulus over clear air, coarse-grained by
regional averages as in Section 4.2).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------
# Scene description records (plain data)
# ----------------------------------------------------------------------------


@dataclass
class FieldDesc:
    nx: int
    ny: int
    nz: int
    x0: float = 0.0
    y0: float = 0.0
    z0: float = 0.0
    dx: float = 0.1
    dy: float = 0.1
    dz: float = 0.1

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def box(self):
        return ((self.x0, self.x0 + self.nx * self.dx),
                (self.y0, self.y0 + self.ny * self.dy),
                (self.z0, self.z0 + self.nz * self.dz))


@dataclass
class GridParams:
    tau_tilde: float = 1.0
    k_gas: float = 0.0
    criterion: int = 0          # 0: kmax*dz_node < tau_tilde, 1: (kmax-kmin)*dz_node < tau_tilde, 2: flat, 3: layered
    flat_level: int = 3         # criteria 2, 3: every node of level <= flat_level is a voxel (2^3-cell supercells)


@dataclass
class Optics:
    ssa: float = 0.999
    g: float = 0.85
    ground_albedo: float = 0.2
    sun_zenith_deg: float = 30.0
    sun_azimuth_deg: float = 0.0
    sun_irradiance: float = 1.0
    majorant_scale: float = 1.0
    max_scatter: int = -1          # -1: unlimited
    max_segments: int = 1_000_000  # per path, counted when hit
    sun_half_angle_deg: float = 0.0  # angular radius of the solar disc (0: directional sun)
    phase_table: object = None       # (mu, p): tabulated phase function instead of HG (cosines -1..1, values)
    kdist: object = None             # (w, k_gas): k-distribution, a quadrature point drawn per path (<= 16 points)


@dataclass
class Camera:
    type: int = 0                  # 0 pinhole, 1 orthographic, 2 horizontal irradiance sensor (looks up)
    pos: tuple = (0.0, 0.0, 0.0)
    target: tuple = (0.0, 0.0, -1.0)
    up: tuple = (0.0, 0.0, 1.0)
    fov_y_deg: float = 60.0
    ortho_w: float = 1.0
    ortho_h: float = 1.0
    width: int = 64
    height: int = 64


@dataclass
class Sampling:
    seed: int = 1
    sample_offset: int = 0
    spp: int = 16
    flags: int = 0
    guide_frac: float = 0.5
    stream: int = 0
    guide_max_order: int = 0    # last guided scattering order (0: all)


@dataclass
class Scene:
    name: str
    desc: FieldDesc
    kc: np.ndarray
    grid: GridParams
    optics: Optics
    camera: Camera | None = None
    sampling: Sampling = field(default_factory=Sampling)

    def replace(self, **kw):
        return dataclasses.replace(self, **kw)


# ----------------------------------------------------------------------------
# Field recipes
# ----------------------------------------------------------------------------


def _gaussian_smooth_wrap(a: np.ndarray, sigma_cells: float) -> np.ndarray:
    """Periodic Gaussian smoothing by FFT (sigma in cells)."""
    spec = np.fft.rfftn(a)
    ks = [np.fft.fftfreq(n) for n in a.shape[:-1]] + [np.fft.rfftfreq(a.shape[-1])]
    grids = np.meshgrid(*ks, indexing="ij")
    k2 = sum(g * g for g in grids)
    spec *= np.exp(-2.0 * np.pi ** 2 * sigma_cells ** 2 * k2)
    return np.fft.irfftn(spec, s=a.shape, axes=tuple(range(a.ndim)))


def lognormal_blob(n: int = 32, cell: float = 0.1, z0: float = 1.0, peak: float = 50.0,
                   clear: float = 0.01, radius: float = 0.5, seed: int = 1):
    """Small cloud: a Gaussian envelope times lognormal noise over clear air.

    k = clear + (peak - clear) * E*M / max(E*M) with E = exp(-|x-c|^2 / (2 r^2))
    about the box centre and M = exp(0.5 G - 0.125), G unit-variance Gaussian
    noise (seeded) smoothed over 1.5 cells.
    """
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((n, n, n))
    G = _gaussian_smooth_wrap(noise, 1.5)
    G = (G - G.mean()) / G.std()
    M = np.exp(0.5 * G - 0.125)
    c = (np.arange(n) + 0.5) * cell
    zc = z0 + c
    ctr = (n * cell / 2.0, n * cell / 2.0, z0 + n * cell / 2.0)
    Z, Y, X = np.meshgrid(zc, c, c, indexing="ij")
    r2 = (X - ctr[0]) ** 2 + (Y - ctr[1]) ** 2 + (Z - ctr[2]) ** 2
    E = np.exp(-r2 / (2.0 * radius ** 2))
    EM = E * M
    k = clear + (peak - clear) * EM / EM.max()
    desc = FieldDesc(n, n, n, 0.0, 0.0, z0, cell, cell, cell)
    return desc, k.astype(np.float32)


def gaussian_random_field(shape, spacing, seed, slope=-11.0 / 6.0, workers=8):
    """Zero-mean, unit-variance Gaussian random field with amplitude |k|^slope.

    An energy spectrum E(k) ~ k^-5/3 in 3D corresponds to an amplitude filter
    |k|^-11/6 on white noise.  `shape` is (nz, ny, nx), `spacing` (dz, dy, dx).
    Computed in float32 with scipy's FFT.
    """
    import scipy.fft as sfft
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(shape, dtype=np.float32)
    spec = sfft.rfftn(noise, workers=workers)
    del noise
    nz, ny, nx = shape
    dz, dy, dx = spacing
    kz = np.fft.fftfreq(nz, d=dz).astype(np.float32)
    ky = np.fft.fftfreq(ny, d=dy).astype(np.float32)
    kx = np.fft.rfftfreq(nx, d=dx).astype(np.float32)
    # build |k|^slope plane by plane to bound memory
    kyx2 = ky[:, None] ** 2 + kx[None, :] ** 2
    for iz in range(nz):
        k2 = kyx2 + kz[iz] ** 2
        with np.errstate(divide="ignore"):
            amp = np.where(k2 > 0, k2 ** (slope / 2.0), 0.0).astype(np.float32)
        spec[iz] *= amp
    G = sfft.irfftn(spec, s=shape, workers=workers).astype(np.float32)
    del spec
    G -= G.mean(dtype=np.float64)
    G /= G.std(dtype=np.float64)
    return G


def cumulus_field(fine=(320, 1024, 1024), pool=2, cell_fine=0.0125, cover=0.15,
                  base=0.5, top=1.5, lwc_rate=2.0, k_per_lwc=150.0, seed=2, workers=8):
    """Broken cumulus field from a thresholded k^-5/3 Gaussian random field.

    Generated on the fine grid `fine` = (nz, ny, nx) with cubic cells of
    `cell_fine` km, then coarse-grained by `pool` x `pool` x `pool` regional
    averages (which preserves the total condensed water, Section 4.2).

    A fine cell is cloudy iff G > t and base <= z <= top, with t chosen so that
    `cover` of the columns hold at least one cloudy cell.  The liquid water
    content follows an adiabatic profile LWC = lwc_rate * (z - base) g m^-3
    (z in km) and the extinction is 1.5 LWC / (rho_w r_eff) = k_per_lwc * LWC
    km^-1 (r_eff = 10 um).  Clear cells are 0 (the gas is a separate constant).
    """
    nz, ny, nx = fine
    G = gaussian_random_field(fine, (cell_fine,) * 3, seed, workers=workers)
    zc = (np.arange(nz, dtype=np.float64) + 0.5) * cell_fine
    layer = (zc >= base) & (zc <= top)
    colmax = G[layer].max(axis=0)
    t = np.quantile(colmax.astype(np.float64), 1.0 - cover)
    lwc = np.where(layer, lwc_rate * (zc - base), 0.0).astype(np.float32)
    k = np.where(G > t, (k_per_lwc * lwc)[:, None, None], np.float32(0.0)).astype(np.float32)
    del G
    if pool > 1:
        k = k.reshape(nz // pool, pool, ny // pool, pool, nx // pool, pool)
        k = k.mean(axis=(1, 3, 5), dtype=np.float64).astype(np.float32)
    c = cell_fine * pool
    desc = FieldDesc(nx // pool, ny // pool, nz // pool, 0.0, 0.0, 0.0, c, c, c)
    return desc, np.ascontiguousarray(k)


def pool_field(desc: FieldDesc, k: np.ndarray, f: int):
    """Coarse-grain a field by f x f x f regional averages."""
    nz, ny, nx = k.shape
    kk = k.reshape(nz // f, f, ny // f, f, nx // f, f).mean(axis=(1, 3, 5), dtype=np.float64)
    d = FieldDesc(nx // f, ny // f, nz // f, desc.x0, desc.y0, desc.z0,
                  desc.dx * f, desc.dy * f, desc.dz * f)
    return d, np.ascontiguousarray(kk.astype(np.float32))


def cylinder_cumulus(n=256, cell=0.02, radius=1.0, base=0.5, top=2.5, tau_min=5.0, tau_max=40.0):
    """Single cumulus: a vertical cylinder about the box centre.

    Inside r < radius and base <= z <= top the extinction is
    (tau_min + (tau_max - tau_min)(1 - r^2/R^2)) / (top - base), so the
    vertical optical depth of a column runs from tau_min at the edge to
    tau_max on the axis.  Outside the cylinder it is 0.
    """
    c = (np.arange(n) + 0.5) * cell
    L = n * cell
    Y, X = np.meshgrid(c, c, indexing="ij")
    r2 = ((X - L / 2) ** 2 + (Y - L / 2) ** 2) / radius ** 2
    col = np.where(r2 < 1.0, (tau_min + (tau_max - tau_min) * (1.0 - r2)) / (top - base), 0.0)
    zin = (c >= base) & (c <= top)
    k = np.where(zin[:, None, None], col[None, :, :], 0.0).astype(np.float32)
    desc = FieldDesc(n, n, n, 0.0, 0.0, 0.0, cell, cell, cell)
    return desc, np.ascontiguousarray(k)


def slab_field(k_layers, dz_layers, width=1.0e4, z0=0.0):
    """Horizontally homogeneous layered slab: one cell per layer, huge in x and y.

    With cells 1e4 km wide, paths essentially never leave the slab sideways,
    so plane-parallel closed forms apply.
    """
    dz = float(dz_layers)
    nz = len(k_layers)
    k = np.asarray(k_layers, dtype=np.float32).reshape(nz, 1, 1)
    desc = FieldDesc(1, 1, nz, -width / 2, -width / 2, z0, width, width, dz)
    return desc, np.ascontiguousarray(k)


# ----------------------------------------------------------------------------
# Ray sets
# ----------------------------------------------------------------------------


def random_rays(desc: FieldDesc, n: int, seed: int, inside_frac=0.5, axis_frac=0.1):
    """Rays (ox,oy,oz,dx,dy,dz) as float32: a mix of origins inside the box,
    outside it aimed at a random interior point, and axis-parallel directions."""
    rng = np.random.default_rng(seed)
    (xa, xb), (ya, yb), (za, zb) = desc.box
    lo = np.array([xa, ya, za])
    hi = np.array([xb, yb, zb])
    ext = hi - lo
    rays = np.zeros((n, 6), dtype=np.float64)
    inside = rng.random(n) < inside_frac
    p_in = lo + rng.random((n, 3)) * ext
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    axis = rng.random(n) < axis_frac
    ax = rng.integers(0, 3, n)
    sgn = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    va = np.zeros((n, 3))
    va[np.arange(n), ax] = sgn
    v = np.where(axis[:, None], va, v)
    far = p_in - v * (1.5 * np.linalg.norm(ext))
    o = np.where(inside[:, None], p_in, far)
    rays[:, :3] = o
    rays[:, 3:] = v
    r32 = rays.astype(np.float32)
    # renormalise in float32 so |d| = 1 to float32 precision
    d = r32[:, 3:].astype(np.float64)
    r32[:, 3:] = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    return r32


def phase_table_tthg(g1=0.92, g2=-0.35, w=0.96, n=181):
    """A synthetic tabulated phase function with the shape of a droplet Mie
    function (strong forward peak, weak backward lobe): a two-term HG mixture
    sampled at n cosines whose angles are uniform in [0, pi] (dense near the
    peak).  Returns (mu ascending from -1 to 1, p) in float64."""
    th = np.linspace(np.pi, 0.0, n)
    mu = np.cos(th)
    mu[0], mu[-1] = -1.0, 1.0

    def hg(g):
        return (1 - g * g) / (4 * np.pi * (1 + g * g - 2 * g * mu) ** 1.5)
    return mu, w * hg(g1) + (1 - w) * hg(g2)


def kdist_synthetic(n=8, k_min=1e-3, k_max=1.0, seed=5):
    """A synthetic k-distribution of one band: n quadrature points whose gas
    extinction spans k_min .. k_max km^-1 geometrically, with Gauss-like
    weights (more weight on the weak lines).  Returns (w, k_gas)."""
    k = np.geomspace(k_min, k_max, n)
    rng = np.random.default_rng(seed)
    w = np.exp(-0.5 * np.linspace(0.0, 2.5, n) ** 2) * (1.0 + 0.1 * rng.random(n))
    return w / w.sum(), k


def sun_direction(zenith_deg, azimuth_deg):
    """Unit vector towards the sun; azimuth from +X towards +Y (Table 3 convention)."""
    t = np.deg2rad(zenith_deg)
    p = np.deg2rad(azimuth_deg)
    return np.array([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)])


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------

SEED_GPU_BASE = 1000
SEED_ORACLE_BASE = 2000


def scene_small(spp=16):
    """32^3 lognormal blob, 100 m voxels, 1 km above ground; 64x64 nadir view."""
    desc, k = lognormal_blob()
    (xa, xb), (ya, yb), (za, zb) = desc.box
    cam = Camera(type=1, pos=((xa + xb) / 2, (ya + yb) / 2, zb), target=((xa + xb) / 2, (ya + yb) / 2, 0.0),
                 up=(0.0, 1.0, 0.0), ortho_w=xb - xa, ortho_h=yb - ya, width=64, height=64)
    return Scene("small_blob_32", desc, k, GridParams(1.0, 0.0, 0),
                 Optics(ssa=0.999, g=0.85, ground_albedo=0.2, sun_zenith_deg=30.0, sun_azimuth_deg=0.0),
                 cam, Sampling(seed=SEED_GPU_BASE + 1, spp=spp))


def scene_cumulus(fine=(320, 1024, 1024), pool=2, width=1024, height=1024, spp=64, workers=8, field=None):
    """Broken cumulus at 25 m (512x512x160) seen by an oblique pinhole camera.
    `field` = (desc, k) replaces the generated field (e.g. another member of
    the refinement family)."""
    desc, k = field if field is not None else cumulus_field(fine=fine, pool=pool, workers=workers)
    (xa, xb), (ya, yb), (za, zb) = desc.box
    cx, cy = (xa + xb) / 2, (ya + yb) / 2
    # camera 3 km outside the -X face at mid-Y, 2 km high, looking at the cloud layer
    cam = Camera(type=0, pos=(xa - 3.0, cy, 2.0), target=(cx, cy, 0.75), up=(0.0, 0.0, 1.0),
                 fov_y_deg=60.0, width=width, height=height)
    return Scene("cumulus_%dx%dx%d" % (desc.nx, desc.ny, desc.nz), desc, k, GridParams(1.0, 0.05, 0),
                 Optics(ssa=0.999, g=0.86, ground_albedo=0.2, sun_zenith_deg=45.0, sun_azimuth_deg=0.0),
                 cam, Sampling(seed=SEED_GPU_BASE + 2, spp=spp))


def scene_cylinder():
    """Single 2 km cumulus cylinder (tau 5-40) on a 256^3 grid, sun at zenith, black ground."""
    desc, k = cylinder_cumulus()
    return Scene("cylinder_256", desc, k, GridParams(1.0, 0.0, 0),
                 Optics(ssa=0.999, g=0.85, ground_albedo=0.0, sun_zenith_deg=0.0, sun_azimuth_deg=0.0,
                        majorant_scale=2.0),
                 None, Sampling(seed=SEED_GPU_BASE + 4, spp=1))


def batch_views(n_views=48, suns=(15.0, 30.0, 45.0, 60.0), centre=(6.4, 6.4), ring=10.0, height=2.0,
                target_z=0.75, base_side=256, side_step=128, side_mod=7):
    """48 views on a ring about the domain centre, of uneven size, times 4 suns."""
    jobs = []
    for s in suns:
        for i in range(n_views):
            a = np.deg2rad(7.5 * i)
            pos = (centre[0] + ring * np.cos(a), centre[1] + ring * np.sin(a), height)
            side = base_side + side_step * (i % side_mod)
            cam = Camera(type=0, pos=pos, target=(centre[0], centre[1], target_z), up=(0.0, 0.0, 1.0),
                         fov_y_deg=60.0, width=side, height=side)
            jobs.append((cam, s))
    return jobs
