"""Seeded synthetic inputs shared by the renderer's tests/bench and the oracle.

This module only *describes* scenes: triangle soups, per-material optical
constants tabulated at the wavelength-bin centres, a sun spectrum, cameras.
It holds none of the rendering arithmetic (no intersection, no Fresnel, no
sampling), so that the oracle and the HIP path stay independent of each other
and meet only on these inputs.

Stand-ins: the paper's Royaumont CAD model and its measured optical data
(ellipsometry n/k of Saint-Just glasses, transmittance maps, solar spectra;
section 3) are not available, so every scene here is procedural and seeded.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SCENE_SEED = 0x19124000
RENDER_SEED = 1
VIEW_SEED = 7

MAT_OPAQUE = 0
MAT_GLASS = 1

# Exact SI values (2019 redefinition) used for the blackbody sun table.
H_PLANCK = 6.62607015e-34
C_LIGHT = 299792458.0
K_BOLTZMANN = 1.380649e-23


def bin_centres(n_bins: int, lambda_min_nm: float = 380.0, lambda_max_nm: float = 780.0) -> np.ndarray:
    """Vacuum wavelengths (nm) of the bin centres: lmin + (j + 1/2) * (lmax - lmin) / B."""
    j = np.arange(n_bins, dtype=np.float64)
    return lambda_min_nm + (j + 0.5) * (lambda_max_nm - lambda_min_nm) / n_bins


def planck(lambda_nm, temperature_k: float = 5778.0):
    """Blackbody spectral radiance 2 h c^2 / lambda^5 / (exp(h c / (lambda k T)) - 1), SI units."""
    lam = np.asarray(lambda_nm, dtype=np.float64) * 1e-9
    return 2.0 * H_PLANCK * C_LIGHT**2 / lam**5 / np.expm1(H_PLANCK * C_LIGHT / (lam * K_BOLTZMANN * temperature_k))


def sun_irradiance(n_bins: int, lambda_min_nm: float = 380.0, lambda_max_nm: float = 780.0,
                   temperature_k: float = 5778.0) -> np.ndarray:
    """Directional-sun spectrum: a 5778 K blackbody point-sampled at the bin centres,
    normalised to 1 at 555 nm (a stand-in for the paper's Rayleigh-derived solar
    spectrum, section 3). FP64 here, handed over as FP32."""
    lam = bin_centres(n_bins, lambda_min_nm, lambda_max_nm)
    return (planck(lam, temperature_k) / planck(555.0, temperature_k)).astype(np.float32)


def sun_direction(elevation_deg: float = 35.0, azimuth_deg: float = -90.0) -> np.ndarray:
    """Unit vector pointing *toward* the sun (plane-wave source, section 3).
    Azimuth is measured from +x toward +y; -90 deg puts the sun beyond y < 0."""
    el, az = math.radians(elevation_deg), math.radians(azimuth_deg)
    v = np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    v[np.abs(v) < 1e-15] = 0.0
    return (v / np.linalg.norm(v)).astype(np.float32)


@dataclass
class Camera:
    eye: tuple
    target: tuple
    up: tuple = (0.0, 0.0, 1.0)
    vfov_deg: float = 60.0
    width: int = 64
    height: int = 64


@dataclass
class Scene:
    """A triangle scene plus its spectral data; every array is what both sides read."""
    verts: np.ndarray            # float32 [N][3][3]
    mat: np.ndarray              # uint16 [N]
    mat_type: np.ndarray         # int32 [n_mat]   0 opaque, 1 thin glass slab
    thickness_m: np.ndarray      # float32 [n_mat] slab thickness (glass only)
    n_tab: np.ndarray            # float32 [n_mat][B] real index n(lambda_j)
    k_tab: np.ndarray            # float32 [n_mat][B] extinction k(lambda_j)
    rho_tab: np.ndarray          # float32 [n_mat][B] diffuse albedo of opaque materials
    lambda_min_nm: float
    lambda_max_nm: float
    sun_dir: np.ndarray          # float32 [3], toward the sun
    sun_E: np.ndarray            # float32 [B]
    env: np.ndarray              # float32 [B] radiance of escaping rays
    name: str = ""
    info: dict = field(default_factory=dict)

    @property
    def n_bins(self) -> int:
        return int(self.n_tab.shape[1])

    @property
    def n_tri(self) -> int:
        return int(self.verts.shape[0])

    @property
    def n_mat(self) -> int:
        return int(self.mat_type.shape[0])

    def check(self) -> "Scene":
        assert self.verts.dtype == np.float32 and self.verts.ndim == 3 and self.verts.shape[1:] == (3, 3)
        assert self.mat.dtype == np.uint16 and self.mat.shape == (self.n_tri,)
        for a in (self.n_tab, self.k_tab, self.rho_tab):
            assert a.dtype == np.float32 and a.shape == (self.n_mat, self.n_bins)
        assert self.sun_E.shape == (self.n_bins,) and self.env.shape == (self.n_bins,)
        for a in ("verts", "mat", "mat_type", "thickness_m", "n_tab", "k_tab", "rho_tab", "sun_dir", "sun_E", "env"):
            setattr(self, a, np.ascontiguousarray(getattr(self, a)))
        return self


# ----------------------------------------------------------------------------------------------
# geometry helpers (pure data construction)
# ----------------------------------------------------------------------------------------------

def _quad_grid(origin, ex, ey, nx, ny, skip=None):
    """Tessellate the parallelogram origin + s*ex + t*ey (s,t in [0,1]) into nx*ny quads,
    two triangles each. `skip(i, j)` drops a quad (window openings)."""
    o, ex, ey = (np.asarray(a, dtype=np.float64) for a in (origin, ex, ey))
    tris = []
    for j in range(ny):
        for i in range(nx):
            if skip is not None and skip(i, j):
                continue
            p00 = o + ex * (i / nx) + ey * (j / ny)
            p10 = o + ex * ((i + 1) / nx) + ey * (j / ny)
            p01 = o + ex * (i / nx) + ey * ((j + 1) / ny)
            p11 = o + ex * ((i + 1) / nx) + ey * ((j + 1) / ny)
            tris.append((p00, p10, p11))
            tris.append((p00, p11, p01))
    return tris


def _box_pillar(cx, cy, w, h, segs):
    """Axis-aligned square pillar: four sides with `segs` vertical segments and a top cap."""
    x0, x1, y0, y1 = cx - w / 2, cx + w / 2, cy - w / 2, cy + w / 2
    tris = []
    tris += _quad_grid((x0, y0, 0), (x1 - x0, 0, 0), (0, 0, h), 1, segs)
    tris += _quad_grid((x1, y0, 0), (0, y1 - y0, 0), (0, 0, h), 1, segs)
    tris += _quad_grid((x1, y1, 0), (x0 - x1, 0, 0), (0, 0, h), 1, segs)
    tris += _quad_grid((x0, y1, 0), (0, y0 - y1, 0), (0, 0, h), 1, segs)
    tris += _quad_grid((x0, y0, h), (x1 - x0, 0, 0), (0, y1 - y0, 0), 1, 1)
    return tris


def _stone_tables(rng, n_bins, n_stone):
    k = rng.uniform(0.01, 0.05, size=(n_stone, n_bins))
    n = np.full((n_stone, n_bins), 1.6)
    rho = 1.0 - 10.0 * k
    return n, k, rho


def _glass_k_linear(lam_nm):
    """k(lambda) rising linearly from 1e-7 at 380 nm to 1e-6 at 780 nm."""
    return 1e-7 + (lam_nm - 380.0) / 400.0 * 9e-7


# ----------------------------------------------------------------------------------------------
# C1: the tiny box nave
# ----------------------------------------------------------------------------------------------

def nave_scene(n_bins: int = 8, seed: int = SCENE_SEED, lambda_min_nm: float = 380.0,
               lambda_max_nm: float = 780.0) -> Scene:
    """Box nave 20 x 10 x 8 m without a ceiling: floor and four walls tessellated at 1 m,
    a 2 x 3 m window opening (x in [9,11], z in [3,6]) in the y=0 wall closed by one glass
    quad (n=1.52, k linear 1e-7..1e-6, 5 mm), and 8 square pillars (0.6 m, 6 m tall, 50
    triangles each) in two rows of four, jittered +-0.5 m. Materials: 0 floor stone,
    1 wall/pillar stone, 2 glass."""
    rng = np.random.default_rng(seed)
    tris, mats = [], []

    def add(ts, m):
        tris.extend(ts)
        mats.extend([m] * len(ts))

    add(_quad_grid((0, 0, 0), (20, 0, 0), (0, 10, 0), 20, 10), 0)                       # floor
    window = lambda i, j: 9 <= i < 11 and 3 <= j < 6
    add(_quad_grid((0, 0, 0), (20, 0, 0), (0, 0, 8), 20, 8, skip=window), 1)          # y=0 wall
    add(_quad_grid((0, 10, 0), (20, 0, 0), (0, 0, 8), 20, 8), 1)                        # y=10 wall
    add(_quad_grid((0, 0, 0), (0, 10, 0), (0, 0, 8), 10, 8), 1)                         # x=0 wall
    add(_quad_grid((20, 0, 0), (0, 10, 0), (0, 0, 8), 10, 8), 1)                        # x=20 wall
    jit = rng.uniform(-0.5, 0.5, size=(8, 2))
    k = 0
    for row_y in (3.5, 6.5):
        for col_x in (4.0, 8.0, 12.0, 16.0):
            add(_box_pillar(col_x + jit[k, 0], row_y + jit[k, 1], 0.6, 6.0, 6), 1)
            k += 1
    add(_quad_grid((9, 0, 3), (2, 0, 0), (0, 0, 3), 1, 1), 2)                           # glass

    lam = bin_centres(n_bins, lambda_min_nm, lambda_max_nm)
    n_s, k_s, rho_s = _stone_tables(rng, n_bins, 2)
    n_tab = np.vstack([n_s, np.full((1, n_bins), 1.52)])
    k_tab = np.vstack([k_s, _glass_k_linear(lam)[None, :]])
    rho_tab = np.vstack([rho_s, np.zeros((1, n_bins))])
    verts = np.asarray(tris, dtype=np.float64).astype(np.float32)
    return Scene(
        verts=verts, mat=np.asarray(mats, dtype=np.uint16),
        mat_type=np.array([MAT_OPAQUE, MAT_OPAQUE, MAT_GLASS], dtype=np.int32),
        thickness_m=np.array([0.0, 0.0, 0.005], dtype=np.float32),
        n_tab=n_tab.astype(np.float32), k_tab=k_tab.astype(np.float32), rho_tab=rho_tab.astype(np.float32),
        lambda_min_nm=lambda_min_nm, lambda_max_nm=lambda_max_nm,
        sun_dir=sun_direction(35.0, -90.0), sun_E=sun_irradiance(n_bins, lambda_min_nm, lambda_max_nm),
        env=np.zeros(n_bins, dtype=np.float32), name="nave",
    ).check()


def nave_camera(width: int = 64, height: int = 64) -> Camera:
    return Camera(eye=(3.0, 8.0, 1.7), target=(12.0, 1.0, 1.5), up=(0.0, 0.0, 1.0), vfov_deg=60.0,
                  width=width, height=height)


# ----------------------------------------------------------------------------------------------
# small analytic scenes used by closed-form pins
# ----------------------------------------------------------------------------------------------

def plane_scene(n_bins=8, size=100.0, z=0.0, n=1.6, k=0.03, rho=0.7, sun_dir=(0.0, 0.0, 1.0),
                window=None, glass_n=1.52, glass_k=1e-6, glass_d=0.005, env=0.0,
                lambda_min_nm=380.0, lambda_max_nm=780.0) -> Scene:
    """One large opaque square at height z (two triangles) and optionally a glass quad
    `window=(zw, half)` centred above the origin at height zw."""
    s = size / 2
    tris = [((-s, -s, z), (s, -s, z), (s, s, z)), ((-s, -s, z), (s, s, z), (-s, s, z))]
    mats = [0, 0]
    if window is not None:
        zw, h = window
        tris += [((-h, -h, zw), (h, -h, zw), (h, h, zw)), ((-h, -h, zw), (h, h, zw), (-h, h, zw))]
        mats += [1, 1]
    B = n_bins
    return Scene(
        verts=np.asarray(tris, dtype=np.float32), mat=np.asarray(mats, dtype=np.uint16),
        mat_type=np.array([MAT_OPAQUE, MAT_GLASS], dtype=np.int32),
        thickness_m=np.array([0.0, glass_d], dtype=np.float32),
        n_tab=np.array([[n] * B, [glass_n] * B], dtype=np.float32),
        k_tab=np.array([[k] * B, [glass_k] * B], dtype=np.float32),
        rho_tab=np.array([[rho] * B, [0.0] * B], dtype=np.float32),
        lambda_min_nm=lambda_min_nm, lambda_max_nm=lambda_max_nm,
        sun_dir=np.asarray(sun_dir, dtype=np.float32) / np.float32(np.linalg.norm(sun_dir)),
        sun_E=sun_irradiance(B, lambda_min_nm, lambda_max_nm),
        env=np.full(B, env, dtype=np.float32), name="plane",
    ).check()


def furnace_scene(n_bins=8, seed=3, n_boxes=6) -> Scene:
    """Open white-furnace scene: a floor, two glass quads and a few boxes; every material is
    lossless and non-dispersive (k = 0, rho = 1), env = 1 and the sun is off."""
    rng = np.random.default_rng(seed)
    tris, mats = [], []
    tris += _quad_grid((-10, -10, 0), (20, 0, 0), (0, 20, 0), 4, 4)
    mats += [0] * (len(tris))
    for _ in range(n_boxes):
        cx, cy = rng.uniform(-6, 6, size=2)
        w, h = rng.uniform(0.5, 2.0), rng.uniform(0.5, 3.0)
        b = _box_pillar(cx, cy, w, h, 2)
        tris += b
        mats += [1] * len(b)
    for _ in range(2):
        cx, cy, cz = rng.uniform(-5, 5), rng.uniform(-5, 5), rng.uniform(1, 4)
        q = _quad_grid((cx - 1, cy, cz - 1), (2, 0, 0), (0, 0.5, 2), 1, 1)
        tris += q
        mats += [2] * len(q)
    B = n_bins
    return Scene(
        verts=np.asarray(tris, dtype=np.float32), mat=np.asarray(mats, dtype=np.uint16),
        mat_type=np.array([MAT_OPAQUE, MAT_OPAQUE, MAT_GLASS], dtype=np.int32),
        thickness_m=np.array([0.0, 0.0, 0.005], dtype=np.float32),
        n_tab=np.array([[1.6] * B, [1.3] * B, [1.52] * B], dtype=np.float32),
        k_tab=np.zeros((3, B), dtype=np.float32),
        rho_tab=np.array([[1.0] * B, [1.0] * B, [0.0] * B], dtype=np.float32),
        lambda_min_nm=380.0, lambda_max_nm=780.0,
        sun_dir=np.array([0, 0, 1], dtype=np.float32), sun_E=np.zeros(B, dtype=np.float32),
        env=np.ones(B, dtype=np.float32), name="furnace",
    ).check()


def random_soup(n_tri: int, seed: int = 11, extent: float = 10.0, size: float = 1.0, n_bins: int = 8) -> Scene:
    """Random triangles in a cube, for intersection tests (one opaque material)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0, extent, size=(n_tri, 1, 3))
    v = c + rng.normal(0, size, size=(n_tri, 3, 3))
    B = n_bins
    return Scene(
        verts=v.astype(np.float32), mat=np.zeros(n_tri, dtype=np.uint16),
        mat_type=np.array([MAT_OPAQUE], dtype=np.int32), thickness_m=np.zeros(1, dtype=np.float32),
        n_tab=np.full((1, B), 1.6, dtype=np.float32), k_tab=np.full((1, B), 0.03, dtype=np.float32),
        rho_tab=np.full((1, B), 0.7, dtype=np.float32), lambda_min_nm=380.0, lambda_max_nm=780.0,
        sun_dir=np.array([0, 0, 1], dtype=np.float32), sun_E=np.ones(B, dtype=np.float32),
        env=np.zeros(B, dtype=np.float32), name="soup",
    ).check()


def random_rays(n: int, seed: int = 5, lo=-2.0, hi=12.0, aim_lo=0.0, aim_hi=10.0):
    """Ray origins in a box around the soup, aimed at random points inside it.
    Returns float32 origins [n][3] and unit directions [n][3]."""
    rng = np.random.default_rng(seed)
    o = rng.uniform(lo, hi, size=(n, 3))
    a = rng.uniform(aim_lo, aim_hi, size=(n, 3))
    d = a - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)
