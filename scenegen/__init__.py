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
    # spectral transmittance maps of glass (optional): per-triangle texture coordinates, the maps
    # (internal transmittance at normal incidence per texel and bin, in [0, 1]) and the map of
    # each material (-1: none; the glass then absorbs by its k)
    uv: np.ndarray | None = None         # float32 [N][3][2]
    textures: list | None = None         # list of float32 [h][w][B]
    mat_tex: np.ndarray | None = None    # int32 [n_mat]

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
        if self.textures is not None:
            assert self.uv is not None and self.mat_tex is not None
            self.uv = np.ascontiguousarray(self.uv, dtype=np.float32)
            assert self.uv.shape == (self.n_tri, 3, 2)
            self.mat_tex = np.ascontiguousarray(self.mat_tex, dtype=np.int32)
            assert self.mat_tex.shape == (self.n_mat,) and self.mat_tex.max() < len(self.textures)
            self.textures = [np.ascontiguousarray(t, dtype=np.float32) for t in self.textures]
            for t in self.textures:
                assert t.ndim == 3 and t.shape[2] == self.n_bins and t.min() >= 0 and t.max() <= 1
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
# the tiny box nave
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


def glass_map(rng, lam_nm, d_m, width=12, height=16, n_spots=6):
    """A seeded stand-in for a measured map of medieval glass (section 3: the spectral
    transmittance measured at points of the samples, accessed by texture coordinates): internal
    transmittance at normal incidence tau0 = exp(-4 pi k d / lambda) with k varying smoothly over
    the pane (a few Gaussian absorption bumps whose strength drifts across it) and darker round
    spots (clusters of micro-bubbles and inclusions) a few texels wide. Returns float32
    [height][width][B] in (0, 1]."""
    B = len(lam_nm)
    s = (np.arange(width) + 0.5) / width
    t = (np.arange(height) + 0.5) / height
    S, T = np.meshgrid(s, t)
    k = np.full((height, width, B), 1e-7)
    for _ in range(rng.integers(1, 4)):
        a = rng.uniform(2e-6, 2e-5)
        mu, sig = rng.uniform(400, 760), rng.uniform(15, 60)
        drift = 1.0 + 0.3 * np.sin(2 * np.pi * (rng.uniform() + S * rng.uniform(0.3, 1.0) + T * rng.uniform(0.2, 0.8)))
        k += a * drift[..., None] * np.exp(-0.5 * ((lam_nm[None, None, :] - mu) / sig) ** 2)
    # spots a few texels wide: a map only resolves features larger than its texel spacing, and
    # its log-transmittance gradient sets how much the FP32 rounding of path vertices moves it
    for _ in range(n_spots):
        cs, ct, r = rng.uniform(0, 1), rng.uniform(0, 1), rng.uniform(0.15, 0.3)
        k += 6e-6 * np.exp(-0.5 * (((S - cs) ** 2 + (T - ct) ** 2) / r**2))[..., None]
    return np.exp(-4 * np.pi * k * d_m / (lam_nm * 1e-9)).astype(np.float32)


def quad_uv(n_tri):
    """Texture coordinates of _quad_grid quads taken one by one ((0,0) (1,0) (1,1) | (0,0) (1,1) (0,1))
    for n_tri // 2 quads, others 0."""
    q = np.array([[(0, 0), (1, 0), (1, 1)], [(0, 0), (1, 1), (0, 1)]], dtype=np.float32)
    return np.tile(q, (n_tri // 2, 1, 1))


def with_glass_maps(sc: Scene, seed=0x6A55, width=12, height=16) -> Scene:
    """The scene with a seeded transmittance map on every glass material and texture coordinates
    (0..1 over each glass quad, whose two triangles come in _quad_grid order). Opaque triangles get
    zero texture coordinates (unused)."""
    import dataclasses
    rng = np.random.default_rng(seed)
    lam = bin_centres(sc.n_bins, sc.lambda_min_nm, sc.lambda_max_nm)
    uv = np.zeros((sc.n_tri, 3, 2), dtype=np.float32)
    mat_tex = np.full(sc.n_mat, -1, dtype=np.int32)
    tex = []
    for m in range(sc.n_mat):
        if sc.mat_type[m] != MAT_GLASS:
            continue
        idx = np.nonzero(sc.mat == m)[0]
        assert len(idx) % 2 == 0
        uv[idx] = quad_uv(len(idx))
        mat_tex[m] = len(tex)
        tex.append(glass_map(rng, lam, float(sc.thickness_m[m]), width, height))
    return dataclasses.replace(sc, uv=uv, textures=tex, mat_tex=mat_tex).check()


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


def caustic_scene(n_bins=3, floor_n=(1.5, 1.9, 2.6), floor_rho=0.0, sun_zenith_deg=30.0, single=False,
                  pane_k=0.0) -> Scene:
    """A caustic under a window: a horizontal glass pane (z = 3, 2 m x 2 m, centred near the
    origin), a large floor at z = 0 (albedo floor_rho; zero albedo makes its mirror lobe certain),
    a diffuse receiver wall x = -6 facing +x, and the sun sun_zenith_deg from the zenith in the x-z
    plane. Sunlight through the pane and off the floor meets the wall. floor_n gives the floor's
    real index per bin (the first n_bins entries, repeated if shorter). With single=True the floor
    and the wall are one large triangle each (no shared edge inside the lit region)."""
    th = math.radians(sun_zenith_deg)
    B = n_bins

    def quad(c00, c10, c11, c01):
        return [(c00, c10, c11), (c00, c11, c01)]

    tris, mats = [], []
    tris += quad((-0.97, -1.03, 3), (1.03, -1.03, 3), (1.03, 0.97, 3), (-0.97, 0.97, 3))
    mats += [0, 0]
    s = 60.0
    if single:
        tris += [((-3 * s, -3 * s, 0), (3 * s, -3 * s, 0), (0, 3 * s, 0))]
        mats += [1]
        tris += [((-6, -3 * s, -1), (-6, 3 * s, -1), (-6, 0, 3 * s))]
        mats += [2]
    else:
        tris += quad((-s, -s, 0), (s, -s, 0), (s, s, 0), (-s, s, 0))
        mats += [1, 1]
        tris += quad((-6, -s, -1), (-6, s, -1), (-6, s, 30), (-6, -s, 30))
        mats += [2, 2]
    fn = [floor_n[j % len(floor_n)] for j in range(B)]
    sun_E = np.array([1.0, 0.8, 0.6][:B] + [0.7] * max(0, B - 3), dtype=np.float32)
    return Scene(
        verts=np.asarray(tris, dtype=np.float32), mat=np.asarray(mats, dtype=np.uint16),
        mat_type=np.array([MAT_GLASS, MAT_OPAQUE, MAT_OPAQUE], dtype=np.int32),
        thickness_m=np.array([0.004, 0, 0], dtype=np.float32),
        n_tab=np.array([[1.52] * B, fn, [1.6] * B], dtype=np.float32),
        k_tab=np.array([[pane_k] * B, [0.1] * B, [0.02] * B], dtype=np.float32),
        rho_tab=np.array([[0.0] * B, [floor_rho] * B, [0.8] * B], dtype=np.float32),
        lambda_min_nm=380.0, lambda_max_nm=780.0,
        sun_dir=np.array([math.sin(th), 0.0, math.cos(th)], dtype=np.float32),
        sun_E=sun_E, env=np.zeros(B, dtype=np.float32), name="caustic",
    ).check()


def window_box_scene(n_bins=4, size=(4.0, 4.0, 3.0), window=(1.2, 1.2), rho=0.6, sun_zenith_deg=25.0,
                     sun_azimuth_deg=30.0, n=1.5, k=0.02, glass_k=2e-7) -> Scene:
    """A closed room lit only through a ceiling window: floor, four walls and a ceiling of one
    diffuse material (index n + ik, albedo rho, constant over the bins), the ceiling pierced by a
    centred glass pane of the given size; the sun enters only through the pane. Floor at z = 0,
    the room spans [0, sx] x [0, sy] x [0, sz]."""
    sx, sy, sz = size
    wx, wy = window
    x0, x1 = (sx - wx) / 2, (sx + wx) / 2
    y0, y1 = (sy - wy) / 2, (sy + wy) / 2
    tris, mats = [], []

    def quad(c00, c10, c11, c01, m):
        tris.extend([(c00, c10, c11), (c00, c11, c01)])
        mats.extend([m, m])

    quad((0, 0, 0), (sx, 0, 0), (sx, sy, 0), (0, sy, 0), 0)            # floor
    quad((0, 0, 0), (0, sy, 0), (0, sy, sz), (0, 0, sz), 0)            # walls
    quad((sx, 0, 0), (sx, 0, sz), (sx, sy, sz), (sx, sy, 0), 0)
    quad((0, 0, 0), (0, 0, sz), (sx, 0, sz), (sx, 0, 0), 0)
    quad((0, sy, 0), (sx, sy, 0), (sx, sy, sz), (0, sy, sz), 0)
    # ceiling around the opening: four rectangles
    quad((0, 0, sz), (0, y0, sz), (sx, y0, sz), (sx, 0, sz), 0)
    quad((0, y1, sz), (0, sy, sz), (sx, sy, sz), (sx, y1, sz), 0)
    quad((0, y0, sz), (0, y1, sz), (x0, y1, sz), (x0, y0, sz), 0)
    quad((x1, y0, sz), (x1, y1, sz), (sx, y1, sz), (sx, y0, sz), 0)
    quad((x0, y0, sz), (x1, y0, sz), (x1, y1, sz), (x0, y1, sz), 1)   # the pane
    B = n_bins
    return Scene(
        verts=np.asarray(tris, dtype=np.float32), mat=np.asarray(mats, dtype=np.uint16),
        mat_type=np.array([MAT_OPAQUE, MAT_GLASS], dtype=np.int32),
        thickness_m=np.array([0.0, 0.005], dtype=np.float32),
        n_tab=np.array([[n] * B, [1.52] * B], dtype=np.float32),
        k_tab=np.array([[k] * B, [glass_k] * B], dtype=np.float32),
        rho_tab=np.array([[rho] * B, [0.0] * B], dtype=np.float32),
        lambda_min_nm=380.0, lambda_max_nm=780.0,
        sun_dir=sun_direction(90.0 - sun_zenith_deg, sun_azimuth_deg),
        sun_E=sun_irradiance(B), env=np.zeros(B, dtype=np.float32), name="window_box",
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


# ----------------------------------------------------------------------------------------------
# procedural church (about 1M triangles, or 10M for the large configuration)
# ----------------------------------------------------------------------------------------------

def _grid_tris(P, skip=None):
    """Two triangles per cell of a point lattice P [nu+1][nv+1][3]; skip [nu][nv] drops cells."""
    a, b = P[:-1, :-1], P[1:, :-1]
    c, d = P[1:, 1:], P[:-1, 1:]
    t1 = np.stack([a, b, c], axis=-2)
    t2 = np.stack([a, c, d], axis=-2)
    t = np.stack([t1, t2], axis=2)          # [nu][nv][2][3][3]
    if skip is not None:
        t = t[~skip]
    return t.reshape(-1, 3, 3)


def _lattice(origin, ex, ey, nu, nv):
    u = np.linspace(0.0, 1.0, nu + 1)[:, None, None]
    v = np.linspace(0.0, 1.0, nv + 1)[None, :, None]
    return np.asarray(origin, float) + u * np.asarray(ex, float) + v * np.asarray(ey, float)


def _pointed_arch(width, rise, n):
    """Two-arc pointed arch over y in [0, width], springing at z = 0, apex at (width/2, rise).
    Returns n+1 points (y, z) along the curve, uniform in angle on each arc."""
    half = width / 2.0
    R = (rise**2 + half**2) / (2 * half)       # arc radius: R^2 = rise^2 + (R - half)^2
    phi_max = math.acos((R - half) / R)
    m = n // 2
    phi = np.linspace(0.0, phi_max, m + 1)
    left = np.column_stack([R - R * np.cos(phi), R * np.sin(phi)])
    right = np.column_stack([width - left[::-1, 0], left[::-1, 1]])
    return np.vstack([left, right[1:]])


def _sweep_square(path, half, n_seg):
    """Square tube of half-width `half` swept along a polyline path [k][3] (4 faces)."""
    path = np.asarray(path, float)
    tng = np.gradient(path, axis=0)
    tng /= np.linalg.norm(tng, axis=1, keepdims=True)
    ref = np.where(np.abs(tng[:, 2:3]) < 0.9, np.array([[0, 0, 1.0]]), np.array([[1.0, 0, 0]]))
    n1 = np.cross(tng, ref)
    n1 /= np.linalg.norm(n1, axis=1, keepdims=True)
    n2 = np.cross(tng, n1)
    corners = [n1 + n2, -n1 + n2, -n1 - n2, n1 - n2, n1 + n2]
    ring = np.stack([path + half * c for c in corners], axis=1)   # [k][5][3]
    return _grid_tris(ring)


def _cylinder(cx, cy, r, h, n_around, n_up):
    th = np.linspace(0.0, 2 * math.pi, n_around + 1)
    z = np.linspace(0.0, h, n_up + 1)
    P = np.stack(np.broadcast_arrays(cx + r * np.cos(th)[:, None], cy + r * np.sin(th)[:, None], z[None, :]), -1)
    return _grid_tris(P)


def _window_spectrum(rng, lam):
    k = np.full_like(lam, 1e-7)
    for _ in range(rng.integers(1, 4)):
        a, mu, sg = rng.uniform(2e-6, 2e-5), rng.uniform(400, 760), rng.uniform(15, 60)
        k += a * np.exp(-((lam - mu) ** 2) / (2 * sg**2))
    return k


def church_scene(n_bins=40, target_tris=1_000_000, seed=SCENE_SEED, length=60.0, width=14.0, wall_h=14.0,
                 rise=10.0, n_bays=10, tiers=2, lambda_min_nm=380.0, lambda_max_nm=780.0) -> Scene:
    """Procedural church: a nave `length` x `width` m whose side walls (height wall_h) carry a
    pointed two-arc barrel vault of the given rise, transverse and diagonal vault ribs at each
    bay, two rows of cylindrical columns, and tiers x n_bays window openings per side closed by
    glass quads with per-window Gaussian-bump absorption spectra. The tessellation density is
    scaled so that the triangle count lands near `target_tris` (the exact count is recorded in
    `info`). Materials: 0 floor, 1 walls, 2 columns, 3 vault and ribs (stone), 4.. glass."""
    rng = np.random.default_rng(seed)
    bay = length / n_bays
    win_w = min(1.6, 0.4 * bay)
    tier_z = [(3.0, 8.0), (9.5, 13.0)][:tiers] if tiers <= 2 else [
        (1.0 + i * (wall_h - 2) / tiers, 1.0 + (i + 0.8) * (wall_h - 2) / tiers) for i in range(tiers)]

    def counts(s):
        fx = max(1, int(round(length * s)))                    # along the nave
        fy = max(1, int(round(width * s)))
        wz = max(1, int(round(wall_h * s)))
        ez = max(1, int(round((wall_h + rise) * s)))
        va = max(2, 2 * int(round(0.6 * (rise + width) * s)))  # around the vault arch (even)
        ca = max(6, int(round(2 * math.pi * 0.6 * s * 0.9)))   # around a column
        cu = max(1, int(round(wall_h * s * 0.9)))
        rs = max(4, int(round((rise + width) * s * 0.5)))      # rib segments
        return fx, fy, wz, ez, va, ca, cu, rs

    def n_tris(s):
        fx, fy, wz, ez, va, ca, cu, rs = counts(s)
        return (2 * fx * fy + 2 * 2 * fx * wz + 2 * 2 * fy * ez + 2 * fx * va + 2 * n_bays * 2 * ca * cu
                + (n_bays + 1 + 2 * n_bays) * 8 * rs)

    lo_s, hi_s = 0.5, 200.0
    for _ in range(60):
        mid = math.sqrt(lo_s * hi_s)
        lo_s, hi_s = (mid, hi_s) if n_tris(mid) < target_tris else (lo_s, mid)
    fx, fy, wz, ez, va, ca, cu, rs = counts(lo_s)

    parts, mats = [], []

    def add(t, m):
        parts.append(np.asarray(t, float).reshape(-1, 3, 3))
        mats.append(np.full(len(parts[-1]), m, dtype=np.int64))

    add(_grid_tris(_lattice((0, 0, 0), (length, 0, 0), (0, width, 0), fx, fy)), 0)
    # side walls with window openings (cells whose centre falls in an opening are dropped)
    uc = (np.arange(fx) + 0.5) * length / fx
    vc = (np.arange(wz) + 0.5) * wall_h / wz
    skip = np.zeros((fx, wz), dtype=bool)
    windows = []
    for side_y in (0.0, width):
        for b in range(n_bays):
            xc = (b + 0.5) * bay
            for (z0, z1) in tier_z:
                # snap the opening to the wall lattice so the glass exactly fills it
                i0 = int(np.floor((xc - win_w / 2) * fx / length + 0.5))
                i1 = max(i0 + 1, int(np.floor((xc + win_w / 2) * fx / length + 0.5)))
                j0 = int(np.floor(z0 * wz / wall_h + 0.5))
                j1 = max(j0 + 1, int(np.floor(z1 * wz / wall_h + 0.5)))
                windows.append((side_y, i0 * length / fx, i1 * length / fx, j0 * wall_h / wz, j1 * wall_h / wz,
                                (i0, i1, j0, j1)))
    for side_y in (0.0, width):
        sk = np.zeros((fx, wz), dtype=bool)
        for (sy, x0, x1, z0, z1, (i0, i1, j0, j1)) in windows:
            if sy == side_y:
                sk[i0:i1, j0:j1] = True
        add(_grid_tris(_lattice((0, side_y, 0), (length, 0, 0), (0, 0, wall_h), fx, wz), skip=sk), 1)
    # end walls up to the vault apex
    for side_x in (0.0, length):
        add(_grid_tris(_lattice((side_x, 0, 0), (0, width, 0), (0, 0, wall_h + rise), fy, ez)), 1)
    # columns: two rows, one per bay
    for b in range(n_bays):
        xc = (b + 0.5) * bay
        for yc in (0.18 * width, 0.82 * width):
            add(_cylinder(xc, yc, 0.6, wall_h, ca, cu), 2)
    # pointed barrel vault
    arch = _pointed_arch(width, rise, va)
    P = np.stack(np.broadcast_arrays(np.linspace(0, length, fx + 1)[:, None], arch[None, :, 0],
                                     wall_h + arch[None, :, 1]), -1)
    add(_grid_tris(P), 3)
    # transverse ribs at the bay boundaries, diagonal ribs across each bay (hanging under the vault)
    rib = _pointed_arch(width, rise, 2 * rs)
    for b in range(n_bays + 1):
        x = b * bay
        path = np.column_stack([np.full(len(rib), x), rib[:, 0], wall_h + rib[:, 1] - 0.2])
        add(_sweep_square(path, 0.15, len(path) - 1), 3)
    for b in range(n_bays):
        for flip in (False, True):
            s = np.linspace(0.0, 1.0, 2 * rs + 1)
            y = s * width
            x = b * bay + (1 - s if flip else s) * bay
            z = wall_h + np.interp(y, rib[:, 0], rib[:, 1]) - 0.25
            add(_sweep_square(np.column_stack([x, y, z]), 0.12, len(s) - 1), 3)
    # glass quads
    for wi, (sy, x0, x1, z0, z1, _) in enumerate(windows):
        add(_grid_tris(_lattice((x0, sy, z0), (x1 - x0, 0, 0), (0, 0, z1 - z0), 1, 1)), 4 + wi)

    verts = np.concatenate(parts).astype(np.float32)
    mat = np.concatenate(mats).astype(np.uint16)
    lam = bin_centres(n_bins, lambda_min_nm, lambda_max_nm)
    n_glass = len(windows)
    n_s, k_s, rho_s = _stone_tables(rng, n_bins, 4)
    k_g = np.stack([_window_spectrum(rng, lam) for _ in range(n_glass)])
    n_tab = np.vstack([n_s, np.full((n_glass, n_bins), 1.52)])
    k_tab = np.vstack([k_s, k_g])
    rho_tab = np.vstack([rho_s, np.zeros((n_glass, n_bins))])
    n_mat = 4 + n_glass
    return Scene(
        verts=verts, mat=mat,
        mat_type=np.array([MAT_OPAQUE] * 4 + [MAT_GLASS] * n_glass, dtype=np.int32),
        thickness_m=np.array([0.0] * 4 + [0.005] * n_glass, dtype=np.float32),
        n_tab=n_tab.astype(np.float32), k_tab=k_tab.astype(np.float32), rho_tab=rho_tab.astype(np.float32),
        lambda_min_nm=lambda_min_nm, lambda_max_nm=lambda_max_nm,
        sun_dir=sun_direction(35.0, -75.0), sun_E=sun_irradiance(n_bins, lambda_min_nm, lambda_max_nm),
        env=np.zeros(n_bins, dtype=np.float32), name="church",
        info=dict(n_tri=int(len(verts)), n_windows=n_glass, n_mat=n_mat, density=lo_s, length=length, width=width,
                  wall_h=wall_h, rise=rise, n_bays=n_bays),
    ).check()


def church_camera(width=1920, height=1080, length=60.0, nave_w=14.0) -> Camera:
    return Camera(eye=(2.0, 0.5 * nave_w, 1.7), target=(0.66 * length, 0.36 * nave_w, 9.0), up=(0.0, 0.0, 1.0),
                  vfov_deg=60.0, width=width, height=height)


RESOLUTIONS = [(256, 256), (512, 512), (640, 480), (800, 600), (1024, 768)]


def batch_views(n_views=32, seed=VIEW_SEED, length=60.0, width=14.0):
    """Seeded cameras inside the nave: eye height 1.2-2.5 m, yaw U[0, 360), pitch U[-10, 40] deg,
    vfov 60, resolution from RESOLUTIONS, spp uniform in 4..64."""
    rng = np.random.default_rng(seed)
    cams, spps = [], []
    for _ in range(n_views):
        eye = np.array([rng.uniform(1.0, length - 1.0), rng.uniform(1.5, width - 1.5), rng.uniform(1.2, 2.5)])
        yaw, pitch = math.radians(rng.uniform(0, 360)), math.radians(rng.uniform(-10, 40))
        d = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
        w, h = RESOLUTIONS[rng.integers(len(RESOLUTIONS))]
        cams.append(Camera(eye=tuple(eye), target=tuple(eye + d), up=(0.0, 0.0, 1.0), vfov_deg=60.0, width=w,
                           height=h))
        spps.append(int(rng.integers(4, 65)))
    return cams, spps
