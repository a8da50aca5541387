"""Pins of the oracle's camera map and sampled directions, by outcomes the geometry fixes.

Every test renders with ``oracle.render`` and checks a value that follows from the scene alone:
  * pixel placement (the pinhole map with y = 0 at the top, the W/H aspect, jitter inside the
    pixel): a small quad placed in the footprint of one pixel darkens exactly that pixel;
  * the cosine lobe: the fraction of cosine-weighted directions that leave through a square
    opening is the view factor of a differential area to a parallel rectangle (a closed form of
    radiative transfer), for several orientations of the surface normal;
  * the mirror lobe: with zero albedo every path takes the mirror bounce, which must leave
    through a small opening at the reflected point, giving exactly F(theta) per bin.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen


def _scene(tris, mats, mat_type, n_tab, k_tab, rho_tab, env=1.0, sun_dir=(0.0, 0.0, 1.0)):
    B = len(n_tab[0])
    return scenegen.Scene(
        verts=np.asarray(tris, dtype=np.float32), mat=np.asarray(mats, dtype=np.uint16),
        mat_type=np.asarray(mat_type, dtype=np.int32), thickness_m=np.full(len(mat_type), 0.005, dtype=np.float32),
        n_tab=np.asarray(n_tab, dtype=np.float32), k_tab=np.asarray(k_tab, dtype=np.float32),
        rho_tab=np.asarray(rho_tab, dtype=np.float32), lambda_min_nm=380.0, lambda_max_nm=780.0,
        sun_dir=np.asarray(sun_dir, dtype=np.float32), sun_E=np.zeros(B, dtype=np.float32),
        env=np.full(B, env, dtype=np.float32), name="pin").check()


def _quad(c00, c10, c11, c01):
    return [(c00, c10, c11), (c00, c11, c01)]


def _rotation(axis, angle_deg):
    a = np.asarray(axis, dtype=np.float64)
    a /= np.linalg.norm(a)
    t = math.radians(angle_deg)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(t) * K + (1 - math.cos(t)) * K @ K


# ---------------------------------------------------------------------------------------------
# pixel placement
# ---------------------------------------------------------------------------------------------

def _pixel_quad(L, tan_half, W, H, x0, y0, margin):
    """Quad on the plane x = L (camera at the origin looking along +x, right = -y, up = +z)
    covering the screen window of pixel (x0, y0) shrunk by `margin` (in pixels) on every side.
    Screen coordinates of a point (L, -L sx, L sy) are (sx, sy); pixel x spans
    sx in (2x/W - 1) t W/H .. (2(x+1)/W - 1) t W/H, and row y spans sy = (1 - 2y/H) t downward."""
    sx = [(2.0 * (x0 + j) / W - 1.0) * tan_half * W / H for j in (margin, 1.0 - margin)]
    sy = [(1.0 - 2.0 * (y0 + j) / H) * tan_half for j in (1.0 - margin, margin)]
    pt = lambda a, b: (L, -L * a, L * b)
    return _quad(pt(sx[0], sy[0]), pt(sx[1], sy[0]), pt(sx[1], sy[1]), pt(sx[0], sy[1]))


@pytest.mark.parametrize("W,H", [(16, 8), (9, 14)])
def test_pixel_placement_rows_from_top_aspect_and_jitter(W, H):
    """A quad in the footprint of pixel (x0, y0) (shrunk by 2 % of a pixel per side) darkens that
    pixel only: with depth 1, no sun and env = 1 a pixel is the fraction of its samples that
    escape. Neighbouring pixels must stay exactly 1 -- a half-pixel jitter offset, a flipped row
    order or an aspect ratio taken as H/W would put samples of other pixels on the quads."""
    vfov = 40.0
    t = math.tan(math.radians(vfov / 2))
    targets = [(3, 1), (W - 2, H - 3)]
    tris = []
    for (x0, y0) in targets:
        tris += _pixel_quad(10.0, t, W, H, x0, y0, 0.02)
    B = 2
    sc = _scene(tris, [0] * len(tris), [0], [[1.6] * B], [[0.0] * B], [[0.5] * B])
    cam = scenegen.Camera(eye=(0.0, 0.0, 0.0), target=(10.0, 0.0, 0.0), up=(0.0, 0.0, 1.0), vfov_deg=vfov,
                          width=W, height=H)
    res = oracle.render(sc, cam, spp=64, max_depth=1, seed=3)
    img = res.image[0]
    dark = np.zeros((H, W), dtype=bool)
    for (x0, y0) in targets:
        dark[y0, x0] = True
        # the quad covers the central 96 % x 96 % of the pixel: about 92 % of its samples hit it
        assert 0.0 <= img[y0, x0] < 0.25, (x0, y0, img[y0, x0])
    np.testing.assert_array_equal(img[~dark], 1.0)
    np.testing.assert_array_equal(res.image[1], res.image[0])


# ---------------------------------------------------------------------------------------------
# cosine lobe: view factor of a square opening
# ---------------------------------------------------------------------------------------------

def _view_factor_corner(X, Y):
    """View factor from a differential area to a parallel rectangle X c by Y c at distance c
    whose corner lies on the area's normal (standard closed form of radiative exchange)."""
    a, b = math.sqrt(1 + X * X), math.sqrt(1 + Y * Y)
    return (X / a * math.atan(Y / a) + Y / b * math.atan(X / b)) / (2 * math.pi)


def test_view_factor_closed_form_limits():
    # an infinite quadrant is a quarter of the cosine-weighted hemisphere
    assert abs(_view_factor_corner(1e7, 1e7) - 0.25) < 1e-6
    # numerical integration of cos(theta)/pi over the square opening at unit distance
    n = 600
    g = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(g, g)
    num = np.sum(1.0 / (math.pi * (1 + X**2 + Y**2) ** 2)) / n**2
    assert abs(num - _view_factor_corner(1.0, 1.0)) < 1e-5


def _opening_scene(R, c, half, height, rho, big=3000.0):
    """Floor (material 0, normal R z) through the origin, a roof at `height` along R z with a
    square opening of half-width `half` centred above the point c = (cx, cy, 0) (material 1,
    black: rho 0, n = 1 so F = 0 at every angle: a path ending on it gathers nothing), all
    rotated by R. c lies off the floor's diagonal, so the camera ray's hit is not on an edge."""
    P = lambda x, y, z: tuple(R @ np.array([x, y, z], dtype=np.float64))
    h, s, z = half, big, height
    cx, cy = c[0], c[1]
    tris = _quad(P(-s, -s, 0), P(s, -s, 0), P(s, s, 0), P(-s, s, 0))
    mats = [0, 0]
    roof = []
    roof += _quad(P(-s, -s, z), P(s, -s, z), P(s, cy - h, z), P(-s, cy - h, z))                  # below the opening
    roof += _quad(P(-s, cy + h, z), P(s, cy + h, z), P(s, s, z), P(-s, s, z))                    # above it
    roof += _quad(P(-s, cy - h, z), P(cx - h, cy - h, z), P(cx - h, cy + h, z), P(-s, cy + h, z))  # left
    roof += _quad(P(cx + h, cy - h, z), P(s, cy - h, z), P(s, cy + h, z), P(cx + h, cy + h, z))    # right
    tris += roof
    mats += [1] * len(roof)
    B = 2
    return _scene(tris, mats, [0, 0], [[1.6] * B, [1.0] * B], [[0.0] * B, [0.0] * B], [[rho] * B, [0.0] * B])


@pytest.mark.parametrize("axis,angle", [((1, 0, 0), 0.0), ((0.3, -0.8, 0.5), 37.0), ((1, 0.2, 0), 131.0)])
def test_cosine_lobe_escape_fraction_is_the_view_factor(axis, angle):
    """Depth 2, env 1, no sun: the camera looks straight down onto the floor through a tiny
    field. The mirror bounce (probability P = F / (F + (1 - F) rho)) leaves through the opening
    with weight F / P; a diffuse bounce leaves with weight (1 - F) rho / (1 - P) exactly when its
    cosine-sampled direction passes the opening. So E[L] = F + (1 - F) rho Fv, Fv the view factor
    of the opening. Orientations: normal +z, a generic tilt, and a normal with negative z (the
    two branches of the orthonormal frame built around the normal)."""
    R = _rotation(axis, angle)
    half, height, rho = 1.0, 1.0, 0.8
    c = np.array([0.31, 0.07, 0.0])
    sc = _opening_scene(R, c, half, height, rho)
    n_w = R @ np.array([0.0, 0.0, 1.0])
    eye = tuple(R @ (c + np.array([0.0, 0.0, 0.5])))
    up = tuple(R @ np.array([0.0, 1.0, 0.0]))
    W = H = 32
    spp = 400
    cam = scenegen.Camera(eye=eye, target=tuple(R @ c), up=up, vfov_deg=1e-4, width=W, height=H)
    res = oracle.render(sc, cam, spp=spp, max_depth=2, seed=11)
    F = ((float(np.float32(1.6)) - 1) / (float(np.float32(1.6)) + 1)) ** 2
    rho32 = float(np.float32(rho))
    Fv = 4 * _view_factor_corner(half / height, half / height)
    expect = F + (1 - F) * rho32 * Fv
    A = F + (1 - F) * rho32                  # every escaping sample carries this weight
    p = expect / A
    N = W * H * spp
    sigma = A * math.sqrt(p * (1 - p) / N)
    got = res.image.mean(axis=(1, 2))
    # a few diffuse rays pass within rounding of the opening's edges (flagged, still counted)
    assert res.stats["tied_paths"] < 1e-3 * N
    assert n_w[2] != 0.0
    for j in range(2):
        assert abs(got[j] - expect) <= 5 * sigma, (axis, angle, got[j], expect, sigma)
    # a uniform-hemisphere lobe would escape with the solid-angle fraction instead: far away
    assert abs(Fv - 0.5541) < 1e-3


# ---------------------------------------------------------------------------------------------
# mirror lobe
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("axis,angle", [((1, 0, 0), 0.0), ((-0.4, 0.7, 0.2), 58.0)])
def test_mirror_lobe_leaves_through_the_reflected_opening(axis, angle):
    """Albedo 0 makes the mirror lobe certain (P = 1, weight F). The camera ray meets the floor
    at 45 degrees; the reflected ray must pass a 10 cm opening in the roof centred on the
    reflected point, 1 m further along x at the roof's height. A basement plane below catches a ray that would pass through the
    floor, and the roof blocks the other reflections. Pixel value = F_j(45 deg) per bin."""
    R = _rotation(axis, angle)
    P = lambda x, y, z: tuple(R @ np.array([x, y, z], dtype=np.float64))
    s, h = 100.0, 0.05
    tris = _quad(P(-s, -s, 0), P(s, -s, 0), P(s, s, 0), P(-s, s, 0))              # mirror floor
    tris += _quad(P(-s, -s, -1), P(s, -s, -1), P(s, s, -1), P(-s, s, -1))          # basement
    ox, oy = 0.31, 0.07              # floor hit point, off the floor's diagonal
    cx, cy = ox + 1.0, oy
    roof = []
    roof += _quad(P(-s, -s, 1), P(s, -s, 1), P(s, cy - h, 1), P(-s, cy - h, 1))
    roof += _quad(P(-s, cy + h, 1), P(s, cy + h, 1), P(s, s, 1), P(-s, s, 1))
    roof += _quad(P(-s, cy - h, 1), P(cx - h, cy - h, 1), P(cx - h, cy + h, 1), P(-s, cy + h, 1))
    roof += _quad(P(cx + h, cy - h, 1), P(s, cy - h, 1), P(s, cy + h, 1), P(cx + h, cy + h, 1))
    tris += roof
    mats = [0, 0, 1, 1] + [1] * len(roof)
    n_tab, k_tab = [[1.5, 1.7, 2.2], [1.0] * 3], [[0.01, 0.2, 1.5], [0.0] * 3]
    sc = _scene(tris, mats, [0, 0], n_tab, k_tab, [[0.0] * 3, [0.0] * 3])
    cam = scenegen.Camera(eye=P(ox - 0.5, oy, 0.5), target=P(ox, oy, 0.0), up=tuple(R[:, 2]), vfov_deg=1e-4,
                          width=3, height=2)
    res = oracle.render(sc, cam, spp=4, max_depth=2, seed=5)
    c45 = math.cos(math.radians(45.0))
    f32 = lambda x: float(np.float32(x))
    exp = np.array([oracle.fresnel(f32(n), f32(k), c45) for n, k in zip(n_tab[0], k_tab[0])])
    assert res.stats["tied_paths"] == 0
    np.testing.assert_allclose(res.image.reshape(3, -1), np.repeat(exp[:, None], 6, axis=1), rtol=2e-5)
    # the expected values are far from zero, so a ray blocked by the roof cannot pass
    assert exp.min() > 0.03
