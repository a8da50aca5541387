"""Pins of the oracle's spectral transmittance maps of glass (section 3: a map of spectral
transmittance measured at points of the medieval samples, read through texture coordinates).

  * A map holding exp(-4 pi k d / lambda) in every texel reproduces the glass that absorbs by k.
  * The direct term under a textured window (sun overhead, camera looking straight down at a
    point of the floor) is the closed form (1 - F0) rho / pi E T_slab(tau0) with tau0 read at the
    point's texture coordinates: a texel's own value at its centre, the mean of two texels
    midway between their centres, the mean of the last and the first texel on the map's
    periodic seam, on both triangles of the quad.
  * At a textured glass vertex the path estimate averages to R + T of the slab under env = 1.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import scenegen

f32 = lambda x: float(np.float32(x))


def _window_scene(tex, zw=2.0, half=1.0, env=0.0, sun=(0.0, 0.0, 1.0), floor=True, uv_scale=1.0, uv_shift=0.0):
    """Opaque floor z = 0 (if floor) under a glass quad z = zw over [-half, half]^2 whose two
    triangles carry texture coordinates uv_shift + uv_scale (0,0) (1,0) (1,1) | (0,0) (1,1) (0,1)."""
    B = tex.shape[2]
    sc = scenegen.plane_scene(n_bins=B, n=1.6, k=0.02, rho=0.8, sun_dir=sun, window=(zw, half), glass_k=3e-6,
                              env=env)
    if not floor:
        sc = dataclasses.replace(sc, verts=sc.verts[2:], mat=sc.mat[2:])
    uv = np.zeros((sc.n_tri, 3, 2), dtype=np.float32)
    uv[-2:] = uv_shift + uv_scale * scenegen.quad_uv(2)
    return dataclasses.replace(sc, uv=uv, textures=[tex], mat_tex=np.array([-1, 0], dtype=np.int32)).check()


def _nee_at(sc, x, y, zw):
    cam = scenegen.Camera(eye=(x, y, 0.5 * zw), target=(x, y, 0.0), up=(0, 1, 0), vfov_deg=1e-7, width=1, height=1)
    r = oracle.render(sc, cam, spp=1, max_depth=1)
    assert r.stats["tied_paths"] == 0
    return r.image[:, 0, 0]


def _expected(sc, tau0):
    B = sc.n_bins
    n, k, rho = f32(1.6), f32(0.02), f32(0.8)
    F0 = ((n - 1) ** 2 + k**2) / ((n + 1) ** 2 + k**2)
    gn, gk = f32(1.52), f32(3e-6)
    G = ((gn - 1) ** 2 + gk**2) / ((gn + 1) ** 2 + gk**2)
    T = (1 - G) ** 2 * tau0 / (1 - G**2 * tau0**2)
    return (1 - F0) * rho / math.pi * sc.sun_E.astype(np.float64) * T


def test_direct_term_through_a_textured_window_closed_form():
    rng = np.random.default_rng(3)
    W, H, B = 4, 3, 2
    tex = rng.uniform(0.3, 0.95, size=(H, W, B)).astype(np.float32)
    zw, half = 2.0, 1.0
    sc = _window_scene(tex, zw, half)
    pos = lambda s, t: (-half + 2 * half * s, -half + 2 * half * t)
    # texel centres ((i + 1/2) / W, (k + 1/2) / H), on the lower-right (s > t) and upper-left triangles
    for (i, k) in [(2, 0), (3, 1), (0, 2), (1, 1)]:
        s, t = (i + 0.5) / W, (k + 0.5) / H
        got = _nee_at(sc, *pos(s, t), zw)
        np.testing.assert_allclose(got, _expected(sc, tex[k, i].astype(np.float64)), rtol=1e-7)
    # midway between two centres along s, and along t
    got = _nee_at(sc, *pos(2.0 / W, 0.5 / H), zw)
    np.testing.assert_allclose(got, _expected(sc, 0.5 * (tex[0, 1] + tex[0, 2]).astype(np.float64)), rtol=1e-7)
    got = _nee_at(sc, *pos(2.5 / W, 2.0 / H), zw)
    np.testing.assert_allclose(got, _expected(sc, 0.5 * (tex[1, 2] + tex[2, 2]).astype(np.float64)), rtol=1e-7)
    # on the periodic seams s = 0 and s = 1 of a window whose coordinates run over [-0.5, 1.5]:
    # the mean of the last and the first texel of the row
    sc2 = _window_scene(tex, zw, half, uv_scale=2.0, uv_shift=-0.5)
    pos2 = lambda s, t: (-half + 2 * half * (s + 0.5) / 2.0, -half + 2 * half * (t + 0.5) / 2.0)
    seam = _expected(sc2, 0.5 * (tex[1, 0] + tex[1, W - 1]).astype(np.float64))
    for s_ in (0.0, 1.0):
        np.testing.assert_allclose(_nee_at(sc2, *pos2(s_, 1.5 / H), zw), seam, rtol=1e-7)
    # and one period further along t the same texel centre
    np.testing.assert_allclose(_nee_at(sc2, *pos2(1.5 / W, 1.0 + 0.5 / H), zw),
                               _expected(sc2, tex[0, 1].astype(np.float64)), rtol=1e-7)


def test_oblique_crossing_raises_the_map_to_one_over_cos_theta_t():
    """Sun at 35 degrees from the zenith: the shadow ray from the floor point crosses the window
    zw tan(35) further along x, at refraction cosine cos(theta_t) = sqrt(1 - sin^2 / n^2), so
    the slab's internal transmittance is tau0^(1 / cos(theta_t)) and its faces reflect by
    F(theta) of the glass."""
    rng = np.random.default_rng(5)
    W, H, B = 4, 4, 2
    tex = rng.uniform(0.3, 0.9, size=(H, W, B)).astype(np.float32)
    zw, half, th = 2.0, 1.0, math.radians(35.0)
    sun = (math.sin(th), 0.0, math.cos(th))
    sc = _window_scene(tex, zw, half, sun=sun)
    ws = sc.sun_dir.astype(np.float64)
    ws /= np.linalg.norm(ws)
    i, k = 2, 1
    s, t = (i + 0.5) / W, (k + 0.5) / H
    xc, yc = -half + 2 * half * s, -half + 2 * half * t        # crossing point on the window
    # floor point below it along the sun; the shadow ray starts eps = 1e-5 (1 + max|p|) above it
    x, y = xc - zw * ws[0] / ws[2], yc - zw * ws[1] / ws[2]
    for _ in range(2):
        eps = 1e-5 * (1 + max(abs(x), abs(y)))
        x, y = xc - (zw - eps) * ws[0] / ws[2], yc - (zw - eps) * ws[1] / ws[2]
    got = _nee_at(sc, x, y, zw)
    gn, gk = f32(1.52), f32(3e-6)
    c = ws[2]
    ct = math.sqrt(1 - (1 - c * c) / gn**2)
    G = oracle.fresnel(gn, gk, c)
    tau = tex[k, i].astype(np.float64) ** (1.0 / ct)
    T = (1 - G) ** 2 * tau / (1 - G**2 * tau**2)
    n, kk, rho = f32(1.6), f32(0.02), f32(0.8)
    F0 = ((n - 1) ** 2 + kk**2) / ((n + 1) ** 2 + kk**2)
    exp = (1 - F0) * rho / math.pi * sc.sun_E.astype(np.float64) * c * T
    np.testing.assert_allclose(got, exp, rtol=2e-6)


def test_constant_map_equals_absorption_by_k():
    sc = scenegen.nave_scene(8)
    g = int(np.nonzero(sc.mat_type == scenegen.MAT_GLASS)[0][0])
    lam = scenegen.bin_centres(8)
    tau0 = np.exp(-4 * np.pi * sc.k_tab[g].astype(np.float64) * float(sc.thickness_m[g]) / (lam * 1e-9))
    tex = np.broadcast_to(tau0.astype(np.float32), (5, 7, 8)).copy()
    uv = np.random.default_rng(1).uniform(-3, 3, size=(sc.n_tri, 3, 2)).astype(np.float32)
    mt = np.full(sc.n_mat, -1, dtype=np.int32)
    mt[g] = 0
    sct = dataclasses.replace(sc, uv=uv, textures=[tex], mat_tex=mt).check()
    cam = scenegen.nave_camera(24, 24)
    a = oracle.render(sc, cam, spp=4, max_depth=5, seed=3)
    b = oracle.render(sct, cam, spp=4, max_depth=5, seed=3)
    assert a.image.max() > 0
    np.testing.assert_allclose(b.image, a.image, rtol=2e-6, atol=1e-12)
    # and the shadow query
    rng = np.random.default_rng(2)
    o = rng.uniform([8, 0.5, 0.2], [12, 6, 2], size=(400, 3)).astype(np.float32)
    d = np.tile(sc.sun_dir, (400, 1)).astype(np.float32)
    va, ta = oracle.shadow(sc, o, d)
    vb, tb = oracle.shadow(sct, o, d)
    np.testing.assert_allclose(vb, va, rtol=2e-6, atol=1e-12)
    assert ((va[:, 0] > 0) & (va[:, 0] < 1)).sum() > 20


def test_textured_glass_vertex_expectation():
    """Looking down through the textured window into an open sky (no floor, env = 1, no sun):
    every path reflects (weight R / P) or transmits (weight T / (1 - P)) and escapes, so the
    mean over samples tends to R + T of the slab at the texel under the camera."""
    rng = np.random.default_rng(7)
    W, H, B = 3, 3, 2
    tex = rng.uniform(0.2, 0.9, size=(H, W, B)).astype(np.float32)
    zw, half = 2.0, 1.0
    sc = _window_scene(tex, zw, half, env=1.0, floor=False)
    sc.sun_E[:] = 0
    s, t = 2.5 / W, 0.5 / H
    x, y = -half + 2 * half * s, -half + 2 * half * t
    cam = scenegen.Camera(eye=(x, y, 5.0), target=(x, y, 0.0), up=(0, 1, 0), vfov_deg=1e-4, width=16, height=16)
    r = oracle.render(sc, cam, spp=200, max_depth=3, seed=4)
    gn, gk = f32(1.52), f32(3e-6)
    G = ((gn - 1) ** 2 + gk**2) / ((gn + 1) ** 2 + gk**2)
    tau = tex[0, 2].astype(np.float64)
    R = G + (1 - G) ** 2 * tau**2 * G / (1 - G**2 * tau**2)
    T = (1 - G) ** 2 * tau / (1 - G**2 * tau**2)
    P = R.mean() / (R.mean() + T.mean())
    n = 16 * 16 * 200
    sig = np.sqrt(P * (1 - P) / n) * np.abs(R / P - T / (1 - P))
    got = r.image.reshape(B, -1).mean(axis=1)
    assert np.all(np.abs(got - (R + T)) <= 5 * sig + 1e-12), (got, R + T, sig)
