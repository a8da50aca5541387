"""Pins of the oracle's caustic photon map (section 4: photon maps filled from the light sources,
one for caustics) by closed forms of geometric optics.

Scene: a horizontal lossless glass pane (the window, z = 3, 2 m x 2 m), a large mirror floor
(zero albedo, so its mirror lobe is certain and weighs F), a diffuse receiver wall x = -6 facing
+x, and the sun 30 degrees from the zenith in the x-z plane. Sunlight passes the pane (slab
transmittance T), reflects on the floor (F) and reaches the wall, where the reflected beam has
irradiance E T F cos(theta_r) with cos(theta_r) = sin 30. Looking at the wall inside the beam, the
caustic part of the pixel (render with the map minus render without) is
(1 - F_w) rho_w / pi * E T F cos(theta_r), within the density estimate's counting noise.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen

f32 = lambda x: float(np.float32(x))


def _quad(c00, c10, c11, c01):
    return [(c00, c10, c11), (c00, c11, c01)]


def _caustic_scene(B=3, floor_n=(1.5, 1.9, 2.6), floor_rho=0.0):
    return scenegen.caustic_scene(B, floor_n, floor_rho)


def _expected_caustic(sc, cos_view):
    B = sc.n_bins
    ws = sc.sun_dir.astype(np.float64)
    ws /= np.linalg.norm(ws)
    c_pane = ws[2]
    T = np.array([oracle.slab(f32(1.52), 0.0, 500.0, f32(0.004), c_pane)[1] for _ in range(B)])
    F = np.array([oracle.fresnel(float(sc.n_tab[1, j]), float(sc.k_tab[1, j]), c_pane) for j in range(B)])
    cos_r = ws[0]                                    # the reflected beam meets the wall x = -6
    Fw = oracle.fresnel(f32(1.6), f32(0.02), cos_view)
    return (1 - Fw) * f32(0.8) / math.pi * sc.sun_E.astype(np.float64) * T * F * cos_r


def _spot_camera(y, z, W=4, H=4):
    # on the receiver wall, looking straight at (−6, y, z) from x = −3 (normal incidence)
    return scenegen.Camera(eye=(-3.0, y, z), target=(-6.0, y, z), up=(0, 0, 1), vfov_deg=1e-4, width=W, height=H)


def test_window_mirror_receiver_caustic_closed_form():
    sc = _caustic_scene()
    N, r = 3_000_000, 0.15
    ph = oracle.photons(sc, N, max_depth=6, seed=7)
    # every photon lands on the wall once: reflected by the pane (vertex 2, a spot at z 11.7 to
    # 15.2) or transmitted, then reflected by the floor (vertex 3, a spot at z 5.7 to 9.1)
    assert len(ph["id"]) == N and set(np.unique(ph["depth"])) == {2, 3}
    t30 = math.tan(math.radians(30.0))
    zc = (6.0 - 3.0 * t30) / t30     # centre of the floor-route spot
    for (y, z) in [(0.03, zc), (-0.45, zc - 0.8), (0.5, zc + 0.9)]:
        cam = _spot_camera(y, z)
        a = oracle.render(sc, cam, spp=1, max_depth=1, seed=1, photons=ph, radius=r)
        b = oracle.render(sc, cam, spp=1, max_depth=1, seed=1)
        got = (a.image - b.image)[:, 0, 0]
        exp = _expected_caustic(sc, 1.0)
        # counting noise: about exp / sqrt(photons in the disc)
        wall_area = 4.0 * math.cos(math.radians(30.0)) / math.sin(math.radians(30.0))
        n_disc = (ph["depth"] == 3).sum() * math.pi * r * r / wall_area
        np.testing.assert_allclose(got, exp, rtol=5.0 / math.sqrt(n_disc))
        assert a.stats["tied_paths"] == 0
        # photons near the gather radius bound how far a different rounding could move the estimate
        assert np.all(a.photon_unc[:, 0, 0] < 0.01 * got)


def test_no_caustic_without_a_reflection():
    """Sun overhead and a floor that reflects nothing (n = 1: F = 0, so P_s = 0) under the pane:
    what the pane reflects leaves straight up, and sunlight only transmitted through thin glass is
    the direct term, so no photon is stored."""
    sc = _caustic_scene(floor_n=(1.0, 1.0, 1.0), floor_rho=0.9)
    sc.k_tab[1] = 0.0
    sc.sun_dir[:] = (0.0, 0.0, 1.0)
    ph = oracle.photons(sc, 50_000, max_depth=6, seed=2)
    assert len(ph["id"]) == 0


def test_emission_flux_and_area():
    """Photon flux: the sun's irradiance times the windows' area projected on its direction, split
    evenly. Every photon reaches the wall once, by the pane's reflection (R) or through the pane
    and off the floor's certain mirror (T F): the stored flux sums to E A (R + T F) in
    expectation; A is the pane's 4 m^2 times cos 30."""
    sc = _caustic_scene()
    ph = oracle.photons(sc, 400_000, max_depth=6, seed=3)
    A = 4.0 * math.cos(math.radians(30.0))
    assert abs(ph["area"] - A) < 1e-6 * A
    ws = sc.sun_dir.astype(np.float64) / np.linalg.norm(sc.sun_dir)
    T = oracle.slab(f32(1.52), 0.0, 500.0, f32(0.004), ws[2])
    F = np.array([oracle.fresnel(float(sc.n_tab[1, j]), float(sc.k_tab[1, j]), ws[2]) for j in range(3)])
    tot = ph["flux"].sum(axis=0)
    exp = sc.sun_E.astype(np.float64) * A * (T[0] + T[1] * F)
    # the transmit/reflect choice at the pane is random (weights R / P_r or T / (1 - P_r)):
    # binomial noise on the split
    P_r = T[0] / (T[0] + T[1])
    wr, wt = T[0] / P_r, T[1] * F / (1 - P_r)
    sd = np.abs(wr - wt) * math.sqrt(P_r * (1 - P_r) / 400_000) * sc.sun_E.astype(np.float64) * A
    assert np.all(np.abs(tot - exp) <= 5 * sd + 1e-12), (tot, exp, sd)


def test_stride_sample_is_the_full_maps_records():
    """Tracing every k-th photon reproduces exactly the records those photons leave in the full
    map (each photon is traced from its own counter; its flux is E A / N for the full N)."""
    sc = scenegen.nave_scene(8)
    full = oracle.photons(sc, 30_000, max_depth=6, seed=3)
    part = oracle.photons(sc, 30_000, max_depth=6, seed=3, stride=7)
    sel = full["id"] % 7 == 0
    assert sel.sum() == len(part["id"]) > 50
    for k in ("id", "depth", "pos", "dir", "flux"):
        assert np.array_equal(full[k][sel], part[k]), k
    assert np.array_equal(full["tied"][::7], part["tied"][::7]) and part["area"] == full["area"]


# -- global photon map ---------------------------------------------------------------------
def _box_with_floor(floor_n, floor_k, walls_n=1.0, walls_k=0.0, size=(4.0, 4.0, 3.0), rho=0.6, B=4):
    """window_box_scene with the floor made a material of its own (index floor_n + i floor_k)."""
    import dataclasses
    sc = scenegen.window_box_scene(B, size=size, n=walls_n, k=walls_k, rho=rho)
    mat = sc.mat.copy()
    mat[:2] = 2                                    # the floor's two triangles
    return dataclasses.replace(
        sc, mat=mat, mat_type=np.array([0, 1, 0], dtype=np.int32),
        thickness_m=np.array([0, 0.005, 0], dtype=np.float32),
        n_tab=np.vstack([sc.n_tab, np.full((1, B), floor_n, np.float32)]),
        k_tab=np.vstack([sc.k_tab, np.full((1, B), floor_k, np.float32)]),
        rho_tab=np.vstack([sc.rho_tab, np.full((1, B), rho, np.float32)])).check()


def _select(ph, keep):
    return {k: v[keep] for k, v in ph.items() if k not in ("tied", "area")}


def test_global_map_direct_irradiance():
    """Sunlight through a ceiling window lands on the floor (the photons' vertex 2): there the
    global map's estimate is (1 - F_v) rho / pi E T(theta_s) cos(theta_s) for a view along the
    normal, within the counting noise of the disc."""
    sc = scenegen.window_box_scene(4)
    ph = oracle.photons(sc, 1_000_000, max_depth=2, seed=5, global_map=True)
    assert set(np.unique(ph["depth"])) == {2}
    ws = sc.sun_dir.astype(np.float64) / np.linalg.norm(sc.sun_dir.astype(np.float64))
    c = (2.0 - 3.0 * ws[0] / ws[2], 2.0 - 3.0 * ws[1] / ws[2])   # centre of the lit patch
    cam = scenegen.Camera(eye=(c[0], c[1], 1.0), target=(c[0], c[1], 0.0), up=(0, 1, 0), vfov_deg=1e-4, width=1,
                          height=1)
    r = 0.08
    got = oracle.render(sc, cam, spp=1, max_depth=1, seed=1, global_photons=ph, global_radius=r,
                        global_depth=1).image[:, 0, 0]
    lam = scenegen.bin_centres(4)
    T = np.array([oracle.slab(f32(1.52), float(sc.k_tab[1, j]), lam[j], f32(0.005), ws[2])[1] for j in range(4)])
    exp = (1 - oracle.fresnel(f32(1.5), f32(0.02), 1.0)) * f32(0.6) / math.pi * sc.sun_E.astype(np.float64) * T * ws[2]
    n_disc = len(ph["id"]) * math.pi * r * r / (1.2 * 1.2)
    np.testing.assert_allclose(got, exp, rtol=4.0 / math.sqrt(n_disc))


def test_global_map_diffuse_bounce_takes_fresnel_of_the_new_direction():
    """The Fresnel-split diffuse lobe weighs light by 1 - F of the direction it leaves in (for a
    camera path, the direction toward the viewer). A photon bouncing diffusely off the lit floor
    must therefore take F at its new direction: then the light it brings to far, grazing ceiling
    points equals what camera paths of two vertices find there (ceiling and walls without a
    Fresnel term, so the camera paths' second vertex is the floor's direct term). The photons that
    took the floor's mirror lobe (sunlight no camera path can reach) are left out."""
    sc = _box_with_floor(1.5, 0.02, size=(6.0, 6.0, 1.0))
    N = 1_000_000
    g = oracle.photons(sc, N, max_depth=3, seed=5, global_map=True)
    c = oracle.photons(sc, N, max_depth=3, seed=5)
    mirror = c["id"][c["depth"] == 3]
    d3 = _select(g, (g["depth"] == 3) & ~np.isin(g["id"], mirror))
    for (tx, ty) in [(5.5, 5.5), (5.5, 1.0), (1.0, 5.5)]:
        cam = scenegen.Camera(eye=(tx, ty, 0.5), target=(tx, ty, 1.0), up=(0, 1, 0), vfov_deg=40, width=8, height=8)
        a = oracle.render(sc, cam, spp=1, max_depth=1, seed=1, global_photons=d3, global_radius=0.15, global_depth=1)
        b = oracle.render(sc, cam, spp=4096, max_depth=2, seed=2)
        # F at the photon's arrival angle instead would give +20 to +30 % here
        assert abs(a.image[0].mean() / b.image[0].mean() - 1.0) < 0.06


def test_global_map_matches_camera_paths():
    """In a closed room without specular surfaces besides the pane (no caustics), the radiance a
    camera path finds with the global map from its first or its second vertex on equals what full
    paths with the direct term find, within the noise of both (4 standard deviations) and 2 % of
    density-estimate blur: on the floor in shadow, on the floor in the sunlit patch (where the map
    carries the direct light the paths get from eq. 3), and on the ceiling, whose second vertices
    fall on the patch too."""
    sc = scenegen.window_box_scene(4, n=1.0, k=0.0)
    g = oracle.photons(sc, 300_000, max_depth=12, seed=5, global_map=True)
    ws = sc.sun_dir.astype(np.float64) / np.linalg.norm(sc.sun_dir.astype(np.float64))
    lit = (2.0 - 3.0 * ws[0] / ws[2], 2.0 - 3.0 * ws[1] / ws[2])
    views = [((3.0, 3.0, 1.0), (3.0, 3.0, 0.0), ((1, 1), (2, 64))),
             ((lit[0], lit[1], 1.0), (lit[0], lit[1], 0.0), ((1, 1),)),
             ((3.0, 3.0, 2.0), (3.0, 3.0, 3.0), ((2, 64),))]
    for eye, target, runs in views:
        cam = scenegen.Camera(eye=eye, target=target, up=(0, 1, 0), vfov_deg=20, width=8, height=8)
        b = oracle.render(sc, cam, spp=2048, max_depth=12, seed=2)
        mb, sb = b.image[0].mean(), b.image[0].std() / 8
        for gd, spp in runs:
            a = oracle.render(sc, cam, spp=spp, max_depth=12, seed=1, global_photons=g, global_radius=0.1,
                              global_depth=gd)
            ma, sa = a.image[0].mean(), a.image[0].std() / 8
            assert abs(ma - mb) < 4.0 * math.hypot(sa, sb) + 0.02 * mb, (target, gd, ma, mb, sa, sb)
