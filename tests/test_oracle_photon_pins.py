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
