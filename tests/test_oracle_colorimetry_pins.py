"""Pins of the oracle's colorimetry (spectral image -> CIE XYZ -> sRGB) by data and standards
outside it: CIE 1931 colour-matching values at five wavelengths (tests/golden, cited there),
the equal-energy white point of XYZ, the sRGB standard's D65 white, its transfer function's
values, and the photopic peak near 555 nm."""
import os

import numpy as np
import pytest

from oracle import colorimetry as col

HERE = os.path.dirname(os.path.abspath(__file__))


def test_fit_matches_cie1931_anchor_values():
    t = np.loadtxt(os.path.join(HERE, "golden", "cie1931_2deg_anchors.txt"))
    v = col.cmf(t[:, 0]).T
    # the multi-lobe fit is accurate to about 1e-2 of the peak values
    np.testing.assert_allclose(v, t[:, 1:], atol=0.015)


def test_photopic_peak_near_555nm():
    lam = np.linspace(380, 780, 4001)
    y = col.cmf(lam)[1]
    assert 550.0 <= lam[np.argmax(y)] <= 560.0
    assert abs(y.max() - 1.0) < 0.01


def test_equal_energy_white():
    """XYZ is defined so that the equal-energy spectrum has X = Y = Z: a flat spectrum of 1 over
    the visible range maps to XYZ close to (1, 1, 1), chromaticity (1/3, 1/3)."""
    B = 400
    img = np.ones((B, 2, 3))
    xyz = col.spectral_to_xyz(img, 380.0, 780.0)
    np.testing.assert_allclose(xyz[1], 1.0, rtol=1e-12)
    np.testing.assert_allclose(xyz[:, 0, 0], 1.0, atol=5e-3)
    xy = xyz[:2, 0, 0] / xyz[:, 0, 0].sum()
    np.testing.assert_allclose(xy, 1 / 3, atol=2e-3)
    # exposure scales linearly
    np.testing.assert_allclose(col.spectral_to_xyz(img, 380.0, 780.0, exposure=2.5), 2.5 * xyz, rtol=1e-12)


def test_d65_white_is_srgb_white():
    """The sRGB primaries are defined with D65 (x, y) = (0.3127, 0.3290) as R = G = B = 1."""
    x, y = 0.3127, 0.3290
    xyz = np.array([x / y, 1.0, (1 - x - y) / y])
    np.testing.assert_allclose(col.xyz_to_linear_srgb(xyz), 1.0, atol=1e-3)
    # and the primaries' chromaticities: the inverse matrix's columns
    inv = np.linalg.inv(col.SRGB_FROM_XYZ)
    prim = inv[:2] / inv.sum(axis=0)
    np.testing.assert_allclose(prim.T, [[0.64, 0.33], [0.30, 0.60], [0.15, 0.06]], atol=1e-3)


def test_srgb_transfer_function_values():
    lin = np.array([0.0, 0.0031308, 0.18, 0.5, 1.0, 2.0, -1.0, 0.01, 0.002])
    enc = col.encode_srgb(lin)
    # 1 % linear encodes to 0.099853 (the power segment); 0.2 % stays on the linear segment
    np.testing.assert_allclose(enc[7], 0.099853, rtol=1e-5)
    np.testing.assert_allclose(enc[8], 0.02584, rtol=1e-9)
    np.testing.assert_allclose(enc[[0, 4, 5, 6]], [0.0, 1.0, 1.0, 0.0], atol=1e-12)
    assert abs(enc[1] - 12.92 * 0.0031308) < 1e-12
    np.testing.assert_allclose(enc[2], 0.46135612950044164, rtol=1e-9)
    np.testing.assert_allclose(enc[3], 0.7353569830524495, rtol=1e-9)
    # continuous at the threshold within the standard's rounding of its constants
    a = 1.055 * 0.0031308 ** (1 / 2.4) - 0.055
    assert abs(a - 12.92 * 0.0031308) < 3e-5


def test_monochromatic_bins_order_of_hues():
    """A single 450 nm, 550 nm or 620 nm bin: blue, green or red dominates the linear sRGB."""
    B = 40
    lam = col.bin_centres(B, 380.0, 780.0)
    for target, ch in ((450.0, 2), (540.0, 1), (620.0, 0)):
        img = np.zeros((B, 1, 1))
        img[np.argmin(np.abs(lam - target))] = 1.0
        rgb = col.xyz_to_linear_srgb(col.spectral_to_xyz(img, 380.0, 780.0))[:, 0, 0]
        assert np.argmax(rgb) == ch, (target, rgb)
