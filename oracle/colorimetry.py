"""Colorimetry of the spectral image, FP64 -- TEST INFRASTRUCTURE ONLY (oracle).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this module; the renderer never does. It is the plain definition of what the library's spectral
to sRGB kernel computes.

The paper renders spectral images and maps them to RGB "by means of colorimetry" for display
(section 6), since the observer's visual adaptation needs colorimetric treatment (section 1).
No colour-matching tables ship here, so the CIE 1931 2-degree standard observer is taken from
the multi-lobe analytic fit of Wyman, Sloan and Shirley ("Simple analytic approximations to the
CIE XYZ color matching functions", JCGT 2(2), 2013): each function is a sum of piecewise
Gaussians g(l; mu, s1, s2) = exp(-((l - mu) / s)^2 / 2) with s = s1 below mu and s2 above.

Steps, per pixel of an image I[B][H][W] sampled at the bin centres l_j (point samples, as
everywhere in the renderer):
  1. XYZ = exposure * sum_j I_j cmf(l_j) / sum_j ybar(l_j)   (a flat spectrum of 1 gives Y = 1)
  2. linear sRGB = M XYZ with the IEC 61966-2-1 (sRGB, D65) matrix
  3. encoded sRGB: clamp to [0, 1], then 12.92 c below 0.0031308, else 1.055 c^(1/2.4) - 0.055
"""
from __future__ import annotations

import numpy as np

# (amplitude, mu, sigma below mu, sigma above mu) of each lobe, nm
_LOBES = {
    "x": ((1.056, 599.8, 37.9, 31.0), (0.362, 442.0, 16.0, 26.7), (-0.065, 501.1, 20.4, 26.2)),
    "y": ((0.821, 568.8, 46.9, 40.5), (0.286, 530.9, 16.3, 31.1)),
    "z": ((1.217, 437.0, 11.8, 36.0), (0.681, 459.0, 26.0, 13.8)),
}

# XYZ (D65) -> linear sRGB, IEC 61966-2-1
SRGB_FROM_XYZ = np.array([[3.2406, -1.5372, -0.4986],
                          [-0.9689, 1.8758, 0.0415],
                          [0.0557, -0.2040, 1.0570]])


def _piecewise_gauss(lam, mu, s1, s2):
    lam = np.asarray(lam, dtype=np.float64)
    s = np.where(lam < mu, s1, s2)
    return np.exp(-0.5 * ((lam - mu) / s) ** 2)


def cmf(lam_nm):
    """xbar, ybar, zbar at wavelengths lam_nm (array), shape [3][n]."""
    lam = np.atleast_1d(np.asarray(lam_nm, dtype=np.float64))
    out = np.zeros((3, lam.size))
    for c, name in enumerate("xyz"):
        for a, mu, s1, s2 in _LOBES[name]:
            out[c] += a * _piecewise_gauss(lam, mu, s1, s2)
    return out


def bin_centres(n_bins, lambda_min_nm, lambda_max_nm):
    j = np.arange(n_bins, dtype=np.float64)
    return lambda_min_nm + (j + 0.5) * (lambda_max_nm - lambda_min_nm) / n_bins


def spectral_to_xyz(image, lambda_min_nm, lambda_max_nm, exposure=1.0):
    """image [B][...] -> XYZ [3][...] (step 1)."""
    img = np.asarray(image, dtype=np.float64)
    B = img.shape[0]
    w = cmf(bin_centres(B, lambda_min_nm, lambda_max_nm))
    w = w / w[1].sum()
    return exposure * np.tensordot(w, img, axes=(1, 0))


def xyz_to_linear_srgb(xyz):
    """XYZ [3][...] -> linear sRGB [3][...] (step 2)."""
    return np.tensordot(SRGB_FROM_XYZ, np.asarray(xyz, dtype=np.float64), axes=(1, 0))


def encode_srgb(lin):
    """Transfer function of sRGB on values clamped to [0, 1] (step 3)."""
    c = np.clip(np.asarray(lin, dtype=np.float64), 0.0, 1.0)
    return np.where(c <= 0.0031308, 12.92 * c, 1.055 * np.power(c, 1.0 / 2.4) - 0.055)


def spectral_to_srgb(image, lambda_min_nm, lambda_max_nm, exposure=1.0):
    """image [B][H][W] -> (XYZ [3][H][W], encoded sRGB [H][W][3])."""
    xyz = spectral_to_xyz(image, lambda_min_nm, lambda_max_nm, exposure)
    rgb = encode_srgb(xyz_to_linear_srgb(xyz))
    return xyz, np.moveaxis(rgb, 0, -1)
