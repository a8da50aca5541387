"""Colorimetry kernel (spectral image -> XYZ -> sRGB) against the FP64 oracle, on the GPU.

Tolerances from the arithmetic: every XYZ component is a sum of at most 128 products of a
weight (FP32, a few ulp from expf and its scaling) and an image value, so its error is below
1e-5 of the sum of the magnitudes of its terms; sRGB mixes XYZ with coefficients below 3.3 in
magnitude and the transfer function's slope is at most 12.92, so encoded values are within
2e-4 for the XYZ below 2 used here.
"""
import numpy as np
import pytest

import oracle
import scenegen
from oracle import colorimetry as col

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1912_04000_amd as sd
    return sd.Context(0)


def _check(ctx, img, lmin, lmax, exposure, label):
    import torch
    dev = torch.from_numpy(np.ascontiguousarray(img, dtype=np.float32)).cuda()
    xyz, rgb = ctx.spectral_to_srgb(dev, lmin, lmax, exposure)
    xyz, rgb = xyz.cpu().numpy(), rgb.cpu().numpy()
    oxyz, orgb = col.spectral_to_srgb(img.astype(np.float32).astype(np.float64), lmin, lmax, exposure)
    B = img.shape[0]
    w = col.cmf(col.bin_centres(B, lmin, lmax))
    w = exposure * np.abs(w) / w[1].sum()
    mag = np.tensordot(w, np.abs(img.astype(np.float64)), axes=(1, 0))
    err_xyz = np.abs(xyz - oxyz)
    assert (err_xyz <= 1e-5 * mag + 1e-30).all(), (label, (err_xyz / np.maximum(mag, 1e-30)).max())
    assert np.abs(rgb - orgb).max() <= 2e-4, (label, np.abs(rgb - orgb).max())
    print(f"[{label}] max XYZ rel {(err_xyz / np.maximum(mag, 1e-30)).max():.2e}, "
          f"max sRGB abs {np.abs(rgb - orgb).max():.2e}", flush=True)
    return xyz, rgb


@pytest.mark.parametrize("B,H,W", [(1, 3, 5), (8, 37, 29), (13, 64, 65), (40, 90, 160), (80, 33, 17), (128, 8, 300)])
def test_random_spectra_match_oracle(ctx, B, H, W):
    rng = np.random.default_rng(B * 1000 + H)
    img = rng.uniform(0.0, 1.0, size=(B, H, W)) * rng.uniform(0.0, 1.5, size=(1, H, W))
    img[:, 0, 0] = 0.0                                  # black
    img[:, 0, 1] = 40.0                                 # clipped white
    _check(ctx, img, 380.0, 780.0, 0.9, f"B={B} {H}x{W}")


def test_narrow_range_and_exposure(ctx):
    rng = np.random.default_rng(5)
    img = rng.uniform(0.0, 2.0, size=(16, 20, 20))
    _check(ctx, img, 520.0, 610.0, 0.3, "520-610 nm, exposure 0.3")


def test_flat_spectrum_gives_y_equal_exposure(ctx):
    import torch
    img = torch.ones((40, 4, 6), dtype=torch.float32, device="cuda")
    xyz, _ = ctx.spectral_to_srgb(img, 380.0, 780.0, 0.5, want_srgb=False)
    np.testing.assert_allclose(xyz[1].cpu().numpy(), 0.5, rtol=2e-6)


def test_rendered_nave_frame(ctx):
    """The nave frame rendered on the GPU, then its colour image on the GPU, against the
    oracle's colorimetry of the same spectral image."""
    import paper_1912_04000_amd as sd
    sc = scenegen.nave_scene(8)
    cam = scenegen.nave_camera()
    S = sd.Scene.from_description(sc, grid=(2, 2, 2))
    ctx.upload(S)
    img = ctx.render(S, sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height),
                     sd.render_params(spp=4, max_depth=4, seed=1))
    _check(ctx, img.cpu().numpy(), 380.0, 780.0, 4.0, "nave frame")


def test_argument_validation(ctx):
    import ctypes as C
    import torch
    import paper_1912_04000_amd as sd
    img = torch.ones((8, 2, 2), dtype=torch.float32, device="cuda")
    out = torch.empty((3, 2, 2), dtype=torch.float32, device="cuda")
    L = sd.lib()
    f = lambda B, lmin, lmax, n, e, o1, o2: L.sdd_spectral_to_srgb(ctx.handle, C.c_void_p(img.data_ptr()), B, lmin,
                                                                   lmax, n, e, o1, o2)
    o = C.c_void_p(out.data_ptr())
    assert f(0, 380.0, 780.0, 4, 1.0, o, None) == -1
    assert f(129, 380.0, 780.0, 4, 1.0, o, None) == -1
    assert f(8, 780.0, 380.0, 4, 1.0, o, None) == -1
    assert f(8, 380.0, 780.0, 0, 1.0, o, None) == -1
    assert f(8, 380.0, 780.0, 4, float("nan"), o, None) == -1
    assert f(8, 380.0, 780.0, 4, 1.0, None, None) == -1
    assert f(8, 380.0, 780.0, 4, 1.0, o, None) == 0
    ctx.finish()
