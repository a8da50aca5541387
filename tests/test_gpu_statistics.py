"""Statistics of the spectral path estimator on the GPU, with random numbers the oracle does not
share (the parity tests use identical streams):

  * unbiasedness: the GPU image with one seed and the oracle's with another estimate the same
    expectation; per bin, the difference of the image means stays within 4 standard errors, the
    per-pixel noise variance estimated from two independent GPU renders;
  * convergence: the RMSE against a high-spp reference falls as spp^-1/2 (least-squares
    log-log slope -0.5 +- 0.05 over 1 .. 64 spp), with the reference's own noise, estimated from
    its two halves, subtracted.
"""
import sys

import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nave():
    import paper_1912_04000_amd as sd
    ctx = sd.Context(0)
    sc = scenegen.nave_scene(8)
    cam = scenegen.nave_camera(64, 64)
    S = sd.Scene.from_description(sc, grid=(2, 2, 2))
    ctx.upload(S)
    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height)
    return sd, ctx, sc, cam, S, c


def _render(nave, spp, seed, first=0):
    sd, ctx, sc, cam, S, c = nave
    return ctx.render(S, c, sd.render_params(spp=spp, max_depth=4, seed=seed, first_sample=first)).cpu().numpy()


def test_gpu_and_oracle_means_agree_with_other_random_numbers(nave):
    sd, ctx, sc, cam, S, c = nave
    spp = 16
    a = _render(nave, spp, 101).astype(np.float64)
    b = _render(nave, spp, 303).astype(np.float64)
    o = oracle.render(sc, cam, spp=spp, max_depth=4, seed=202).image
    B = a.shape[0]
    npix = a.shape[1] * a.shape[2]
    noise_var = np.mean(((a - b) ** 2).reshape(B, -1), axis=1) / 2.0   # per-pixel variance of one render
    se = np.sqrt(2.0 * noise_var / npix)                               # of the difference of two means
    d = a.reshape(B, -1).mean(axis=1) - o.reshape(B, -1).mean(axis=1)
    say(f"mean differences {np.round(d / se, 2)} standard errors; image means {a.reshape(B, -1).mean(axis=1)}")
    assert np.all(noise_var > 0)
    assert np.all(np.abs(d) <= 4.0 * se), (d, se)


def test_rmse_falls_as_inverse_square_root_of_spp(nave):
    B = 8
    # reference: two independent 1024-spp halves (samples 0..1023 and 1024..2047 of seed 9)
    h0 = _render(nave, 1024, 9, first=0).astype(np.float64)
    h1 = _render(nave, 1024, 9, first=1024).astype(np.float64)
    ref = 0.5 * (h0 + h1)
    ref_var = np.mean((h0 - h1) ** 2) / 4.0
    spps = np.array([1, 2, 4, 8, 16, 32, 64])
    rmse = []
    for k in spps:
        img = _render(nave, int(k), 77).astype(np.float64)
        rmse.append(np.sqrt(max(np.mean((img - ref) ** 2) - ref_var, 0.0)))
    rmse = np.array(rmse)
    slope = np.polyfit(np.log(spps), np.log(rmse), 1)[0]
    say(f"RMSE {rmse}, log-log slope {slope:.3f}, reference noise RMS {np.sqrt(ref_var):.2e}")
    assert abs(slope + 0.5) <= 0.05
    assert ref.shape[0] == B and rmse[-1] < rmse[0] / 6.0
