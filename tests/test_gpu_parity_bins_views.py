"""Parity against the oracle of the shading paths other bin counts take, and of batched views.

  * Bin counts other than 8 and 40 take the generic opaque-shading kernel (no compile-time
    quad count, tables read from memory): the nave at 13 bins (a ragged last quad of the padded
    rows) and at 80 bins (the large configuration's 5 nm bins), with n, k and rho all varying
    over wavelength. 8 and 40 bins are checked with their tables staged in LDS (few materials)
    and read from memory (many materials; test_gpu_parity.py).
  * Batches: views of different size and spp share the wavefronts; view v draws its random
    numbers with view index v, so each view must equal oracle.render(view=v), eager and replayed
    from the captured graph.
Bars as in test_gpu_parity.py: |a - b| <= 1e-4 max(|b|, 1e-3 mean_bin) on tie-free pixels.
"""
import dataclasses
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
def ctx():
    import paper_1912_04000_amd as sd
    return sd.Context(0)


def _scene(ctx, sc, grid):
    import paper_1912_04000_amd as sd
    S = sd.Scene.from_description(sc, grid=grid)
    ctx.upload(S)
    return S


def _pixel_parity(img, ref, tied, label):
    B = ref.shape[0]
    mean_bin = ref.reshape(B, -1).mean(axis=1)
    tol = 1e-4 * np.maximum(np.abs(ref), 1e-3 * mean_bin.reshape((B,) + (1,) * (ref.ndim - 1)))
    ok = tied == 0
    bad = (np.abs(img - ref) > tol) & ok[None]
    rel = np.abs(img - ref)[:, ok] / np.maximum(np.abs(ref)[:, ok], 1e-12)
    say(f"[{label}] pixels={ok.size} tie-free={ok.sum()} bad={bad.reshape(B, -1).any(axis=0).sum()} "
        f"max rel={rel.max() if rel.size else 0:.3e}")
    assert not bad.any(), np.argwhere(bad)[:10]
    return ok


def _dispersive_nave(B):
    """The nave with every optical table varying over the bins: stone n = 1.6 + 0.04 sin, glass
    n = 1.52 + 0.02 (1 - t) (normal dispersion), rho already per-bin from k."""
    sc = scenegen.nave_scene(B)
    t = (np.arange(B) + 0.5) / B
    n = sc.n_tab.copy()
    for m in range(sc.n_mat):
        if sc.mat_type[m] == scenegen.MAT_GLASS:
            n[m] = 1.52 + 0.02 * (1.0 - t)
        else:
            n[m] = 1.6 + 0.04 * np.sin(7.0 * t + m)
    return dataclasses.replace(sc, n_tab=n.astype(np.float32)).check()


@pytest.mark.parametrize("B", [13, 80])
def test_generic_shading_kernel_parity(ctx, B):
    import paper_1912_04000_amd as sd
    sc = _dispersive_nave(B)
    assert sc.n_tab.std(axis=1).min() > 0 and sc.k_tab.std(axis=1).min() > 0
    cam = scenegen.nave_camera(48, 40)
    S = _scene(ctx, sc, (2, 2, 2))
    img = ctx.render(S, sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height),
                     sd.render_params(spp=2, max_depth=6, seed=21)).cpu().numpy()
    ref = oracle.render(sc, cam, spp=2, max_depth=6, seed=21)
    ok = _pixel_parity(img, ref.image, ref.tied, f"{B} bins, generic shading kernel")
    assert ok.mean() > 0.9
    # the bins really differ (a wrong quad or bin index would not hide behind equal bins)
    assert np.abs(np.diff(ref.image, axis=0)).max() > 1e-3 * ref.image.max()


@pytest.mark.parametrize("B", [8, 40])
def test_lds_table_shading_parity_dispersive(ctx, B):
    """8 and 40 bins with few materials: the opaque shading kernel stages n, k, rho in LDS."""
    import paper_1912_04000_amd as sd
    sc = _dispersive_nave(B)
    bp = (B + 3) // 4 * 4
    assert 3 * sc.n_mat * bp + bp <= 8192
    cam = scenegen.nave_camera(40, 32)
    S = _scene(ctx, sc, (2, 2, 2))
    img = ctx.render(S, sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height),
                     sd.render_params(spp=2, max_depth=6, seed=22)).cpu().numpy()
    ref = oracle.render(sc, cam, spp=2, max_depth=6, seed=22)
    ok = _pixel_parity(img, ref.image, ref.tied, f"{B} bins, tables in LDS")
    assert ok.mean() > 0.9


def _views(sd):
    return [sd.camera((3.0, 8.0, 1.7), (12.0, 1.0, 1.5), (0, 0, 1), 60, 40, 30),
            sd.camera((15.0, 2.0, 3.0), (5.0, 8.0, 1.0), (0, 0, 1), 75, 17, 23),
            sd.camera((10.0, 5.0, 6.0), (10.0, 5.0, 0.0), (0, 1, 0), 90, 32, 32)]


def _oracle_cam(c):
    return scenegen.Camera(eye=tuple(c.eye), target=tuple(c.target), up=tuple(c.up), vfov_deg=c.vfov_deg,
                           width=c.width, height=c.height)


@pytest.mark.parametrize("use_graph", [0, 1])
def test_batch_views_match_oracle_per_view(ctx, use_graph):
    """Three views of uneven size and spp in one batch (wavefronts of 1500 paths, so wavefronts
    straddle views); view v is compared with oracle.render(view=v). In graph mode the capture
    is replayed twice, with an eager render in between, and both replays are compared."""
    import paper_1912_04000_amd as sd
    sc = scenegen.nave_scene(8)
    S = _scene(ctx, sc, (2, 2, 2))
    cams = _views(sd)
    spp = [3, 1, 5]
    refs = [oracle.render(sc, _oracle_cam(c), spp=s, max_depth=5, seed=9, view=v)
            for v, (c, s) in enumerate(zip(cams, spp))]
    p = sd.render_params(max_depth=5, seed=9, wave_paths=1500, use_graph=use_graph)
    outs = None
    for rep in range(2 if use_graph else 1):
        outs = ctx.render_batch(S, cams, spp, p, outs=outs)
        for v in range(len(cams)):
            ok = _pixel_parity(outs[v].cpu().numpy(), refs[v].image, refs[v].tied,
                               f"batch view {v} ({cams[v].width}x{cams[v].height}, {spp[v]} spp) graph={use_graph} "
                               f"replay {rep}")
            assert ok.mean() > 0.9
        ctx.render(S, cams[1], sd.render_params(spp=1, max_depth=3, seed=rep))
    if use_graph:
        assert ctx.stats()["graph_launches"] >= 2
