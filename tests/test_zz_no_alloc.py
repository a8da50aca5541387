"""sdd_render_noalloc (the render with the library's static device workspace) against sdd_render,
through the C ABI, on the GPU: two calls in a row, the second with a smaller frame, each equal
to the allocating entry point's image within the renderer's 1e-4 relative bar (and to the
oracle on tie-free pixels); a wavefront that does not fit the static workspace is refused."""
import ctypes as C
import sys

import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _close(a, ref, label):
    B = ref.shape[0]
    mean_bin = ref.reshape(B, -1).mean(axis=1)
    tol = 1e-4 * np.maximum(np.abs(ref), 1e-3 * mean_bin[:, None, None])
    bad = np.abs(a - ref) > tol
    say(f"[{label}] max |diff| {np.abs(a - ref).max():.3e}, bad {bad.sum()}")
    assert not bad.any()


def test_render_noalloc_matches_render_twice_then_smaller():
    import torch
    import paper_1912_04000_amd as sd
    ctx = sd.Context(0)
    sc = scenegen.nave_scene(8)
    S = sd.Scene.from_description(sc, grid=(2, 2, 2))
    ctx.upload(S)
    for (W, H, spp, seed) in ((64, 48, 3, 5), (24, 16, 1, 6)):
        cam = scenegen.nave_camera(W, H)
        c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, W, H)
        p = sd.render_params(spp=spp, max_depth=5, seed=seed)
        ref = ctx.render(S, c, p).cpu().numpy()
        out = torch.full((sc.n_bins, H, W), float("nan"), dtype=torch.float32, device="cuda")
        got = ctx.render_noalloc(S, c, p, out).cpu().numpy()
        _close(got, ref, f"noalloc {W}x{H} {spp} spp vs sdd_render")
        o = oracle.render(sc, cam, spp=spp, max_depth=5, seed=seed)
        ok = o.tied == 0
        mean_bin = o.image.reshape(sc.n_bins, -1).mean(axis=1)
        tol = 1e-4 * np.maximum(np.abs(o.image), 1e-3 * mean_bin[:, None, None])
        assert ok.mean() > 0.9 and not ((np.abs(got - o.image) > tol) & ok[None]).any()
    # a wavefront whose workspace exceeds the static array is refused with a clear error
    cam = scenegen.nave_camera(64, 64)
    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, 64, 64)
    out = torch.empty((sc.n_bins, 64, 64), dtype=torch.float32, device="cuda")
    p = sd.render_params(spp=64, max_depth=4, seed=1, wave_paths=1 << 20)
    rc = sd.lib().sdd_render_noalloc(ctx.handle, S.handle, C.byref(c), C.byref(p), C.c_void_p(out.data_ptr()))
    msg = sd.lib().sdd_last_error(ctx.handle).decode()
    say(f"refused: rc={rc} {msg}")
    assert rc == -3 and "static workspace" in msg
    # and graph mode is refused (instantiating a graph allocates)
    p = sd.render_params(spp=1, max_depth=4, seed=1, use_graph=1)
    rc = sd.lib().sdd_render_noalloc(ctx.handle, S.handle, C.byref(c), C.byref(p), C.c_void_p(out.data_ptr()))
    assert rc == -1
