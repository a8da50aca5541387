"""Cell scheduling of the traversal: the tile list built fullest cells first (section 5: the
sub-model with the most waiting rays is taken next) against the oracle, and against the cell
index order, whose images it must reproduce bit for bit (a ray's result does not depend on which
workgroup traces it or when, and the image update runs in slot order).
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
def ctx():
    import paper_1912_04000_amd as sd
    return sd.Context(0)


def _pixel_parity(img, ref, tied, label):
    B = ref.shape[0]
    mean_bin = ref.reshape(B, -1).mean(axis=1)
    tol = 1e-4 * np.maximum(np.abs(ref), 1e-3 * mean_bin[:, None, None])
    ok = tied == 0
    bad = (np.abs(img - ref) > tol) & ok[None]
    say(f"[{label}] pixels={ok.size} tie-free={ok.sum()} bad={bad.any(axis=0).sum()}")
    assert not bad.any(), np.argwhere(bad)[:10]
    return ok


# (2, 2, 2): counts staged in LDS; (8, 8, 8): 12288 queue keys, read from memory; (3, 2, 5): a
# ragged grid; three rounds: rays migrate through the queues between cells
@pytest.mark.parametrize("grid,rounds,wave", [((2, 2, 2), 0, 0), ((8, 8, 8), 0, 777), ((3, 2, 5), 3, 0),
                                              ((8, 8, 8), 4, 0)])
def test_fullest_first_matches_oracle_and_index_order(ctx, grid, rounds, wave):
    import paper_1912_04000_amd as sd
    sc = scenegen.nave_scene(8)
    cam = scenegen.nave_camera(48, 40)
    S = sd.Scene.from_description(sc, grid=grid)
    ctx.upload(S)
    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height)
    say(f"fullest first: grid={grid} rounds={rounds} wave={wave}")
    imgs = [ctx.render(S, c, sd.render_params(spp=2, max_depth=6, seed=5, wave_paths=wave, queue_rounds=rounds,
                                               cell_order=order)).cpu().numpy() for order in (0, 1)]
    assert np.array_equal(imgs[0], imgs[1])
    ref = oracle.render(sc, cam, spp=2, max_depth=6, seed=5)
    ok = _pixel_parity(imgs[1], ref.image, ref.tied, f"grid={grid} rounds={rounds}")
    assert ok.mean() > 0.9


def test_fullest_first_church_one_spp_identical(ctx):
    """The church frame (8 x 4 x 4 cells, 2^25-path wavefronts) at 1 spp in both orders: the same
    image bit for bit, and the same traversal work counted."""
    import paper_1912_04000_amd as sd
    sc = scenegen.church_scene(40)
    cam = scenegen.church_camera()
    S = sd.Scene.from_description(sc, grid=(8, 4, 4))
    ctx.upload(S)
    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height)
    imgs, stats = [], []
    for order in (0, 1):
        say(f"church 1 spp, cell_order={order}")
        ctx.finish()
        ctx.reset_stats()
        imgs.append(ctx.render(S, c, sd.render_params(spp=1, max_depth=8, seed=3, wave_paths=1 << 25,
                                                      cell_order=order)).cpu().numpy())
        ctx.finish()
        stats.append(ctx.stats())
    assert np.array_equal(imgs[0], imgs[1])
    for k in ("cell_visits", "node_visits", "tri_tests", "vertices", "shadow_rays"):
        assert stats[0][k] == stats[1][k], (k, stats[0][k], stats[1][k])


def test_cell_order_out_of_range_is_rejected(ctx):
    import paper_1912_04000_amd as sd
    sc = scenegen.nave_scene(8)
    cam = scenegen.nave_camera(8, 8)
    S = sd.Scene.from_description(sc, grid=(2, 2, 2))
    ctx.upload(S)
    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height)
    with pytest.raises(sd.SddError, match="cell_order"):
        ctx.render(S, c, sd.render_params(spp=1, max_depth=2, seed=1, cell_order=2))


def test_smaller_workspace_orders_coarser_and_renders_the_same(ctx):
    """A workspace below sdd_workspace_bytes gets fewer origin blocks per queue key (the most whose
    counters fit, down to none): only the order of rays inside a key changes, so the image equals
    the full workspace's bit for bit; a workspace below the plan without blocks is refused. The
    96 x 96 x 8-spp render keeps 73,728 paths in flight, enough for two block levels on 8 cells."""
    import ctypes as C
    import torch
    import paper_1912_04000_amd as sd
    sc = scenegen.nave_scene(8)
    cam = scenegen.nave_camera(96, 96)
    S = sd.Scene.from_description(sc, grid=(2, 2, 2))
    ctx.upload(S)
    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height)
    # as many paths in flight as the frame has samples, so that sdd_workspace_bytes (which knows no
    # camera) sizes the same wavefront as the render
    p = sd.render_params(spp=8, max_depth=5, seed=3, wave_paths=96 * 96 * 8)
    full = ctx.workspace_bytes(S, p)
    ref = ctx.render(S, c, p).cpu().numpy()
    ws = ctx.workspace(full)
    img = torch.empty((8, cam.height, cam.width), dtype=torch.float32, device="cuda")
    rendered, refused = 0, 0
    for cut in (1, 1 << 10, 1 << 14, 1 << 17, 1 << 18, 1 << 19, 3 << 18, 1 << 20, 1 << 21):
        nbytes = full - cut
        rc = sd.lib().sdd_render(ctx.handle, S.handle, C.byref(c), C.byref(p), C.c_void_p(ws.data_ptr()),
                                 nbytes, C.c_void_p(img.data_ptr()))
        if rc != 0:
            with pytest.raises(sd.SddError, match="workspace too small"):
                ctx._err(rc)
            say(f"workspace {nbytes} of {full} bytes: refused")
            refused += 1
            break
        ctx.finish()
        same = np.array_equal(img.cpu().numpy(), ref)
        say(f"workspace {nbytes} of {full} bytes: identical={same}")
        assert same
        rendered += 1
    assert rendered >= 2 and refused == 1


def test_noalloc_church_fits_the_static_workspace_and_matches(ctx):
    """The church (128 cells, 40 bins, 1920 x 1080) through sdd_render_noalloc: its 64 MiB static
    workspace cannot hold the full-depth queue sub-ranges (75 MB) beside a wavefront, so the render
    takes fewer origin blocks and fewer paths in flight. At 1 spp every pixel holds one sample, so
    the image equals sdd_render's (full workspace, 2^20 paths in flight) bit for bit."""
    import torch
    import paper_1912_04000_amd as sd
    sc = scenegen.church_scene(40)
    cam = scenegen.church_camera()
    S = sd.Scene.from_description(sc, grid=(8, 4, 4))
    ctx.upload(S)
    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height)
    p = sd.render_params(spp=1, max_depth=8, seed=5)
    say("church 1 spp: sdd_render, then sdd_render_noalloc")
    ref = ctx.render(S, c, p).cpu().numpy()
    out = torch.empty((40, cam.height, cam.width), dtype=torch.float32, device="cuda")
    img = ctx.render_noalloc(S, c, p, out=out).cpu().numpy()
    same = np.array_equal(img, ref)
    say(f"church noalloc identical={same} mean={float(ref.mean()):.4e}")
    assert same and float(ref.mean()) > 0.0
