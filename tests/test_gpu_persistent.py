"""The persistent batched render (one kernel for a whole batch of views, lanes taking
(view, 8 x 8 tile, sample) items from a device work list) against the oracle.

Each lane carries one path through all its vertices with the wavefront kernels' random-number
counters and arithmetic, so every view must equal oracle.render(view=v) within the parity bar
(|a - b| <= 1e-4 max(|b|, 1e-3 mean_bin) on tie-free pixels); pixels are accumulated with float
atomics, so only the order of the spp additions into a pixel differs from the wavefront path.
Cases: ragged views (edges cutting 8 x 8 tiles), a batch of uneven sizes and spp (eager and a
replayed graph), fewer lanes than paths (lanes take many items), more lanes than paths, a
non-zero sky, glass with transmittance maps, dispersive 13 and 80 bins, an 8x8x8 grid whose cell
table is read from memory, and sampled pixels of the full-size church frame.
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


def _cam(sd, cam):
    return sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height)


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


@pytest.mark.parametrize("grid,lanes,size", [((2, 2, 2), 0, (45, 37)), ((4, 2, 2), 2048, (48, 40)),
                                             ((3, 5, 7), 6144, (31, 9)), ((8, 8, 8), 0, (24, 20)),
                                             ((1, 1, 1), 0, (8, 8))])
def test_persistent_single_view(ctx, grid, lanes, size):
    import paper_1912_04000_amd as sd
    sc = scenegen.nave_scene(8)
    cam = scenegen.nave_camera(*size)
    S = _scene(ctx, sc, grid)
    say(f"persistent: grid={grid} lanes={lanes} size={size}")
    ctx.reset_stats()
    img = ctx.render(S, _cam(sd, cam), sd.render_params(spp=3, max_depth=6, seed=21, wave_paths=lanes,
                                                        persistent=1)).cpu().numpy()
    st = ctx.stats()
    ref = oracle.render(sc, cam, spp=3, max_depth=6, seed=21)
    ok = _pixel_parity(img, ref.image, ref.tied, f"persistent grid={grid} lanes={lanes} {size}")
    assert ok.mean() > 0.9
    assert st["paths"] == size[0] * size[1] * 3
    assert st["trace_launches"] == 1 and st["shade_launches"] == 0
    assert st["err_nonfinite"] == 0 and st["err_cross_overflow"] == 0


def _views(sd):
    return [sd.camera((3.0, 8.0, 1.7), (12.0, 1.0, 1.5), (0, 0, 1), 60, 40, 30),
            sd.camera((15.0, 2.0, 3.0), (5.0, 8.0, 1.0), (0, 0, 1), 75, 17, 23),
            sd.camera((10.0, 5.0, 6.0), (10.0, 5.0, 0.0), (0, 1, 0), 90, 32, 32)]


def _oracle_cam(c):
    return scenegen.Camera(eye=tuple(c.eye), target=tuple(c.target), up=tuple(c.up), vfov_deg=c.vfov_deg,
                           width=c.width, height=c.height)


@pytest.mark.parametrize("use_graph", [0, 1])
def test_persistent_batch_matches_oracle_per_view(ctx, use_graph):
    """Three views of uneven size and spp in one persistent launch; view v against
    oracle.render(view=v). In graph mode the capture is replayed twice with an eager render of
    another kind in between."""
    import paper_1912_04000_amd as sd
    sc = scenegen.nave_scene(8)
    S = _scene(ctx, sc, (2, 2, 2))
    cams = _views(sd)
    spp = [3, 1, 5]
    refs = [oracle.render(sc, _oracle_cam(c), spp=s, max_depth=5, seed=9, view=v)
            for v, (c, s) in enumerate(zip(cams, spp))]
    p = sd.render_params(max_depth=5, seed=9, wave_paths=4096, use_graph=use_graph, persistent=1)
    outs = None
    for rep in range(2 if use_graph else 1):
        outs = ctx.render_batch(S, cams, spp, p, outs=outs)
        for v in range(len(cams)):
            ok = _pixel_parity(outs[v].cpu().numpy(), refs[v].image, refs[v].tied,
                               f"persistent view {v} ({cams[v].width}x{cams[v].height}, {spp[v]} spp) "
                               f"graph={use_graph} replay {rep}")
            assert ok.mean() > 0.9
        ctx.render(S, cams[1], sd.render_params(spp=1, max_depth=3, seed=rep))
    if use_graph:
        assert ctx.stats()["graph_launches"] >= 2


def test_persistent_environment_and_glass_maps(ctx):
    """A non-zero sky (escapes add it) and transmittance maps on the window (glass shading and
    the shadow rays' crossings read them)."""
    import paper_1912_04000_amd as sd
    sc = scenegen.with_glass_maps(scenegen.nave_scene(8))
    sc.env = np.linspace(0.2, 0.6, 8).astype(np.float32)
    cam = scenegen.nave_camera(40, 33)
    S = _scene(ctx, sc, (2, 2, 2))
    img = ctx.render(S, _cam(sd, cam), sd.render_params(spp=2, max_depth=6, seed=31, persistent=1)).cpu().numpy()
    ref = oracle.render(sc, cam, spp=2, max_depth=6, seed=31)
    ok = _pixel_parity(img, ref.image, ref.tied, "persistent env + maps")
    assert ok.mean() > 0.9


@pytest.mark.parametrize("B", [13, 80])
def test_persistent_dispersive_bins(ctx, B):
    import paper_1912_04000_amd as sd
    sc = scenegen.nave_scene(B)
    t = (np.arange(B) + 0.5) / B
    n = sc.n_tab.copy()
    for m in range(sc.n_mat):
        n[m] = 1.52 + 0.02 * (1.0 - t) if sc.mat_type[m] == scenegen.MAT_GLASS else 1.6 + 0.04 * np.sin(7.0 * t + m)
    sc = dataclasses.replace(sc, n_tab=n.astype(np.float32)).check()
    cam = scenegen.nave_camera(32, 24)
    S = _scene(ctx, sc, (2, 2, 2))
    img = ctx.render(S, _cam(sd, cam), sd.render_params(spp=2, max_depth=6, seed=8, persistent=1)).cpu().numpy()
    ref = oracle.render(sc, cam, spp=2, max_depth=6, seed=8)
    ok = _pixel_parity(img, ref.image, ref.tied, f"persistent B={B}")
    assert ok.mean() > 0.9


def test_persistent_church_sampled(ctx):
    """The church frame (1920 x 1080, 40 bins, depth 8, 8 x 4 x 4 cells) at 2 spp in one
    persistent launch, 4000 sampled pixels against the oracle."""
    import paper_1912_04000_amd as sd
    import torch
    sc = scenegen.church_scene(40)
    cam = scenegen.church_camera()
    S = _scene(ctx, sc, (8, 4, 4))
    say("persistent church 2 spp")
    img = ctx.render(S, _cam(sd, cam), sd.render_params(spp=2, max_depth=8, seed=13, persistent=1))
    rng = np.random.default_rng(4)
    px = np.sort(rng.choice(cam.width * cam.height, 4000, replace=False))
    g = img.reshape(40, -1)[:, torch.from_numpy(px).cuda()].cpu().numpy()
    ref = oracle.render(sc, cam, spp=2, max_depth=8, seed=13, pixels=px)
    mean_bin = ref.image.mean(axis=1)
    tol = 1e-4 * np.maximum(np.abs(ref.image), 1e-3 * mean_bin[:, None])
    ok = ref.tied == 0
    bad = ((np.abs(g - ref.image) > tol) & ok[None]).any(axis=0)
    say(f"persistent church: sampled={len(px)} tie-free={ok.sum()} bad={bad.sum()}")
    # two samples of up to 8 vertices each: about one pixel in eight has a tied sample
    assert ok.mean() > 0.8 and not bad.any()


def test_persistent_rejected_where_unsupported(ctx):
    import paper_1912_04000_amd as sd
    sc = scenegen.nave_scene(8)
    cam = scenegen.nave_camera(8, 8)
    S = _scene(ctx, sc, (2, 2, 2))
    c = _cam(sd, cam)
    with pytest.raises(sd.SddError, match="noalloc"):
        import torch
        ctx.render_noalloc(S, c, sd.render_params(spp=1, max_depth=2, seed=1, persistent=1),
                           out=torch.empty((8, 8, 8), dtype=torch.float32, device="cuda"))
    with pytest.raises(sd.SddError, match="persistent"):
        ctx.render(S, c, sd.render_params(spp=1, max_depth=2, seed=1, persistent=2))
    with pytest.raises(sd.SddError, match="2\\^19"):
        ctx.render(S, c, sd.render_params(spp=1, max_depth=2, seed=1, persistent=1, wave_paths=1 << 20))
