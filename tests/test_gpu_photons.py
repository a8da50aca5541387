"""Caustic photon map on the GPU against the oracle (section 4: photon maps filled from the
light sources, one of them for caustics, and the caustic part of the reflected radiance taken
from it).

Records: both sides follow the same photon paths (the same Philox draws, the window chosen by the
same integer thresholds), so for every photon the oracle does not flag as tied the set of
(photon, vertex) records is equal. Values: positions within 2e-5 (1 + |p|) (FP32 path vertices
after a few bounces), directions within 1e-5, flux within 1e-4 relative (FP32 slab and Fresnel
factors) above 1e-6 of the largest flux.

Gathering: the oracle's records, rounded to FP32, are loaded into a GPU map and rendered; the
oracle renders with the same rounded records. Per pixel (tie-free) the two agree within 1e-4
relative (the bar of the plain renderer) plus the flux of the photons that lie within
r (1 +- tie_radius) of a shading point, which FP32 vertices may count on either side of r
(photon_unc). tie_radius = 1e-3: path vertices carry up to ~1e-5 m of FP32 error, 1e-4 of the
gather radii used here.
"""
import sys

import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.gpu

TIE_RADIUS = 1e-3


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


def _cam(c):
    import paper_1912_04000_amd as sd
    return sd.camera(c.eye, c.target, c.up, c.vfov_deg, c.width, c.height)


def _incidence(sc, ref):
    """Per oracle record: |cos| between the photon's direction and its triangle's normal, and the
    smallest such cosine over the photon's records up to this one (records come in photon, vertex
    order)."""
    v = sc.verts.astype(np.float64)[ref["tri"]]
    nrm = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    c = np.abs(np.einsum("ij,ij->i", nrm, ref["dir"]))
    run = c.copy()
    for k in range(1, len(c)):
        if ref["id"][k] == ref["id"][k - 1]:
            run[k] = min(run[k], run[k - 1])
    return nrm, v[:, 0], run


def _compare_records(gpu, ref, label, sc=None):
    """gpu: (pos, dir, flux, id, vertex) from the map; ref: oracle.photons(...). With the scene
    given, the position bar of a record is divided by the smallest incidence cosine of its photon
    so far (a grazing hit moves the hit point along the surface by the ray's rounding over that
    cosine, and the next rays start there), and every GPU position must lie on the oracle's
    triangle's plane within 1e-5 (1 + |p|)."""
    gpos, gdir, gflux, gid, gvx = gpu
    tied_ids = set(np.nonzero(ref["tied"])[0].tolist())
    gkeys = {(int(i), int(v)): k for k, (i, v) in enumerate(zip(gid, gvx))}
    okeys = {(int(i), int(v)): k for k, (i, v) in enumerate(zip(ref["id"], ref["depth"]))}
    assert len(gkeys) == len(gid), "a (photon, vertex) pair was stored twice"
    g_free = {k for k in gkeys if k[0] not in tied_ids}
    o_free = {k for k in okeys if k[0] not in tied_ids}
    say(f"[{label}] records gpu {len(gid)} oracle {len(ref['id'])}, tied photons {len(tied_ids)}, "
        f"untied records gpu {len(g_free)} oracle {len(o_free)}")
    assert g_free == o_free, (sorted(g_free - o_free)[:5], sorted(o_free - g_free)[:5])
    keys = sorted(o_free)
    gi = np.array([gkeys[k] for k in keys], dtype=np.int64)
    oi = np.array([okeys[k] for k in keys], dtype=np.int64)
    dp = np.abs(gpos[gi] - ref["pos"][oi]).max(axis=1) / (1.0 + np.abs(ref["pos"][oi]).max(axis=1))
    if sc is not None:
        nrm, v0, run = _incidence(sc, ref)
        plane = np.abs(np.einsum("ij,ij->i", gpos[gi].astype(np.float64) - v0[oi], nrm[oi]))
        plane /= 1.0 + np.abs(ref["pos"][oi]).max(axis=1)
        say(f"[{label}] max off-plane {plane.max():.2e}, smallest incidence cos {run[oi].min():.2e}")
        assert plane.max() <= 1e-5
        dp = dp * np.minimum(1.0, run[oi])
    dd = np.abs(gdir[gi] - ref["dir"][oi]).max(axis=1)
    fo = ref["flux"][oi]
    big = np.abs(fo) > 1e-6 * np.abs(fo).max()
    df = np.where(big, np.abs(gflux[gi] - fo) / np.maximum(np.abs(fo), 1e-300), 0.0)
    say(f"[{label}] max pos err {dp.max():.2e}, dir err {dd.max():.2e}, flux rel err {df.max():.2e}")
    assert dp.max() <= 2e-5 and dd.max() <= 1e-5 and df.max() <= 1e-4
    return len(keys)


@pytest.mark.parametrize("n_photons,wave,grid,single", [(50_001, 16_384, (2, 2, 2), False),
                                                        (20_000, 0, (1, 1, 1), True)])
def test_records_window_mirror_receiver(ctx, n_photons, wave, grid, single):
    """Emission through the pane, its reflect/transmit choice, the floor's mirror lobe and the
    storage on the wall; several wavefronts with a ragged last one."""
    import paper_1912_04000_amd as sd
    sc = scenegen.caustic_scene(3, single=single)
    S = _scene(ctx, sc, grid)
    say(f"build: caustic scene, {n_photons} photons, wave {wave}, grid {grid}")
    m = ctx.photon_map(S, sd.photon_params(n_photons, radius=0.15, max_depth=6, seed=7, wave_paths=wave))
    info = m.info()
    ref = oracle.photons(sc, n_photons, max_depth=6, seed=7)
    assert info["n_windows"] == 2 and abs(info["window_area"] - ref["area"]) <= 1e-12 * ref["area"]
    assert info["dropped"] == 0
    n = _compare_records(m.records(), ref, "caustic")
    assert n > 0.99 * n_photons


@pytest.mark.parametrize("B,grid,maps", [(8, (2, 2, 2), False), (13, (4, 2, 2), True)])
def test_records_nave(ctx, B, grid, maps):
    """The nave's window (with a seeded transmittance map when maps is set): photons through it,
    mostly off the stone floor's mirror lobe onto the walls and pillars."""
    import paper_1912_04000_amd as sd
    sc = scenegen.nave_scene(B)
    if maps:
        sc = scenegen.with_glass_maps(sc)
    S = _scene(ctx, sc, grid)
    N = 60_000
    say(f"build: nave {B} bins, maps {maps}, grid {grid}, {N} photons")
    m = ctx.photon_map(S, sd.photon_params(N, radius=0.2, max_depth=7, seed=11, wave_paths=25_000))
    ref = oracle.photons(sc, N, max_depth=7, seed=11)
    n = _compare_records(m.records(), ref, f"nave {B} bins maps {maps}")
    assert n > 1000


def _f32_records(ph):
    out = dict(ph)
    for k in ("pos", "dir", "flux"):
        out[k] = ph[k].astype(np.float32).astype(np.float64)
    return out


def _gather_parity(img, ref, label, min_ok=0.9):
    B = ref.image.shape[0]
    mean_bin = ref.image.reshape(B, -1).mean(axis=1).reshape((B,) + (1,) * (ref.image.ndim - 1))
    tol = 1e-4 * np.maximum(np.abs(ref.image), 1e-3 * mean_bin) + 1.0001 * ref.photon_unc
    ok = ref.tied == 0
    bad = (np.abs(img - ref.image) > tol) & ok[None]
    rel = np.abs(img - ref.image)[:, ok] / np.maximum(np.abs(ref.image)[:, ok], 1e-3 * mean_bin.reshape(B, 1))
    say(f"[{label}] tie-free {ok.mean():.3f}, bad {int(bad.any(axis=0).sum())}, max rel {rel.max():.2e}, "
        f"pixels with an uncertain photon {int((ref.photon_unc > 0).any(axis=0).sum())}")
    assert ok.mean() > min_ok and not bad.any(), np.argwhere(bad)[:5]


def test_gather_caustic_on_the_wall(ctx):
    """The oracle's map loaded into the GPU: a camera over the lit spots on the receiver wall, and
    a path depth that also sees the wall through the floor's mirror."""
    import paper_1912_04000_amd as sd
    sc = scenegen.caustic_scene(3, floor_rho=0.3)
    S = _scene(ctx, sc, (2, 2, 2))
    ph = _f32_records(oracle.photons(sc, 200_000, max_depth=6, seed=7))
    m = sd.PhotonMap(ctx, S, sd.photon_params(200_000, radius=0.15, max_depth=6, seed=7,
                                              capacity=len(ph["id"]) + 10))
    m.load(ph["pos"], ph["dir"], ph["flux"], ph["id"], ph["depth"])
    assert m.info()["stored"] == len(ph["id"])
    cam = scenegen.Camera(eye=(-1.0, 0.0, 8.0), target=(-6.0, 0.0, 9.0), up=(0, 0, 1), vfov_deg=70, width=40,
                          height=32)
    for depth in (1, 3):
        say(f"render: caustic wall, depth {depth}")
        img = ctx.render_photons(S, m, _cam(cam), sd.render_params(spp=2, max_depth=depth, seed=3)).cpu().numpy()
        ref = oracle.render(sc, cam, spp=2, max_depth=depth, seed=3, photons=ph, radius=0.15, tie_radius=TIE_RADIUS)
        _gather_parity(img, ref, f"caustic wall depth {depth}")
        plain = oracle.render(sc, cam, spp=2, max_depth=depth, seed=3)
        assert (ref.image - plain.image).max() > 0.05 * ref.image.max()   # the caustic is in the frame
    # vertices in the dense spots went through the wave-wide pass (more than 48 entries to test)
    assert ctx.stats()["photon_candidates_max"] > 48


@pytest.mark.parametrize("B,grid,radius", [(8, (2, 2, 2), 0.25), (40, (4, 2, 2), 0.1)])
def test_gather_nave(ctx, B, grid, radius):
    import paper_1912_04000_amd as sd
    sc = scenegen.nave_scene(B)
    S = _scene(ctx, sc, grid)
    ph = _f32_records(oracle.photons(sc, 150_000, max_depth=7, seed=5))
    m = sd.PhotonMap(ctx, S, sd.photon_params(150_000, radius=radius, max_depth=7, seed=5))
    m.load(ph["pos"], ph["dir"], ph["flux"], ph["id"], ph["depth"])
    cam = scenegen.nave_camera(48, 40)
    say(f"render: nave {B} bins, radius {radius}, {len(ph['id'])} records")
    img = ctx.render_photons(S, m, _cam(cam), sd.render_params(spp=2, max_depth=5, seed=8)).cpu().numpy()
    ref = oracle.render(sc, cam, spp=2, max_depth=5, seed=8, photons=ph, radius=radius, tie_radius=TIE_RADIUS)
    _gather_parity(img, ref, f"nave {B} bins r {radius}")


def test_empty_map_renders_like_plain(ctx):
    """No photon is stored when the only light through the pane is transmitted (overhead sun, a
    floor that reflects nothing): the render with the empty map equals the plain render bit for
    bit, in eager and graph mode; so does a scene without glass."""
    import paper_1912_04000_amd as sd
    sc = scenegen.caustic_scene(3, floor_n=(1.0,), floor_rho=0.9)
    sc.k_tab[1] = 0.0
    sc.sun_dir[:] = (0.0, 0.0, 1.0)
    S = _scene(ctx, sc, (2, 2, 2))
    m = ctx.photon_map(S, sd.photon_params(30_000, radius=0.2, max_depth=6, seed=2))
    assert m.info()["stored"] == 0 and m.info()["n_windows"] == 2
    cam = _cam(scenegen.Camera(eye=(0.5, 0.2, 2.0), target=(0.0, 0.0, 0.0), up=(0, 1, 0), vfov_deg=80, width=32,
                               height=32))
    p = sd.render_params(spp=2, max_depth=4, seed=4)
    a = ctx.render(S, cam, p).cpu().numpy()
    b = ctx.render_photons(S, m, cam, p).cpu().numpy()
    assert np.array_equal(a, b)
    sc2 = scenegen.plane_scene(n_bins=8)
    S2 = _scene(ctx, sc2, (1, 1, 1))
    m2 = ctx.photon_map(S2, sd.photon_params(1000, radius=0.2, max_depth=4, seed=2))
    assert m2.info()["n_windows"] == 0 and m2.info()["stored"] == 0
    p2 = sd.render_params(spp=1, max_depth=3, seed=4, use_graph=1)
    c2 = _cam(scenegen.Camera(eye=(0, 0, 5), target=(0, 0, 0), up=(0, 1, 0), vfov_deg=60, width=16, height=16))
    assert np.array_equal(ctx.render(S2, c2, p2).cpu().numpy(), ctx.render_photons(S2, m2, c2, p2).cpu().numpy())


def test_graph_replays_equal_eager(ctx):
    import paper_1912_04000_amd as sd
    sc = scenegen.caustic_scene(3, floor_rho=0.3)
    S = _scene(ctx, sc, (2, 2, 2))
    m = ctx.photon_map(S, sd.photon_params(40_000, radius=0.2, max_depth=6, seed=9))
    cam = _cam(scenegen.Camera(eye=(-1.0, 0.0, 8.0), target=(-6.0, 0.0, 9.0), up=(0, 0, 1), vfov_deg=70, width=24,
                               height=24))
    eager = ctx.render_photons(S, m, cam, sd.render_params(spp=2, max_depth=3, seed=1)).cpu().numpy()
    pg = sd.render_params(spp=2, max_depth=3, seed=1, use_graph=1)
    out = None
    for rep in range(3):
        out = ctx.render_photons(S, m, cam, pg, out=out)
        ctx.torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), rep
    assert ctx.stats()["graph_launches"] >= 3


def test_capacity_and_errors(ctx):
    import paper_1912_04000_amd as sd
    sc = scenegen.caustic_scene(3)
    S = _scene(ctx, sc, (2, 2, 2))
    ref = oracle.photons(sc, 5000, max_depth=6, seed=4)
    m = ctx.photon_map(S, sd.photon_params(5000, radius=0.2, max_depth=6, seed=4, capacity=300))
    info = m.info()
    n_tied = int(ref["tied"].sum())
    say(f"capacity 300: stored {info['stored']}, dropped {info['dropped']}, oracle records {len(ref['id'])}")
    assert info["stored"] == 300 and abs(info["stored"] + info["dropped"] - len(ref["id"])) <= 2 * n_tied
    # records of the kept photons are still the oracle's
    pos, dr, fl, pid, vx = m.records(300)
    okeys = {(int(i), int(v)): k for k, (i, v) in enumerate(zip(ref["id"], ref["depth"]))}
    tied = set(np.nonzero(ref["tied"])[0].tolist())
    for k in range(300):
        if int(pid[k]) in tied:
            continue
        o = okeys[(int(pid[k]), int(vx[k]))]
        assert np.abs(fl[k] - ref["flux"][o]).max() <= 1e-4 * np.abs(ref["flux"][o]).max()
    with pytest.raises(sd.SddError):
        m.records(301)
    cam = _cam(scenegen.Camera(eye=(0, 0, 5), target=(0, 0, 0), up=(0, 1, 0), vfov_deg=60, width=8, height=8))
    unbuilt = sd.PhotonMap(ctx, S, sd.photon_params(100, radius=0.2))
    with pytest.raises(sd.SddError) as e:
        ctx.render_photons(S, unbuilt, cam, sd.render_params())
    assert e.value.code == -5
    S8 = _scene(ctx, scenegen.caustic_scene(8), (2, 2, 2))
    with pytest.raises(sd.SddError) as e:
        ctx.render_photons(S8, m, cam, sd.render_params())
    assert e.value.code == -5
    with pytest.raises(sd.SddError):
        ctx.render_photons(S, m, cam, sd.render_params(mode=sd.MODE_CACHED))


def test_church_photons_full_size(ctx):
    """The benchmarked church (979,664 triangles, 40 windows, 40 bins, 8x4x4 cells) and its caustic
    map as bench.py builds it: 4M photons, depth 8, radius 0.1 m, 2^20 photons in flight. Records
    of every 16th photon against the oracle's (a sample it traces one photon at a time). Then that
    sample, loaded as a map of its own with a 0.5 m radius, gathered in the benchmarked frame
    (1920x1080, 8 spp, depth 8, 2^24 paths in flight) on 300 sampled pixels against the oracle."""
    import paper_1912_04000_amd as sd
    import torch
    sc = scenegen.church_scene(40)
    S = _scene(ctx, sc, (8, 4, 4))
    N = 4_000_000
    say("build: church, 4M photons")
    m = ctx.photon_map(S, sd.photon_params(N, radius=0.1, max_depth=8, seed=1, capacity=N // 4))
    info = m.info()
    assert info["dropped"] == 0 and info["n_windows"] == 80
    pos, dr, fl, pid, vx = m.records()
    keep = pid % 16 == 0
    say(f"church map: {info['stored']} records, {int(keep.sum())} of sampled photons; oracle sample ...")
    ref = oracle.photons(sc, N, max_depth=8, seed=1, stride=16)
    _compare_records((pos[keep], dr[keep], fl[keep], pid[keep], vx[keep]), ref, "church 4M, every 16th photon")
    assert abs(info["window_area"] - ref["area"]) <= 1e-12 * ref["area"]

    ph = _f32_records(ref)
    m2 = sd.PhotonMap(ctx, S, sd.photon_params(N, radius=0.5, max_depth=8, seed=1, capacity=len(ph["id"]) + 1))
    m2.load(ph["pos"], ph["dir"], ph["flux"], ph["id"], ph["depth"])
    cam = scenegen.church_camera()
    say("render: church 1920x1080 8 spp depth 8 with the sampled map")
    img = ctx.render_photons(S, m2, _cam(cam), sd.render_params(spp=8, max_depth=8, seed=5, wave_paths=1 << 24))
    px = np.sort(np.random.default_rng(21).choice(cam.width * cam.height, 300, replace=False))
    g = img.reshape(40, -1)[:, torch.from_numpy(px).cuda()].cpu().numpy()
    r = oracle.render(sc, cam, spp=8, max_depth=8, seed=5, pixels=px, photons=ph, radius=0.5,
                      tie_radius=TIE_RADIUS)
    plain = oracle.render(sc, cam, spp=8, max_depth=8, seed=5, pixels=px)
    lit = ((r.image - plain.image) > 1e-3 * r.image).any(axis=0) & (r.tied == 0)
    say(f"sampled pixels with caustic light: {int(lit.sum())}")
    assert lit.sum() >= 5
    # 8 samples of 8 vertices in a million-triangle mesh: a pixel is tied when any of its samples
    # passes near an edge or a lobe threshold (as in the church test of the plain renderer)
    _gather_parity(g, r, "church frame, sampled map r 0.5", min_ok=0.5)


# -- global maps ---------------------------------------------------------------------------
@pytest.mark.parametrize("B,grid,wave", [(4, (2, 2, 2), 30_000), (13, (1, 1, 1), 0)])
def test_global_records_window_box(ctx, B, grid, wave):
    """A closed room lit through a ceiling window: every photon stored at every opaque vertex it
    reaches, continued by the mirror or the diffuse lobe (Fresnel factor of the new direction)."""
    import paper_1912_04000_amd as sd
    sc = scenegen.window_box_scene(B)
    S = _scene(ctx, sc, grid)
    N = 40_001
    say(f"build: window box {B} bins, global map, {N} photons, wave {wave}")
    m = ctx.photon_map(S, sd.photon_params(N, radius=0.1, max_depth=8, seed=3, wave_paths=wave,
                                           kind=sd.PHOTON_GLOBAL))
    ref = oracle.photons(sc, N, max_depth=8, seed=3, global_map=True)
    assert m.info()["dropped"] == 0
    n = _compare_records(m.records(), ref, f"global window box {B} bins", sc)
    assert n > 5 * N


def test_global_records_nave_with_maps(ctx):
    import paper_1912_04000_amd as sd
    sc = scenegen.with_glass_maps(scenegen.nave_scene(8))
    S = _scene(ctx, sc, (4, 2, 2))
    N = 30_000
    m = ctx.photon_map(S, sd.photon_params(N, radius=0.2, max_depth=6, seed=12, kind=sd.PHOTON_GLOBAL))
    ref = oracle.photons(sc, N, max_depth=6, seed=12, global_map=True)
    _compare_records(m.records(), ref, "global nave with glass maps", sc)


def _load(ctx, S, ph, radius, kind):
    import paper_1912_04000_amd as sd
    m = sd.PhotonMap(ctx, S, sd.photon_params(max(1, len(ph["id"])), radius=radius, capacity=len(ph["id"]) + 1,
                                              kind=kind))
    m.load(ph["pos"], ph["dir"], ph["flux"], ph["id"], ph["depth"])
    return m


@pytest.mark.parametrize("gl_from,spp", [(1, 2), (2, 2), (3, 1)])
def test_global_gather_window_box(ctx, gl_from, spp):
    """The oracle's global and caustic maps (rounded to FP32) loaded into GPU maps; camera paths
    with the caustic map before vertex gl_from and the global map from there on, against the
    oracle with the same maps."""
    import paper_1912_04000_amd as sd
    sc = scenegen.window_box_scene(4)
    S = _scene(ctx, sc, (2, 2, 2))
    g = _f32_records(oracle.photons(sc, 60_000, max_depth=10, seed=5, global_map=True))
    c = _f32_records(oracle.photons(sc, 200_000, max_depth=10, seed=6))
    mg = _load(ctx, S, g, 0.1, sd.PHOTON_GLOBAL)
    mc = _load(ctx, S, c, 0.15, sd.PHOTON_CAUSTIC)
    cam = scenegen.Camera(eye=(3.5, 3.5, 2.5), target=(1.0, 1.2, 0.0), up=(0, 0, 1), vfov_deg=75, width=40,
                          height=32)
    say(f"render: window box, global from vertex {gl_from}, {len(g['id'])} + {len(c['id'])} records")
    img = ctx.render_photons(S, mc, _cam(cam), sd.render_params(spp=spp, max_depth=8, seed=4), global_map=mg,
                             global_from=gl_from).cpu().numpy()
    # the oracle takes one tie radius for both maps; the global gather reports its bound there too
    ref = oracle.render(sc, cam, spp=spp, max_depth=8, seed=4, photons=c, radius=0.15, tie_radius=TIE_RADIUS,
                        global_photons=g, global_radius=0.1, global_depth=gl_from)
    _gather_parity(img, ref, f"window box global from {gl_from}")


def test_global_gather_nave_and_graph(ctx):
    import paper_1912_04000_amd as sd
    sc = scenegen.nave_scene(8)
    S = _scene(ctx, sc, (2, 2, 2))
    g = _f32_records(oracle.photons(sc, 60_000, max_depth=8, seed=9, global_map=True))
    mg = _load(ctx, S, g, 0.25, sd.PHOTON_GLOBAL)
    cam = scenegen.nave_camera(40, 32)
    p = sd.render_params(spp=2, max_depth=6, seed=8)
    img = ctx.render_photons(S, None, _cam(cam), p, global_map=mg, global_from=2).cpu().numpy()
    ref = oracle.render(sc, cam, spp=2, max_depth=6, seed=8, global_photons=g, global_radius=0.25,
                        tie_radius=TIE_RADIUS, global_depth=2)
    _gather_parity(img, ref, "nave global from vertex 2")
    pg = sd.render_params(spp=2, max_depth=6, seed=8, use_graph=1)
    out = None
    for rep in range(2):
        out = ctx.render_photons(S, None, _cam(cam), pg, out=out, global_map=mg, global_from=2)
        ctx.torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), img), rep
    # argument errors: kinds swapped, no map, global_from < 1
    mc = _load(ctx, S, g, 0.25, sd.PHOTON_CAUSTIC)
    for kw in (dict(pmap=mg), dict(pmap=None, global_map=mc, global_from=1), dict(pmap=None),
               dict(pmap=None, global_map=mg, global_from=0)):
        pm = kw.pop("pmap")
        with pytest.raises(sd.SddError) as e:
            ctx.render_photons(S, pm, _cam(cam), p, **kw)
        assert e.value.code == -1


def test_church_global_map_full_size(ctx):
    """The benchmarked church's global map as bench.py builds it (2M photons, depth 8, radius
    0.15 m, 2^20 photons in flight): records of every 32nd photon against the oracle's sample; then
    that sample loaded with a 0.5 m radius and gathered from vertex 2 on in the benchmarked frame
    (1920x1080, 8 spp, depth 8, 2^24 paths in flight) on 200 sampled pixels."""
    import paper_1912_04000_amd as sd
    import torch
    sc = scenegen.church_scene(40)
    S = _scene(ctx, sc, (8, 4, 4))
    N = 2_000_000
    say("build: church global map, 2M photons")
    m = ctx.photon_map(S, sd.photon_params(N, radius=0.15, max_depth=8, seed=1, capacity=6 * N,
                                           kind=sd.PHOTON_GLOBAL))
    info = m.info()
    assert info["dropped"] == 0
    pos, dr, fl, pid, vx = m.records()
    keep = pid % 32 == 0
    say(f"church global map: {info['stored']} records; oracle sample ...")
    ref = oracle.photons(sc, N, max_depth=8, seed=1, stride=32, global_map=True)
    _compare_records((pos[keep], dr[keep], fl[keep], pid[keep], vx[keep]), ref, "church global, every 32nd photon",
                     sc)
    ph = _f32_records(ref)
    m2 = _load(ctx, S, ph, 0.5, sd.PHOTON_GLOBAL)
    cam = scenegen.church_camera()
    say("render: church 1920x1080 8 spp depth 8, global map from vertex 2")
    img = ctx.render_photons(S, None, _cam(cam), sd.render_params(spp=8, max_depth=8, seed=5, wave_paths=1 << 24),
                             global_map=m2, global_from=2)
    px = np.sort(np.random.default_rng(22).choice(cam.width * cam.height, 200, replace=False))
    g = img.reshape(40, -1)[:, torch.from_numpy(px).cuda()].cpu().numpy()
    r = oracle.render(sc, cam, spp=8, max_depth=8, seed=5, pixels=px, global_photons=ph, global_radius=0.5,
                      tie_radius=TIE_RADIUS, global_depth=2)
    _gather_parity(g, r, "church frame, global sample map from vertex 2", min_ok=0.5)
