"""Radiance cache on the GPU (through the C ABI) against the FP64 oracle of oracle/mlp.py.

Bars (bf16 matrix-core arithmetic with FP32 accumulation against FP64 with the same bf16
roundings; see the tolerance derivation in the design notes):
  network outputs   relative L2 <= 1e-2, max |error| <= 3e-2 max |y|
  gradients         per tensor cosine >= 0.999 and relative L2 <= 2e-2
  first Adam step   closed form p - lr g / (|g| + eps) on the GPU's own gradient, FP32 rounding
  training records  validity and material exact, position / direction within 1e-5, targets within
                    the renderer's 1e-4 bar, on paths the oracle does not flag as tied
"""
import sys

import numpy as np
import pytest

import oracle
import scenegen
from oracle import mlp

pytestmark = pytest.mark.gpu

SMALL = dict(levels_pos=4, log2_table_pos=12, nmin_pos=2.0, nmax_pos=64.0, levels_dir=3, log2_table_dir=8,
             nmin_dir=2.0, nmax_dir=32.0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_1912_04000_amd as sd
    return sd.Context(0)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _ocfg(kw):
    return mlp.CacheConfig(levels_pos=kw["levels_pos"], log2_table_pos=kw["log2_table_pos"], nmin_pos=kw["nmin_pos"],
                           nmax_pos=kw["nmax_pos"], levels_dir=kw["levels_dir"], log2_table_dir=kw["log2_table_dir"],
                           nmin_dir=kw["nmin_dir"], nmax_dir=kw["nmax_dir"])


def _params(kw, n_mat, seed, grid_scale=3e3):
    """Oracle parameters that FP32 masters hold exactly, grids bf16-representable (the renderer
    interpolates bf16 grid values)."""
    P = mlp.CacheParams(_ocfg(kw), n_mat).init(seed)
    P.arrays["pos"] *= grid_scale
    P.arrays["dir"] *= grid_scale
    for k in P.arrays:
        P.arrays[k] = P.arrays[k].astype(np.float32).astype(np.float64)
    P.arrays["pos"] = mlp.bf16(P.arrays["pos"])
    P.arrays["dir"] = mlp.bf16(P.arrays["dir"])
    return P


def _records(n, seed, lo, hi, n_mat, B):
    rng = np.random.default_rng(seed)
    x = rng.uniform(lo, hi, size=(n, 3)).astype(np.float32)
    w = rng.normal(size=(n, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    w = w.astype(np.float32)
    mat = rng.integers(0, n_mat, n).astype(np.int32)
    t = rng.uniform(0.0, 1.5, size=(n, B)).astype(np.float32)
    return x, w, mat, t


def _oracle_rows(P, x, w, mat, lo, hi, B):
    n = x.shape[0]
    xs = np.repeat(x.astype(np.float64), B, axis=0)
    ws = np.repeat(w.astype(np.float64), B, axis=0)
    ms = np.repeat(mat, B)
    lt = np.tile((np.arange(B) + 0.5) / B, n)
    inp, taps = mlp.encode(P, xs, ws, ms, lo, hi, lt)
    return inp, taps, ms


def _make_cache(ctx, kw, n_mat, lo, hi, B, **extra):
    import paper_1912_04000_amd as sd
    cfg = sd.cache_config(n_mat, lo, hi, max_bins=B, **{**kw, **extra})
    return sd.Cache(ctx, cfg)


@pytest.mark.parametrize("kw,B,n", [(SMALL, 8, 200), (SMALL, 13, 77),
                                    (dict(levels_pos=12, log2_table_pos=19, nmin_pos=16.0, nmax_pos=2048.0,
                                          levels_dir=12, log2_table_dir=14, nmin_dir=4.0, nmax_dir=256.0), 40, 160),
                                    (dict(levels_pos=12, log2_table_pos=19, nmin_pos=16.0, nmax_pos=2048.0,
                                          levels_dir=12, log2_table_dir=14, nmin_dir=4.0, nmax_dir=256.0), 80, 97)])
def test_cache_eval_matches_oracle(ctx, kw, B, n):
    lo, hi, n_mat = [-3.0, -1.0, 0.0], [17.0, 11.0, 8.5], 5
    P = _params(kw, n_mat, 3)
    cache = _make_cache(ctx, kw, n_mat, lo, hi, B, max_records=4096, max_step=1024)
    assert cache.n_param == P.size()
    info = cache.info()
    c = _ocfg(kw)
    assert info["npos"] == mlp.level_resolutions(c.nmin_pos, c.nmax_pos, c.levels_pos)
    assert info["ndir"] == mlp.level_resolutions(c.nmin_dir, c.nmax_dir, c.levels_dir)
    cache.set_params(P.flat())
    np.testing.assert_array_equal(cache.params(), P.flat().astype(np.float32))
    x, w, mat, _ = _records(n, 4, lo, hi, n_mat, B)
    y = cache.eval(_dev(x), _dev(w), _dev(mat), B).cpu().numpy()
    inp, _, _ = _oracle_rows(P, x, w, mat, lo, hi, B)
    yo, _ = mlp.forward(P, inp, bf=True)
    yo = yo.reshape(n, B)
    err = np.abs(y - yo)
    rel_l2 = np.linalg.norm(y - yo) / np.linalg.norm(yo)
    say(f"eval B={B} n={n}: |y| max {np.abs(yo).max():.3e}, rel L2 {rel_l2:.2e}, max err {err.max():.2e}")
    assert rel_l2 <= 1e-2
    assert err.max() <= 3e-2 * np.abs(yo).max()


def test_cache_eval_ragged_and_tiny(ctx):
    """One vertex, one bin; and a count that leaves a partial wave."""
    lo, hi, n_mat = [0.0, 0.0, 0.0], [1.0, 1.0, 1.0], 2
    P = _params(SMALL, n_mat, 9)
    cache = _make_cache(ctx, SMALL, n_mat, lo, hi, 3, max_records=64, max_step=32)
    cache.set_params(P.flat())
    for n, B in ((1, 1), (33, 3)):
        x, w, mat, _ = _records(n, 5 + n, lo, hi, n_mat, B)
        y = cache.eval(_dev(x), _dev(w), _dev(mat), B).cpu().numpy()
        inp, _, _ = _oracle_rows(P, x, w, mat, lo, hi, B)
        yo, _ = mlp.forward(P, inp, bf=True)
        np.testing.assert_allclose(y.ravel(), yo, rtol=3e-2, atol=3e-2 * np.abs(yo).max())


@pytest.mark.parametrize("B,n", [(8, 300), (5, 1024)])
def test_cache_gradients_match_oracle(ctx, B, n):
    lo, hi, n_mat = [-3.0, -1.0, 0.0], [17.0, 11.0, 8.5], 4
    P = _params(SMALL, n_mat, 11)
    cache = _make_cache(ctx, SMALL, n_mat, lo, hi, B, max_records=2048, max_step=1024)
    cache.set_params(P.flat())
    x, w, mat, t = _records(n, 12, lo, hi, n_mat, B)
    cache.backward(_dev(x), _dev(w), _dev(mat), _dev(t))
    g = cache.grads()
    loss = cache.loss()
    inp, taps, ms = _oracle_rows(P, x, w, mat, lo, hi, B)
    y, cch = mlp.forward(P, inp, bf=True)
    go = mlp.backward(P, taps, cch, y, t.ravel().astype(np.float64), ms, bf=True)
    lo_ = mlp.rel_l2(y, t.ravel())
    say(f"grad B={B} n={n}: loss gpu {loss:.6f} oracle {lo_:.6f}")
    assert loss == pytest.approx(lo_, rel=2e-2)
    off = 0
    for k, shape in P.shapes:
        size = int(np.prod(shape))
        a = g[off:off + size].astype(np.float64)
        b = go[k].ravel()
        off += size
        nb = np.linalg.norm(b)
        assert nb > 0, k
        cos = a @ b / (np.linalg.norm(a) * nb)
        rel = np.linalg.norm(a - b) / nb
        say(f"  {k:4s} cos {cos:.6f} rel L2 {rel:.2e}")
        assert cos >= 0.999 and rel <= 2e-2, k


def test_first_adam_step_closed_form(ctx):
    lo, hi, n_mat, B = [0.0, 0.0, 0.0], [4.0, 4.0, 4.0], 3, 6
    P = _params(SMALL, n_mat, 21)
    cache = _make_cache(ctx, SMALL, n_mat, lo, hi, B, max_records=512, max_step=256, lr=1e-3)
    cache.set_params(P.flat())
    x, w, mat, t = _records(256, 22, lo, hi, n_mat, B)
    cache.backward(_dev(x), _dev(w), _dev(mat), _dev(t))
    g = cache.grads().astype(np.float64)
    p0 = cache.params().astype(np.float64)
    cache.step()
    p1 = cache.params().astype(np.float64)
    assert cache.info()["adam_steps"] == 1
    expect = p0 - 1e-3 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(p1, expect, rtol=0, atol=2e-7 * np.maximum(1.0, np.abs(p0)).max())
    # the gradient buffer is cleared by the step
    assert np.all(cache.grads() == 0.0)


def test_training_fits_a_smooth_field(ctx):
    """Online Adam on records of a smooth radiance-like field: the loss falls by an order of
    magnitude and the network reproduces held-out records."""
    lo, hi, n_mat, B = [0.0, 0.0, 0.0], [10.0, 6.0, 4.0], 3, 8
    cache = _make_cache(ctx, SMALL, n_mat, lo, hi, B, max_records=8192, max_step=2048, lr=1e-2)
    cache.init(7)

    def field(x, w, mat):
        lam = (np.arange(B) + 0.5) / B
        s = 0.4 + 0.25 * np.sin(0.6 * x[:, 0:1]) * np.cos(0.8 * x[:, 1:2]) + 0.1 * w[:, 2:3] + 0.05 * mat[:, None]
        return (s * (0.6 + 0.4 * lam[None, :])).astype(np.float32)

    losses = []
    for it in range(120):
        x, w, mat, _ = _records(8192, 100 + it, lo, hi, n_mat, B)
        cache.train(_dev(x), _dev(w), _dev(mat), _dev(field(x, w, mat)))
        losses.append(cache.loss())
    say(f"training loss first {losses[0]:.4e} last {losses[-1]:.4e}, adam steps {cache.info()['adam_steps']}")
    assert losses[-1] < 0.1 * losses[0]
    x, w, mat, _ = _records(1000, 9999, lo, hi, n_mat, B)
    y = cache.eval(_dev(x), _dev(w), _dev(mat), B).cpu().numpy()
    t = field(x, w, mat)
    rel = np.linalg.norm(y - t) / np.linalg.norm(t)
    say(f"held-out relative error {rel:.3e}")
    assert rel < 0.1


def _nave_setup(ctx, B=8, grid=(2, 2, 2)):
    import paper_1912_04000_amd as sd
    sc = scenegen.nave_scene(B)
    S = sd.Scene.from_description(sc, grid=grid)
    ctx.upload(S)
    lo, hi = sc.verts.reshape(-1, 3).min(0) - 0.01, sc.verts.reshape(-1, 3).max(0) + 0.01
    return sc, S, lo, hi


def test_training_records_match_oracle(ctx):
    import paper_1912_04000_amd as sd
    sc, S, lo, hi = _nave_setup(ctx)
    cam = scenegen.nave_camera(48, 32)
    n_mat = len(sc.mat_type)
    cache = _make_cache(ctx, SMALL, n_mat, lo, hi, sc.n_bins, max_records=4096, max_step=1024)
    cache.init(3)
    nt, seed, D = 3000, 77, 8
    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height)
    p = sd.render_params(spp=1, max_depth=D, seed=seed, mode=sd.MODE_CACHED, wave_paths=4096)
    tp = sd.train_params(train_paths=nt, step_records=1024, steps=2)
    ctx.render_cached(S, cache, c, p, tp)
    rx, rw, tg = cache.records(nt)
    P = cam.width * cam.height
    key = (seed & 0xFFFFFFFF, seed >> 32)
    pix = (oracle.philox_stream((0, 0, 2 << 24, 0), key, nt)[:, 0] % P).astype(np.int64)
    rec = oracle.training_records(sc, cam, pix, 0, max_depth=D, seed=seed)
    ok = rec["tied"] == 0
    valid = rw[:, 3] != 0
    say(f"training paths {nt}: tied {int((~ok).sum())}, reached vertex 3: gpu {valid.sum()} oracle {rec['valid'].sum()}")
    np.testing.assert_array_equal(valid[ok], rec["valid"][ok])
    v = ok & valid
    # vertex positions carry the FP32 hit distance error (1e-5 relative) of up to three bounces
    xt = 3e-5 * (1.0 + np.abs(rec["x"][v]).max())
    np.testing.assert_allclose(rx[v, :3], rec["x"][v], rtol=0, atol=xt)
    np.testing.assert_allclose(rw[v, :3], rec["wo"][v], rtol=0, atol=1e-5)
    np.testing.assert_array_equal(rx[v, 3].view(np.uint32), rec["mat"][v].astype(np.uint32))
    tgt = tg[v, :sc.n_bins].astype(np.float64)
    ref = rec["target"][v]
    scale = 1e-3 * np.maximum(ref.mean(axis=0), 1e-12)
    bad = np.abs(tgt - ref) > 1e-4 * np.maximum(np.abs(ref), scale[None, :])
    say(f"targets: {v.sum()} records, {bad.any(axis=1).sum()} outside the bar, max |target| {ref.max():.3e}")
    assert bad.sum() == 0


def test_cached_render_matches_oracle(ctx):
    """Frozen cache: vertices 1-2 as the plain path, then beta max(y, 0) at vertex 3."""
    import paper_1912_04000_amd as sd
    sc, S, lo, hi = _nave_setup(ctx)
    cam = scenegen.nave_camera(40, 24)
    n_mat, B = len(sc.mat_type), sc.n_bins
    Pm = _params(SMALL, n_mat, 5, grid_scale=1e3)
    Pm.arrays["w4"] = np.abs(Pm.arrays["w4"]).astype(np.float32).astype(np.float64)  # mostly positive outputs
    cache = _make_cache(ctx, SMALL, n_mat, lo, hi, B, max_records=1024, max_step=512)
    cache.set_params(Pm.flat())
    spp, seed = 2, 9
    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height)
    img = ctx.render_cached(S, cache, c, sd.render_params(spp=spp, max_depth=8, seed=seed, mode=sd.MODE_CACHED))
    img = img.cpu().numpy().reshape(B, -1)
    st = ctx.stats()
    pre = oracle.render(sc, cam, spp=spp, max_depth=8, seed=seed, cached=True)
    q = pre.queries
    valid = q["valid"].astype(bool)
    yq = np.zeros((valid.size, B))
    yq[valid] = mlp.predict(Pm, q["x"][valid], q["wo"][valid], q["mat"][valid], lo, hi,
                            scenegen.bin_centres(B), sc.lambda_min_nm, sc.lambda_max_nm, bf=True)
    cache_part = (q["beta"] * yq).reshape(-1, spp, B).sum(axis=1).T / spp
    prefix = pre.image.reshape(B, -1)
    ref = prefix + cache_part
    tied = pre.tied.ravel() > 0
    ok = ~tied
    tol = 1e-4 * np.abs(prefix) + 3e-2 * np.abs(cache_part) + 1e-6
    bad = (np.abs(img - ref) > tol)[:, ok]
    say(f"cached render: {valid.sum()} queries (gpu counted {st['cache_queries']}), tied px {tied.sum()}, "
        f"cache share {cache_part.sum() / ref.sum():.3f}, bad {bad.sum()}")
    assert bad.sum() == 0
    assert cache_part.sum() > 0.05 * ref.sum()


def test_cache_gain_over_untrained_and_truncated(ctx):
    """The ablation of the learned part: trained cache vs the same network untrained vs paths
    truncated after two bounces with no cache (all parameters zero), RMSE against a 1024-spp
    plain render of the same view."""
    import paper_1912_04000_amd as sd
    sc, S, lo, hi = _nave_setup(ctx)
    cam = scenegen.nave_camera(48, 32)
    n_mat, B = len(sc.mat_type), sc.n_bins
    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height)
    ref = ctx.render(S, c, sd.render_params(spp=1024, max_depth=8, seed=101)).cpu().numpy()
    kw = dict(levels_pos=8, log2_table_pos=16, nmin_pos=4.0, nmax_pos=256.0, levels_dir=6, log2_table_dir=12,
              nmin_dir=2.0, nmax_dir=32.0)

    def rmse(img):
        return float(np.sqrt(np.mean((img - ref) ** 2)))

    def render(cache, spp=64, seed=202, train=None, first=0):
        return ctx.render_cached(S, cache, c, sd.render_params(spp=spp, max_depth=8, seed=seed, mode=sd.MODE_CACHED,
                                                                wave_paths=8192, first_sample=first),
                                 train).cpu().numpy()

    trained = _make_cache(ctx, kw, n_mat, lo, hi, B, max_records=8192, max_step=2048, lr=3e-3)
    trained.init(1)
    tp = sd.train_params(train_paths=8192, step_records=2048, steps=4)
    for f in range(40):
        render(trained, spp=4, seed=300 + f, train=tp)
    untrained = _make_cache(ctx, kw, n_mat, lo, hi, B, max_records=8192, max_step=2048)
    untrained.init(1)
    zero = _make_cache(ctx, kw, n_mat, lo, hi, B, max_records=8192, max_step=2048)
    zero.set_params(np.zeros(zero.n_param, dtype=np.float32))
    r_t, r_u, r_z = rmse(render(trained)), rmse(render(untrained)), rmse(render(zero))
    say(f"gain: RMSE trained {r_t:.4e}, untrained {r_u:.4e}, truncated {r_z:.4e}; "
        f"adam steps {trained.info()['adam_steps']}")
    assert r_t < r_z and r_t < r_u
