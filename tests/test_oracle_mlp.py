"""Pins of the FP64 radiance-cache oracle (oracle/mlp.py)."""
import math

import numpy as np
import pytest

from oracle import mlp

SMALL = mlp.CacheConfig(levels_pos=3, features=2, log2_table_pos=10, nmin_pos=2, nmax_pos=40, levels_dir=2,
                        log2_table_dir=6, nmin_dir=2, nmax_dir=16, mat_dim=8, blob_bins=8, width=64)


def _rows(n, seed=0, n_mat=3):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-2, 3, size=(n, 3))
    w = rng.normal(size=(n, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    mat = rng.integers(0, n_mat, n)
    lt = rng.uniform(0, 1, n)
    t = rng.uniform(0, 2, n)
    return x, w, mat, lt, t


def test_level_resolutions_geometric():
    N = mlp.level_resolutions(16, 2048, 12)
    assert N[0] == 16 and N[-1] == 2048
    b = math.exp((math.log(2048) - math.log(16)) / 11)
    assert all(N[l] == math.floor(16 * b**l) for l in range(12))


def test_hash_matches_hand_arithmetic():
    c = np.array([[3, 7, 11], [123456, 654321, 999999], [0, 0, 0]])
    T = 1 << 19
    got = mlp.hash_index(c, T)
    for i, (x, y, z) in enumerate(c):
        h = (x * 1 % 2**32) ^ (y * 2654435761 % 2**32) ^ (z * 805459861 % 2**32)
        assert got[i] == h % T


def test_dense_levels_reproduce_linear_fields():
    """Where (N+1)^dim <= T the table is indexed densely and trilinear interpolation of vertex
    values of a linear function is exact."""
    N_list = [3, 5, 9]
    T = 1 << 12
    rng = np.random.default_rng(1)
    table = np.zeros((3, T, 2))
    coef = rng.normal(size=(3, 2, 3))
    off = rng.normal(size=(3, 2))
    for l, N in enumerate(N_list):
        g = np.stack(np.meshgrid(*[np.arange(N + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
        idx = mlp.grid_index(g, N, T)
        assert len(set(idx.tolist())) == len(idx)  # dense: no collisions
        table[l, idx] = g @ coef[l].T + off[l]
    p = rng.uniform(0, 1 - 1e-9, size=(200, 3))
    feats, _ = mlp.grid_encode(p, table, N_list, T)
    for l, N in enumerate(N_list):
        exp = (p * N) @ coef[l].T + off[l]
        np.testing.assert_allclose(feats[:, 2 * l:2 * l + 2], exp, atol=1e-12)


def test_octahedral_map():
    w = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, 0, -1.0]])
    uv = mlp.octahedral(w)
    np.testing.assert_allclose(uv, [[0.5, 0.5], [1, 0.5], [0.5, 1], [0, 0.5], [1, 1]])
    # continuous across the equator and inside the unit square everywhere
    rng = np.random.default_rng(2)
    d = rng.normal(size=(1000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    uv = mlp.octahedral(d)
    assert uv.min() >= 0 and uv.max() <= 1
    e = np.array([[0.6, 0.8, 1e-9], [0.6, 0.8, -1e-9]])
    a = mlp.octahedral(e)
    np.testing.assert_allclose(a[0], a[1], atol=1e-8)


def test_one_blob():
    b = mlp.one_blob(np.array([0.0625, 0.5, 0.9375]))
    assert b[0].argmax() == 0 and b[2].argmax() == 7 and b[0, 0] == pytest.approx(1.0)
    np.testing.assert_allclose(b[1, 3], b[1, 4])  # t = 0.5 sits between bins 3 and 4
    np.testing.assert_allclose(b[1, 3], math.exp(-0.5 * 0.5**2))


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2**-8, 1.0 + 2**-7, 1.0 + 3 * 2**-8, 3.14159265])
    r = mlp.bf16(v)
    # ties go to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    np.testing.assert_array_equal(r[:4], [1.0, 1.0, 1.0 + 2**-7, 1.0 + 2**-6])
    assert abs(r[4] - 3.14159265) < 2**-7 * 2


def _loss_fixed(params, x, w, mat, lt, t, denom, box):
    inp, _ = mlp.encode(params, x, w, mat, box[0], box[1], lt)
    y, _ = mlp.forward(params, inp, bf=False)
    return np.mean((y - t) ** 2 / denom)


def test_backward_matches_finite_differences():
    params = mlp.CacheParams(SMALL, 3).init(5)
    params.arrays["pos"] *= 1e3  # features large enough to matter
    params.arrays["dir"] *= 1e3
    x, w, mat, lt, t = _rows(24, 3)
    box = ([-2, -2, -2], [3, 3, 3])
    inp, taps = mlp.encode(params, x, w, mat, box[0], box[1], lt)
    y, cache = mlp.forward(params, inp, bf=False)
    g = mlp.backward(params, taps, cache, y, t, mat, bf=False)
    denom = y**2 + 0.01
    rng = np.random.default_rng(7)
    checked = 0
    for k in ["pos", "dir", "mat", "W0", "W1", "W2", "W3", "w4"]:
        gk = g[k].ravel()
        # the loss is piecewise quadratic in each parameter, so central differences are exact
        # up to rounding; test the entries whose gradient dwarfs the forward pass's rounding
        cand = np.argsort(-np.abs(gk))[:12]
        for j in rng.choice(cand, 6, replace=False):
            orig = params.arrays[k].ravel()[j]
            h = 1e-6 * max(1.0, abs(orig))
            flat = params.arrays[k].reshape(-1)
            flat[j] = orig + h
            lp = _loss_fixed(params, x, w, mat, lt, t, denom, box)
            flat[j] = orig - h
            lm = _loss_fixed(params, x, w, mat, lt, t, denom, box)
            flat[j] = orig
            fd = (lp - lm) / (2 * h)
            assert fd == pytest.approx(gk[j], rel=1e-6, abs=1e-12), (k, j)
            checked += 1
    assert checked >= 40


def test_first_adam_step_closed_form():
    params = mlp.CacheParams(SMALL, 2).init(1)
    before = params.flat().copy()
    rng = np.random.default_rng(0)
    g = {k: rng.normal(size=v.shape) for k, v in params.arrays.items()}
    opt = mlp.Adam(lr=1e-3)
    opt.step(params, g)
    gf = np.concatenate([g[k].ravel() for k, _ in params.shapes])
    np.testing.assert_allclose(params.flat() - before, -1e-3 * gf / (np.abs(gf) + 1e-8), rtol=1e-9)


def test_bf16_forward_close_to_fp64():
    params = mlp.CacheParams(SMALL, 3).init(2)
    x, w, mat, lt, t = _rows(64, 4)
    inp, _ = mlp.encode(params, x, w, mat, [-2] * 3, [3] * 3, lt)
    y64, _ = mlp.forward(params, inp, bf=False)
    y16, _ = mlp.forward(params, inp, bf=True)
    assert np.abs(y16 - y64).max() <= 0.05 * np.abs(y64).max()
