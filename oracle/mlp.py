"""FP64 reference of the learned spectral radiance cache -- TEST INFRASTRUCTURE ONLY.

The cache replaces the photon maps' role of supplying indirect radiance (section 4 of the paper
computes global illumination from photon maps; here paths end after two bounces in a learned
estimate instead). It predicts, for a surface point x, the direction toward the previous vertex
w, the material and a wavelength bin, the outgoing spectral radiance L(x, w, lambda).

Network (the renderer implements the same):
  input (64) = [position hash grid (L_p levels x F), octahedral direction hash grid (L_d x F),
                material embedding (8), wavelength one-blob (8)]
  h1..h4 = ReLU(W_l h_{l-1}) with 64 x 64 matrices and no biases, y = w4 . h4 (one output)
Multiresolution hash encoding (Mueller, Evans, Schied, Keller 2022): level l has resolution
N_l = floor(N_min b^l), b = exp((ln N_max - ln N_min)/(L - 1)); its vertices are indexed densely
when (N_l + 1)^dim <= T, else by the spatial hash (x * 1 xor y * 2654435761 xor z * 805459861)
mod T in 32-bit unsigned arithmetic; features are interpolated (tri/bi-linearly).
Loss: relative L2, (y - t)^2 / (sg(y)^2 + 0.01), averaged over rows. Optimizer: Adam
(Kingma & Ba 2015) with bias correction.

With bf16=True the forward and backward passes round to bfloat16 (round to nearest even) where
the renderer feeds its matrix cores: layer inputs, weights and back-propagated deltas.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

PRIMES = (1, 2654435761, 805459861)


@dataclass
class CacheConfig:
    levels_pos: int = 12
    features: int = 2
    log2_table_pos: int = 19
    nmin_pos: float = 16.0
    nmax_pos: float = 2048.0
    levels_dir: int = 12
    log2_table_dir: int = 14
    nmin_dir: float = 4.0
    nmax_dir: float = 256.0
    mat_dim: int = 8
    blob_bins: int = 8
    width: int = 64

    @property
    def n_in(self):
        return (self.levels_pos + self.levels_dir) * self.features + self.mat_dim + self.blob_bins


def bf16(a):
    """Round float64/float32 values to bfloat16 (nearest even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def level_resolutions(nmin, nmax, L):
    b = math.exp((math.log(nmax) - math.log(nmin)) / (L - 1)) if L > 1 else 1.0
    return [int(math.floor(nmin * b**l)) for l in range(L)]


def hash_index(corner, T):
    """Spatial hash of integer vertex coordinates (uint32 products, xor, mod T)."""
    h = np.zeros(corner.shape[0], dtype=np.uint64)
    for a in range(corner.shape[1]):
        h ^= (corner[:, a].astype(np.uint64) * np.uint64(PRIMES[a])) & np.uint64(0xFFFFFFFF)
    return (h % np.uint64(T)).astype(np.int64)


def grid_index(corner, N, T):
    dim = corner.shape[1]
    if (N + 1) ** dim <= T:
        idx = np.zeros(corner.shape[0], dtype=np.int64)
        stride = 1
        for a in range(dim):
            idx += corner[:, a].astype(np.int64) * stride
            stride *= N + 1
        return idx
    return hash_index(corner, T)


def octahedral(w):
    """Unit directions [n][3] -> [0,1]^2 (octahedral map, lower hemisphere folded outward)."""
    w = np.asarray(w, dtype=np.float64)
    s = np.abs(w).sum(axis=1)
    px, py = w[:, 0] / s, w[:, 1] / s
    neg = w[:, 2] < 0
    fx = (1 - np.abs(py)) * np.copysign(1.0, px)
    fy = (1 - np.abs(px)) * np.copysign(1.0, py)
    px, py = np.where(neg, fx, px), np.where(neg, fy, py)
    return np.column_stack([(px + 1) * 0.5, (py + 1) * 0.5])


def one_blob(t, k=8):
    """One-blob encoding of t in [0,1]: Gaussians of width 1/k at the k bin centres."""
    c = (np.arange(k) + 0.5) / k
    return np.exp(-((np.asarray(t, dtype=np.float64)[:, None] - c[None, :]) ** 2) / (2 * (1.0 / k) ** 2))


def grid_encode(p, table, N_list, T):
    """Interpolated features of points p in [0,1]^dim from the level tables [L][T][F].
    Returns features [n][L*F] and, per level, the (index, weight) lists for the backward pass."""
    n, dim = p.shape
    L, _, F = table.shape
    p = np.clip(p, 0.0, 1.0 - 2.0**-20)
    feats = np.zeros((n, L * F))
    taps = []
    for l, N in enumerate(N_list):
        x = p * N
        i0 = np.floor(x).astype(np.int64)
        f = x - i0
        lvl = []
        for c in range(2**dim):
            off = np.array([(c >> a) & 1 for a in range(dim)])
            w = np.prod(np.where(off[None, :] == 1, f, 1 - f), axis=1)
            idx = grid_index(i0 + off[None, :], N, T)
            feats[:, l * F:(l + 1) * F] += w[:, None] * table[l, idx, :]
            lvl.append((idx, w))
        taps.append(lvl)
    return feats, taps


class CacheParams:
    """All trainable parameters (FP64 masters). Flat layout (shared with the renderer's ABI):
    pos grid [Lp][Tp][F], dir grid [Ld][Td][F], material embedding [n_mat][8],
    W0..W3 [64 out][64 in], w4 [64]."""

    def __init__(self, cfg: CacheConfig, n_mat: int):
        self.cfg, self.n_mat = cfg, n_mat
        c = cfg
        self.shapes = [("pos", (c.levels_pos, 1 << c.log2_table_pos, c.features)),
                       ("dir", (c.levels_dir, 1 << c.log2_table_dir, c.features)),
                       ("mat", (n_mat, c.mat_dim))] + \
                      [(f"W{i}", (c.width, c.width if i else c.n_in)) for i in range(4)] + [("w4", (c.width,))]
        self.arrays = {k: np.zeros(s) for k, s in self.shapes}

    def size(self):
        return sum(int(np.prod(s)) for _, s in self.shapes)

    def flat(self):
        return np.concatenate([self.arrays[k].ravel() for k, _ in self.shapes])

    def set_flat(self, v):
        v = np.asarray(v, dtype=np.float64)
        o = 0
        for k, s in self.shapes:
            n = int(np.prod(s))
            self.arrays[k] = v[o:o + n].reshape(s).copy()
            o += n
        assert o == v.size

    def init(self, seed=0):
        rng = np.random.default_rng(seed)
        a = self.arrays
        a["pos"] = rng.uniform(-1e-4, 1e-4, a["pos"].shape)
        a["dir"] = rng.uniform(-1e-4, 1e-4, a["dir"].shape)
        a["mat"] = rng.uniform(-1.0, 1.0, a["mat"].shape)
        for i in range(4):
            fi, fo = a[f"W{i}"].shape[1], a[f"W{i}"].shape[0]
            lim = math.sqrt(6.0 / (fi + fo))
            a[f"W{i}"] = rng.uniform(-lim, lim, a[f"W{i}"].shape)
        a["w4"] = rng.uniform(-math.sqrt(6.0 / 65), math.sqrt(6.0 / 65), a["w4"].shape)
        return self


def encode(params: CacheParams, x, w, mat, box_lo, box_hi, lam_t):
    """Network inputs for rows (x [n][3], w [n][3], mat [n], lam_t [n] in [0,1])."""
    c = params.cfg
    a = params.arrays
    p = (np.asarray(x, np.float64) - np.asarray(box_lo, np.float64)) / (np.asarray(box_hi, np.float64) -
                                                                          np.asarray(box_lo, np.float64))
    fp, tp = grid_encode(p, a["pos"], level_resolutions(c.nmin_pos, c.nmax_pos, c.levels_pos), 1 << c.log2_table_pos)
    fd, td = grid_encode(octahedral(w), a["dir"], level_resolutions(c.nmin_dir, c.nmax_dir, c.levels_dir),
                         1 << c.log2_table_dir)
    fm = a["mat"][np.asarray(mat, np.int64)]
    fb = one_blob(lam_t, c.blob_bins)
    return np.concatenate([fp, fd, fm, fb], axis=1), (tp, td)


def forward(params: CacheParams, inp, bf=True):
    """Returns y [n] and the cache of layer inputs / pre-activations."""
    r = bf16 if bf else (lambda v: np.asarray(v, np.float64))
    a = params.arrays
    hs = [r(inp)]
    pre = []
    h = hs[0]
    for i in range(4):
        z = h @ r(a[f"W{i}"]).T
        pre.append(z)
        h = r(np.maximum(z, 0.0))
        hs.append(h)
    y = h @ r(a["w4"])
    return y, (hs, pre)


def rel_l2(y, t):
    return np.mean((y - t) ** 2 / (y**2 + 0.01))


def backward(params: CacheParams, inp_taps, cache, y, t, mat, bf=True):
    """Gradients of the mean relative-L2 loss (the denominator treated as a constant) with
    respect to every parameter, as a dict of arrays shaped like the parameters."""
    r = bf16 if bf else (lambda v: np.asarray(v, np.float64))
    a = params.arrays
    c = params.cfg
    hs, pre = cache
    n = y.shape[0]
    dy = 2.0 * (y - t) / (y**2 + 0.01) / n
    g = {k: np.zeros_like(v) for k, v in a.items()}
    g["w4"] = dy @ hs[4]
    delta = np.outer(dy, r(a["w4"])) * (pre[3] > 0)
    for i in (3, 2, 1, 0):
        g[f"W{i}"] = r(delta).T @ hs[i]
        dh = r(delta) @ r(a[f"W{i}"])
        if i > 0:
            delta = dh * (pre[i - 1] > 0)
    d_in = dh
    Lp, F, Ld = c.levels_pos, c.features, c.levels_dir
    tp, td = inp_taps
    for l in range(Lp):
        for idx, w in tp[l]:
            np.add.at(g["pos"][l], idx, w[:, None] * d_in[:, l * F:(l + 1) * F])
    o = Lp * F
    for l in range(Ld):
        for idx, w in td[l]:
            np.add.at(g["dir"][l], idx, w[:, None] * d_in[:, o + l * F:o + (l + 1) * F])
    o += Ld * F
    np.add.at(g["mat"], np.asarray(mat, np.int64), d_in[:, o:o + c.mat_dim])
    return g


class Adam:
    def __init__(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = None
        self.v = None

    def step(self, params: CacheParams, grads: dict):
        if self.m is None:
            self.m = {k: np.zeros_like(v) for k, v in params.arrays.items()}
            self.v = {k: np.zeros_like(v) for k, v in params.arrays.items()}
        self.t += 1
        for k in params.arrays:
            g = grads[k]
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * g
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * g * g
            mh = self.m[k] / (1 - self.b1**self.t)
            vh = self.v[k] / (1 - self.b2**self.t)
            params.arrays[k] = params.arrays[k] - self.lr * mh / (np.sqrt(vh) + self.eps)


def predict(params: CacheParams, x, w, mat, box_lo, box_hi, lambdas, lmin, lmax, bf=True):
    """Cache output for every (vertex, bin): [n][B], clamped at 0 (radiance)."""
    x = np.asarray(x, np.float64)
    n, B = x.shape[0], len(lambdas)
    xs = np.repeat(x, B, axis=0)
    ws = np.repeat(np.asarray(w, np.float64), B, axis=0)
    ms = np.repeat(np.asarray(mat), B)
    lt = np.tile((np.asarray(lambdas, np.float64) - lmin) / (lmax - lmin), n)
    inp, _ = encode(params, xs, ws, ms, box_lo, box_hi, lt)
    y, _ = forward(params, inp, bf)
    return np.maximum(y, 0.0).reshape(n, B)
