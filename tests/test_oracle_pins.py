"""Pins of the CPU oracle against closed forms, published vectors, brute force and invariants.

Each check uses a computation that is independent of the oracle's own formula (a special
case, a different algebraic route, a series summed term by term, a geometric construction),
so that a dropped term, a wrong sign or a swapped operand inside the oracle fails here.
"""
import math
import os

import numpy as np
import pytest

import oracle
import scenegen
from oracle.philox_generic import philox4, uniform24

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------------------------
# Philox4x32-10 (counter-based RNG of the path decisions)
# ---------------------------------------------------------------------------------------------

def _kat():
    rows = []
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        lhs, rhs = line.split("->")
        a = [int(x, 16) for x in lhs.split()]
        b = [int(x, 16) for x in rhs.split()]
        rows.append((a[:4], a[4:], b))
    return rows


def test_philox_generic_64_matches_numpy():
    # NumPy's Philox4x64-10 increments the 256-bit counter before producing each block.
    key = (0x0123456789ABCDEF, 0x0FEDCBA987654321)
    ctr = (5, 7, 11, 13)
    bg = np.random.Philox(counter=np.array(ctr, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    raw = [int(x) for x in bg.random_raw(8)]
    assert list(philox4((6, 7, 11, 13), key, 64)) == raw[:4]
    assert list(philox4((7, 7, 11, 13), key, 64)) == raw[4:]


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox4x32_kat(ctr, key, out):
    assert list(philox4(ctr, key, 32)) == out
    assert [int(x) for x in oracle.philox4x32_10(ctr, key)] == out


def test_philox_cpp_matches_generic_stream():
    key = (0xDEADBEEF, 0x12345678)
    base = (1000, 3, (2 << 24) | 5, 9)
    got = oracle.philox_stream(base, key, 512)
    rng = np.random.default_rng(0)
    for i in rng.choice(512, 64, replace=False):
        exp = philox4((base[0] + int(i), base[1], base[2], base[3]), key, 32)
        assert tuple(int(x) for x in got[i]) == exp


def test_philox_uniformity_chi2():
    out = oracle.philox_stream((0, 0, 0, 0), (1, 0), 1 << 16).ravel()
    u = (out >> 8).astype(np.float64) * 2.0**-24
    assert u.min() >= 0.0 and u.max() < 1.0
    h, _ = np.histogram(u, bins=64, range=(0, 1))
    e = u.size / 64
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 < 120  # 63 dof: p ~ 1e-5
    assert uniform24(0xFFFFFFFF) == (2**24 - 1) / 2**24


# ---------------------------------------------------------------------------------------------
# Fresnel at the interface air -> n + ik (eq. 1)
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("n,k,anchor", [(1.52, 0.0, 0.042579995), (1.6, 0.01, 0.053268443),
                                        (1.6, 0.03, 0.053380467), (1.6, 0.05, 0.053604436)])
def test_fresnel_normal_incidence_closed_form(n, k, anchor):
    closed = ((n - 1) ** 2 + k**2) / ((n + 1) ** 2 + k**2)
    assert oracle.fresnel(n, k, 1.0) == pytest.approx(closed, rel=1e-12)
    assert closed == pytest.approx(anchor, abs=1e-9)


def _real_fresnel_snell(n, cos_i):
    sin_t = math.sqrt(1 - cos_i**2) / n
    cos_t = math.sqrt(1 - sin_t**2)
    rs = (cos_i - n * cos_t) / (cos_i + n * cos_t)
    rp = (n * cos_i - cos_t) / (n * cos_i + cos_t)
    ts = 2 * cos_i / (cos_i + n * cos_t)
    tp = 2 * cos_i / (n * cos_i + cos_t)
    R = 0.5 * (rs * rs + rp * rp)
    T = n * cos_t / cos_i * 0.5 * (ts * ts + tp * tp)
    return R, T


@pytest.mark.parametrize("deg", [0.0, 10.0, 30.0, 45.0, 60.0, 75.0, 85.0, 89.0])
@pytest.mark.parametrize("n", [1.33, 1.52, 1.6, 2.4])
def test_fresnel_lossless_matches_snell_and_energy(deg, n):
    c = math.cos(math.radians(deg))
    R, T = _real_fresnel_snell(n, c)
    assert R + T == pytest.approx(1.0, abs=1e-12)
    assert oracle.fresnel(n, 0.0, c) == pytest.approx(R, rel=1e-11, abs=1e-14)


def test_fresnel_anchor_values():
    assert oracle.fresnel(1.52, 0.0, math.cos(math.radians(45))) == pytest.approx(0.053045232, abs=1e-9)
    assert oracle.fresnel(1.52, 0.0, math.cos(math.radians(80))) == pytest.approx(0.390949863, abs=1e-9)
    assert oracle.fresnel(1.6, 0.03, math.cos(math.radians(45))) == pytest.approx(0.064576281, abs=1e-9)


@pytest.mark.parametrize("n,k", [(1.6, 0.01), (1.6, 0.05), (1.52, 1e-6), (0.2, 3.0), (2.5, 0.7)])
@pytest.mark.parametrize("deg", [0.0, 20.0, 50.0, 70.0, 88.0])
def test_fresnel_complex_via_complex_snell(n, k, deg):
    # Independent route: complex Snell's law cos_t = sqrt(1 - sin^2/eta^2) with NumPy complex
    # arithmetic, r_s = (cos - eta cos_t)/(cos + eta cos_t), r_p = (eta cos - cos_t)/(eta cos + cos_t).
    eta = complex(n, k)
    ci = math.cos(math.radians(deg))
    si2 = 1 - ci * ci
    ct = np.sqrt(1 - si2 / eta**2)
    if ct.imag < 0 or (ct.imag == 0 and ct.real < 0):
        ct = -ct
    rs = (ci - eta * ct) / (ci + eta * ct)
    rp = (eta * ci - ct) / (eta * ci + ct)
    R = 0.5 * (abs(rs) ** 2 + abs(rp) ** 2)
    assert oracle.fresnel(n, k, ci) == pytest.approx(R, rel=1e-10)


def test_fresnel_grazing_limit_and_monotone_tail():
    vals = [oracle.fresnel(1.6, 0.03, c) for c in (1e-3, 1e-5, 1e-8)]
    assert vals[-1] > 0.9999 and vals[0] < vals[1] < vals[2]
    assert oracle.fresnel(1.6, 0.03, 0.0) == pytest.approx(1.0, abs=1e-12)


# ---------------------------------------------------------------------------------------------
# Thin glass slab with Beer-Lambert absorption (section 3: spectral absorption of glass)
# ---------------------------------------------------------------------------------------------

def _slab_series(R1, tau, terms=400):
    # multiple reflections summed bounce by bounce
    R = R1
    T = 0.0
    for m in range(terms):
        T += (1 - R1) ** 2 * tau * (R1 * tau) ** (2 * m)
        R += (1 - R1) ** 2 * R1 * tau**2 * (R1 * tau) ** (2 * m)
    return R, T


def test_slab_lossless_closed_form():
    R, T = oracle.slab(1.52, 0.0, 500.0, 0.005, 1.0)
    R1 = ((1.52 - 1) / (1.52 + 1)) ** 2
    assert R == pytest.approx(2 * R1 / (1 + R1), rel=1e-12)
    assert R + T == pytest.approx(1.0, abs=1e-14)
    assert (R, T) == (pytest.approx(0.081681972, abs=1e-9), pytest.approx(0.918318028, abs=1e-9))


@pytest.mark.parametrize("deg", [0.0, 30.0, 60.0, 80.0])
@pytest.mark.parametrize("k", [1e-7, 1e-6, 2e-5])
def test_slab_matches_bounce_series_and_snell_path(deg, k):
    n, lam, d = 1.52, 555.0, 0.005
    ci = math.cos(math.radians(deg))
    sin_t = math.sqrt(1 - ci * ci) / n
    cos_t = math.sqrt(1 - sin_t * sin_t)
    tau = math.exp(-4 * math.pi * k / (lam * 1e-9) * d / cos_t)
    R1 = oracle.fresnel(n, k, ci)
    Rs, Ts = _slab_series(R1, tau)
    R, T = oracle.slab(n, k, lam, d, ci)
    assert R == pytest.approx(Rs, rel=1e-12)
    assert T == pytest.approx(Ts, rel=1e-12)
    assert R + T <= 1.0 + 1e-15


def test_beer_lambert_c1_anchors():
    lam = scenegen.bin_centres(8)
    sc = scenegen.nave_scene(8)
    k = sc.k_tab[2].astype(np.float64)
    tau = np.exp(-4 * np.pi * k * 0.005 / (lam * 1e-9))
    np.testing.assert_allclose(tau, [0.976051, 0.963568, 0.953673, 0.945636, 0.938979, 0.933376, 0.928594,
                                     0.924465], atol=1e-6)
    T = np.array([oracle.slab(1.52, float(k[j]), lam[j], 0.005, 1.0)[1] for j in range(8)])
    assert T[0] == pytest.approx(0.896248, abs=1e-6) and T[-1] == pytest.approx(0.848729, abs=1e-6)
    # as the interface reflection vanishes (n -> 1) the slab transmits exactly exp(-alpha d)
    T1 = np.array([oracle.slab(1.0, float(k[j]), lam[j], 0.005, 1.0)[1] for j in range(8)])
    np.testing.assert_allclose(T1, tau, rtol=1e-12)


# ---------------------------------------------------------------------------------------------
# Sun spectrum (scenegen input): 5778 K blackbody normalised at 555 nm
# ---------------------------------------------------------------------------------------------

def test_sun_planck_wien_and_anchors():
    from scipy.optimize import minimize_scalar
    r = minimize_scalar(lambda l: -scenegen.planck(l), bounds=(300, 800), method="bounded",
                        options=dict(xatol=1e-6))
    assert r.x == pytest.approx(2.897771955e-3 / 5778 * 1e9, abs=1e-3)  # Wien's law b/T
    E = scenegen.sun_irradiance(8)
    assert E[0] == pytest.approx(0.908916, abs=1e-6) and E[-1] == pytest.approx(0.723323, abs=1e-6)
    assert E[3] == pytest.approx(1.0, abs=1e-7)  # the bin centred at 555 nm


# ---------------------------------------------------------------------------------------------
# Closest hit and shadow visibility
# ---------------------------------------------------------------------------------------------

def test_plane_hits_closed_form():
    sc = scenegen.plane_scene(size=100.0, z=2.5)
    rng = np.random.default_rng(1)
    o = np.column_stack([rng.uniform(-5, 5, 200), rng.uniform(-5, 5, 200), rng.uniform(4, 9, 200)])
    d = np.column_stack([rng.normal(0, 0.3, 200), rng.normal(0, 0.3, 200), -np.ones(200)])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o32, d32 = o.astype(np.float32), d.astype(np.float32)
    t, ids, u, v, tie = oracle.intersect(sc, o32, d32)
    exp = (2.5 - o32[:, 2].astype(np.float64)) / d32[:, 2].astype(np.float64)
    assert np.all(ids >= 0)
    np.testing.assert_allclose(t, exp, rtol=1e-12)
    # rays pointing away never hit
    t2, ids2, *_ = oracle.intersect(sc, o32, -d32)
    assert np.all(ids2 == -1) and np.all(np.isinf(t2))


def _icosphere(r, levels=2):
    phi = (1 + 5**0.5) / 2
    V = [(-1, phi, 0), (1, phi, 0), (-1, -phi, 0), (1, -phi, 0), (0, -1, phi), (0, 1, phi), (0, -1, -phi),
         (0, 1, -phi), (phi, 0, -1), (phi, 0, 1), (-phi, 0, -1), (-phi, 0, 1)]
    V = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in V]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6),
         (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
         (8, 6, 7), (9, 8, 1)]
    for _ in range(levels):
        cache = {}
        nf = []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = nf
    V = np.array(V) * r
    return np.array([[V[a], V[b], V[c]] for a, b, c in F])


def test_icosphere_hit_bounds():
    r = 2.0
    tris = _icosphere(r, 2)
    # inscribed radius: smallest distance from the centre to a face plane
    nrm = np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    r_in = np.abs(np.einsum("ij,ij->i", nrm, tris[:, 0])).min()
    sc = scenegen.random_soup(4)
    sc.verts = tris.astype(np.float32)
    sc.mat = np.zeros(len(tris), dtype=np.uint16)
    rng = np.random.default_rng(2)
    o = rng.normal(size=(300, 3))
    o = o / np.linalg.norm(o, axis=1, keepdims=True) * 6.0
    aim = rng.normal(scale=0.5, size=(300, 3))
    d = aim - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o32, d32 = o.astype(np.float32), d.astype(np.float32)
    t, ids, u, v, tie = oracle.intersect(sc, o32, d32)
    oo, dd = o32.astype(np.float64), d32.astype(np.float64)
    b = np.einsum("ij,ij->i", oo, dd)
    cc = np.einsum("ij,ij->i", oo, oo)

    def tsph(R):
        disc = b * b - (cc - R * R)
        return np.where(disc >= 0, -b - np.sqrt(np.maximum(disc, 0)), np.inf)
    t_out, t_in = tsph(r), tsph(r_in)
    inner = np.isfinite(t_in)
    assert np.all(ids[inner] >= 0)
    hit = ids >= 0
    assert np.all(t[hit] >= t_out[hit] - 1e-9) and np.all(t[hit] <= t_in[hit] + 1e-9)
    # the normal of the face hit is within the facet angle of the radial direction
    p = oo[hit] + t[hit, None] * dd[hit]
    cosang = np.abs(np.einsum("ij,ij->i", nrm[ids[hit]], p / np.linalg.norm(p, axis=1, keepdims=True)))
    assert cosang.min() > r_in / r - 1e-9


def test_bvh_equals_brute_force():
    sc = scenegen.random_soup(3000, seed=4, extent=10.0, size=0.6)
    o, d = scenegen.random_rays(4000, seed=9)
    a = oracle.intersect(sc, o, d, force_bvh=0)
    b = oracle.intersect(sc, o, d, force_bvh=1)
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[4], b[4])
    assert (a[1] >= 0).mean() > 0.3


def test_skip_triangle_and_tie_break():
    # two coincident triangles: equal t -> the smaller id wins; skipping it exposes the other
    tri = np.array([[[0, 0, 0], [4, 0, 0], [0, 4, 0]]], dtype=np.float32)
    sc = scenegen.random_soup(2)
    sc.verts = np.concatenate([tri, tri])
    sc.mat = np.zeros(2, dtype=np.uint16)
    o = np.array([[1, 1, 3]], dtype=np.float32)
    d = np.array([[0, 0, -1]], dtype=np.float32)
    t, ids, u, v, tie = oracle.intersect(sc, o, d)
    assert ids[0] == 0 and t[0] == 3.0 and tie[0]
    t, ids, u, v, tie = oracle.intersect(sc, o, d, skip=np.array([0], dtype=np.int32))
    assert ids[0] == 1
    # barycentrics: p = (1-u-v) v0 + u v1 + v v2
    t, ids, u, v, tie = oracle.intersect(sc, o, d, skip=np.array([1], dtype=np.int32))
    assert (u[0], v[0]) == (0.25, 0.25)


def test_shadow_visibility_glass_product_and_block():
    sc = scenegen.plane_scene(n_bins=8, window=(5.0, 3.0), glass_k=2e-6)
    lam = scenegen.bin_centres(8)
    o = np.array([[0.3, 0.2, 1e-3], [20.0, 20.0, 1e-3]], dtype=np.float32)
    d = np.array([[0, 0, 1], [0, 0, 1]], dtype=np.float32)
    vis, tie = oracle.shadow(sc, o, d)
    T = [oracle.slab(float(np.float32(1.52)), float(np.float32(2e-6)), lam[j], float(np.float32(0.005)), 1.0)[1]
         for j in range(8)]
    np.testing.assert_allclose(vis[0], T, rtol=1e-12)
    np.testing.assert_allclose(vis[1], 1.0)
    # an opaque plane between point and sun blocks everything
    o2 = np.array([[0.3, 0.2, -1.0]], dtype=np.float32)
    vis2, _ = oracle.shadow(sc, o2, d[:1])
    assert np.all(vis2 == 0)


# ---------------------------------------------------------------------------------------------
# Whole-estimator pins
# ---------------------------------------------------------------------------------------------

def test_nee_single_plane_closed_form():
    """Depth 1 over one opaque plane, camera looking straight down through a very narrow
    field: every pixel is exactly the direct term (eq. 3) with F at normal incidence."""
    B = 8
    n, k, rho = 1.6, 0.03, 0.7
    sdir = np.array([0.3, -0.2, 0.9])
    sc = scenegen.plane_scene(n_bins=B, n=n, k=k, rho=rho, sun_dir=sdir)
    cam = scenegen.Camera(eye=(0.1, 0.2, 10.0), target=(0.1, 0.2, 0.0), up=(0, 1, 0), vfov_deg=1e-4, width=4,
                          height=4)
    res = oracle.render(sc, cam, spp=2, max_depth=1)
    n32, k32, rho32 = (float(np.float32(x)) for x in (n, k, rho))
    F0 = ((n32 - 1) ** 2 + k32**2) / ((n32 + 1) ** 2 + k32**2)
    ws = sc.sun_dir.astype(np.float64)
    ws /= np.linalg.norm(ws)
    exp = (1 - F0) * rho32 / math.pi * sc.sun_E.astype(np.float64) * ws[2]
    np.testing.assert_allclose(res.image, np.broadcast_to(exp[:, None, None], res.image.shape), rtol=1e-9)


def test_nee_through_glass_window_closed_form():
    B = 8
    sc = scenegen.plane_scene(n_bins=B, n=1.6, k=0.02, rho=0.8, sun_dir=(0, 0, 1), window=(6.0, 4.0),
                              glass_k=3e-6)
    cam = scenegen.Camera(eye=(0.0, 0.3, 3.0), target=(0.0, 0.3, 0.0), up=(0, 1, 0), vfov_deg=1e-4, width=2,
                          height=2)
    res = oracle.render(sc, cam, spp=1, max_depth=1)
    lam = scenegen.bin_centres(B)
    f = lambda x: float(np.float32(x))
    n, k, rho, gk, gd = f(1.6), f(0.02), f(0.8), f(3e-6), f(0.005)
    F0 = ((n - 1) ** 2 + k**2) / ((n + 1) ** 2 + k**2)
    G1 = ((f(1.52) - 1) ** 2 + gk**2) / ((f(1.52) + 1) ** 2 + gk**2)
    tau = np.exp(-4 * np.pi * gk / (lam * 1e-9) * gd)
    T = (1 - G1) ** 2 * tau / (1 - G1**2 * tau**2)
    exp = (1 - F0) * rho / math.pi * sc.sun_E.astype(np.float64) * T
    np.testing.assert_allclose(res.image[:, 0, 0], exp, rtol=1e-9)


def test_white_furnace():
    sc = scenegen.furnace_scene(n_bins=4)
    cam = scenegen.Camera(eye=(0.0, -14.0, 6.0), target=(0.0, 0.0, 0.5), up=(0, 0, 1), vfov_deg=70, width=24,
                          height=24)
    res = oracle.render(sc, cam, spp=4, max_depth=64)
    np.testing.assert_allclose(res.image, 1.0, atol=1e-12)
    assert res.stats["vertices"] > 0.5 * res.stats["paths"]  # most camera paths hit geometry


def test_single_bounce_expectation_under_uniform_env():
    """Opaque plane under env = 1, no sun, depth 2: E[L] = F(theta_o) + (1 - F) rho per bin
    (the Fresnel-split Lambertian's albedo), which pins the lobe-selection weights."""
    B = 2
    sc = scenegen.plane_scene(n_bins=B, n=1.6, k=0.05, rho=0.6, sun_dir=(0, 0, 1), env=1.0)
    sc.sun_E[:] = 0
    c = math.cos(math.radians(60))
    cam = scenegen.Camera(eye=(0.0, -10 * math.tan(math.radians(60)), 10.0), target=(0.0, 0.0, 0.0), up=(0, 0, 1),
                          vfov_deg=1e-4, width=1, height=1)
    res = oracle.render(sc, cam, spp=20000, max_depth=2)
    F = oracle.fresnel(float(np.float32(1.6)), float(np.float32(0.05)), c)
    exp = F + (1 - F) * float(np.float32(0.6))
    # per-sample weight is F/P or (1-F)rho/(1-P), P = F/(F+(1-F)rho): both equal F + (1-F)rho
    np.testing.assert_allclose(res.image[:, 0, 0], exp, rtol=1e-6)


def test_nave_geometry_counts():
    sc = scenegen.nave_scene(8)
    assert sc.n_tri == 1750
    assert np.bincount(sc.mat).tolist() == [400, 948 + 400, 2]  # floor, walls + pillars, glass
    lo, hi = sc.verts.reshape(-1, 3).min(0), sc.verts.reshape(-1, 3).max(0)
    np.testing.assert_allclose(lo, [0, 0, 0])
    np.testing.assert_allclose(hi, [20, 10, 8])
