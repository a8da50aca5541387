"""Plain CPU oracle of the spectral path tracer -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package. The renderer (``paper_1912_04000_amd``) never imports it and shares no
code with it; the two meet only on the seeded inputs of ``scenegen``.

Contents:
  * ``oracle.cpp`` -- FP64 C++17: Philox4x32-10, unpolarised complex Fresnel (section 3,
    eq. 1 for n + ik), thin-slab Beer-Lambert glass (absorbing by k, or by a spectral
    transmittance map read at the hit's texture coordinates, section 3), Moeller-Trumbore closest hit / shadow
    visibility (brute force or a median-split BVH), and the path estimator whose direct term
    is eq. 3 (section 4), with tie flags for paths that FP32 rounding could flip.
  * ``philox_generic.py`` -- a word-size-generic Philox used to pin the C++ generator.
  * ``mlp.py`` -- FP64 reference of the learned radiance cache (hash-grid encoding, MLP,
    relative-L2 loss, backward pass, Adam).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C++ oracle with g++ (in-tree)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _Scene(C.Structure):
    _fields_ = [("verts", C.c_void_p), ("n_tri", C.c_int64), ("mat", C.c_void_p), ("n_mat", C.c_int32),
                ("mat_type", C.c_void_p), ("thickness_m", C.c_void_p), ("n_tab", C.c_void_p),
                ("k_tab", C.c_void_p), ("rho_tab", C.c_void_p), ("n_bins", C.c_int32),
                ("lambda_min_nm", C.c_double), ("lambda_max_nm", C.c_double), ("sun_dir", C.c_void_p),
                ("sun_E", C.c_void_p), ("env", C.c_void_p), ("uv", C.c_void_p), ("n_tex", C.c_int32),
                ("tex_dims", C.c_void_p), ("tex_offset", C.c_void_p), ("texels", C.c_void_p),
                ("mat_tex", C.c_void_p)]


class _Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("target", C.c_double * 3), ("up", C.c_double * 3),
                ("vfov_deg", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("spp", C.c_int32), ("max_depth", C.c_int32), ("seed", C.c_uint64), ("view", C.c_uint32),
                ("threads", C.c_int32), ("force_bvh", C.c_int32), ("tie_t_rel", C.c_double),
                ("tie_edge_abs", C.c_double), ("tie_edge_rel_t", C.c_double), ("tie_lobe", C.c_double),
                ("tie_cos_sun", C.c_double), ("cached", C.c_int32), ("first_sample", C.c_int32),
                ("purpose", C.c_uint32), ("record_depth", C.c_int32), ("sample_per_entry", C.c_int32),
                ("ph_pos", C.c_void_p), ("ph_dir", C.c_void_p), ("ph_flux", C.c_void_p), ("n_photons", C.c_int64),
                ("ph_radius", C.c_double), ("tie_radius", C.c_double), ("ph_unc", C.c_void_p),
                ("gl_pos", C.c_void_p), ("gl_dir", C.c_void_p), ("gl_flux", C.c_void_p), ("n_global", C.c_int64),
                ("gl_radius", C.c_double), ("gl_depth", C.c_int32), ("pad_gl", C.c_int32)]


class _PhotonParams(C.Structure):
    _fields_ = [("n_photons", C.c_int64), ("max_depth", C.c_int32), ("seed", C.c_uint64), ("threads", C.c_int32),
                ("tie_t_rel", C.c_double), ("tie_edge_abs", C.c_double), ("tie_edge_rel_t", C.c_double),
                ("tie_lobe", C.c_double), ("tie_cos_sun", C.c_double), ("stride", C.c_int64),
                ("global_map", C.c_int32), ("pad", C.c_int32)]


class _Queries(C.Structure):
    _fields_ = [("x", C.c_void_p), ("wo", C.c_void_p), ("mat", C.c_void_p), ("beta", C.c_void_p),
                ("valid", C.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_philox_stream.argtypes = [vp, vp, i64, vp]
        L.orc_fresnel.argtypes = [dbl, dbl, dbl]
        L.orc_fresnel.restype = dbl
        L.orc_slab.argtypes = [dbl, dbl, dbl, dbl, dbl, vp, vp]
        L.orc_intersect.argtypes = [vp, vp, vp, vp, i64, i32, dbl, dbl, dbl, i32, vp, vp, vp, vp, vp]
        L.orc_intersect.restype = i32
        L.orc_shadow.argtypes = [vp, vp, vp, vp, i64, dbl, dbl, vp, vp]
        L.orc_shadow.restype = i32
        L.orc_render.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, vp]
        L.orc_render.restype = i32
        L.orc_photons.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_photons.restype = i64
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


@dataclass
class TieParams:
    """Margins that decide when FP32 rounding could change a path's outcome."""
    t_rel: float = 1e-5
    edge_abs: float = 2e-6
    edge_rel_t: float = 2e-6
    lobe: float = 2e-5
    cos_sun: float = 1e-6      # also: grazing hits and normals with 0 < |n_z| below it


def _scene_struct(sc):
    keep = dict(
        verts=np.ascontiguousarray(sc.verts, dtype=np.float32), mat=np.ascontiguousarray(sc.mat, dtype=np.uint16),
        mat_type=np.ascontiguousarray(sc.mat_type, dtype=np.int32),
        thickness=np.ascontiguousarray(sc.thickness_m, dtype=np.float32),
        n=np.ascontiguousarray(sc.n_tab, dtype=np.float32), k=np.ascontiguousarray(sc.k_tab, dtype=np.float32),
        rho=np.ascontiguousarray(sc.rho_tab, dtype=np.float32),
        sun_dir=np.ascontiguousarray(sc.sun_dir, dtype=np.float32),
        sun_E=np.ascontiguousarray(sc.sun_E, dtype=np.float32), env=np.ascontiguousarray(sc.env, dtype=np.float32))
    s = _Scene(_p(keep["verts"]).value, sc.n_tri, _p(keep["mat"]).value, sc.n_mat, _p(keep["mat_type"]).value,
               _p(keep["thickness"]).value, _p(keep["n"]).value, _p(keep["k"]).value, _p(keep["rho"]).value,
               sc.n_bins, float(sc.lambda_min_nm), float(sc.lambda_max_nm), _p(keep["sun_dir"]).value,
               _p(keep["sun_E"]).value, _p(keep["env"]).value, None, 0, None, None, None, None)
    tex = getattr(sc, "textures", None)
    if tex:
        keep["uv"] = np.ascontiguousarray(sc.uv, dtype=np.float32)
        keep["tex_dims"] = np.ascontiguousarray([[t.shape[1], t.shape[0]] for t in tex], dtype=np.int32)
        sizes = [t.size for t in tex]
        keep["tex_offset"] = np.ascontiguousarray(np.concatenate([[0], np.cumsum(sizes)[:-1]]), dtype=np.int64)
        keep["texels"] = np.ascontiguousarray(np.concatenate([np.asarray(t, dtype=np.float32).ravel() for t in tex]))
        keep["mat_tex"] = np.ascontiguousarray(sc.mat_tex, dtype=np.int32)
        s.uv, s.n_tex = _p(keep["uv"]).value, len(tex)
        s.tex_dims, s.tex_offset = _p(keep["tex_dims"]).value, _p(keep["tex_offset"]).value
        s.texels, s.mat_tex = _p(keep["texels"]).value, _p(keep["mat_tex"]).value
    return s, keep


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def philox_stream(ctr_base, key, n):
    c = np.ascontiguousarray(ctr_base, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros((n, 4), dtype=np.uint32)
    lib().orc_philox_stream(_p(c), _p(k), n, _p(out))
    return out


def fresnel(n, k, cos_t):
    return lib().orc_fresnel(float(n), float(k), float(cos_t))


def slab(n, k, lambda_nm, d_m, cos_t):
    R, T = C.c_double(), C.c_double()
    lib().orc_slab(float(n), float(k), float(lambda_nm), float(d_m), float(cos_t), C.byref(R), C.byref(T))
    return R.value, T.value


def intersect(scene, orig, dirs, skip=None, force_bvh=-1, tie: TieParams = TieParams(), threads=None):
    """Closest hit per ray: t (inf on miss), triangle id (-1), u, v, tie flag."""
    s, keep = _scene_struct(scene)
    o = np.ascontiguousarray(orig, dtype=np.float32)
    d = np.ascontiguousarray(dirs, dtype=np.float32)
    n = o.shape[0]
    sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.int32)
    t = np.zeros(n)
    ids = np.zeros(n, dtype=np.int64)
    u = np.zeros(n)
    v = np.zeros(n)
    tie_f = np.zeros(n, dtype=np.uint8)
    th = threads or min(8, os.cpu_count() or 1)
    lib().orc_intersect(C.byref(s), _p(o), _p(d), None if sk is None else _p(sk), n, force_bvh, tie.t_rel,
                        tie.edge_abs, tie.edge_rel_t, th, _p(t), _p(ids), _p(u), _p(v), _p(tie_f))
    return t, ids, u, v, tie_f.astype(bool)


def shadow(scene, orig, dirs, skip=None, tie: TieParams = TieParams()):
    """Sun visibility per ray and bin (0 if an opaque triangle blocks, else the product of the
    slab transmittances of the glass crossed) and a tie flag."""
    s, keep = _scene_struct(scene)
    o = np.ascontiguousarray(orig, dtype=np.float32)
    d = np.ascontiguousarray(dirs, dtype=np.float32)
    n = o.shape[0]
    sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.int32)
    vis = np.zeros((n, scene.n_bins))
    tie_f = np.zeros(n, dtype=np.uint8)
    lib().orc_shadow(C.byref(s), _p(o), _p(d), None if sk is None else _p(sk), n, tie.edge_abs, tie.edge_rel_t,
                     _p(vis), _p(tie_f))
    return vis, tie_f.astype(bool)


@dataclass
class RenderResult:
    image: np.ndarray      # [B][H][W] (full frame) or [B][n_pixels] (subset), FP64
    tied: np.ndarray       # number of tied samples per pixel
    stats: dict
    queries: dict | None = None
    photon_unc: np.ndarray | None = None   # like image: caustic radiance of photons near the radius


def render(scene, camera, spp=1, max_depth=4, seed=1, view=0, pixels=None, threads=None,
           tie: TieParams = TieParams(), force_bvh=-1, cached=False, first_sample=0, purpose=0,
           sample_per_entry=False, photons=None, radius=0.0, tie_radius=1e-4, global_photons=None,
           global_radius=0.0, global_depth=0) -> RenderResult:
    """Reference spectral image (mean of spp path samples per pixel), FP64 accumulation.
    With cached=True the paths stop at the vertex after bounce 2 and the query there
    (position, direction toward the previous vertex, material, throughput) is returned.
    purpose is added to the depth word of every random-number counter; with sample_per_entry
    entry i of ``pixels`` is one path (spp = 1) with sample index first_sample + i.
    photons / radius: a caustic map gathered at every opaque vertex; global_photons /
    global_radius / global_depth: from vertex global_depth on, the diffuse radiance of every opaque
    vertex comes from the global map (no direct term or caustic map there) and the path continues
    by the mirror lobe only (global_depth 0 with a map given: as 0, no global mode)."""
    s, keep = _scene_struct(scene)
    cam = _Camera((C.c_double * 3)(*camera.eye), (C.c_double * 3)(*camera.target), (C.c_double * 3)(*camera.up),
                  float(camera.vfov_deg), int(camera.width), int(camera.height))
    th = threads or min(8, os.cpu_count() or 1)
    prm = _Params(int(spp), int(max_depth), int(seed), int(view), int(th), int(force_bvh), tie.t_rel, tie.edge_abs,
                  tie.edge_rel_t, tie.lobe, tie.cos_sun, 1 if cached else 0, int(first_sample), int(purpose), 0,
                  1 if sample_per_entry else 0, None, None, None, 0, float(radius), float(tie_radius), None,
                  None, None, None, 0, float(global_radius), int(global_depth), 0)
    unc = None
    if photons is not None and len(photons["id"]) > 0:
        keep_ph = [np.ascontiguousarray(photons[k], dtype=np.float64) for k in ("pos", "dir", "flux")]
        prm.ph_pos, prm.ph_dir, prm.ph_flux = (_p(a).value for a in keep_ph)
        prm.n_photons = len(photons["id"])
    if global_photons is not None and len(global_photons["id"]) > 0:
        keep_gl = [np.ascontiguousarray(global_photons[k], dtype=np.float64) for k in ("pos", "dir", "flux")]
        prm.gl_pos, prm.gl_dir, prm.gl_flux = (_p(a).value for a in keep_gl)
        prm.n_global = len(global_photons["id"])
    B = scene.n_bins
    if pixels is None:
        npx = camera.width * camera.height
        px = None
    else:
        px = np.ascontiguousarray(pixels, dtype=np.int64)
        npx = px.shape[0]
    img = np.zeros((B, npx))
    tied = np.zeros(npx, dtype=np.int32)
    st = np.zeros(4, dtype=np.int64)
    if prm.n_photons > 0 or prm.n_global > 0:
        unc = np.zeros((B, npx))
        prm.ph_unc = _p(unc).value
    q = None
    qs = None
    if cached:
        nq = npx * spp
        q = dict(x=np.zeros((nq, 3)), wo=np.zeros((nq, 3)), mat=np.full(nq, -1, dtype=np.int32),
                 beta=np.zeros((nq, B)), valid=np.zeros(nq, dtype=np.uint8))
        qs = _Queries(_p(q["x"]).value, _p(q["wo"]).value, _p(q["mat"]).value, _p(q["beta"]).value,
                      _p(q["valid"]).value)
    lib().orc_render(C.byref(s), C.byref(cam), C.byref(prm), None if px is None else _p(px), npx, _p(img),
                     _p(tied), _p(st), None if qs is None else C.byref(qs))
    if pixels is None:
        img = img.reshape(B, camera.height, camera.width)
        tied = tied.reshape(camera.height, camera.width)
        if unc is not None:
            unc = unc.reshape(B, camera.height, camera.width)
    stats = dict(paths=int(st[0]), vertices=int(st[1]), shadow_rays=int(st[2]), tied_paths=int(st[3]))
    return RenderResult(img, tied, stats, q, unc)


def photons(scene, n_photons, max_depth=8, seed=1, threads=None, tie: TieParams = TieParams(), stride=1,
            global_map=False):
    """Caustic photon map (see orc_photons): records of photons stored at opaque vertices after at
    least one reflection, ordered by (photon, vertex): pos [n][3], dir [n][3] (direction of
    travel), flux [n][B], id [n] (photon index), depth [n] (vertex), tri [n] (the triangle it lies
    on); tied [n_photons] flags
    photons whose path FP32 rounding could change; area = the windows' projected area A. With
    stride k only photons 0, k, 2k, ... are traced (their records are those of the full map).
    global_map: every opaque vertex stores, and the diffuse lobe continues the photon."""
    s, keep = _scene_struct(scene)
    B = scene.n_bins
    th = threads or min(8, os.cpu_count() or 1)
    pp = _PhotonParams(int(n_photons), int(max_depth), int(seed), int(th), tie.t_rel, tie.edge_abs, tie.edge_rel_t,
                       tie.lobe, tie.cos_sun, int(stride), 1 if global_map else 0, 0)
    cap = max(1024, int(n_photons) // 2)
    while True:
        pos, dirs = np.zeros((cap, 3)), np.zeros((cap, 3))
        flux = np.zeros((cap, B))
        pid, dep = np.zeros(cap, dtype=np.int64), np.zeros(cap, dtype=np.int32)
        tri = np.zeros(cap, dtype=np.int32)
        tied = np.zeros(int(n_photons), dtype=np.uint8)
        area = C.c_double()
        n = lib().orc_photons(C.byref(s), C.byref(pp), cap, _p(pos), _p(dirs), _p(flux), _p(pid), _p(dep), _p(tri),
                              _p(tied),
                              C.byref(area))
        if n <= cap:
            break
        cap = int(n)
    return dict(pos=pos[:n], dir=dirs[:n], flux=flux[:n], id=pid[:n], depth=dep[:n], tri=tri[:n], tied=tied.astype(bool),
                area=area.value)


def training_records(scene, camera, pixels, first_path, max_depth=8, seed=1, view=0, record_depth=3, threads=None,
                     tie: TieParams = TieParams()):
    """Training paths of the radiance cache: entry i of ``pixels`` is path g = first_path + i,
    traced with random-number purpose 1 (bit 24 of the depth word of the counter
    (pixel, g, depth | purpose, view)) to full depth. At vertex ``record_depth`` the path records
    (position, direction toward the previous vertex, material) and restarts its throughput at
    one and its gathered radiance at zero; the radiance gathered from there on is the target.
    Returns x [n][3], wo [n][3], mat [n], valid [n] (vertex reached), target [n][B], tied [n]."""
    s, keep = _scene_struct(scene)
    cam = _Camera((C.c_double * 3)(*camera.eye), (C.c_double * 3)(*camera.target), (C.c_double * 3)(*camera.up),
                  float(camera.vfov_deg), int(camera.width), int(camera.height))
    th = threads or min(8, os.cpu_count() or 1)
    prm = _Params(1, int(max_depth), int(seed), int(view), int(th), -1, tie.t_rel, tie.edge_abs, tie.edge_rel_t,
                  tie.lobe, tie.cos_sun, 0, int(first_path), 1 << 24, int(record_depth), 1, None, None, None, 0, 0.0, 0.0,
                  None)
    B = scene.n_bins
    px = np.ascontiguousarray(pixels, dtype=np.int64)
    n = px.shape[0]
    img = np.zeros((B, n))
    tied = np.zeros(n, dtype=np.int32)
    st = np.zeros(4, dtype=np.int64)
    q = dict(x=np.zeros((n, 3)), wo=np.zeros((n, 3)), mat=np.full(n, -1, dtype=np.int32), beta=np.zeros((n, B)),
             valid=np.zeros(n, dtype=np.uint8))
    qs = _Queries(_p(q["x"]).value, _p(q["wo"]).value, _p(q["mat"]).value, _p(q["beta"]).value, _p(q["valid"]).value)
    lib().orc_render(C.byref(s), C.byref(cam), C.byref(prm), _p(px), n, _p(img), _p(tied), _p(st), C.byref(qs))
    return dict(x=q["x"], wo=q["wo"], mat=q["mat"], valid=q["valid"].astype(bool), target=img.T.copy(), tied=tied)
