"""ctypes binding of libspecdd.so -- argument marshalling only.

Every step of the rendering path runs in the library's HIP kernels; this module only turns
arrays and tensors into pointers, PyTorch provides the device memory and the stream. If the
library is missing the import fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspecdd.so")

SDD_OK = 0
ERRORS = {-1: "SDD_ERR_INVALID_ARG", -2: "SDD_ERR_HIP", -3: "SDD_ERR_WORKSPACE", -4: "SDD_ERR_QUEUE_OVERFLOW",
          -5: "SDD_ERR_NOT_READY", -6: "SDD_ERR_INTERNAL", -7: "SDD_ERR_DEVICE"}

MODE_PLAIN = 0
MODE_CACHED = 1


class SddError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Material(C.Structure):
    _fields_ = [("type", C.c_int32), ("thickness_m", C.c_float)]


class SceneDesc(C.Structure):
    _fields_ = [("verts", C.c_void_p), ("mat", C.c_void_p), ("n_tri", C.c_int64), ("materials", C.c_void_p),
                ("n_mat", C.c_int32), ("n_tab", C.c_void_p), ("k_tab", C.c_void_p), ("rho_tab", C.c_void_p),
                ("n_bins", C.c_int32), ("lambda_min_nm", C.c_float), ("lambda_max_nm", C.c_float),
                ("sun_dir", C.c_float * 3), ("sun_irradiance", C.c_void_p), ("env_radiance", C.c_void_p),
                ("grid", C.c_int32 * 3), ("uv", C.c_void_p), ("n_tex", C.c_int32), ("textures", C.c_void_p),
                ("mat_texture", C.c_void_p)]


class Texture(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("tau0", C.c_void_p)]


class Daylight(C.Structure):
    _fields_ = [("day_of_year", C.c_int32), ("clock_hours", C.c_float), ("utc_offset_hours", C.c_float),
                ("latitude_deg", C.c_float), ("longitude_deg", C.c_float), ("scene_x_azimuth_deg", C.c_float),
                ("temperature_k", C.c_float), ("pressure_ratio", C.c_float)]


class DaylightInfo(C.Structure):
    _fields_ = [("elevation_deg", C.c_float), ("azimuth_deg", C.c_float), ("air_mass", C.c_float),
                ("distance_factor", C.c_float)]


def daylight(day_of_year=172, clock_hours=12.0, utc_offset_hours=0.0, latitude_deg=49.14, longitude_deg=2.38,
             scene_x_azimuth_deg=90.0, temperature_k=5778.0, pressure_ratio=1.0) -> Daylight:
    d = Daylight()
    d.day_of_year, d.clock_hours, d.utc_offset_hours = int(day_of_year), clock_hours, utc_offset_hours
    d.latitude_deg, d.longitude_deg, d.scene_x_azimuth_deg = latitude_deg, longitude_deg, scene_x_azimuth_deg
    d.temperature_k, d.pressure_ratio = temperature_k, pressure_ratio
    return d


def daylight_sun(params: Daylight, n_bins, lambda_min_nm=380.0, lambda_max_nm=780.0):
    """The library's sun for a date and time (host computation): (direction [3], E [n_bins], info)."""
    d = (C.c_float * 3)()
    E = np.zeros(n_bins, dtype=np.float32)
    info = DaylightInfo()
    _check(lib().sdd_daylight_sun(C.byref(params), int(n_bins), float(lambda_min_nm), float(lambda_max_nm), d,
                                  _ptr(E), C.byref(info)))
    return np.array(d[:], dtype=np.float32), E, {n: getattr(info, n) for n, _ in DaylightInfo._fields_}


class SceneInfo(C.Structure):
    _fields_ = [("n_tri", C.c_int64), ("n_refs", C.c_int64), ("n_nodes", C.c_int64), ("n_cells", C.c_int64),
                ("n_empty_cells", C.c_int64), ("max_depth", C.c_int32), ("max_leaf", C.c_int32),
                ("device_bytes", C.c_size_t), ("grid_lo", C.c_float * 3), ("grid_hi", C.c_float * 3)]


class Camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("target", C.c_float * 3), ("up", C.c_float * 3), ("vfov_deg", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32)]


class RenderParams(C.Structure):
    _fields_ = [("spp", C.c_int32), ("max_depth", C.c_int32), ("seed", C.c_uint64), ("mode", C.c_int32),
                ("wave_paths", C.c_int32), ("queue_rounds", C.c_int32), ("view", C.c_uint32),
                ("timing", C.c_int32), ("first_sample", C.c_int32), ("use_graph", C.c_int32),
                ("cell_order", C.c_int32), ("persistent", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "paths", "vertices", "ext_rays", "shadow_rays", "cell_visits", "migrations", "escapes", "glass_crossings",
        "trace_launches", "shade_launches", "wavefronts", "err_cross_overflow", "err_nonfinite", "err_stack",
        "node_visits", "tri_tests")] + [
        ("trace_ms", C.c_double), ("shade_ms", C.c_double), ("graph_launches", C.c_uint64), ("graph_ms", C.c_double),
        ("cache_queries", C.c_uint64), ("query_launches", C.c_uint64), ("train_batches", C.c_uint64),
        ("query_ms", C.c_double), ("train_ms", C.c_double), ("photon_vertices", C.c_uint64),
        ("photons_found", C.c_uint64), ("photon_lit_vertices", C.c_uint64), ("photon_candidates", C.c_uint64),
        ("photon_candidates_max", C.c_uint64), ("photon_launches", C.c_uint64),
        ("photon_ms", C.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class TuneSpace(C.Structure):
    _fields_ = [("n_waves", C.c_int32), ("wave_paths", C.c_int32 * 8), ("n_grids", C.c_int32),
                ("grids", (C.c_int32 * 3) * 8), ("n_rounds", C.c_int32), ("queue_rounds", C.c_int32 * 4),
                ("calib_spp", C.c_int32), ("reps", C.c_int32), ("n_orders", C.c_int32),
                ("cell_orders", C.c_int32 * 2), ("try_persistent", C.c_int32)]


class TunePoint(C.Structure):
    _fields_ = [("grid", C.c_int32 * 3), ("wave_paths", C.c_int32), ("queue_rounds", C.c_int32),
                ("cell_order", C.c_int32), ("persistent", C.c_int32), ("pad", C.c_int32),
                ("samples_per_s", C.c_double)]

    def as_dict(self):
        return dict(grid=list(self.grid), wave_paths=self.wave_paths, queue_rounds=self.queue_rounds,
                    cell_order=self.cell_order, persistent=self.persistent, samples_per_s=self.samples_per_s)


class TuneResult(C.Structure):
    _fields_ = [("best", TunePoint), ("from_cache", C.c_int32), ("n_tried", C.c_int32), ("tried", TunePoint * 128)]


class CacheConfig(C.Structure):
    _fields_ = [("levels_pos", C.c_int32), ("log2_table_pos", C.c_int32), ("nmin_pos", C.c_float),
                ("nmax_pos", C.c_float), ("levels_dir", C.c_int32), ("log2_table_dir", C.c_int32),
                ("nmin_dir", C.c_float), ("nmax_dir", C.c_float), ("n_mat", C.c_int32), ("max_bins", C.c_int32),
                ("max_records", C.c_int32), ("max_step", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("box_lo", C.c_float * 3), ("box_hi", C.c_float * 3)]


class CacheInfo(C.Structure):
    _fields_ = [("n_param", C.c_int64), ("device_bytes", C.c_size_t), ("n_in", C.c_int32),
                ("npos", C.c_int32 * 16), ("ndir", C.c_int32 * 16), ("dense_pos", C.c_uint32),
                ("dense_dir", C.c_uint32), ("adam_steps", C.c_int64), ("train_paths_done", C.c_int64)]


class TrainParams(C.Structure):
    _fields_ = [("train_paths", C.c_int32), ("step_records", C.c_int32), ("steps", C.c_int32), ("every", C.c_int32)]


class PhotonParams(C.Structure):
    _fields_ = [("n_photons", C.c_int64), ("max_depth", C.c_int32), ("radius", C.c_float), ("seed", C.c_uint64),
                ("capacity", C.c_int64), ("wave_paths", C.c_int32), ("queue_rounds", C.c_int32),
                ("kind", C.c_int32), ("pad", C.c_int32)]


class PhotonInfo(C.Structure):
    _fields_ = [("stored", C.c_int64), ("dropped", C.c_int64), ("n_windows", C.c_int32), ("n_buckets", C.c_int32),
                ("window_area", C.c_double), ("device_bytes", C.c_size_t)]


PHOTON_CAUSTIC, PHOTON_GLOBAL = 0, 1


def photon_params(n_photons, radius, max_depth=8, seed=1, capacity=None, wave_paths=0, queue_rounds=0,
                  kind=PHOTON_CAUSTIC) -> PhotonParams:
    cap = int(capacity) if capacity is not None else int(n_photons) * (int(max_depth) - 1)
    return PhotonParams(int(n_photons), int(max_depth), float(radius), int(seed), max(1, min(cap, 1 << 28)),
                        int(wave_paths), int(queue_rounds), int(kind), 0)


# Every exported function: (name, restype, argtypes)
_vp, _i32, _i64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
SIGNATURES = [
    ("sdd_scene_create", _i32, [_vp, _vp]),
    ("sdd_scene_destroy", None, [_vp]),
    ("sdd_scene_get_info", _i32, [_vp, _vp]),
    ("sdd_scene_device_bytes", _i32, [_vp, _vp]),
    ("sdd_scene_host_image", _i32, [_vp, _vp, _vp]),
    ("sdd_create", _i32, [_vp, C.c_int, _vp]),
    ("sdd_destroy", None, [_vp]),
    ("sdd_set_stream", _i32, [_vp, _vp]),
    ("sdd_scene_upload", _i32, [_vp, _vp, _vp, _sz]),
    ("sdd_workspace_bytes", _i32, [_vp, _vp, _vp]),
    ("sdd_set_sun", _i32, [_vp, _vp, _vp, _vp]),
    ("sdd_set_env", _i32, [_vp, _vp, _vp]),
    ("sdd_daylight_sun", _i32, [_vp, _i32, C.c_float, C.c_float, _vp, _vp, _vp]),
    ("sdd_set_daylight", _i32, [_vp, _vp, _vp, _vp]),
    ("sdd_render", _i32, [_vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    ("sdd_render_batch", _i32, [_vp, _vp, _vp, _vp, _i32, _vp, _vp, _sz, _vp]),
    ("sdd_render_noalloc", _i32, [_vp, _vp, _vp, _vp, _vp]),
    ("sdd_query_workspace_bytes", _i32, [_vp, _i64, _vp]),
    ("sdd_trace", _i32, [_vp, _vp, _vp, _vp, _vp, _i64, _vp, _sz, _vp, _vp, _vp, _vp]),
    ("sdd_shadow", _i32, [_vp, _vp, _vp, _vp, _vp, _i64, _vp, _sz, _vp]),
    ("sdd_philox", _i32, [_vp, _vp, _vp, _i64, _vp]),
    ("sdd_finish", _i32, [_vp]),
    ("sdd_spectral_to_srgb", _i32, [_vp, _vp, _i32, C.c_float, C.c_float, _i64, C.c_float, _vp, _vp]),
    ("sdd_get_stats", _i32, [_vp, _vp]),
    ("sdd_reset_stats", _i32, [_vp]),
    ("sdd_last_error", C.c_char_p, [_vp]),
    ("sdd_autotune", _i32, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _sz, _vp, _sz, _vp, C.c_char_p, _vp]),
    ("sdd_cache_param_count", _i32, [_vp, _vp]),
    ("sdd_cache_bytes", _i32, [_vp, _vp]),
    ("sdd_cache_create", _i32, [_vp, _vp, _vp, _sz, _vp]),
    ("sdd_cache_destroy", None, [_vp]),
    ("sdd_cache_get_info", _i32, [_vp, _vp, _vp]),
    ("sdd_cache_init", _i32, [_vp, _vp, C.c_uint64]),
    ("sdd_cache_set_params", _i32, [_vp, _vp, _vp, _i64]),
    ("sdd_cache_get_params", _i32, [_vp, _vp, _vp, _i64]),
    ("sdd_cache_get_grads", _i32, [_vp, _vp, _vp, _i64]),
    ("sdd_cache_eval", _i32, [_vp, _vp, _vp, _vp, _vp, _i64, _i32, _vp]),
    ("sdd_cache_backward", _i32, [_vp, _vp, _vp, _vp, _vp, _vp, _i64, _i32]),
    ("sdd_cache_step", _i32, [_vp, _vp]),
    ("sdd_cache_train", _i32, [_vp, _vp, _vp, _vp, _vp, _vp, _i64, _i32]),
    ("sdd_cache_loss", _i32, [_vp, _vp, _vp]),
    ("sdd_render_cached", _i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    ("sdd_cache_get_records", _i32, [_vp, _vp, _i64, _vp, _vp, _vp]),
    ("sdd_photon_map_bytes", _i32, [_vp, _vp, _vp]),
    ("sdd_photon_workspace_bytes", _i32, [_vp, _vp, _vp]),
    ("sdd_photon_map_create", _i32, [_vp, _vp, _vp, _vp, _sz, _vp]),
    ("sdd_photon_map_destroy", None, [_vp]),
    ("sdd_photon_map_build", _i32, [_vp, _vp, _vp, _vp, _sz]),
    ("sdd_photon_map_info", _i32, [_vp, _vp, _vp]),
    ("sdd_photon_map_records", _i32, [_vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    ("sdd_photon_map_load", _i32, [_vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    ("sdd_render_photons", _i32, [_vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _sz, _vp]),
]

_lib = None


def lib():
    """Load libspecdd.so (built in-tree by ``paper_1912_04000_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1912_04000_amd.build` "
                              "(there is no fallback implementation)")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != SDD_OK:
        msg = lib().sdd_last_error(ctx)
        raise SddError(rc, msg.decode() if msg else "")


def _ptr(a):
    """Pointer of a contiguous numpy array or torch tensor."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    assert a.is_contiguous()
    return a.data_ptr()


def make_desc(verts, mat, mat_type, thickness_m, n_tab, k_tab, rho_tab, lambda_min_nm, lambda_max_nm, sun_dir, sun_E,
              env=None, grid=(2, 2, 2), uv=None, textures=None, mat_tex=None):
    """sdd_scene_desc over host arrays; returns the struct and the arrays it points into."""
    keep = dict(
        verts=np.ascontiguousarray(verts, dtype=np.float32), mat=np.ascontiguousarray(mat, dtype=np.uint16),
        n=np.ascontiguousarray(n_tab, dtype=np.float32), k=np.ascontiguousarray(k_tab, dtype=np.float32),
        rho=np.ascontiguousarray(rho_tab, dtype=np.float32), E=np.ascontiguousarray(sun_E, dtype=np.float32),
        env=None if env is None else np.ascontiguousarray(env, dtype=np.float32))
    n_mat = len(mat_type)
    mats = (Material * n_mat)()
    for i in range(n_mat):
        mats[i].type = int(mat_type[i])
        mats[i].thickness_m = float(thickness_m[i])
    keep["mats"] = mats
    d = SceneDesc()
    d.verts = _ptr(keep["verts"])
    d.mat = _ptr(keep["mat"])
    d.n_tri = keep["verts"].shape[0]
    d.materials = C.cast(mats, C.c_void_p)
    d.n_mat = n_mat
    d.n_tab, d.k_tab, d.rho_tab = _ptr(keep["n"]), _ptr(keep["k"]), _ptr(keep["rho"])
    d.n_bins = int(keep["n"].shape[1])
    d.lambda_min_nm, d.lambda_max_nm = float(lambda_min_nm), float(lambda_max_nm)
    d.sun_dir[:] = [float(x) for x in sun_dir]
    d.sun_irradiance = _ptr(keep["E"])
    d.env_radiance = _ptr(keep["env"]) if keep["env"] is not None else None
    d.grid[:] = [int(g) for g in grid]
    if textures:
        keep["uv"] = np.ascontiguousarray(uv, dtype=np.float32)
        keep["tex_data"] = [np.ascontiguousarray(t, dtype=np.float32) for t in textures]
        tx = (Texture * len(textures))()
        for i, t in enumerate(keep["tex_data"]):
            tx[i].height, tx[i].width = int(t.shape[0]), int(t.shape[1])
            tx[i].tau0 = _ptr(t)
        keep["tex"] = tx
        keep["mat_tex"] = np.ascontiguousarray(mat_tex, dtype=np.int32)
        d.uv = _ptr(keep["uv"])
        d.n_tex = len(textures)
        d.textures = C.cast(tx, C.c_void_p)
        d.mat_texture = _ptr(keep["mat_tex"])
    return d, keep


def desc_from(sc, grid=(2, 2, 2)):
    return make_desc(sc.verts, sc.mat, sc.mat_type, sc.thickness_m, sc.n_tab, sc.k_tab, sc.rho_tab, sc.lambda_min_nm,
                     sc.lambda_max_nm, sc.sun_dir, sc.sun_E, sc.env, grid, getattr(sc, "uv", None),
                     getattr(sc, "textures", None), getattr(sc, "mat_tex", None))


class Scene:
    """Host-built cell-decomposed scene (``sdd_scene``), optionally uploaded to a device buffer."""

    def __init__(self, verts, mat, mat_type, thickness_m, n_tab, k_tab, rho_tab, lambda_min_nm, lambda_max_nm,
                 sun_dir, sun_E, env=None, grid=(2, 2, 2), uv=None, textures=None, mat_tex=None):
        d, self._keep = make_desc(verts, mat, mat_type, thickness_m, n_tab, k_tab, rho_tab, lambda_min_nm,
                                  lambda_max_nm, sun_dir, sun_E, env, grid, uv, textures, mat_tex)
        self.n_bins = d.n_bins
        h = C.c_void_p()
        _check(lib().sdd_scene_create(C.byref(d), C.byref(h)))
        self._desc = d
        self.handle = h
        self.grid = tuple(int(g) for g in grid)
        self.device_buffer = None

    @classmethod
    def from_description(cls, sc, grid=(2, 2, 2)):
        """Build from any object carrying the scene arrays by name (verts, mat, mat_type, ...)."""
        return cls(sc.verts, sc.mat, sc.mat_type, sc.thickness_m, sc.n_tab, sc.k_tab, sc.rho_tab, sc.lambda_min_nm,
                   sc.lambda_max_nm, sc.sun_dir, sc.sun_E, sc.env, grid, getattr(sc, "uv", None),
                   getattr(sc, "textures", None), getattr(sc, "mat_tex", None))

    def info(self) -> dict:
        i = SceneInfo()
        _check(lib().sdd_scene_get_info(self.handle, C.byref(i)))
        return dict(n_tri=i.n_tri, n_refs=i.n_refs, n_nodes=i.n_nodes, n_cells=i.n_cells,
                    n_empty_cells=i.n_empty_cells, max_depth=i.max_depth, max_leaf=i.max_leaf,
                    device_bytes=i.device_bytes, grid_lo=list(i.grid_lo), grid_hi=list(i.grid_hi))

    def device_bytes(self) -> int:
        b = C.c_size_t()
        _check(lib().sdd_scene_device_bytes(self.handle, C.byref(b)))
        return b.value

    def host_image(self) -> np.ndarray:
        p, b = C.c_void_p(), C.c_size_t()
        _check(lib().sdd_scene_host_image(self.handle, C.byref(p), C.byref(b)))
        return np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_uint8)), shape=(b.value,)).copy()

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.sdd_scene_destroy(self.handle)
            self.handle = None


def camera(eye, target, up=(0.0, 0.0, 1.0), vfov_deg=60.0, width=64, height=64) -> Camera:
    c = Camera()
    c.eye[:] = [float(x) for x in eye]
    c.target[:] = [float(x) for x in target]
    c.up[:] = [float(x) for x in up]
    c.vfov_deg = float(vfov_deg)
    c.width, c.height = int(width), int(height)
    return c


def cache_config(n_mat, box_lo, box_hi, levels_pos=12, log2_table_pos=19, nmin_pos=16.0, nmax_pos=2048.0,
                 levels_dir=12, log2_table_dir=14, nmin_dir=4.0, nmax_dir=256.0, max_bins=40, max_records=1 << 17,
                 max_step=1 << 14, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8) -> CacheConfig:
    c = CacheConfig()
    c.levels_pos, c.log2_table_pos, c.nmin_pos, c.nmax_pos = int(levels_pos), int(log2_table_pos), nmin_pos, nmax_pos
    c.levels_dir, c.log2_table_dir, c.nmin_dir, c.nmax_dir = int(levels_dir), int(log2_table_dir), nmin_dir, nmax_dir
    c.n_mat, c.max_bins, c.max_records, c.max_step = int(n_mat), int(max_bins), int(max_records), int(max_step)
    c.lr, c.beta1, c.beta2, c.eps = lr, beta1, beta2, eps
    c.box_lo[:] = [float(x) for x in box_lo]
    c.box_hi[:] = [float(x) for x in box_hi]
    return c


def train_params(train_paths=0, step_records=1 << 14, steps=4, every=0) -> TrainParams:
    t = TrainParams()
    t.train_paths, t.step_records, t.steps, t.every = int(train_paths), int(step_records), int(steps), int(every)
    return t


def render_params(spp=1, max_depth=4, seed=1, mode=MODE_PLAIN, wave_paths=0, queue_rounds=0, view=0, timing=0,
                  first_sample=0, use_graph=0, cell_order=0, persistent=0):
    p = RenderParams()
    p.cell_order = int(cell_order)
    p.persistent = int(persistent)
    p.first_sample = int(first_sample)
    p.use_graph = int(use_graph)
    p.spp, p.max_depth, p.seed, p.mode = int(spp), int(max_depth), int(seed), int(mode)
    p.wave_paths, p.queue_rounds, p.view, p.timing = int(wave_paths), int(queue_rounds), int(view), int(timing)
    return p


class Context:
    """``sdd_ctx`` on a torch CUDA (HIP) device; device memory comes from torch allocations."""

    def __init__(self, device=0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(lib().sdd_create(C.byref(h), int(device), C.c_void_p(self.stream.cuda_stream)))
        self.handle = h
        self._ws = None

    def _err(self, rc):
        _check(rc, self.handle)

    def upload(self, scene: Scene):
        nbytes = scene.device_bytes()
        buf = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        view = buf[off:off + nbytes]
        self._err(lib().sdd_scene_upload(self.handle, scene.handle, C.c_void_p(view.data_ptr()), nbytes))
        scene.device_buffer = buf
        return scene

    def set_sun(self, scene: Scene, dir_to_sun, irradiance):
        d = (C.c_float * 3)(*[float(x) for x in dir_to_sun])
        E = np.ascontiguousarray(irradiance, dtype=np.float32)
        assert E.shape == (scene.n_bins,)
        self._err(lib().sdd_set_sun(self.handle, scene.handle, d, _ptr(E)))

    def set_daylight(self, scene: Scene, params: Daylight) -> dict:
        info = DaylightInfo()
        self._err(lib().sdd_set_daylight(self.handle, scene.handle, C.byref(params), C.byref(info)))
        return {n: getattr(info, n) for n, _ in DaylightInfo._fields_}

    def set_env(self, scene: Scene, radiance=None):
        L = None if radiance is None else np.ascontiguousarray(radiance, dtype=np.float32)
        assert L is None or L.shape == (scene.n_bins,)
        self._err(lib().sdd_set_env(self.handle, scene.handle, _ptr(L)))

    def workspace(self, nbytes):
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
        return self._ws

    def workspace_bytes(self, scene: Scene, params: RenderParams) -> int:
        b = C.c_size_t()
        _check(lib().sdd_workspace_bytes(scene.handle, C.byref(params), C.byref(b)))
        return b.value

    def render(self, scene: Scene, cam: Camera, params: RenderParams, out=None, finish=True):
        ws = self.workspace(self.workspace_bytes(scene, params))
        img = out if out is not None else self.torch.empty((scene.n_bins, cam.height, cam.width),
                                                           dtype=self.torch.float32, device=self.device)
        self._err(lib().sdd_render(self.handle, scene.handle, C.byref(cam), C.byref(params),
                                   C.c_void_p(ws.data_ptr()), ws.numel(), C.c_void_p(img.data_ptr())))
        if finish:
            self.finish()
        return img

    def render_noalloc(self, scene: Scene, cam: Camera, params: RenderParams, out, finish=True):
        """sdd_render with the library's static device workspace (no allocation by the library);
        `out` is the caller's [n_bins][H][W] float32 device tensor."""
        self._err(lib().sdd_render_noalloc(self.handle, scene.handle, C.byref(cam), C.byref(params),
                                           C.c_void_p(out.data_ptr())))
        if finish:
            self.finish()
        return out

    def render_batch(self, scene: Scene, cams, spp, params: RenderParams, outs=None, finish=True):
        n = len(cams)
        arr = (Camera * n)(*cams)
        spp_arr = (C.c_int32 * n)(*[int(s) for s in spp])
        if outs is None:
            outs = [self.torch.empty((scene.n_bins, c.height, c.width), dtype=self.torch.float32, device=self.device)
                    for c in cams]
        ptrs = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
        ws = self.workspace(self.workspace_bytes(scene, params))
        self._err(lib().sdd_render_batch(self.handle, scene.handle, arr, spp_arr, n, C.byref(params),
                                         C.c_void_p(ws.data_ptr()), ws.numel(), ptrs))
        if finish:
            self.finish()
        return outs

    def autotune(self, scene_description, cams, base: RenderParams, waves, grids, rounds=(1, 2), calib_spp=1,
                 reps=2, cache_path=None, scene_bytes=None, ws_bytes=None, orders=(), try_persistent=False):
        """Measure (grid, wavefront size, queue rounds, cell order) candidates, and with
        try_persistent the persistent kernel on every grid, on calibration renders of the views
        and return the fastest (the library's autotuner; cached in cache_path). An empty `orders`
        keeps the base parameters' cell order."""
        torch = self.torch
        d, keep = desc_from(scene_description)
        sp = TuneSpace()
        sp.n_waves = len(waves)
        for i, wv in enumerate(waves):
            sp.wave_paths[i] = int(wv)
        sp.n_grids = len(grids)
        for i, g in enumerate(grids):
            sp.grids[i][:] = [int(x) for x in g]
        sp.n_rounds = len(rounds)
        for i, r in enumerate(rounds):
            sp.queue_rounds[i] = int(r)
        sp.calib_spp, sp.reps = int(calib_spp), int(reps)
        sp.n_orders = len(orders)
        for i, o in enumerate(orders):
            sp.cell_orders[i] = int(o)
        sp.try_persistent = int(bool(try_persistent))
        if scene_bytes is None:
            # finest grid bounds the scene size (more duplicated references): measure it once
            finest = max(grids, key=lambda g: g[0] * g[1] * g[2])
            probe = Scene.from_description(scene_description, grid=finest)
            scene_bytes = int(probe.device_bytes() * 1.25) + (1 << 20)
        if ws_bytes is None:
            p = RenderParams()
            C.memmove(C.byref(p), C.byref(base), C.sizeof(RenderParams))
            p.wave_paths = int(max(waves))
            b = C.c_size_t()
            probe = probe if "probe" in locals() else Scene.from_description(scene_description)
            _check(lib().sdd_workspace_bytes(probe.handle, C.byref(p), C.byref(b)))
            ws_bytes = b.value
            if try_persistent:
                p.wave_paths, p.persistent = 0, 1
                _check(lib().sdd_workspace_bytes(probe.handle, C.byref(p), C.byref(b)))
                ws_bytes = max(ws_bytes, b.value)
        sbuf = torch.empty(scene_bytes + 256, dtype=torch.uint8, device=self.device)
        soff = (-sbuf.data_ptr()) % 256
        ws = self.workspace(ws_bytes)
        n = len(cams)
        arr = (Camera * n)(*cams)
        outs = [torch.empty((d.n_bins, c.height, c.width), dtype=torch.float32, device=self.device) for c in cams]
        ptrs = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
        res = TuneResult()
        self._err(lib().sdd_autotune(self.handle, C.byref(d), arr, n, C.byref(base), C.byref(sp),
                                     C.c_void_p(sbuf.data_ptr() + soff), scene_bytes, C.c_void_p(ws.data_ptr()),
                                     ws.numel(), ptrs, None if cache_path is None else cache_path.encode(),
                                     C.byref(res)))
        return dict(best=res.best.as_dict(), from_cache=bool(res.from_cache),
                    tried=[res.tried[i].as_dict() for i in range(res.n_tried)])

    def _query_ws(self, scene, n):
        b = C.c_size_t()
        _check(lib().sdd_query_workspace_bytes(scene.handle, int(n), C.byref(b)))
        return self.workspace(b.value)

    def trace(self, scene: Scene, orig, dirs, skip=None):
        """Closest hits of device rays (float32 [n][3]); returns (t, id, u, v) tensors."""
        torch = self.torch
        n = orig.shape[0]
        ws = self._query_ws(scene, n)
        t = torch.empty(n, dtype=torch.float32, device=self.device)
        ids = torch.empty(n, dtype=torch.int32, device=self.device)
        u = torch.empty_like(t)
        v = torch.empty_like(t)
        self._err(lib().sdd_trace(self.handle, scene.handle, C.c_void_p(orig.data_ptr()), C.c_void_p(dirs.data_ptr()),
                                  None if skip is None else C.c_void_p(skip.data_ptr()), n, C.c_void_p(ws.data_ptr()),
                                  ws.numel(), C.c_void_p(t.data_ptr()), C.c_void_p(ids.data_ptr()),
                                  C.c_void_p(u.data_ptr()), C.c_void_p(v.data_ptr())))
        self.finish()
        return t, ids, u, v

    def shadow(self, scene: Scene, orig, dirs, skip=None):
        torch = self.torch
        n = orig.shape[0]
        ws = self._query_ws(scene, n)
        vis = torch.empty((n, scene.n_bins), dtype=torch.float32, device=self.device)
        self._err(lib().sdd_shadow(self.handle, scene.handle, C.c_void_p(orig.data_ptr()),
                                   C.c_void_p(dirs.data_ptr()), None if skip is None else C.c_void_p(skip.data_ptr()),
                                   n, C.c_void_p(ws.data_ptr()), ws.numel(), C.c_void_p(vis.data_ptr())))
        self.finish()
        return vis

    def philox(self, ctr, key, n):
        torch = self.torch
        out = torch.empty((n, 4), dtype=torch.int32, device=self.device)
        c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
        k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
        self._err(lib().sdd_philox(self.handle, c, k, int(n), C.c_void_p(out.data_ptr())))
        self.finish()
        return out

    def finish(self):
        self._err(lib().sdd_finish(self.handle))

    def spectral_to_srgb(self, image, lambda_min_nm=380.0, lambda_max_nm=780.0, exposure=1.0, want_xyz=True,
                         want_srgb=True, finish=True, xyz_out=None, srgb_out=None):
        """Colorimetry of a device image [B][H][W]: (XYZ [3][H][W] or None, sRGB [H][W][3] or None)."""
        torch = self.torch
        assert image.dtype == torch.float32 and image.is_contiguous() and image.dim() == 3
        B, H, W = image.shape
        xyz = xyz_out if xyz_out is not None else (
            torch.empty((3, H, W), dtype=torch.float32, device=self.device) if want_xyz else None)
        rgb = srgb_out if srgb_out is not None else (
            torch.empty((H, W, 3), dtype=torch.float32, device=self.device) if want_srgb else None)
        self._err(lib().sdd_spectral_to_srgb(self.handle, C.c_void_p(image.data_ptr()), int(B), float(lambda_min_nm),
                                             float(lambda_max_nm), int(H * W), float(exposure),
                                             None if xyz is None else C.c_void_p(xyz.data_ptr()),
                                             None if rgb is None else C.c_void_p(rgb.data_ptr())))
        if finish:
            self.finish()
        return xyz, rgb

    # -- learned radiance cache ------------------------------------------------------------
    def cache(self, cfg: CacheConfig, seed=None):
        """Create a radiance cache in a torch device buffer; random init when seed is given."""
        return Cache(self, cfg, seed)

    def render_cached(self, scene: Scene, cache, cam: Camera, params: RenderParams, train: TrainParams = None,
                      out=None, finish=True):
        ws = self.workspace(self.workspace_bytes(scene, params))
        img = out if out is not None else self.torch.empty((scene.n_bins, cam.height, cam.width),
                                                           dtype=self.torch.float32, device=self.device)
        self._err(lib().sdd_render_cached(self.handle, scene.handle, cache.handle, C.byref(cam), C.byref(params),
                                          None if train is None else C.byref(train), C.c_void_p(ws.data_ptr()),
                                          ws.numel(), C.c_void_p(img.data_ptr())))
        if finish:
            self.finish()
        return img

    # -- caustic photon map ----------------------------------------------------------------
    def photon_map(self, scene: Scene, params: PhotonParams, build=True, finish=True):
        """A caustic photon map for `scene` in a torch device buffer, built at once by default."""
        m = PhotonMap(self, scene, params)
        if build:
            m.build(scene, finish=finish)
        return m

    def render_photons(self, scene: Scene, pmap, cam: Camera, params: RenderParams, out=None, finish=True,
                       global_map=None, global_from=0):
        """sdd_render_photons: `pmap` the caustic map (or None), `global_map` a global map used
        from vertex `global_from` on."""
        ws = self.workspace(self.workspace_bytes(scene, params))
        img = out if out is not None else self.torch.empty((scene.n_bins, cam.height, cam.width),
                                                           dtype=self.torch.float32, device=self.device)
        self._err(lib().sdd_render_photons(self.handle, scene.handle, None if pmap is None else pmap.handle,
                                           None if global_map is None else global_map.handle, int(global_from),
                                           C.byref(cam), C.byref(params), C.c_void_p(ws.data_ptr()), ws.numel(),
                                           C.c_void_p(img.data_ptr())))
        if finish:
            self.finish()
        return img

    def stats(self) -> dict:
        s = Stats()
        self._err(lib().sdd_get_stats(self.handle, C.byref(s)))
        return s.as_dict()

    def reset_stats(self):
        self._err(lib().sdd_reset_stats(self.handle))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.sdd_destroy(self.handle)
            self.handle = None


def param_count(cfg: CacheConfig) -> int:
    n = C.c_int64()
    _check(lib().sdd_cache_param_count(C.byref(cfg), C.byref(n)))
    return n.value


class Cache:
    """``sdd_cache`` bound to a torch device buffer."""

    def __init__(self, ctx: Context, cfg: CacheConfig, seed=None):
        torch = ctx.torch
        self.ctx, self.cfg = ctx, cfg
        b = C.c_size_t()
        _check(lib().sdd_cache_bytes(C.byref(cfg), C.byref(b)))
        self.buffer = torch.empty(b.value + 256, dtype=torch.uint8, device=ctx.device)
        off = (-self.buffer.data_ptr()) % 256
        h = C.c_void_p()
        ctx._err(lib().sdd_cache_create(ctx.handle, C.byref(cfg), C.c_void_p(self.buffer.data_ptr() + off), b.value,
                                        C.byref(h)))
        self.handle = h
        self.n_param = param_count(cfg)
        if seed is not None:
            self.init(seed)

    def init(self, seed):
        self.ctx._err(lib().sdd_cache_init(self.ctx.handle, self.handle, int(seed)))

    def info(self) -> dict:
        i = CacheInfo()
        self.ctx._err(lib().sdd_cache_get_info(self.ctx.handle, self.handle, C.byref(i)))
        return dict(n_param=i.n_param, device_bytes=i.device_bytes, n_in=i.n_in,
                    npos=list(i.npos)[:self.cfg.levels_pos], ndir=list(i.ndir)[:self.cfg.levels_dir],
                    dense_pos=i.dense_pos, dense_dir=i.dense_dir, adam_steps=i.adam_steps,
                    train_paths_done=i.train_paths_done)

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        self.ctx._err(lib().sdd_cache_set_params(self.ctx.handle, self.handle, _ptr(a), a.size))

    def params(self) -> np.ndarray:
        a = np.empty(self.n_param, dtype=np.float32)
        self.ctx._err(lib().sdd_cache_get_params(self.ctx.handle, self.handle, _ptr(a), a.size))
        return a

    def grads(self) -> np.ndarray:
        a = np.empty(self.n_param, dtype=np.float32)
        self.ctx._err(lib().sdd_cache_get_grads(self.ctx.handle, self.handle, _ptr(a), a.size))
        return a

    def eval(self, x, wo, mat, n_bins):
        """Network outputs [n][n_bins] for device tensors x, wo (float32 [n][3]) and mat (int32 [n])."""
        out = self.ctx.torch.empty((x.shape[0], n_bins), dtype=self.ctx.torch.float32, device=self.ctx.device)
        self.ctx._err(lib().sdd_cache_eval(self.ctx.handle, self.handle, C.c_void_p(x.data_ptr()),
                                           C.c_void_p(wo.data_ptr()), C.c_void_p(mat.data_ptr()), x.shape[0],
                                           int(n_bins), C.c_void_p(out.data_ptr())))
        self.ctx.finish()
        return out

    def backward(self, x, wo, mat, target):
        self.ctx._err(lib().sdd_cache_backward(self.ctx.handle, self.handle, C.c_void_p(x.data_ptr()),
                                               C.c_void_p(wo.data_ptr()), C.c_void_p(mat.data_ptr()),
                                               C.c_void_p(target.data_ptr()), x.shape[0], target.shape[1]))

    def step(self):
        self.ctx._err(lib().sdd_cache_step(self.ctx.handle, self.handle))

    def train(self, x, wo, mat, target):
        self.ctx._err(lib().sdd_cache_train(self.ctx.handle, self.handle, C.c_void_p(x.data_ptr()),
                                            C.c_void_p(wo.data_ptr()), C.c_void_p(mat.data_ptr()),
                                            C.c_void_p(target.data_ptr()), x.shape[0], target.shape[1]))

    def loss(self) -> float:
        d = C.c_double()
        self.ctx._err(lib().sdd_cache_loss(self.ctx.handle, self.handle, C.byref(d)))
        return d.value

    def records(self, n):
        """Training records of the last batch (slot order): rec_x [n][4], rec_w [n][4], target [n][max_bins]."""
        rx = np.empty((n, 4), dtype=np.float32)
        rw = np.empty((n, 4), dtype=np.float32)
        t = np.empty((n, self.cfg.max_bins), dtype=np.float32)
        self.ctx._err(lib().sdd_cache_get_records(self.ctx.handle, self.handle, int(n), _ptr(rx), _ptr(rw), _ptr(t)))
        return rx, rw, t

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.sdd_cache_destroy(self.handle)
            self.handle = None


class PhotonMap:
    """``sdd_photon_map`` bound to a torch device buffer."""

    def __init__(self, ctx: Context, scene: Scene, params: PhotonParams):
        torch = ctx.torch
        self.ctx, self.params, self.n_bins = ctx, params, scene.n_bins
        b = C.c_size_t()
        _check(lib().sdd_photon_map_bytes(scene.handle, C.byref(params), C.byref(b)))
        self.buffer = torch.empty(b.value + 256, dtype=torch.uint8, device=ctx.device)
        off = (-self.buffer.data_ptr()) % 256
        h = C.c_void_p()
        ctx._err(lib().sdd_photon_map_create(ctx.handle, scene.handle, C.byref(params),
                                             C.c_void_p(self.buffer.data_ptr() + off), b.value, C.byref(h)))
        self.handle = h

    def workspace_bytes(self, scene: Scene) -> int:
        b = C.c_size_t()
        _check(lib().sdd_photon_workspace_bytes(scene.handle, C.byref(self.params), C.byref(b)))
        return b.value

    def build(self, scene: Scene, finish=True):
        ws = self.ctx.workspace(self.workspace_bytes(scene))
        self.ctx._err(lib().sdd_photon_map_build(self.ctx.handle, scene.handle, self.handle,
                                                 C.c_void_p(ws.data_ptr()), ws.numel()))
        if finish:
            self.ctx.finish()

    def info(self) -> dict:
        i = PhotonInfo()
        self.ctx._err(lib().sdd_photon_map_info(self.ctx.handle, self.handle, C.byref(i)))
        return dict(stored=i.stored, dropped=i.dropped, n_windows=i.n_windows, n_buckets=i.n_buckets,
                    window_area=i.window_area, device_bytes=i.device_bytes)

    def records(self, n=None):
        """Stored records (any order): pos [n][3], dir [n][3], flux [n][n_bins], id [n], vertex [n]."""
        if n is None:
            n = self.info()["stored"]
        pos = np.empty((n, 3), dtype=np.float32)
        dr = np.empty((n, 3), dtype=np.float32)
        fl = np.empty((n, self.n_bins), dtype=np.float32)
        pid = np.empty(n, dtype=np.int64)
        vx = np.empty(n, dtype=np.int32)
        self.ctx._err(lib().sdd_photon_map_records(self.ctx.handle, self.handle, int(n), _ptr(pos), _ptr(dr),
                                                   _ptr(fl), _ptr(pid), _ptr(vx)))
        return pos, dr, fl, pid, vx

    def load(self, pos, dirs, flux, pid=None, vertex=None):
        """Replace the records with host arrays (pos [n][3], dirs [n][3], flux [n][n_bins] float32;
        pid int64 [n], vertex int32 [n] optional) and rebuild the grid."""
        pos = np.ascontiguousarray(pos, dtype=np.float32)
        dirs = np.ascontiguousarray(dirs, dtype=np.float32)
        flux = np.ascontiguousarray(flux, dtype=np.float32)
        assert flux.shape == (len(pos), self.n_bins) and dirs.shape == pos.shape == (len(pos), 3)
        pid = None if pid is None else np.ascontiguousarray(pid, dtype=np.int64)
        vertex = None if vertex is None else np.ascontiguousarray(vertex, dtype=np.int32)
        self.ctx._err(lib().sdd_photon_map_load(self.ctx.handle, self.handle, len(pos), _ptr(pos), _ptr(dirs),
                                                _ptr(flux), _ptr(pid), _ptr(vertex)))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.sdd_photon_map_destroy(self.handle)
            self.handle = None
