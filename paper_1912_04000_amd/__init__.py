"""specdd: spectral path tracing over a cell-decomposed triangle scene on one MI355X.

The compute path is libspecdd.so (hand-written HIP for gfx950 behind a C ABI, declared in
include/specdd.h); this package is its thin ctypes binding. PyTorch supplies device memory and
the stream only.
"""
from ._binding import (MODE_CACHED, MODE_PLAIN, Cache, CacheConfig, Camera, Context, Daylight, PhotonMap,
                       PhotonParams, RenderParams, Scene, SddError, TrainParams, cache_config, camera, daylight,
                       daylight_sun, lib, param_count, photon_params, render_params, train_params, PHOTON_CAUSTIC, PHOTON_GLOBAL)

__all__ = ["Scene", "Context", "Camera", "RenderParams", "SddError", "camera", "render_params", "lib",
           "MODE_PLAIN", "MODE_CACHED", "Cache", "CacheConfig", "TrainParams", "cache_config", "train_params",
           "param_count", "Daylight", "daylight", "daylight_sun", "PhotonMap", "PhotonParams", "photon_params",
           "PHOTON_CAUSTIC", "PHOTON_GLOBAL"]
