"""Host side of the caustic photon map (no GPU): parameter validation and the map's buffer size."""
import ctypes as C

import pytest

import paper_1912_04000_amd as sd
import scenegen
from paper_1912_04000_amd import _binding


def _bytes(S, p):
    b = C.c_size_t()
    rc = _binding.lib().sdd_photon_map_bytes(S.handle, C.byref(p), C.byref(b))
    return rc, b.value


@pytest.mark.parametrize("field,value", [("n_photons", 0), ("max_depth", 1), ("max_depth", 65), ("radius", 0.0),
                                         ("radius", float("inf")), ("capacity", 0), ("capacity", (1 << 28) + 1),
                                         ("wave_paths", 63), ("queue_rounds", -1)])
def test_photon_params_validation(field, value):
    S = sd.Scene.from_description(scenegen.caustic_scene(3))
    p = sd.photon_params(1000, radius=0.1)
    setattr(p, field, value)
    rc, _ = _bytes(S, p)
    assert rc == -1


def test_photon_count_bound():
    """Stored-record counters are 32-bit: n_photons (max_depth - 1) must stay below 2^32."""
    S = sd.Scene.from_description(scenegen.caustic_scene(3))
    assert _bytes(S, sd.photon_params(1 << 28, radius=0.1, max_depth=17, capacity=1000))[0] == -1
    assert _bytes(S, sd.photon_params(1 << 28, radius=0.1, max_depth=16, capacity=1000))[0] == 0


def test_map_bytes_grow_with_capacity_and_bins():
    S3 = sd.Scene.from_description(scenegen.caustic_scene(3))
    S40 = sd.Scene.from_description(scenegen.caustic_scene(40))
    _, a = _bytes(S3, sd.photon_params(1000, radius=0.1, capacity=10_000))
    _, b = _bytes(S3, sd.photon_params(1000, radius=0.1, capacity=20_000))
    _, c = _bytes(S40, sd.photon_params(1000, radius=0.1, capacity=10_000))
    # a record is (position, direction, flux quads): 48 bytes at 3 bins, 192 at 40; plus its index
    assert 10_000 * 52 <= a and b - a >= 10_000 * 52 and c - a >= 10_000 * 144
    ws = C.c_size_t()
    assert _binding.lib().sdd_photon_workspace_bytes(S3.handle, C.byref(sd.photon_params(1000, radius=0.1)),
                                                     C.byref(ws)) == 0
    assert ws.value > 0


def test_photon_kind_validation():
    S = sd.Scene.from_description(scenegen.caustic_scene(3))
    assert _bytes(S, sd.photon_params(1000, radius=0.1, kind=sd.PHOTON_GLOBAL))[0] == 0
    assert _bytes(S, sd.photon_params(1000, radius=0.1, kind=2))[0] == -1
