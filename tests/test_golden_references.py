"""The oracle's stored RMSE references (written by tests/golden/make_c4_reference.py and
make_c5_reference.py, which call only the oracle) have the layout the benchmark scores against:
the documented pixel subset in row-major order, every bin, the sample count and seeds, a finite
non-negative radiance, and a positive noise estimate from the two independent halves."""
import os

import numpy as np
import pytest

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("name,stride,width,height,bins,spp", [
    ("c4_reference.npz", 4, 1920, 1080, 40, 1024),
    ("c5_reference.npz", 32, 3840, 2160, 80, 2048)])
def test_reference_layout(name, stride, width, height, bins, spp):
    f = np.load(os.path.join(HERE, name))
    assert int(f["stride"]) == stride and int(f["width"]) == width and int(f["height"]) == height
    assert int(f["n_bins"]) == bins and int(f["spp"]) == spp and int(f["depth"]) == 8
    ys, xs = np.meshgrid(np.arange(0, height, stride), np.arange(0, width, stride), indexing="ij")
    assert np.array_equal(f["pixels"], (ys * width + xs).ravel())
    img = f["image"]
    assert img.shape == (bins, len(f["pixels"])) and img.dtype == np.float32
    assert np.all(np.isfinite(img)) and img.min() >= 0.0 and img.max() > 0.0
    nv = float(f["noise_var"])
    # the halves' difference estimates the mean's noise: positive, and below a tenth of the
    # signal's power (the large view is dark: its reference noise is 22 % of the RMS radiance)
    assert 0.0 < nv < 0.1 * float(np.mean(img.astype(np.float64) ** 2))
    assert len(f["seeds"]) == 2 and f["seeds"][0] != f["seeds"][1]
