"""Pins of the oracle's training paths for the radiance cache (records and suffix targets)."""
import numpy as np

import oracle
import scenegen


def _paths(n=300, seed=5):
    sc = scenegen.nave_scene(8)
    cam = scenegen.nave_camera(width=48, height=32)
    rng = np.random.default_rng(seed)
    px = rng.integers(0, cam.width * cam.height, n)
    return sc, cam, px


def test_full_path_is_prefix_plus_throughput_times_suffix():
    """Path-space decomposition: with the same random numbers, a full-depth path's radiance equals
    what it gathers before its third vertex plus the throughput there times the radiance the
    training path gathers after restarting at that vertex."""
    sc, cam, px = _paths()
    g0, D = 1000, 8
    full = oracle.render(sc, cam, spp=1, max_depth=D, pixels=px, first_sample=g0, purpose=1 << 24,
                         sample_per_entry=True)
    pre = oracle.render(sc, cam, spp=1, max_depth=D, pixels=px, first_sample=g0, purpose=1 << 24,
                        sample_per_entry=True, cached=True)
    rec = oracle.training_records(sc, cam, px, g0, max_depth=D)
    q = pre.queries
    valid = q["valid"].astype(bool)
    assert valid.sum() > 100 and (~valid).sum() > 0
    np.testing.assert_array_equal(valid, rec["valid"])
    np.testing.assert_allclose(q["x"][valid], rec["x"][valid], rtol=0, atol=0)
    np.testing.assert_array_equal(q["mat"][valid], rec["mat"][valid])
    expect = pre.image.T + np.where(valid[:, None], q["beta"] * rec["target"], 0.0)
    np.testing.assert_allclose(full.image.T, expect, rtol=1e-12, atol=1e-14)
    # a path that never reached the vertex never restarted: what it gathered is the full radiance
    np.testing.assert_array_equal(rec["target"][~valid], full.image.T[~valid])


def test_purpose_changes_the_random_numbers():
    sc, cam, px = _paths(64)
    a = oracle.render(sc, cam, spp=1, max_depth=6, pixels=px, first_sample=7, sample_per_entry=True)
    b = oracle.render(sc, cam, spp=1, max_depth=6, pixels=px, first_sample=7, purpose=1 << 24,
                      sample_per_entry=True)
    assert not np.allclose(a.image, b.image)


def test_sample_per_entry_matches_single_pixel_renders():
    sc, cam, px = _paths(12)
    a = oracle.render(sc, cam, spp=1, max_depth=5, pixels=px, first_sample=40, sample_per_entry=True)
    for i, p in enumerate(px):
        b = oracle.render(sc, cam, spp=1, max_depth=5, pixels=[p], first_sample=40 + i)
        np.testing.assert_array_equal(a.image[:, i], b.image[:, 0])
