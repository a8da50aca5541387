"""Writes c4_reference.npz: the oracle's FP64-accumulated 1024-spp spectral radiance of the
church-1M view (1920x1080, 40 bins 380-780 nm, depth 8) on the pixel subset x % 16 == 0 and
y % 16 == 0 (120 x 68 = 8160 pixels), the reference against which the plain and the
cache-terminated renders are scored by RMSE. Calls only the oracle; the seed (0xC4) differs from
every seed the renders use, so the reference noise is independent of theirs.

    python tests/golden/make_c4_reference.py [--threads N]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import scenegen  # noqa: E402

STRIDE, SPP, DEPTH, SEED = 16, 1024, 8, 0xC4


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    sc = scenegen.church_scene(40)
    cam = scenegen.church_camera()
    ys, xs = np.meshgrid(np.arange(0, cam.height, STRIDE), np.arange(0, cam.width, STRIDE), indexing="ij")
    px = (ys * cam.width + xs).ravel().astype(np.int64)
    t0 = time.time()
    r = oracle.render(sc, cam, spp=SPP, max_depth=DEPTH, seed=SEED, pixels=px, threads=a.threads)
    dt = time.time() - t0
    np.savez_compressed(os.path.join(HERE, "c4_reference.npz"), pixels=px, image=r.image.astype(np.float32),
                        spp=SPP, depth=DEPTH, seed=SEED, stride=STRIDE, width=cam.width, height=cam.height,
                        n_bins=sc.n_bins)
    print(f"{len(px)} pixels x {SPP} spp in {dt:.0f} s with {a.threads} threads")


if __name__ == "__main__":
    main()
