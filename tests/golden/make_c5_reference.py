"""Writes c5_reference.npz: the oracle's FP64-accumulated spectral radiance of the large church
view (9.9 M triangles, 200 windows, 3840x2160, 80 bins 380-780 nm, depth 8) on the pixel subset
x % 32 == 0 and y % 32 == 0 (120 x 68 = 8160 pixels), the reference against which the plain and
the cache-terminated renders of that view are scored by RMSE. Two independent halves of 1024
samples each (seeds 0xC5 and 0xC50, differing from every seed the renders use) give the mean and
an unbiased estimate of the mean's own noise: noise_var = mean((A - B)^2) / 4 over every pixel and
bin, which a score subtracts from a measured mean squared error. Calls only the oracle.

    python tests/golden/make_c5_reference.py [--threads N]
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

STRIDE, SPP_HALF, DEPTH, SEEDS = 32, 1024, 8, (0xC5, 0xC50)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    sc = scenegen.church_scene(n_bins=80, target_tris=10_000_000, n_bays=50, tiers=2)
    cam = scenegen.church_camera(3840, 2160)
    ys, xs = np.meshgrid(np.arange(0, cam.height, STRIDE), np.arange(0, cam.width, STRIDE), indexing="ij")
    px = (ys * cam.width + xs).ravel().astype(np.int64)
    t0 = time.time()
    halves = [oracle.render(sc, cam, spp=SPP_HALF, max_depth=DEPTH, seed=s, pixels=px, threads=a.threads).image
              for s in SEEDS]
    dt = time.time() - t0
    mean = 0.5 * (halves[0] + halves[1])
    noise_var = float(np.mean((halves[0] - halves[1]) ** 2) / 4.0)
    np.savez_compressed(os.path.join(HERE, "c5_reference.npz"), pixels=px, image=mean.astype(np.float32),
                        noise_var=noise_var, spp=2 * SPP_HALF, depth=DEPTH, seeds=np.array(SEEDS), stride=STRIDE,
                        width=cam.width, height=cam.height, n_bins=sc.n_bins, n_tri=sc.n_tri)
    print(f"{len(px)} pixels x {2 * SPP_HALF} spp in {dt:.0f} s with {a.threads} threads; "
          f"RMS of the reference's noise {np.sqrt(noise_var):.3e}")


if __name__ == "__main__":
    main()
