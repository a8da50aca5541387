"""Writes c4_reference.npz: the oracle's FP64-accumulated 1024-spp spectral radiance of the
church-1M view (1920x1080, 40 bins 380-780 nm, depth 8) on the pixel subset x % 4 == 0 and
y % 4 == 0 (480 x 270 = 129,600 pixels), the reference against which the plain and the
cache-terminated renders are scored by RMSE. Two independent halves of 512 samples each (seeds
0xC4 and 0xC40, differing from every seed the renders use) give the mean and an unbiased
estimate of the mean's own noise: noise_var = mean((A - B)^2) / 4 over every pixel and bin, which
a score subtracts from a measured mean squared error. Calls only the oracle.

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

STRIDE, SPP_HALF, DEPTH, SEEDS = 4, 512, 8, (0xC4, 0xC40)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    sc = scenegen.church_scene(40)
    cam = scenegen.church_camera()
    ys, xs = np.meshgrid(np.arange(0, cam.height, STRIDE), np.arange(0, cam.width, STRIDE), indexing="ij")
    px = (ys * cam.width + xs).ravel().astype(np.int64)
    t0 = time.time()
    halves = [oracle.render(sc, cam, spp=SPP_HALF, max_depth=DEPTH, seed=s, pixels=px, threads=a.threads).image
              for s in SEEDS]
    dt = time.time() - t0
    mean = 0.5 * (halves[0] + halves[1])
    noise_var = float(np.mean((halves[0] - halves[1]) ** 2) / 4.0)
    np.savez_compressed(os.path.join(HERE, "c4_reference.npz"), pixels=px, image=mean.astype(np.float32),
                        noise_var=noise_var, spp=2 * SPP_HALF, depth=DEPTH, seeds=np.array(SEEDS), stride=STRIDE,
                        width=cam.width, height=cam.height, n_bins=sc.n_bins)
    print(f"{len(px)} pixels x {2 * SPP_HALF} spp in {dt:.0f} s with {a.threads} threads; "
          f"RMS of the reference's noise {np.sqrt(noise_var):.3e}")


if __name__ == "__main__":
    main()
