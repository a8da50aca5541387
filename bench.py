#!/usr/bin/env python
"""Benchmark of the spectral path tracer on one MI355X.

Workload (default): the seeded procedural church of 979,664 triangles (40 coloured glass windows),
1920x1080 pixels, 40 wavelength bins over 380-780 nm, 64 samples per pixel, 8 surface vertices
per path, 8x4x4 cells, 2^25 paths in flight. One step = one full plain frame (132.7 M spectral
path samples, each carrying all 40 bins); `value` is the plain path's samples/s. The same line
carries `equal_rmse`: the cache-terminated path on the same view (untrained cache, eight 1-spp
online-training frames, then a 64-spp frame, all timed) scored against the oracle's 1024-spp
reference, with the plain time to reach the same RMSE. Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload church|nave|batch|cached] [--no-cpu-baseline]
                  [--no-cached]
  python bench.py --copy-calibration 1.0   # a plain 1 GiB device copy (for PMC byte scaling)
  python bench.py --pmc-summary F.csv W.csv CF.csv CW.csv   # HBM bytes of k_trace from rocprofv3 --pmc
      (FETCH_SIZE and WRITE_SIZE runs of this bench, then of --copy-calibration; writes
       profiles/k_trace_church1M_pmc.json, which later bench lines report as roofline.traffic)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spectral path samples/s on 1 GPU, plain vs MLP-cached at equal RMSE; HBM GB/s"
HBM_PEAK_GBPS = 8000.0
# Non-packed FP32 VALU issue rate of MI355X: 256 CUs x 64 lanes x 2.4 GHz (ops/s, 1 op = 1 flop).
# The 157.3 TFLOP/s vector figure counts an FMA as 2 flops on packed (2-wide) lanes.
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
BF16_PEAK_TFLOPS = 2500.0   # dense bf16 matrix-core peak of MI355X
# Algorithmic VALU operations per unit of traversal work (counted from the kernel source):
OPS_PER_NODE = 104      # four robust slab tests (6 sub, 6 mul, 12 min/max, 1 slop mul, 1 cmp each)
OPS_PER_TRI = 56        # watertight test: translate, shear, 3 edge functions, signs, det, t, u, v


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="church", choices=["church", "nave", "batch", "cached", "large"])
    ap.add_argument("--cached-spp", type=int, default=64, help="cached workload: samples per pixel of the scored frame")
    ap.add_argument("--warm-frames", type=int, default=8, help="cached workload: 1-spp training frames before it")
    ap.add_argument("--train-paths", type=int, default=1 << 17, help="cached workload: training paths per batch")
    ap.add_argument("--train-steps", type=int, default=None,
                    help="cached and large workloads: Adam steps of 2^14 records per batch (default 4 / 8)")
    ap.add_argument("--cache-lr", type=float, default=None,
                    help="cached and large workloads: Adam learning rate (default 1e-3 / 3e-3)")
    ap.add_argument("--cache-log2-pos", type=int, default=None,
                    help="cached and large workloads: log2 entries per level of the position grid (default 19 / 21)")
    ap.add_argument("--train-every", type=int, default=0,
                    help="cached path: wavefronts between training batches (0: one batch per frame)")
    ap.add_argument("--tune-cache", default=os.path.join(os.path.expanduser("~"), ".cache", "specdd",
                                                          "tune_cache.json"))
    ap.add_argument("--spp", type=int, default=None, help="override samples per pixel (profiling runs)")
    ap.add_argument("--wave-paths", type=int, default=1 << 25,
                    help="paths per wavefront (church frame: 1046 / 925 / 889 / 838 / 821 ms at 2^21 .. 2^25)")
    ap.add_argument("--queue-rounds", type=int, default=0)
    ap.add_argument("--persistent", type=int, default=0, choices=[0, 1],
                    help="church/nave workloads: render with the one persistent kernel instead of the wavefronts")
    ap.add_argument("--cell-order", type=int, default=1, choices=[0, 1],
                    help="tile order of the traversal: 0 cell index, 1 fullest cells first")
    ap.add_argument("--large-train-frames", type=int, default=0,
                    help="large workload: frames trained one batch each before the period applies (0: every frame)")
    ap.add_argument("--large-train-period", type=int, default=1,
                    help="large workload: after those frames, one training batch every this many frames")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cached", action="store_true", help="skip the cached-path comparison of the default run")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the colorimetry, glass-map and photon-map measurements (profiling runs of the "
                         "frame alone)")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="GiB: only run a plain device-to-device copy of that size (PMC calibration)")
    ap.add_argument("--pmc-summary", nargs=4, default=None, metavar="CSV",
                    help="counter_collection.csv of FETCH_SIZE, WRITE_SIZE (bench), FETCH_SIZE, WRITE_SIZE (copy)")
    ap.add_argument("--pmc-command", default="", help="the rocprofv3 command lines, recorded in the summary")
    return ap.parse_args()


def workload(name, spp_override):
    import scenegen
    if name == "church":
        sc = scenegen.church_scene(40)
        cam = scenegen.church_camera()
        cfg = dict(spp=64, max_depth=8, grid=(8, 4, 4))
        label = "church-1M plain: 1920x1080, 40 bins 380-780 nm, 64 spp, depth 8, 8x4x4 cells"
    else:
        sc = scenegen.nave_scene(8)
        cam = scenegen.nave_camera()
        cfg = dict(spp=1, max_depth=4, grid=(2, 2, 2))
        label = "nave-1.75k plain: 64x64, 8 bins 380-780 nm, 1 spp, depth 4, 2x2x2 cells"
    if spp_override:
        cfg["spp"] = spp_override
        label += f" (spp overridden to {spp_override})"
    return sc, cam, cfg, label


# Record sizes of the wavefront design: ray R = 32 B, hit H = 16 B, queue entry Q = 4 B.
REC_R, REC_H, REC_Q = 32, 16, 4
# Algorithmic bytes of one cell visit of a ray: the ray record read, its queue entry written by
# the scatter and read by the traversal.
BYTES_PER_CELL_VISIT = REC_R + 2 * REC_Q


def path_bytes(st, B):
    """Algorithmic HBM bytes of the whole path, from the device counters: per path the camera
    ray R and the throughput initialisation S, then the image read-modify-write 2 S; per vertex
    the extension and shadow rays written (2 R), the hit record written and read (2 H) and the
    spectral state 6 S (throughput, direct-term weight and gathered radiance, each read and
    written); per cell visit of any ray 40 B (ray read, queue entry written and read). S = 4 B
    per bin. This is R + 3 S + V (2 R + 2 H + 6 S) + 40 visits per path, the cell visits
    counted instead of assumed (2 + mean migrations per vertex)."""
    S = 4 * B
    return (st["paths"] * (REC_R + 3 * S) + st["vertices"] * (2 * REC_R + 2 * REC_H + 6 * S)
            + st["cell_visits"] * BYTES_PER_CELL_VISIT)


def trace_bytes(st):
    """Algorithmic HBM bytes of the traversal kernel: 40 B per cell visit and the 16 B hit record
    every extension ray writes (hit or miss)."""
    return st["cell_visits"] * BYTES_PER_CELL_VISIT + st["ext_rays"] * REC_H


def _oracle_rate(sc, cam, spp, depth, px, threads):
    """Spectral path samples/s of the oracle on a pixel list, its fixed per-call cost (the FP64
    BVH build over the scene) measured on a one-pixel call and subtracted."""
    import oracle
    t0 = time.perf_counter()
    oracle.render(sc, cam, spp=1, max_depth=depth, seed=1, pixels=px[:1], threads=threads)
    fixed = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = oracle.render(sc, cam, spp=spp, max_depth=depth, seed=1, pixels=px, threads=threads)
    dt = max(time.perf_counter() - t0 - fixed, 1e-9)
    n = len(px) * spp
    return n / dt, dt, fixed, r.stats["vertices"] / n


def cpu_baseline(sc, cam, cfg, threads):
    """The oracle as it stands, timed on the host: all-core (`threads` workers over pixel rows,
    the paper's static image-space partition) on the pixel subset x % 4 == 0, y % 4 == 0 at 8 spp
    of the same frame, single-thread on the subset x % 8 == 0, y % 8 == 0 at 1 spp, and the small
    64 x 64 nave frame (8 bins, 1 spp, depth 4) in full, single-thread and all-core."""
    import scenegen
    ys, xs = np.meshgrid(np.arange(0, cam.height, 4), np.arange(0, cam.width, 4), indexing="ij")
    px4 = (ys * cam.width + xs).ravel()
    ys, xs = np.meshgrid(np.arange(0, cam.height, 8), np.arange(0, cam.width, 8), indexing="ij")
    px8 = (ys * cam.width + xs).ravel()
    spp = min(8, cfg["spp"])
    D = cfg["max_depth"]
    rate, dt, fixed, vpp = _oracle_rate(sc, cam, spp, D, px4, threads)
    rate1, dt1, _, _ = _oracle_rate(sc, cam, 1, D, px8, 1)
    nave, ncam = scenegen.nave_scene(8), scenegen.nave_camera()
    allpx = np.arange(ncam.width * ncam.height)
    c1_all, _, _, _ = _oracle_rate(nave, ncam, 1, 4, allpx, threads)
    c1_one, _, _, _ = _oracle_rate(nave, ncam, 1, 4, allpx, 1)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"value": rate, "unit": "spectral path samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(px4)} pixels (every 4th row and column) x {spp} spp of the same frame, "
                      f"{len(px4) * spp} paths in {dt:.1f} s on {threads} threads (+{fixed:.1f} s BVH build "
                      f"excluded), FP64",
            "nproc": os.cpu_count(), "affinity_cpus": affinity,
            "single_thread": {"value": rate1, "sample": f"{len(px8)} pixels (every 8th row and column) x 1 spp, "
                                                          f"{len(px8)} paths in {dt1:.1f} s"},
            "nave_64x64_full_frame": {"all_core": c1_all, "single_thread": c1_one,
                                      "sample": "64x64 nave, 8 bins, 1 spp, depth 4, whole frame"},
            "vertices_per_path": vpp}


def traffic_from_profiles(kernel_src_hash):
    """HBM bytes per k_trace launch from the committed PMC summary, if it was taken on the
    current kernel source."""
    p = os.path.join(ROOT, "profiles", "k_trace_church1M_pmc.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_sha256") != kernel_src_hash:
        return None
    return d.get("hbm_bytes_per_launch")


def copy_calibration(gib):
    import torch
    n = int(gib * (1 << 30)) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 4, "copy_calibration_bytes_written": n * 4, "launches": 3}))


def _pmc_per_kernel(path, counter):
    """Mean counter value (KiB per dispatch) and dispatch count per kernel name."""
    import csv
    acc = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        k = r["Kernel_Name"].split("(")[0].strip()
        if k.startswith("void "):
            k = k[5:]
        v = acc.setdefault(k, [0.0, 0])
        v[0] += float(r["Counter_Value"])
        v[1] += 1
    return {k: (v[0] / v[1], v[1]) for k, v in acc.items()}


def pmc_summary(args):
    """HBM bytes per k_trace launch: FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by
    what the same counter reads for a plain device copy of known size."""
    f_csv, w_csv, cf_csv, cw_csv = args.pmc_summary
    copy_bytes = 3 * (1 << 30)  # three 1 GiB copies (bench.py --copy-calibration 1)
    cf = _pmc_per_kernel(cf_csv, "FETCH_SIZE")["__amd_rocclr_copyBuffer"]
    cw = _pmc_per_kernel(cw_csv, "WRITE_SIZE")["__amd_rocclr_copyBuffer"]
    f_scale = copy_bytes / (cf[0] * cf[1] * 1024)
    w_scale = copy_bytes / (cw[0] * cw[1] * 1024)
    fk = _pmc_per_kernel(f_csv, "FETCH_SIZE")
    wk = _pmc_per_kernel(w_csv, "WRITE_SIZE")
    kernels = {}
    for k in sorted(set(fk) & set(wk)):
        if not k.startswith("sdd::"):
            continue
        rd = fk[k][0] * 1024 * f_scale
        wr = wk[k][0] * 1024 * w_scale
        kernels[k] = {"dispatches": fk[k][1], "fetch_kib_raw": fk[k][0], "write_kib_raw": wk[k][0],
                      "read_bytes": rd, "write_bytes": wr, "hbm_bytes_per_launch": rd + wr}
    src = open(os.path.join(ROOT, "paper_1912_04000_amd", "csrc", "kernels.hip"), "rb").read()
    out = {"kernel": "sdd::k_trace", "kernel_source_sha256": hashlib.sha256(src).hexdigest(),
           "hbm_bytes_per_launch": kernels["sdd::k_trace"]["hbm_bytes_per_launch"],
           "fetch_scale": f_scale, "write_scale": w_scale,
           "calibration": "FETCH_SIZE / WRITE_SIZE of three 1 GiB torch device copies "
                          "(__amd_rocclr_copyBuffer) against their known 3 GiB read and written",
           "command": args.pmc_command, "kernels": kernels}
    p = os.path.join(ROOT, "profiles", "k_trace_church1M_pmc.json")
    os.makedirs(os.path.dirname(p), exist_ok=True)
    with open(p, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({k: round(v["hbm_bytes_per_launch"] / 1e6, 3) for k, v in kernels.items()}))


_REF_NOISE_VAR = 0.0   # noise variance of the loaded reference's mean (subtracted from every MSE)


def _rmse(img, ref, px):
    """RMSE over (subset pixel, bin) of an image [B][H][W] against the reference [B][n], with the
    reference's own noise variance (estimated from its two independent halves) subtracted."""
    B = ref.shape[0]
    sub = img.reshape(B, -1)[:, px]
    return float(np.sqrt(max(np.mean((sub.astype(np.float64) - ref) ** 2) - _REF_NOISE_VAR, 0.0)))


def load_reference():
    """The oracle's reference of the church view for the cached comparison
    (tests/golden/c4_reference.npz): pixel indices, the mean image [B][n] of its two halves, and
    their noise variance, which _rmse subtracts from then on."""
    global _REF_NOISE_VAR
    ref_f = np.load(os.path.join(ROOT, "tests", "golden", "c4_reference.npz"))
    _REF_NOISE_VAR = float(ref_f["noise_var"]) if "noise_var" in ref_f.files else 0.0
    return ref_f["pixels"], ref_f["image"].astype(np.float64)


def reference_note():
    ref_f = np.load(os.path.join(ROOT, "tests", "golden", "c4_reference.npz"))
    st = int(ref_f["stride"])
    return (f"oracle FP64 {int(ref_f['spp'])} spp, pixels x%{st}==0 and y%{st}==0 ({len(ref_f['pixels'])}), "
            f"its noise variance {float(ref_f['noise_var']) if 'noise_var' in ref_f.files else 0.0:.3e} subtracted")


def plain_curve(ctx, S, c, img, px, ref, wave, spps, W, H):
    """Plain frames (seed 1) at each spp, their RMSE against the reference, and the least-squares
    fit RMSE = a / sqrt(spp) with the log-log slope (-0.5 for an unbiased estimator)."""
    import paper_1912_04000_amd as sd
    plain = []
    for spp in spps:
        dt = _timed(lambda: ctx.render(S, c, sd.render_params(spp=spp, max_depth=8, seed=1, wave_paths=wave,
                                                              cell_order=1), out=img))
        plain.append(dict(spp=spp, seconds=dt, rmse=_rmse(img.cpu().numpy(), ref, px)))
    sp = np.array([q["spp"] for q in plain], dtype=np.float64)
    rm = np.array([q["rmse"] for q in plain])
    a = float(np.sum(rm * sp ** -0.5) / np.sum(1.0 / sp))   # least squares of rmse = a spp^-1/2
    slope = float(np.polyfit(np.log(sp), np.log(np.maximum(rm, 1e-30)), 1)[0])
    return plain, a, slope


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def run_cached(ctx, S, sc, cam, img, args, px, ref, wave):
    """The cache-terminated path on the church view: an untrained cache, warm_frames 1-spp frames,
    then one scored frame of cached_spp samples, all timed; every frame (render call) trains the
    cache once on 2^16 records (--train-every 0). Then the scored frame again with training off
    (inference-only throughput, the steady state of a converged cache)."""
    import paper_1912_04000_amd as sd
    B, W, H = sc.n_bins, cam.width, cam.height
    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, W, H)
    lo = sc.verts.reshape(-1, 3).min(0) - 0.05
    hi = sc.verts.reshape(-1, 3).max(0) + 0.05
    cache = sd.Cache(ctx, sd.cache_config(len(sc.mat_type), lo, hi, max_bins=B,
                                          max_records=max(args.train_paths, 1 << 14), max_step=1 << 14,
                                          lr=args.cache_lr or 1e-3, log2_table_pos=args.cache_log2_pos or 19),
                     seed=12345)
    tp = sd.train_params(train_paths=args.train_paths, step_records=1 << 14, steps=args.train_steps or 4,
                         every=args.train_every)
    ctx.reset_stats()
    frames, t_total = [], 0.0
    for f in range(args.warm_frames):
        dt = _timed(lambda: ctx.render_cached(S, cache, c, sd.render_params(spp=1, max_depth=8, seed=1000 + f,
                                                                           mode=sd.MODE_CACHED, wave_paths=wave),
                                              tp, out=img))
        t_total += dt
        frames.append(dict(frame=f, spp=1, seconds=dt, rmse=_rmse(img.cpu().numpy(), ref, px)))
    n_spp = args.cached_spp
    ctx.finish()
    ctx.reset_stats()   # the statistics below cover the scored frame only
    p = sd.render_params(spp=n_spp, max_depth=8, seed=1, mode=sd.MODE_CACHED, wave_paths=wave, timing=1)
    dt = _timed(lambda: ctx.render_cached(S, cache, c, p, tp, out=img))
    t_total += dt
    r_c = _rmse(img.cpu().numpy(), ref, px)
    frames.append(dict(frame=args.warm_frames, spp=n_spp, seconds=dt, rmse=r_c))
    st = ctx.stats()
    dt_inf = _timed(lambda: ctx.render_cached(S, cache, c, sd.render_params(spp=n_spp, max_depth=8, seed=1,
                                                                             mode=sd.MODE_CACHED, wave_paths=wave),
                                              None, out=img))
    r_inf = _rmse(img.cpu().numpy(), ref, px)
    # matrix-core roofline of the query kernel in the scored frame: MFMA flops per queried vertex
    # = 2*64*64 (z = W0 e) + B * 3 * 2*64*64 (three 64x64 layers per bin)
    flops = st["cache_queries"] * (2 * 64 * 64 + B * 3 * 2 * 64 * 64)
    q_s = st["query_ms"] / 1e3
    achieved = flops / q_s / 1e12 if q_s > 0 else 0.0
    roof = {"kernel": "k_cache_query", "bound": "mfma", "achieved": achieved, "peak": BF16_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / BF16_PEAK_TFLOPS, "launches": st["query_launches"],
            "avg_launch_ms": st["query_ms"] / max(1, st["query_launches"]),
            "queries_per_launch": st["cache_queries"] / max(1, st["query_launches"]),
            "note": "algorithmic MFMA flops (2*64*64 per vertex + 3*2*64*64 per vertex and bin) of the scored "
                    "frame's queries over the HIP-event time of its query launches; peak = bf16 dense"}
    return dict(rmse=r_c, seconds=t_total, frames=frames, inference_rmse=r_inf, inference_seconds=dt_inf,
                spp=n_spp, adam_steps=cache.info()["adam_steps"], train_ms=st["train_ms"],
                train_batches=st["train_batches"], cache_queries=st["cache_queries"], roofline=roof)


def equal_rmse(cached, a, plain_rate, W, H, warm_frames):
    """Plain spp that reaches the cached frame's RMSE under RMSE = a / sqrt(spp), and the times."""
    spp_eq = (a / cached["rmse"]) ** 2
    t_plain = W * H * spp_eq / plain_rate
    return {"rmse_cached": cached["rmse"], "plain_fit_a": a, "spp_plain_equivalent": spp_eq,
            "time_cached_s": cached["seconds"], "time_plain_equivalent_s": t_plain,
            "speedup": t_plain / cached["seconds"],
            "plain_equivalent_samples_per_s": W * H * spp_eq / cached["seconds"],
            "cached_samples_per_s": W * H * (cached["spp"] + warm_frames) / cached["seconds"],
            "plain_samples_per_s": plain_rate,
            "rmse_cached_inference_only": cached["inference_rmse"],
            "inference_only_frame_s": cached["inference_seconds"],
            "adam_steps": cached["adam_steps"], "train_ms": cached["train_ms"],
            "train_batches": cached["train_batches"], "cache_roofline": cached["roofline"]}


def bench_cached(args):
    """Equal-RMSE comparison of the plain full-depth path and the cache-terminated path on the
    church-1M view (1920x1080, 40 bins, depth 8). Both are scored by RMSE against the
    oracle's FP64 1024-spp reference on the pixel subset x % 4 == 0, y % 4 == 0
    (tests/golden/c4_reference.npz, its own noise variance subtracted). Plain: RMSE at spp = 1 .. 256 gives the least-squares fit
    RMSE = a / sqrt(spp) and the frame rate. Cached: the cache starts untrained and is trained
    online once per frame (2^16 records, 4 Adam steps of 2^14, lr 1e-3) during warm_frames 1-spp
    frames and the scored frame; the time of every warm-up and scored frame counts.
    value = W H spp_eq / time_cached, with spp_eq = (a / RMSE_cached)^2 the plain samples per
    pixel that reach the cached frame's RMSE: plain-equivalent samples per second."""
    import torch
    import paper_1912_04000_amd as sd
    import scenegen
    px, ref = load_reference()
    sc = scenegen.church_scene(40)
    cam = scenegen.church_camera()
    B, W, H = sc.n_bins, cam.width, cam.height
    ctx = sd.Context(0)
    S = sd.Scene.from_description(sc, grid=(8, 4, 4))
    ctx.upload(S)
    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, W, H)
    img = torch.empty((B, H, W), dtype=torch.float32, device="cuda")
    wave = args.wave_paths
    ctx.render(S, c, sd.render_params(spp=1, max_depth=8, seed=1, wave_paths=wave), out=img)  # warm-up
    plain, a, slope = plain_curve(ctx, S, c, img, px, ref, wave, (1, 2, 4, 8, 16, 32, 64, 128, 256), W, H)
    plain_rate = W * H * 64 / [q for q in plain if q["spp"] == 64][0]["seconds"]
    cached = run_cached(ctx, S, sc, cam, img, args, px, ref, wave)
    eq = equal_rmse(cached, a, plain_rate, W, H, args.warm_frames)
    out = {
        "metric": METRIC, "value": eq["plain_equivalent_samples_per_s"],
        "unit": "plain-equivalent spectral path samples/s", "n_gpus": 1,
        "steps": 1, "warmup": args.warm_frames, "ms_per_step": cached["seconds"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16 (cache MLP) / f32 (tracer)",
        "data": f"synthetic (seeded procedural scene, {sc.n_tri} triangles)",
        "config": {"workload": "church-1M cached vs plain at equal RMSE: 1920x1080, 40 bins, depth 8, cache at vertex 3, "
                               f"{args.warm_frames} 1-spp warm-up frames + one {args.cached_spp}-spp frame, "
                               "online training once per frame",
                   "reference": reference_note(),
                   "train_paths_per_batch": args.train_paths, "train_every": args.train_every,
                   "records_per_batch": 4 << 14},
        "equal_rmse": eq, "plain_curve": plain, "plain_loglog_slope": slope, "cached_frames": cached["frames"],
    }
    print(json.dumps(out), flush=True)


def bench_colorimetry(ctx, img, sc, reps=20):
    """The frame's colour image (spectral -> CIE XYZ -> sRGB, one HBM pass): HIP-event time of
    `reps` launches on the library stream, against the algorithmic bytes per launch (the B
    planes read, 3 XYZ planes and the 3-channel sRGB image written)."""
    import torch
    B, H, W = img.shape
    xyz = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
    rgb = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    run = lambda: ctx.spectral_to_srgb(img, sc.lambda_min_nm, sc.lambda_max_nm, 1.0, finish=False, xyz_out=xyz,
                                       srgb_out=rgb)
    run()
    ctx.finish()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        run()
    e1.record()
    torch.cuda.synchronize()
    ctx.finish()
    ms = e0.elapsed_time(e1) / reps
    nbytes = H * W * (4 * B + 12 + 12)
    gbps = nbytes / (ms * 1e-3) / 1e9
    return {"kernel": "k_spectral_to_srgb", "bound": "hbm", "avg_launch_ms": ms, "achieved": gbps,
            "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS,
            "algorithmic_bytes_per_launch": nbytes, "launches": reps,
            "note": "per pixel 4 B x bins read, 12 B XYZ and 12 B sRGB written; HIP events on the library stream"}


def bench_glass_maps(ctx, sc, cam, cfg, wave, spp=8):
    """The same church with a seeded spectral transmittance map on each window (glass absorbing
    by the map at the hit's texture coordinates instead of by k): samples/s of an spp-sample frame
    against the plain scene at the same spp, HIP-event timed on the library stream."""
    import torch
    import paper_1912_04000_amd as sd
    import scenegen
    st = scenegen.with_glass_maps(sc)
    S = sd.Scene.from_description(st, grid=cfg["grid"])
    ctx.upload(S)
    S0 = sd.Scene.from_description(sc, grid=cfg["grid"])
    ctx.upload(S0)
    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height)
    img = torch.empty((sc.n_bins, cam.height, cam.width), dtype=torch.float32, device="cuda")
    p = sd.render_params(spp=spp, max_depth=cfg["max_depth"], seed=1, wave_paths=wave)
    out = {}
    for name, scene in (("maps", S), ("plain", S0)):
        ctx.render(scene, c, p, out=img)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.render(scene, c, p, out=img, finish=False)
        e1.record()
        torch.cuda.synchronize()
        ctx.finish()
        out[name] = cam.width * cam.height * spp / (e0.elapsed_time(e1) * 1e-3)
    return {"samples_per_s": out["maps"], "plain_samples_per_s_same_spp": out["plain"],
            "relative_cost": out["plain"] / out["maps"], "spp": spp,
            "maps": f"{len(st.textures)} maps of {st.textures[0].shape[1]}x{st.textures[0].shape[0]} texels x "
                    f"{sc.n_bins} bins"}


def bench_photons(ctx, S, sc, cam, cfg, wave, n_photons=4_000_000, radius=0.1, spp=8):
    """Caustic photon map (section 4) of the benchmarked view: HIP-event time of building an
    n_photons map (emission through the windows, photon paths through the cell queues, storage,
    hashed-grid sort), then of an spp-sample frame that gathers from it at every shaded opaque
    vertex against the same frame without it. Gather roofline: algorithmic bytes from the device
    counters (per gathering vertex its list entry, hit, ray and triangle, 100 B; per vertex that
    found a record its throughput row read and radiance row read and written, 12 Bp B; per record
    found its grid entry, direction and flux row, 32 + 4 Bp B; grid bounds and the entries tested
    outside the ball are search overhead, not counted) over the HIP-event time of the gather
    launches (both passes)."""
    import torch
    import paper_1912_04000_amd as sd
    Bp = (sc.n_bins + 3) // 4 * 4
    pp = sd.photon_params(n_photons, radius=radius, max_depth=cfg["max_depth"], seed=1, capacity=n_photons // 4)
    m = sd.PhotonMap(ctx, S, pp)
    m.build(S)                                   # first touch of the map and the workspace
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    m.build(S, finish=False)
    e1.record()
    torch.cuda.synchronize()
    ctx.finish()
    build_ms = e0.elapsed_time(e1)
    info = m.info()
    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height)
    img = torch.empty((sc.n_bins, cam.height, cam.width), dtype=torch.float32, device="cuda")
    p = sd.render_params(spp=spp, max_depth=cfg["max_depth"], seed=1, wave_paths=wave, timing=1)
    rate, st = {}, None
    for name in ("photons", "plain"):
        run = ((lambda: ctx.render_photons(S, m, c, p, out=img, finish=False)) if name == "photons" else
               (lambda: ctx.render(S, c, p, out=img, finish=False)))
        run()
        ctx.finish()
        ctx.reset_stats()
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        ctx.finish()
        rate[name] = cam.width * cam.height * spp / (e0.elapsed_time(e1) * 1e-3)
        if name == "photons":
            st = ctx.stats()
    launches = max(1, st["photon_launches"])
    alg = (st["photon_vertices"] * 100 + st["photon_lit_vertices"] * 12 * Bp
           + st["photons_found"] * (32 + 4 * Bp))
    gbps = alg / (st["photon_ms"] * 1e-3) / 1e9 if st["photon_ms"] > 0 else 0.0
    return {"photons": n_photons, "radius_m": radius, "max_depth": cfg["max_depth"],
            "build_ms": build_ms, "photons_per_s": n_photons / (build_ms * 1e-3),
            "records": info["stored"], "dropped": info["dropped"], "windows": info["n_windows"],
            "spp": spp, "samples_per_s": rate["photons"], "plain_samples_per_s_same_spp": rate["plain"],
            "relative_cost": rate["plain"] / rate["photons"],
            "gather": {"kernel": "k_photon_gather", "bound": "hbm", "launches": st["photon_launches"],
                       "avg_launch_ms": st["photon_ms"] / launches, "achieved": gbps, "peak": HBM_PEAK_GBPS,
                       "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS,
                       "algorithmic_bytes_per_launch": alg / launches,
                       "vertices_per_launch": st["photon_vertices"] / launches,
                       "records_found_per_vertex": st["photons_found"] / max(1, st["photon_vertices"]),
                       "entries_tested_per_vertex": st["photon_candidates"] / max(1, st["photon_vertices"]),
                       "entries_tested_max": st["photon_candidates_max"],
                       "lit_fraction": st["photon_lit_vertices"] / max(1, st["photon_vertices"])}}


def bench_batch_leg(ctx, S, sc, steps=2):
    """The 32-view batch on the church scene already uploaded (8x4x4 cells, the grid the autotuner
    picks for it; --workload batch runs the tuner): 32 seeded views of uneven size and spp, one
    graph launch per step of the wavefront sequence (2^24 paths, one round, fullest cells first),
    then the same views as one graph-launched persistent kernel per step."""
    import torch
    import paper_1912_04000_amd as sd
    import scenegen
    views, spp = scenegen.batch_views(32)
    cams = [sd.camera(v.eye, v.target, v.up, v.vfov_deg, v.width, v.height) for v in views]
    outs = [torch.empty((sc.n_bins, c.height, c.width), dtype=torch.float32, device="cuda") for c in cams]
    samples = sum(c.width * c.height * k for c, k in zip(cams, spp))
    res = {}
    for name, p in (("wavefront_graph", sd.render_params(max_depth=8, seed=1, wave_paths=1 << 24, queue_rounds=1,
                                                          cell_order=1, use_graph=1)),
                    ("persistent", sd.render_params(max_depth=8, seed=1, use_graph=1, persistent=1))):
        ctx.render_batch(S, cams, spp, p, outs=outs)   # captures the graph
        ctx.finish()
        n = steps if name == "wavefront_graph" else 1
        dt = _timed(lambda: [ctx.render_batch(S, cams, spp, p, outs=outs, finish=False) for _ in range(n)])
        ctx.finish()
        res[name] = {"samples_per_s": samples * n / dt, "ms_per_step": dt / n * 1e3, "steps": n}
    res["views"] = len(cams)
    res["samples_per_step"] = samples
    res["persistent_relative"] = res["persistent"]["samples_per_s"] / res["wavefront_graph"]["samples_per_s"]
    res["note"] = ("32 seeded views 256x256..1024x768, 4..64 spp, 40 bins, depth 8, church 8x4x4 cells; "
                   "one graph launch per step")
    return res


def bench_global_map(ctx, S, sc, cam, cfg, wave, n_photons=2_000_000, radius=0.15, spp=8, gm_from=2):
    """Global photon map (section 4) of the benchmarked view: HIP-event time of building it, then
    of an spp-sample frame whose paths take the diffuse light of vertex gm_from on from it (final
    gathering over the first bounce), against the plain frame at the same spp."""
    import torch
    import paper_1912_04000_amd as sd
    pp = sd.photon_params(n_photons, radius=radius, max_depth=cfg["max_depth"], seed=1, capacity=6 * n_photons,
                          kind=sd.PHOTON_GLOBAL)
    m = sd.PhotonMap(ctx, S, pp)
    m.build(S)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    m.build(S, finish=False)
    e1.record()
    torch.cuda.synchronize()
    ctx.finish()
    build_ms = e0.elapsed_time(e1)
    info = m.info()
    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height)
    img = torch.empty((sc.n_bins, cam.height, cam.width), dtype=torch.float32, device="cuda")
    p = sd.render_params(spp=spp, max_depth=cfg["max_depth"], seed=1, wave_paths=wave, timing=1)
    run = lambda: ctx.render_photons(S, None, c, p, out=img, finish=False, global_map=m, global_from=gm_from)
    run()
    ctx.finish()
    ctx.reset_stats()
    e0.record()
    run()
    e1.record()
    torch.cuda.synchronize()
    ctx.finish()
    st = ctx.stats()
    ms = e0.elapsed_time(e1)
    return {"photons": n_photons, "radius_m": radius, "max_depth": cfg["max_depth"], "from_vertex": gm_from,
            "build_ms": build_ms, "photons_per_s": n_photons / (build_ms * 1e-3), "records": info["stored"],
            "spp": spp, "samples_per_s": cam.width * cam.height * spp / (ms * 1e-3),
            "gather_ms_per_launch": st["photon_ms"] / max(1, st["photon_launches"]),
            "records_found_per_vertex": st["photons_found"] / max(1, st["photon_vertices"]),
            "vertices_per_launch": st["photon_vertices"] / max(1, st["photon_launches"])}


def _progress(msg):
    # long workloads report their steps on stderr (the JSON line stays the only stdout line)
    print(msg, file=sys.stderr, flush=True)


def bench_large(args):
    print(json.dumps(large_result(args)), flush=True)


def large_result(args):
    """The large configuration: procedural church of ~10M triangles (200 windows), 80 bins (5 nm), 3840x2160, 16x8x8
    cells, depth 8. Plain 256 spp against the cache-terminated path given the same wall time
    (untrained cache; 1-spp frames, accumulated, until the plain time is used up; every frame
    trains the cache once: 8 Adam steps of 2^14 records, lr 3e-3, position grids of 2^21 entries
    per level -- the configuration leaves the cache's training open, and the larger scene and
    frame want more of it than the 1080p church). RMSE over the pixels x % 32 == 0, y % 32 == 0
    against the oracle's FP64 2048-spp reference of them (tests/golden/c5_reference.npz, two
    independent 1024-spp halves); the reference's own noise variance, estimated from its halves,
    is subtracted from each mean squared error. value = plain samples/s of the 256-spp frame."""
    import torch
    import paper_1912_04000_amd as sd
    import scenegen
    t0 = time.perf_counter()
    sc = scenegen.church_scene(n_bins=80, target_tris=10_000_000, n_bays=50, tiers=2)
    cam = scenegen.church_camera(3840, 2160)
    S = sd.Scene.from_description(sc, grid=(16, 8, 8))
    build_s = time.perf_counter() - t0
    B, W, H = sc.n_bins, cam.width, cam.height
    ctx = sd.Context(0)
    ctx.upload(S)
    wave = args.wave_paths
    rf = np.load(os.path.join(ROOT, "tests", "golden", "c5_reference.npz"))
    assert int(rf["n_tri"]) == sc.n_tri and int(rf["width"]) == W and int(rf["n_bins"]) == B
    ref_px, ref, noise_var = rf["pixels"], rf["image"].astype(np.float64), float(rf["noise_var"])
    px_t = torch.from_numpy(ref_px).cuda()
    _progress(f"large: scene {sc.n_tri} triangles built in {build_s:.1f} s")

    def rmse_window(img):
        sub = img.reshape(B, -1)[:, px_t].double().cpu().numpy()
        return float(np.sqrt(max(np.mean((sub - ref) ** 2) - noise_var, 0.0)))

    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, W, H)
    img = torch.empty((B, H, W), dtype=torch.float32, device="cuda")
    ctx.render(S, c, sd.render_params(spp=1, max_depth=8, seed=7, wave_paths=wave), out=img)  # warm-up
    spp_plain = 256
    ctx.reset_stats()
    t_plain = _timed(lambda: ctx.render(S, c, sd.render_params(spp=spp_plain, max_depth=8, seed=1, wave_paths=wave,
                                                                timing=1), out=img))
    st_plain = ctx.stats()
    r_plain = rmse_window(img)
    _progress(f"large: plain {spp_plain} spp in {t_plain:.1f} s, RMSE {r_plain:.3e}")
    # cached, same wall time
    lo = sc.verts.reshape(-1, 3).min(0) - 0.05
    hi = sc.verts.reshape(-1, 3).max(0) + 0.05
    cache = sd.Cache(ctx, sd.cache_config(len(sc.mat_type), lo, hi, max_bins=B,
                                          max_records=max(args.train_paths, 1 << 17), max_step=1 << 14,
                                          lr=args.cache_lr or 3e-3, log2_table_pos=args.cache_log2_pos or 21),
                     seed=12345)
    tp = sd.train_params(train_paths=args.train_paths, step_records=1 << 14, steps=args.train_steps or 8, every=0)
    acc = torch.zeros((B, H, W), dtype=torch.float32, device="cuda")
    chunk, done_spp, t_cached, chunks = 1, 0, 0.0, []
    ctx.reset_stats()
    frame = 0
    while t_cached < t_plain:
        train = (args.large_train_frames <= 0 or frame < args.large_train_frames
                 or (frame - args.large_train_frames) % max(1, args.large_train_period) == 0)
        dt = _timed(lambda: ctx.render_cached(S, cache, c, sd.render_params(spp=chunk, max_depth=8, seed=1,
                                                                             mode=sd.MODE_CACHED, wave_paths=wave,
                                                                             first_sample=done_spp, timing=1),
                                              tp if train else None, out=img))
        frame += 1
        acc.mul_(done_spp / (done_spp + chunk)).add_(img, alpha=chunk / (done_spp + chunk))
        done_spp += chunk
        t_cached += dt
        if done_spp & (done_spp - 1) == 0:
            chunks.append(dict(spp=done_spp, seconds=t_cached, rmse=rmse_window(acc)))
            _progress(f"large: cached {done_spp} spp after {t_cached:.1f} s")
    st_c = ctx.stats()
    r_cached = rmse_window(acc)
    chunks.append(dict(spp=done_spp, seconds=t_cached, rmse=r_cached))
    # plain spp for the cached RMSE (RMSE ~ spp^-1/2 through the measured 256-spp point)
    spp_eq = spp_plain * (r_plain / r_cached) ** 2
    t_eq = t_plain * spp_eq / spp_plain
    value = W * H * spp_plain / t_plain
    out = {
        "metric": METRIC, "value": value, "unit": "spectral path samples/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": t_plain * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (tracer) / bf16 (cache MLP)", "data": f"synthetic (seeded procedural scene, {sc.n_tri} triangles)",
        "config": {"workload": "church-10M large: 3840x2160, 80 bins 380-780 nm, depth 8, 16x8x8 cells, 200 windows; "
                               "plain 256 spp vs cached at equal wall time",
                   "triangles": sc.n_tri, "materials": len(sc.mat_type),
                   "reference": f"oracle FP64, {int(rf['spp'])} spp, pixels x % 32 == y % 32 == 0 "
                                f"({len(ref_px)} pixels), its noise variance {noise_var:.3e} subtracted",
                   "scene_build_s": build_s},
        "equal_time": {"plain_spp": spp_plain, "plain_s": t_plain, "rmse_plain": r_plain,
                       "cached_spp": done_spp, "cached_s": t_cached, "rmse_cached": r_cached,
                       "rmse_ratio_plain_over_cached": r_plain / r_cached,
                       "spp_plain_equivalent": spp_eq, "time_plain_equivalent_s": t_eq,
                       "speedup_at_equal_rmse": t_eq / t_cached,
                       "adam_steps": cache.info()["adam_steps"], "train_batches": st_c["train_batches"],
                       "cache": {"lr": args.cache_lr or 3e-3, "log2_table_pos": args.cache_log2_pos or 21,
                                 "steps_per_batch": args.train_steps or 8, "records_per_step": 1 << 14},
                       "training": ("one batch per frame" if args.large_train_frames <= 0 else
                                    f"one batch per frame for {args.large_train_frames} frames, then one every "
                                    f"{args.large_train_period}")},
        "timing_split_ms": {"plain_trace": st_plain["trace_ms"], "plain_shade": st_plain["shade_ms"],
                            "cached_trace": st_c["trace_ms"], "cached_shade": st_c["shade_ms"],
                            "cached_query": st_c["query_ms"], "cached_train_steps": st_c["train_ms"]},
        "cached_progress": chunks,
    }
    return out


def bench_batch(args):
    """32 seeded views of the church with uneven resolutions (256x256 .. 1024x768) and spp (4..64),
    rendered together in one graph launch per step, with the grid, wavefront size and queue rounds
    picked by the autotuner (cached per scene and device)."""
    import torch
    import paper_1912_04000_amd as sd
    import scenegen
    sc = scenegen.church_scene(40)
    views, spp = scenegen.batch_views(32)
    cams = [sd.camera(v.eye, v.target, v.up, v.vfov_deg, v.width, v.height) for v in views]
    ctx = sd.Context(0)
    os.makedirs(os.path.dirname(args.tune_cache), exist_ok=True)
    t0 = time.perf_counter()
    tune = ctx.autotune(sc, cams, sd.render_params(max_depth=8, seed=1),
                        waves=[1 << 22, 1 << 23, 1 << 24],
                        grids=[(4, 4, 4), (8, 8, 8), (16, 16, 16), (8, 4, 4)], rounds=(1, 2), orders=(0, 1),
                        try_persistent=True, calib_spp=1, reps=2, cache_path=args.tune_cache)
    tune_s = time.perf_counter() - t0
    best = tune["best"]
    S = sd.Scene.from_description(sc, grid=tuple(best["grid"]))
    ctx.upload(S)
    p = sd.render_params(max_depth=8, seed=1, wave_paths=best["wave_paths"], queue_rounds=best["queue_rounds"],
                         cell_order=best["cell_order"], persistent=best["persistent"], use_graph=1, timing=1)
    outs = [torch.empty((sc.n_bins, c.height, c.width), dtype=torch.float32, device="cuda") for c in cams]
    for _ in range(max(1, args.warmup)):   # the first call captures the graph
        ctx.render_batch(S, cams, spp, p, outs=outs)
    ctx.finish()
    ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.render_batch(S, cams, spp, p, outs=outs, finish=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.finish()
    st = ctx.stats()
    samples = sum(c.width * c.height * s for c, s in zip(cams, spp)) * args.steps
    value = samples / dt
    # the same batch as one persistent kernel (work list of (view, tile, sample) items), also one
    # graph launch per step, on the tuned grid
    pp = sd.render_params(max_depth=8, seed=1, use_graph=1, timing=1, persistent=1)
    ctx.render_batch(S, cams, spp, pp, outs=outs)   # captures its graph
    ctx.finish()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        ctx.render_batch(S, cams, spp, pp, outs=outs, finish=False)
    torch.cuda.synchronize()
    dt_p = time.perf_counter() - t1
    ctx.finish()
    out = {
        "metric": METRIC, "value": value, "unit": "spectral path samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": f"synthetic (seeded procedural scene, {sc.n_tri} triangles)",
        "config": {"workload": "church-1M batch: 32 seeded views 256x256..1024x768, spp 4..64, 40 bins, depth 8, "
                               "one graph launch per step, autotuned grid / wavefront / rounds",
                   "views": len(cams), "samples_per_step": samples // args.steps, "tuned": best,
                   "tune_from_cache": tune["from_cache"], "tune_seconds": tune_s,
                   "tune_candidates": len(tune["tried"])},
        "graph_ms_per_step": st["graph_ms"] / max(1, st["graph_launches"]),
        "persistent": {"samples_per_s": samples / dt_p, "ms_per_step": dt_p / args.steps * 1e3,
                       "relative_to_wavefront": (samples / dt_p) / value,
                       "note": "the same 32 views as one persistent kernel per step (lanes taking (view, 8x8 "
                               "tile, sample) items from a device work list), graph-launched, tuned grid"},
        "tune_table": tune["tried"],
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this renderer runs on one GPU only (asked for --gpus {args.gpus}); sharding the "
              "path over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return
    if args.pmc_summary:
        pmc_summary(args)
        return
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "cached":
        bench_cached(args)
        return
    if args.workload == "large":
        bench_large(args)
        return
    import torch
    import paper_1912_04000_amd as sd

    sc, cam, cfg, label = workload(args.workload, args.spp)
    ctx = sd.Context(0)
    t0 = time.perf_counter()
    S = sd.Scene.from_description(sc, grid=cfg["grid"])
    build_s = time.perf_counter() - t0
    ctx.upload(S)
    c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height)
    wave = min(args.wave_paths, cam.width * cam.height * cfg["spp"])
    p = sd.render_params(spp=cfg["spp"], max_depth=cfg["max_depth"], seed=1,
                         wave_paths=0 if args.persistent else max(64, wave),
                         queue_rounds=args.queue_rounds, timing=1, cell_order=args.cell_order,
                         persistent=args.persistent)
    img = torch.empty((sc.n_bins, cam.height, cam.width), dtype=torch.float32, device="cuda")
    for _ in range(args.warmup):
        ctx.render(S, c, p, out=img)
    ctx.finish()
    ctx.reset_stats()
    # per-step HIP events on the stream the library launches on (torch's current stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(args.steps):
        ctx.render(S, c, p, out=img, finish=False)
        ev[k + 1].record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.finish()
    step_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    st = ctx.stats()
    samples = cam.width * cam.height * cfg["spp"] * args.steps
    value = samples / dt
    B = sc.n_bins
    # dominant kernel: the cell-local traversal (k_trace); its launches are bracketed by HIP events
    # on the library's stream (timing = 1)
    launches = max(1, st["trace_launches"])
    trace_s = st["trace_ms"] / 1e3
    tb = trace_bytes(st)
    achieved = tb / trace_s / 1e9 if trace_s > 0 else 0.0
    ops = OPS_PER_NODE * st["node_visits"] + OPS_PER_TRI * st["tri_tests"]
    alu = ops / trace_s / 1e12 if trace_s > 0 else 0.0
    src = open(os.path.join(ROOT, "paper_1912_04000_amd", "csrc", "kernels.hip"), "rb").read()
    traffic = traffic_from_profiles(hashlib.sha256(src).hexdigest())
    ab = path_bytes(st, B)
    out = {
        "metric": METRIC, "value": value, "unit": "spectral path samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": f"synthetic (seeded procedural scene, {sc.n_tri} triangles)",
        "config": {"workload": label, "triangles": sc.n_tri, "width": cam.width, "height": cam.height,
                   "spp": cfg["spp"], "bins": B, "max_depth": cfg["max_depth"], "grid": list(cfg["grid"]),
                   "wave_paths": p.wave_paths, "queue_rounds": args.queue_rounds or 1,
                   "cell_order": args.cell_order, "persistent": args.persistent},
        "ms_per_step_median": float(np.median(step_ms)), "ms_per_step_events": step_ms,
        "bin_samples_per_s": value * B,
        "roofline": {"kernel": "k_trace", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic, "traffic_over_algorithmic": (traffic / (tb / launches)) if traffic else None,
                     "launches": st["trace_launches"], "avg_launch_ms": st["trace_ms"] / launches,
                     "algorithmic_bytes_per_launch": tb / launches,
                     "cell_visits_per_launch": st["cell_visits"] / launches,
                     "note": "algorithmic bytes per launch (40 B per device-counted cell visit: ray record read, "
                             "queue entry written and read; 16 B hit record per extension ray) over the HIP-event "
                             "time of the k_trace launches on the library stream; traffic = HBM bytes per launch "
                             "from rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by a copy calibration, null unless "
                             "taken on this kernel source"},
        "roofline_alu": {"kernel": "k_trace", "bound": "alu", "achieved": alu, "peak": ALU_PEAK_TOPS,
                         "unit": "TOP/s", "frac": alu / ALU_PEAK_TOPS,
                         "note": "secondary: algorithmic FP32 VALU ops (104 per 4-wide BVH node, 56 per triangle "
                                 "test) over the same time; peak = non-packed VALU issue rate 256 CU x 64 x 2.4 GHz"},
        "path_hbm": {"algorithmic_bytes_per_sample": ab / max(1, st["paths"]),
                     "achieved_GBps": ab / dt / 1e9, "peak_GBps": HBM_PEAK_GBPS,
                     "frac": ab / dt / 1e9 / HBM_PEAK_GBPS,
                     "formula": "R + 3S + V(2R + 2H + 6S) + 40 B x cell visits per path, S = 4 B x bins, "
                                "V and cell visits counted on the device"},
        "timing_split_ms": {"trace": st["trace_ms"] / args.steps, "shade": st["shade_ms"] / args.steps},
        "per_path": {"vertices": st["vertices"] / max(1, st["paths"]),
                     "shadow_rays": st["shadow_rays"] / max(1, st["paths"]),
                     "cell_visits_per_ray": st["cell_visits"] / max(1, st["ext_rays"] + st["shadow_rays"]),
                     "nodes_per_ray": st["node_visits"] / max(1, st["ext_rays"] + st["shadow_rays"]),
                     "tri_tests_per_ray": st["tri_tests"] / max(1, st["ext_rays"] + st["shadow_rays"])},
        "scene_build_s": build_s,
    }
    if not args.no_extras:
        out["colorimetry"] = bench_colorimetry(ctx, img, sc)
        if args.workload == "church":
            out["glass_maps"] = bench_glass_maps(ctx, sc, cam, cfg, p.wave_paths)
            out["photon_map"] = bench_photons(ctx, S, sc, cam, cfg, p.wave_paths)
            out["global_map"] = bench_global_map(ctx, S, sc, cam, cfg, p.wave_paths)
            out["batch"] = bench_batch_leg(ctx, S, sc)
            # the large configuration as one more leg: its own scene, context and workspace
            try:
                lg = large_result(args)
                out["large"] = {"samples_per_s": lg["value"], "plain_s": lg["ms_per_step"] / 1e3,
                                "config": lg["config"], "equal_time": lg["equal_time"],
                                "timing_split_ms": lg["timing_split_ms"]}
            except Exception as e:  # recorded, so that the church line above still prints
                out["large"] = {"error": f"{type(e).__name__}: {e}"}
    if args.workload == "church" and not args.no_cached:
        # the cached half of the metric on the same view: plain frames at 1 .. 256 spp fix a in the
        # least-squares fit RMSE = a / sqrt(spp) of the plain estimator; the plain rate is the one
        # just measured
        px, ref = load_reference()
        r64 = _rmse(img.cpu().numpy(), ref, px)
        c = sd.camera(cam.eye, cam.target, cam.up, cam.vfov_deg, cam.width, cam.height)
        curve, a, slope = plain_curve(ctx, S, c, img, px, ref, p.wave_paths, (1, 2, 4, 8, 16, 32, 64, 128, 256),
                                      cam.width, cam.height)
        cached = run_cached(ctx, S, sc, cam, img, args, px, ref, p.wave_paths)
        out["equal_rmse"] = equal_rmse(cached, a, value, cam.width, cam.height, args.warm_frames)
        out["equal_rmse"]["rmse_plain_frame"] = r64
        out["equal_rmse"]["plain_curve"] = [{"spp": q["spp"], "rmse": q["rmse"]} for q in curve]
        out["equal_rmse"]["plain_loglog_slope"] = slope
        out["equal_rmse"]["reference"] = reference_note()
    if not args.no_cpu_baseline:
        # the host cores this job may use: its CPU affinity (a one-GPU machine allots 16), unless given
        try:
            avail = len(os.sched_getaffinity(0))
        except AttributeError:
            avail = os.cpu_count() or 1
        threads = args.cpu_threads or min(16, avail)
        out["cpu_baseline"] = cpu_baseline(sc, cam, cfg, threads)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
