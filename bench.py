#!/usr/bin/env python
"""Benchmark of the plain spectral path tracer on one MI355X.

Workload (default): the seeded procedural church of 979,664 triangles (40 coloured glass windows),
1920x1080 pixels, 40 wavelength bins over 380-780 nm, 64 samples per pixel, 8 surface vertices
per path, 8x4x4 cells, 2^21 paths in flight. One step = one full frame (132.7 M spectral path
samples, each carrying all 40 bins). Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload church|nave] [--no-cpu-baseline]
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

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spectral path samples/s on 1 GPU, plain vs MLP-cached at equal RMSE; HBM GB/s"
HBM_PEAK_GBPS = 8000.0
# Non-packed FP32 VALU issue rate of MI355X: 256 CUs x 64 lanes x 2.4 GHz (ops/s, 1 op = 1 flop).
# The 157.3 TFLOP/s vector figure counts an FMA as 2 flops on packed (2-wide) lanes.
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Algorithmic VALU operations per unit of traversal work (counted from the kernel source):
OPS_PER_NODE = 52       # two robust slab tests (6 sub, 6 mul, 12 min/max, 1 slop mul, 1 cmp each)
OPS_PER_TRI = 56        # watertight test: translate, shear, 3 edge functions, signs, det, t, u, v


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="church", choices=["church", "nave", "batch"])
    ap.add_argument("--tune-cache", default=os.path.join(os.path.expanduser("~"), ".cache", "specdd",
                                                          "tune_cache.json"))
    ap.add_argument("--spp", type=int, default=None, help="override samples per pixel (profiling runs)")
    ap.add_argument("--wave-paths", type=int, default=1 << 21)
    ap.add_argument("--queue-rounds", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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


def algorithmic_bytes(st, B):
    """HBM bytes the wavefront design must move, from the device counters (record sizes:
    ray R = 32 B, hit H = 16 B, queue entry 4 B, produced list entry 12 B, spectral value 4 B
    per bin, triangle record 48 B)."""
    R, H, S = 32, 16, 4 * B
    produced = st["ext_rays"] + st["shadow_rays"]
    b = 0
    b += st["paths"] * (R + S + 16)                 # raygen: ray, beta = 1, path state
    b += produced * (12 + 12 + 4)                   # list write, scatter read, queue write
    b += st["cell_visits"] * (4 + R)                # traversal: queue entry + ray record
    b += st["migrations"] * 12                      # re-queued entries
    b += st["ext_rays"] * 2 * H                     # hit record written, read by shading
    b += st["vertices"] * (48 + 2 * S + R + 16)     # triangle, beta read+write, new ray, state
    b += st["shadow_rays"] * (R + 3 * S)            # shadow ray, NEE weight write+read, image
    return b


def cpu_baseline(sc, cam, cfg, threads):
    """The oracle as it stands, on the host cores, on the pixel subset x%4==0, y%4==0 at 32 spp
    (a bounded sample of the same frame, ~10-30 s of CPU work); its fixed per-call cost (BVH
    build) is subtracted."""
    import numpy as np
    import oracle
    ys, xs = np.meshgrid(np.arange(0, cam.height, 4), np.arange(0, cam.width, 4), indexing="ij")
    px = (ys * cam.width + xs).ravel()
    spp = min(32, cfg["spp"])
    t0 = time.perf_counter()
    oracle.render(sc, cam, spp=1, max_depth=cfg["max_depth"], seed=1, pixels=px[:1], threads=threads)
    fixed = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = oracle.render(sc, cam, spp=spp, max_depth=cfg["max_depth"], seed=1, pixels=px, threads=threads)
    dt = time.perf_counter() - t0 - fixed
    n = len(px) * spp
    return {"value": n / dt, "unit": "spectral path samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(px)} pixels (every 4th row and column) x {spp} spp of the same frame, "
                      f"{n} paths in {dt:.1f} s (+{fixed:.1f} s BVH build excluded), FP64",
            "vertices_per_path": r.stats["vertices"] / n}


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
                        waves=[1 << 18, 1 << 20, 1 << 21, 1 << 22],
                        grids=[(4, 4, 4), (8, 8, 8), (16, 16, 16), (8, 4, 4)], rounds=(1, 2), calib_spp=1, reps=2,
                        cache_path=args.tune_cache)
    tune_s = time.perf_counter() - t0
    best = tune["best"]
    S = sd.Scene.from_description(sc, grid=tuple(best["grid"]))
    ctx.upload(S)
    p = sd.render_params(max_depth=8, seed=1, wave_paths=best["wave_paths"], queue_rounds=best["queue_rounds"],
                         use_graph=1, timing=1)
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
    p = sd.render_params(spp=cfg["spp"], max_depth=cfg["max_depth"], seed=1, wave_paths=max(64, wave),
                         queue_rounds=args.queue_rounds, timing=1)
    img = torch.empty((sc.n_bins, cam.height, cam.width), dtype=torch.float32, device="cuda")
    for _ in range(args.warmup):
        ctx.render(S, c, p, out=img)
    ctx.finish()
    ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.render(S, c, p, out=img, finish=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.finish()
    st = ctx.stats()
    samples = cam.width * cam.height * cfg["spp"] * args.steps
    value = samples / dt
    B = sc.n_bins
    # dominant kernel: the cell-local traversal (k_trace); its launches are bracketed by HIP events
    ops = OPS_PER_NODE * st["node_visits"] + OPS_PER_TRI * st["tri_tests"]
    trace_s = st["trace_ms"] / 1e3
    achieved = ops / trace_s / 1e12 if trace_s > 0 else 0.0
    src = open(os.path.join(ROOT, "paper_1912_04000_amd", "csrc", "kernels.hip"), "rb").read()
    traffic = traffic_from_profiles(hashlib.sha256(src).hexdigest())
    ab = algorithmic_bytes(st, B)
    out = {
        "metric": METRIC, "value": value, "unit": "spectral path samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": f"synthetic (seeded procedural scene, {sc.n_tri} triangles)",
        "config": {"workload": label, "triangles": sc.n_tri, "width": cam.width, "height": cam.height,
                   "spp": cfg["spp"], "bins": B, "max_depth": cfg["max_depth"], "grid": list(cfg["grid"]),
                   "wave_paths": p.wave_paths, "queue_rounds": args.queue_rounds or 2},
        "bin_samples_per_s": value * B,
        "roofline": {"kernel": "k_trace", "bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS,
                     "unit": "TFLOP/s", "frac": achieved / ALU_PEAK_TOPS, "traffic": traffic,
                     "launches": st["trace_launches"], "avg_launch_ms": st["trace_ms"] / max(1, st["trace_launches"]),
                     "ops_per_launch": ops / max(1, st["trace_launches"]),
                     "note": "algorithmic FP32 VALU ops (52 per BVH node, 56 per triangle test) over the "
                             "HIP-event time of the k_trace launches; peak = non-packed VALU issue rate"},
        "path_hbm": {"algorithmic_bytes_per_sample": ab / max(1, st["paths"]),
                     "achieved_GBps": ab / dt / 1e9, "peak_GBps": HBM_PEAK_GBPS,
                     "frac": ab / dt / 1e9 / HBM_PEAK_GBPS},
        "timing_split_ms": {"trace": st["trace_ms"] / args.steps, "shade": st["shade_ms"] / args.steps},
        "per_path": {"vertices": st["vertices"] / max(1, st["paths"]),
                     "shadow_rays": st["shadow_rays"] / max(1, st["paths"]),
                     "cell_visits_per_ray": st["cell_visits"] / max(1, st["ext_rays"] + st["shadow_rays"]),
                     "nodes_per_ray": st["node_visits"] / max(1, st["ext_rays"] + st["shadow_rays"])},
        "scene_build_s": build_s,
    }
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(sc, cam, cfg, threads)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
