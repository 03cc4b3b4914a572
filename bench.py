#!/usr/bin/env python3
"""Throughput of the exact squared EDT + feature transform on one MI355X.

One step = one edt_feature call (site predicate, vertical pass, lower envelope
and fill: squared distance and nearest-site index for every pixel) on one
synthetic image already resident in HBM.  The default workload is the
16384 x 16384 image with 30 random object points, the single-image size at
which the HBM roofline is measured.

Prints ONE JSON line (see the keys below).  --gpus N > 1 is refused: this
build runs on one GPU.
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

METRIC = "Gpixel/s exact sq-EDT+feature transform and % HBM roofline; batched vs per-image"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak

PATH_BYTES_PER_PX = 13.0  # 1 mask + 2 + 2 intermediate + 4 D + 4 F


def algo_bytes(kernel: str, H: int, W: int, n: int, with_dist: bool = True) -> int:
    """Algorithmic HBM bytes of one launch of `kernel` on an H x W image whose
    sites occupy n columns: what the kernel must read and write at minimum
    given its inputs and outputs ('Roofline')."""
    nb = (H + 63) // 64
    if kernel == "k_band_bits":          # mask in, one site bit per pixel out
        return H * W + nb * W * 8
    if kernel == "k_band_carry":         # site bits in, two int16 carries per band out
        return nb * W * 8 + nb * W * 4 + W * 4
    if kernel == "k_col_compact":        # column flags in, column list out
        return W * 4 + n * 2
    if kernel == "k_nearest_row":        # bits + carries of listed columns in, int16 rows out
        return nb * n * 12 + H * n * 2
    if kernel.startswith("k_row_"):      # int16 rows in, int32 D and F out
        return H * n * 2 + H * W * (8 if with_dist else 4)
    raise KeyError(kernel)


def site_columns(mask, polarity) -> int:
    """Number of columns holding at least one site (input statistics)."""
    import numpy as np
    site = (mask != 0) if polarity == 0 else (mask == 0)
    return int(np.count_nonzero(site.any(axis=0)))

WORKLOADS = {
    "points16k": dict(
        H=16384, W=16384, polarity=0,
        desc="16384x16384 uint8 mask, 30 uniform random object points (Voronoi-style); "
             "int32 squared distance + int32 nearest-object index per pixel"),
    "disks4k": dict(
        H=4096, W=4096, polarity=0,
        desc="4096x4096 uint8 mask, 200 random filled disks (r 5-200) + Bernoulli(1e-4) "
             "points; distances outside objects"),
    "disks4k_inside": dict(
        H=4096, W=4096, polarity=1,
        desc="4096x4096 uint8 mask, 200 random filled disks (r 5-200) + Bernoulli(1e-4) "
             "points; distances inside objects"),
    "bernoulli256": dict(
        H=256, W=256, polarity=0,
        desc="256x256 uint8 mask, Bernoulli(0.01) object pixels"),
}


def make_mask(name):
    import workloads
    if name == "points16k":
        return workloads.points(16384, 16384, 30)
    if name.startswith("disks4k"):
        return workloads.disks(4096, 4096)
    if name == "bernoulli256":
        return workloads.bernoulli(256, 256, 0.01)
    raise SystemExit(f"unknown workload {name}")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2106_03503_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    ent = t.get("kernels", {}).get(workload, {}).get(kernel)
    if not ent or t.get("source_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(mask, polarity, units_px):
    import oracle
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    oracle.separable(mask, polarity, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(units_px / dt / 1e9, 5), "unit": "Gpixel/s", "cores": threads,
            "kind": "oracle",
            "sample": f"one full pass of the oracle's separable transform (vertical pass + "
                      f"lower envelope + fill) over the whole {mask.shape[0]}x{mask.shape[1]} "
                      f"image, {threads} POSIX threads, {dt:.2f} s"}


def copy_calibration(steps):
    """Plain device-to-device copy of a known size, for scaling the rocprofv3
    FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = 1 << 30
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(steps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "launches": steps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="points16k", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the cpu_baseline leg")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(see DESIGN.md, 'More than one GPU').", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2106_03503_amd as edt

    if args.copy_calibration:
        copy_calibration(args.steps)
        return

    wl = WORKLOADS[args.workload]
    H, W, pol = wl["H"], wl["W"], wl["polarity"]
    mask_np = make_mask(args.workload)
    dev = torch.device("cuda:0")
    mask = torch.from_numpy(mask_np).to(dev)
    D = torch.empty((H, W), dtype=torch.int32, device=dev)
    F = torch.empty((H, W), dtype=torch.int32, device=dev)
    ws = torch.empty(edt.workspace_bytes(H, W, True), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        edt.feature(mask, polarity=pol, out_dist=D, out_feat=F, workspace=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    edt.profile_begin()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = edt.profile_end()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    px = H * W
    value = px / (ms_per_step * 1e-3) / 1e9

    # dominant kernel and its roofline
    dom = max(kt, key=lambda k: kt[k][1])
    launches, total_ms = kt[dom]
    avg_ms = total_ms / launches
    algo = algo_bytes(dom, H, W, site_columns(mask_np, pol))
    achieved = algo / (avg_ms * 1e-3) / 1e9
    traffic = traffic_from_profiles(dom, args.workload)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "algorithmic_bytes_per_launch": int(algo),
                "avg_launch_ms": round(avg_ms, 4)}

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "H": H, "W": W, "polarity": pol,
                   "call": "edt_feature", "parallelism": "single GPU"},
        "roofline": roofline,
        "path_hbm": {"bytes_per_px": PATH_BYTES_PER_PX,
                     "achieved_GBs": round(PATH_BYTES_PER_PX * px / (ms_per_step * 1e-3) / 1e9, 1),
                     "frac": round(PATH_BYTES_PER_PX * px / (ms_per_step * 1e-3) / 1e9
                                   / HBM_PEAK_GBS, 4)},
        "kernels_ms_per_step": {k: round(v[1] / max(1, v[0]) * v[0] / args.steps, 4)
                                for k, v in sorted(kt.items())},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mask_np, pol, px)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
