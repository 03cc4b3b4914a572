#!/usr/bin/env python3
"""Throughput of the exact squared EDT + feature transform on one MI355X.

Workloads (--workload):
  points16k (default)  one step = one edt_feature call on a 16384 x 16384 image
                       with 30 random object points: the single-image size at
                       which the HBM roofline is measured.  The default line
                       also carries, as extra keys, shorter runs of the rest of
                       the metric: "batch2048" (batched against per-image
                       launches), "serve" (the request server at 5000 req/s and
                       all at once, against per-image launches of the same
                       requests) and "dense16k" (--no-extras skips them);
  dense16k             a 16384 x 16384 image of 3200 random disks (the 4096^2
                       disk image's density over 16 times the area);
  points16k_sq         the same image through edt_sq (distances only);
  points16k_f32, dense16k_f32
                       the points and dense images through edt_dist_f32 (fp32
                       Euclidean distances written by the row pass, and features);
  disks4k, disks4k_inside, bernoulli256
  disks4k_regions      the disks image through edt_feature and then edt_regions
  disks1k_danielsson   a 1024^2 disks image through Danielsson's approximate transform,
                       with its error against the exact one
  disks4k_chamfer      the disks image through edt_sq with the chamfer 4-3 metric,
                       with its error against the exact Euclidean distance
                       other single images (4096^2 disks outside / inside,
                       256^2 Bernoulli(0.01));
  batch2048            one step = one edt_batch_submit over 2048 images of
                       uneven size (sides 64..1024, 5-60 ellipses, mixed
                       polarity), replayed as a captured graph, after
                       edt_batch_autotune picked the schedule; the same
                       images launched one by one through edt_feature are
                       timed beside it ("per_image").
  serve                one step = one replay of a Poisson request stream
                       (--rate requests/s, --requests of them; square masks
                       of side 128..8192 log-uniform, Bernoulli or ellipses,
                       half distance-only) through the request server; reports
                       throughput and p50/p99 latency (submission to observed
                       completion).
Inputs are resident in HBM before the timed region.  Prints ONE JSON line.
--gpus N > 1 is refused: the library has no multi-GPU path, so the benchmark runs
on one GPU.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpixel/s exact sq-EDT+feature transform and % HBM roofline; batched vs per-image"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak
SWEEP_RATES = (100.0, 250.0, 500.0, 1000.0, 2000.0, 5000.0)


def path_bytes(H: int, W: int, n: int, with_feature: bool = True, lanes: bool = False) -> int:
    """Bytes the method itself must move for one image: the mask read once, the
    outputs written once (4 B of distance, plus 4 B of feature), and the
    intermediate as this design holds it -- the nearest site row (int16) of
    each of the n columns holding a site, written by the vertical pass and
    read by the row pass; for a batch image of the one-lane-per-row pass,
    which works the rows out itself, the band bits and carries (12 B per
    column per 64-row band) written and read once instead."""
    inter = 2 * 12 * ((H + 63) // 64) * W if lanes else 2 * 2 * H * n
    return H * W * (1 + 4 + (4 if with_feature else 0)) + inter


def algo_bytes(kernel: str, H: int, W: int, n: int, with_dist: bool = True) -> int:
    """Algorithmic HBM bytes of one launch of `kernel` on an H x W image whose
    sites occupy n columns: what the kernel must read and write at minimum
    given its inputs and outputs."""
    nb = (H + 63) // 64
    if kernel == "k_band_bits":          # mask in, one site bit per pixel out
        return H * W + nb * W * 8
    if kernel == "k_band_carry":         # site bits in, two int16 carries per band out
        return nb * W * 8 + nb * W * 4 + W
    if kernel == "k_col_compact":        # column flags in, column list out
        return W + n * 2
    if kernel == "k_nearest_row":        # bits + carries of listed columns in, int16 rows out
        return nb * n * 12 + H * n * 2
    if kernel == "k_row_segscan":        # int16 rows in (segment envelopes stay on chip or spill)
        return H * n * 2
    if kernel in ("k_reg_init", "k_reg_union", "k_reg_flatten", "k_reg_sites"):
        return H * W                     # the mask (site slots are a small part)
    if kernel == "k_reg_others":         # mask and F in, labels out
        return H * W * 9
    if kernel == "k_danielsson":         # mask in; positions written, read back, written; D out
        return H * W * 21
    if kernel in ("k_row_segfill", "k_row_segwin"):  # int32 D and F (or D only) out
        return H * W * (8 if with_dist else 4)
    if kernel in ("k_row_lanes", "k_row_sparse"):  # bits + carries of listed columns in, D, F out
        return nb * n * 12 + H * W * (8 if with_dist else 4)
    if kernel.startswith("k_row_"):      # int16 rows in, int32 D and F (or D only) out
        return H * n * 2 + H * W * (8 if with_dist else 4)
    raise KeyError(kernel)


def site_columns(mask, polarity) -> int:
    """Number of columns holding at least one site (input statistics)."""
    import numpy as np
    site = (mask != 0) if polarity == 0 else (mask == 0)
    return int(np.count_nonzero(site.any(axis=0)))


SINGLE = {
    "points16k": dict(
        H=16384, W=16384, polarity=0,
        desc="16384x16384 uint8 mask, 30 uniform random object points (Voronoi-style); "
             "int32 squared distance + int32 nearest-object index per pixel"),
    "points16k_sq": dict(
        H=16384, W=16384, polarity=0, call="edt_sq",
        desc="16384x16384 uint8 mask, 30 uniform random object points; int32 squared "
             "distance only (edt_sq)"),
    "points16k_f32": dict(
        H=16384, W=16384, polarity=0, call="edt_dist_f32",
        desc="16384x16384 uint8 mask, 30 uniform random object points; fp32 Euclidean "
             "distance written by the row pass + int32 nearest-object index (edt_dist_f32)"),
    "dense16k_f32": dict(
        H=16384, W=16384, polarity=0, call="edt_dist_f32",
        desc="16384x16384 uint8 mask, 3200 random filled disks (r 5-200) + Bernoulli(1e-4) "
             "points; fp32 Euclidean distance written by the row pass + int32 nearest-object "
             "index (edt_dist_f32)"),
    "disks4k": dict(
        H=4096, W=4096, polarity=0,
        desc="4096x4096 uint8 mask, 200 random filled disks (r 5-200) + Bernoulli(1e-4) "
             "points; distances outside objects"),
    "dense16k": dict(
        H=16384, W=16384, polarity=0,
        desc="16384x16384 uint8 mask, 3200 random filled disks (r 5-200) + Bernoulli(1e-4) "
             "points (the 4096^2 disk image's density of disks over 16 times the area); "
             "distances outside objects"),
    "disks4k_inside": dict(
        H=4096, W=4096, polarity=1,
        desc="4096x4096 uint8 mask, 200 random filled disks (r 5-200) + Bernoulli(1e-4) "
             "points; distances inside objects"),
    "bernoulli256": dict(
        H=256, W=256, polarity=0,
        desc="256x256 uint8 mask, Bernoulli(0.01) object pixels"),
    "disks4k_regions": dict(
        H=4096, W=4096, polarity=0, regions=8,
        desc="4096x4096 uint8 mask, 200 random filled disks (r 5-200) + Bernoulli(1e-4) "
             "points; int32 squared distance + nearest-object index (edt_feature), then the "
             "Voronoi region of every pixel under 8-neighbourhood (edt_regions)"),
    "disks1k_danielsson": dict(
        H=1024, W=1024, polarity=0, call="edt_danielsson",
        desc="1024x1024 uint8 mask, 40 random filled disks (r 5-100) + Bernoulli(1e-4) points; "
             "Danielsson's approximate squared distances and propagated positions "
             "(edt_danielsson, one workgroup per image)"),
    "disks4k_chamfer": dict(
        H=4096, W=4096, polarity=0, call="edt_sq", metric=3,
        desc="4096x4096 uint8 mask, 200 random filled disks (r 5-200) + Bernoulli(1e-4) "
             "points; int32 chamfer 4-3 distances (scaled by 3) outside objects (edt_sq)"),
}
BATCH_DESC = ("2048 uint8 masks of uneven size (H, W uniform in 64..1024), 5-60 overlapping "
              "random ellipses each (semi-axes 4-80), polarity Bernoulli(0.5); int32 squared "
              "distance + int32 nearest-site index per pixel")
SERVE_DESC = ("{n} requests arriving as a Poisson stream at {rate:g}/s: square uint8 masks of "
              "side round(exp(U(ln 128, ln 8192))), Bernoulli or ellipses (50/50) at "
              "log-uniform density 1e-4..0.3; half int32 squared distance only, half distance + "
              "nearest-site index")


def make_mask(name):
    import workloads
    if name in ("points16k", "points16k_sq", "points16k_f32"):
        return workloads.points(16384, 16384, 30)
    if name in ("dense16k", "dense16k_f32"):
        return workloads.disks(16384, 16384, n_disks=3200)
    if name.startswith("disks4k"):
        return workloads.disks(4096, 4096)
    if name == "disks1k_danielsson":
        return workloads.disks(1024, 1024, n_disks=40, rmin=5, rmax=100)
    if name == "bernoulli256":
        return workloads.bernoulli(256, 256, 0.01)
    raise SystemExit(f"unknown workload {name}")


# Source files that define each kernel (its own file and the shared header).
KERNEL_SOURCES = {
    "k_band_bits": ("edt_column.hip",), "k_band_carry": ("edt_column.hip",),
    "k_col_compact": ("edt_column.hip",), "k_nearest_row": ("edt_column.hip",),
    "k_row_sparse": ("edt_row.hip",), "k_row_dense": ("edt_row.hip",),
    "k_row_dense_global": ("edt_row.hip",), "k_row_lanes": ("edt_row_lanes.hip",),
    "k_row_segscan": ("edt_row_lanes.hip",), "k_row_segfill": ("edt_row.hip",),
    "k_row_segwin": ("edt_row.hip",),
    "k_sqrt": ("edt_api.hip",),
    **{k: ("edt_regions.hip",) for k in ("k_reg_init", "k_reg_union", "k_reg_flatten",
                                         "k_reg_others", "k_reg_sites")},
    "k_danielsson": ("edt_danielsson.hip",),
}


def kernel_source_hash(kernel: str) -> str:
    """Hash of the sources of `kernel`: counters taken before a change to them
    no longer describe it."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2106_03503_amd", "csrc")
    for f in KERNEL_SOURCES.get(kernel, tuple(sorted(os.listdir(csrc)))) + ("edt_internal.h",):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    ent = t.get("kernels", {}).get(workload, {}).get(kernel)
    if not ent or ent.get("source_hash") != kernel_source_hash(kernel):
        return None
    return ent.get("bytes_per_launch")


def cpu_threads() -> int:
    import oracle
    return oracle.default_threads()


def cpu_baseline(images, units_px, metric=0):
    """The oracle over the images on the host cores: its separable transform,
    or for the chamfer 4-3 metric its two raster scans (one thread)."""
    import oracle
    threads = cpu_threads() if metric == 0 else 1
    t0 = time.perf_counter()
    for m, pol in images:
        if metric == 3:
            oracle.chamfer_scans(m, pol)
        elif metric == "danielsson":
            oracle.danielsson(m, pol)
        else:
            oracle.separable(m, pol, nthreads=threads)
    dt = time.perf_counter() - t0
    what = (f"the whole {images[0][0].shape[0]}x{images[0][0].shape[1]} image" if len(images) == 1
            else f"all {len(images)} images of the batch, one after the other")
    how = ("the oracle's two raster scans of the chamfer 4-3 transform" if metric == 3 else
           "the oracle's two propagation scans of Danielsson's transform" if metric == "danielsson"
           else "the oracle's separable transform (vertical pass + lower envelope + fill)")
    return {"value": round(units_px / dt / 1e9, 5), "unit": "Gpixel/s", "cores": threads,
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"one full pass of {how} over {what}, {threads} thread(s), {dt:.2f} s"}


def approx_error(mask, pol, D, ws, stream, scale=3.0, squared=False):
    """An approximate distance (chamfer 4-3 d / 3, or the square root of
    Danielsson's d^2) against the exact Euclidean distance of the same image
    (computed once by edt_sq, outside the timed region), over the pixels that
    have a site: mean and largest absolute error in pixels, the range of the
    relative error, and the share of pixels where they differ."""
    import torch
    import paper_2106_03503_amd as edt
    E = edt.sq(mask, polarity=pol, workspace=ws, stream=stream)
    ok = E != edt.EDT_INF_SQ
    c = D[ok].double().sqrt() if squared else D[ok].double() / scale
    e = E[ok].double().sqrt()
    err = c - e
    pos = e > 0
    rel = err[pos] / e[pos]
    out = {"vs": "exact Euclidean distance (edt_sq, squared Euclidean metric)",
           "mean_abs_px": round(float(err.abs().mean()), 4),
           "max_abs_px": round(float(err.abs().max()), 4),
           "rel_min": round(float(rel.min()), 4), "rel_max": round(float(rel.max()), 4),
           "frac_differs": round(float((err.abs() > 1e-9).double().mean()), 4)}
    torch.cuda.synchronize()
    return out


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


def timed(step, steps, warmup, profile=True):
    """Warm up, then time `steps` calls between two device synchronisations;
    returns (ms per step, per-kernel {name: (launches, total ms)})."""
    import torch
    import paper_2106_03503_amd as edt
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if profile:
        edt.profile_begin()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = edt.profile_end() if profile else {}
    return (t1 - t0) * 1e3 / steps, kt


def roofline(kt, algo_per_launch, workload):
    dom = max(kt, key=lambda k: kt[k][1])
    launches, total_ms = kt[dom]
    avg_ms = total_ms / launches
    algo = algo_per_launch(dom)
    achieved = algo / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profiles(dom, workload),
            "algorithmic_bytes_per_launch": int(algo), "avg_launch_ms": round(avg_ms, 4)}


def path_hbm(nbytes: int, ms: float) -> dict:
    """The whole step against the bytes the method must move (path_bytes)."""
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"bytes_per_step": int(nbytes), "achieved_GBs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "basis": "mask read once, outputs written once, int16 nearest site row of each "
                     "column holding a site written and read once (band bits and carries for "
                     "batch images of the one-lane-per-row pass)"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def base_line(args, value, ms, config):
    return {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic", "config": config,
    }


def run_single(args):
    import torch
    import paper_2106_03503_amd as edt
    wl = SINGLE[args.workload]
    H, W, pol = wl["H"], wl["W"], wl["polarity"]
    mask_np = make_mask(args.workload)
    n = site_columns(mask_np, pol)
    dev = torch.device("cuda:0")
    mask = torch.from_numpy(mask_np).to(dev)
    D = torch.empty((H, W), dtype=torch.int32, device=dev)
    F = torch.empty((H, W), dtype=torch.int32, device=dev)
    ws = torch.empty(edt.workspace_bytes(H, W, True), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    sq_only = wl.get("call") == "edt_sq"
    metric = wl.get("metric", 0)

    conn = wl.get("regions", 0)
    L = torch.empty((H, W), dtype=torch.int32, device=dev) if conn else None

    dan = wl.get("call") == "edt_danielsson"
    f32 = wl.get("call") == "edt_dist_f32"
    Df = torch.empty((H, W), dtype=torch.float32, device=dev) if f32 else None

    def step():
        if f32:
            edt.dist_f32(mask, polarity=pol, want_feature=True, out_dist=Df, out_feat=F,
                         workspace=ws, stream=stream)
            return
        if dan:
            edt.danielsson(mask, polarity=pol, out_dist=D, out_rel=F, stream=stream)
            return
        if sq_only:
            edt.sq(mask, polarity=pol, metric=metric, out=D, workspace=ws, stream=stream)
        else:
            edt.feature(mask, polarity=pol, metric=metric, out_dist=D, out_feat=F, workspace=ws,
                        stream=stream)
        if conn:
            edt.regions(mask, F, polarity=pol, connectivity=conn, out=L, stream=stream)

    # value from K plain steps; the per-kernel HIP events (two per launch) add
    # about 55 us to a step, so kernel durations come from K more steps with
    # the events on
    ms, _ = timed(step, args.steps, args.warmup, profile=False)
    ms_prof, kt = timed(step, args.steps, 1, profile=True)
    px = H * W
    out = base_line(args, px / (ms * 1e-3) / 1e9, ms,
                    {"workload": wl["desc"], "H": H, "W": W, "polarity": pol,
                     "call": "edt_danielsson" if dan else "edt_dist_f32" if f32 else (
                         ("edt_sq" if sq_only else "edt_feature")
                         + (f" + edt_regions ({conn}-neighbourhood)" if conn else "")),
                     "metric": "Danielsson's approximate squared distance" if dan else
                               ["squared Euclidean", "city-block", "chessboard",
                                "chamfer 4-3"][metric],
                     "parallelism": "single GPU"})
    out["roofline"] = roofline(kt, lambda k: algo_bytes(k, H, W, n, with_dist=not sq_only),
                               args.workload)
    out["roofline"]["scope"] = "the dominant kernel of the step"
    if not dan and not conn:
        out["path_hbm"] = path_hbm(path_bytes(H, W, n, with_feature=not sq_only), ms)
    out["roofline"]["kernel_timing"] = (f"HIP events around every launch, in a second timed "
                                        f"region of {args.steps} steps")
    out["kernels_ms_per_step"] = {k: round(v[1] / args.steps, 4) for k, v in sorted(kt.items())}
    out["ms_per_step_with_kernel_events"] = round(ms_prof, 4)
    if metric == 3:
        out["approx_error"] = approx_error(mask, pol, D, ws, stream)
    if dan:
        out["approx_error"] = approx_error(mask, pol, D, ws, stream, scale=1.0, squared=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline([(mask_np, pol)], px, "danielsson" if dan else metric)
    return out


def run_batch(args):
    import numpy as np
    import torch
    import paper_2106_03503_amd as edt
    from paper_2106_03503_amd import _lib
    import workloads
    imgs = workloads.ragged_batch(2048)
    dev = torch.device("cuda:0")
    plan = edt.BatchPlan([(m.shape[0], m.shape[1], p, True) for m, p in imgs])
    mask = plan.pack([m for m, _ in imgs], dev)
    D, F = plan.outputs(dev)
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    px = sum(m.size for m, _ in imgs)

    tune = None
    if args.schedule:
        knobs = [int(x) for x in args.schedule.split(",")]
        lw, lf, br, wsg, tr = (knobs + [1, 1, 0, 0][len(knobs) - 1:])[:5]
        plan.set_schedule(lw, bool(lf), br, bool(wsg), bool(tr))
        tune = {"fixed": {"lane_w": lw, "largest_first": bool(lf), "branches": br,
                          "wide_single": bool(wsg), "transpose": bool(tr)}}
    elif not args.no_autotune:
        cands, chosen = plan.autotune(mask, D, F, workspace=ws, stream=stream)
        tune = {"candidates": cands, "chosen": chosen}

    def step():
        plan.submit(mask, D, F, workspace=ws, stream=stream)

    ms, _ = timed(step, args.steps, args.warmup, profile=False)      # graph replays
    ms_prof, kt = timed(step, max(3, args.steps // 4), 1, profile=True)  # per-kernel times

    # the same images, one edt_feature call each (plain per-image launches)
    wsz = max(edt.workspace_bytes(m.shape[0], m.shape[1]) for m, _ in imgs)
    ws1 = torch.empty(wsz, dtype=torch.uint8, device=dev)
    calls = []
    for q, (m, pol) in enumerate(imgs):
        h, w = m.shape
        calls.append((mask.data_ptr() + plan.mask_off[q], h, w, plan.mask_pitch[q], pol, 0,
                      D.data_ptr() + 4 * plan.out_off[q], F.data_ptr() + 4 * plan.out_off[q],
                      plan.out_pitch[q], ws1.data_ptr(), wsz, stream.cuda_stream))
    fn = _lib.lib.edt_feature

    def per_image():
        for c in calls:
            if fn(*c) != 0:
                raise RuntimeError("edt_feature failed")

    ms_single = None
    if not args.no_per_image:
        ms_single, _ = timed(per_image, max(2, args.steps // 5), 1, profile=False)

    ns = [site_columns(m, p) for m, p in imgs]
    out = base_line(args, px / (ms * 1e-3) / 1e9, ms,
                    {"workload": BATCH_DESC, "images": len(imgs), "pixels": int(px),
                     "call": "edt_batch_submit (graph replay)", "parallelism": "single GPU"})
    out["roofline"] = roofline(
        kt, lambda k: sum(algo_bytes(k, m.shape[0], m.shape[1], n) for (m, _), n in zip(imgs, ns)),
        args.workload)
    out["roofline"]["kernel_timing"] = (
        f"HIP events around every launch (the plan launches its kernels one by one while they "
        f"are on), in a second timed region of {max(3, args.steps // 4)} steps")
    out["roofline"]["scope"] = "the dominant kernel of the step"
    # the images the chosen schedule gives the one-lane-per-row pass
    knobs = (tune["fixed"] if tune and "fixed" in tune
             else tune["candidates"][tune["chosen"]] if tune else {"lane_w": 1024})
    lane_w = knobs["lane_w"]
    out["path_hbm"] = path_hbm(sum(path_bytes(m.shape[0], m.shape[1], n,
                                              lanes=m.shape[1] <= lane_w and m.shape[0] <= 4096)
                                   for (m, _), n in zip(imgs, ns)), ms)
    if ms_single is not None:
        out["per_image"] = {"value": round(px / (ms_single * 1e-3) / 1e9, 3),
                            "ms_per_step": round(ms_single, 4), "call": "edt_feature per image"}
        out["batched_over_per_image"] = round(ms_single / ms, 2)
    out["kernels_ms_per_step"] = {k: round(v[1] / max(3, args.steps // 4), 4)
                                  for k, v in sorted(kt.items())}
    if tune is not None:
        out["autotune"] = tune
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(imgs, px)
    plan.close()
    return out


def run_serve(args):
    import numpy as np
    import torch
    import paper_2106_03503_amd as edt
    from paper_2106_03503_amd import _lib
    import workloads
    burst = args.rate <= 0  # every request at t = 0: the server's capacity
    # arrival times drawn at 1000/s and scaled: the masks do not depend on the rate
    reqs = workloads.serving_requests(args.requests, 1000.0)
    scale = 0.0 if burst else 1000.0 / args.rate
    dev = torch.device("cuda:0")
    print(f"serve: drawing {len(reqs)} request masks", file=sys.stderr, flush=True)
    masks_np = [workloads.request_mask(r) for r in reqs]
    masks = [torch.from_numpy(m).to(dev) for m in masks_np]
    outs = []
    for r in reqs:
        s_ = r["side"]
        D = torch.empty((s_, s_), dtype=torch.int32, device=dev)
        F = torch.empty((s_, s_), dtype=torch.int32, device=dev) if r["want_feature"] else None
        outs.append((D, F))
    torch.cuda.synchronize()
    px = sum(m.numel() for m in masks)
    bytes_path = sum(path_bytes(r["side"], r["side"], site_columns(m, r["polarity"]),
                                r["want_feature"]) for m, r in zip(masks_np, reqs))
    budget = int(args.budget_gib * (1 << 30))
    stream = torch.cuda.current_stream()

    def replay(srv, sc):
        t0 = time.perf_counter()
        tickets = []
        for r, m, (D, F) in zip(reqs, masks, outs):
            while time.perf_counter() - t0 < r["t"] * sc:
                pass
            while True:
                try:
                    tickets.append(srv.submit_raw(m, D, F, polarity=r["polarity"], stream=stream))
                    break
                except edt.EDTError as e:
                    if e.status != -5:  # busy: retry
                        raise
                    time.sleep(50e-6)
        for t in tickets:
            srv.wait(t)
        return time.perf_counter() - t0, srv.stats()

    def replays(sc, k, label):
        runs = []
        for q in range(k):
            with edt.Server(budget, n_streams=args.streams) as srv:
                wall, st = replay(srv, sc)
            runs.append((wall, st))
            print(f"serve: {label} replay {q + 1}/{k} {wall * 1e3:.1f} ms", file=sys.stderr,
                  flush=True)
        walls = [w for w, _ in runs]
        med = sorted(range(len(runs)), key=lambda q: walls[q])[len(runs) // 2]
        return runs[med][0], runs[med][1], walls

    if args.warmup > 0:  # one warm-up replay
        with edt.Server(budget, n_streams=args.streams) as srv:
            replay(srv, scale)
    wall, st, walls = replays(scale, args.steps, "burst" if burst else f"{args.rate:g}/s")
    value = st["gpix_per_s"]

    # the same requests one after the other through edt_feature / edt_sq on one
    # stream (plain per-image launches)
    wsz = max(edt.workspace_bytes(r["side"], r["side"]) for r in reqs)
    ws1 = torch.empty(wsz, dtype=torch.uint8, device=dev)
    lib = _lib.lib

    def per_image():
        for r, m, (D, F) in zip(reqs, masks, outs):
            s_ = r["side"]
            if F is not None:
                st_ = lib.edt_feature(m.data_ptr(), s_, s_, s_, r["polarity"], 0, D.data_ptr(),
                                      F.data_ptr(), s_, ws1.data_ptr(), wsz, stream.cuda_stream)
            else:
                st_ = lib.edt_sq(m.data_ptr(), s_, s_, s_, r["polarity"], 0, D.data_ptr(), s_,
                                 ws1.data_ptr(), wsz, stream.cuda_stream)
            if st_ != 0:
                raise RuntimeError("per-image call failed")
    ms_single, _ = timed(per_image, 2, 1, profile=False)

    out = base_line(args, value, wall * 1e3,
                    {"workload": SERVE_DESC.format(n=len(reqs), rate=args.rate) if not burst else
                     SERVE_DESC.replace("arriving as a Poisson stream at {rate:g}/s",
                                        "submitted at once").format(n=len(reqs)),
                     "requests": len(reqs), "pixels": int(px), "rate_per_s": args.rate,
                     "hbm_budget_GiB": args.budget_gib, "streams": args.streams,
                     "call": "edt_serve_submit / edt_serve_wait", "parallelism": "single GPU"})
    out["scaling"] = "strong"
    offered = px / (reqs[-1]["t"] * scale) / 1e9 if not burst else None
    out["serve"] = serve_summary(st, walls, offered)
    out["per_image"] = {"value": round(px / (ms_single * 1e-3) / 1e9, 3),
                        "ms_per_pass": round(ms_single, 3),
                        "call": "edt_feature / edt_sq per request, one stream"}
    out["served_over_per_image"] = round(value / out["per_image"]["value"], 2)
    out["path_hbm"] = path_hbm(bytes_path, wall * 1e3)
    if args.capacity and not burst:
        cwall, cst, cwalls = replays(0.0, args.steps, "burst")
        out["capacity"] = {"gpix_per_s": round(cst["gpix_per_s"], 3),
                           "over_per_image": round(cst["gpix_per_s"] / out["per_image"]["value"], 2),
                           **serve_summary(cst, cwalls, None)}
    if args.sweep and not burst:
        # the same requests at other rates: the arrival times scale with 1/rate
        sweep = []
        for rate in SWEEP_RATES:
            with edt.Server(budget, n_streams=args.streams) as srv:
                w, st_r = replay(srv, 1000.0 / rate)
            sweep.append({"rate_per_s": rate,
                          "offered_gpix_per_s": round(px / (reqs[-1]["t"] * 1000.0 / rate) / 1e9, 3),
                          "gpix_per_s": round(st_r["gpix_per_s"], 3),
                          "p50_ms": round(st_r["p50_ns"] / 1e6, 3),
                          "p99_ms": round(st_r["p99_ns"] / 1e6, 3),
                          "launches": st_r["launches"]})
            print(f"serve: sweep {rate:g}/s {w * 1e3:.1f} ms", file=sys.stderr, flush=True)
        out["serve"]["sweep"] = sweep
    if not args.no_cpu:
        # a bounded sample: the requests in arrival order up to ~1e8 pixels
        sample, acc = [], 0
        for m, r in zip(masks_np, reqs):
            if acc + m.size > 1e8 and sample:
                break
            sample.append((m, r["polarity"]))
            acc += m.size
        cb = cpu_baseline(sample, acc)
        cb["sample"] = (f"the first {len(sample)} requests of the stream ({acc} pixels), "
                        f"one after the other: " + cb["sample"])
        out["cpu_baseline"] = cb
    return out


def serve_summary(st, walls, offered):
    return {"offered_gpix_per_s": round(offered, 3) if offered else "burst",
            "p50_ms": round(st["p50_ns"] / 1e6, 3), "p99_ms": round(st["p99_ns"] / 1e6, 3),
            "mean_ms": round(st["mean_ns"] / 1e6, 3), "max_ms": round(st["max_ns"] / 1e6, 3),
            "launches": st["launches"], "done": st["done"], "failed": st["failed"],
            "rejected_busy": st["rejected_busy"],
            "hbm_high_water_GiB": round(st["hbm_high_water"] / (1 << 30), 3),
            "replay_ms": [round(w * 1e3, 2) for w in walls]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="points16k",
                    choices=sorted(list(SINGLE) + ["batch2048", "serve"]))
    ap.add_argument("--rate", type=float, default=5000.0,
                    help="serve: requests per second (0: all at once, the capacity)")
    ap.add_argument("--requests", type=int, default=400, help="serve: requests per replay")
    ap.add_argument("--budget-gib", type=float, default=16.0, help="serve: memory budget")
    ap.add_argument("--streams", type=int, default=4, help="serve: server streams")
    ap.add_argument("--sweep", action="store_true",
                    help="serve: also replay the same requests at 100..5000 req/s")
    ap.add_argument("--no-cpu", action="store_true", help="skip the cpu_baseline leg")
    ap.add_argument("--no-per-image", action="store_true",
                    help="batch2048: skip the per-image edt_feature leg")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batch2048: keep the default schedule instead of autotuning it")
    ap.add_argument("--schedule", default="",
                    help="batch2048: use this schedule 'lane_w,largest_first[,branches"
                         "[,wide_single[,transpose]]]' instead of autotuning (e.g. 1024,1,2)")
    ap.add_argument("--capacity", action="store_true",
                    help="serve: also replay the requests all at once (the capacity)")
    ap.add_argument("--no-extras", action="store_true",
                    help="points16k: skip the batch2048, serve and dense16k legs that the "
                         "default line carries beside the headline")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported.",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.steps)
        return
    if args.workload == "batch2048":
        out = run_batch(args)
    elif args.workload == "serve":
        out = run_serve(args)
    else:
        out = run_single(args)
        if args.workload == "points16k" and not args.no_extras:
            out.update(extras(args))
    print(json.dumps(out), flush=True)


def leg_args(args, **kw):
    a = argparse.Namespace(**vars(args))
    a.no_cpu = True
    for k, v in kw.items():
        setattr(a, k, v)
    return a


def extras(args):
    """The rest of the metric beside the headline: the ragged batch against
    per-image launches, the request server against per-image launches of the
    same requests, and a dense single image at 16384^2 (shorter runs)."""
    keep = ("value", "unit", "ms_per_step", "config", "roofline", "path_hbm",
            "kernels_ms_per_step", "per_image")
    print("bench: batch2048 leg", file=sys.stderr, flush=True)
    b = run_batch(leg_args(args, workload="batch2048", steps=10, warmup=2, schedule="",
                           no_autotune=False, no_per_image=False))
    batch = {k: b[k] for k in keep if k in b}
    batch["batched_over_per_image"] = b.get("batched_over_per_image")
    batch["autotune_chosen"] = b["autotune"]["candidates"][b["autotune"]["chosen"]]
    print("bench: serve leg", file=sys.stderr, flush=True)
    v = run_serve(leg_args(args, workload="serve", steps=3, warmup=1, rate=5000.0,
                           requests=400, capacity=True, sweep=False))
    serve = {"value": v["value"], "unit": v["unit"], "config": v["config"],
             "at_5000_per_s": v["serve"], "capacity": v["capacity"], "per_image": v["per_image"],
             "served_over_per_image": v["served_over_per_image"], "path_hbm": v["path_hbm"]}
    print("bench: dense16k leg", file=sys.stderr, flush=True)
    d = run_single(leg_args(args, workload="dense16k", steps=20, warmup=3))
    dense = {k: d[k] for k in keep if k in d}
    return {"batch2048": batch, "serve": serve, "dense16k": dense}


if __name__ == "__main__":
    main()
