#!/usr/bin/env python
"""Throughput of the clustering hot path on one MI355X.

One step = Euclidean MST (Boruvka screen + exact recheck + contraction + FP64
lengths + rooting) followed by the optimal k-subpartition of the tree
(speculative bisection over Algorithm 1, labels), on the image-like workload
n = 200,000 points, d = 784, k = 10, sigma = median MST edge, points resident
in HBM before the timed region.  Prints one JSON line (rank 0).

    python bench.py [--steps K] [--warmup W] [--precision fp32|bf16]
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

METRIC = "points/s for MST+subpartition (n=200k,d=784) BF16-refined vs FP32; % MFMA peak"
WORKLOAD = 3
PEAKS_TFLOPS = {"int8": 5000.0, "fp8": 5000.0, "bf16": 2500.0, "fp32": 157.3}  # dense MFMA peaks of MI355X
# one screen launch = the diagonal tile pairs' dispatch followed by the off-diagonal one
SCREEN_KERNEL = "k_screen_pairs<%s> (diagonal + off-diagonal dispatch)"
SCREEN_SOURCES = ["paper_1702_04739_amd/csrc/screen_pairs.hip", "paper_1702_04739_amd/csrc/screen.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def screen_source_sha():
    h = hashlib.sha256()
    for p in SCREEN_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(precision):
    """HBM bytes per screen launch from committed rocprofv3 counter runs, or
    None when absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "screen_%s_traffic.json" % precision)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha") != screen_source_sha():
        return None
    return rec.get("hbm_bytes_per_launch")


def traffic_report(fetch_dir, write_dir, precision, copy_mib):
    """Per-launch HBM bytes of the screen kernel from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch), each scaled by what the
    same counter reads for the plain device copy of copy_mib MiB that the
    profiled command ran first (--calibrate-copy)."""
    import csv
    import glob

    prefix = "k_screen_pairs<%d, " % {"fp32": 0, "bf16": 1, "fp8": 2, "int8": 3}[precision]

    def per_kernel(d, counter):
        """Summed counter over the screen's dispatches (diagonal and
        off-diagonal), the number of screen rounds, and the copy's value."""
        total, rounds, copy = 0.0, 0, None
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"])
                if prefix in r["Kernel_Name"]:
                    total += v
                    rounds += 1 if (prefix + "false") in r["Kernel_Name"] else 0
                elif "copyBuffer" in r["Kernel_Name"] and copy is None and v > 0.25 * copy_mib * 1024:
                    copy = v
        return total, rounds, copy

    ft, fr, fc = per_kernel(fetch_dir, "FETCH_SIZE")
    wt, wr, wc = per_kernel(write_dir, "WRITE_SIZE")
    nbytes = copy_mib * (1 << 20)
    f_scale = nbytes / (fc * 1024.0)
    w_scale = nbytes / (wc * 1024.0)
    fetch = ft / fr * 1024.0 * f_scale
    write = wt / wr * 1024.0 * w_scale
    rec = {"kernel": SCREEN_KERNEL % precision, "source_sha": screen_source_sha(),
           "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "hbm_bytes_per_launch": fetch + write, "launches": fr,
           "copy_calibration": {"bytes": nbytes, "fetch_kib": fc, "write_kib": wc, "fetch_scale": f_scale,
                                "write_scale": w_scale},
           "commands": [
               "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE -f csv -d <fetch_dir> -o run -- python3 "
               "<repo>/bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-compare --all-k 0 --paper-prim-n 0 "
               "--calibrate-copy %d --precision %s" % (copy_mib, precision),
               "(the same with --pmc WRITE_SIZE -d <write_dir>)",
               "python bench.py --traffic-report <fetch_dir> <write_dir> --precision %s --calibrate-copy %d"
               % (precision, copy_mib)],
           "note": "FETCH_SIZE and WRITE_SIZE summed over the screen's dispatches of every screened round (the "
                   "plain first round, the second round that also builds the neighbour lists, the final round) "
                   "and divided by the number of those rounds; each counter is scaled by what it reads for the "
                   "plain device copy run first in the same process (FETCH_SIZE counts half the copied bytes, "
                   "WRITE_SIZE all).  The algorithmic minimum is one read of the BF16 representation (n_pad x "
                   "d_pad x 2 bytes, 314 MB) per screen; the rest are tile re-reads that miss L2."}
    return rec


def cpu_baseline(n_full, k, sample_n):
    """The FP64 oracle (single thread) on a subsample of the same recipe; the
    O(n^2 d) MST cost is scaled to the full n."""
    import oracle
    from paper_1702_04739_amd import datagen
    X = datagen.config(WORKLOAD, n=sample_n)
    t0 = time.perf_counter()
    parent, length, _, _ = oracle.prim_mst(X)
    t1 = time.perf_counter()
    oracle.subpartition(parent, length, k)
    t2 = time.perf_counter()
    t_full = (t1 - t0) * (n_full / sample_n) ** 2 + (t2 - t1) * (n_full / sample_n)
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": n_full / t_full,
        "unit": "points/s",
        "cores": 1,
        "cpu": cpu_model,
        "kind": "oracle",
        "sample": "same recipe at n=%d (MST %.2f s, tree search %.3f s, single thread); MST time scaled by "
                  "(n/%d)^2 and tree time by n/%d to n=%d" % (sample_n, t1 - t0, t2 - t1, sample_n, sample_n, n_full),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16", "fp8", "int8"])
    ap.add_argument("--no-compare", action="store_true", help="skip the FP32 and INT8 screen comparison steps")
    ap.add_argument("--recheck", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--n", type=int, default=None, help="smaller n of the same recipe (not the benchmark)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--paper-prim-n", type=int, default=20000, metavar="M",
                    help="time the paper's Prim MST against this path's MST on an M-point sample (0: skip)")
    ap.add_argument("--all-k", type=int, default=10, metavar="K",
                    help="after the timed steps, time the all-k sweep k = 2..K on the last tree (0: skip)")
    ap.add_argument("--cpu-sample-n", type=int, default=8000)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before the steps, run one plain device copy of MIB MiB (reference for HBM counters)")
    ap.add_argument("--traffic-report", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs into profiles/screen_<precision>_traffic.json and exit")
    args = ap.parse_args()

    if args.traffic_report:
        rec = traffic_report(args.traffic_report[0], args.traffic_report[1], args.precision,
                             args.calibrate_copy or 1024)
        path = os.path.join(ROOT, "profiles", "screen_%s_traffic.json" % args.precision)
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the MST screen shards over tile pairs with one min-all-reduce per "
              "Boruvka round, but no multi-GPU path is built; run with --gpus 1", flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1702_04739_amd as iso
    from paper_1702_04739_amd import _lib, datagen

    cfg = datagen.CONFIGS[WORKLOAD]
    n = args.n or cfg["n"]
    d, k = cfg["d"], cfg["k"]
    log("generating %s n=%d d=%d" % (cfg["name"], n, d))
    X = torch.from_numpy(datagen.config(WORKLOAD, n=n)).cuda()
    torch.cuda.synchronize()

    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read, %d bytes written" % (src.numel() * 4, dst.numel() * 4))
        del src, dst

    def step():
        return iso.cluster(X, k, precision=args.precision, recheck=args.recheck)

    for w in range(args.warmup):
        log("warmup %d" % w)
        step()
    torch.cuda.synchronize()
    _lib.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for s in range(args.steps):
        last = step()
        log("step %d done" % s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    T = _lib.timing_read()
    _lib.timing_enable(False)
    ms = (t1 - t0) * 1e3 / args.steps
    value = n / (ms / 1e3)

    labels, ik, info = last
    flops = 2.0 * d * T["screen_pairs"]
    achieved = flops / (T["screen_ms"] * 1e-3) / 1e12 if T["screen_ms"] > 0 else None
    bound, peak = "mfma", PEAKS_TFLOPS[args.precision]
    launches = max(T["screen_launches"], 1)
    tb = traffic_from_profiles(args.precision)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": cfg["name"] if args.n is None else "%s@n=%d" % (cfg["name"], n), "n": n, "d": d,
                   "k": k, "sigma": "median MST edge", "screen": args.precision, "recheck": args.recheck,
                   "tree": "f64", "parallelism": "none"},
        "roofline": {
            "kernel": SCREEN_KERNEL % args.precision,
            "bound": bound,
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": (achieved / peak) if achieved else None,
            "traffic": tb,
            "flops_per_launch": flops / launches,
            "avg_launch_ms": T["screen_ms"] / launches,
            "launches": T["screen_launches"],
        },
        "phases": {"mst_ms_per_step": T["mst_ms"] / max(T["mst_calls"], 1),
                   "sub_ms_per_step": T["sub_ms"] / max(T["sub_calls"], 1),
                   "screen_ms_per_step": T["screen_ms"] / args.steps,
                   "rounds": info["mst"]["rounds"], "list_rounds": info["mst"]["list_rounds"],
                   "candidates": info["mst"]["candidates"],
                   "rescanned_rows": info["mst"]["rescanned_rows"], "bisection_iters": info["sub"]["iters"],
                   "passes": info["sub"]["passes"], "max_depth": info["sub"]["max_depth"],
                   "i_k": ik, "mst_weight": info["mst"]["mst_weight"]},
    }
    if not args.no_compare:
        # the same step with other screen precisions (FP32: the reference
        # precision; INT8: exact integer Gram tiles, for 8-bit data like this
        # workload's q/256 coordinates), one warm-up + one step each
        out["compare"] = []
        for prec in ("fp32", "int8"):
            if prec == args.precision:
                continue
            log("comparison: %s screen, 1 warm-up + 1 step" % prec)
            iso.cluster(X, k, precision=prec, recheck=args.recheck)
            torch.cuda.synchronize()
            c0 = time.perf_counter()
            labc, ikc, infoc = iso.cluster(X, k, precision=prec, recheck=args.recheck)
            torch.cuda.synchronize()
            c1 = time.perf_counter()
            out["compare"].append({"screen": prec, "value": n / (c1 - c0), "ms_per_step": (c1 - c0) * 1e3,
                                   "value_ratio": value / (n / (c1 - c0)),
                                   "same_tree": bool(torch.equal(infoc["parent"], info["parent"])),
                                   "same_labels": bool(torch.equal(labc, labels)), "i_k": ikc})
    if args.paper_prim_n > 0:
        # the paper's own MST construction (Prim, one min-reduction per step)
        # against this path's Boruvka MST, on a subsample of the same recipe
        m = min(args.paper_prim_n, n)
        Xs = torch.from_numpy(datagen.config(WORKLOAD, n=m)).cuda()
        iso.mst(Xs, precision=args.precision, recheck="fp64")
        torch.cuda.synchronize()
        b0 = time.perf_counter()
        bp, bl, _ = iso.mst(Xs, precision=args.precision, recheck="fp64")
        torch.cuda.synchronize()
        b1 = time.perf_counter()
        pp, pl = iso.mst_prim(Xs)
        torch.cuda.synchronize()
        b2 = time.perf_counter()
        out["paper_mst"] = {"n": m, "algorithm": "Prim from vertex 0, FP64 (Algorithm 3)", "prim_ms": (b2 - b1) * 1e3,
                            "boruvka_ms": (b1 - b0) * 1e3, "boruvka_screen": args.precision, "recheck": "fp64",
                            "same_tree": bool(torch.equal(pp, bp) and torch.equal(pl, bl))}
    if args.all_k >= 2:
        # every k = 2 .. K of the last step's tree in shared passes, against
        # separate single-k calls (outside the timed region)
        parent, length = last[2]["parent"], last[2]["length"]
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        ik_all, _, passes = iso.subpartition_all_k(parent, length, args.all_k)
        torch.cuda.synchronize()
        a1 = time.perf_counter()
        sep_passes = 0
        for kk in range(2, args.all_k + 1):
            _, ik1, info1 = iso.isoperimetric_subpartition(parent, length, kk)
            sep_passes += info1["passes"]
            if ik1 != ik_all[kk - 2]:
                raise RuntimeError("all-k sweep differs from the single-k result at k=%d" % kk)
        torch.cuda.synchronize()
        a2 = time.perf_counter()
        out["all_k"] = {"kmax": args.all_k, "ms": (a1 - a0) * 1e3, "passes": passes,
                        "separate_calls_ms": (a2 - a1) * 1e3, "separate_calls_passes": sep_passes,
                        "i_k": [float(v) for v in ik_all]}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, n=%d sample)" % args.cpu_sample_n)
        out["cpu_baseline"] = cpu_baseline(n, k, args.cpu_sample_n)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
