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
# one screen "launch" = one screened round: its two phases (the tile pairs whose
# bounding balls meet, then those the bound does not exclude), each with the
# off-diagonal dispatch and the diagonal (masked) one
SCREEN_KERNEL = "k_screen_pairs<%s> (one screened round: both phases, masked + unmasked dispatches)"
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
        """Summed counter over the screen's dispatches (both phases of a round,
        diagonal and off-diagonal), the number of screened rounds, and the
        copy's value.  A screened round is a run of consecutive screen
        dispatches of one mode (the profiled step's rounds are plain, list
        building and final, so the mode changes at every round)."""
        import re
        total, copy, modes = 0.0, None, []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"])
                if prefix in r["Kernel_Name"]:
                    total += v
                    m = re.search(r"k_screen_pairs<\d+, \w+, (\d+)", r["Kernel_Name"])
                    modes.append((int(r["Dispatch_Id"]), m.group(1) if m else "?"))
                elif "copyBuffer" in r["Kernel_Name"] and copy is None and v > 0.25 * copy_mib * 1024:
                    copy = v
        modes.sort()
        rounds = sum(1 for i, (_, md) in enumerate(modes) if i == 0 or md != modes[i - 1][1])
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
               "<repo>/bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-compare --all-k 0 --paper-prim-n 0 "
               "--no-extras --calibrate-copy %d --precision %s" % (copy_mib, precision),
               "(the same with --pmc WRITE_SIZE -d <write_dir>)",
               "python bench.py --traffic-report <fetch_dir> <write_dir> --precision %s --calibrate-copy %d"
               % (precision, copy_mib)],
           "note": "FETCH_SIZE and WRITE_SIZE summed over the screen's dispatches of every screened round (the "
                   "plain first round, the second round that also builds the neighbour lists, the final round; "
                   "each round's two phases and its masked and unmasked dispatches) "
                   "and divided by the number of those rounds; each counter is scaled by what it reads for the "
                   "plain device copy run first in the same process (FETCH_SIZE counts half the copied bytes, "
                   "WRITE_SIZE all).  The algorithmic minimum is one read of the BF16 representation (n_pad x "
                   "d_pad x 2 bytes, 314 MB) per screen; the rest are tile re-reads that miss L2."}
    return rec


def kernel_traffic_table(fetch_dir, write_dir, stats_csv, copy_mib, patterns=()):
    """Markdown table of HBM bytes and rates per kernel from two rocprofv3
    --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, each scaled by
    what it reads for the plain device copy of copy_mib MiB run first) and the
    kernel statistics of a --kernel-trace --stats run of the same command."""
    import collections
    import csv
    import glob
    import re

    def per_kernel(d, counter):
        tot, calls, copy = collections.defaultdict(float), collections.defaultdict(int), None
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter:
                    continue
                v, k = float(r["Counter_Value"]), r["Kernel_Name"]
                if "copyBuffer" in k and copy is None and v > 0.25 * copy_mib * 1024:
                    copy = v
                    continue
                tot[k] += v
                calls[k] += 1
        return tot, calls, copy

    ft, fc, fcopy = per_kernel(fetch_dir, "FETCH_SIZE")
    wt, _, wcopy = per_kernel(write_dir, "WRITE_SIZE")
    nb = copy_mib * (1 << 20)
    fs, ws = nb / (fcopy * 1024.0), nb / (wcopy * 1024.0)
    dur = {r["Name"]: float(r["TotalDurationNs"]) for r in csv.DictReader(open(stats_csv))}
    lines = ["copy calibration: FETCH_SIZE x %.4f, WRITE_SIZE x %.4f" % (fs, ws), "",
             "| kernel | calls | fetch MB | write MB | kernel ms | GB/s |", "|---|---:|---:|---:|---:|---:|"]
    for k in sorted(set(ft) | set(wt), key=lambda k: -(ft.get(k, 0) + wt.get(k, 0))):
        m = re.search(r"(k_\w+|__amd\w+)(<[^()]*>)?", k)
        name = m.group(0) if m else k[:60]
        if patterns and not any(p in name for p in patterns):
            continue
        fb, wb, ns = ft.get(k, 0) * 1024 * fs, wt.get(k, 0) * 1024 * ws, dur.get(k, 0.0)
        lines.append("| `%s` | %d | %.1f | %.1f | %.3f | %s |" % (name, fc.get(k, 0), fb / 1e6, wb / 1e6, ns / 1e6,
                                                              "%.0f" % ((fb + wb) / ns) if ns > 0 else "-"))
    return "\n".join(lines)


def cpu_baseline(n_full, k, sample_ns, tree=None):
    """The FP64 oracle (single thread) on subsamples of the same recipe: its
    O(n^2 d) MST time is measured at each sample size, the exponent fitted
    between the two, and the largest sample's time scaled by (n/sample)^2.
    With ``tree`` (the timed step's parent and length arrays) the oracle's
    tree search also runs once at the full size, on that tree: its time enters
    the baseline unscaled, and its MISO_k is returned for the i_k check."""
    import math

    import oracle
    from paper_1702_04739_amd import datagen
    mst_s = []
    for m in sample_ns:
        X = datagen.config(WORKLOAD, n=m)
        t0 = time.perf_counter()
        parent, length, _, _ = oracle.prim_mst(X)
        mst_s.append(time.perf_counter() - t0)
    sample_n = sample_ns[-1]
    expo = (math.log(mst_s[-1] / mst_s[0]) / math.log(sample_ns[-1] / sample_ns[0])) if len(sample_ns) > 1 else None
    ik_oracle = None
    if tree is not None:
        t1 = time.perf_counter()
        ref = oracle.subpartition(tree[0], tree[1], k)
        t_tree = time.perf_counter() - t1
        ik_oracle = ref.i_k
        t_full = mst_s[-1] * (n_full / sample_n) ** 2 + t_tree
    else:
        t1 = time.perf_counter()
        oracle.subpartition(parent, length, k)
        t_tree = time.perf_counter() - t1
        t_full = mst_s[-1] * (n_full / sample_n) ** 2 + t_tree * (n_full / sample_n)
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
        "nproc": os.cpu_count(),
        "cpu": cpu_model,
        "kind": "oracle",
        "sample": "oracle MST (dense Prim, one thread) on the same recipe at n=%s: %s s (fitted exponent %s); "
                  "the n=%d time scaled by (n/%d)^2 to n=%d; tree search %s %.3f s" % (
                      "/".join(str(m) for m in sample_ns), "/".join("%.2f" % t for t in mst_s),
                      "%.2f" % expo if expo is not None else "n/a", sample_n, sample_n, n_full,
                      "on the timed step's tree at full n" if tree is not None else "at the sample size, scaled by n",
                      t_tree),
        "mst_sample_s": dict(zip([str(m) for m in sample_ns], mst_s)),
        "tree_search_s": t_tree,
        "_ik_oracle": ik_oracle,
    }


def _timed(fn, reps=3):
    """Median wall time (ms) of reps calls after one warm-up call, with device
    synchronisation around each."""
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    ts.sort()
    return ts[len(ts) // 2]


def oracle_digest_parity(info, n):
    """The timed step's MST against the FP64 oracle's, as stored by the
    oracle-only digest script: parent-array identity (SHA-256) and the
    relative error of the MST weight."""
    path = os.path.join(ROOT, "tests", "golden", "mst_digest_image-like_n%d.json" % n)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    p = info["parent"].cpu().numpy().astype("<i4")
    w = info["mst"]["mst_weight"]
    return {"oracle_digest": os.path.relpath(path, ROOT),
            "parent_identical_to_oracle": hashlib.sha256(p.tobytes()).hexdigest() == rec["parent_sha256"],
            "mst_weight": w, "mst_weight_oracle": rec["weight"],
            "mst_weight_rel_err_vs_oracle": abs(w - rec["weight"]) / rec["weight"]}


def other_workloads():
    """MST + subpartition at full size on the Gaussian-mixture (n = 2000,
    d = 16), anisotropic-mixture (n = 50,000, d = 64) and blobs (n = 20,000,
    d = 128) workloads with the FP32 screen and FP32 recheck (their values lie
    on no binary grid, so a BF16 request hands over to FP32); for the blobs
    workload also the forward pass plus the adjoint through MSTIsoCost (the
    gradient of W + i_k with respect to the points and sigma)."""
    import torch

    import paper_1702_04739_amd as iso
    from paper_1702_04739_amd import datagen
    out = {}
    for cfg in (1, 2, 5):
        c = datagen.CONFIGS[cfg]
        log("workload %s" % c["name"])
        X = torch.from_numpy(datagen.config(cfg)).cuda()
        ms = _timed(lambda: iso.cluster(X, c["k"], precision="fp32", recheck="fp32"))
        rec = {"n": c["n"], "d": c["d"], "k": c["k"], "screen": "fp32", "recheck": "fp32", "ms": ms,
               "points_per_s": c["n"] / (ms * 1e-3)}
        if cfg == 5:
            _, _, info = iso.cluster(X, c["k"])
            sig0 = info["sub"]["sigma"]

            def fwd_bwd():
                pts = X.clone().requires_grad_(True)
                sig = torch.tensor(sig0, dtype=torch.float64, device=X.device, requires_grad=True)
                W, I, _ = iso.MSTIsoCost.apply(pts, sig, c["k"])
                (W + I).backward()

            rec["forward_adjoint_ms"] = _timed(fwd_bwd)
            labels, _, info = iso.cluster(X, c["k"])
            rec["adjoint_ms"] = _timed(lambda: iso.adjoint(X, info["parent"], labels, info["sub"]["jstar"], sig0))
        out[c["name"]] = rec
    return out


def precision_sparse_communities():
    """The MST of the sparse-communities workload (n = 100,000, d = 4096) with
    the FP32, BF16 and FP8 screens (FP32 recheck): one call each after one
    FP32 warm-up.  The rows' norms are heavy tailed, so BF16 takes each pair's
    own error bound in its thresholds (pair_bounds); a screen whose bound is
    still too loose for the data (FP8) hands over to FP32 (screen_precision
    tells which one built the tree); the tree is the same in every case."""
    import torch

    import paper_1702_04739_amd as iso
    from paper_1702_04739_amd import datagen
    c = datagen.CONFIGS[4]
    log("precision comparison %s" % c["name"])
    X = torch.from_numpy(datagen.config(4)).cuda()
    iso.mst(X, precision="fp32")
    torch.cuda.synchronize()
    out = {"workload": c["name"], "n": c["n"], "d": c["d"], "recheck": "fp32"}
    ref = None
    for prec in ("fp32", "bf16", "fp8"):
        t0 = time.perf_counter()
        parent, _, info = iso.mst(X, precision=prec)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        if ref is None:
            ref = parent
        out[prec] = {"ms": ms, "points_per_s": c["n"] / (ms * 1e-3), "screen_precision": info["screen_precision"],
                     "pair_bounds": info["pair_bounds"], "rounds": info["rounds"],
                     "candidates_per_point": info["candidates"] / c["n"],
                     "rescanned_rows": info["rescanned_rows"], "same_tree_as_fp32": bool(torch.equal(parent, ref))}
    del X
    torch.cuda.empty_cache()
    return out


def graph_weights_timing():
    """Full-graph vertex weights and potential (eqs. 2.2-2.3, FP64 on the
    vector units) at the blobs (n = 20,000, d = 128) and anisotropic-mixture
    (n = 50,000, d = 64) sizes: time and FP64 rate, counting 3 d flops per
    ordered pair of points (difference, square, sum) against the 78.6 TFLOP/s
    FP64 vector peak."""
    import torch

    import paper_1702_04739_amd as iso
    from paper_1702_04739_amd import datagen
    out = {}
    for cfg in (5, 2):
        c = datagen.CONFIGS[cfg]
        log("graph weights %s" % c["name"])
        X = torch.from_numpy(datagen.config(cfg)).cuda()
        ms = _timed(lambda: iso.graph_weights(X, 1.0, alpha=0.05), reps=1)
        fl = 3.0 * c["d"] * c["n"] * (c["n"] - 1)
        out[c["name"]] = {"n": c["n"], "d": c["d"], "ms": ms, "fp64_tflops": fl / (ms * 1e-3) / 1e12,
                          "frac_fp64_peak": fl / (ms * 1e-3) / 78.6e12}
    return out


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
    ap.add_argument("--no-prune", action="store_true",
                    help="screen every tile pair (no bounding-ball test); the tree is the same")
    ap.add_argument("--paper-prim-n", type=int, default=20000, metavar="M",
                    help="time the paper's Prim MST against this path's MST on an M-point sample (0: skip)")
    ap.add_argument("--all-k", type=int, default=10, metavar="K",
                    help="after the timed steps, time the all-k sweep k = 2..K on the last tree (0: skip)")
    ap.add_argument("--cpu-sample-n", type=int, nargs="+", default=[4000, 8000])
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads, the sparse-communities precision comparison and graph weights")
    ap.add_argument("--only-graph-weights", action="store_true",
                    help="time only the full-graph weights at the blobs and anisotropic-mixture sizes and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before the steps, run one plain device copy of MIB MiB (reference for HBM counters)")
    ap.add_argument("--traffic-report", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs into profiles/screen_<precision>_traffic.json and exit")
    ap.add_argument("--kernel-traffic", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "STATS_CSV"),
                    help="print the per-kernel HBM table of two rocprofv3 --pmc runs and a --stats run, and exit")
    ap.add_argument("--kernels", nargs="*", default=[], help="with --kernel-traffic: kernel name substrings to keep")
    args = ap.parse_args()

    if args.traffic_report:
        rec = traffic_report(args.traffic_report[0], args.traffic_report[1], args.precision,
                             args.calibrate_copy or 1024)
        path = os.path.join(ROOT, "profiles", "screen_%s_traffic.json" % args.precision)
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec))
        return

    if args.kernel_traffic:
        print(kernel_traffic_table(*args.kernel_traffic, args.calibrate_copy or 1024, args.kernels))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the MST screen shards over tile pairs with one min-all-reduce per "
              "Boruvka round, but no multi-GPU path is built; run with --gpus 1", flush=True)
        sys.exit(2)

    if args.only_graph_weights:
        print(json.dumps({"graph_weights": graph_weights_timing()}), flush=True)
        return

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

    prune = not args.no_prune

    def step():
        return iso.cluster(X, k, precision=args.precision, recheck=args.recheck, prune=prune)

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
                   "i_k": ik, "mst_weight": info["mst"]["mst_weight"],
                   "prune": prune, "tile_pairs": info["mst"]["tile_pairs"],
                   "tile_pairs_full": info["mst"]["tile_pairs_full"]},
    }
    if not args.no_compare:
        # the same step with other screen precisions (FP32: the reference
        # precision; INT8: exact integer Gram tiles, for 8-bit data like this
        # workload's q/256 coordinates), one warm-up + one step each
        out["compare"] = []
        runs = [(prec, prune) for prec in ("fp32", "int8") if prec != args.precision]
        runs.append((args.precision, not prune))  # the same screen with the other pruning setting
        runs.append(("fp32", False))              # plain FP32, every tile pair
        for prec, pr in runs:
            log("comparison: %s screen%s, 1 warm-up + 1 step" % (prec, "" if pr else ", every tile pair"))
            iso.cluster(X, k, precision=prec, recheck=args.recheck, prune=pr)
            torch.cuda.synchronize()
            _lib.timing_enable(True)
            c0 = time.perf_counter()
            labc, ikc, infoc = iso.cluster(X, k, precision=prec, recheck=args.recheck, prune=pr)
            torch.cuda.synchronize()
            c1 = time.perf_counter()
            Tc = _lib.timing_read()
            _lib.timing_enable(False)
            # the same screen's roofline in this configuration (its own peak)
            ach = 2.0 * d * Tc["screen_pairs"] / (Tc["screen_ms"] * 1e-3) / 1e12 if Tc["screen_ms"] > 0 else None
            out["compare"].append({"screen": prec, "prune": pr, "value": n / (c1 - c0),
                                   "ms_per_step": (c1 - c0) * 1e3, "value_ratio": value / (n / (c1 - c0)),
                                   "tile_pairs": infoc["mst"]["tile_pairs"],
                                   "screen_ms": Tc["screen_ms"], "screen_tflops": ach,
                                   "screen_frac": ach / PEAKS_TFLOPS[prec] if ach else None,
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
    if args.n is None:
        out["parity"] = oracle_digest_parity(info, n)
    if not args.no_extras:
        out["workloads"] = other_workloads()
        out["precision_sparse_communities"] = precision_sparse_communities()
        out["graph_weights"] = graph_weights_timing()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, n=%s samples)" % args.cpu_sample_n)
        tree = (info["parent"].cpu().numpy(), info["length"].cpu().numpy())
        cb = cpu_baseline(n, k, args.cpu_sample_n, tree=tree)
        ik_or = cb.pop("_ik_oracle")
        out["cpu_baseline"] = cb
        if ik_or is not None and "parity" in out:
            out["parity"]["ik_oracle_on_this_tree"] = ik_or
            out["parity"]["ik_rel_err_vs_oracle"] = abs(ik - ik_or) / ik_or
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
