"""Benchmark of the block-wise LGF convolution on one MI355X.

Workload: the 1272-block plate-and-wake set (blocks of 16^3 cells inside an
ellipsoid around an aspect-ratio-2 flat plate at 30 degrees plus a downstream
cone; 5,210,112 cells per component), three components (the staggered vector
Poisson solve as three scalar solves), FP32 sources drawn N(0,1) within 4 cells
of the plate and 1e-3 N(0,1) elsewhere.  One step = one vector apply
u = G * f (3 components) through lgf_poisson_apply, inputs resident in HBM.

Prints one JSON line.  Extra objects: ``roofline`` for the dominant kernel
(HIP events on the launch stream over the timed region), ``cpu_baseline``
(the FP64 oracle's direct sum on a bounded sample of target cells, all host
cores), the measured error on a sample of targets, and the integrating-factor
apply E(0.1) f on the same block set.
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

METRIC = "LGF conv active Gcells/s + % roofline at 1e-5 err; IB force-solve ms, learned vs plain"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def conv_model_bytes(blocks, B, ncomp, es):
    """Algorithmic HBM bytes per kernel of one box-FFT apply (sources = targets).

    Every pass reads its input once and writes its output once; padding
    columns (Kxp - Kx) and rows without sources/targets are not counted."""
    b = np.asarray(blocks)
    lo = b.min(0)
    span = b.max(0) - lo + 1

    def smooth(n):
        m = n
        while True:
            r = m
            for p in (2, 3, 5):
                while r % p == 0:
                    r //= p
            if r == 1:
                return m
            m += 1

    nb = [smooth(int(s)) for s in span]
    N = [n * B for n in nb]
    P = [2 * n for n in N]
    Kx = P[0] // 2 + 1
    rows = {(int(y), int(z)) for _, y, z in (b - lo)}
    rows_cells = len(rows) * B * B            # box rows (y, z) holding sources (= targets)
    zplanes = len({z for _, z in rows}) * B   # z-planes holding targets
    cells = len(b) * B ** 3
    cx = 2 * es
    by = {
        "k_xfwd": ncomp * (cells * es + rows_cells * Kx * cx),
        "k_yfwd": ncomp * (rows_cells * Kx * cx + N[2] * P[1] * Kx * cx),
        "k_zconv": ncomp * (2 * N[2] * P[1] * Kx * cx) + (N[2] + 1) * (N[1] + 1) * Kx * es,
        "k_yinv": ncomp * (zplanes * P[1] * Kx * cx + rows_cells * Kx * cx),
        "k_xinv": ncomp * (rows_cells * Kx * cx + cells * es),
    }
    return by, N, P


def kernel_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, "paper_1604_01814_amd", "csrc", rec["source"]), "rb").read()
        if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
            return None
        k = rec["kernels"].get(kernel)
        return None if k is None else float(k["bytes_per_launch"])
    except Exception:
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (3x) to scale HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the box-FFT convolution is measured on a single "
              "MI355X; --gpus %d is not supported." % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1604_01814_amd as lg
    import workloads

    B, ncomp = 16, 3
    blocks = workloads.plate_blocks(B)
    nblk = len(blocks)
    cells = nblk * B ** 3
    log("workload: %d blocks of %d^3, %d cells/component, %d components" % (nblk, B, cells, ncomp))
    f64 = workloads.plate_sources(blocks, B, ncomp=ncomp)
    f = torch.from_numpy(f64.astype(np.float32)).cuda()
    u = torch.zeros_like(f)
    ctx = lg.Context(0)
    span = (blocks.max(0) - blocks.min(0) + 1) * B - 1
    t0 = time.time()
    tbl = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, tuple(int(v) for v in span))
    log("LGF table %s built in %.2f s" % (tuple(int(v) for v in span), time.time() - t0))
    stream = torch.cuda.current_stream()

    for i in range(args.warmup):
        lg.lgf_poisson_apply(ctx, tbl, B, blocks, blocks, f, u, stream=stream)
    torch.cuda.synchronize()
    log("warmup done (%d steps)" % args.warmup)

    lg.lgfib_profile_reset(ctx)
    lg.lgfib_profile_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        lg.lgf_poisson_apply(ctx, tbl, B, blocks, blocks, f, u, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lg.lgfib_profile_enable(ctx, False)
    prof = lg.lgfib_profile_read(ctx)
    ms = (t1 - t0) * 1e3 / args.steps
    value = ncomp * cells / (ms * 1e-3) / 1e9
    log("timed %d steps: %.4f ms/step, %.2f Gcells/s" % (args.steps, ms, value))

    model, N, P = conv_model_bytes(blocks, B, ncomp, 4)
    kern = {}
    for k, (cnt, tot) in prof.items():
        if k in model and cnt:
            avg = tot / cnt
            kern[k] = {"avg_ms": avg, "model_bytes": model[k], "GBs": model[k] / (avg * 1e-3) / 1e9}
    dom = max(kern, key=lambda k: kern[k]["avg_ms"])
    ach = kern[dom]["GBs"]
    step_bytes = sum(model.values())
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": kernel_traffic(dom),
                "bytes_per_launch": model[dom], "avg_launch_ms": round(kern[dom]["avg_ms"], 5)}
    for k in kern:
        log("  %-8s %8.4f ms  %7.1f GB/s (model %.1f MB)" % (k, kern[k]["avg_ms"], kern[k]["GBs"],
                                                            model[k] / 1e6))

    # accuracy on a seeded sample of targets, and the CPU oracle timed on it
    import oracle
    torch.cuda.synchronize()
    uh = u.cpu().numpy().astype(np.float64)
    cellsxyz = workloads.block_cells(blocks, B)
    near = workloads.plate_near_blocks(blocks, B, 8)
    g = np.random.Generator(np.random.PCG64(1604))
    t0 = time.time()
    G = oracle.lgf_table(*[int(v) for v in span])
    log("oracle LGF table built in %.1f s" % (time.time() - t0))
    cpu = None
    errs = []
    if not args.no_cpu_baseline:
        nprobe = 2 * oracle.num_threads()
        probe = g.choice(cells, nprobe, replace=False)
        t0 = time.perf_counter()
        oracle.conv_direct(G, cellsxyz, f64[0].reshape(-1), cellsxyz[probe])
        per = (time.perf_counter() - t0) / nprobe
        nt = int(max(8, min(20000, args.cpu_seconds / (ncomp * per))))
        picks = [int(b) * B ** 3 + int(v) for b in near for v in g.choice(B ** 3, max(1, nt // 16), replace=False)]
        rnd = g.choice(cells, max(0, nt - len(picks)), replace=False)
        sample = np.unique(np.concatenate([picks, rnd]).astype(np.int64))
        log("oracle sample: %d target cells x %d components (~%.0f s)" % (len(sample), ncomp,
                                                                           per * ncomp * len(sample)))
        t0 = time.perf_counter()
        refs = [oracle.conv_direct(G, cellsxyz, f64[c].reshape(-1), cellsxyz[sample]) for c in range(ncomp)]
        tcpu = time.perf_counter() - t0
        for c in range(ncomp):
            got = uh[c].reshape(-1)[sample]
            errs.append(float(np.max(np.abs(got - refs[c])) / np.max(np.abs(refs[c]))))
        cpu = {"value": round(len(sample) * ncomp / tcpu / 1e9, 9), "unit": "Gcells/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "%d target cells (%d next to the plate, rest seeded uniform) x %d components, FP64 "
                         "direct sum over all %d source cells; %.1f s" % (len(sample), len(picks), ncomp, cells, tcpu)}
        log("oracle: %.1f s, rel err per component %s" % (tcpu, ["%.2e" % e for e in errs]))

    # integrating factor E(a) f on the same block set (a = 0.1, radius 8)
    fi = torch.zeros_like(f)
    for _ in range(2):
        lg.lgf_if_apply(ctx, 0.1, B, blocks, blocks, f, fi, stream=stream)
    lg.lgfib_profile_reset(ctx)
    lg.lgfib_profile_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nif = max(5, args.steps)
    for _ in range(nif):
        lg.lgf_if_apply(ctx, 0.1, B, blocks, blocks, f, fi, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lg.lgfib_profile_enable(ctx, False)
    pif = lg.lgfib_profile_read(ctx).get("k_if_apply", (1, 0.0))
    ms_if = (t1 - t0) * 1e3 / nif
    if_bytes = ncomp * cells * 8
    if_avg = pif[1] / max(1, pif[0])
    if_apply = {"a": 0.1, "ms": round(ms_if, 5), "Gcells_per_s": round(ncomp * cells / (ms_if * 1e-3) / 1e9, 2),
                "roofline": {"bound": "hbm", "achieved": round(if_bytes / (if_avg * 1e-3) / 1e9, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(if_bytes / (if_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                             "bytes_per_launch": if_bytes, "avg_launch_ms": round(if_avg, 5)}}
    log("E(0.1) apply: %.4f ms, %.1f Gcells/s" % (ms_if, if_apply["Gcells_per_s"]))

    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 256 MiB device-to-device copies")

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gcells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "plate_wake_vector_poisson", "blocks": nblk, "B": B, "cells_per_component": cells,
                   "components": ncomp, "box_cells": N, "fft": P, "path": "box_fft"},
        "roofline": roofline,
        "step_model_GBs": round(step_bytes / (ms * 1e-3) / 1e9, 1),
        "kernels": {k: {"avg_ms": round(v["avg_ms"], 5), "GBs": round(v["GBs"], 1)} for k, v in kern.items()},
        "max_rel_err": max(errs) if errs else None,
        "cpu_baseline": cpu,
        "if_apply": if_apply,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
