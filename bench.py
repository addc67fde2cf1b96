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
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
# FP32 vector FMAs without packed instructions: 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
FP32_FMA_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0


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
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))["kernels"].get(kernel)
        if rec is None:
            return None
        h = hashlib.sha256()
        for f in rec["sources"]:
            h.update(open(os.path.join(ROOT, "paper_1604_01814_amd", "csrc", f), "rb").read())
        if h.hexdigest() != rec["sources_sha256"]:
            return None
        return float(rec["bytes_per_launch"])
    except Exception:
        return None


def to_blocks8(blocks16, f16):
    """Re-lay fields on 16^3 blocks as 8^3 blocks (each split into eight)."""
    out_b, out_f = [], []
    for i, b in enumerate(blocks16):
        for dz in range(2):
            for dy in range(2):
                for dx in range(2):
                    out_b.append((2 * b[0] + dx, 2 * b[1] + dy, 2 * b[2] + dz))
                    out_f.append(f16[:, i, 8 * dz:8 * dz + 8, 8 * dy:8 * dy + 8, 8 * dx:8 * dx + 8])
    return np.array(out_b, dtype=np.int32), np.stack(out_f, axis=1)


def precision_bench(lg, torch, workloads, ctx, args, f64_all, blocks, B, tbl, G):
    """Precision sweep on the full plate-and-wake set (1272 blocks of 16^3, 3
    components of the plate sources): box FFT in FP64 and FP32, and the
    block-pair form on the same set re-blocked to 8^3 (10,176 blocks) with
    FP32 or split-BF16 matrix-core DFTs; error per component against the FP64
    direct sum on seeded targets (half of them next to the plate).  Then
    E(a) for a in {0.02, 0.1, 0.5}, FP32, against the windowed direct sum."""
    import oracle
    f = f64_all
    ncomp = f.shape[0]
    g = np.random.Generator(np.random.PCG64(1604 + 3))
    ncell = len(blocks) * B ** 3
    near = workloads.plate_near_blocks(blocks, B, 8)
    near_cells = np.array([int(b) * B ** 3 + v for b in near for v in range(B ** 3)], dtype=np.int64)
    sample = np.unique(np.concatenate([g.choice(near_cells, 128, replace=False), g.choice(ncell, 128, replace=False)]))
    cells = workloads.block_cells(blocks, B)
    t0 = time.time()
    refs = [oracle.conv_direct(G, cells, f[c].reshape(-1), cells[sample]) for c in range(ncomp)]
    log("precision: oracle on %d target cells x %d components in %.1f s" % (len(sample), ncomp, time.time() - t0))
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {"workload": "plate_wake_vector_poisson", "blocks": int(len(blocks)), "cells_per_component": int(ncell),
           "components": ncomp, "targets_sampled": int(len(sample)), "variants": {}}

    def record(name, u16, ms):
        errs = [float(np.max(np.abs(u16[c].reshape(-1)[sample] - refs[c])) / np.max(np.abs(refs[c])))
                for c in range(ncomp)]
        out["variants"][name] = {"ms": round(ms, 4), "max_rel_err_per_component": ["%.2e" % e for e in errs],
                                 "Gcells_per_s": round(ncomp * ncell / (ms * 1e-3) / 1e9, 2)}
        log("precision %-14s %8.4f ms  err %s" % (name, ms, out["variants"][name]["max_rel_err_per_component"]))

    for name, dt in (("box_fft_f64", torch.float64), ("box_fft_f32", torch.float32)):
        fd = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float64 if dt == torch.float64 else np.float32)).cuda()
        ud = torch.zeros_like(fd)
        ms = timed(lambda: lg.lgf_poisson_apply(ctx, tbl, B, blocks, blocks, fd, ud, stream=stream))
        record(name, ud.cpu().numpy().astype(np.float64), ms)
        del fd, ud
    b8, f8 = to_blocks8(blocks, f)
    fd = torch.from_numpy(np.ascontiguousarray(f8, dtype=np.float32)).cuda()
    ud = torch.zeros_like(fd)
    n8 = len(b8)
    for name, dft in (("pair_fft32", lg.LGF_DFT_FFT32), ("pair_bf16x3", lg.LGF_DFT_BF16X3)):
        ms = timed(lambda: lg.lgf_pair_apply(ctx, tbl, 8, b8, b8, fd, ud, dft=dft, stream=stream), reps=2)
        # per-kernel times of the same apply (HIP events on the launch stream)
        lg.lgfib_profile_reset(ctx)
        lg.lgfib_profile_enable(ctx, True)
        for _ in range(2):
            lg.lgf_pair_apply(ctx, tbl, 8, b8, b8, fd, ud, dft=dft, stream=stream)
        torch.cuda.synchronize()
        lg.lgfib_profile_enable(ctx, False)
        prof = lg.lgfib_profile_read(ctx)
        u8 = ud.cpu().numpy().astype(np.float64)
        u16 = np.zeros_like(f)
        for dz in range(2):
            for dy in range(2):
                for dx in range(2):
                    j = 4 * dz + 2 * dy + dx
                    u16[:, :, 8 * dz:8 * dz + 8, 8 * dy:8 * dy + 8, 8 * dx:8 * dx + 8] = u8[:, j::8]
        record(name, u16, ms)
        # the spectral multiply-accumulate: 8 flop per complex MAC, 2304
        # half-spectrum values per block pair and component; FP32 FMAs on
        # the vector units (no packed FP32 in this build): 78.6 TFLOP/s
        cnt, tot = prof.get("k_pair_mac", (1, 0.0))
        mac_ms = tot / max(cnt, 1)
        flop = 8.0 * n8 * n8 * 2304 * ncomp
        ach = flop / (mac_ms * 1e-3) / 1e12 if mac_ms > 0 else 0.0
        kern = {k: round(v[1] / max(v[0], 1), 4) for k, v in prof.items() if k.startswith("k_pair")}
        var = out["variants"][name]
        var["kernels_ms"] = kern
        var["roofline_mac"] = {"bound": "alu", "achieved": round(ach, 2), "peak": FP32_FMA_TFLOPS,
                               "unit": "TFLOP/s", "frac": round(ach / FP32_FMA_TFLOPS, 4),
                               "flop_per_launch": flop, "avg_launch_ms": round(mac_ms, 4)}
        if dft == lg.LGF_DFT_BF16X3:
            # matrix-core work of the block transforms: 28 complex 16 x 16 x 16
            # products per block and component each way (x: 4, y: 8, z: 16
            # column groups), 24 bf16 MFMAs of 2 * 16^3 flop per product
            mflop = 28 * 24 * 2.0 * 16 ** 3 * n8 * ncomp
            for kname in ("k_pair_fwd", "k_pair_inv"):
                kms = kern.get(kname, 0.0)
                if kms > 0:
                    var["roofline_" + kname + "_mfma"] = {
                        "bound": "mfma", "achieved": round(mflop / (kms * 1e-3) / 1e12, 1), "peak": BF16_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(mflop / (kms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS, 4),
                        "flop_per_launch": mflop, "avg_launch_ms": kms}
        log("  %s kernels %s; MAC %.1f TFLOP/s" % (name, kern, ach))
    del fd, ud
    # E(a) on the full plate set
    fa = torch.from_numpy(np.ascontiguousarray(f64_all, dtype=np.float32)).cuda()
    ua = torch.zeros_like(fa)
    allcells = workloads.block_cells(blocks, B)
    samp = np.unique(g.choice(len(blocks) * B ** 3, 128, replace=False))
    out["if_apply"] = {}
    for a in (0.02, 0.1, 0.5):
        ms = timed(lambda: lg.lgf_if_apply(ctx, a, B, blocks, blocks, fa, ua, stream=stream))
        u = ua.cpu().numpy()
        ker = oracle.if_kernel_table(a)
        errs = []
        for c in range(f64_all.shape[0]):
            lo, box, _ = workloads.dense_box(blocks, B, f64_all[c])
            ref = oracle.conv_window(ker, box, lo, allcells[samp])
            errs.append(float(np.max(np.abs(u[c].reshape(-1)[samp] - ref)) / np.max(np.abs(ref))))
        ncl = f64_all.shape[0] * len(blocks) * B ** 3
        out["if_apply"]["a=%g" % a] = {"radius": lg.lgf_if_weights(ctx, a, lg.IF_CUTOFF_F32)[0],
                                       "ms": round(ms, 4), "Gcells_per_s": round(ncl / (ms * 1e-3) / 1e9, 1),
                                       "max_rel_err_per_component": ["%.2e" % e for e in errs]}
        log("E(%g): %.4f ms, err %s" % (a, ms, ["%.2e" % e for e in errs]))
    return out


def refresh_bench(lg, torch, workloads, ctx, args, tbl, blocks, B, f, stream):
    """Velocity refresh (Sec. 4.1) on the plate-and-wake flow set, FP32, with
    the vorticity kept on the blocks whose lower neighbours are flow blocks
    (so the source side stays inside the flow set's box).  Timed in place on
    one field; the stencil kernel's roofline uses its algorithmic bytes: read
    u and write r = -C^T (C u) once over the source blocks, 3 components."""
    vort = workloads.lower_closed_blocks(blocks)
    src = np.unique(np.concatenate([vort] + [vort - np.eye(3, dtype=np.int32)[a] for a in range(3)]), axis=0)
    u = f.clone()
    for _ in range(2):
        lg.lgf_velocity_refresh(ctx, tbl, B, vort, blocks, u, stream=stream)
    lg.lgfib_profile_reset(ctx)
    lg.lgfib_profile_enable(ctx, True)
    torch.cuda.synchronize()
    n = max(5, args.steps)
    t0 = time.perf_counter()
    for _ in range(n):
        lg.lgf_velocity_refresh(ctx, tbl, B, vort, blocks, u, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lg.lgfib_profile_enable(ctx, False)
    prof = lg.lgfib_profile_read(ctx)
    ms = (t1 - t0) * 1e3 / n
    cells = len(blocks) * B ** 3
    cnt, tot = prof.get("k_refresh_src", (1, 0.0))
    avg = tot / max(1, cnt)
    nbytes = 2 * 3 * len(src) * B ** 3 * 4
    out = {"flow_blocks": len(blocks), "vorticity_blocks": len(vort), "source_blocks": len(src),
           "ms": round(ms, 5), "Gcells_per_s": round(3 * cells / (ms * 1e-3) / 1e9, 2),
           "finite": bool(torch.isfinite(u).all().item()),
           "kernels_ms": {k: round(v[1] / max(1, v[0]), 5) for k, v in prof.items()},
           "roofline": {"bound": "hbm", "kernel": "k_refresh_src", "achieved": round(nbytes / (avg * 1e-3) / 1e9, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(nbytes / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        "traffic": kernel_traffic("k_refresh_src"), "bytes_per_launch": nbytes,
                        "avg_launch_ms": round(avg, 5)}}
    log("velocity refresh: %.4f ms (%d flow, %d vorticity, %d source blocks), k_refresh_src %.4f ms %.0f GB/s"
        % (ms, len(blocks), len(vort), len(src), avg, out["roofline"]["achieved"]))
    # the nonlinear term (C u) x u_a on the same blocks: read u, write the term
    lam = torch.empty_like(f)
    for _ in range(2):
        lg.lgf_lamb_vector(ctx, B, blocks, f, lam, (0.1, 0.0, 0.0), stream=stream)
    lg.lgfib_profile_reset(ctx)
    lg.lgfib_profile_enable(ctx, True)
    for _ in range(n):
        lg.lgf_lamb_vector(ctx, B, blocks, f, lam, (0.1, 0.0, 0.0), stream=stream)
    torch.cuda.synchronize()
    lg.lgfib_profile_enable(ctx, False)
    cnt, tot = lg.lgfib_profile_read(ctx).get("k_lamb", (1, 0.0))
    lavg = tot / max(1, cnt)
    lbytes = 2 * 3 * cells * 4
    out["lamb_vector"] = {"avg_launch_ms": round(lavg, 5), "Gcells_per_s": round(3 * cells / (lavg * 1e-3) / 1e9, 1),
                          "roofline": {"bound": "hbm", "kernel": "k_lamb",
                                       "achieved": round(lbytes / (lavg * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                                       "unit": "GB/s",
                                       "frac": round(lbytes / (lavg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                       "traffic": kernel_traffic("k_lamb"), "bytes_per_launch": lbytes}}
    log("nonlinear term: k_lamb %.4f ms %.0f GB/s" % (lavg, out["lamb_vector"]["roofline"]["achieved"]))
    return out


def multilevel_bench(lg, torch, workloads, ctx, args):
    """Multilevel interpolation evaluator (FP64) on a sparse set: the blocks
    of 8^3 within one block of a sphere surface of diameter --ml-diameter
    cells, sources = targets, against the exact FP64 box-FFT apply on the
    same set.  The roofline is that of the neighbour sum on the matrix cores
    (k_ml_near_mfma): 2 B^6 flops per neighbouring block pair against the
    dense FP64 matrix peak."""
    B = 8
    blocks = workloads.shell_blocks(float(args.ml_diameter), B)
    nblk = len(blocks)
    cells = nblk * B ** 3
    # the table must reach the nodes of the top-level clusters (at most 4 per axis)
    lo, hi = blocks.min(0), blocks.max(0)
    top = 0
    while np.any((hi >> top) - (lo >> top) + 1 > 4):
        top += 1
    ext = [int(v) for v in ((hi >> top) - (lo >> top) + 1) * (B << top) - 1]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tbl = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, ext)
    t_table = time.perf_counter() - t0
    f = torch.from_numpy(workloads.normal_sources(nblk, B, config=6)).cuda()
    u_ex = torch.empty_like(f)
    u = torch.empty_like(f)
    n = max(5, args.steps)

    def timed(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / n

    try:   # the exact box FFT takes spans of at most 512 cells per axis
        ms_exact = timed(lambda: lg.lgf_poisson_apply(ctx, tbl, B, blocks, blocks, f, u_ex))
    except lg.LgfibError as e:
        if e.code != lg.LGFIB_ERANGE:
            raise
        ms_exact = None
        log("multilevel: no exact box-FFT apply for this set (%s)" % e)
    out = {"workload": "sphere_shell_d%d" % args.ml_diameter, "blocks": nblk, "B": B, "table_extent": ext,
           "table_build_s": round(t_table, 3),
           "exact_box_fft_f64_ms": None if ms_exact is None else round(ms_exact, 4), "orders": {}}
    scale = None if ms_exact is None else float(u_ex.abs().max().item())
    for p, near in ((4, lg.LGF_F64), (5, lg.LGF_F64), (6, lg.LGF_F64), (4, lg.LGF_F32), (6, lg.LGF_F32)):
        t0 = time.perf_counter()
        ml = lg.lgf_ml_create(ctx, tbl, B, p, blocks, blocks, pair_prec=near)
        t_plan = time.perf_counter() - t0
        ms = timed(lambda: ml.apply(f, u))
        lg.lgfib_profile_reset(ctx)
        lg.lgfib_profile_enable(ctx, True)
        for _ in range(n):
            ml.apply(f, u)
        torch.cuda.synchronize()
        lg.lgfib_profile_enable(ctx, False)
        prof = lg.lgfib_profile_read(ctx)
        info = ml.info()
        err = None if scale is None else float((u - u_ex).abs().max().item()) / scale
        cnt, tot = prof.get("k_ml_near_mfma", (1, 0.0))
        avg = tot / max(1, cnt)
        flops = 2.0 * info["near_pairs"] * B ** 6
        ach = flops / (avg * 1e-3) / 1e12
        peak = FP64_PEAK_TFLOPS if near == lg.LGF_F64 else FP32_PEAK_TFLOPS
        out["orders"][str(p) if near == lg.LGF_F64 else "%d_pairs_f32" % p] = {
            "ms": round(ms, 4), "Gcells_per_s": round(cells / (ms * 1e-3) / 1e9, 3),
            "speedup_vs_exact": None if ms_exact is None else round(ms_exact / ms, 2), "max_rel_err_vs_exact": err,
            "plan_s": round(t_plan, 3),
            "tree": info,
            "kernels_ms_per_apply": {k: round(v[1] / n, 5) for k, v in prof.items()},
            "roofline": {"bound": "mfma", "kernel": "k_ml_near_mfma", "dtype": "f64" if near == lg.LGF_F64 else "f32",
                         "achieved": round(ach, 2), "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 4),
                         "traffic": kernel_traffic("k_ml_near_mfma") if near == lg.LGF_F64 else None,
                         "flops_per_launch": flops,
                         "avg_launch_ms": round(avg, 5)}}
        log("multilevel p=%d%s: %.3f ms (exact box FFT %s ms), err %s, neighbour sum %.3f ms %.1f TFLOP/s, %s"
            % (p, "" if near == lg.LGF_F64 else " (FP32 pair products)", ms, "n/a" if ms_exact is None else "%.3f" % ms_exact, "n/a" if err is None else "%.2e" % err,
               avg, ach, info))
        ml.close()
    return out


def batch_bench(lg, torch, workloads, ctx, args):
    """64 independent scalar FP32 Poisson applies on compact blobs of K_i blocks
    of 16^3 (K_i log-uniform in [1, 400], random anisotropic metric in a
    16^3-block region), f ~ N(0,1): one autotuned, graph-captured batch launch
    against the same instances as 64 separate lgf_poisson_apply calls."""
    B = 16
    sets = workloads.blob_instances(n_inst=64, kmin=1, kmax=400, region=16, config=4)
    g = np.random.Generator(np.random.PCG64(1604 + 4))
    f_d = [torch.from_numpy(g.standard_normal((len(s), B, B, B)).astype(np.float32)).cuda() for s in sets]
    u_d = [torch.zeros_like(f) for f in f_d]
    cells = sum(len(s) for s in sets) * B ** 3
    tbl = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, (16 * B + 2 * B,) * 3)
    t0 = time.time()
    batch = lg.lgf_batch_create(ctx, tbl, B, list(zip(sets, f_d, u_d)), autotune=True, nbranch=args.batch_branches)
    t_tune = time.time() - t0
    picks = [batch.info(i) for i in range(len(sets))]
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    reps = max(5, args.steps)
    ms_graph = timed(lambda: batch.run(stream=stream), reps)
    ms_eager = timed(lambda: batch.run(eager=True, stream=stream), reps)
    # the same instances with the box convolutions as batched passes (one
    # persistent launch per pass and FFT length)
    t0 = time.time()
    bpass = lg.lgf_batch_create(ctx, tbl, B, list(zip(sets, f_d, u_d)), autotune=True, nbranch=args.batch_branches,
                                passes=True)
    t_tune_p = time.time() - t0
    ms_pass = timed(lambda: bpass.run(stream=stream), reps)
    bpass.close()
    one = [(s, f.unsqueeze(0), u.unsqueeze(0)) for s, f, u in zip(sets, f_d, u_d)]

    def separate():
        for s, f, u in one:
            lg.lgf_poisson_apply(ctx, tbl, B, s, s, f, u, stream=stream)

    ms_sep = timed(separate, reps)
    hist = {}
    for p in picks:
        key = "pair8" if p["path"] == "pair" else "B%d_tx%d_ty%d" % (p["block"], p["tiles_x"], p["tiles_y"])
        hist[key] = hist.get(key, 0) + 1
    out = {"workload": "64_blobs_K1_400_B16", "instances": len(sets), "blocks": int(sum(len(s) for s in sets)),
           "cells": int(cells), "graph_ms": round(ms_graph, 4), "eager_same_kernels_ms": round(ms_eager, 4),
           "separate_applies_ms": round(ms_sep, 4), "Gcells_per_s": round(cells / (ms_graph * 1e-3) / 1e9, 2),
           "speedup_vs_separate": round(ms_sep / ms_graph, 3), "autotune_s": round(t_tune, 2), "picks": hist,
           "branches": args.batch_branches,
           "batched_passes": {"graph_ms": round(ms_pass, 4), "Gcells_per_s": round(cells / (ms_pass * 1e-3) / 1e9, 2),
                              "autotune_s": round(t_tune_p, 2)},
           "best": {"form": "batched_passes" if ms_pass < ms_graph else "per_instance_graph",
                    "ms": round(min(ms_pass, ms_graph), 4),
                    "Gcells_per_s": round(cells / (min(ms_pass, ms_graph) * 1e-3) / 1e9, 2)}}
    log("batch: %d instances, %d blocks: graph %.3f ms, eager %.3f ms, separate %.3f ms (%.1f Gcells/s); "
        "batched passes %.3f ms" % (len(sets), out["blocks"], ms_graph, ms_eager, ms_sep, out["Gcells_per_s"], ms_pass))
    batch.close()
    return out


def lanczos_extremes(apply, n, its, seed, torch):
    """Extreme Ritz values of a symmetric operator after ``its`` Lanczos steps
    with full reorthogonalisation (FP64 on the device): estimates of
    lambda_min and lambda_max, hence of the condition number."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    q = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
    q /= torch.linalg.vector_norm(q)
    Q = [q]
    al, be = [], []
    w = torch.empty_like(q)
    for j in range(its):
        apply(Q[-1], w)
        a = float(torch.dot(w, Q[-1]))
        al.append(a)
        w -= a * Q[-1]
        if j:
            w -= be[-1] * Q[-2]
        for v in Q:                       # full reorthogonalisation
            w -= torch.dot(w, v) * v
        b = float(torch.linalg.vector_norm(w))
        if b < 1e-12 * abs(a):
            break
        be.append(b)
        Q.append(w / b)
        w = torch.empty_like(q)
    k = len(al)
    T = np.diag(al) + np.diag(be[:k - 1], 1) + np.diag(be[:k - 1], -1)
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])


def ib_force_bench(lg, torch, workloads, ctx, args, NL, history_direct=False, stride=1, maxit=4000, extras=True):
    """Force solves of the heaving-sphere Stokes driver: a sphere of diameter
    32 cells with NL Fibonacci markers (3-point Roma kernel) in a body-fixed
    frame, body blocks of 8^3, a = 0.05, flow on 12^3 blocks of 8^3 around it.
    The body heaves with amplitude 0.25 D and period 200 steps, which enters as
    the marker velocity u_B = U(t) e_y.  Steps 0..ntrain-1 generate the force
    history that trains the warm-start network; on the later steps the same
    force systems C f = b_k are solved to 1e-8 relative residual (FP32
    matvecs, FP64 dots and true residual) from a cold start, from the
    previous step's force, from a linear extrapolation of the last two, and
    from the network's prediction.  With history_direct the history's force
    solves use the dense Cholesky factor of C (Sec. 3.2) instead of CG (the
    listed 4000-marker sphere, where cold CG needs thousands of iterations);
    the evaluated solves are every stride-th step of the rest."""
    B, alpha, D = 8, 0.05, 32.0
    X = workloads.sphere_markers(D, NL)
    normals = torch.from_numpy((X - workloads.SPHERE_CENTER) / (D / 2)).cuda()
    blocks = lg.ib_body_blocks(lg.IB_ROMA3, X, B)
    t0 = time.time()
    sys_ = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, alpha)
    fb = np.array([(x, y, z) for z in range(-1, 11) for y in range(-1, 11) for x in range(-1, 11)], dtype=np.int32)
    fl = lg.ib_flow_create(ctx, sys_, fb)
    log("IB: %d markers, %d body blocks, %d flow blocks of %d^3; set-up %.2f s" % (NL, len(blocks), len(fb), B,
                                                                               time.time() - t0))
    t_factor = None
    if history_direct:
        torch.cuda.synchronize()
        t0 = time.time()
        lg.ib_system_factor(ctx, sys_)
        torch.cuda.synchronize()
        t_factor = time.time() - t0
        log("IB: dense C (%d unknowns) built and factored in %.2f s" % (3 * NL, t_factor))
    nsteps, ntrain = args.ib_steps, args.ib_train
    U = [workloads.heave_velocity(k, D) for k in range(nsteps + 2)]   # U[-1] = U(t_{-1}) is never used
    u = torch.zeros((3, len(fb), B, B, B), dtype=torch.float64, device="cuda")
    F = torch.zeros((nsteps, NL, 3), dtype=torch.float64, device="cuda")
    Bk = torch.zeros_like(F)
    ub = torch.zeros((NL, 3), dtype=torch.float64, device="cuda")
    gen_its = []
    t0 = time.time()
    for k in range(nsteps):
        ub[:, 1] = U[k + 1]
        x0 = F[k - 1] if k else None
        st = lg.ib_flow_step(ctx, fl, u, ub, F[k], x0=x0, rtol=1e-8, maxit=maxit,
                             prec=lg.IB_SOLVE_DIRECT if history_direct else lg.LGF_F32, b_out=Bk[k])
        gen_its.append(st["iterations"])
        if (k + 1) % 100 == 0:
            log("IB history: step %d/%d, %.1f s, last solve %d its" % (k + 1, nsteps, time.time() - t0,
                                                                      st["iterations"]))
    t_gen = time.time() - t0

    # training set: the solves of steps ib_skip..ntrain-1 (the impulsive start,
    # whose force jumps dwarf the later ones, is left out); target: the error
    # of the linear extrapolation, f_k - (2 f_{k-1} - f_{k-2})
    nin, nh, nout = 12, 256, 3
    rows = list(range(args.ib_skip, ntrain))
    Xtr = torch.zeros((len(rows) * NL, nin), dtype=torch.float32, device="cuda")
    for i, k in enumerate(rows):
        lg.ib_mlp_features(ctx, normals, (U[k + 1], U[k], U[k - 1], U[k - 2]), F[k - 1], F[k - 2],
                           Xtr[i * NL:(i + 1) * NL])
    Ttr = (F[rows] - 2.0 * F[[k - 1 for k in rows]] + F[[k - 2 for k in rows]]).reshape(-1, 3).float().contiguous()
    ins, inc = Xtr.mean(0), Xtr.std(0).clamp_min(1e-6)
    ots, otc = Ttr.mean(0), Ttr.std(0).clamp_min(1e-12)
    g = np.random.Generator(np.random.PCG64(1604))
    p0 = []
    for fo, fi in ((nh, nin), (nh, nh), (nout, nh)):
        lim = 1.0 / np.sqrt(fi)
        p0 += [g.uniform(-lim, lim, fo * fi), np.zeros(fo)]
    net = lg.ib_mlp_create(ctx, nin, nh, nout, np.concatenate(p0), ins.cpu().numpy(), inc.cpu().numpy(),
                           ots.cpu().numpy(), otc.cpu().numpy())
    torch.cuda.synchronize()
    t0 = time.time()
    loss = lg.ib_mlp_train(ctx, net, Xtr, Ttr, epochs=args.ib_epochs, batch=4096, lr=1e-3, seed=1604)
    t_train = time.time() - t0
    log("IB: trained on %d rows, %d epochs in %.1f s, loss %.3e" % (Xtr.shape[0], args.ib_epochs, t_train, loss))
    del Xtr, Ttr

    feats = torch.zeros((NL, nin), dtype=torch.float32, device="cuda")
    x0 = torch.zeros((NL, 3), dtype=torch.float64, device="cuda")
    f = torch.zeros_like(x0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {m: {"ms": [], "its": [], "fallback": 0, "x0_err": [], "err": []} for m in ("cold", "prev", "extrap", "mlp")}
    evals = list(range(max(ntrain, 2), nsteps, stride))
    for k in evals:
        ref = F[k]
        nref = float(torch.linalg.vector_norm(ref))
        for m in res:
            ms_pre = 0.0
            if m == "cold":
                guess = None
            elif m == "prev":
                guess = F[k - 1]
            elif m == "extrap":
                e0.record()
                torch.mul(F[k - 1], 2.0, out=x0)
                x0.sub_(F[k - 2])
                e1.record()
                e1.synchronize()
                ms_pre = e0.elapsed_time(e1)
                guess = x0
            else:
                e0.record()
                lg.ib_mlp_features(ctx, normals, (U[k + 1], U[k], U[k - 1], U[k - 2]), F[k - 1], F[k - 2], feats)
                lg.ib_mlp_warmstart(ctx, net, feats, F[k - 1], F[k - 2], x0)
                e1.record()
                e1.synchronize()
                ms_pre = e0.elapsed_time(e1)
                guess = x0
            st = lg.ib_force_solve(ctx, sys_, Bk[k], f, x0=guess, rtol=1e-8, maxit=maxit, prec=lg.LGF_F32,
                                   raise_on_noconv=False)
            r = res[m]
            r["ms"].append(ms_pre + st["ms"])
            r["its"].append(st["iterations"])
            r.setdefault("restarts", []).append(st["restarts"])
            r["fallback"] += st["fallback"]
            r["noconv"] = r.get("noconv", 0) + int(st["rel_residual"] > 1e-8)
            r["err"].append(float(torch.linalg.vector_norm(f - ref)) / nref)
            if guess is not None:
                r["x0_err"].append(float(torch.linalg.vector_norm(guess - ref)) / nref)
    if history_direct:
        lg.ib_system_factor(ctx, sys_, False)   # free the dense factor before the next legs
    dense = dense_solve_bench(lg, torch, ctx, sys_, NL, F, Bk, evals, args) if extras else None
    herk = herk_bench(lg, torch, workloads, ctx, X, B, blocks, fb, alpha, u, nsteps, D, args) if extras else None
    # condition number of the Schur complement (Lanczos, FP64 matvec)
    def capply(q, w):
        lg.ib_schur_apply(ctx, sys_, q.view(NL, 3), w.view(NL, 3))
    lmin, lmax = lanczos_extremes(capply, 3 * NL, args.ib_lanczos, 7, torch)
    out = {"workload": "sphere_heave_D32_NL%d" % NL, "markers": NL, "a": alpha, "B": B, "body_blocks": len(blocks),
           "flow_blocks": len(fb), "steps": nsteps, "train_steps": ntrain, "eval_steps": len(evals),
           "eval_stride": stride, "maxit": maxit, "history_solver": "dense_cholesky" if history_direct else "cg",
           "dense_factor_s": None if t_factor is None else round(t_factor, 3),
           "rtol": 1e-8, "matvec": "f32", "history_s": round(t_gen, 2),
           "history_mean_its": round(float(np.mean(gen_its)), 1), "train_s": round(t_train, 2),
           "train_loss": loss, "kappa": round(lmax / lmin, 1), "lambda": [lmin, lmax]}
    for m, r in res.items():
        out[m] = {"ms": round(float(np.mean(r["ms"])), 4), "iterations": round(float(np.mean(r["its"])), 2),
                  "restarts": round(float(np.mean(r["restarts"])), 2),
                  "fallbacks": r["fallback"], "not_converged": r.get("noconv", 0),
                  "max_err_vs_history": float(np.max(r["err"]))}
        if r["x0_err"]:
            out[m]["x0_rel_err"] = float(np.mean(r["x0_err"]))
        log("IB %-6s %8.3f ms  %6.1f its  fallbacks %d" % (m, out[m]["ms"], out[m]["iterations"], r["fallback"]))
    out["speedup_mlp_vs_cold"] = round(out["cold"]["ms"] / out["mlp"]["ms"], 3)
    out["direct"] = dense
    out["herk"] = herk
    net.close()
    fl.close()
    sys_.close()
    return out


def herk_bench(lg, torch, workloads, ctx, X, B, blocks, fb, alpha, u, k0, D, args):
    """The paper's time integrator on the same configuration: Scheme A
    IF-HERK steps (three stages, two distinct integrating factors, one the
    identity; Sec. 2.3, App. B) with dense direct force solves, continuing the
    force history's flow for args.herk_steps steps."""
    at, ct = lg.ib_herk_tableau("A")
    torch.cuda.synchronize()
    t0 = time.time()
    hk = lg.ib_herk_create(ctx, lg.IB_ROMA3, X, B, blocks, fb, alpha, at, ct, direct=True)
    t_create = time.time() - t0
    NL = len(X)
    ub = torch.zeros((len(ct), NL, 3), dtype=torch.float64, device="cuda")
    f = torch.zeros((NL, 3), dtype=torch.float64, device="cuda")
    uu = u.clone()
    n = args.herk_steps
    for k in range(2):   # warm-up
        lg.ib_herk_step(ctx, hk, uu, ub, f)
    torch.cuda.synchronize()
    t0 = time.time()
    for k in range(n):
        for i, c in enumerate(ct):
            ub[i, :, 1] = workloads.heave_velocity(k0 + k + c, D)
        lg.ib_herk_step(ctx, hk, uu, ub, f)
    torch.cuda.synchronize()
    ms = (time.time() - t0) / n * 1e3
    # the same steps with the nonlinear term (Navier-Stokes on the fixed flow
    # set): dt / dx = 1, so the heave velocity gives a Courant number of 0.25
    lg.ib_herk_convection(ctx, hk, 1.0)
    lg.ib_herk_step(ctx, hk, uu, ub, f)
    torch.cuda.synchronize()
    t0 = time.time()
    for k in range(n):
        for i, c in enumerate(ct):
            ub[i, :, 1] = workloads.heave_velocity(k0 + n + k + c, D)
        lg.ib_herk_step(ctx, hk, uu, ub, f)
    torch.cuda.synchronize()
    ms_ns = (time.time() - t0) / n * 1e3
    # the adaptive-domain update on the resulting flow (Sec. 4.1): the
    # per-block support (max |C u|, max |D-bar N~|), then the weights and the
    # new D_flow / D_xflow, all on the GPU; the host form of the update is
    # timed beside it (same lists)
    mu = torch.zeros(len(fb), dtype=torch.float64, device="cuda")
    nu = torch.zeros_like(mu)
    lg.lgf_block_support(ctx, B, fb, uu, mu, nu)
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float64)).cuda()
    fnew, xnew = lg.ib_adapt_flow_dev(ctx, Xd, B, fb, mu, nu, 1.0, D, 1e-3, blocks, 1)
    lg.lgfib_profile_reset(ctx)
    lg.lgfib_profile_enable(ctx, True)
    for _ in range(n):
        lg.lgf_block_support(ctx, B, fb, uu, mu, nu)
    torch.cuda.synchronize()
    lg.lgfib_profile_enable(ctx, False)
    cnt, tot = lg.lgfib_profile_read(ctx).get("k_block_support", (1, 0.0))
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(n):
        fnew, xnew = lg.ib_adapt_flow_dev(ctx, Xd, B, fb, mu, nu, 1.0, D, 1e-3, blocks, 1)
    t_dev = (time.time() - t0) / n * 1e3
    t0 = time.time()
    wts = lg.ib_block_weights(X, B, fb, 1.0, D)
    fh, xh = lg.ib_adapt_flow(fb, mu.cpu().numpy(), nu.cpu().numpy(), wts, 1e-3, blocks, 1)
    t_host = (time.time() - t0) * 1e3
    same = bool(np.array_equal(fh, fnew) and np.array_equal(xh, xnew))
    hk.close()
    out = {"scheme": "A", "stages": 3, "distinct_factors": 2, "force_solve": "direct", "create_s": round(t_create, 2),
           "steps": n, "ms_per_step": round(ms, 3), "ms_per_step_with_nonlinear_term": round(ms_ns, 3),
           "nonlinear_dt_over_dx": 1.0,
           "adapt": {"support_kernel_ms": round(tot / max(1, cnt), 4), "device_update_ms": round(t_dev, 3),
                     "host_update_ms": round(t_host, 2), "host_lists_equal": same,
                     "eps_supp": 1e-3, "eta": 1.0, "nbuf": 1, "flow_blocks_in": len(fb),
                     "flow_blocks_out": len(fnew), "xflow_blocks_out": len(xnew)}}
    log("IB HERK A: created in %.2f s (2 dense factors), %.2f ms per step, %.2f ms with the nonlinear term"
        % (t_create, ms, ms_ns))
    log("IB adaptive domain: support %.4f ms, device update %.3f ms (host form %.2f ms, same lists: %s), "
        "D_flow %d -> %d blocks (D_xflow %d)" % (out["adapt"]["support_kernel_ms"], t_dev, t_host, same, len(fb),
                                                 len(fnew), len(xnew)))
    return out


def dense_solve_bench(lg, torch, ctx, sys_, NL, F, Bk, evals, args):
    """The paper's own force solver (Sec. 3.2): C built once column by column
    (FP64 matvecs), factored by FP64 Cholesky with the inverse factor W kept,
    then every step's force is f = W^T (W b).  Timed on the same right-hand
    sides as the CG legs."""
    n = 3 * NL
    torch.cuda.synchronize()
    t0 = time.time()
    Cd = torch.empty((n, n), dtype=torch.float64, device="cuda")
    lg.ib_schur_dense(ctx, sys_, Cd)
    t_build = time.time() - t0
    Wd = torch.empty_like(Cd)
    C0 = Cd.clone()
    lg.ib_chol_factor(ctx, Cd, Wd)   # first factorisation: workspaces allocated
    # timed factorisation (warm), then one more with per-kernel events
    Cd.copy_(C0)
    torch.cuda.synchronize()
    t0 = time.time()
    lg.ib_chol_factor(ctx, Cd, Wd)
    t_fac = time.time() - t0
    Cd.copy_(C0)
    lg.lgfib_profile_reset(ctx)
    lg.lgfib_profile_enable(ctx, True)
    lg.ib_chol_factor(ctx, Cd, Wd)
    lg.lgfib_profile_enable(ctx, False)
    pf = lg.lgfib_profile_read(ctx)
    del Cd, C0
    gemm_ms = pf.get("k_gemm_f64", (0, 0.0))[1]
    leaf_ms = pf.get("k_chol_leaf", (0, 0.0))[1]
    # algorithmic work: n^3/3 for the factor and n^3/3 for its inverse
    flop = 2.0 * n ** 3 / 3.0
    f = torch.zeros((NL, 3), dtype=torch.float64, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms, errs = [], []
    for k in evals:
        e0.record()
        lg.ib_chol_solve(ctx, Wd, Bk[k].view(-1), f.view(-1))
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
        errs.append(float(torch.linalg.vector_norm(f - F[k]) / torch.linalg.vector_norm(F[k])))
    lg.lgfib_profile_reset(ctx)
    lg.lgfib_profile_enable(ctx, True)
    reps = 20
    for _ in range(reps):
        lg.ib_chol_solve(ctx, Wd, Bk[evals[0]].view(-1), f.view(-1))
    torch.cuda.synchronize()
    lg.lgfib_profile_enable(ctx, False)
    ps = lg.lgfib_profile_read(ctx)
    solve_ms = sum(v[1] for k_, v in ps.items() if k_.startswith("k_trmv")) / reps
    nbytes = 8.0 * n * (n + 1)   # each half of W read once per product
    del Wd
    out = {"unknowns": n, "dense_build_s": round(t_build, 3), "factor_s": round(t_fac, 4),
           "factor_kernels_ms": {"k_gemm_f64": round(gemm_ms, 2), "k_chol_leaf": round(leaf_ms, 2)},
           "factor_roofline": {"bound": "mfma", "achieved": round(flop / (t_fac * 1e12), 2), "peak": 78.6,
                               "unit": "TFLOP/s", "frac": round(flop / (t_fac * 1e12) / 78.6, 4),
                               "flop": flop},
           "solve_ms": round(float(np.mean(ms)), 4), "max_err_vs_history": float(np.max(errs)),
           "solve_roofline": {"bound": "hbm", "achieved": round(nbytes / (solve_ms * 1e-3) / 1e9, 1),
                              "peak": 8000.0, "unit": "GB/s",
                              "frac": round(nbytes / (solve_ms * 1e-3) / 1e9 / 8000.0, 4),
                              "bytes_per_solve": nbytes, "avg_kernel_ms": round(solve_ms, 4)}}
    log("IB direct: C built in %.2f s, factored in %.3f s (%.1f TFLOP/s), solve %.4f ms (%.0f GB/s), err %.1e"
        % (t_build, t_fac, out["factor_roofline"]["achieved"], out["solve_ms"],
           out["solve_roofline"]["achieved"], out["max_err_vs_history"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--settle", type=float, default=0.5,
                    help="keep warming up until this many seconds of GPU work have run")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ib", action="store_true", help="skip the immersed-boundary force-solve section")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-applies section")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision sweep")
    ap.add_argument("--no-refresh", action="store_true", help="skip the velocity-refresh section")
    ap.add_argument("--no-multilevel", action="store_true", help="skip the multilevel-evaluator section")
    ap.add_argument("--ml-diameter", type=int, default=256, help="sphere diameter (cells) of the multilevel set")
    ap.add_argument("--batch-branches", type=int, default=4, help="concurrent graph branches of the batched launch")
    ap.add_argument("--ib-markers", type=int, default=2200,
                    help="markers on the D = 32 sphere (2200: minimum spacing 1.055 dx)")
    ap.add_argument("--ib-steps", type=int, default=1000)
    ap.add_argument("--ib-train", type=int, default=500)
    ap.add_argument("--ib-epochs", type=int, default=20)
    ap.add_argument("--herk-steps", type=int, default=20, help="Scheme A IF-HERK steps timed in the IB section")
    ap.add_argument("--ib-skip", type=int, default=20,
                    help="first training step (the impulsive start is left out of the training set)")
    ap.add_argument("--ib-eval-stride", type=int, default=1)
    ap.add_argument("--ib-listed-markers", type=int, default=4000,
                    help="markers of the listed sphere leg (history by dense Cholesky; 0 skips it)")
    ap.add_argument("--ib-listed-stride", type=int, default=25,
                    help="evaluate every n-th step of the listed sphere leg")
    ap.add_argument("--ib-listed-maxit", type=int, default=30000)
    ap.add_argument("--ib-lanczos", type=int, default=200)
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

    # untimed warmup: at least W steps, and until the GPU has run for
    # settle seconds (a fresh box raises its clocks over the first ~0.1 s of
    # work; the first steps of a cold process run up to 3x slower)
    nwarm = 0
    tw0 = time.perf_counter()
    while nwarm < args.warmup or time.perf_counter() - tw0 < args.settle:
        lg.lgf_poisson_apply(ctx, tbl, B, blocks, blocks, f, u, stream=stream)
        nwarm += 1
        if nwarm % 16 == 0:
            torch.cuda.synchronize()
    # one more untimed step with the kernel timers on, so their events exist
    lg.lgfib_profile_enable(ctx, True)
    lg.lgf_poisson_apply(ctx, tbl, B, blocks, blocks, f, u, stream=stream)
    torch.cuda.synchronize()
    lg.lgfib_profile_enable(ctx, False)
    log("warmup done (%d steps, %.2f s)" % (nwarm, time.perf_counter() - tw0))

    # the timed steps (no kernel timers), then the same steps again with the
    # kernel timers on for the per-kernel figures
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        lg.lgf_poisson_apply(ctx, tbl, B, blocks, blocks, f, u, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    value = ncomp * cells / (ms * 1e-3) / 1e9
    log("timed %d steps: %.4f ms/step, %.2f Gcells/s" % (args.steps, ms, value))
    lg.lgfib_profile_reset(ctx)
    lg.lgfib_profile_enable(ctx, True)
    for i in range(args.steps):
        lg.lgf_poisson_apply(ctx, tbl, B, blocks, blocks, f, u, stream=stream)
    torch.cuda.synchronize()
    lg.lgfib_profile_enable(ctx, False)
    prof = lg.lgfib_profile_read(ctx)

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
        # a bounded, time-boxed sample: chunks of seeded targets (half next to
        # the plate, half uniform) until about cpu_seconds of oracle work
        chunk = 8 * oracle.num_threads()
        near_cells = np.array([int(b) * B ** 3 + int(v) for b in near for v in range(B ** 3)], dtype=np.int64)
        nn = min(20000, len(near_cells))
        order = np.stack([g.permutation(near_cells)[:nn], g.choice(cells, nn, replace=False)], axis=1).reshape(-1)
        _, first = np.unique(order, return_index=True)   # interleaved near / uniform, first occurrences
        order = order[np.sort(first)]
        refs = [[] for _ in range(ncomp)]
        done = 0
        t0 = time.perf_counter()
        while done < len(order) and time.perf_counter() - t0 < args.cpu_seconds:
            part = order[done:done + chunk]
            for c in range(ncomp):
                refs[c].append(oracle.conv_direct(G, cellsxyz, f64[c].reshape(-1), cellsxyz[part]))
            done += len(part)
        tcpu = time.perf_counter() - t0
        sample = order[:done]
        refs = [np.concatenate(r) for r in refs]
        picks = np.intersect1d(sample, near_cells)
        log("oracle sample: %d target cells x %d components in %.1f s" % (len(sample), ncomp, tcpu))
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
                             "traffic": kernel_traffic("k_if_apply"),
                             "bytes_per_launch": if_bytes, "avg_launch_ms": round(if_avg, 5)}}
    log("E(0.1) apply: %.4f ms, %.1f Gcells/s" % (ms_if, if_apply["Gcells_per_s"]))

    refresh = None if args.no_refresh else refresh_bench(lg, torch, workloads, ctx, args, tbl, blocks, B, f, stream)
    precision = None if args.no_precision else precision_bench(lg, torch, workloads, ctx, args, f64, blocks, B,
                                                                  tbl, G)
    batched = None if args.no_batch else batch_bench(lg, torch, workloads, ctx, args)
    multilevel = None if args.no_multilevel else multilevel_bench(lg, torch, workloads, ctx, args)
    ib = None if args.no_ib else ib_force_bench(lg, torch, workloads, ctx, args, args.ib_markers,
                                                stride=args.ib_eval_stride)
    ib_listed = None
    if not args.no_ib and args.ib_listed_markers > 0:
        ib_listed = ib_force_bench(lg, torch, workloads, ctx, args, args.ib_listed_markers, history_direct=True,
                                   stride=args.ib_listed_stride, maxit=args.ib_listed_maxit, extras=False)

    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 256 MiB device-to-device copies")

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gcells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "warmup_run": {"steps": nwarm, "settle_s": args.settle},
        "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "plate_wake_vector_poisson", "blocks": nblk, "B": B, "cells_per_component": cells,
                   "components": ncomp, "box_cells": N, "fft": P, "path": "box_fft"},
        "roofline": roofline,
        "step_model_GBs": round(step_bytes / (ms * 1e-3) / 1e9, 1),
        "kernels": {k: {"avg_ms": round(v["avg_ms"], 5), "GBs": round(v["GBs"], 1)} for k, v in kern.items()},
        "max_rel_err": max(errs) if errs else None,
        "cpu_baseline": cpu,
        "if_apply": if_apply,
        "velocity_refresh": refresh,
        "fp64_apply": (precision or {}).get("variants", {}).get("box_fft_f64"),
        "precision": precision,
        "batched": batched,
        "multilevel": multilevel,
        "ib_force_solve": ib,
        "ib_force_solve_listed": ib_listed,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
