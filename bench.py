"""Benchmark: compressed (DIT) SpMV vs plain ELL on MI355X, plus CG time to 1e-10.

Workload (default): the HPCG 27-point stencil matrix on a 104^3 grid
(n = 1,124,864, nnz = 29,791,000, diagonal 26, neighbours -1), x ~ U[-1, 1]
(seed 0).  One step = one y = A x over the DIT-compressed matrix (pattern ID +
terminal indices per row, value table {-1, 26}).  Inputs are resident in HBM
before the timed region.  The same matrix as FP64 ELL is timed beside it, and
(unless --no-cg) CG to 1e-10 on the 192^3 grid with b = A*1: FP64, mixed
precision, preconditioned by one SymGS sweep, and preconditioned by one
multigrid V-cycle over the 192/96/48/24 grid hierarchy.

Prints one JSON line (see the repository's design notes for the fields).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COLD_REPS = 50  # cold-MALL launches of the DIT kernel quoted against the HBM roof
PROFILE_PMC = os.path.join(ROOT, "profiles", "dit_spmv_stencil104_cold_pmc.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1612_00530_amd", "csrc", "spmv.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profile(kernel, rows_per_block):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it was
    taken from this kernel source in this launch configuration (else None)."""
    if not os.path.exists(PROFILE_PMC):
        return None
    txt = open(PROFILE_PMC).read()

    def field(name):
        m = re.search(name + r":\s*(\S+)", txt)
        return m.group(1) if m else None

    if field("kernel_source_sha256_16") != kernel_source_hash():
        return None
    m = re.search(r"^traffic:\s+" + re.escape(kernel) + r"\s+" + str(int(rows_per_block)) + r"\s+(\d+)\s+(\d+)\s*$",
                  txt, re.M)
    if m is None:
        return None
    return float(m.group(1)) + float(m.group(2))


def time_launches(fn, reps, torch):
    """Mean duration (ms) of one launch, from a HIP event pair around each launch on its stream."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    return float(t.mean()), float(np.median(t)), float(t.min())


def time_batch(fn, reps, torch):
    """Mean duration (ms) of one launch over `reps` back-to-back launches (one event pair)."""
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def time_cold(fn, reps, torch, flush):
    """Duration (ms) of one launch after the 256 MB last-level (MALL) cache has
    been overwritten by a 1 GiB fill, so that the launch reads HBM, not MALL.

    An event recorded between the fill and the launch would add the dispatch
    gap of a launch that starts from an idle queue, so the kernel time is
    taken as a difference: event pairs around [fill, launch] and around
    [fill] alone, interleaved; kernel = mean(fill + launch) - mean(fill).
    Returns (difference mean, single-launch event pair median) in ms."""
    mk = lambda: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    both, alone, single = [mk() for _ in range(reps)], [mk() for _ in range(reps)], [mk() for _ in range(reps)]
    for r in range(reps):
        a, b = alone[r]
        a.record()
        flush.fill_(1.0)
        b.record()
        a, b = both[r]
        a.record()
        flush.fill_(1.0)
        fn()
        b.record()
        flush.fill_(1.0)
        a, b = single[r]
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t_both = np.array([a.elapsed_time(b) for a, b in both])
    t_alone = np.array([a.elapsed_time(b) for a, b in alone])
    t_single = np.array([a.elapsed_time(b) for a, b in single])
    return float(t_both.mean() - t_alone.mean()), float(np.median(t_single))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--grid", type=int, default=104)
    ap.add_argument("--cg-grid", type=int, default=192)
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-irregular", action="store_true")
    ap.add_argument("--no-reorder", action="store_true")
    ap.add_argument("--batched-systems", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 512 MiB read+write elementwise kernel (counter calibration)")
    ap.add_argument("--cold-only", action="store_true",
                    help="counter runs: compress and tune the 104^3 DIT matrix, then only the cold-MALL "
                         "launches of the roofline (each after a 1 GiB fill), and exit")
    ap.add_argument("--pmc-configs", action="store_true",
                    help="with --cold-only: before the roofline launches, also launch the FP64 DIT kernel "
                         "cold in each tuner candidate configuration (register kernel at 256/512/768/1024 "
                         "rows per block, plane-marching kernel at 256/512/1024) so that one counter run "
                         "covers whichever the tuner picks")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1612_00530_amd as P
    from synthetic import stencil27, uniform_vector

    P.load()  # fails loudly when the HIP library is missing
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.calib_copy:
        a = torch.ones(64 << 20, dtype=torch.float64, device=dev)  # 512 MiB
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    g = args.grid
    log(f"[bench] generating 27-point stencil {g}^3")
    A = stencil27(g, g, g)
    n, nnz = A.n_rows, A.nnz
    rp, col, val = (torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col, A.val))
    x = torch.from_numpy(uniform_vector(n, seed=0)).to(dev)
    y = torch.empty(n, dtype=torch.float64, device=dev)

    log("[bench] compressing (DIT, ELL)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    D = P.compress(rp, col, val, n_cols=n, fmt="DIT")
    torch.cuda.synchronize()
    t_compress = time.perf_counter() - t0
    E = P.compress(rp, col, val, n_cols=n, fmt="ELL")
    del rp, col, val
    tuned = None
    if not args.no_tune:
        tuned = D.tune(torch.float64)
        tuned_f32 = D.tune(torch.float32)
        log(f"[bench] tuned DIT: FP64 {tuned}, FP32 {tuned_f32}")
    dinf, einf = D.info(), E.info()
    if args.cold_only:
        # counter and trace runs of the roofline launches: cold launches only
        # (each of the tuner's candidate configurations with --pmc-configs, then
        # the tuned -- or, with --no-tune, the default 512-row -- configuration)
        flush = torch.empty(128 << 20, dtype=torch.float64, device=dev)
        if args.no_tune:
            D.set_config(512, 1)
        keep = D.info()
        if args.pmc_configs:
            time_cold(lambda: D.spmv(x, y), 5, torch, flush)  # first-use costs out of the first config
            for lds, rows_list in ((1, (256, 512, 768, 1024)), (2, (256, 512, 1024))):
                for rows in rows_list:
                    D.set_config(rows, lds)
                    cm, _ = time_cold(lambda: D.spmv(x, y), COLD_REPS, torch, flush)
                    log(f"[bench] cold {D.info()['kernel_name']} {rows} rows: kernel {cm * 1000:.3f} us")
            D.set_config(keep["rows_per_block"], {0: 0, 1: 1, 2: 1, 3: 2}[keep["kernel"]])
        c_mean, c_med = time_cold(lambda: D.spmv(x, y), COLD_REPS, torch, flush)
        log(f"[bench] cold-only: {keep['kernel_name']} {keep['rows_per_block']} rows, {2 * COLD_REPS} cold "
            f"launches, kernel {c_mean * 1000:.3f} us (fill + launch minus fill), single-launch event pair "
            f"median {c_med * 1000:.3f} us")
        return

    # timed region: K back-to-back compressed SpMVs, bracketed by host clock and
    # by a HIP event pair on the stream the kernel is launched on
    for _ in range(args.warmup):
        D.spmv(x, y)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        D.spmv(x, y)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1000.0 * wall / args.steps
    gflops = 2.0 * nnz / (ms_per_step * 1e-3) / 1e9
    log(f"[bench] DIT: {ms_per_step * 1000:.2f} us/step, {gflops:.1f} Gflops")

    # dominant kernel: average launch duration over the timed region (events);
    # single-launch event pairs give the spread
    k_mean = ev0.elapsed_time(ev1) / args.steps
    _, k_med, k_min = time_launches(lambda: D.spmv(x, y), args.steps, torch)
    alg_dit = dinf["bytes_stream"] + 8 * n + 8 * n
    achieved = alg_dit / (k_mean * 1e-3) / 1e9
    traffic = traffic_from_profile(dinf["kernel_name"], dinf["rows_per_block"])

    # ELL baseline, same matrix and vectors
    for _ in range(args.warmup):
        E.spmv(x, y)
    e_mean = time_batch(lambda: E.spmv(x, y), max(20, args.steps // 2), torch)
    alg_ell = einf["bytes_stream"] + 8 * n + 8 * n
    ell_gflops = 2.0 * nnz / (e_mean * 1e-3) / 1e9
    log(f"[bench] ELL: {e_mean * 1000:.2f} us/launch, {ell_gflops:.1f} Gflops, "
        f"{alg_ell / (e_mean * 1e-3) / 1e9:.0f} GB/s")

    # parity spot check of this very launch configuration against the oracle
    out = {}
    if not args.no_cpu:
        import oracle

        yref = oracle.spmv(A, x.cpu().numpy())
        yg = D.spmv(x, y).cpu().numpy()
        rows = np.repeat(np.arange(n), np.diff(A.row_ptr))
        scale = np.bincount(rows, weights=np.abs(A.val) * np.abs(x.cpu().numpy()[A.col]), minlength=n)
        out["parity_max_rel_err"] = float((np.abs(yg - yref) / scale).max())
        # CPU baseline: the oracle as it stands, timed on the host cores
        reps, t_cpu = 0, 0.0
        xh = x.cpu().numpy()
        t0 = time.perf_counter()
        while reps < 3 or (time.perf_counter() - t0) < args.cpu_seconds:
            oracle.spmv(A, xh)
            reps += 1
        t_cpu = (time.perf_counter() - t0) / reps
        # and on one thread (a few repetitions)
        nthr = oracle.threads()
        oracle.set_threads(1)
        reps1, t1 = 0, time.perf_counter()
        while reps1 < 2 or (time.perf_counter() - t1) < min(3.0, args.cpu_seconds):
            oracle.spmv(A, xh)
            reps1 += 1
        t_cpu1 = (time.perf_counter() - t1) / reps1
        oracle.set_threads(nthr)
        cpu_model = ""
        try:
            with open("/proc/cpuinfo") as f:
                cpu_model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
        except OSError:
            pass
        out["cpu_baseline"] = {"value": 2.0 * nnz / t_cpu / 1e9, "unit": "Gflops", "cores": nthr,
                               "cpu_model": cpu_model,
                               "kind": "oracle",
                               "sample": f"{reps} full CSR SpMVs of the {g}^3 stencil matrix (FP64, OpenMP rows)",
                               "value_1thread": round(2.0 * nnz / t_cpu1 / 1e9, 3),
                               "sample_1thread": f"{reps1} full CSR SpMVs on one thread"}
        log(f"[bench] CPU oracle: {out['cpu_baseline']['value']:.2f} Gflops on {oracle.threads()} threads")

    # FP32 DIT SpMV of the same matrix (the inner kernel of the mixed-precision CG)
    x32, y32 = x.float(), y.float()
    for _ in range(5):
        D.spmv(x32, y32)
    f_mean = time_batch(lambda: D.spmv(x32, y32), max(20, args.steps // 2), torch)

    # DITV: the values registered in the pattern table too, a row stores only its ID
    rp, col, val = (torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col, A.val))
    DV = P.compress(rp, col, val, n_cols=n, fmt="DITV")
    del rp, col, val
    tuned_v = DV.tune(torch.float64) if not args.no_tune else None
    vinf = DV.info()
    for _ in range(5):
        DV.spmv(x, y)
    v_mean = time_batch(lambda: DV.spmv(x, y), max(20, args.steps // 2), torch)
    alg_v = vinf["bytes_stream"] + 8 * n + 8 * n
    ditv = {"launch_us_mean": round(v_mean * 1000, 3), "gflops": round(2.0 * nnz / (v_mean * 1e-3) / 1e9, 1),
            "bytes_per_row": round(vinf["bytes_stream"] / n, 3), "bytes_per_launch": alg_v,
            "GBps": round(alg_v / (v_mean * 1e-3) / 1e9, 1), "speedup_vs_ell": round(e_mean / v_mean, 3),
            "kernel": vinf["kernel_name"], "tuned": tuned_v}
    log(f"[bench] DITV: {ditv['launch_us_mean']} us, {ditv['gflops']} Gflops, {ditv['bytes_per_row']} B/row")
    del DV

    # BMASK: a bitmask per row over the matrix's 27 displacements, plus the V[1] mask
    rp, col, val = (torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col, A.val))
    DB = P.compress(rp, col, val, n_cols=n, fmt="BMASK")
    del rp, col, val
    tuned_b = DB.tune(torch.float64) if not args.no_tune else None
    binf = DB.info()
    for _ in range(5):
        DB.spmv(x, y)
    bm_mean = time_batch(lambda: DB.spmv(x, y), max(20, args.steps // 2), torch)
    alg_b = binf["bytes_stream"] + 8 * n + 8 * n
    bmask = {"launch_us_mean": round(bm_mean * 1000, 3), "gflops": round(2.0 * nnz / (bm_mean * 1e-3) / 1e9, 1),
             "bytes_per_row": round(binf["bytes_stream"] / n, 3), "bytes_per_launch": alg_b,
             "GBps": round(alg_b / (bm_mean * 1e-3) / 1e9, 1), "speedup_vs_ell": round(e_mean / bm_mean, 3),
             "kernel": binf["kernel_name"], "displacements": binf["P"], "tuned": tuned_b}
    log(f"[bench] BMASK: {bmask['launch_us_mean']} us, {bmask['gflops']} Gflops, {bmask['bytes_per_row']} B/row")
    del DB

    # multicolor symmetric Gauss-Seidel, one sweep (colors forward, then backward): DIT and ELL
    bgs = torch.from_numpy(uniform_vector(n, seed=6)).to(dev)
    xgs = torch.zeros(n, dtype=torch.float64, device=dev)
    n_colors = D.colors()[0]
    E.colors()
    D.symgs(bgs, xgs)
    E.symgs(bgs, xgs)
    g_dit = time_batch(lambda: D.symgs(bgs, xgs), max(10, args.steps // 10), torch)
    g_ell = time_batch(lambda: E.symgs(bgs, xgs), max(10, args.steps // 10), torch)
    # the same sweep on the color-ordered twin (each color one contiguous range
    # of rows): what the preconditioned solvers run
    DC, cperm = D.color_order()
    bgs_c, xgs_c = bgs[cperm.long()].contiguous(), xgs[cperm.long()].contiguous()
    DC.symgs(bgs_c, xgs_c)
    g_ord = time_batch(lambda: DC.symgs(bgs_c, xgs_c), max(10, args.steps // 10), torch)
    del DC, cperm, bgs_c, xgs_c
    symgs = {"colors": n_colors, "launches_per_sweep": max(2 * n_colors - 1, 0),
             "dit_us": round(g_dit * 1000, 3), "dit_gflops": round(4.0 * nnz / (g_dit * 1e-3) / 1e9, 1),
             "dit_color_ordered_us": round(g_ord * 1000, 3),
             "dit_color_ordered_gflops": round(4.0 * nnz / (g_ord * 1e-3) / 1e9, 1),
             "ell_us": round(g_ell * 1000, 3), "ell_gflops": round(4.0 * nnz / (g_ell * 1e-3) / 1e9, 1),
             "speedup_vs_ell": round(g_ell / g_dit, 3)}
    log(f"[bench] SymGS sweep: DIT {symgs['dit_us']} us (color-ordered {symgs['dit_color_ordered_us']} us), "
        f"ELL {symgs['ell_us']} us ({n_colors} colors)")
    del bgs, xgs

    # block SpMV, 8 right-hand sides (row-interleaved), same matrix: DIT and ELL
    X8 = torch.from_numpy(np.random.default_rng(5).uniform(-1.0, 1.0, (n, 8))).to(dev)
    Y8 = torch.empty((n, 8), dtype=torch.float64, device=dev)
    tuned_block = D.tune(torch.float64, nrhs=8) if not args.no_tune else None
    for _ in range(5):
        D.spmv_block(X8, Y8)
        E.spmv_block(X8, Y8)
    b_dit = time_batch(lambda: D.spmv_block(X8, Y8), max(20, args.steps // 4), torch)
    b_ell = time_batch(lambda: E.spmv_block(X8, Y8), max(20, args.steps // 4), torch)
    block8 = {"nrhs": 8, "dit_us": round(b_dit * 1000, 3), "dit_gflops": round(16.0 * nnz / (b_dit * 1e-3) / 1e9, 1),
              "ell_us": round(b_ell * 1000, 3), "ell_gflops": round(16.0 * nnz / (b_ell * 1e-3) / 1e9, 1),
              "dit_GBps": round((dinf["bytes_stream"] + 128 * n) / (b_dit * 1e-3) / 1e9, 1),
              "tuned": tuned_block}
    log(f"[bench] block SpMV x8: DIT {block8['dit_us']} us ({block8['dit_gflops']} Gflops), "
        f"ELL {block8['ell_us']} us ({block8['ell_gflops']} Gflops)")
    del X8, Y8

    # practical HBM rate on this machine: a 1 GiB -> 1 GiB device copy (4x the MALL)
    src = torch.ones(128 << 20, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    c_ms = time_batch(lambda: dst.copy_(src), 10, torch)
    practical_gbs = 2.0 * src.numel() * 8 / (c_ms * 1e-3) / 1e9
    log(f"[bench] 1 GiB device copy: {practical_gbs:.0f} GB/s (read + write)")
    del src, dst

    # cold-cache launches: the MALL flushed before each one.  These are the
    # launches the roofline quotes against HBM (a warm launch reads its 21 MB
    # working set from the 256 MB MALL, not from HBM).
    flush = torch.empty(128 << 20, dtype=torch.float64, device=dev)
    time_cold(lambda: D.spmv(x, y), 5, torch, flush)  # first-use costs and clocks out of the measurement
    c_dit_mean, c_dit = time_cold(lambda: D.spmv(x, y), COLD_REPS, torch, flush)
    c_ell_mean, c_ell = time_cold(lambda: E.spmv(x, y), 30, torch, flush)
    del flush
    achieved_cold = alg_dit / (c_dit_mean * 1e-3) / 1e9
    # kernel times by difference (fill + launch minus fill); the single-launch
    # event pairs (which add the dispatch gap of an idle queue) beside them
    cold = {"dit_us": round(c_dit_mean * 1000, 3), "dit_gflops": round(2.0 * nnz / (c_dit_mean * 1e-3) / 1e9, 1),
            "dit_GBps": round(alg_dit / (c_dit_mean * 1e-3) / 1e9, 1),
            "ell_us": round(c_ell_mean * 1000, 3), "ell_gflops": round(2.0 * nnz / (c_ell_mean * 1e-3) / 1e9, 1),
            "ell_GBps": round(alg_ell / (c_ell_mean * 1e-3) / 1e9, 1),
            "speedup_vs_ell": round(c_ell_mean / c_dit_mean, 2),
            "single_event_pair_us_median": {"dit": round(c_dit * 1000, 3), "ell": round(c_ell * 1000, 3)}}
    log(f"[bench] cold MALL: DIT {cold['dit_us']} us, ELL {cold['ell_us']} us ({cold['ell_GBps']} GB/s); "
        f"single event pairs {cold['single_event_pair_us_median']}")

    irregular = None
    if not args.no_irregular:
        irregular = run_irregular(P, torch, dev, args.steps)
    reordered = None
    if not args.no_reorder:
        reordered = run_reorder(P, torch, dev, args.steps)
    cg = None
    if not args.no_cg:
        cg = run_cg(args.cg_grid, P, torch, dev)
    batched = None
    if not args.no_batched:
        batched = run_batched(P, torch, dev, args.batched_systems)

    res = {
        "metric": "SpMV Gflops + effective HBM GB/s, compressed vs plain ELL; CG time to 1e-10",
        "value": round(gflops, 2),
        "unit": "Gflops",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"27-point stencil {g}^3 (HPCG matrix), DIT-compressed FP64 SpMV",
                   "grid": [g, g, g], "n": n, "nnz": nnz, "format": "DIT",
                   "rows_per_block": dinf["rows_per_block"], "lds_windows": dinf["lds_windows"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved_cold, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved_cold / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "mode": f"cold MALL: {COLD_REPS} launches, each right after a 1 GiB fill; kernel time = "
                             f"mean of HIP event pairs around [fill, launch] minus those around [fill] alone, "
                             f"on the launch stream",
                     "practical_peak_GBps": round(practical_gbs, 1),
                     "frac_of_practical": round(achieved_cold / practical_gbs, 4),
                     "kernel": dinf["kernel_name"], "algorithmic_bytes_per_launch": alg_dit,
                     "launch_us_mean": round(c_dit_mean * 1000, 3),
                     "single_launch_event_us_median": round(c_dit * 1000, 3),
                     "warm_mall": {"achieved": round(achieved, 1), "frac": round(achieved / HBM_PEAK_GBS, 4),
                                   "launch_us_mean": round(k_mean * 1000, 3),
                                   "single_launch_event_us_median": round(k_med * 1000, 3),
                                   "note": "back-to-back launches of the timed region; the 21 MB working "
                                           "set is resident in the 256 MB MALL, so this is not an HBM rate"}},
        "cpu_baseline": out.get("cpu_baseline"),
        "effective_GBps_actual": round(alg_dit / (ms_per_step * 1e-3) / 1e9, 1),
        "effective_GBps_equiv_uncompressed": round(alg_ell / (ms_per_step * 1e-3) / 1e9, 1),
        "ell": {"gflops": round(ell_gflops, 2), "launch_us_mean": round(e_mean * 1000, 3),
                "GBps": round(alg_ell / (e_mean * 1e-3) / 1e9, 1), "bytes_per_launch": alg_ell,
                "hbm_frac": round(alg_ell / (e_mean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "speedup_vs_ell": round(gflops / ell_gflops, 3),
        "compress_seconds": round(t_compress, 3),
        "bytes_per_row": {"DIT": round(dinf["bytes_stream"] / n, 3), "ELL": round(einf["bytes_stream"] / n, 3),
                          "DIT_paper_widths": round(dinf["bytes_paper"] / n, 3)},
        "parity_max_rel_err": out.get("parity_max_rel_err"),
        "tuned": tuned,
        "cold_mall": cold,
        "block_spmv": block8,
        "dit_f32": {"launch_us_mean": round(f_mean * 1000, 3), "gflops": round(2.0 * nnz / (f_mean * 1e-3) / 1e9, 2)},
        "ditv": ditv,
        "bmask": bmask,
        "symgs": symgs,
        "irregular": irregular,
        "reorder": reordered,
        "cg": cg,
        "batched_cg": batched,
        "paper_context_gflops_per_chip": {"uncompressed": 11.6, "compressed": 32.4, "hardware": "PEZY-SC"},
    }
    print(json.dumps(res), flush=True)


def run_irregular(P, torch, dev, steps):
    """SpMV on the irregularised 128^3 stencil: DIT (pattern IDs + raw values + escapes) vs ELL."""
    from synthetic import stencil27_irregular, uniform_vector

    log("[bench] irregular 128^3")
    A = stencil27_irregular(128, 128, 128, seed=0)
    rp, col, val = (torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col, A.val))
    D = P.compress(rp, col, val, n_cols=A.n_cols, fmt="DIT")
    E = P.compress(rp, col, val, n_cols=A.n_cols, fmt="ELL")
    B = P.compress(rp, col, val, n_cols=A.n_cols, fmt="BMASK")
    del rp, col, val
    tuned = D.tune(torch.float64)
    tuned_b = B.tune(torch.float64)
    x = torch.from_numpy(uniform_vector(A.n_cols, seed=0)).to(dev)
    y = torch.empty(A.n_rows, dtype=torch.float64, device=dev)
    d_us = time_batch(lambda: D.spmv(x, y), max(20, steps // 2), torch) * 1000
    e_us = time_batch(lambda: E.spmv(x, y), max(20, steps // 2), torch) * 1000
    b_us = time_batch(lambda: B.spmv(x, y), max(20, steps // 2), torch) * 1000
    di, ei, bi = D.info(), E.info(), B.info()
    res = {"grid": [128, 128, 128], "n": A.n_rows, "nnz": A.nnz, "P": di["P"], "K": di["K"],
           "escape_rows": di["n_escape_rows"], "dit_us": round(d_us, 3), "ell_us": round(e_us, 3),
           "dit_gflops": round(2.0 * A.nnz / (d_us * 1e-6) / 1e9, 2),
           "ell_gflops": round(2.0 * A.nnz / (e_us * 1e-6) / 1e9, 2), "speedup": round(e_us / d_us, 3),
           "dit_bytes": di["bytes_stream"] + 16 * A.n_rows, "ell_bytes": ei["bytes_stream"] + 16 * A.n_rows,
           "dit_GBps": round((di["bytes_stream"] + 16 * A.n_rows) / (d_us * 1e-6) / 1e9, 1), "tuned": tuned,
           "bmask": {"us": round(b_us, 3), "gflops": round(2.0 * A.nnz / (b_us * 1e-6) / 1e9, 2),
                     "bytes": bi["bytes_stream"] + 16 * A.n_rows,
                     "GBps": round((bi["bytes_stream"] + 16 * A.n_rows) / (b_us * 1e-6) / 1e9, 1),
                     "hbm_frac": round((bi["bytes_stream"] + 16 * A.n_rows) / (b_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                     "speedup_vs_ell": round(e_us / b_us, 3), "speedup_vs_dit": round(d_us / b_us, 3),
                     "escape_rows": bi["n_escape_rows"], "displacements": bi["P"], "mask_bytes": bi["id_bytes"],
                     "tuned": tuned_b}}
    log(f"[bench] irregular: DIT {d_us:.1f} us vs ELL {e_us:.1f} us vs BMASK {b_us:.1f} us")
    return res


def run_reorder(P, torch, dev, steps):
    """The 104^3 stencil under a random row/column labelling (seed 0, applied with
    the library's own permute): SpMV as given vs after reverse Cuthill-McKee
    (spmv_rcm + spmv_permute), each compressed with format AUTO."""
    from synthetic import stencil27, uniform_vector

    log("[bench] reorder: scrambled 104^3")
    A = stencil27(104, 104, 104)
    rp, col, val = (torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col, A.val))
    scramble = torch.from_numpy(np.random.default_rng(0).permutation(A.n_rows).astype(np.int32)).to(dev)
    srp, scol, sval = P.permute(rp, col, val, scramble)
    del rp, col, val
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    perm = P.rcm(srp, scol)
    torch.cuda.synchronize()
    t_rcm = time.perf_counter() - t0
    t0 = time.perf_counter()
    brp, bcol, bval = P.permute(srp, scol, sval, perm)
    torch.cuda.synchronize()
    t_perm = time.perf_counter() - t0

    def bandwidth(rp_, col_):
        rows = torch.repeat_interleave(torch.arange(A.n_rows, device=dev), rp_[1:] - rp_[:-1])
        return int((rows - col_.long()).abs().max().item())

    res = {"grid": [104, 104, 104], "n": A.n_rows, "nnz": A.nnz, "rcm_seconds": round(t_rcm, 4),
           "permute_seconds": round(t_perm, 4)}
    x = torch.from_numpy(uniform_vector(A.n_cols, seed=0)).to(dev)
    y = torch.empty(A.n_rows, dtype=torch.float64, device=dev)
    for name, (r_, c_, v_) in (("scrambled", (srp, scol, sval)), ("rcm", (brp, bcol, bval))):
        M = P.compress(r_, c_, v_, n_cols=A.n_cols, fmt="AUTO")
        M.tune(torch.float64)
        us = time_batch(lambda: M.spmv(x, y), max(20, steps // 2), torch) * 1000
        info = M.info()
        res[name] = {"format": info["fmt_name"] if "fmt_name" in info else info.get("fmt"), "P": info["P"],
                     "escape_rows": info["n_escape_rows"], "bandwidth": bandwidth(r_, c_), "us": round(us, 3),
                     "gflops": round(2.0 * A.nnz / (us * 1e-6) / 1e9, 2)}
        log(f"[bench] reorder {name}: {us:.1f} us, bandwidth {res[name]['bandwidth']}, format {res[name]['format']}")
        del M
    res["speedup"] = round(res["scrambled"]["us"] / res["rcm"]["us"], 3)
    return res


def run_batched(P, torch, dev, n_sys):
    """64 systems, grid dims U{16..96} (seed 0), 8 right-hand sides U[-1,1]: batched CG to 1e-10."""
    from synthetic import batched_grids, stencil27

    grids = batched_grids(n_sys, 16, 96, seed=0)
    log(f"[bench] batched: generating {n_sys} systems")
    mats, bs = [], []
    rows = nnz = 0
    for s, g in enumerate(grids):
        A = stencil27(*g)
        rows += A.n_rows
        nnz += A.nnz
        rp, col, val = (torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col, A.val))
        mats.append(P.compress(rp, col, val, n_cols=A.n_cols, fmt="DIT"))
        rng = np.random.default_rng(1000 + s)
        bs.append(torch.from_numpy(rng.uniform(-1.0, 1.0, (A.n_rows, 8))).to(dev))
    res = {"systems": n_sys, "nrhs": 8, "rows": rows, "nnz": nnz, "rtol": 1e-10}
    P.cg_solve(mats, bs, nrhs=8, batched=2, max_iter=4)  # warm the code path
    for name, mode in (("graph", 2), ("batched_kernels", 1), ("sequential", 0)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, xs, stats = P.cg_solve(mats, bs, nrhs=8, batched=mode, max_iter=5000)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        its = [q["iters"] for q in stats]
        res[name] = {"status": st, "seconds": round(t, 4), "iters_min": min(its), "iters_max": max(its),
                     "relres_true_max": max(q["relres_true"] for q in stats)}
        log(f"[bench] batched {name}: {t * 1000:.1f} ms, iters {min(its)}..{max(its)}")
    res["speedup_graph_vs_sequential"] = round(res["sequential"]["seconds"] / res["graph"]["seconds"], 2)
    res["tuned_spmv"] = P.batched_config()  # form: 0 window-phased, 1 lane groups (rhs pairs), 2 lane groups
    return res


def run_cg(g, P, torch, dev):
    """CG to 1e-10 on the g^3 stencil with b = A*1: FP64 DIT, mixed precision DIT (iterative
    refinement; reliable updates), FP64 ELL."""
    from synthetic import stencil27, stencil_hierarchy

    log(f"[bench] CG: generating {g}^3")
    mg_levels = 4 if g % 8 == 0 else 1
    mats, f2c = stencil_hierarchy(g, g, g, mg_levels)
    A = mats[0]
    rp, col, val = (torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col, A.val))
    D = P.compress(rp, col, val, n_cols=A.n_cols, fmt="DIT")
    E = P.compress(rp, col, val, n_cols=A.n_cols, fmt="ELL")
    del rp, col, val
    res_tune = {"f64": D.tune(torch.float64), "f32": D.tune(torch.float32)}
    ones = torch.ones(A.n_cols, dtype=torch.float64, device=dev)
    b = D.spmv(ones)
    res = {"grid": [g, g, g], "n": A.n_rows, "nnz": A.nnz, "rtol": 1e-10, "tuned": res_tune}
    for name, M, mode, inner in (("fp64_dit", D, 0, 1e-5), ("mixed_dit", D, 1, 1e-5),
                                 ("mixed_reliable_dit", D, 3, 1e-2), ("fp64_ell", E, 0, 1e-5)):
        P.cg_solve(M, b, mode=mode, inner_rtol=inner, max_iter=20)  # warm-up of the code path
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, xs, stats = P.cg_solve(M, b, mode=mode, inner_rtol=inner, max_iter=5000)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        err = float((xs[0] - 1.0).abs().max().item())
        res[name] = {"status": st, "seconds": round(t, 5), "iters": stats[0]["iters"],
                     "outer_iters": stats[0]["outer_iters"], "relres_true_fp64": stats[0]["relres_true"],
                     "max_abs_err_vs_ones": err}
        log(f"[bench] CG {name}: {t * 1000:.2f} ms, {stats[0]['iters']} iters, relres {stats[0]['relres_true']:.2e}")
    for name in ("mixed_dit", "mixed_reliable_dit"):
        res[name]["speedup_vs_fp64_dit"] = round(res["fp64_dit"]["seconds"] / res[name]["seconds"], 3)
    # preconditioned: one SymGS sweep (mode 2); one V-cycle over the grid hierarchy
    levels = [D] + [P.compress(*(torch.from_numpy(a).to(dev) for a in (m.row_ptr, m.col, m.val)),
                               n_cols=m.n_cols, fmt="DIT") for m in mats[1:]]
    maps = [torch.from_numpy(f).to(dev) for f in f2c]
    for name, run in (("pcg_symgs_dit", lambda it: P.cg_solve(D, b, mode=2, max_iter=it)),
                      ("mg_pcg_dit", lambda it: P.cg_solve_mg(levels, maps, b, max_iter=it))):
        run(3)  # warm-up: coloring and code path
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = run(5000)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        st = out[0]
        x = out[1][0] if isinstance(out[1], list) else out[1]
        s0 = out[2][0] if isinstance(out[2], list) else out[2]
        res[name] = {"status": st, "seconds": round(t, 5), "iters": s0["iters"],
                     "relres_true_fp64": s0["relres_true"],
                     "max_abs_err_vs_ones": float((x - 1.0).abs().max().item())}
        if name == "mg_pcg_dit":
            res[name]["levels"] = [[m.grid[0], m.grid[1], m.grid[2]] for m in mats]
        log(f"[bench] CG {name}: {t * 1000:.2f} ms, {s0['iters']} iters, relres {s0['relres_true']:.2e}")
    return res


if __name__ == "__main__":
    main()
