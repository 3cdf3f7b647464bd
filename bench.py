#!/usr/bin/env python3
"""Benchmark of the band-arrowhead tile Cholesky on one MI355X.

Default workload (one "step" = the whole hot path on one matrix):
  variable-bandwidth SPD block-arrowhead matrix, n = 200,000 band rows whose
  half-width is piecewise constant per 5,000-row segment and uniform in
  [200, 800] (seed 2), a dense arrow of 100 rows (N = 200,100), values N(0,1)
  with diagonal = absolute row sum + 1; tile 64;
  step = value scatter + factorization and solve with 8 right-hand sides
  (seed 102) as one launch of the merged task graph + log-determinant.
Inputs are resident in HBM before the timed region.  `value` is TFLOP/s of
the algorithmic factorization flops F = sum_j (eta_j + 1)^2 over the whole
step time; the roofline object reports the merged factorization + solve
launch (algorithmic flops: F + 4 nnz(L) nrhs for the two solve sweeps).

Other workloads (--workload): small (n=2,000, w=50, a=10, 1 RHS, tile and ordering autotuned),
batch (512 uneven matrices in one launch), mixed (n=500,000, w=1,000,
a=200, FP32 updates + FP64 refinement, 16 RHS), spde (spatio-temporal CSC
input: 40 x 40 grid x 60 time steps, arrow 50), selinv (selected inversion
of the variable-bandwidth matrix's factor: A^{-1} on the tile pattern of L
and its diagonal; F = sum_j 2 eta_j (eta_j + 1)), serve (Poisson request
stream over 8 resident patterns, FP64 and mixed precision, p50/p99 latency),
ooc (out-of-core factorization of the variable-bandwidth matrix by band
segments, host values in and host factor out), banded (host context: LAPACK
band Cholesky plus the arrow on the host cores, beside the GPU's FP64
factorization of the same constant-width matrices), copycal (a device copy
of known size, to calibrate the HBM byte counters).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

UBLOCK = 0           # columns per 2 x 2 block update task (0: library default)
FP64_PEAK = 78.6     # TFLOP/s, MI355X dense FP64 (vector = matrix)
FP32_PEAK = 157.3    # TFLOP/s, MI355X dense FP32 matrix
HBM_PEAK = 8000.0    # GB/s


def flops_alg(f):
    """sum_j (eta_j + 1)^2, eta_j = entries below the diagonal in column j."""
    N = f.shape[0]
    d = np.zeros(N + 1, dtype=np.int64)
    np.add.at(d, f, 1)
    np.add.at(d, np.arange(N), -1)
    eta = np.cumsum(d)[:N]
    return float(np.sum((eta.astype(np.float64) + 1.0) ** 2))


def to_device_cols(B):
    import torch
    t = torch.empty((B.shape[1], B.shape[0]), dtype=torch.float64, device="cuda")
    t.copy_(torch.from_numpy(np.ascontiguousarray(B.T)))
    return t.t()


def measured_traffic(workload, tile):
    """HBM bytes per factorization launch from the committed rocprofv3 --pmc
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a copy of known size), or
    None when there is none for this workload or the kernel source changed
    since the counters were taken."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    src = os.path.join(root, "paper_2501_02483_amd", "csrc", "kernels.hip")
    prof = os.path.join(root, "profiles")
    if not os.path.isdir(prof):
        return None
    sha = hashlib.sha1(open(src, "rb").read()).hexdigest()
    for name in sorted(os.listdir(prof)):
        if not name.startswith("hbm_traffic_"):
            continue
        kv = {}
        for line in open(os.path.join(prof, name)):
            if ":" in line and not line.startswith(("#", "|", "-", " ")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get("workload") == "%s_T%d" % (workload, tile) and kv.get("kernels_sha1") == sha:
            return {"bytes": int(kv["traffic_bytes_per_launch"]), "fetch": int(kv["fetch_bytes_per_launch"]),
                    "write": int(kv["write_bytes_per_launch"]), "source": "profiles/" + name}
    return None


def cpu_threads():
    try:
        return int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    except ValueError:
        return os.cpu_count()


def cpu_model():
    """The host CPU's model name (lscpu), or the platform string."""
    import platform
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return platform.processor() or platform.machine()


def cpu_baseline_single(p, vals, B):
    """The oracle on the same matrix: factorization + solve + logdet, timed on
    all host threads (the full matrix: about 5-20 s of CPU work); and, for the
    per-core rate, the oracle's factorization with one thread on a sample of
    the same law (the first 20,000 band rows with their half-widths, and the
    arrow), timed also with all threads."""
    import oracle
    from paper_2501_02483_amd import inputs as I
    nt = cpu_threads()
    t0 = time.perf_counter()
    L, info = oracle.factor(p.f, vals, nthreads=nt)
    t1 = time.perf_counter()
    X = oracle.solve(p.f, L, B)
    ld = oracle.logdet(p.f, L)
    t2 = time.perf_counter()
    F = flops_alg(p.f)
    res = {"value": F / (t2 - t0) / 1e12, "unit": "TFLOP/s", "cores": nt, "kind": "oracle",
           "sample": "the full workload, one step (factorize %.2f s with %d threads + sequential "
                     "%d-RHS solve and logdet %.2f s)" % (t1 - t0, nt, B.shape[1], t2 - t1),
           "factorize_s": t1 - t0, "step_s": t2 - t0, "info": info, "cpu_model": cpu_model()}
    ns = min(p.n, 20000)
    if ns < p.n:
        fs = np.concatenate([p.f[:ns], np.zeros(p.a, dtype=np.int64)])
        ps = I.Pattern(ns, p.a, fs, name=p.name + "_sample")
        vs = I.make_values(ps, seed=2)
        Fs = flops_alg(ps.f)
        times = {}
        for thr in (1, nt):
            t3 = time.perf_counter()
            oracle.factor(ps.f, vs, nthreads=thr)
            times[thr] = time.perf_counter() - t3
        res["one_thread"] = {"value": Fs / times[1] / 1e12, "unit": "TFLOP/s", "cores": 1,
                             "sample": "factorization of the first %d band rows and the %d arrow rows "
                                       "(%.3g flops): %.2f s on 1 thread, %.2f s on %d threads"
                                       % (ns, p.a, Fs, times[1], times[nt], nt),
                             "all_threads_value": Fs / times[nt] / 1e12}
    return res, (L, X, ld)


def bench_single(args):
    import torch

    import paper_2501_02483_amd as S
    from paper_2501_02483_amd import inputs as I

    if args.workload == "small":
        p, seed, nrhs, rseed = I.single_small(), 1, 1, 101
    else:
        p, seed, nrhs, rseed = I.variable_band(), 2, 8, 102
    vals = I.make_values(p, seed=seed)
    B = I.rhs(p.N, nrhs, seed=rseed)
    tuned = None
    if args.tile == 0:
        # autotune tile size and ordering on this matrix (timed on the device)
        from paper_2501_02483_amd import autotune
        best, tried = autotune.tune_single(p, vals, reps=2)
        args.tile, args.ordering, args.parts = best["tile"], best["ordering"], best["nd_parts"]
        tuned = tried
    ordering = {"none": S.STILES_ORDER_NONE, "nd": S.STILES_ORDER_ADAPTABLE_ND}[args.ordering]
    sym = S.Symbolic.from_pattern(p, tile=args.tile, tree_min_ratio=args.tree_ratio, ordering=ordering,
                                  ublock=args.ublock,
                                  nd_parts=args.parts)
    fac = S.Factor(sym, S.STILES_FP64, nrhs_max=nrhs)
    dv = torch.from_numpy(vals).cuda()
    dB0 = to_device_cols(B)
    work = to_device_cols(B)
    ld = torch.empty(1, dtype=torch.float64, device="cuda")
    F = sym.info.flops_alg

    def step(ev=None):
        # factorization and solve as one launch of the merged task graph
        # (FP64): rows whose factor is final are solved while the rest is
        # still being factored
        work.copy_(dB0)
        if ev:
            ev[0].record()
        fac.factorize_solve(dv, work)
        if ev:
            ev[1].record()
        if ev:
            ev[2].record()
        fac.logdet(ld)
        if ev:
            ev[3].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert fac.info() == 0
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    info = fac.info()
    fact_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    logdet_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    ms = (t1 - t0) / args.steps * 1e3
    # the merged executor launch alone: HIP events recorded by the library
    # around that launch, on the same stream, over K further steps; and, for
    # reference, the factorization and solve launches of separate calls
    S.stiles_factor_set_timing(fac.handle, True)
    kms = []
    for _ in range(args.steps):
        step()
        kms.append(S.stiles_factor_kernel_ms(fac.handle, 0))
    sep_f, sep_s = [], []
    for _ in range(args.steps):
        fac.factorize(dv)
        work.copy_(dB0)
        fac.solve(work)
        sep_f.append(S.stiles_factor_kernel_ms(fac.handle, 0))
        sep_s.append(S.stiles_factor_kernel_ms(fac.handle, 1))
    S.stiles_factor_set_timing(fac.handle, False)
    kernel_ms = float(np.mean(kms))
    solve_kernel_ms = float(np.mean(sep_s))
    # algorithmic solve flops: two sweeps, a multiply and an add per entry of
    # the method's L (the envelope before ND) and right-hand side; executed:
    # the same over every stored tile entry
    F_solve = 4.0 * sym.info.nnz_L_alg * nrhs
    F_solve_exec = 4.0 * sym.info.tiles * args.tile * args.tile * nrhs
    achieved = (F + F_solve) / (kernel_ms * 1e-3) / 1e12
    res = {
        "metric": "arrowhead Cholesky TFLOP/s (factorize+solve+logdet step)",
        "value": F / (ms * 1e-3) / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": p.name, "n": p.n, "arrow": p.a, "N": p.N, "tile": args.tile, "nrhs": nrhs,
                   "ordering": {1: "none", 3: "adaptable_nd"}.get(sym.info.ordering_used, "other"),
                   "nd_parts": sym.info.nd_parts, "autotune": tuned,
                   "value_seed": seed, "rhs_seed": rseed, "ops": "factorize+solve+logdet",
                   "parallelism": "single GPU, persistent DAG executor"},
        "factorizations_per_s": 1e3 / ms,
        "factorize_solve_ms": fact_ms,
        "separate_launches_ms": {"factorization": float(np.mean(sep_f)), "solve": solve_kernel_ms},
        "logdet_ms": logdet_ms,
        "flops_alg": F,
        "flops_exec": sym.info.flops_exec,
        "solve_flops_alg": F_solve,
        "solve_flops_exec": F_solve_exec,
        "nnz_L_alg": sym.info.nnz_L_alg,
        "info": info,
        "roofline": {"bound": "mfma", "kernel": "exec_kernel<%d,3> (merged factorization + solve DAG)" % args.tile,
                     "achieved": achieved, "peak": FP64_PEAK, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK,
                     "traffic": None, "kernel_ms": kernel_ms, "flops_per_launch": F + F_solve,
                     "bytes_alg": 16 * p.nnz},
    }
    order_key = "nd%d" % sym.info.nd_parts if sym.info.nd_parts > 1 else "none"
    tr = measured_traffic("%s_n%d_a%d_%s" % (p.name.split("_")[0].rstrip("0123456789"), p.n, p.a, order_key),
                          args.tile)
    if tr is not None:
        res["roofline"]["traffic"] = tr["bytes"]
        res["roofline"]["traffic_detail"] = tr
    if not args.no_cpu_baseline:
        cb, _ = cpu_baseline_single(p, vals, B)
        res["cpu_baseline"] = cb
    del fac, dv, dB0, work
    if args.workload == "varband" and not args.no_large:
        # the largest single-GPU workload (n = 500,000, half-width 1,000,
        # arrow 200, Laplacian law): FP64 and mixed factorization kernels and
        # the refined 16-RHS solve, so that their times are observed in the
        # same run
        torch.cuda.empty_cache()
        res["large_n500k"] = mixed_runs(500_000, args.tile, S.STILES_ORDER_ADAPTABLE_ND, 0, steps=3)
    return res


def bench_selinv(args):
    """Selected inversion on the variable-bandwidth workload: the factor is
    computed once (untimed); a step is one selected inversion (Sigma = A^{-1}
    on the stored tiles of L) plus the diagonal of A^{-1} in the original
    ordering."""
    import torch

    import paper_2501_02483_amd as S
    from paper_2501_02483_amd import inputs as I

    p, seed = I.variable_band(), 2
    vals = I.make_values(p, seed=seed)
    ordering = {"none": S.STILES_ORDER_NONE, "nd": S.STILES_ORDER_ADAPTABLE_ND}[args.ordering]
    sym = S.Symbolic.from_pattern(p, tile=args.tile, tree_min_ratio=args.tree_ratio, ordering=ordering,
                                  ublock=args.ublock,
                                  nd_parts=args.parts)
    fac = S.Factor(sym, S.STILES_FP64)
    fac.factorize(torch.from_numpy(vals).cuda())
    assert fac.info() == 0
    ntasks, F, Fexec = S.stiles_selinv_query(sym.handle)
    si = S.SelInv(fac)
    diag = torch.empty(p.N, dtype=torch.float64, device="cuda")

    def step():
        si.compute()
        si.diag(diag)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) / args.steps * 1e3
    si.set_timing(True)
    kms = []
    for _ in range(args.steps):
        step()
        kms.append(si.kernel_ms())
    si.set_timing(False)
    kernel_ms = float(np.mean(kms))
    achieved = F / (kernel_ms * 1e-3) / 1e12
    res = {
        "metric": "selected inversion TFLOP/s (A^{-1} on the factor pattern + its diagonal)",
        "value": F / (ms * 1e-3) / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": p.name, "n": p.n, "arrow": p.a, "N": p.N, "tile": args.tile,
                   "ordering": {1: "none", 3: "adaptable_nd"}.get(sym.info.ordering_used, "other"),
                   "nd_parts": sym.info.nd_parts, "value_seed": seed, "ops": "selected inversion + diagonal",
                   "parallelism": "single GPU, persistent DAG executor"},
        "flops_alg": F,
        "flops_exec": Fexec,
        "tasks": ntasks,
        "roofline": {"bound": "mfma", "kernel": "exec_kernel<%d,2> (selected-inversion DAG)" % args.tile,
                     "achieved": achieved, "peak": FP64_PEAK, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK,
                     "traffic": None, "kernel_ms": kernel_ms, "bytes_alg": 16 * p.nnz},
    }
    order_key = "nd%d" % sym.info.nd_parts if sym.info.nd_parts > 1 else "none"
    tr = measured_traffic("selinv_varband_n%d_a%d_%s" % (p.n, p.a, order_key), args.tile)
    if tr is not None:
        res["roofline"]["traffic"] = tr["bytes"]
        res["roofline"]["traffic_detail"] = tr
    if not args.no_cpu_baseline:
        import oracle
        nt = cpu_threads()
        L, info = oracle.factor(p.f, vals, nthreads=nt)
        t2 = time.perf_counter()
        Sg = oracle.selinv(p.f, L, nthreads=nt)
        t3 = time.perf_counter()
        del Sg
        res["cpu_baseline"] = {"value": F / (t3 - t2) / 1e12, "unit": "TFLOP/s", "cores": nt, "kind": "oracle",
                               "sample": "the full workload, one selected inversion of the oracle's factor "
                                         "(%.2f s with %d threads; the factorization is not counted)" % (t3 - t2, nt)}
    return res


def bench_spde(args):
    """Spatio-temporal (SPDE-shaped) CSC input: 40 x 40 grid, 60 time steps,
    arrow 50 (n = 96,000); a step = scatter through the value map +
    factorization and 8-RHS solve (one merged launch) + logdet."""
    import torch

    import paper_2501_02483_amd as S
    from paper_2501_02483_amd import inputs as I

    nx, ny, nt, a = 40, 40, 60, 50
    g = I.spde_space_time(nx, ny, nt, a, seed=6)
    ordering = {"none": S.STILES_ORDER_AUTO, "nd": S.STILES_ORDER_ADAPTABLE_ND}[args.ordering]
    sym = S.Symbolic.from_csc(g["N"], g["a"], g["colptr"], g["rowind"], tile=args.tile, ordering=ordering,
                              ublock=args.ublock,
                              nd_parts=args.parts)
    fac = S.Factor(sym, S.STILES_FP64, nrhs_max=8)
    dv = torch.from_numpy(g["values"]).cuda()
    B = I.rhs(g["N"], 8, seed=106)
    dB0 = to_device_cols(B)
    work = to_device_cols(B)
    ld = torch.empty(1, dtype=torch.float64, device="cuda")
    F = sym.info.flops_alg

    def step():
        work.copy_(dB0)
        fac.factorize_solve(dv, work)
        fac.logdet(ld)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert fac.info() == 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) / args.steps * 1e3
    S.stiles_factor_set_timing(fac.handle, True)
    kms = []
    for _ in range(args.steps):
        step()
        kms.append(S.stiles_factor_kernel_ms(fac.handle, 0))
    S.stiles_factor_set_timing(fac.handle, False)
    kernel_ms = float(np.mean(kms))
    F_solve = 4.0 * sym.info.nnz_L * 8
    achieved = (F + F_solve) / (kernel_ms * 1e-3) / 1e12
    res = {
        "metric": "arrowhead Cholesky TFLOP/s (factorize+solve+logdet step, CSC input)",
        "value": F / (ms * 1e-3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": g["pattern"].name, "n": g["n"], "arrow": a, "N": g["N"], "nnz_lower": int(len(g["rowind"])),
                   "nnz_envelope": int(g["pattern"].nnz), "tile": args.tile,
                   "ordering": {1: "none", 2: "partial_rcm", 3: "adaptable_nd"}.get(sym.info.ordering_used, "other"),
                   "nd_parts": sym.info.nd_parts, "value_seed": 6, "rhs_seed": 106,
                   "ops": "factorize+solve+logdet", "parallelism": "single GPU, persistent DAG executor"},
        "flops_alg": F, "flops_exec": sym.info.flops_exec,
        "roofline": {"bound": "mfma", "kernel": "exec_kernel<%d,3> (merged factorization + solve DAG)" % args.tile,
                     "achieved": achieved, "peak": FP64_PEAK, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK,
                     "traffic": None, "kernel_ms": kernel_ms, "flops_per_launch": F + F_solve},
    }
    if not args.no_cpu_baseline:
        # bounded sample: the same generator with 10 time steps (n = 16,000)
        import oracle
        gs = I.spde_space_time(nx, ny, 10, a, seed=6)
        ps = gs["pattern"]
        nthr = cpu_threads()
        t2 = time.perf_counter()
        L, info = oracle.factor(ps.f, gs["profile_values"], nthreads=nthr)
        t3 = time.perf_counter()
        res["cpu_baseline"] = {"value": flops_alg(ps.f) / (t3 - t2) / 1e12, "unit": "TFLOP/s", "cores": nthr,
                               "kind": "oracle", "sample": "factorization of the same generator with 10 time steps "
                               "(n = 16,000; %.2f s with %d threads)" % (t3 - t2, nthr)}
    return res


def bench_batch(args):
    """512 uneven matrices in one persistent launch; tile size by the autotuner."""
    import torch

    import paper_2501_02483_amd as S
    from paper_2501_02483_amd import autotune
    from paper_2501_02483_amd import inputs as I
    from paper_2501_02483_amd.devgen import DevicePattern

    pats = I.batch_patterns()[:args.count]
    # values drawn on the device (seed 3000 + b), same law as the host generator
    dvals = [DevicePattern(p).values(p.meta["value_seed"]) for p in pats]
    torch.cuda.synchronize()
    best, tried = autotune.tune_batch(pats, dvals, reps=2) if args.tile == 0 \
        else ({"tile": args.tile, "nd_min_rows": args.nd_min_rows}, [])
    T = best["tile"]
    syms = autotune.batch_symbolics(pats, T, best["nd_min_rows"])
    facs = [S.Factor(s) for s in syms]
    batch = S.Batch(facs)
    lds = torch.empty(len(facs), dtype=torch.float64, device="cuda")

    def step():
        batch.factorize(dvals)
        batch.logdet(lds)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    infos = [f.info() for f in facs]
    F = sum(s.info.flops_alg for s in syms)
    ms = (t1 - t0) / args.steps * 1e3
    # the batched executor launch alone (library event pair on its stream)
    S.stiles_factor_set_timing(facs[0].handle, True)
    kms = []
    for _ in range(args.steps):
        step()
        kms.append(S.stiles_factor_kernel_ms(facs[0].handle, 0))
    S.stiles_factor_set_timing(facs[0].handle, False)
    kernel_ms = float(np.mean(kms))
    achieved = F / (kernel_ms * 1e-3) / 1e12
    return {"metric": "batched arrowhead Cholesky TFLOP/s (factorize+logdet of every matrix)",
            "value": F / (ms * 1e-3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic (device-generated values)",
            "config": {"workload": "batch%d_uneven" % len(pats), "matrices": len(pats), "tile": T,
                       "nd_min_rows": best["nd_min_rows"],
                       "nd_matrices": sum(1 for s in syms if s.info.nd_parts > 1),
                       "autotune": tried, "parallelism": "single GPU, one persistent launch"},
            "factorizations_per_s": len(pats) * 1e3 / ms, "flops_alg": F,
            "failed": int(sum(1 for i in infos if i != 0)),
            "logdet_finite": bool(torch.isfinite(lds).all().item()),
            "roofline": {"bound": "mfma", "kernel": "exec_kernel<%d,0> (batched factorization DAG)" % T,
                         "achieved": achieved, "peak": FP64_PEAK, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK,
                         "traffic": None, "kernel_ms": kernel_ms}}


def mixed_runs(n, tile, ordering, parts, steps, law="laplacian"):
    """n band rows, half-width 1,000, arrow 200; values by `law` (Laplacian:
    kappa ~ 1e6) drawn on the device: FP64 and mixed factorization kernel
    times (library event pair around the launch), the 16-RHS solve (refined
    in mixed mode), factorize + solve end to end, and the mixed results'
    differences from the FP64 ones."""
    import torch

    import paper_2501_02483_amd as S
    from paper_2501_02483_amd import inputs as I
    from paper_2501_02483_amd.devgen import DevicePattern

    p = I.mixed_large(n=n)
    nrhs = 16
    dp = DevicePattern(p)
    dv = dp.values(4, law=law, kappa=1e6)
    B = torch.randn(nrhs, p.N, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(104)).t()
    out = {}
    for prec, name in ((S.STILES_FP64, "fp64"), (S.STILES_MIXED32, "mixed"), (S.STILES_MIXED32_FULL, "mixed_corner_fp32")):
        sym = S.Symbolic.from_pattern(p, tile=tile or 64, ordering=ordering, nd_parts=parts, ublock=UBLOCK)
        fac = S.Factor(sym, prec, nrhs_max=nrhs)
        fac.factorize(dv)
        torch.cuda.synchronize()
        S.stiles_factor_set_timing(fac.handle, True)
        fms = []
        for _ in range(max(1, steps)):
            fac.factorize(dv)
            fms.append(S.stiles_factor_kernel_ms(fac.handle, 0))
        S.stiles_factor_set_timing(fac.handle, False)
        X = B.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = fac.solve(X)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ld = fac.logdet().item()
        # end to end: factorization (scatter included) + solve, host clock
        X2 = B.clone()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fac.factorize(dv)
        fac.solve(X2)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        # the same in one launch of the merged graph (mixed: its solve is the
        # first iterate of the refinement)
        X3 = B.clone()
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        fac.factorize_solve(dv, X3)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        fk = float(np.median(fms))
        out[name] = {"factor_kernel_ms": fk, "tflops": sym.info.flops_alg / fk / 1e9,
                     "solve_ms": (t1 - t0) * 1e3, "factorize_solve_ms": (t3 - t2) * 1e3,
                     "factorize_solve_merged_ms": (t5 - t4) * 1e3,
                     "iterations": rep.iterations, "converged": rep.converged,
                     "backward_error": rep.backward_error, "logdet": ld, "info": fac.info(), "X": X,
                     "L": fac.extract() if n <= 200_000 else None, "nd_parts": sym.info.nd_parts}
        del fac
    # both placements of the arrow-corner accumulation (FP64 in "mixed",
    # FP32 in "mixed_corner_fp32"): differences from the FP64 results
    xf, Lf = out["fp64"].pop("X"), out["fp64"].pop("L")
    for name in ("mixed", "mixed_corner_fp32"):
        xm, Lm = out[name].pop("X"), out[name].pop("L")
        out[name]["x_rel_diff_vs_fp64"] = float(torch.linalg.norm(xm - xf) / torch.linalg.norm(xf))
        out[name]["logdet_rel_diff_vs_fp64"] = abs(out[name]["logdet"] - out["fp64"]["logdet"]) / abs(out["fp64"]["logdet"])
        if Lf is not None:
            out[name]["L_rel_diff_vs_fp64"] = float(torch.linalg.norm(Lm - Lf) / torch.linalg.norm(Lf))
    out["flops_alg"] = sym.info.flops_alg
    out["workload"] = p.name
    out["law"] = law
    return out


def bench_mixed(args):
    """n=500,000, w=1,000, a=200, Laplacian law (kappa ~ 1e6): mixed-precision
    factorization and 16-RHS refined solve vs the FP64 path on the same GPU."""
    import paper_2501_02483_amd as S
    from paper_2501_02483_amd import inputs as I

    p = I.mixed_large(n=args.n or 500_000)
    nrhs = 16
    ordering = {"none": S.STILES_ORDER_NONE, "nd": S.STILES_ORDER_ADAPTABLE_ND}[args.ordering]
    out = mixed_runs(args.n or 500_000, args.tile, ordering, args.parts, args.steps, law=args.law)
    F = out["flops_alg"]
    v = out["mixed"]["tflops"]
    return {"metric": "mixed-precision arrowhead Cholesky TFLOP/s (factorization kernel)", "value": v,
            "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
            "ms_per_step": out["mixed"]["factor_kernel_ms"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32-updates/f64",
            "data": "synthetic (device-generated, %s law)" % args.law,
            "config": {"workload": p.name, "n": p.n, "arrow": p.a, "half_width": 1000, "nrhs": nrhs,
                       "tile": args.tile or 64, "ordering": args.ordering, "nd_parts": out["mixed"]["nd_parts"],
                       "law": args.law},
            "flops_alg": F, "runs": out,
            "roofline": {"bound": "mfma", "achieved": v, "peak": FP32_PEAK, "unit": "TFLOP/s",
                         "frac": v / FP32_PEAK, "traffic": None}}


HOST_THREADS = {"auto": None, "on": True, "off": False}


def bench_serve(args):
    """Poisson arrivals over 8 resident patterns (continuous batching), FP64
    and mixed-precision serving, each at 0.5 and 0.8 x its own saturation."""
    import torch

    import paper_2501_02483_amd as S
    from paper_2501_02483_amd import inputs as I
    from paper_2501_02483_amd.serve import GpuExecutor, Request, Server, summarize

    pats = I.serving_patterns()
    if args.max_n:
        pats = [p for p in pats if p.n <= args.max_n]
    budget = int(args.budget_gb * 2 ** 30)
    ordering = S.STILES_ORDER_ADAPTABLE_ND if args.ordering == "nd" else S.STILES_ORDER_NONE
    precisions = {"fp64": [S.STILES_FP64], "mixed": [S.STILES_MIXED32],
                  "both": [S.STILES_FP64, S.STILES_MIXED32]}[args.serve_precision]
    policies = {"sjf": ["sjf"], "fifo": ["fifo"], "both": ["fifo", "sjf"]}[args.serve_policy]

    def serve_one(prec):
        name = "fp64" if prec == S.STILES_FP64 else "mixed"
        # slots per precision (measured over 2000-request runs: FP64 peaks at
        # 2 concurrent requests, mixed precision at 4)
        slots = args.slots or (2 if prec == S.STILES_FP64 else 4)
        ex = GpuExecutor(pats, tile=args.tile or 64, precision=prec, slots=slots, ordering=ordering,
                         keep_results=False, host_threads=HOST_THREADS[args.host_threads])
        # warm-up: one request per pattern and slot, so every workspace the
        # runs below need is allocated and initialized before any clock starts
        warm = [Request(rid=i, arrival=0.0, pattern=i // slots, op=i % 3, seed=4000 + i, precision=prec)
                for i in range(len(pats) * slots)]
        Server(ex, budget, slots).run(warm)
        torch.cuda.synchronize()
        # closed loop: saturation rate with every slot busy
        nsat = max(args.requests // 2, 1)
        rng = np.random.default_rng(5)
        sat = [Request(rid=i, arrival=0.0, pattern=int(rng.integers(len(pats))), op=int(rng.integers(3)),
                       seed=5000 + i, precision=prec) for i in range(nsat)]
        done = Server(ex, budget, slots).run(sat)
        mu = len(done) / max(r.t_done for r in done)
        print("[serve %s] saturation %.1f req/s over %d requests" % (name, mu, nsat), file=sys.stderr, flush=True)
        res = {"saturation_rps": mu, "slots": slots, "syms_nd_parts": [s.info.nd_parts for s in ex.syms],
               "policies": {}}
        flops = lambda r: ex.flops(r.pattern)
        for policy in policies:
            out = res["policies"][policy] = {}
            for frac in (0.5, 0.8):
                reqs = [Request(rid=i, arrival=t, pattern=pi, op=op, seed=sd, precision=prec)
                        for i, (t, pi, op, sd) in enumerate(I.serving_requests(len(pats), args.requests, frac * mu))]
                srv = Server(ex, budget, slots, policy=policy)
                d = srv.run(reqs)
                bad = sum(1 for r in d if r.result.get("info", 0) != 0)
                out["load_%.1f" % frac] = dict(summarize(d, flops), failed=bad, max_used_gb=srv.max_used / 2 ** 30)
                print("[serve %s %s] load %.1f: %d requests, p50 %.1f ms, p99 %.1f ms, mean %.1f ms" % (
                    name, policy, frac, len(d), out["load_%.1f" % frac]["p50_ms"],
                    out["load_%.1f" % frac]["p99_ms"], out["load_%.1f" % frac]["mean_ms"]),
                    file=sys.stderr, flush=True)
        # the first policy's figures are the precision's headline
        res.update(res["policies"][policies[0]])
        ex.close()
        del ex
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return name, res

    res = dict(serve_one(p) for p in precisions)
    head = res["fp64"] if "fp64" in res else res["mixed"]
    main = head["load_0.8"]
    return {"metric": "serving p50/p99 request latency (ms) at 0.8 x saturation", "value": main["p99_ms"],
            "unit": "ms (p99)", "n_gpus": 1, "steps": args.requests, "warmup": 0, "ms_per_step": main["mean_ms"],
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if "fp64" in res else "f32+f64",
            "data": "synthetic (device-generated values per request)",
            "config": {"workload": "serve8", "patterns": [(p.n, int(p.n - p.f[p.n - 1]), p.a) for p in pats],
                       "slots": args.slots, "budget_gb": args.budget_gb, "requests": args.requests,
                       "precisions": list(res), "host_threads": args.host_threads, "policies": policies},
            "results": res}


def lapack_banded(p, vals):
    """Context row (not the oracle): LAPACK's band Cholesky (pbtrf through
    scipy.linalg.cholesky_banded, multithreaded BLAS) on the band block B of a
    constant-half-width arrowhead matrix [[B, C^T], [C, D]], then the arrow
    in NumPy: X = L_B^{-1} C^T by blocked forward substitution (row blocks of
    w: a triangular solve with the diagonal block and a product with the
    block to its left), S = D - X^T X, L_D = chol(S).  Returns the seconds of
    each part and log det A.  The inputs are converted to LAPACK's lower band
    storage before the clock starts."""
    from numpy.lib.stride_tricks import as_strided
    from scipy.linalg import blas, cholesky, cholesky_banded

    n, a = p.n, p.a
    f = p.f
    w = int(np.max(np.arange(n) - f[:n]))
    rp = p.row_ptr()
    # lower band storage, column-major: ab[d, j] = A[j + d, j]; entry (i, j)
    # of the band sits at flat index i + j w
    ab = np.zeros((w + 1, n), order="F")
    flat = ab.reshape(-1, order="F")
    step = 1 << 20
    for r0 in range(0, n, step):
        r1 = min(n, r0 + step)
        lens = rp[r0 + 1:r1 + 1] - rp[r0:r1]
        rows = np.repeat(np.arange(r0, r1, dtype=np.int64), lens)
        cols = np.arange(rp[r0], rp[r1], dtype=np.int64) - rp[rows] + f[rows]
        flat[rows + cols * w] = vals[rp[r0]:rp[r1]]
    C = np.zeros((a, n))
    D = np.zeros((a, a))
    for r in range(a):
        i = n + r
        row = vals[rp[i]:rp[i + 1]]          # columns 0 .. i (dense arrow)
        C[r] = row[:n]
        D[r, :r + 1] = row[n:]
    t0 = time.perf_counter()
    Lb = cholesky_banded(ab, lower=True, overwrite_ab=True, check_finite=False)
    t1 = time.perf_counter()
    Lf = np.asfortranarray(Lb).reshape(-1, order="F")

    def view(r0, r1, c0, c1):
        # L[r0:r1, c0:c1] read through the band storage as a column-major
        # matrix (leading dimension w); entries outside the band (j > i or
        # i - j > w) alias other storage, so only the triangle that lies in
        # the band is handed to BLAS
        return as_strided(Lf[r0 + c0 * w:], shape=(r1 - r0, c1 - c0), strides=(8, 8 * w))

    # row blocks of w rows: X_k = L_kk^{-1} (C_k^T - U_k X_(k-1)), with L_kk
    # the lower triangular diagonal block and U_k the upper triangular block
    # to its left (the previous w columns); S = D - sum_k X_k^T X_k
    b = max(w, 1)
    Sc = np.asfortranarray(D)      # lower triangle; S is formed there (syrk)
    Xprev = None
    for s0 in range(0, n, b):
        s1 = min(n, s0 + b)
        rhs = np.asfortranarray(C[:, s0:s1].T)
        if Xprev is not None:
            U = view(s0, s1, s0 - b, s0)
            if s1 - s0 < b:      # short last block: its rows of U, then a plain product
                rhs -= np.triu(U) @ Xprev
            else:
                rhs -= blas.dtrmm(1.0, U, Xprev, side=0, lower=0)
        Xk = blas.dtrsm(1.0, view(s0, s1, s0, s1), rhs, side=0, lower=1, overwrite_b=1)
        Sc = blas.dsyrk(-1.0, Xk, beta=1.0, c=Sc, trans=1, lower=1, overwrite_c=1)
        Xprev = Xk
    Ld = cholesky(Sc, lower=True, check_finite=False)
    t2 = time.perf_counter()
    logdet = 2.0 * (np.sum(np.log(Lb[0])) + np.sum(np.log(np.diag(Ld))))
    return {"band_pbtrf_s": t1 - t0, "arrow_s": t2 - t1, "total_s": t2 - t0, "logdet": float(logdet), "w": w}


def bench_banded(args):
    """Context row: LAPACK band Cholesky + NumPy arrow on the host cores, on
    the constant-half-width workloads (n = 2,000, w = 50, a = 10 and
    n = 500,000, w = 1,000, a = 200), beside the GPU's FP64 factorization +
    log-determinant of the same matrices (adaptable ND, T = 64)."""
    from paper_2501_02483_amd import inputs as I

    pats = [I.single_small(), I.mixed_large(n=args.n or 500_000)]
    rows = []
    for p in pats:
        vals = I.make_values(p, seed=4 if p.n > 100_000 else 1)
        F = flops_alg(p.f)
        reps = 3 if p.n <= 100_000 else 1
        ts = [lapack_banded(p, vals) for _ in range(reps)]
        best = min(ts, key=lambda r: r["total_s"])
        row = {"workload": p.name, "n": p.n, "arrow": p.a, "half_width": best["w"], "flops_alg": F,
               "lapack": best, "lapack_tflops": F / best["total_s"] / 1e12, "threads": cpu_threads(),
               "cpu_model": cpu_model()}
        gpu = gpu_fp64_factor(p, vals)
        if gpu is not None:
            row["gpu"] = gpu
            row["gpu_tflops"] = F / (gpu["step_ms"] * 1e-3) / 1e12
            row["gpu_over_lapack"] = best["total_s"] / (gpu["step_ms"] * 1e-3)
            row["logdet_rel_diff"] = abs(gpu["logdet"] - best["logdet"]) / abs(best["logdet"])
        rows.append(row)
        print(json.dumps({"context_row": row}), file=sys.stderr, flush=True)
    big = rows[-1]
    return {"metric": "LAPACK band Cholesky + arrow, TFLOP/s (host context)", "value": big["lapack_tflops"],
            "unit": "TFLOP/s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": big["lapack"]["total_s"] * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic (host-generated, dominant law)",
            "config": {"workload": "banded_context", "rows": [r["workload"] for r in rows]}, "rows": rows}


def gpu_fp64_factor(p, vals):
    """The library's FP64 scatter + factorization + log-determinant of the
    same matrix on the GPU (values resident; adaptable ND, T = 64), median
    of 5 after one warm-up, or None without a GPU."""
    try:
        import torch
        if not torch.cuda.is_available():
            return None
    except ImportError:
        return None
    import paper_2501_02483_amd as S
    sym = S.Symbolic.from_pattern(p, tile=64, ordering=S.STILES_ORDER_ADAPTABLE_ND)
    fac = S.Factor(sym)
    dv = torch.from_numpy(vals).cuda()
    ts, ld = [], None
    for it in range(6):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fac.factorize(dv)
        ld = fac.logdet()
        e1.record()
        torch.cuda.synchronize()
        if it:
            ts.append(e0.elapsed_time(e1))
    info = fac.info()
    del fac, sym, dv
    torch.cuda.empty_cache()
    return {"step_ms": float(np.median(ts)), "min_ms": float(np.min(ts)), "logdet": float(ld.item()), "info": int(info)}


def bench_ooc(args):
    """Out-of-core factorization of the variable-band matrix (host values in,
    host factor out): time per factorization and device footprint for a few
    segment lengths, against the in-core factorization's workspace."""
    import torch

    import paper_2501_02483_amd as S
    from paper_2501_02483_amd import inputs as I

    p, seed = I.variable_band(), 2
    vals = I.make_values(p, seed=seed)
    sym = S.Symbolic.from_pattern(p, tile=64, ordering=S.STILES_ORDER_NONE)
    in_core = sym.workspace_size(S.STILES_FP64, 1)
    F = sym.info.flops_alg
    runs = {}
    Lout = np.empty_like(vals)       # the host factor, reused across calls
    # the same work in core, also from host values to a host factor: upload,
    # factorization (natural order, as the segments), extraction, download
    fac = S.Factor(sym)
    ts = []
    for it in range(max(1, args.steps) + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fac.factorize(torch.from_numpy(vals).cuda())
        fac.extract().cpu()
        ts.append(time.perf_counter() - t0)
    in_core_host_ms = float(np.median(ts[1:])) * 1e3
    del fac
    torch.cuda.empty_cache()
    print("[ooc] in core, host values in and factor out: %.1f ms" % in_core_host_ms, file=sys.stderr, flush=True)
    for seg in (args.seg_rows or [10000, 20000, 50000]):
        S.stiles_factorize_ooc(p.n, p.a, p.f[:p.n], vals, seg, out=Lout)          # warm-up
        ts = []
        for _ in range(max(1, args.steps)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, ld, info, peak = S.stiles_factorize_ooc(p.n, p.a, p.f[:p.n], vals, seg, out=Lout)
            ts.append(time.perf_counter() - t0)
        runs[str(seg)] = {"ms": float(np.median(ts)) * 1e3, "peak_device_mb": peak / 2 ** 20, "info": info,
                          "logdet": ld, "segments": -(-p.n // seg)}
        print("[ooc] segments of %d rows: %.1f ms, %.1f MB" % (seg, runs[str(seg)]["ms"], peak / 2 ** 20),
              file=sys.stderr, flush=True)
    best = min(runs.values(), key=lambda r: r["ms"])
    return {"metric": "out-of-core arrowhead Cholesky TFLOP/s (host values -> host factor)",
            "value": F / (best["ms"] * 1e-3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
            "warmup": 1, "ms_per_step": best["ms"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "varband%d_a%d_ooc" % (p.n, p.a), "n": p.n, "arrow": p.a, "tile": 64,
                       "ordering": "natural"},
            "in_core_workspace_mb": in_core / 2 ** 20, "in_core_host_ms": in_core_host_ms, "runs": runs}


def bench_copycal(args):
    """Plain device copy of a known size (counter calibration for HBM traffic)."""
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gbs = 2 * nbytes * args.steps / (t1 - t0) / 1e9
    return {"metric": "device copy GB/s (calibration)", "value": gbs, "unit": "GB/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 0, "ms_per_step": (t1 - t0) / args.steps * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "copy_1GiB", "bytes_read": nbytes, "bytes_written": nbytes}}


def rocpd_summary(path):
    """Per-kernel table from a rocprofv3 rocpd database (kernel trace)."""
    import sqlite3
    db = sqlite3.connect(path)
    rows = db.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration), "
        "max(vgpr_count), max(accum_vgpr_count), max(sgpr_count), max(lds_size), max(grid_x), max(workgroup_x) "
        "from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1
    print("%-62s %6s %11s %11s %11s %11s %5s %5s %5s %6s %8s %4s %6s" % (
        "kernel", "calls", "total_ms", "avg_us", "min_us", "max_us", "vgpr", "agpr", "sgpr", "lds", "grid", "wg", "pct"))
    for r in rows:
        name = r[0] if len(r[0]) <= 62 else r[0][:59] + "..."
        print("%-62s %6d %11.3f %11.2f %11.2f %11.2f %5d %5d %5d %6d %8d %4d %6.2f" % (
            name, r[1], r[2] / 1e6, r[3] / 1e3, r[4] / 1e3, r[5] / 1e3, r[6] or 0, r[7] or 0, r[8] or 0,
            r[9] or 0, r[10] or 0, r[11] or 0, 100.0 * r[2] / total))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tile", type=int, default=-1,
                    help="tile size; 0 = autotune (tile and ordering, or tile and ND threshold for the batch); "
                         "default: 64, autotuned for the batch and small workloads")
    ap.add_argument("--tree-ratio", type=int, default=2)
    ap.add_argument("--ordering", default="nd", choices=["none", "nd"],
                    help="single-matrix workloads: natural order or adaptable nested dissection")
    ap.add_argument("--parts", type=int, default=0, help="adaptable ND partitions (0 = chosen by the analysis)")
    ap.add_argument("--workload", default="varband", choices=["varband", "small", "batch", "mixed", "serve", "copycal", "selinv", "spde", "ooc", "banded"])
    ap.add_argument("--rocpd-summary", default="", help="print a per-kernel table of a rocprofv3 database and exit")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ublock", type=int, default=0,
                    help="columns per 2 x 2 block update task (0: library default, -1: no blocks)")
    ap.add_argument("--count", type=int, default=512, help="batch: number of matrices")
    ap.add_argument("--nd-min-rows", type=int, default=0,
                    help="batch: adaptable ND for matrices with at least this many band tile rows (0 = none)")
    ap.add_argument("--n", type=int, default=0, help="mixed: band rows (default 500,000)")
    ap.add_argument("--law", default="laplacian", choices=["laplacian", "scaled"],
                    help="mixed: value law (Laplacian, kappa ~ 1e6; or S A0 S with s_i = 10^(-3 u_i))")
    ap.add_argument("--no-large", action="store_true",
                    help="varband: skip the n = 500,000 FP64/mixed runs reported beside the main line")
    ap.add_argument("--slots", type=int, default=0,
                    help="serve: concurrent request slots (0: 2 for FP64, 4 for mixed precision)")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serve: HBM budget for in-flight requests")
    ap.add_argument("--requests", type=int, default=2000, help="serve: timed requests per load point")
    ap.add_argument("--host-threads", default="auto", choices=list(HOST_THREADS),
                    help="serve: issue requests from one host thread per slot (auto: mixed precision only)")
    ap.add_argument("--serve-precision", default="both", choices=["fp64", "mixed", "both"],
                    help="serve: FP64 factors, mixed precision (FP32 updates, FP64 refinement), or both in turn")
    ap.add_argument("--serve-policy", default="both", choices=["sjf", "fifo", "both"],
                    help="serve: admission order, arrival order (fifo) or least expected work first (sjf); "
                         "both: fifo (the headline) then sjf")
    ap.add_argument("--max-n", type=int, default=0, help="serve: keep patterns with n <= max-n")
    ap.add_argument("--seg-rows", type=int, nargs="*", default=None,
                    help="ooc: band rows per segment (default: 10000 20000 50000)")
    args = ap.parse_args()
    global UBLOCK
    UBLOCK = args.ublock
    if args.tile < 0:
        args.tile = 0 if args.workload in ("batch", "small") else 64
    if args.rocpd_summary:
        rocpd_summary(args.rocpd_summary)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(independent factorizations shard across GPUs without exchange; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    if args.workload in ("varband", "small"):
        res = bench_single(args)
    elif args.workload == "batch":
        res = bench_batch(args)
    elif args.workload == "mixed":
        res = bench_mixed(args)
    elif args.workload == "copycal":
        res = bench_copycal(args)
    elif args.workload == "selinv":
        res = bench_selinv(args)
    elif args.workload == "spde":
        res = bench_spde(args)
    elif args.workload == "ooc":
        res = bench_ooc(args)
    elif args.workload == "banded":
        res = bench_banded(args)
    else:
        res = bench_serve(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
