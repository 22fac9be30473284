#!/usr/bin/env python3
"""Benchmark of the mirror-symmetric Poisson solve on one MI355X.

Workload (default): 128^3 cell-centred Poisson on the unit cube, y stretched
by tanh (gamma = 1.5), homogeneous Dirichlet walls, s = 3 mirror symmetries
(8 decoupled subsystems), 4 seeded uniform[-1, 1] right-hand sides solved
together (32 SpMM columns), low-rank corrections of rank k per subsystem,
tolerance 1e-10 relative residual per right-hand side.

A step is one complete solve (Q_s transforms, PCG to tolerance with the shared
V-cycle and corrections, back transform) with the right-hand sides already
resident in GPU memory.  The headline value is the solve time of the mixed
solver (FP32 V-cycle, FP64 outer PCG); the plain FP64 solve is timed beside
it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "solve time to 1e-10 rel-res, 128^3 s=3; mixed vs FP64 plain; V-cycle HBM GB/s"


PRECISION_NOTE = {"mixed": "mixed (FP32 V-cycle, FP64 PCG)",
                  "mixed_bf16": "mixed (V-cycle multivectors bfloat16 with FP32 arithmetic, FP32 matrices and "
                                "coarsest inverses, FP64 PCG)"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_solves(sv, b, steps, warmup, torch, markers=False):
    """Mean time of `steps` solves after `warmup` untimed ones; with markers, the
    window fills bracket the timed solves (for profiling.py window)."""
    for _ in range(warmup):
        sv.solve(b)
    torch.cuda.synchronize()
    if markers:
        window_marker(torch)
    t0 = time.perf_counter()
    for _ in range(steps):
        x = sv.solve(b)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if markers:
        window_marker(torch)
        torch.cuda.synchronize()
    return (t1 - t0) / steps, x


def kernel_breakdown(sv, b):
    """One fully instrumented solve: per timer class (kind) its launches, time,
    algorithmic bytes and kernel function; and the same grouped by kernel
    function (several classes can run one function, e.g. the level-0
    operator and smoother products)."""
    sv.reset_timing()
    sv.set_timing(True)
    sv.solve(b)
    sv.set_timing(False)
    tm = sv.timing()
    names = sv.timing_kernels()
    sv.reset_timing()
    funcs = {}
    for kind, (cnt, ms, by) in tm.items():
        f = funcs.setdefault(names[kind], dict(kinds=[], launches=0, ms=0.0, bytes=0.0))
        f["kinds"].append(kind)
        f["launches"] += cnt
        f["ms"] += ms
        f["bytes"] += by
    return tm, names, funcs


def committed_traffic(kernel):
    """Calibrated HBM bytes per launch of a kernel function from the committed
    rocprofv3 counter summary, if it was taken on the current library source."""
    import glob
    from paper_2407_05930_amd.profiling import source_hash
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_traffic.json")):
        try:
            info = json.load(open(path))
        except Exception:
            continue
        if info.get("kernel") == kernel and info.get("source_hash") == source_hash():
            return int(info["traffic_bytes_per_launch"])
    return None


def copy_ceiling(torch, nbytes=1 << 30, reps=10):
    """Achievable bandwidth of a plain device copy of nbytes (read + write
    counted), timed with events on the current stream."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return dict(bytes_moved=2 * nbytes, ms=round(ms, 4), GBs=round(2 * nbytes / (ms * 1e-3) / 1e9, 1))


def same_size_copy(torch, nbytes, reps=11, flush_bytes=512 << 20):
    """A plain device copy moving nbytes (nbytes / 2 read, nbytes / 2 written),
    the dominant kernel's algorithmic bytes per launch: median time per copy
    with the caches holding its operands (hot), and after a 512 MB write that
    evicts them from L2 and the memory-side cache (cold), as the solve's
    kernels find their operands after the PCG vectors have streamed through."""
    half = max(int(nbytes) // 2 // 8, 1)
    src = torch.ones(half, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    junk = torch.empty(flush_bytes // 4, dtype=torch.float32, device="cuda")
    out = {}
    for mode in ("hot", "cold"):
        ts = []
        dst.copy_(src)
        for _ in range(reps):
            if mode == "cold":
                junk.fill_(1.0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            dst.copy_(src)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = sorted(ts)[reps // 2]
        out[mode] = dict(ms=round(ms, 5), GBs=round(2 * half * 8 / (ms * 1e-3) / 1e9, 1))
    del src, dst, junk
    torch.cuda.empty_cache()
    out["bytes_moved"] = 2 * half * 8
    return out


def device_columns(torch, a):
    """An (n, m) host array as a CUDA tensor in the n x m column-major layout
    the library takes (so the binding passes it without a transposing copy)."""
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()


def window_marker(torch):
    """A tiny int16 fill launched just before and just after the timed steps of
    the headline solve, so that a kernel trace of this command can be cut to
    exactly those steps (profiling.py window).  The other workloads place them
    around their bfloat16-multivector solves (the adjoint: its timed forward and
    backward passes)."""
    torch.empty(1, dtype=torch.int16, device="cuda").fill_(7)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(problem, k, pc, extra):
    """The FP64 oracle on the host, on the same workload with the same
    preconditioner and correction rank: setup (hierarchy and Lanczos) timed
    on its own, then one complete solve to 1e-10, measured.  BLAS (dense
    products of the oracle) may use every core; SciPy's sparse products, the
    bulk of the work, run on one core."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import amg, krylov
    ncpu = os.cpu_count() or 1
    with threadpool_limits(limits=ncpu):
        blas = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
        t0 = time.perf_counter()
        ctx = krylov.setup(problem.A, problem.img, amg.AMGOptions(**extra), precond=pc, k=k)
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        ref = krylov.solve(ctx, problem.b, tol=1e-10)
        t_solve = time.perf_counter() - t0
    its = int(ref.iters.max())
    sample = (f"the whole headline workload: oracle setup ({pc}, k={k}: hierarchy and Lanczos) {t_setup:.1f} s, timed "
              f"apart; then one complete FP64 solve to 1e-10 ({its} iterations), measured, not extrapolated; "
              f"{ncpu} host cores, BLAS pool {blas} threads, SciPy sparse products on 1 core")
    return dict(value=round(t_solve, 3), unit="s", cores=int(blas), kind="oracle", sample=sample,
                setup_s=round(t_setup, 2), iters=its, s_per_iteration=round(t_solve / max(its, 1), 3),
                host_cpu_count=ncpu, host_cpu_model=cpu_model(), x=ref.x)


def bench_jitter(args, torch, np):
    """192^3 jittered octant, lognormal kappa, s = 3, k = 16: FP64 vs mixed
    (FP32 V-cycle) vs mixed with bfloat16 smoother values."""
    from gen import config_problem
    from paper_2407_05930_amd import Solver
    log("building workload jitter3d_192_s3")
    k = 16 if args.k is None else args.k
    p = config_problem("jitter3d_192_s3")
    b = device_columns(torch, p.b)
    out = {}
    for prec in ("fp64", "mixed", "mixed_bf16g", "mixed_bf16"):
        sv = Solver(p.A, p.img, tol=1e-10, precision=prec, k=k, pc=args.pc, **args.extra)
        t, x = timed_solves(sv, b, args.steps, args.warmup, torch, markers=prec == "mixed_bf16")
        xs = x.cpu().numpy()
        rr = float(np.max(np.linalg.norm(p.b - p.A @ xs, axis=0) / np.linalg.norm(p.b, axis=0)))
        out[prec] = dict(solve_s=round(t, 6), iters=sv.last.iters, true_relres=rr, setup_s=round(sv.stats.t_setup_s, 3))
        if prec == "fp64":
            x64 = xs
        else:
            out[prec]["rel_diff_vs_fp64"] = float(np.linalg.norm(xs - x64) / np.linalg.norm(x64))
        log(f"  {prec}: {t * 1e3:.2f} ms, {sv.last.iters} its, relres {rr:.2e}")
        sv.close()
    return {"metric": f"solve time to 1e-10 rel-res, 192^3 jittered s=3, k={k}", "value": out["mixed_bf16g"]["solve_s"],
            "unit": "s", "higher_is_better": False, "dtype": "f64+f32+bf16",
            "config": {"workload": "jitter3d_192_s3", "afsai_nnz": args.afsai, "emin_steps": args.emin, "grid": list(p.N), "s": 3, "rhs": 1, "lrc_k": k,
                       "unknowns": int(p.n), "preconditioner": args.pc}, "variants": out}


def dominant_roofline(sv, b, steps, torch):
    """Roofline of the dominant kernel function of a solve: the function with
    the largest share of one fully instrumented solve, then its launches alone
    bracketed by HIP events on the solve's stream over ``steps`` more solves."""
    tm_all, names, funcs = kernel_breakdown(sv, b)
    top = max(funcs, key=lambda f: funcs[f]["ms"])
    for kind in funcs[top]["kinds"]:
        sv.set_timing(True, kind)
    for _ in range(steps):
        sv.solve(b)
    torch.cuda.synchronize()
    live = sv.timing()
    sv.set_timing(False)
    sv.reset_timing()
    cnt = sum(live[kd][0] for kd in funcs[top]["kinds"] if kd in live)
    ms = sum(live[kd][1] for kd in funcs[top]["kinds"] if kd in live)
    by = sum(live[kd][2] for kd in funcs[top]["kinds"] if kd in live)
    avg_ms, per = ms / cnt, by / cnt
    achieved = per / (avg_ms * 1e-3) / 1e9
    same = same_size_copy(torch, per)
    from paper_2407_05930_amd import Solver
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": committed_traffic(top), "kernel": top,
            "classes": [Solver.kind_name(kk) for kk in funcs[top]["kinds"]], "avg_ms": round(avg_ms, 5),
            "algorithmic_bytes_per_launch": int(per), "launches": cnt, "same_size_copy": same,
            "frac_of_same_size_copy": {m: round(achieved / same[m]["GBs"], 4) for m in ("hot", "cold")},
            "kernel_functions": {f: dict(launches=v["launches"], ms=round(v["ms"], 3),
                                         classes=[Solver.kind_name(kk) for kk in v["kinds"]])
                                 for f, v in sorted(funcs.items(), key=lambda kv: -kv[1]["ms"])}}


def headline_resetup(args, torch, np, p, svm, k):
    """Numeric re-setup on the device (msp_refresh) of the headline solver for
    a lognormal coefficient on the same mesh, against a fresh host setup of
    that matrix: time, iterations and true residual of the solve after it."""
    from gen import make_problem
    from gen.problems import CONFIG_SEED0
    from paper_2407_05930_amd import Solver
    log("re-setup for a lognormal kappa on the same mesh")
    pk = make_problem(p.N, s=p.s, m=int(p.b.shape[1]), seed=CONFIG_SEED0 + 7, y_stretch=1.5, kappa="lognormal")
    assert np.array_equal(pk.A.indices, p.A.indices) and np.array_equal(pk.A.indptr, p.A.indptr)
    vals = torch.from_numpy(pk.A.data).cuda()
    bk = device_columns(torch, pk.b)
    t_rs = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        svm.refresh(vals)
        torch.cuda.synchronize()
        t_rs.append(time.perf_counter() - t0)
    drift = int(svm.stats.split_drift)
    drift1 = int(svm.stats.split_drift1)
    t_solve, x = timed_solves(svm, bk, args.steps, args.warmup, torch)
    xs = x.cpu().numpy()
    rr = float(np.max(np.linalg.norm(pk.b - pk.A @ xs, axis=0) / np.linalg.norm(pk.b, axis=0)))
    its = svm.last.iters
    fresh = Solver(pk.A, pk.img, tol=1e-10, precision=args.mixed, k=k, pc=args.pc, **args.extra)
    t_fresh, _ = timed_solves(fresh, bk, args.steps, args.warmup, torch)
    res = {"device_resetup_first_s": round(t_rs[0], 4), "device_resetup_s": round(min(t_rs[1:]), 4),
           "host_setup_s": round(fresh.stats.t_setup_s, 3),
           "solve_after_resetup_s": round(t_solve, 6), "iters_after_resetup": its, "true_relres_max": rr,
           "split_drift": drift, "base_cells": int(p.n_b),
           "split_drift_level1": drift1, "level1_points": int(svm.stats.rows[1]),
           "fresh_setup_solve_s": round(t_fresh, 6), "iters_fresh_setup": fresh.last.iters,
           "kappa": "lognormal(0, 1) per cell, same mesh",
           "note": "first re-setup includes building its device structure; lrc_k corrections rebuilt each time"}
    log(f"  re-setup {res['device_resetup_s'] * 1e3:.1f} ms (first {res['device_resetup_first_s'] * 1e3:.1f} ms), "
        f"host setup {res['host_setup_s']:.2f} s; solve {t_solve * 1e3:.2f} ms, {its} its "
        f"(fresh setup {t_fresh * 1e3:.2f} ms, {fresh.last.iters} its)")
    fresh.close()
    return res


def bench_copies(args, torch, np):
    """AMGR in the original basis on a domain made of copies (msp_setup_copies):
    8 translated copies of a 64^3 box side by side, lognormal kappa repeated in
    every copy, walls that differ between copies (the low axis-1 wall insulated
    in odd copies and the far end wall), 4 right-hand sides: 2.1 M unknowns, the
    headline's size, in a geometry Q_s cannot decouple.  FP64, FP32 and
    bfloat16 V-cycle vectors; no low-rank correction."""
    from gen import make_repeated_problem
    from gen.problems import CONFIG_SEED0
    from paper_2407_05930_amd import Solver
    log("building workload copies3d_8x64")
    p = make_repeated_problem((64, 64, 64), 8, m=4, seed=CONFIG_SEED0 + 5, walls="mixed")
    b = device_columns(torch, p.b)
    out = {}
    x64 = None
    svh = None
    for prec in ("fp64", "mixed", "mixed_bf16"):
        sv = Solver.from_copies(p.A, p.sub, tol=1e-10, precision=prec, **args.extra)
        t, x = timed_solves(sv, b, args.steps, args.warmup, torch, markers=prec == "mixed_bf16")
        xs = x.cpu().numpy()
        rr = float(np.max(np.linalg.norm(p.b - p.A @ xs, axis=0) / np.linalg.norm(p.b, axis=0)))
        out[prec] = dict(solve_s=round(t, 6), iters=sv.last.iters, true_relres=rr,
                         setup_s=round(sv.stats.t_setup_s, 3))
        if prec == "fp64":
            x64 = xs
        else:
            out[prec]["rel_diff_vs_fp64"] = float(np.linalg.norm(xs - x64) / np.linalg.norm(x64))
        log(f"  copies {prec}: {t * 1e3:.2f} ms, {sv.last.iters} its, relres {rr:.2e}")
        if prec == "mixed_bf16":
            svh = sv
        else:
            sv.close()
    st = svh.stats
    iface = svh.export_outer()[1]
    roof = dominant_roofline(svh, b, args.steps, torch)
    svh.close()
    return {"metric": "solve time to 1e-10 rel-res, 8 translated copies of 64^3 with differing walls, 4 RHS",
            "value": out["mixed_bf16"]["solve_s"], "unit": "s", "higher_is_better": False,
            "dtype": "f64+f32+bf16",
            "config": {"workload": "copies3d_8x64", "afsai_nnz": args.afsai, "emin_steps": args.emin, "copy_grid": [64, 64, 64], "copies": 8, "rhs": 4,
                       "unknowns": int(p.n), "preconditioner": "amgr (original basis, populated interface)",
                       "interface_fraction": round(float(iface.mean()), 4),
                       "levels": int(st.nlev), "op_complexity": round(st.op_complexity, 3)},
            "variants": out, "roofline": roof}


def bench_amgs(args, torch, np):
    """AMGS, the Schur-complement AMG of Sec. 3.1, on the headline problem
    (128^3, s = 3, 4 RHS) with k low-rank corrections of the decoupled Schur
    blocks, FP64: the symmetric form under PCG and the light form under
    flexible CG, beside AMGR (per-subsystem cycle, FP64) on the same systems."""
    from gen import config_problem
    from paper_2407_05930_amd import Solver
    log("building workload amgs3d_128_s3")
    p = config_problem("channel3d_128_s3")
    b = device_columns(torch, p.b)
    out = {}
    svh = None
    for label, opts in (("amgs", dict(pc="amgs", amgs_light=0)), ("amgs_light", dict(pc="amgs", amgs_light=1)),
                        ("amgr_sub", dict(pc="amgr_sub"))):
        sv = Solver(p.A, p.img, tol=1e-10, precision="fp64", k=8 if args.k is None else args.k, **opts)
        t, x = timed_solves(sv, b, args.steps, args.warmup, torch)
        xs = x.cpu().numpy()
        rr = float(np.max(np.linalg.norm(p.b - p.A @ xs, axis=0) / np.linalg.norm(p.b, axis=0)))
        out[label] = dict(solve_s=round(t, 6), iters=sv.last.iters, true_relres=rr,
                          setup_s=round(sv.stats.t_setup_s, 3))
        log(f"  {label}: {t * 1e3:.2f} ms, {sv.last.iters} its, relres {rr:.2e}")
        if label == "amgs":
            svh = sv
        else:
            sv.close()
    roof = dominant_roofline(svh, b, args.steps, torch)
    svh.close()
    return {"metric": "solve time to 1e-10 rel-res, 128^3 s=3, 4 RHS, AMGS (Schur-complement AMG), FP64",
            "value": out["amgs"]["solve_s"], "unit": "s", "higher_is_better": False, "dtype": "f64",
            "config": {"workload": "amgs3d_128_s3", "grid": list(p.N), "s": p.s, "rhs": int(p.b.shape[1]),
                       "schur_lrc_k": 8 if args.k is None else args.k, "unknowns": int(p.n)},
            "variants": out, "roofline": roof}


def bench_batch(args, torch, np):
    """64 uneven cubic Dirichlet systems (N in even 32..96, s in 1..3, m in
    1..8) solved as one batch: one launch of a captured graph whose
    iterations are gated per system on the device.  The headline is the FP32
    V-cycle with FP64 PCG; bfloat16 V-cycle vectors and the same systems
    solved one after another are timed beside it."""
    from gen import batch_problems
    from paper_2407_05930_amd import BatchSolver, Solver
    log("building 64 systems")
    probs = batch_problems(64)
    bs = [device_columns(torch, pr.b) for pr in probs]
    unk = sum(pr.n * pr.b.shape[1] for pr in probs)

    def run_batch(prec):
        t0 = time.perf_counter()
        bsol = BatchSolver([(pr.A, pr.img) for pr in probs], tol=1e-10, precision=prec, pc=args.pc, **args.extra)
        t_setup = time.perf_counter() - t0
        for _ in range(max(args.warmup, 1)):
            bsol.solve(bs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            xs = bsol.solve(bs)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        worst = 0.0
        for pr, x in zip(probs, xs):
            xh = x.cpu().numpy()
            worst = max(worst, float(np.max(np.linalg.norm(pr.b - pr.A @ xh, axis=0) / np.linalg.norm(pr.b, axis=0))))
        its = [bsol.stats[i].iters for i in range(len(probs))]
        out = dict(solve_s=round(t, 6), iters_min_max=[min(its), max(its)], true_relres_max=worst,
                   graph_launches_per_solve=bsol.last_launches, setup_s=round(t_setup, 2),
                   unknown_rhs_per_s=round(unk / t, 1))
        log(f"  batch {prec}: {t * 1e3:.2f} ms, iterations {min(its)}..{max(its)}, {bsol.last_launches} launch(es)")
        bsol.close()
        return out

    head = run_batch("mixed")
    alt = run_batch("mixed_bf16")
    # the same systems one after another, one context each (no batching)
    sols = [Solver(pr.A, pr.img, tol=1e-10, precision="mixed", pc=args.pc, **args.extra) for pr in probs]
    for sv, b in zip(sols, bs):
        sv.solve(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for sv, b in zip(sols, bs):
            sv.solve(b)
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / args.steps
    for sv in sols:
        sv.close()
    return {"metric": "batched solve time to 1e-10 rel-res, 64 uneven systems", "value": head["solve_s"], "unit": "s",
            "higher_is_better": False, "dtype": "f64+f32",
            "config": {"workload": "batch64", "afsai_nnz": args.afsai, "emin_steps": args.emin, "systems": len(probs), "unknowns": int(sum(pr.n for pr in probs)),
                       "rhs_total": int(sum(pr.b.shape[1] for pr in probs)), "preconditioner": args.pc,
                       "precision": PRECISION_NOTE["mixed"]},
            **{k: v for k, v in head.items() if k != "solve_s"},
            "bf16_vcycle_vectors": {"precision": PRECISION_NOTE["mixed_bf16"], **alt},
            "sequential_single_solves_s": round(t_seq, 6),
            "batch_speedup_vs_sequential": round(t_seq / head["solve_s"], 3)}


def bench_adjoint(args, torch, np):
    """256^3, s = 3, lognormal kappa: forward solve and adjoint (dL/df,
    dL/dkappa) through torch.autograd, FP64."""
    from gen import config_problem
    from gen.problems import CONFIG_SEED0
    from paper_2407_05930_amd.adjoint import DifferentiablePoisson
    log("building workload adjoint3d_256_s3 (geometry only)")
    pr = config_problem("adjoint3d_256_s3", assemble=False)
    t0 = time.perf_counter()
    dp = DifferentiablePoisson(pr.faces, pr.img, tol=1e-10, pc=args.pc, **args.extra)
    f = torch.from_numpy(pr.b).cuda()
    pst = torch.from_numpy(pr.p_target[:, None]).cuda()
    kap = torch.from_numpy(pr.kappa_base).cuda().requires_grad_(True)
    dp.solver_for(kap)
    t_setup = time.perf_counter() - t0
    times = []
    for it in range(args.warmup + args.steps):
        kap.grad = None
        fr = f.clone().requires_grad_(True)
        torch.cuda.synchronize()
        if it == args.warmup:
            window_marker(torch)
        t0 = time.perf_counter()
        p = dp(fr, kap)
        loss = 0.5 * ((p - pst) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        if it >= args.warmup:
            times.append(time.perf_counter() - t0)
    window_marker(torch)
    torch.cuda.synchronize()
    t = sum(times) / len(times)
    its_host = dp.solver.last.iters
    g64 = kap.grad.clone()
    # the same passes with the bfloat16-multivector V-cycle under the FP64 PCG
    log("forward + adjoint with the bfloat16-multivector V-cycle")
    dpm = DifferentiablePoisson(pr.faces, pr.img, tol=1e-10, pc=args.pc, precision="mixed_bf16", **args.extra)
    dpm.solver_for(kap)
    tm = []
    for it in range(args.warmup + args.steps):
        kap.grad = None
        fm = f.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pm = dpm(fm, kap)
        (0.5 * ((pm - pst) ** 2).sum()).backward()
        torch.cuda.synchronize()
        if it >= args.warmup:
            tm.append(time.perf_counter() - t0)
    mixed = {"value_s": round(sum(tm) / len(tm), 6), "iters": dpm.solver.last.iters,
             "grad_kappa_rel_diff_vs_fp64": float((kap.grad - g64).norm().item() / g64.norm().item())}
    log(f"  mixed_bf16: {mixed['value_s'] * 1e3:.1f} ms, {mixed['iters']} its")
    dpm.solver.close()
    dpm.op.close()
    del dpm, pm
    kap.grad = g64
    loss_host = float(loss.item())
    gk_host = float(kap.grad.norm().item())
    # Per-kappa rebuild for an optimisation step: the host path (assembly and
    # setup of a fresh solver) against the device re-setup on the first
    # setup's structure (device assembly, then msp_refresh).  Kappa steps are
    # lognormal perturbations exp(0.1 z) of the base field.
    log("per-kappa rebuild: host assembly + setup")
    rng = np.random.default_rng(CONFIG_SEED0 + 6)
    steps_k = [torch.from_numpy(pr.kappa_base * np.exp(0.1 * rng.standard_normal(pr.n_b))).cuda()
               for _ in range(3)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    host_dp = DifferentiablePoisson(pr.faces, pr.img, tol=1e-10, pc=args.pc, **args.extra)
    host_dp.solver_for(steps_k[0])
    torch.cuda.synchronize()
    t_host_rebuild = time.perf_counter() - t0
    kap0 = steps_k[0].clone().requires_grad_(True)
    p0 = host_dp(f, kap0)
    (0.5 * ((p0 - pst) ** 2).sum()).backward()
    its_fresh = host_dp.solver.last.iters
    g_fresh = kap0.grad.clone()
    host_dp.solver.close()
    host_dp.op.close()
    del host_dp, p0
    log("per-kappa rebuild: device assembly + re-setup")
    dp.resetup = "device"
    t_dev = []
    drift = []
    drift1 = []
    for kk in steps_k:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dp.solver_for(kk)
        torch.cuda.synchronize()
        t_dev.append(time.perf_counter() - t0)
        drift.append(int(dp.solver.stats.split_drift))
        drift1.append(int(dp.solver.stats.split_drift1))
        log(f"  re-setup {t_dev[-1]:.3f} s, split drift {drift[-1]} of {pr.n_b} base cells, "
            f"level 1: {drift1[-1]} of {dp.solver.stats.rows[1]}")
    # back to the first step's kappa: its gradient against the fresh setup's
    dp.solver_for(steps_k[0])
    kap1 = steps_k[0].clone().requires_grad_(True)
    p1 = dp(f, kap1)
    (0.5 * ((p1 - pst) ** 2).sum()).backward()
    its_dev = dp.solver.last.iters
    g_rel = float((kap1.grad - g_fresh).norm().item() / g_fresh.norm().item())
    # the levels below the reduction level rebuilt on the host for this kappa (msp_rebuild_below)
    log("rebuild below the reduction level")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dp.solver.rebuild_below()
    torch.cuda.synchronize()
    t_rb_host = time.perf_counter() - t0
    kap_h = steps_k[0].clone().requires_grad_(True)
    (0.5 * ((dp(f, kap_h) - pst) ** 2).sum()).backward()
    its_rb_host = dp.solver.last.iters
    # the same with the per-subsystem values and corrections from a device re-setup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dp.solver.rebuild_below(dp._vals)
    torch.cuda.synchronize()
    t_rb = time.perf_counter() - t0
    kap2 = steps_k[0].clone().requires_grad_(True)
    p2 = dp(f, kap2)
    (0.5 * ((p2 - pst) ** 2).sum()).backward()
    its_rb = dp.solver.last.iters
    g_rel_rb = float((kap2.grad - g_fresh).norm().item() / g_fresh.norm().item())
    log(f"  rebuild {t_rb:.2f} s with device values ({t_rb_host:.2f} s on the host, {its_rb_host} iterations), "
        f"{its_rb} iterations (re-setup {its_dev}, fresh setup {its_fresh})")
    resetup = {"host_assembly_and_setup_s": round(t_host_rebuild, 3),
               "device_first_s": round(t_dev[0], 3),
               "device_s": round(sum(t_dev[1:]) / len(t_dev[1:]), 4),
               "iters_fresh_setup": its_fresh, "iters_device_resetup": its_dev,
               "split_drift_per_step": drift, "base_cells": int(pr.n_b),
               "split_drift_level1_per_step": drift1, "level1_points": int(dp.solver.stats.rows[1]),
               "grad_kappa_rel_diff_vs_fresh_setup": g_rel,
               "rebuild_below_s": round(t_rb, 3), "iters_after_rebuild_below": its_rb,
               "rebuild_below_host_values_s": round(t_rb_host, 3), "iters_after_host_rebuild": its_rb_host,
               "grad_kappa_rel_diff_after_rebuild_vs_fresh_setup": g_rel_rb,
               "kappa_step": "kappa_base * exp(0.1 z), z ~ N(0, 1) per base cell",
               "note": "device_first_s includes building the position map and the re-setup's device structure"}
    return {"metric": "forward + adjoint solve time, 256^3 s=3 lognormal kappa", "value": round(t, 6), "unit": "s",
            "higher_is_better": False, "dtype": "f64",
            "config": {"workload": "adjoint3d_256_s3", "afsai_nnz": args.afsai, "emin_steps": args.emin, "grid": list(pr.N), "s": 3, "unknowns": int(pr.n),
                       "preconditioner": args.pc},
            "iters": its_host, "setup_s": round(t_setup, 2), "loss": loss_host,
            "grad_kappa_norm": gk_host, "grad_f_norm": float(fr.grad.norm().item()), "resetup": resetup,
            "mixed_bf16_vcycle": mixed}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="channel3d_128_s3")
    ap.add_argument("--k", type=int, default=None,
                    help="low-rank correction rank per subsystem (default: 16 for jitter3d_192_s3, else 8)")
    ap.add_argument("--pc", default="amgr_sub", choices=["amgr", "amgr_sub"],
                    help="AMGR per subsystem below the shared reduction level (default), or the AMGR "
                         "hierarchy of A_inn shared by every subsystem")
    ap.add_argument("--mixed", default="mixed_bf16", choices=["mixed", "mixed_bf16"],
                    help="mixed-precision variant of the headline: V-cycle multivectors in bfloat16 (default) or "
                         "FP32; the other one is timed beside it")
    ap.add_argument("--afsai", type=int, default=5,
                    help="adaptive FSAI smoothers with at most this many entries per row, as in the paper's "
                         "experiments (0: static FSAI on the strong lower pattern)")
    ap.add_argument("--emin", type=int, default=4,
                    help="energy-minimisation steps on every interpolation (0: none)")
    ap.add_argument("--trunc0", type=float, default=None,
                    help="reduction-level interpolation truncation (library default when omitted)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip timing the other preconditioner beside the headline one")
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the headline mixed solve (for profiler runs): no other precision, no "
                         "comparison, no copy ceiling, no CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain 1 GiB device copy (reference for the traffic counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}): this solver has no "
              "multi-GPU path (the base cells would be split over GPUs with halo exchanges, one process each)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from gen import config_problem
    from paper_2407_05930_amd import Solver

    rank = int(os.environ.get("RANK", "0"))
    extra = {"afsai_nnz": args.afsai, "emin_steps": args.emin}
    if args.trunc0 is not None:
        extra["trunc0"] = args.trunc0
    args.extra = extra
    other = {"jitter3d_192_s3": bench_jitter, "batch64": bench_batch, "adjoint3d_256_s3": bench_adjoint,
             "copies3d_8x64": bench_copies, "amgs3d_128_s3": bench_amgs}
    if args.workload in other:
        res = other[args.workload](args, torch, np)
        res.update({"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "data": "synthetic", "vs_baseline": None})
        print(json.dumps(res), flush=True)
        return
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {src.numel() * 8} bytes read, {dst.numel() * 8} bytes written")
        del src, dst
    log(f"building workload {args.workload}")
    p = config_problem(args.workload)
    b = device_columns(torch, p.b)
    k = 8 if args.k is None else args.k
    head = args.mixed   # the mixed-precision variant reported as the headline
    alt = "mixed" if head == "mixed_bf16" else "mixed_bf16"

    def run(pc, prec, label=None, markers=False, **opts):
        label = label or prec
        log(f"setup {pc} {label} k={k}")
        sv = Solver(p.A, p.img, tol=1e-10, precision=prec, k=k, pc=pc, **args.extra, **opts)
        log(f"timing {pc} {label}: warmup {args.warmup}, steps {args.steps}")
        for _ in range(args.warmup):
            sv.solve(b)
        torch.cuda.synchronize()
        if markers:
            window_marker(torch)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            x = sv.solve(b)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        if markers:
            window_marker(torch)
            torch.cuda.synchronize()
        xs = x.cpu().numpy()
        true_rr = np.linalg.norm(p.b - p.A @ xs, axis=0) / np.linalg.norm(p.b, axis=0)
        log(f"  {pc} {label}: {t * 1e3:.3f} ms/solve, {sv.last.iters} iterations, true rel res {true_rr.max():.2e}")
        return dict(sv=sv, t=t, iters=sv.last.iters, true_relres=true_rr.tolist(), t_setup=sv.stats.t_setup_s, x=xs)

    res = {}
    res["mixed"] = run(args.pc, head, markers=True)
    if args.headline_only:
        print(json.dumps({"metric": METRIC, "value": round(res["mixed"]["t"], 6), "unit": "s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "iters": res["mixed"]["iters"],
                          "note": "headline solve only (profiler run)"}), flush=True)
        return
    res["fp64"] = run(args.pc, "fp64")
    res["alt"] = run(args.pc, alt)
    res["alt"]["sv"].close()
    ns = run(args.pc, "mixed", label="mixed_fp64_coarsest", coarse64=1) if args.pc == "amgr_sub" else None
    if ns is not None:
        ns["sv"].close()
    other_pc = "amgr" if args.pc == "amgr_sub" else "amgr_sub"
    other = None
    if not args.no_compare:
        other = {prec: run(other_pc, prec) for prec in ("fp64", "mixed")}
        for v in other.values():
            v["sv"].close()

    # Roofline of the dominant kernel function of the headline solve: the
    # function with the largest share of one fully instrumented solve; then
    # its launches alone are bracketed by HIP events on the solve's stream
    # during a second run of the timed steps.
    svm = res["mixed"]["sv"]
    tm_all, names, funcs = kernel_breakdown(svm, b)
    top = max(funcs, key=lambda f: funcs[f]["ms"])
    for kind in funcs[top]["kinds"]:
        svm.set_timing(True, kind)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        svm.solve(b)
    torch.cuda.synchronize()
    t_head = (time.perf_counter() - t0) / args.steps
    svm.set_timing(False)
    live = svm.timing()
    svm.reset_timing()
    cnt = sum(live[kd][0] for kd in funcs[top]["kinds"] if kd in live)
    ms = sum(live[kd][1] for kd in funcs[top]["kinds"] if kd in live)
    by = sum(live[kd][2] for kd in funcs[top]["kinds"] if kd in live)
    avg_ms = ms / cnt
    bytes_per_launch = by / cnt
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    ceiling = copy_ceiling(torch)
    log(f"copy ceiling: {ceiling['GBs']} GB/s")
    same = same_size_copy(torch, bytes_per_launch)
    log(f"copy of the dominant kernel's bytes per launch: hot {same['hot']['GBs']} GB/s, "
        f"cold {same['cold']['GBs']} GB/s")
    breakdown = {Solver.kind_name(kk): dict(launches=v[0], ms=round(v[1], 3), kernel=names[kk],
                                            GBs=round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None)
                 for kk, v in sorted(tm_all.items(), key=lambda kv: -kv[1][1])}
    by_function = {f: dict(launches=v["launches"], ms=round(v["ms"], 3),
                           classes=[Solver.kind_name(kk) for kk in v["kinds"]],
                           GBs=round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None)
                   for f, v in sorted(funcs.items(), key=lambda kv: -kv[1]["ms"])}
    # V-cycle aggregate GB/s: all level kernels and the dense coarsest solve
    vc_ms = sum(v[1] for kk, v in tm_all.items() if kk >= 16 or kk == 6)
    vc_by = sum(v[2] for kk, v in tm_all.items() if kk >= 16 or kk == 6)
    vc_gbs = vc_by / (vc_ms * 1e-3) / 1e9 if vc_ms > 0 else None

    t_mixed = res["mixed"]["t"]
    t_fp64 = res["fp64"]["t"]
    x64 = res["fp64"]["x"]

    def rel(x, y):
        return float(np.linalg.norm(x - y) / np.linalg.norm(y))

    out = {
        "metric": METRIC,
        "value": round(t_mixed, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_mixed * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32+bf16" if head == "mixed_bf16" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": list(p.N), "s": p.s, "rhs": int(p.b.shape[1]),
                   "subsystem_columns": int((1 << p.s) * p.b.shape[1]), "lrc_k": k, "tol": 1e-10,
                   "preconditioner": args.pc, "afsai_nnz": args.afsai, "emin_steps": args.emin,
                   "precision": PRECISION_NOTE[head], "unknowns": int(p.n)},
        "other_mixed_variant": {"precision": PRECISION_NOTE[alt], "solve_s": round(res["alt"]["t"], 6),
                                "iters": res["alt"]["iters"], "true_relres_max": max(res["alt"]["true_relres"]),
                                "rel_diff_vs_fp64": rel(res["alt"]["x"], x64)},
        "fp64_solve_s": round(t_fp64, 6),
        "mixed_speedup_vs_fp64": round(t_fp64 / t_mixed, 3),
        "iters": {"fp64": res["fp64"]["iters"], "mixed": res["mixed"]["iters"]},
        "true_relres_max": {kk: max(res[kk]["true_relres"]) for kk in ("fp64", "mixed")},
        "mixed_vs_fp64_rel_diff": rel(res["mixed"]["x"], x64),
        "setup_s": {kk: round(res[kk]["t_setup"], 3) for kk in ("fp64", "mixed")},
        "vcycle_GBs": round(vc_gbs, 1) if vc_gbs else None,
        "vcycle_frac": round(vc_gbs / HBM_PEAK_GBS, 4) if vc_gbs else None,
        "vcycle_frac_of_copy_ceiling": round(vc_gbs / ceiling["GBs"], 4) if vc_gbs else None,
        "copy_ceiling": ceiling,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": committed_traffic(top),
                     "kernel": top, "classes": [Solver.kind_name(kk) for kk in funcs[top]["kinds"]],
                     "avg_ms": round(avg_ms, 5), "algorithmic_bytes_per_launch": int(bytes_per_launch),
                     "launches": cnt, "frac_of_copy_ceiling": round(achieved / ceiling["GBs"], 4),
                     "same_size_copy": same,
                     "frac_of_same_size_copy": {m: round(achieved / same[m]["GBs"], 4) for m in ("hot", "cold")}},
        "kernel_functions_mixed": by_function,
        "kernel_breakdown_mixed": breakdown,
        "timed_solve_with_kernel_events_s": round(t_head, 6),
    }
    if ns is not None:
        out["mixed_fp32_vcycle_fp64_coarsest"] = {
            "precision": "mixed (FP32 V-cycle: FP32 matrices, vectors and accumulation; FP64 coarsest solve; FP64 PCG)",
            "solve_s": round(ns["t"], 6), "iters": ns["iters"], "true_relres_max": max(ns["true_relres"]),
            "rel_diff_vs_fp64": rel(ns["x"], x64), "speedup_vs_fp64": round(t_fp64 / ns["t"], 3)}
    if other is not None:
        out[{"amgr": "shared_cycle", "amgr_sub": "per_subsystem_cycle"}[other_pc]] = {
            "preconditioner": other_pc,
            "mixed_solve_s": round(other["mixed"]["t"], 6), "fp64_solve_s": round(other["fp64"]["t"], 6),
            "iters": {kk: v["iters"] for kk, v in other.items()},
            "true_relres_max": {kk: max(v["true_relres"]) for kk, v in other.items()},
            "mixed_vs_headline_rel_diff": rel(other["mixed"]["x"], res["mixed"]["x"]),
        }
    if not args.no_compare:
        out["resetup"] = headline_resetup(args, torch, np, p, svm, k)
    if not args.no_cpu_baseline and rank == 0:
        log("cpu baseline (oracle, same workload, preconditioner and k)")
        cb = cpu_baseline(p, k, args.pc, args.extra)
        xo = cb.pop("x")
        cb["gpu_fp64_vs_oracle_rel_diff"] = rel(x64, xo)
        cb["gpu_mixed_vs_oracle_rel_diff"] = rel(res["mixed"]["x"], xo)
        out["cpu_baseline"] = cb
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
