"""GPU parity of the HIP solve path against the FP64 oracle at the
configurations' own shapes and column counts, through the C interface
(Python binding -> libmsp.so -> HIP kernels).

Both sides solve to a relative residual of 1e-13, so that the 1e-9 bar
measures the difference between two converged solutions rather than the
solver tolerance: iteration counts are equal without low-rank corrections
(within one with them, whose Ritz vectors differ by rounding), the solutions
agree to 1e-9 in the 2-norm and element by element (max |x - x_ref| <=
1e-9 max |x_ref| for every right-hand side)."""
import os
import sys

import numpy as np
import pytest

from gen import batch_problems, config_problem, make_problem
from oracle import amg, krylov

pytestmark = pytest.mark.gpu

TOL = 1e-13


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _agree(x, xr, bound=1e-9):
    """2-norm and element-wise agreement per right-hand side."""
    x = x.reshape(x.shape[0], -1)
    xr = xr.reshape(xr.shape[0], -1)
    rel = np.linalg.norm(x - xr) / np.linalg.norm(xr)
    elem = np.abs(x - xr).max(axis=0) / np.abs(xr).max(axis=0)
    _say("  rel 2-norm", rel, "element-wise", elem.max())
    assert rel <= bound, rel
    assert np.all(elem <= bound), elem


def _solve_gpu(p, **opts):
    torch = _torch()
    from paper_2407_05930_amd import Solver
    sv = Solver(p.A, p.img, **opts)
    x = sv.solve(torch.from_numpy(p.b).cuda()).cpu().numpy()
    return sv, x


def _check_ritz(sv, ctx, S):
    kept, ritz = sv.export_lrc()
    for a in range(S):
        ref = ctx["lrc"].ritz[a]
        assert np.abs(ritz[a] - ref).max() <= 1e-8 * max(1.0, np.abs(ref).max()), (a, ritz[a], ref)
        assert kept[a] == ctx["lrc"].U[a].shape[1]


@pytest.mark.parametrize("f3", [False, True], ids=["static_fsai", "afsai5_emin4"])
def test_headline_workload_fp64_matches_oracle(f3):
    """The headline workload at its full size (128^3, y stretched, s = 3,
    4 right-hand sides: 32 columns) with the per-subsystem cycle in FP64,
    without low-rank corrections (they change no iteration count there);
    also with the adaptive FSAI smoothers and energy-minimised interpolation
    that the headline measurement uses."""
    _torch()
    p = config_problem("channel3d_128_s3")
    opt = dict(afsai_nnz=5, emin_steps=4) if f3 else {}
    _say("oracle setup 128^3", opt)
    ctx = krylov.setup(p.A, p.img, amg.AMGOptions(**opt), precond="amgr_sub")
    ref = krylov.solve(ctx, p.b, tol=TOL)
    _say("oracle iterations", int(ref.iters.max()))
    sv, x = _solve_gpu(p, tol=TOL, pc="amgr_sub", **opt)
    _say("gpu iterations", sv.last.iters)
    assert sv.num_levels() == ref.hierarchy.nlev
    assert sv.last.iters == int(ref.iters.max())
    _agree(x, ref.x)
    sv.close()


@pytest.mark.parametrize("pc", ["amgr", "amgr_sub"])
def test_2d_workload_full_size_matches_oracle(pc):
    """The 2D workload at its full size: 128^2, s = 1, one right-hand side."""
    p = config_problem("poisson2d_128_s1")
    ctx = krylov.setup(p.A, p.img, amg.AMGOptions(), precond=pc)
    ref = krylov.solve(ctx, p.b, tol=TOL)
    sv, x = _solve_gpu(p, tol=TOL, pc=pc)
    _say(pc, "iterations gpu", sv.last.iters, "oracle", int(ref.iters.max()))
    assert sv.last.iters == int(ref.iters.max())
    _agree(x, ref.x)


@pytest.mark.parametrize("shape", [
    dict(N=(48, 48, 48), s=3, m=4, k=8, kw=dict(y_stretch=1.5), opt=dict(coarse_max=256)),
    dict(N=(24, 24, 24), s=3, m=8, k=8, kw=dict(y_stretch=1.5), opt=dict(coarse_max=64)),
    dict(N=(32, 32, 32), s=3, m=1, k=16, kw=dict(jitter=0.2, kappa="lognormal"), opt=dict(coarse_max=64)),
    dict(N=(32, 32, 32), s=3, m=2, k=16, kw=dict(jitter=0.2, kappa="lognormal"), opt=dict(coarse_max=64)),
], ids=["48c_s3_m4_k8_32cols", "24c_s3_m8_k8_64cols", "32c_jitter_s3_m1_k16", "32c_jitter_s3_m2_k16"])
def test_fp64_per_subsystem_lrc_matches_oracle(shape):
    """Per-subsystem cycle with low-rank corrections in FP64 at the column
    counts the workloads use (8, 16, 32 and 64 columns) and both correction
    ranks of the kernels (k = 8, and k = 16 of the jittered workload):
    Ritz values of the device Lanczos equal the oracle's to 1e-8, the
    iteration counts are within one and the solutions agree to 1e-9."""
    p = make_problem(shape["N"], s=shape["s"], m=shape["m"], seed=41, **shape["kw"])
    ctx = krylov.setup(p.A, p.img, amg.AMGOptions(**shape["opt"]), precond="amgr_sub", k=shape["k"])
    ref = krylov.solve(ctx, p.b, tol=TOL)
    sv, x = _solve_gpu(p, tol=TOL, pc="amgr_sub", k=shape["k"], **shape["opt"])
    _say(shape["N"], "k", shape["k"], "iterations gpu", sv.last.iters, "oracle", int(ref.iters.max()))
    _check_ritz(sv, ctx, 1 << shape["s"])
    assert abs(sv.last.iters - int(ref.iters.max())) <= 1
    _agree(x, ref.x)
    sv.close()


VARIANTS = [dict(MSP_SPMM_SPLIT="1", MSP_SPMM_WIDE="0", MSP_SPMM_SELL="0", MSP_OP_SELL="0", MSP_DENSE_ROWS="1"),
            dict(MSP_SPMM_SPLIT="1", MSP_SPMM_WIDE="1", MSP_SPMM_SELL="0", MSP_OP_SELL="1", MSP_DENSE_ROWS="2"),
            dict(MSP_SPMM_SPLIT="2", MSP_SPMM_WIDE="0", MSP_SPMM_SELL="0", MSP_OP_SELL="0", MSP_DENSE_ROWS="4"),
            dict(MSP_SPMM_SPLIT="4", MSP_SPMM_WIDE="0", MSP_SPMM_SELL="0", MSP_OP_SELL="1", MSP_DENSE_ROWS="8"),
            dict(MSP_SPMM_SPLIT="16", MSP_SPMM_WIDE="0", MSP_SPMM_SELL="0", MSP_OP_SELL="0", MSP_DENSE_ROWS="8"),
            dict(MSP_SPMM_SPLIT="64", MSP_SPMM_WIDE="0", MSP_SPMM_SELL="0", MSP_OP_SELL="1", MSP_DENSE_ROWS="8"),
            dict(MSP_SPMM_SELL="1", MSP_SPMM_WIDE="0", MSP_OP_SELL="1", MSP_DENSE_ROWS="8"),
            dict(MSP_SPMM_SELL="1", MSP_SPMM_WIDE="1", MSP_OP_SELL="1", MSP_DENSE_ROWS="8"),
            dict(MSP_SPMM_SELL="2", MSP_SPMM_WIDE="0", MSP_OP_SELL="0", MSP_DENSE_ROWS="8"),
            dict(MSP_SPMM_SELL="4", MSP_SPMM_WIDE="1", MSP_OP_SELL="1", MSP_DENSE_ROWS="8"),
            dict(MSP_SPMM_SELL="8", MSP_SPMM_WIDE="0", MSP_OP_SELL="1", MSP_DENSE_ROWS="8"),
            dict(MSP_SPMM_SELL="16", MSP_SPMM_WIDE="1", MSP_OP_SELL="1", MSP_DENSE_ROWS="8")]
SHAPES = [dict(N=(20, 20, 20), s=3, m=4, kw=dict(y_stretch=1.5), opt=dict(coarse_max=48)),    # 32 columns
          dict(N=(48, 40), s=1, m=3, kw=dict(), opt=dict(coarse_max=40)),                      # 6 of 8 columns
          dict(N=(16, 12, 20), s=2, m=1, kw=dict(jitter=0.2, kappa="lognormal"), opt=dict(coarse_max=40))]


_REFS = {}


def _vid(v):
    if v.get("MSP_SPMM_SELL", "0") != "0":
        return f"sliced{v['MSP_SPMM_SELL']}_wide{v['MSP_SPMM_WIDE']}_op{v['MSP_OP_SELL']}"
    return f"split{v['MSP_SPMM_SPLIT']}_wide{v['MSP_SPMM_WIDE']}_op{v['MSP_OP_SELL']}_rows{v['MSP_DENSE_ROWS']}"


@pytest.mark.parametrize("shape", range(len(SHAPES)), ids=["3d_32cols", "2d_8cols", "3d_jitter_4cols"])
@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_bf16"])
@pytest.mark.parametrize("var", VARIANTS, ids=[_vid(v) for v in VARIANTS])
def test_every_spmm_variant_matches_oracle(var, prec, shape, monkeypatch):
    """Each kernel variant the autotuner can pick for the V-cycle products
    (CSR with lane groups per row, 16-byte lanes, the sliced-ELL form with
    rows split G ways; rows per wavefront of the coarsest solves) and for the
    operator (CSR or sliced), forced for every matrix: FP64 solves match the
    oracle to 1e-9 with equal iteration counts, the mixed modes reach the
    tolerance and stay within 1e-7 of it."""
    for key, val in var.items():
        monkeypatch.setenv(key, val)
    sh = SHAPES[shape]
    if shape not in _REFS:   # one oracle solve per shape for every variant
        p = make_problem(sh["N"], s=sh["s"], m=sh["m"], seed=43, **sh["kw"])
        ctx = krylov.setup(p.A, p.img, amg.AMGOptions(**sh["opt"]), precond="amgr_sub")
        _REFS[shape] = (p, krylov.solve(ctx, p.b, tol=TOL))
    p, ref = _REFS[shape]
    if prec == "fp64":
        sv, x = _solve_gpu(p, tol=TOL, pc="amgr_sub", **sh["opt"])
        assert sv.last.iters == int(ref.iters.max())
        _agree(x, ref.x)
    else:
        sv, x = _solve_gpu(p, tol=1e-10, pc="amgr_sub", precision=prec, **sh["opt"])
        assert np.all(krylov.true_relres(p.A, x, p.b) <= 1.5e-10)
        _agree(x, ref.x, 1e-7)
    sv.close()


def test_tuning_file_reproduces_the_chosen_kernels(tmp_path, monkeypatch):
    """MSP_TUNE_SAVE records the autotuner's choices; a second context with
    MSP_TUNE_LOAD launches the same kernel functions without timing and gives
    the same bits."""
    torch = _torch()
    from paper_2407_05930_amd import Solver
    path = str(tmp_path / "tune.txt")
    p = make_problem((24, 24, 24), s=3, m=4, seed=44, y_stretch=1.5)
    b = torch.from_numpy(p.b).cuda()
    names = []
    xs = []
    for env in ("MSP_TUNE_SAVE", "MSP_TUNE_LOAD"):
        monkeypatch.delenv("MSP_TUNE_SAVE", raising=False)
        monkeypatch.delenv("MSP_TUNE_LOAD", raising=False)
        monkeypatch.setenv(env, path)
        sv = Solver(p.A, p.img, tol=1e-10, pc="amgr_sub", coarse_max=48, precision="mixed_bf16", k=8)
        sv.set_timing(True)
        xs.append(sv.solve(b))
        names.append(sv.timing_kernels())
        sv.close()
    assert open(path).read().count("=") >= 10
    assert names[0] == names[1]
    assert torch.equal(xs[0], xs[1])


def test_batched_systems_match_oracle_one_by_one():
    """Uneven systems (sizes, s, m) solved as one batch in FP64: every system
    equals its own oracle solve (iterations and solution); in the mixed mode
    (FP32 V-cycle) every system reaches the tolerance and is within 1e-7 of
    the oracle."""
    torch = _torch()
    from paper_2407_05930_amd import BatchSolver
    probs = [make_problem((N, N, N), s=s, m=m, seed=60 + i) for i, (N, s, m) in
             enumerate([(16, 1, 3), (24, 3, 2), (20, 2, 1), (12, 3, 8), (18, 1, 5), (22, 2, 7)])]
    refs = []
    for p in probs:
        ctx = krylov.setup(p.A, p.img, amg.AMGOptions(coarse_max=48), precond="amgr_sub")
        refs.append(krylov.solve(ctx, p.b, tol=TOL))
    bs_in = [torch.from_numpy(p.b).cuda() for p in probs]
    bs = BatchSolver([(p.A, p.img) for p in probs], tol=TOL, pc="amgr_sub", coarse_max=48)
    bs.set_chunk(4)   # the first solve's graph holds too few iterations: one-iteration launches finish it
    xs = bs.solve(bs_in)
    _say("first batched solve: graph launches", bs.last_launches)
    assert bs.last_launches > 1
    for i, (p, x, ref) in enumerate(zip(probs, xs, refs)):
        _say("batch fp64 system", i, "iterations", bs.stats[i].iters, "oracle", int(ref.iters.max()))
        assert bs.stats[i].iters == int(ref.iters.max())
        _agree(x.cpu().numpy(), ref.x)
    # the next solve's graph holds every iteration: one launch, the systems converging at their own
    # iteration counts inside it, and the same bits
    xs2 = bs.solve(bs_in)
    assert bs.last_launches == 1
    its = [bs.stats[i].iters for i in range(len(probs))]
    assert len(set(its)) > 1, its
    for x, x2 in zip(xs, xs2):
        assert torch.equal(x, x2)
    bs.close()
    bm = BatchSolver([(p.A, p.img) for p in probs], tol=1e-10, pc="amgr_sub", coarse_max=48, precision="mixed")
    xs = bm.solve(bs_in)
    for i, (p, x, ref) in enumerate(zip(probs, xs, refs)):
        xh = x.cpu().numpy()
        assert np.all(krylov.true_relres(p.A, xh, p.b) <= 1.5e-10), i
        _agree(xh, ref.x, 1e-7)
    bm.close()


@pytest.mark.parametrize("f3", [False, True], ids=["static_fsai", "afsai5_emin4"])
def test_batch_workload_fp32_vcycle_full_size(f3):
    """The batched workload itself: 64 uneven systems (N in even 32..96,
    s in 1..3, m in 1..8) with the FP32 V-cycle and FP64 PCG in one batch:
    every system reaches a true relative residual of 1e-10, and the four
    smallest are within 1e-7 of their FP64 oracle solutions (also with the
    adaptive FSAI and energy minimisation the bench uses)."""
    torch = _torch()
    from paper_2407_05930_amd import BatchSolver
    probs = batch_problems(64)
    opt = dict(afsai_nnz=5, emin_steps=4) if f3 else {}
    bs = BatchSolver([(p.A, p.img) for p in probs], tol=1e-10, pc="amgr_sub", precision="mixed", **opt)
    b_in = [torch.from_numpy(p.b).cuda() for p in probs]
    bs.solve(b_in)
    xs = bs.solve(b_in)
    _say("batch64 graph launches", bs.last_launches)
    assert bs.last_launches == 1
    xh = [x.cpu().numpy() for x in xs]
    worst = max(float(krylov.true_relres(p.A, x, p.b).max()) for p, x in zip(probs, xh))
    _say("batch64 worst true relres", worst)
    assert worst <= 1.5e-10
    for i in sorted(range(len(probs)), key=lambda j: probs[j].n)[:4]:
        ctx = krylov.setup(probs[i].A, probs[i].img, amg.AMGOptions(**opt), precond="amgr_sub")
        ref = krylov.solve(ctx, probs[i].b, tol=1e-12)
        _say("batch64 system", i, "N", probs[i].N, "s", probs[i].s)
        _agree(xh[i], ref.x, 1e-7)
    bs.close()
