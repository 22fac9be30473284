"""GPU parity of solves preconditioned with the adaptive FSAI smoothers and
energy-minimising interpolation (options afsai_nnz, emin_steps) against the
FP64 oracle, through the C interface."""
import sys

import numpy as np
import pytest

from gen import make_problem
from oracle import amg, krylov, refresh

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
    x = x.reshape(x.shape[0], -1)
    xr = xr.reshape(xr.shape[0], -1)
    assert np.linalg.norm(x - xr) <= bound * np.linalg.norm(xr)
    assert np.all(np.abs(x - xr).max(axis=0) <= bound * np.abs(xr).max(axis=0))


CASES = [
    dict(name="amgr_sub_s3_m4", pc="amgr_sub", k=0, N=(24, 20, 16), s=3, m=4, kw=dict(y_stretch=1.5), af=5, em=4),
    dict(name="amgr_s3_m2", pc="amgr", k=0, N=(24, 20, 16), s=3, m=2, kw=dict(y_stretch=1.5), af=5, em=4),
    dict(name="amgr_sub_s2_jitter", pc="amgr_sub", k=0, N=(28, 24, 20), s=2, m=1,
         kw=dict(jitter=0.2, kappa="lognormal"), af=5, em=4),
    dict(name="amgr_sub_s3_lrc4", pc="amgr_sub", k=4, N=(16, 16, 16), s=3, m=2, kw=dict(y_stretch=1.5), af=5,
         em=4),
    dict(name="amgr_afsai_only", pc="amgr_sub", k=0, N=(24, 20, 16), s=3, m=1, kw=dict(kappa="lognormal"), af=5,
         em=0),
    dict(name="amgr_emin_only", pc="amgr_sub", k=0, N=(24, 20, 16), s=3, m=1, kw=dict(kappa="lognormal"), af=0,
         em=6),
]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_adaptive_fp64_solve_matches_oracle(case):
    """Both sides solve to 1e-13: equal iteration counts (within one with
    low-rank corrections), x element-wise within 1e-9 x max|x|."""
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("adaptive case", case["name"])
    p = make_problem(case["N"], s=case["s"], m=case["m"], seed=27, **case["kw"])
    opt = dict(coarse_max=48, afsai_nnz=case["af"], emin_steps=case["em"])
    ctx = krylov.setup(p.A, p.img, amg.AMGOptions(**opt), precond=case["pc"], k=case["k"])
    ref = krylov.solve(ctx, p.b, tol=TOL)
    sv = Solver(p.A, p.img, tol=TOL, pc=case["pc"], k=case["k"], **opt)
    if case["k"]:
        kept, ritz = sv.export_lrc()
        for a in range(1 << p.s):
            r_or = np.asarray(ctx["lrc"].ritz[a])
            assert np.abs(ritz[a][:r_or.size] - r_or).max() <= 1e-8 * max(1.0, np.abs(r_or).max())
    x = sv.solve(torch.from_numpy(p.b).cuda()).cpu().numpy()
    _say("its gpu", sv.last.iters, "oracle", ref.iters.max())
    assert abs(sv.last.iters - int(ref.iters.max())) <= (1 if case["k"] else 0)
    _agree(x, ref.x)
    assert np.all(krylov.true_relres(p.A, x, p.b) <= 1e-11)


@pytest.mark.parametrize("prec", ["mixed", "mixed_bf16"])
def test_adaptive_mixed_precision_reaches_tolerance(prec):
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("adaptive mixed", prec)
    p = make_problem((32, 32, 32), s=3, m=2, seed=28, y_stretch=1.5, kappa="lognormal")
    opt = dict(coarse_max=64, afsai_nnz=5, emin_steps=4)
    ctx = krylov.setup(p.A, p.img, amg.AMGOptions(**opt), precond="amgr_sub")
    ref = krylov.solve(ctx, p.b, tol=1e-12)
    sv = Solver(p.A, p.img, tol=1e-10, precision=prec, pc="amgr_sub", k=8, **opt)
    x = sv.solve(torch.from_numpy(p.b).cuda()).cpu().numpy()
    rr = krylov.true_relres(p.A, x, p.b)
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    _say("its", sv.last.iters, "oracle (k = 0)", ref.iters.max(), "relres", rr, "err", err)
    assert np.all(rr <= 1.5e-10)
    assert err <= 1e-7


def test_refresh_with_adaptive_fsai_and_emin_matches_the_oracle():
    """The device re-setup keeps the adaptive FSAI patterns (static FSAI on
    them for the new values) and repeats the energy minimisation on the kept
    interpolation patterns, as the oracle's re-setup does."""
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("adaptive refresh")
    kw = dict(y_stretch=1.5, kappa="lognormal")
    p0 = make_problem((24, 20, 16), s=3, m=2, seed=29, **kw)
    p1 = make_problem((24, 20, 16), s=3, m=2, seed=30, **kw)
    opt = dict(coarse_max=48, afsai_nnz=5, emin_steps=4)
    ctx1 = refresh.refresh(krylov.setup(p0.A, p0.img, amg.AMGOptions(**opt), precond="amgr_sub"), p1.A)
    ref = krylov.solve(ctx1, p1.b, tol=TOL)
    sv = Solver(p0.A, p0.img, tol=TOL, pc="amgr_sub", **opt)
    sv.refresh(torch.from_numpy(p1.A.data).cuda())
    x = sv.solve(torch.from_numpy(p1.b).cuda()).cpu().numpy()
    _say("its gpu", sv.last.iters, "oracle", ref.iters.max())
    assert sv.last.iters == int(ref.iters.max())
    _agree(x, ref.x)
    H = ctx1["hier"]
    e0 = sv.export_level(0)
    for key in ("P", "G"):
        M = getattr(H.levels[0], key)
        assert np.array_equal(e0[key].indices, M.indices) and np.array_equal(e0[key].indptr, M.indptr)
        assert np.abs(e0[key].data - M.data).max() <= 1e-12 * 10 * np.abs(M.data).max()
    for a, SH in enumerate(ctx1["sub"].subs):
        for lev in range(1, H.nlev - 1):
            e = sv.export_sub_level(lev, a)
            L = SH.levels[lev - 1]
            assert np.abs(e["P"].data - L.P.data).max() <= 1e-10 * np.abs(L.P.data).max()
            assert np.abs(e["G"].data - L.G.data).max() <= 1e-10 * np.abs(L.G.data).max()
