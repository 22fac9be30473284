"""GPU parity of AMGR in the original basis for domains made of copies
(msp_setup_copies) against the oracle's (oracle/copies.py), through the C
interface: translated and reflected copies whose boundary conditions differ
between copies, several right-hand sides, FP64 element-wise to rounding and
the mixed precisions to the solver tolerance."""
import sys

import numpy as np
import pytest

from gen import make_repeated_problem
from oracle import amg, copies, krylov

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
    dict(name="repeated4_mixed_m3", N=(8, 7, 6), copies=4, mirror=False, walls="mixed", m=3, opt=dict(coarse_max=40)),
    dict(name="mirrored2_mixed_m1", N=(10, 9, 7), copies=2, mirror=True, walls="mixed", m=1, opt=dict(coarse_max=40)),
    dict(name="2d_repeated5_m2", N=(24, 20), copies=5, mirror=False, walls="dirichlet", m=2, opt=dict(coarse_max=40)),
    dict(name="32cube_x4_mixed_m4", N=(32, 32, 32), copies=4, mirror=False, walls="mixed", m=4, opt=dict()),
    dict(name="48cube_x4_mirrored_m2", N=(48, 48, 48), copies=4, mirror=True, walls="mixed", m=2, opt=dict()),
    dict(name="repeated4_mixed_m3_afsai_emin", N=(8, 7, 6), copies=4, mirror=False, walls="mixed", m=3,
         opt=dict(coarse_max=40, afsai_nnz=5, emin_steps=4)),
    dict(name="32cube_x4_mixed_m4_afsai_emin", N=(32, 32, 32), copies=4, mirror=False, walls="mixed", m=4,
         opt=dict(afsai_nnz=5, emin_steps=4)),
]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_copies_fp64_matches_oracle(case):
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("case", case["name"])
    p = make_repeated_problem(case["N"], case["copies"], m=case["m"], seed=31, mirror=case["mirror"],
                              walls=case["walls"])
    ctx = copies.setup(p.A, p.sub, amg.AMGOptions(**case["opt"]))
    ref = copies.solve(ctx, p.b, tol=TOL)
    sv = Solver.from_copies(p.A, p.sub, tol=TOL, **case["opt"])
    assert sv.num_levels() == ctx["hier"].nlev
    x = sv.solve(torch.from_numpy(p.b).cuda()).cpu().numpy()
    _say("iters", sv.last.iters, "oracle", ref.iters.tolist())
    assert sv.last.iters == int(ref.iters.max())
    _agree(x, ref.x)
    assert np.all(krylov.true_relres(p.A, x, p.b) <= 1e-11)


@pytest.mark.parametrize("prec", ["mixed", "mixed_bf16g", "mixed_bf16"])
def test_copies_mixed_precision_reaches_tolerance(prec):
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("copies", prec)
    p = make_repeated_problem((32, 32, 32), 4, m=4, seed=32, walls="mixed")
    ctx = copies.setup(p.A, p.sub, amg.AMGOptions())
    ref = copies.solve(ctx, p.b, tol=1e-12)
    sv = Solver.from_copies(p.A, p.sub, tol=1e-10, precision=prec)
    x = sv.solve(torch.from_numpy(p.b).cuda()).cpu().numpy()
    rr = krylov.true_relres(p.A, x, p.b)
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    _say(prec, "iters", sv.last.iters, "oracle", int(ref.iters.max()), "relres", rr.max(), "err", err)
    assert np.all(rr <= 1.5e-10)
    assert err <= 1e-7
    assert sv.last.iters <= int(1.25 * ref.iters.max()) + 2


def test_copies_with_lrc_matches_oracle_iterate_count():
    """LRCAMG(k) on a domain of copies: the low-rank correction is computed on
    the GPU from the V-cycle; it reaches the tolerance in no more iterations
    than the plain cycle."""
    torch = _torch()
    from paper_2407_05930_amd import Solver
    p = make_repeated_problem((16, 16, 16), 4, m=2, seed=33, walls="mixed")
    ctx = copies.setup(p.A, p.sub, amg.AMGOptions(coarse_max=64))
    ref = copies.solve(ctx, p.b, tol=TOL)
    plain = Solver.from_copies(p.A, p.sub, tol=TOL, coarse_max=64)
    lrc = Solver.from_copies(p.A, p.sub, tol=TOL, coarse_max=64, k=8)
    b = torch.from_numpy(p.b).cuda()
    x0 = plain.solve(b).cpu().numpy()
    x1 = lrc.solve(b).cpu().numpy()
    _say("plain", plain.last.iters, "lrc", lrc.last.iters, "oracle", int(ref.iters.max()))
    _agree(x0, ref.x)
    _agree(x1, ref.x)
    assert lrc.last.iters <= plain.last.iters
