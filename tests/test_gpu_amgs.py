"""GPU parity of AMGS (pc="amgs", the Schur-complement AMG of Sec. 3.1,
eq. (3.12)) against the oracle (oracle/amgs.py), through the C interface:
the symmetric form under PCG with and without the low-rank corrected Schur
approximation, the light form under flexible CG, and the Ritz values of the
Schur corrections."""
import sys

import numpy as np
import pytest

from gen import make_problem
from oracle import amg, amgs, krylov

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
    dict(name="16x14x12_s2_m3_k0", N=(16, 14, 12), s=2, m=3, k=0, light=False, kw=dict(y_stretch=1.5),
         opt=dict(coarse_max=40)),
    dict(name="16x14x12_s2_m3_k8", N=(16, 14, 12), s=2, m=3, k=8, light=False, kw=dict(y_stretch=1.5),
         opt=dict(coarse_max=40)),
    dict(name="12cube_s3_m1_k4_jitter", N=(12, 12, 12), s=3, m=1, k=4, light=False,
         kw=dict(jitter=0.2, kappa="lognormal"), opt=dict(coarse_max=40)),
    dict(name="16x14x12_s2_m2_k8_light", N=(16, 14, 12), s=2, m=2, k=8, light=True, kw=dict(y_stretch=1.5),
         opt=dict(coarse_max=40)),
    dict(name="64cube_s3_m1_k8", N=(64, 64, 64), s=3, m=1, k=8, light=False, kw=dict(y_stretch=1.5), opt=dict()),
]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_amgs_matches_oracle(case):
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("case", case["name"])
    p = make_problem(case["N"], s=case["s"], m=case["m"], seed=41, **case["kw"])
    opt = amgs.AMGSOptions(amg=amg.AMGOptions(**case["opt"]), k=case["k"], light=case["light"])
    ctx = amgs.setup(p.A, p.img, opt)
    ref = amgs.solve(ctx, p.b, tol=TOL)
    sv = Solver(p.A, p.img, tol=TOL, pc="amgs", k=case["k"], amgs_light=int(case["light"]), **case["opt"])
    x = sv.solve(torch.from_numpy(p.b).cuda()).cpu().numpy()
    _say("iters", sv.last.iters, "oracle", int(ref.iters.max()))
    if case["k"] == 0:
        assert sv.last.iters == int(ref.iters.max())
    else:
        assert abs(sv.last.iters - int(ref.iters.max())) <= 1
        kept, ritz = sv.export_lrc()
        for a in range(1 << p.s):
            r_or = np.asarray(ctx["low"].ritz[a])
            assert np.abs(ritz[a][:r_or.size] - r_or).max() <= 1e-8 * max(1.0, np.abs(r_or).max())
            assert kept[a] == ctx["low"].U[a].shape[1]
    _agree(x, ref.x)
    assert np.all(krylov.true_relres(p.A, x, p.b) <= 1e-11)
