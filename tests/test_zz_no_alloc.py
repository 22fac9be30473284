"""The allocation-free solve (msp_solve_device_noalloc) against the ordinary
device solve (msp_solve_device), called through the C interface: two calls
in a row on one context, the second with fewer right-hand sides (a smaller
workspace carved from the same static array), then a smaller system on
another context, in FP64 and with bfloat16 V-cycle multivectors.  The FP64
solutions agree to 1e-9 element by element (and in fact bit for bit: the
same kernels with the same tuned shapes), the mixed ones to the same bar
against the ordinary call."""
import ctypes
import sys

import numpy as np
import pytest

from gen import make_problem
from oracle import krylov

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _call(fn, sv, B, torch):
    """One solve of the n x m right-hand sides B (numpy) through fn, which is
    msp_solve_device or msp_solve_device_noalloc; returns (rc, x, stats)."""
    from paper_2407_05930_amd import _lib
    bt = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
    xt = torch.full_like(bt, float("nan"))
    st = _lib.msp_stats()
    stream = torch.cuda.current_stream()
    rc = fn(sv._ctx, B.shape[1], ctypes.c_void_p(bt.data_ptr()), ctypes.c_void_p(xt.data_ptr()),
            ctypes.c_void_p(stream.cuda_stream), ctypes.byref(st))
    torch.cuda.synchronize()
    return rc, xt.t().cpu().numpy(), st


def _agree(x, xr, bound):
    assert np.all(np.isfinite(x))
    assert np.all(np.abs(x - xr).max(axis=0) <= bound * np.abs(xr).max(axis=0))


@pytest.mark.parametrize("prec", ["fp64", "mixed_bf16"])
def test_noalloc_solve_matches_device_solve(prec):
    torch = _torch()
    from paper_2407_05930_amd import Solver, _lib
    lib = _lib.lib
    p = make_problem((20, 20, 20), s=3, m=4, seed=51, y_stretch=1.5)
    sv = Solver(p.A, p.img, tol=1e-12 if prec == "fp64" else 1e-10, pc="amgr_sub", coarse_max=48, k=8,
                precision=prec)
    for m in (4, 2):   # the second call is smaller: 16 instead of 32 columns
        B = p.b[:, :m]
        _say(prec, "m", m)
        rc0, x0, st0 = _call(lib.msp_solve_device, sv, B, torch)
        rc1, x1, st1 = _call(lib.msp_solve_device_noalloc, sv, B, torch)
        assert rc0 == 0 and rc1 == 0, (rc0, rc1, lib.msp_last_error())
        assert st1.iters == st0.iters
        _agree(x1, x0, 1e-9)
        if prec == "fp64":
            assert np.array_equal(x1, x0)
        assert np.all(krylov.true_relres(p.A, x1, B) <= (1e-11 if prec == "fp64" else 1.5e-10))
    # a smaller system on another context reuses the same array
    q = make_problem((12, 12, 12), s=2, m=3, seed=52)
    sq = Solver(q.A, q.img, tol=1e-12, pc="amgr_sub", coarse_max=32, precision=prec)
    rc0, x0, _ = _call(lib.msp_solve_device, sq, q.b, torch)
    rc1, x1, _ = _call(lib.msp_solve_device_noalloc, sq, q.b, torch)
    assert rc0 == 0 and rc1 == 0
    _agree(x1, x0, 1e-9)
    sq.close()
    sv.close()


def test_noalloc_solve_rejects_a_workspace_beyond_the_array():
    """64^3 with s = 3 and 8 right-hand sides needs more than the 128 MiB
    array: MSP_ERR_UNSUPPORTED with both sizes in the message, nothing
    launched, and the context still solves through the ordinary call."""
    torch = _torch()
    from paper_2407_05930_amd import Solver, _lib
    lib = _lib.lib
    p = make_problem((64, 64, 64), s=3, m=8, seed=53)
    sv = Solver(p.A, p.img, tol=1e-10, pc="amgr_sub")
    rc, _, _ = _call(lib.msp_solve_device_noalloc, sv, p.b, torch)
    msg = lib.msp_last_error().decode()
    _say("rc", rc, msg)
    assert rc == -8 and "bytes" in msg and str(128 << 20) in msg
    rc0, x0, _ = _call(lib.msp_solve_device, sv, p.b, torch)
    assert rc0 == 0
    assert np.all(krylov.true_relres(p.A, x0, p.b) <= 1.5e-10)
    sv.close()


def test_noalloc_solve_after_a_device_resetup():
    """After msp_refresh to a new coefficient the allocation-free solve
    equals the ordinary one bit for bit (FP64), and after a refused
    re-setup it refuses to solve as the ordinary call does."""
    torch = _torch()
    from paper_2407_05930_amd import MspError, Solver, _lib
    lib = _lib.lib
    kw = dict(y_stretch=1.5, kappa="lognormal")
    p0 = make_problem((20, 16, 16), s=3, m=2, seed=54, **kw)
    p1 = make_problem((20, 16, 16), s=3, m=2, seed=55, **kw)
    sv = Solver(p0.A, p0.img, tol=1e-12, pc="amgr_sub", coarse_max=48, k=4)
    sv.refresh(torch.from_numpy(p1.A.data).cuda())
    rc0, x0, st0 = _call(lib.msp_solve_device, sv, p1.b, torch)
    rc1, x1, st1 = _call(lib.msp_solve_device_noalloc, sv, p1.b, torch)
    assert rc0 == 0 and rc1 == 0, lib.msp_last_error()
    assert st1.iters == st0.iters and np.array_equal(x1, x0)
    assert np.all(krylov.true_relres(p1.A, x1, p1.b) <= 1e-11)
    with pytest.raises(MspError):
        sv.refresh(torch.from_numpy(-p1.A.data).cuda())
    rc, _, _ = _call(lib.msp_solve_device_noalloc, sv, p1.b, torch)
    assert rc == -1
    sv.close()
