"""Pins of the oracle's rebuild below the reduction level
(oracle/refresh.py: rebuild_below): it must reproduce a fresh setup whenever
the kept reduction level is what a fresh setup would build.

Two such cases: the setup itself (rebuilding from unchanged values), and a
matrix changed on the diagonal only.  A diagonal shift leaves the strength of
connection (off-diagonal entries against the row's largest off-diagonal
one), hence Alg. 2's split and the strength-based smoother pattern, as they
are; without truncation the interpolation pattern is symbolic, so the
re-set-up reduction level is the fresh one.  Its Galerkin operator A_1 does
change, and with it level 1's split: the kept-structure re-setup then differs
from the fresh setup below the reduction level, and the rebuild must close
exactly that gap."""
import numpy as np
import pytest

from gen import make_problem
from oracle import amg, krylov, refresh


def _same_level(L1, L2):
    for key in ("A", "P", "R", "G"):
        M1, M2 = getattr(L1, key), getattr(L2, key)
        if M1 is None or M2 is None:
            assert M1 is None and M2 is None, key
            continue
        assert np.array_equal(M1.indptr, M2.indptr) and np.array_equal(M1.indices, M2.indices), key
        assert np.array_equal(M1.data, M2.data), key
    if L1.C is None or L2.C is None:
        assert L1.C is None and L2.C is None
    else:
        assert np.array_equal(L1.C, L2.C)
        assert L1.omega == L2.omega


def _same_ctx(c1, c2):
    H1, H2 = c1["hier"], c2["hier"]
    assert H1.nlev == H2.nlev
    for L1, L2 in zip(H1.levels, H2.levels):
        _same_level(L1, L2)
    if c1["sub"] is not None:
        for S1, S2 in zip(c1["sub"].subs, c2["sub"].subs):
            assert len(S1.levels) == len(S2.levels)
            for L1, L2 in zip(S1.levels, S2.levels):
                _same_level(L1, L2)


def _diagonal_shift(p, seed, scale):
    """p.A plus delta_i on every image of base cell i (the mirror structure
    is kept), delta >= 0 so the matrix stays positive definite."""
    rng = np.random.default_rng(seed)
    A = p.A.tocsr(copy=True)
    delta = scale * rng.uniform(0.0, 1.0, p.img.shape[0]) * np.abs(A.diagonal()).max()
    d = np.zeros(A.shape[0])
    for a in range(p.img.shape[1]):
        d[p.img[:, a]] = delta
    A.setdiag(A.diagonal() + d)
    A.sort_indices()
    return A


@pytest.mark.parametrize("pc", ["amgr", "amgr_sub"])
@pytest.mark.parametrize("f3", [False, True], ids=["static", "afsai_emin"])
def test_rebuild_of_a_setup_is_the_setup(pc, f3):
    p = make_problem((20, 16, 14), s=2, m=1, seed=61, y_stretch=1.5, kappa="lognormal")
    opt = amg.AMGOptions(coarse_max=40, afsai_nnz=5 if f3 else 0, emin_steps=4 if f3 else 0)
    ctx = krylov.setup(p.A, p.img, opt, precond=pc, k=4)
    assert ctx["hier"].nlev >= 4
    rb = refresh.rebuild_below(ctx)
    _same_ctx(rb, ctx)
    for r1, r2 in zip(rb["lrc"].ritz, ctx["lrc"].ritz):
        assert np.array_equal(np.asarray(r1), np.asarray(r2))


@pytest.mark.parametrize("pc", ["amgr", "amgr_sub"])
def test_rebuild_after_a_diagonal_shift_is_the_fresh_setup(pc):
    p = make_problem((24, 20, 16), s=2, m=1, seed=62, y_stretch=1.5, kappa="lognormal")
    opt = amg.AMGOptions(coarse_max=40, trunc0=0.0)
    A1 = _diagonal_shift(p, 5, 0.3)
    ctx0 = krylov.setup(p.A, p.img, opt, precond=pc)
    fresh = krylov.setup(A1, p.img, opt, precond=pc)
    kept = refresh.refresh(ctx0, A1)
    # the reduction level is the fresh one, level 1's split is not
    _same_level(kept["hier"].levels[0], fresh["hier"].levels[0])
    assert np.array_equal(kept["hier"].levels[1].A.data, fresh["hier"].levels[1].A.data)
    assert np.any(kept["hier"].levels[1].C != fresh["hier"].levels[1].C)
    rb = refresh.rebuild_below(kept)
    _same_ctx(rb, fresh)
    x_rb = krylov.solve(rb, p.b, tol=1e-12)
    x_fr = krylov.solve(fresh, p.b, tol=1e-12)
    assert np.array_equal(x_rb.iters, x_fr.iters)
    assert np.array_equal(x_rb.x, x_fr.x)
