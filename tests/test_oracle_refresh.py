"""Pins of the oracle's numeric re-setup (oracle/refresh.py): it equals a
fresh setup whenever the fresh setup makes the same structural decisions
(the same matrix; the matrix scaled by 2), and for a new coefficient field on
the same mesh every level keeps the defining identities (Galerkin product,
FSAI normalisation, P = [W; I] with rescaled row sums, symmetric V-cycle)
and the solve reaches the direct solution."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gen import make_problem
from oracle import amg, krylov, refresh

OPT = amg.AMGOptions(coarse_max=40)


def _equal_hier(H1, H2):
    assert H1.nlev == H2.nlev
    for L1, L2 in zip(H1.levels, H2.levels):
        for M1, M2 in ((L1.A, L2.A), (L1.P, L2.P), (L1.G, L2.G)):
            if M2 is None:
                assert M1 is None
                continue
            assert np.array_equal(M1.indptr, M2.indptr) and np.array_equal(M1.indices, M2.indices)
            assert np.array_equal(M1.data, M2.data)
        if L2.C is not None:
            assert np.array_equal(L1.C, L2.C) and L1.omega == L2.omega
    assert np.array_equal(H1.coarse_factor[0], H2.coarse_factor[0])


F3 = amg.AMGOptions(coarse_max=40, afsai_nnz=5, emin_steps=4)


@pytest.mark.parametrize("precond,k,opt", [("amgr", 0, OPT), ("amgr_sub", 0, OPT), ("amgr_sub", 4, OPT),
                                           ("amgr", 0, F3), ("amgr_sub", 4, F3)])
def test_refresh_with_the_same_matrix_is_the_setup(precond, k, opt):
    """With adaptive FSAI and energy minimisation too: the kept adaptive
    patterns are the ones the setup chose, and the minimisation repeats the
    setup's steps from the same start."""
    p = make_problem((16, 14, 12), s=2, seed=3, y_stretch=1.5, kappa="lognormal")
    ctx = krylov.setup(p.A, p.img, opt, precond=precond, k=k)
    new = refresh.refresh(ctx, p.A)
    _equal_hier(new["hier"], ctx["hier"])
    if ctx["sub"] is not None:
        for S1, S2 in zip(new["sub"].subs, ctx["sub"].subs):
            _equal_hier(S1, S2)
    if k:
        for r1, r2 in zip(new["lrc"].ritz, ctx["lrc"].ritz):
            assert np.array_equal(r1, r2)


@pytest.mark.parametrize("opt", [OPT, F3])
def test_refresh_of_a_scaled_matrix_is_its_fresh_setup(opt):
    """Scaling by 2 is exact: the adaptive FSAI scores and the energy
    minimisation's gradients double, its step lengths do not change."""
    p = make_problem((14, 12, 10), s=1, seed=4, jitter=0.2, kappa="lognormal")
    ctx = krylov.setup(p.A, p.img, opt, precond="amgr_sub")
    A2 = (2.0 * p.A).tocsr()
    fresh = krylov.setup(A2, p.img, opt, precond="amgr_sub")
    new = refresh.refresh(ctx, A2)
    _equal_hier(new["hier"], fresh["hier"])
    for S1, S2 in zip(new["sub"].subs, fresh["sub"].subs):
        _equal_hier(S1, S2)


def test_refresh_for_a_new_coefficient_keeps_the_identities_and_solves():
    p0 = make_problem((16, 14, 12), s=2, m=2, seed=5, kappa="lognormal")
    p1 = make_problem((16, 14, 12), s=2, m=2, seed=6, kappa="lognormal")
    assert np.array_equal(p0.A.indices, p1.A.indices) and not np.array_equal(p0.A.data, p1.A.data)
    ctx = krylov.setup(p0.A, p0.img, OPT, precond="amgr_sub", k=4)
    new = refresh.refresh(ctx, p1.A)
    H = new["hier"]
    for lev in range(H.nlev - 1):
        L = H.levels[lev]
        Pd = L.P.toarray()
        Ad = L.A.toarray()
        Ac = H.levels[lev + 1].A.toarray()
        assert np.abs(Pd.T @ Ad @ Pd - Ac).max() <= 1e-12 * np.abs(Ac).max()
        Gd = L.G.toarray()
        assert np.abs(np.diag(Gd @ Ad @ Gd.T) - 1).max() < 1e-12
        cidx = np.flatnonzero(L.C)
        assert np.array_equal(Pd[cidx], np.eye(cidx.size))
        fidx = np.flatnonzero(~L.C)
        off = Ad.sum(axis=1) - np.diag(Ad)
        rho = -off / np.diag(Ad)
        ws = Pd[fidx].sum(axis=1)
        nz = ws != 0
        assert np.abs(ws[nz] - rho[fidx][nz]).max() <= 1e-12 * np.abs(rho).max()
        assert (L.G != ctx["hier"].levels[lev].G).nnz > 0            # values really changed
    for S0, S1 in zip(ctx["sub"].subs, new["sub"].subs):        # kept FSAI patterns per subsystem
        for L0, L1 in zip(S0.levels, S1.levels):
            if L0.G is not None:
                assert np.array_equal(L0.G.indptr, L1.G.indptr) and np.array_equal(L0.G.indices, L1.G.indices)
                Gd, Ad = L1.G.toarray(), L1.A.toarray()
                assert np.abs(np.diag(Gd @ Ad @ Gd.T) - 1).max() < 1e-12
    n = p1.n_b
    V = np.stack([amg.vcycle(H, e) for e in np.eye(n)], axis=1)
    assert np.abs(V - V.T).max() <= 1e-12 * np.abs(V).max()
    res = krylov.solve(new, p1.b, tol=1e-12)
    ref = spla.splu(p1.A.tocsc()).solve(p1.b)
    assert np.linalg.norm(res.x - ref) <= 1e-9 * np.linalg.norm(ref)


def test_refresh_rejects_a_different_sparsity():
    p0 = make_problem((12, 10, 8), s=1, seed=7)
    p1 = make_problem((12, 10, 10), s=1, seed=7)
    ctx = krylov.setup(p0.A, p0.img, OPT)
    with pytest.raises(Exception):
        refresh.refresh(ctx, p1.A)
