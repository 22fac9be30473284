"""Pins of the low-rank corrections (Thm. 2.1 / eq. (2.24) and Thm. 2.2 /
eq. (2.32)) on inputs small enough for dense eigendecompositions."""
import numpy as np
import pytest

from gen import make_problem
from oracle import amg, krylov, lrc, symmetry


def _ctx(N=(8, 8), s=1, **kw):
    p = make_problem(N, s=s, m=1, seed=6, y_stretch=1.5, **kw)
    ctx = krylov.setup(p.A, p.img, amg.AMGOptions(coarse_max=8))
    return p, ctx


def _vmat(hier, n):
    return np.column_stack([amg.vcycle(hier, e) for e in np.eye(n)])


def test_ritz_values_are_dense_eigenvalues():
    """With as many Lanczos steps as unknowns, the Ritz values of M^{-1} A_a
    are its eigenvalues (dense generalised eigenproblem)."""
    p, ctx = _ctx()
    Ainn, outs, hier = ctx["Ainn"], ctx["outs"], ctx["hier"]
    n = Ainn.shape[0]
    assert hier.nlev >= 2
    low = lrc.build_lrcamg(hier, Ainn, outs, k=6, seed=1)
    Vm = _vmat(hier, n)
    for a in range(len(outs)):
        Ah = (Ainn + outs[a]).toarray()
        ev = np.sort(np.linalg.eigvals(Vm @ Ah).real)
        assert np.abs(low.ritz[a] - ev[:6]).max() < 1e-8


def test_lrcamg_full_rank_is_exact_inverse():
    """Thm. 2.2 with every eigenpair: M^{-1} + U diag(1 - lam) U^T = A_a^{-1},
    so PCG converges in one iteration."""
    p, ctx = _ctx()
    Ainn, outs, hier = ctx["Ainn"], ctx["outs"], ctx["hier"]
    n = Ainn.shape[0]
    low = lrc.build_lrcamg(hier, Ainn, outs, k=n, seed=1, keep_all=True, steps=n)
    Vm = _vmat(hier, n)
    for a in range(len(outs)):
        Ah = (Ainn + outs[a]).toarray()
        U, c = low.U[a], low.coef[a]
        Minv = Vm + U @ np.diag(c) @ U.T
        assert np.abs(Minv @ Ah - np.eye(n)).max() < 1e-9
    ctx["lrc"] = low
    r = krylov.solve(ctx, p.b, tol=1e-9)
    assert r.iters.max() <= 2


def test_lrcamg_symmetric_form_equals_paper_form():
    """For exact eigenpairs, (I + U Theta V^T) M^{-1} with V = M U (biorthonormal,
    V^T U = I) and Theta = Lambda^{-1} - I equals M^{-1} + U diag(1-lam) U^T
    when U^T A U = I."""
    p, ctx = _ctx()
    Ainn, outs, hier = ctx["Ainn"], ctx["outs"], ctx["hier"]
    n = Ainn.shape[0]
    low = lrc.build_lrcamg(hier, Ainn, outs, k=5, seed=1, keep_all=True, steps=n)
    Vm = _vmat(hier, n)
    Mm = np.linalg.inv(Vm)
    for a in range(len(outs)):
        Ah = (Ainn + outs[a]).toarray()
        U = low.U[a]
        lam = 1.0 - low.coef[a]
        assert np.abs(U.T @ Ah @ U - np.eye(U.shape[1])).max() < 1e-10
        V = Mm @ U @ np.linalg.inv(U.T @ Mm @ U)        # = M U Lambda = A_a U
        assert np.abs(V - Ah @ U).max() < 1e-8 * np.abs(V).max()
        assert np.abs(V.T @ U - np.eye(U.shape[1])).max() < 1e-10
        paper = (np.eye(n) + U @ np.diag(1.0 / lam - 1.0) @ V.T) @ Vm
        sym = Vm + U @ np.diag(1.0 - lam) @ U.T
        assert np.abs(paper - sym).max() < 1e-9 * np.abs(sym).max()


def test_partial_correction_maps_corrected_eigenvalues_to_one():
    p, ctx = _ctx()
    Ainn, outs, hier = ctx["Ainn"], ctx["outs"], ctx["hier"]
    n = Ainn.shape[0]
    k = 4
    low = lrc.build_lrcamg(hier, Ainn, outs, k=k, seed=1, steps=n)
    Vm = _vmat(hier, n)
    for a in range(len(outs)):
        Ah = (Ainn + outs[a]).toarray()
        ev0 = np.sort(np.linalg.eigvals(Vm @ Ah).real)
        U, c = low.U[a], low.coef[a]
        ev1 = np.sort(np.linalg.eigvals((Vm + U @ np.diag(c) @ U.T) @ Ah).real)
        kept = U.shape[1]
        want = np.sort(np.concatenate([np.ones(kept), ev0[kept:]]))
        assert np.abs(ev1 - want).max() < 1e-8


def test_lrcfsai_full_rank_is_exact_inverse():
    """Thm. 2.1 with every eigenpair of G A_a G^T: G^T G + Z Theta Z^T = A_a^{-1}."""
    p = make_problem((8, 8), s=1, m=1, seed=6, y_stretch=1.5)
    ctx = krylov.setup(p.A, p.img, precond="fsai")
    Ainn, outs, G = ctx["Ainn"], ctx["outs"], ctx["G"]
    n = Ainn.shape[0]
    low = lrc.build_lrcfsai(G, Ainn, outs, k=n, seed=1, keep_all=True, steps=n)
    Gd = G.toarray()
    for a in range(len(outs)):
        Ah = (Ainn + outs[a]).toarray()
        Minv = Gd.T @ Gd + low.U[a] @ np.diag(low.coef[a]) @ low.U[a].T
        assert np.abs(Minv @ Ah - np.eye(n)).max() < 1e-9


def test_lrc_reduces_iterations():
    """Table 1/2 trend: corrections lower the PCG iteration count."""
    p = make_problem((16, 16, 16), s=3, m=1, seed=2, y_stretch=1.5)
    its = []
    for k in (0, 8):
        ctx = krylov.setup(p.A, p.img, amg.AMGOptions(coarse_max=64), k=k)
        its.append(krylov.solve(ctx, p.b, tol=1e-10).iters.max())
    assert its[1] < its[0]
