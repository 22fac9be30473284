"""Pins of the oracle's AMGS (oracle/amgs.py, Sec. 3.1): the block LDU inverse
of eq. (3.2) and its preconditioner form eq. (3.12), the decoupled Schur
complement (eqs. (3.5)-(3.7)), the FSAI-based Schur approximation (eq. (3.4)),
the low-rank corrected Schur inverse (eq. (3.11), Thm. 2.2), symmetry of the
symmetric form and end-to-end convergence to a direct solve."""
import dataclasses

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gen import make_problem
from oracle import amg, amgs, symmetry


def _ctx(N=(10, 10, 8), s=2, k=0, light=False, seed=3, **kw):
    p = make_problem(N, s=s, seed=seed, **kw)
    opt = amgs.AMGSOptions(amg=amg.AMGOptions(coarse_max=40), k=k, light=light)
    return p, amgs.setup(p.A, p.img, opt)


def _subsystems(ctx):
    return [(ctx["Ainn"] + o).toarray() for o in ctx["outs"]]


def test_exact_inverses_make_the_preconditioner_the_inverse():
    """Eq. (3.12) with K1 = K2 = K^{-1} and the exact decoupled Schur
    complement is the LDU inverse of eq. (3.2): M A_a = I."""
    p, ctx = _ctx((8, 6, 6), s=2)
    Kinv = np.linalg.inv(ctx["K"].toarray())
    Bd, C1 = ctx["B"].toarray(), ctx["C1"].toarray()
    Sinv = [np.linalg.inv(C1 + np.diag(ctx["sigma_g"][:, a]) - Bd.T @ Kinv @ Bd) for a in range(len(ctx["outs"]))]
    for a, Aa in enumerate(_subsystems(ctx)):
        n = Aa.shape[0]
        M = amgs.apply_with(ctx, np.eye(n), n, lambda X: Kinv @ X, lambda b, Q: Sinv[a] @ Q, lambda X: Kinv @ X)
        assert np.abs(M @ Aa - np.eye(n)).max() < 1e-9


def test_schur_complement_decouples_in_the_transformed_basis():
    """The Schur complement of the inner block of the full matrix (every
    image's inner cells against every image's interface cells), taken to the
    Q_s basis, is block diagonal with blocks C_1 + Sigma_a - B^T K^{-1} B."""
    p, ctx = _ctx((6, 6, 5), s=2)
    A = p.A.toarray()
    img = p.img
    S = img.shape[1]
    inner, ifc = ctx["inner"], ctx["ifc"]
    I_all = img[inner].T.ravel()     # image by image
    G_all = img[ifc].T.ravel()
    Sbar = A[np.ix_(G_all, G_all)] - A[np.ix_(G_all, I_all)] @ np.linalg.solve(A[np.ix_(I_all, I_all)],
                                                                                A[np.ix_(I_all, G_all)])
    Q = np.kron(symmetry.hadamard(S), np.eye(ifc.size)) / np.sqrt(S)
    Sh = Q @ Sbar @ Q.T
    Kinv = np.linalg.inv(ctx["K"].toarray())
    Bd, C1 = ctx["B"].toarray(), ctx["C1"].toarray()
    g = ifc.size
    for a in range(S):
        for b in range(S):
            blk = Sh[a * g:(a + 1) * g, b * g:(b + 1) * g]
            if a == b:
                ref = C1 + np.diag(ctx["sigma_g"][:, a]) - Bd.T @ Kinv @ Bd
                assert np.abs(blk - ref).max() < 1e-10 * np.abs(ref).max()
            else:
                assert np.abs(blk).max() < 1e-10 * np.abs(Sh).max()


def test_schur_g_with_the_exact_inverse_factor_is_the_schur_complement():
    """S_G1 = C_1 - B^T G^T G B equals C_1 - B^T K^{-1} B when G is the exact
    inverse Cholesky factor (G^T G = K^{-1}), and is symmetric."""
    p, ctx = _ctx((8, 8, 6), s=1)
    K = ctx["K"].toarray()
    L = np.linalg.cholesky(K)
    G = np.linalg.inv(L)
    import scipy.sparse as sp
    S = amgs.schur_g(ctx["C1"], ctx["B"], sp.csr_matrix(G)).toarray()
    ref = ctx["C1"].toarray() - ctx["B"].toarray().T @ np.linalg.solve(K, ctx["B"].toarray())
    assert np.abs(S - ref).max() < 1e-10 * np.abs(ref).max()
    Sg = ctx["SG1"].toarray()
    assert np.array_equal(Sg, Sg.T)


def test_fsai_factors_are_lower_with_unit_scaled_diagonal():
    """G_K and G_S1 are lower triangular on their stated patterns and
    diag(G A G^T) = 1 (the FSAI normalisation); the K pattern reaches
    distance-2 neighbours."""
    p, ctx = _ctx((10, 8, 7), s=2, y_stretch=1.5)
    for G, A in ((ctx["GK"], ctx["K"]), (ctx["GS1"], ctx["SG1"])):
        Gd = G.toarray()
        assert np.all(np.triu(Gd, 1) == 0)
        d = np.diag(Gd @ A.toarray() @ Gd.T)
        assert np.abs(d - 1).max() < 1e-12
    K = ctx["K"]
    P2 = (abs(K) @ abs(K)).tocsr()
    low = np.tril(P2.toarray() != 0)
    assert np.array_equal(ctx["GK"].toarray() != 0, low)
    Sf = amgs.filtered_pattern(ctx["SG1"], 0.01)
    lowS = np.tril((Sf @ Sf @ Sf).toarray() != 0)
    assert np.array_equal(ctx["GS1"].toarray() != 0, lowS)
    assert np.tril((Sf @ Sf).toarray() != 0).sum() < lowS.sum()


def test_filter_drops_small_couplings_symmetrically():
    import scipy.sparse as sp
    M = sp.csr_matrix(np.array([[4.0, -1e-3, -1.0], [-1e-3, 4.0, -0.5], [-1.0, -0.5, 9.0]]))
    P = amgs.filtered_pattern(M, 0.01).toarray()
    assert P[0, 1] == 0 and P[1, 0] == 0            # 1e-3 < 0.01 * 4
    assert P[0, 2] == 1 and P[2, 0] == 1 and P[1, 2] == 1 and np.all(np.diag(P) == 1)


def test_full_rank_correction_gives_the_amg_schur_inverse():
    """Thm. 2.2: with every eigenpair of G S_AMG,a G^T kept, the corrected
    FSAI is S_AMG,a^{-1} exactly (up to the Lanczos basis' rounding)."""
    p, ctx = _ctx((6, 5, 4), s=1)
    n = ctx["ifc"].size
    low = amgs.build_schur_lrc(ctx, n, 7, keep_all=True, steps=n)
    G = ctx["GS1"].toarray()
    for a in range(2):
        Sam = np.column_stack([amgs.schur_amg(ctx, a, e[:, None])[:, 0] for e in np.eye(n)])
        Minv = G.T @ G + low.U[a] @ np.diag(low.coef[a]) @ low.U[a].T
        assert np.abs(Minv @ Sam - np.eye(n)).max() < 1e-7


def test_symmetric_form_is_spd_and_light_form_is_not_symmetric():
    p, ctx = _ctx((8, 6, 6), s=1, k=4)
    n = p.n_b
    M = amgs.apply(ctx, np.eye(n), n)
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
    ctx_l = dict(ctx, opt=dataclasses.replace(ctx["opt"], light=True))
    Ml = amgs.apply(ctx_l, np.eye(n), n)
    assert np.abs(Ml - Ml.T).max() > 1e-6 * np.abs(Ml).max()


@pytest.mark.parametrize("light", [False, True], ids=["symmetric", "light"])
def test_solve_matches_direct_solve_and_corrections_help(light):
    """PCG (symmetric form) / flexible CG (light form) with AMGS reaches the
    sparse direct solution; the low-rank corrected Schur approximation needs
    no more iterations than the plain FSAI one (Table 3's ordering)."""
    p = make_problem((16, 14, 12), s=2, m=2, seed=5, y_stretch=1.5)
    ref = spla.splu(p.A.tocsc()).solve(p.b)
    its = {}
    for k in (0, 8):
        opt = amgs.AMGSOptions(amg=amg.AMGOptions(coarse_max=40), k=k, light=light)
        ctx = amgs.setup(p.A, p.img, opt)
        res = amgs.solve(ctx, p.b, tol=1e-12)
        assert np.linalg.norm(res.x - ref) <= 1e-9 * np.linalg.norm(ref)
        its[k] = int(res.iters.max())
    assert its[8] <= its[0] < 200
