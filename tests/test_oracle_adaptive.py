"""Pins of the oracle's adaptive FSAI pattern and energy-minimising
interpolation (oracle/amg.py: afsai_pattern, emin), the options for the
smoother and interpolation that the paper's experiments use (Sec. 5) and
cite without defining.

aFSAI: the trivial and the complete pattern reduce to Jacobi and to the
inverse Cholesky factor; a worked anisotropic 5-point example fixes the
greedy choice in closed form; the first choice equals a brute-force search
over all pairs; patterns are nested and the diagonal of G grows with the
entry budget.  EMIN: pattern and row sums are kept, the energy falls step by
step, and enough steps reach the equality-constrained minimiser of a dense
KKT system."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from gen import make_problem
from oracle import amg, krylov


def _lap2d(nx, ny, ax, ay):
    """5-point operator on an nx x ny grid (x fastest), Dirichlet all round:
    diagonal 2 ax + 2 ay, -ax to x-neighbours, -ay to y-neighbours."""
    Tx = sp.diags([-np.ones(nx - 1), 2 * np.ones(nx), -np.ones(nx - 1)], [-1, 0, 1])
    Ty = sp.diags([-np.ones(ny - 1), 2 * np.ones(ny), -np.ones(ny - 1)], [-1, 0, 1])
    A = (ax * sp.kron(sp.identity(ny), Tx) + ay * sp.kron(Ty, sp.identity(nx))).tocsr()
    A.sort_indices()
    return A


def _random_spd_graph(n, seed):
    """A sparse SPD matrix: weighted graph Laplacian of a random graph plus a
    positive diagonal shift."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for i in range(n):
        for j in rng.choice(n, size=3, replace=False):
            if j != i:
                w = rng.uniform(0.1, 2.0)
                rows += [i, j]
                cols += [j, i]
                vals += [-w, -w]
    W = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    W.sum_duplicates()
    d = -np.asarray(W.sum(axis=1)).ravel() + rng.uniform(0.1, 1.0, n)
    A = (W + sp.diags(d)).tocsr()
    A.sort_indices()
    return A


def _row_pattern(S, i):
    return list(S.indices[S.indptr[i]:S.indptr[i + 1]])


def test_afsai_with_one_entry_is_jacobi():
    A = _lap2d(7, 5, 1.0, 3.0)
    n = A.shape[0]
    S = amg.afsai_pattern(A, np.zeros(n, np.int64), 1)
    assert S.nnz == n and np.array_equal(S.indices, np.arange(n))
    G = amg.fsai(A, S, np.zeros(n, np.int64))
    assert np.allclose(G.diagonal(), 1.0 / np.sqrt(A.diagonal()), rtol=1e-15, atol=0)


def test_afsai_with_a_full_budget_is_the_inverse_cholesky_factor():
    """With room for every lower entry the search stops only when A g vanishes
    on every lower index outside the pattern, i.e. at the exact row of
    L^{-1} (A = L L^T)."""
    A = _random_spd_graph(40, 3)
    n = A.shape[0]
    S = amg.afsai_pattern(A, np.zeros(n, np.int64), n)
    G = amg.fsai(A, S, np.zeros(n, np.int64)).toarray()
    Linv = np.linalg.inv(np.linalg.cholesky(A.toarray()))
    Gfull = np.zeros_like(Linv)
    Gfull[:, :] = G
    assert np.abs(Gfull - Linv).max() <= 1e-10 * np.abs(Linv).max()
    assert np.abs(G @ A.toarray() @ G.T - np.eye(n)).max() <= 1e-10


@pytest.mark.parametrize("ax,ay,third", [(1.0, 4.0, "south-south"), (1.0, 2.0, "west")])
def test_afsai_worked_anisotropic_example(ax, ay, third):
    """Interior row i of the 5-point operator, d = 2 ax + 2 ay.  Step 1: the
    candidates are west (A g = -ax) and south (-ay): with ay > ax south is
    taken.  Step 2: with g = e_i + (ay/d) e_south, A g is -ax at west,
    -ay^2/d at south-south and -ax ay/d at the two x-neighbours of south;
    scores ax^2, ay^4/d^2, ax^2 ay^2/d^2 (over d).  ax = 1, ay = 4: 2.56 > 1,
    south-south; ax = 1, ay = 2: 0.44 < 1, west."""
    nx, ny = 9, 8
    A = _lap2d(nx, ny, ax, ay)
    n = A.shape[0]
    S2 = amg.afsai_pattern(A, np.zeros(n, np.int64), 2)
    S3 = amg.afsai_pattern(A, np.zeros(n, np.int64), 3)
    i = 4 * nx + 4                       # x = 4, y = 4
    assert _row_pattern(S2, i) == [i - nx, i]
    expect = {"south-south": i - 2 * nx, "west": i - 1}[third]
    assert _row_pattern(S3, i) == sorted([i - nx, expect, i])
    # boundary rows: no south neighbour -> west; no west neighbour -> south
    assert _row_pattern(S2, 3) == [2, 3]
    assert _row_pattern(S2, 2 * nx) == [nx, 2 * nx]
    assert _row_pattern(S2, 0) == [0]


def test_afsai_first_choice_is_the_best_pair_by_brute_force():
    """After one step the row's G_ii (= (min g^T A g)^(-1/2)) is the largest
    over all patterns {j, i}, j < i: checked against static FSAI on every
    such pair."""
    A = _random_spd_graph(30, 5)
    n = A.shape[0]
    z = np.zeros(n, np.int64)
    G2 = amg.fsai(A, amg.afsai_pattern(A, z, 2), z)
    Ad = A.toarray()
    for i in range(1, n):
        best = 1.0 / np.sqrt(Ad[i, i])
        for j in range(i):
            Sp = sp.csr_matrix(([1.0, 1.0], ([i, i], [j, i])), shape=(n, n))
            gii = amg.fsai(A, Sp, z)[i, i]
            best = max(best, gii)
        assert G2[i, i] >= best * (1 - 1e-9), (i, G2[i, i], best)


def test_afsai_patterns_are_nested_and_the_diagonal_grows():
    A = _random_spd_graph(60, 7)
    n = A.shape[0]
    z = np.zeros(n, np.int64)
    prev_S, prev_d = None, None
    for k in range(1, 7):
        S = amg.afsai_pattern(A, z, k)
        assert np.all(np.diff(S.indptr) <= k)
        rows = np.repeat(np.arange(n), np.diff(S.indptr))
        assert np.all(S.indices <= rows)
        G = amg.fsai(A, S, z)
        d = G.diagonal()
        assert np.abs((G @ A @ G.T).diagonal() - 1.0).max() < 1e-12
        if prev_S is not None:
            assert (prev_S - prev_S.multiply(S)).nnz == 0          # nested
            assert np.all(d >= prev_d * (1 - 1e-12))               # min g^T A g does not grow
        prev_S, prev_d = S, d


def test_afsai_respects_the_blocks():
    A = _lap2d(8, 8, 1.0, 1.0)
    n = A.shape[0]
    block = (np.arange(n) % 3 == 0).astype(np.int64)
    S = amg.afsai_pattern(A, block, 5)
    rows = np.repeat(np.arange(n), np.diff(S.indptr))
    assert np.all(block[rows] == block[S.indices])


def _split_problem(nx=10, ny=9, seed=2):
    rng = np.random.default_rng(seed)
    A = _lap2d(nx, ny, 1.0, 1.0)
    A = (sp.diags(np.exp(0.3 * rng.standard_normal(A.shape[0]))) @ A @
         sp.diags(np.exp(0.3 * rng.standard_normal(A.shape[0])))).tocsr()
    A = ((A + A.T) * 0.5).tocsr()
    A = (A + sp.diags(np.abs(A).sum(axis=1).A.ravel() * 0.01)).tocsr()
    A.sort_indices()
    C = amg.coarsen_standard(A, 1, 0.25, 5)
    return A, C


def _energy(A, P):
    return float((P.T @ A @ P).diagonal().sum())


def test_emin_keeps_pattern_row_sums_and_lowers_the_energy_every_step():
    A, C = _split_problem()
    P0 = amg.interpolation(A, C, 2)
    e_prev = _energy(A, P0)
    for k in range(1, 8):
        P = amg.emin(A, C, P0, k)
        assert np.array_equal(P.indptr, P0.indptr) and np.array_equal(P.indices, P0.indices)
        assert np.allclose(np.asarray(P.sum(axis=1)).ravel(), np.asarray(P0.sum(axis=1)).ravel(),
                           rtol=1e-13, atol=1e-14)
        assert np.array_equal(P.toarray()[C], np.eye(int(C.sum())))
        e = _energy(A, P)
        assert e <= e_prev * (1 + 1e-14), (k, e, e_prev)
        e_prev = e
    assert e_prev < _energy(A, P0)
    assert amg.emin(A, C, P0, 0).toarray().tolist() == P0.toarray().tolist()


def test_emin_reaches_the_constrained_minimiser_of_the_kkt_system():
    """minimise w^T (I (x) A_FF) w + 2 b^T w over the pattern entries w of W
    subject to the row sums of W, solved as one dense KKT system."""
    A, C = _split_problem(7, 6, 4)
    P0 = amg.interpolation(A, C, 2)
    fidx, cidx = np.flatnonzero(~C), np.flatnonzero(C)
    W0 = P0.tocsr()[fidx].tocsr()
    W0.sort_indices()
    wr = np.repeat(np.arange(fidx.size), np.diff(W0.indptr))
    wc = W0.indices
    m = wr.size
    Ad = A.toarray()
    AFF = Ad[np.ix_(fidx, fidx)]
    AFC = Ad[np.ix_(fidx, cidx)]
    H = np.zeros((m, m))
    for p in range(m):
        for q in range(m):
            if wc[p] == wc[q]:
                H[p, q] = AFF[wr[p], wr[q]]
    b = AFC[wr, wc]
    B = np.zeros((fidx.size, m))
    B[wr, np.arange(m)] = 1.0
    s = np.asarray(W0.sum(axis=1)).ravel()
    K = np.block([[H, B.T], [B, np.zeros((fidx.size, fidx.size))]])
    sol = np.linalg.lstsq(K, np.concatenate([-b, s]), rcond=None)[0]
    w_star = sol[:m]
    P = amg.emin(A, C, P0, 4 * m)
    W = P.tocsr()[fidx].tocsr()
    W.sort_indices()
    assert np.abs(W.data - w_star).max() <= 1e-8 * np.abs(w_star).max()


@pytest.mark.parametrize("pc", ["amgr", "amgr_sub"])
def test_hierarchy_with_adaptive_fsai_and_emin_keeps_the_identities_and_solves(pc):
    p = make_problem((16, 14, 12), s=2, m=2, seed=8, y_stretch=1.5, kappa="lognormal")
    opt = amg.AMGOptions(coarse_max=40, afsai_nnz=5, emin_steps=4)
    ctx = krylov.setup(p.A, p.img, opt, precond=pc)
    H = ctx["hier"]
    assert H.nlev >= 3
    for lev in range(H.nlev - 1):
        L = H.levels[lev]
        assert np.all(np.diff(L.G.indptr) <= 5)
        Ad = L.A.toarray()
        Gd = L.G.toarray()
        assert np.abs(np.diag(Gd @ Ad @ Gd.T) - 1).max() < 1e-12
        Pd = L.P.toarray()
        assert np.abs(Pd.T @ Ad @ Pd - H.levels[lev + 1].A.toarray()).max() <= 1e-12 * np.abs(Ad).max()
    if ctx["sub"] is not None:
        for SH in ctx["sub"].subs:
            for lev, L in enumerate(SH.levels[:-1], start=1):
                assert np.array_equal(L.G.indices, H.levels[lev].G.indices)
    res = krylov.solve(ctx, p.b, tol=1e-12)
    ref = spla.splu(p.A.tocsc()).solve(p.b)
    assert np.linalg.norm(res.x - ref) <= 1e-9 * np.linalg.norm(ref)
