"""Pins of the multigrid-reduction part of the oracle (Sec. 3.2: Alg. 2,
eqs. (3.13)-(3.15), Alg. 3) against invariants, special cases that reduce
to textbook formulas, and brute force."""
import dataclasses
import itertools

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from gen import make_problem
from oracle import amg, krylov, symmetry


def _inner(N=(12, 12, 12), s=3, **kw):
    p = make_problem(N, s=s, seed=4, **kw)
    H = symmetry.base_blocks(p.A, p.img)
    Ainn, _ = symmetry.inner_outer(H)
    return Ainn.tocsr(), symmetry.interface_rows(H)


# ----------------------------------------------------------------- strength

def test_strength_uniform_all_neighbours_strong():
    """Uniform 7-point stencil: every off-diagonal entry has the same size, so
    every neighbour is strong."""
    A, _ = _inner()
    S = amg.strength(A, 0.25)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    assert S.nnz == int((A.indices != rows).sum())


def test_strength_anisotropic_drops_weak_direction():
    """Cells with aspect ratio 1:3 in 2D: x-couplings are 9x the y-couplings
    (area/distance), above 1/theta = 4, so only x-neighbours are strong."""
    p = make_problem((12, 4), s=1, seed=1)      # hx = 1/12, hy = 1/4: T_x = hy/hx = 3, T_y = 1/3
    A = p.A.tocsr()
    S = amg.strength(A, 0.25)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(S.indptr))
    assert S.nnz > 0
    assert np.all(np.isclose(A[rows, S.indices].A1, -3.0))


def test_strength_threshold_is_inclusive():
    A = sp.csr_matrix(np.array([[4.0, -1.0, -0.25, 0.0], [-1.0, 4.0, -0.5, -0.1],
                                [-0.25, -0.5, 4.0, 0.0], [0.0, -0.1, 0.0, 1.0]]))
    S = amg.strength(A, 0.25).toarray()
    assert S[0].tolist() == [0, 1, 1, 0]         # 0.25 >= 0.25 * 1
    assert S[1].tolist() == [1, 0, 1, 0]         # 0.1 < 0.25
    assert S[3].tolist() == [0, 1, 0, 0]


# ----------------------------------------------------------------- independent sets

def _brute_lexfirst(G, rank):
    """Among all maximal independent sets, the one whose indicator vector,
    read in decreasing rank order, is lexicographically largest."""
    n = G.shape[0]
    Gd = G.toarray() != 0
    order = np.argsort(-rank)
    best = None
    for bits in itertools.product([0, 1], repeat=n):
        x = np.array(bits, dtype=bool)
        if np.any(Gd[np.ix_(x, x)]):
            continue
        # maximal: every excluded node has a taken neighbour
        if np.any(~x & ~(Gd[:, x].any(axis=1))):
            continue
        key = tuple(x[order])
        if best is None or key > best[0]:
            best = (key, x)
    return best[1]


@pytest.mark.parametrize("seed", range(6))
def test_mis_lexicographically_first_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = 12
    M = (rng.random((n, n)) < 0.25)
    M = np.triu(M, 1)
    M = M | M.T
    G = sp.csr_matrix(M.astype(float))
    rank = rng.permutation(n)
    want = _brute_lexfirst(G, rank)
    assert np.array_equal(amg.mis_greedy(G, rank), want)
    assert np.array_equal(amg.mis_rounds(G, rank), want)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_mis_distance_d_independent_and_maximal(d):
    A, iface = _inner((10, 10, 10), y_stretch=1.5)
    S = amg.strength(A, 0.25)
    T = amg.symmetrise(S)
    inner = np.flatnonzero(~iface)
    Tin = T[inner][:, inner].tocsr()
    Gd = amg.distance_graph(Tin, d)
    rank = np.random.default_rng(d).permutation(inner.size)
    m1 = amg.mis_greedy(Gd, rank)
    m2 = amg.mis_rounds(Gd, rank)
    assert np.array_equal(m1, m2)
    # independence at distance d and maximality, checked by BFS in T_in
    dist = sp.csgraph.shortest_path(Tin, unweighted=True)
    sel = np.flatnonzero(m1)
    sub = dist[np.ix_(sel, sel)]
    np.fill_diagonal(sub, np.inf)
    assert sub.min() > d
    notsel = np.flatnonzero(~m1)
    assert np.all(dist[np.ix_(notsel, sel)].min(axis=1) <= d)


def test_coarse_priorities_count_dependants_not_dependencies():
    """Levels below the reduction rank a node by how many nodes depend on it
    strongly, #{j : i in S_j} (a column count of S), ties broken by the hash.
    On a hand-built asymmetric strength graph the row count (how many nodes i
    depends on) orders the nodes differently, so this fixes the direction."""
    from oracle.splitmix import splitmix64
    # S_0 = {1}, S_1 = {0}, S_2 = {1}, S_3 = {1}, S_4 = {3}: node 1 is a strong
    # dependency of 0, 2 and 3; every row has exactly one entry
    rows = np.array([0, 1, 2, 3, 4])
    cols = np.array([1, 0, 1, 1, 3])
    S = sp.csr_matrix((np.ones(5), (rows, cols)), shape=(5, 5))
    seed, level = 77, 2
    rank = amg.priorities_coarse(S, level, seed)
    dependants = np.array([1, 3, 0, 1, 0])            # column counts, worked out by hand
    h = splitmix64(np.uint64(seed) ^ (np.uint64(level) << np.uint64(40)) ^ np.arange(5, dtype=np.uint64))
    expect = sorted(range(5), key=lambda i: (dependants[i], int(h[i])))
    assert [int(i) for i in np.argsort(rank)] == expect
    assert int(np.argmax(rank)) == 1
    assert sorted(rank.tolist()) == list(range(5))


def test_distance_graph_matches_bfs():
    A, iface = _inner((8, 8, 8))
    T = amg.symmetrise(amg.strength(A, 0.25))
    G2 = amg.distance_graph(T, 2).toarray() != 0
    dist = sp.csgraph.shortest_path(T, unweighted=True)
    want = (dist >= 1) & (dist <= 2)
    assert np.array_equal(G2, want)


def test_level0_coarse_set_contains_interface():
    A, iface = _inner((16, 16, 16), y_stretch=1.5)
    C = amg.coarsen_level0(A, iface, 0.25, 2, 99)
    assert np.all(C[iface])
    # the mis is the same computed both ways
    assert np.array_equal(C, amg.coarsen_level0(A, iface, 0.25, 2, 99, method="greedy"))


# ----------------------------------------------------------------- interpolation

@pytest.mark.parametrize("steps", [1, 2, 3])
def test_interpolation_structure(steps):
    A, iface = _inner((12, 12, 12), y_stretch=1.5)
    C = amg.coarsen_level0(A, iface, 0.25, 2, 5)
    P = amg.interpolation(A, C, steps)
    cidx = np.flatnonzero(C)
    # C rows are unit rows
    Pc = P[cidx].toarray()
    assert np.array_equal(Pc, np.eye(cidx.size))
    # no empty F row when steps >= d
    F = np.flatnonzero(~C)
    if steps >= 2:
        assert np.all(np.diff(P[F].indptr) > 0)
    # row sums equal the direct-interpolation sum rho_i (nonempty rows)
    Ad = A.toarray()
    rho = -(Ad.sum(axis=1) - np.diag(Ad)) / np.diag(Ad)
    rs = np.asarray(P.sum(axis=1)).ravel()
    nonempty = np.diff(P.indptr) > 0
    assert np.abs(rs[nonempty] - np.where(C, 1.0, rho)[nonempty]).max() < 1e-14


def test_interpolation_one_step_is_direct_interpolation():
    """steps = 1: w_ij = -(sum_{l != i} a_il / sum_{k in C} a_ik) a_ij / a_ii,
    the textbook direct interpolation."""
    p = make_problem((10, 10), s=1, seed=2, y_stretch=1.5)
    A = p.A.tocsr()
    S = amg.strength(A, 0.25)
    C = amg.mis_greedy(amg.symmetrise(S), np.arange(A.shape[0]))
    P = amg.interpolation(A, C, 1).toarray()
    Ad = A.toarray()
    cidx = np.flatnonzero(C)
    for i in np.flatnonzero(~C):
        row = Ad[i].copy()
        off = row.sum() - row[i]
        cs = row[cidx].sum()
        if cs == 0:
            assert not P[i].any()
            continue
        want = -(off / cs) * row[cidx] / row[i]
        assert np.abs(P[i] - want).max() < 1e-14


def test_interpolation_many_steps_tends_to_ideal():
    """Without the row rescaling, the Jacobi iteration converges to the ideal
    interpolation -A_FF^{-1} A_FC; with it, rows keep the direction of the
    ideal rows."""
    A, iface = _inner((8, 8, 8))
    C = amg.coarsen_level0(A, iface, 0.25, 2, 1)
    F = ~C
    Ad = A.toarray()
    ideal = -np.linalg.solve(Ad[np.ix_(F, F)], Ad[np.ix_(F, C)])
    P = amg.interpolation(A, C, 200).toarray()[F]
    rs_ideal = ideal.sum(axis=1, keepdims=True)
    rs_P = P.sum(axis=1, keepdims=True)
    assert np.abs(P / rs_P - ideal / rs_ideal).max() < 1e-8


# ----------------------------------------------------------------- Galerkin

def test_galerkin_four_term_expansion():
    """A_c = W^T A_FF W + W^T A_FC + A_CF W + A_CC (eq. (3.15)), symmetric and
    positive definite."""
    A, iface = _inner((12, 12, 12), y_stretch=1.5)
    C = amg.coarsen_level0(A, iface, 0.25, 2, 3)
    P = amg.interpolation(A, C, 2)
    Ac = amg.galerkin(A, P).toarray()
    Ad = A.toarray()
    F = ~C
    W = P.toarray()[F]
    want = (W.T @ Ad[np.ix_(F, F)] @ W + W.T @ Ad[np.ix_(F, C)] + Ad[np.ix_(C, F)] @ W
            + Ad[np.ix_(C, C)])
    assert np.abs(Ac - want).max() < 1e-13 * np.abs(want).max()
    assert np.abs(Ac - Ac.T).max() < 1e-15 * np.abs(Ac).max()
    np.linalg.cholesky(Ac)


def test_symbolic_pattern_keeps_cancellations():
    A = sp.csr_matrix(np.array([[1.0, 1.0], [0.0, 1.0]]))
    B = sp.csr_matrix(np.array([[1.0, 0.0], [-1.0, 0.0]]))
    C = amg.sym_matmul(A, B)
    assert C.nnz == 2 and C[0, 0] == 0.0 and C[1, 0] == -1.0


# ----------------------------------------------------------------- FSAI

def test_fsai_unit_diagonal():
    A, iface = _inner((10, 10, 10), y_stretch=1.5)
    C = amg.coarsen_level0(A, iface, 0.25, 2, 3)
    S = amg.strength(A, 0.25)
    G = amg.fsai(A, S, C.astype(np.int64))
    d = (G @ A @ G.T).diagonal()
    assert np.abs(d - 1.0).max() < 1e-14
    # block diagonal: no F-C entries, lower triangular
    Gc = G.tocoo()
    assert np.all(Gc.col <= Gc.row)
    assert np.all(C[Gc.col] == C[Gc.row])


def test_fsai_full_pattern_is_inverse_cholesky():
    """With the full lower pattern, FSAI gives G = L^{-1}, A = L L^T."""
    rng = np.random.default_rng(0)
    n = 9
    M = rng.standard_normal((n, n))
    Ad = M @ M.T + n * np.eye(n)
    A = sp.csr_matrix(Ad)
    S = sp.csr_matrix(np.ones((n, n)) - np.eye(n))
    G = amg.fsai(A, S, np.zeros(n, dtype=np.int64)).toarray()
    L = np.linalg.cholesky(Ad)
    assert np.abs(G - np.linalg.inv(L)).max() < 1e-12


def test_damping_power_iteration_bound():
    A, iface = _inner((8, 8, 8))
    S = amg.strength(A, 0.25)
    G = amg.fsai(A, S, np.zeros(A.shape[0], dtype=np.int64))
    om = amg.damping(A, G, 7)
    lam = 4.0 / (3.0 * om)
    lmax = np.linalg.eigvalsh((G @ A @ G.T).toarray()).max()
    assert 0.8 * lmax <= lam <= lmax * (1 + 1e-12)


# ----------------------------------------------------------------- V-cycle

def _hier(N=(12, 12, 12), **kw):
    A, iface = _inner(N, **kw)
    opt = amg.AMGOptions(coarse_max=40, jacobi=1)
    return A, amg.build_hierarchy(A, iface, opt)


def test_vcycle_symmetric_positive_definite():
    A, H = _hier(y_stretch=1.5)
    assert H.nlev >= 3
    n = A.shape[0]
    rng = np.random.default_rng(1)
    x = rng.standard_normal(n)
    y = rng.standard_normal(n)
    vx, vy = amg.vcycle(H, x), amg.vcycle(H, y)
    assert abs(x @ vy - y @ vx) <= 1e-12 * abs(x @ vy)
    assert x @ vx > 0 and y @ vy > 0


def test_vcycle_contracts_error():
    """The error propagator I - V A has A-norm below 1 (Alg. 3 is a convergent
    iteration on the system it was built for)."""
    A, H = _hier((8, 8, 8))
    n = A.shape[0]
    Ad = A.toarray()
    V = np.column_stack([amg.vcycle(H, e) for e in np.eye(n)])
    E = np.eye(n) - V @ Ad
    L = np.linalg.cholesky(Ad)
    Et = L.T @ E @ np.linalg.inv(L.T)
    assert np.linalg.norm(Et, 2) < 0.9


def test_two_grid_exact_coarse_solve():
    """Coarsest level = level 0 (n <= coarse_max): the V-cycle is A^{-1}."""
    A, iface = _inner((6, 6, 6))
    H = amg.build_hierarchy(A, iface, amg.AMGOptions(coarse_max=10**6))
    assert H.nlev == 1
    y = np.random.default_rng(2).standard_normal(A.shape[0])
    x = amg.vcycle(H, y)
    assert np.abs(A @ x - y).max() < 1e-12 * np.abs(y).max()


# ----------------------------------------------------------------- AMGR per subsystem

def _sub(N=(12, 12, 12), coarse_max=40, **kw):
    p = make_problem(N, s=3, seed=4, **kw)
    H = symmetry.base_blocks(p.A, p.img)
    Ainn, outs = symmetry.inner_outer(H)
    iface = symmetry.interface_rows(H)
    opt = amg.AMGOptions(coarse_max=coarse_max)
    hier = amg.build_hierarchy(Ainn.tocsr(), iface, opt)
    sigma = np.stack([o.diagonal() for o in outs], axis=1)
    Ahat = [(Ainn + o).tocsr() for o in outs]
    return hier, sigma, Ahat, opt


def test_sub_reduced_operator_is_galerkin_of_each_subsystem():
    """The interface is coarse and P_0 = [W; I], so P_0^T (A_inn + diag sigma_a) P_0
    differs from P_0^T A_inn P_0 only by sigma_a on the coarse interface points:
    the shortcut A_1 + diag(sigma_a[C]) must equal the plain product."""
    hier, sigma, Ahat, opt = _sub(y_stretch=1.5)
    SH = amg.build_sub_hierarchy(hier, sigma, opt)
    P0 = hier.levels[0].P.toarray()
    for a, Aa in enumerate(Ahat):
        ref = P0.T @ Aa.toarray() @ P0
        got = SH.subs[a].levels[0].A.toarray()
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_sub_zero_shift_reproduces_shared_levels():
    hier, sigma, _, opt = _sub()
    SH = amg.build_sub_hierarchy(hier, np.zeros_like(sigma), opt)
    for sub in SH.subs:
        assert len(sub.levels) == hier.nlev - 1
        for Ls, Lh in zip(sub.levels, hier.levels[1:]):
            assert (Ls.A != Lh.A).nnz == 0
            if Lh.P is not None:
                assert (Ls.P != Lh.P).nnz == 0 and (Ls.G != Lh.G).nnz == 0
                assert Ls.omega == Lh.omega


def test_sub_patterns_equal_shared_patterns():
    hier, sigma, _, opt = _sub(y_stretch=1.5)
    SH = amg.build_sub_hierarchy(hier, sigma, opt)
    for sub in SH.subs:
        for Ls, Lh in zip(sub.levels, hier.levels[1:]):
            for X, Y in ((Ls.A, Lh.A), (Ls.P, Lh.P), (Ls.G, Lh.G)):
                if Y is None:
                    continue
                assert np.array_equal(X.indptr, Y.indptr) and np.array_equal(X.indices, Y.indices)


def test_sub_two_grid_is_exact_two_grid_of_subsystem():
    """With two levels the per-subsystem cycle is the two-grid method for
    A_a with the Galerkin coarse operator solved exactly:
    I - V A_a = (I - M A_a)(I - P (P^T A_a P)^{-1} P^T A_a)(I - M A_a)."""
    hier, sigma, Ahat, opt = _sub(coarse_max=200)
    assert hier.nlev == 2
    SH = amg.build_sub_hierarchy(hier, sigma, opt)
    L0 = hier.levels[0]
    n = L0.A.shape[0]
    P = L0.P.toarray()
    G = L0.G.toarray()
    M = L0.omega * G.T @ G
    I = np.eye(n)
    for a in (0, 3, 7):
        Aa = Ahat[a].toarray()
        V = np.column_stack([amg.vcycle_sub(SH, Ahat[a], a, e) for e in I])
        Kc = P @ np.linalg.solve(P.T @ Aa @ P, P.T @ Aa)
        E = (I - M @ Aa) @ (I - Kc) @ (I - M @ Aa)
        assert np.abs((I - V @ Aa) - E).max() < 1e-10


def test_sub_vcycle_symmetric_and_contracts():
    hier, sigma, Ahat, opt = _sub((10, 10, 10), coarse_max=20, y_stretch=1.5)
    assert hier.nlev >= 3
    SH = amg.build_sub_hierarchy(hier, sigma, opt)
    n = Ahat[0].shape[0]
    I = np.eye(n)
    for a in (1, 6):
        Aa = Ahat[a].toarray()
        V = np.column_stack([amg.vcycle_sub(SH, Ahat[a], a, e) for e in I])
        assert np.abs(V - V.T).max() <= 1e-12 * np.abs(V).max()
        assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0
        L = np.linalg.cholesky(Aa)
        E = I - V @ Aa
        assert np.linalg.norm(L.T @ E @ np.linalg.inv(L.T), 2) < 0.9


def test_interpolation_truncation_keeps_large_weights_and_row_sums():
    """With trunc > 0 an F row keeps exactly the weights of the untruncated
    row with |w| >= trunc * max|w| (the row-sum rescaling multiplies a row by
    one factor, so the relative test reads the same before and after it) and
    is rescaled to the same row sum rho_i."""
    A, iface = _inner(y_stretch=1.5)
    C = amg.coarsen_level0(A, iface, 0.25, 2, 7, "rounds")
    full = amg.interpolation(A, C, 3)
    for tr in (0.0, 0.05, 0.1, 0.3):
        P = amg.interpolation(A, C, 3, tr)
        assert P.shape == full.shape
        for i in np.flatnonzero(~C)[::7]:
            fr = full[i].toarray().ravel()
            pr = P[i].toarray().ravel()
            mx = np.abs(fr).max()
            expect = set(full.indices[full.indptr[i]:full.indptr[i + 1]][
                np.abs(full.data[full.indptr[i]:full.indptr[i + 1]]) >= tr * mx])
            got = set(P.indices[P.indptr[i]:P.indptr[i + 1]])
            assert got == expect, (tr, i)
            if abs(fr.sum()) > 1e-12:
                assert abs(pr.sum() - fr.sum()) <= 1e-12 * np.abs(fr).sum()
            if tr == 0.0:
                assert np.array_equal(pr, fr)
        for i in np.flatnonzero(C)[::11]:
            assert P[i].nnz == 1 and P[i].data[0] == 1.0


def test_truncated_reduction_keeps_convergence():
    """Dropping small reduction-level weights (trunc0 = 0.05) thins the reduced
    operator but leaves the per-subsystem cycle's PCG iteration count within
    one of the untruncated cycle's."""
    p = make_problem((24, 24, 24), s=3, m=1, seed=5, y_stretch=1.5)
    res = {}
    for tr in (0.0, 0.05):
        ctx = krylov.setup(p.A, p.img, amg.AMGOptions(coarse_max=64, trunc0=tr), precond="amgr_sub")
        r = krylov.solve(ctx, p.b, tol=1e-10)
        res[tr] = (int(r.iters.max()), ctx["hier"].levels[1].A.nnz)
    assert res[0.05][1] < res[0.0][1]
    assert res[0.05][0] <= res[0.0][0] + 1


# ----------------------------------------------------------------- nu1 / nu2 sweeps (Alg. 3)

def test_two_grid_with_two_sweeps_matches_error_propagation():
    """Two levels, nu1 = nu2 = 2: I - V A = (I - M A)^2 (I - P A_c^{-1} P^T A) (I - M A)^2,
    for the shared cycle and for the per-subsystem cycle."""
    hier, sigma, Ahat, opt = _sub(coarse_max=200)
    opt2 = dataclasses.replace(opt, nu1=2, nu2=2)
    # shared cycle on A_inn with its interface
    p = make_problem((12, 12, 12), s=3, seed=4)
    Hb = symmetry.base_blocks(p.A, p.img)
    Ainn, _ = symmetry.inner_outer(Hb)
    iface = symmetry.interface_rows(Hb)
    Hs = amg.build_hierarchy(Ainn.tocsr(), iface, opt2)
    assert Hs.nlev == 2 and Hs.nu1 == 2
    L0 = Hs.levels[0]
    n = L0.A.shape[0]
    I = np.eye(n)
    Ad = L0.A.toarray()
    P = L0.P.toarray()
    M = L0.omega * L0.G.toarray().T @ L0.G.toarray()
    V = np.column_stack([amg.vcycle(Hs, e) for e in I])
    S = (I - M @ Ad) @ (I - M @ Ad)
    E = S @ (I - P @ np.linalg.solve(P.T @ Ad @ P, P.T @ Ad)) @ S
    assert np.abs((I - V @ Ad) - E).max() < 1e-10
    # one sweep fewer on either side is a different operator
    S1 = I - M @ Ad
    assert np.abs((I - V @ Ad) - S1 @ (I - P @ np.linalg.solve(P.T @ Ad @ P, P.T @ Ad)) @ S).max() > 1e-3
    SH = amg.build_sub_hierarchy(hier, sigma, opt2)
    G = hier.levels[0].G.toarray()
    Mh = hier.levels[0].omega * G.T @ G
    Ph = hier.levels[0].P.toarray()
    Ih = np.eye(Ph.shape[0])
    for a in (0, 5):
        Aa = Ahat[a].toarray()
        Va = np.column_stack([amg.vcycle_sub(SH, Ahat[a], a, e) for e in Ih])
        Sa = (Ih - Mh @ Aa) @ (Ih - Mh @ Aa)
        Ea = Sa @ (Ih - Ph @ np.linalg.solve(Ph.T @ Aa @ Ph, Ph.T @ Aa)) @ Sa
        assert np.abs((Ih - Va @ Aa) - Ea).max() < 1e-10


def test_symmetric_sweeps_keep_the_cycle_symmetric_and_help_pcg():
    """V(2,2) on three or more levels is symmetric positive definite, and PCG
    needs no more iterations with it than with V(1,1)."""
    A, iface = _inner((10, 10, 10))
    opt1 = amg.AMGOptions(coarse_max=20)
    opt2 = dataclasses.replace(opt1, nu1=2, nu2=2)
    H1 = amg.build_hierarchy(A, iface, opt1)
    H2 = amg.build_hierarchy(A, iface, opt2)
    assert H2.nlev >= 3
    I = np.eye(A.shape[0])
    V = np.column_stack([amg.vcycle(H2, e) for e in I])
    assert np.abs(V - V.T).max() <= 1e-12 * np.abs(V).max()
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0
    b = np.random.default_rng(3).standard_normal((A.shape[0], 1))
    thr = 1e-10 * np.linalg.norm(b, axis=0)
    r1 = krylov.pcg_columns(lambda X: A @ X, lambda R: amg.vcycle(H1, R), b, thr, 200)
    r2 = krylov.pcg_columns(lambda X: A @ X, lambda R: amg.vcycle(H2, R), b, thr, 200)
    assert r2.converged.all() and r2.iters.max() <= r1.iters.max()
