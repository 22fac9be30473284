"""Pins of the oracle's AMGR in the original basis for domains made of copies
(oracle/copies.py): the inner-interface structure of eq. (3.1), the
replicated populated interface of Alg. 2, P = [W; I] (eq. (3.13)), the
four-term reduced operator (eq. (3.15)), the symmetric V-cycle of Alg. 3,
and the solve against a sparse direct solve on repeated and reflected
domains whose boundary conditions differ between copies."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from gen import make_problem, make_repeated_problem
from oracle import amg, copies, symmetry


def _expected_interface(p, walls):
    """By hand: a base cell is interface when it touches a face between
    copies (x0 = 0 or x0 = N0 - 1 of a copy with neighbours on both sides),
    or, with the mixed walls, the low wall of axis 1 (insulated in odd
    copies) or the far wall of axis 0 (insulated in the last copy only)."""
    N = p.N
    idx = np.stack(np.meshgrid(*[np.arange(v) for v in N], indexing="ij"), axis=-1).reshape(-1, len(N))
    base = idx @ np.cumprod((1,) + N[:-1])
    x0, y0 = idx[:, 0], idx[:, 1]
    exp = (x0 == 0) | (x0 == N[0] - 1)
    if walls == "mixed":
        exp |= y0 == 0
    out = np.zeros(p.n_b, dtype=bool)
    out[base] = exp
    return out


@pytest.mark.parametrize("walls", ["dirichlet", "mixed"])
def test_interface_of_repeated_copies_is_the_hand_derived_set(walls):
    p = make_repeated_problem((6, 5, 4), 3, seed=1, walls=walls)
    assert np.array_equal(copies.interface_of_copies(p.A, p.sub), _expected_interface(p, walls))


def test_inner_blocks_of_every_copy_are_identical():
    """K-bar = I (x) K (eq. (3.1)): the inner-inner block of every copy, read in
    base numbering, equals the base copy's bit for bit, and inner unknowns of
    different copies are not coupled."""
    p = make_repeated_problem((6, 5, 4), 4, seed=2, walls="mixed", mirror=True)
    ifc = copies.interface_of_copies(p.A, p.sub)
    inner = np.flatnonzero(~ifc)
    K0 = copies.copy_block(p.A, p.sub, 0)[inner][:, inner]
    for a in range(p.copies):
        Ka = copies.copy_block(p.A, p.sub, a)[inner][:, inner]
        assert (Ka != K0).nnz == 0
    glob_inner = p.sub[inner].T.ravel()   # copy by copy
    blk = p.A[glob_inner][:, glob_inner].tocsr()
    ni = inner.size
    for a in range(p.copies):
        for b in range(p.copies):
            if a != b:
                assert blk[a * ni:(a + 1) * ni, b * ni:(b + 1) * ni].nnz == 0


def test_one_copy_is_the_plain_reduction_level():
    """A single copy has no interface: the hierarchy is amg.build_hierarchy of
    the whole matrix with an empty interface, level by level."""
    p = make_problem((12, 10, 8), s=0, seed=3, y_stretch=1.5)
    sub = np.arange(p.n, dtype=np.int64)[:, None]
    opt = amg.AMGOptions(coarse_max=40)
    ctx = copies.setup(p.A, sub, opt)
    assert not ctx["interface"].any()
    ref = amg.build_hierarchy(p.A.tocsr(), np.zeros(p.n, dtype=bool), opt)
    assert ctx["hier"].nlev == ref.nlev
    for L1, L2 in zip(ctx["hier"].levels, ref.levels):
        assert (L1.A != L2.A).nnz == 0
        if L2.C is not None:
            assert np.array_equal(L1.C, L2.C)
            assert (L1.P != L2.P).nnz == 0


def test_populated_interface_is_replicated_and_independent():
    """The coarse set (Alg. 2) holds the whole interface and the same inner
    base cells in every copy; those inner cells are a maximal independent set
    of T^2 restricted to the inner cells of the base copy."""
    p = make_repeated_problem((8, 7, 5), 3, seed=4, walls="mixed")
    opt = amg.AMGOptions(coarse_max=40)
    ctx = copies.setup(p.A, p.sub, opt)
    C = ctx["C"]
    Cb = C[p.sub]
    assert np.all(Cb == Cb[:, :1])
    assert np.all(C[ctx["interface"]])
    inner = np.flatnonzero(~ctx["interface_base"])
    A00 = copies.copy_block(p.A, p.sub, 0)
    T = amg.symmetrise(amg.strength(A00, opt.theta))[inner][:, inner].tocsr()
    G2 = amg.distance_graph(T, 2)
    mis = Cb[inner, 0]
    rows = np.repeat(np.arange(inner.size), np.diff(G2.indptr))
    assert not np.any(mis[rows] & mis[G2.indices])                 # independent
    covered = mis.copy()
    covered[G2.indices[mis[rows]]] = True
    assert np.all(covered)                                         # maximal


def test_prolongation_is_w_over_identity_and_repeats_away_from_the_interface():
    """P = [W-bar; I] (eq. (3.13)): a coarse row is a unit row.  An F row whose
    weights only reach inner coarse points of its own copy is the same row in
    every copy (the I (x) W part that an SpMM over the copies would apply)."""
    p = make_repeated_problem((8, 6, 5), 3, seed=5)
    ctx = copies.setup(p.A, p.sub, amg.AMGOptions(coarse_max=40))
    L0 = ctx["hier"].levels[0]
    P, C = L0.P.tocsr(), L0.C
    cnum = -np.ones(p.n, dtype=np.int64)
    cnum[np.flatnonzero(C)] = np.arange(int(C.sum()))
    for g in np.flatnonzero(C):
        row = P[g]
        assert row.nnz == 1 and row.indices[0] == cnum[g] and row.data[0] == 1.0
    copy_of, base_of = copies._index_maps(p.sub)
    fine_of_c = np.flatnonzero(C)
    inner_c = ~ctx["interface"][fine_of_c]
    checked = 0
    for i in np.flatnonzero(~ctx["interface_base"] & ~C[p.sub[:, 0]]):
        rows = [P[p.sub[i, a]] for a in range(p.copies)]
        if not all(np.all(inner_c[r.indices]) for r in rows):
            continue
        keys = [sorted(zip(base_of[fine_of_c[r.indices]].tolist(), r.data.tolist())) for r in rows]
        assert all(k == keys[0] for k in keys)
        checked += 1
    assert checked > 20


def test_reduced_operator_is_the_four_term_sum():
    """A_c = W^T K W + W^T B + B^T W + C (eq. (3.15)) with the F/C blocks of
    the level-0 split, against the Galerkin product the hierarchy holds."""
    p = make_repeated_problem((6, 6, 4), 3, seed=6, walls="mixed", mirror=True)
    ctx = copies.setup(p.A, p.sub, amg.AMGOptions(coarse_max=40))
    L0 = ctx["hier"].levels[0]
    F, C = np.flatnonzero(~L0.C), np.flatnonzero(L0.C)
    A = ctx["A"]
    K, B, Cb = A[F][:, F], A[F][:, C], A[C][:, C]
    W = L0.P.tocsr()[F]
    four = (W.T @ K @ W + W.T @ B + B.T @ W + Cb).toarray()
    Ac = ctx["hier"].levels[1].A.toarray()
    assert np.abs(four - Ac).max() <= 1e-12 * np.abs(Ac).max()


def test_vcycle_is_symmetric_positive_definite():
    p = make_repeated_problem((6, 5, 4), 3, seed=7, walls="mixed")
    ctx = copies.setup(p.A, p.sub, amg.AMGOptions(coarse_max=30))
    H = ctx["hier"]
    M = np.stack([amg.vcycle(H, e) for e in np.eye(p.n)], axis=1)
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


@pytest.mark.parametrize("shape", [
    dict(N=(8, 7, 6), copies=4, mirror=False, walls="mixed"),
    dict(N=(10, 9, 7), copies=2, mirror=True, walls="mixed"),
    dict(N=(24, 20), copies=5, mirror=False, walls="dirichlet"),
], ids=["repeated4_mixed", "mirrored2_mixed", "2d_repeated5"])
def test_solve_matches_direct_solve(shape):
    """PCG with AMGR in the original basis reaches the sparse direct
    solution; the reflected pair with walls that differ between its halves
    is a case the change of basis Q_s cannot take (its blocks are not
    mirror images), which the symmetry oracle confirms by rejecting it."""
    p = make_repeated_problem(shape["N"], shape["copies"], m=2, seed=8, mirror=shape["mirror"],
                              walls=shape["walls"])
    ctx = copies.setup(p.A, p.sub, amg.AMGOptions(coarse_max=40))
    res = copies.solve(ctx, p.b, tol=1e-12)
    ref = spla.splu(p.A.tocsc()).solve(p.b)
    assert np.linalg.norm(res.x - ref) <= 1e-9 * np.linalg.norm(ref)
    assert res.converged.all() and res.iters.max() < 40
    if shape["mirror"] and shape["copies"] == 2:
        with pytest.raises(Exception):
            symmetry.base_blocks(p.A, p.sub)
