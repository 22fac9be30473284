"""Sec. 3.2 of the paper: the multigrid-reduction hierarchy (AMGR) built on
the shared inner block A_inn, and its V-cycle (Alg. 3).

Readings taken where the paper names a method without defining it (each is
listed with its reason in the design notes):
  * strength: classical, S_i = {j != i : -a_ij >= theta * max_{l != i} -a_il},
    symmetrised to the graph T = S u S^T (Alg. 2, first two steps);
  * "maximum independent set" = the lexicographically-first maximal
    independent set under hash priorities (Alg. 2, fourth step);
  * level 0 (the reduction): independent set of T^d taken inside the inner
    (non-interface) nodes, coarse set = MIS u interface (Alg. 2, last step);
    levels >= 1: independent set of T (distance 1) with PMIS-style priorities
    (number of strong dependants, then hash);
  * interpolation: the ideal interpolation -A_FF^{-1} A_FC truncated after a
    few Jacobi steps, with symbolic patterns, rows rescaled to the direct
    interpolation row sum; P = [W; I] (eq. (3.13));
  * smoother: static-pattern FSAI, block-diagonal over F/C at level 0
    (eq. (3.14)), damped by 4/(3 lambda_max(G A G^T));
  * reduced operator A_c = P^T A P (eq. (3.15)), symbolic pattern;
  * coarsest level: dense Cholesky.
Options for the methods the experiments use (Sec. 5: an adaptive FSAI
smoother with five entries per row, energy minimisation of the
interpolation), which the paper cites without defining:
  * afsai_nnz > 0: the FSAI pattern grown row by row by the greedy search of
    adaptive FSAI (largest decrease of the row's quadratic form per added
    entry), then the static FSAI on it;
  * emin_steps > 0: every interpolation refined by projected, Jacobi-
    preconditioned conjugate gradients on tr(P^T A P) with its pattern and
    row sums fixed.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .splitmix import splitmix64, unit_centered


# ---------------------------------------------------------------------------
# sparse helpers (structure-preserving)
# ---------------------------------------------------------------------------

def _ones_like(A: sp.csr_matrix) -> sp.csr_matrix:
    return sp.csr_matrix((np.ones(A.nnz), A.indices.copy(), A.indptr.copy()), shape=A.shape)


def _keys(A: sp.csr_matrix) -> np.ndarray:
    rows = np.repeat(np.arange(A.shape[0], dtype=np.int64), np.diff(A.indptr))
    return rows * np.int64(A.shape[1]) + A.indices.astype(np.int64)


def embed(values: sp.csr_matrix, pattern: sp.csr_matrix) -> sp.csr_matrix:
    """Return a matrix with the structure of ``pattern`` holding the entries
    of ``values`` (absent entries become explicit zeros).  Requires
    structure(values) to be a subset of structure(pattern)."""
    values = values.tocsr()
    values.sort_indices()
    pattern = pattern.tocsr()
    pattern.sort_indices()
    kp = _keys(pattern)
    kv = _keys(values)
    pos = np.searchsorted(kp, kv)
    if kv.size and (pos.max() >= kp.size or np.any(kp[pos] != kv)):
        raise AssertionError("values outside the symbolic pattern")
    data = np.zeros(pattern.nnz)
    data[pos] = values.data
    return sp.csr_matrix((data, pattern.indices.copy(), pattern.indptr.copy()), shape=pattern.shape)


def sym_matmul(A: sp.csr_matrix, B: sp.csr_matrix) -> sp.csr_matrix:
    """A @ B with the *structural* pattern (every reachable (i, j) is kept,
    exact cancellations included as explicit zeros)."""
    pat = (_ones_like(A) @ _ones_like(B)).tocsr()
    val = (A @ B).tocsr()
    return embed(val, pat)


def sym_add(A: sp.csr_matrix, B: sp.csr_matrix) -> sp.csr_matrix:
    pat = (_ones_like(A) + _ones_like(B)).tocsr()
    val = (A + B).tocsr()
    val.eliminate_zeros()
    return embed(val, pat)


def lookup(A: sp.csr_matrix, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """A[rows, cols] elementwise (0 where not stored); A sorted CSR."""
    k = _keys(A)
    q = rows.astype(np.int64) * np.int64(A.shape[1]) + cols.astype(np.int64)
    pos = np.searchsorted(k, q)
    pos = np.minimum(pos, k.size - 1)
    hit = k[pos] == q
    out = np.where(hit, A.data[pos], 0.0)
    return out


# ---------------------------------------------------------------------------
# Alg. 2 steps 1-2: strength of connection and the filtered graph T
# ---------------------------------------------------------------------------

def strength(A: sp.csr_matrix, theta: float) -> sp.csr_matrix:
    """Classical strength: j in S_i iff j != i and -a_ij >= theta*max_{l!=i}(-a_il);
    S_i is empty when that maximum is <= 0.  Returns a 0/1 CSR matrix S
    with S[i, j] = 1 for j in S_i.  theta*max is one FP64 multiply and the
    comparison is exact."""
    A = A.tocsr()
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    off = A.indices != rows
    neg = -A.data
    negoff = np.where(off, neg, -np.inf)
    mx = np.full(n, -np.inf)
    np.maximum.at(mx, rows, negoff)
    thr = theta * mx
    strong = off & (mx[rows] > 0) & (neg >= thr[rows])
    S = sp.csr_matrix((np.ones(int(strong.sum())), (rows[strong], A.indices[strong])), shape=(n, n))
    S.sort_indices()
    return S


def symmetrise(S: sp.csr_matrix) -> sp.csr_matrix:
    """T = S u S^T as a 0/1 matrix."""
    T = (_ones_like(S) + _ones_like(S).T).tocsr()
    T.data[:] = 1.0
    T.sort_indices()
    return T


def distance_graph(T: sp.csr_matrix, d: int) -> sp.csr_matrix:
    """Symbolic power: i ~ j iff 1 <= dist_T(i, j) <= d (Alg. 2, step 3)."""
    n = T.shape[0]
    I = sp.identity(n, format="csr")
    R = (I + _ones_like(T)).tocsr()
    Rk = R.copy()
    for _ in range(d - 1):
        Rk = (Rk @ R).tocsr()
    Rk.data[:] = 1.0
    Rk = Rk - sp.diags(Rk.diagonal())
    Rk = Rk.tocsr()
    Rk.eliminate_zeros()
    Rk.sort_indices()
    return Rk


# ---------------------------------------------------------------------------
# Alg. 2 step 4: independent sets
# ---------------------------------------------------------------------------

def mis_greedy(G: sp.csr_matrix, rank: np.ndarray) -> np.ndarray:
    """Lexicographically-first maximal independent set of graph G under
    decreasing ``rank`` (distinct integers): scan the nodes by decreasing rank
    and take a node when none of its neighbours has been taken.  Pure Python
    loop; for small graphs."""
    n = G.shape[0]
    taken = np.zeros(n, dtype=bool)
    for i in np.argsort(-np.asarray(rank, dtype=np.int64), kind="stable"):
        nb = G.indices[G.indptr[i]:G.indptr[i + 1]]
        if not taken[nb].any():
            taken[i] = True
    return taken


def mis_rounds(G: sp.csr_matrix, rank: np.ndarray) -> np.ndarray:
    """The same set by rounds: every undecided node whose rank beats all its
    undecided neighbours is taken, then its undecided neighbours are removed.
    Adjacency stays that of the fixed graph G (removal does not shorten or
    lengthen any distance)."""
    n = G.shape[0]
    rank = np.asarray(rank, dtype=np.int64)
    state = np.zeros(n, dtype=np.int8)      # 0 undecided, 1 taken, -1 removed
    rows = np.repeat(np.arange(n), np.diff(G.indptr))
    cols = G.indices
    while np.any(state == 0):
        und = state == 0
        live = und[rows] & und[cols]
        best = np.full(n, -1, dtype=np.int64)
        np.maximum.at(best, rows[live], rank[cols[live]])
        sel = und & (rank > best)
        state[sel] = 1
        nb = cols[sel[rows]]
        nb = nb[state[nb] == 0]
        state[nb] = -1
    return state == 1


def priorities_level0(n: int, seed: int) -> np.ndarray:
    """Hash priorities pi_i = splitmix64(seed xor i)."""
    return splitmix64(np.uint64(seed) ^ np.arange(n, dtype=np.uint64))


def priorities_coarse(S: sp.csr_matrix, level: int, seed: int) -> np.ndarray:
    """PMIS-style priorities: (#{j : i in S_j}, splitmix64(seed xor (level<<40)
    xor i)) compared lexicographically; returned as dense ranks (int64)."""
    n = S.shape[0]
    lam = np.asarray(_ones_like(S).sum(axis=0)).ravel().astype(np.int64)
    h = splitmix64(np.uint64(seed) ^ (np.uint64(level) << np.uint64(40)) ^ np.arange(n, dtype=np.uint64))
    order = np.lexsort((h, lam))            # increasing (lam, h)
    rank = np.empty(n, dtype=np.int64)
    rank[order] = np.arange(n)
    return rank


def coarsen_level0(A: sp.csr_matrix, interface: np.ndarray, theta: float, d: int, seed: int,
                   method: str = "rounds") -> np.ndarray:
    """Alg. 2 (populated coarsening at interpolation distance d): coarse set
    = MIS(T^d restricted to inner nodes) disjoint-union interface.  Returns a
    boolean C mask."""
    n = A.shape[0]
    S = strength(A, theta)
    T = symmetrise(S)
    inner = np.flatnonzero(~interface)
    Tin = T[inner][:, inner].tocsr()
    Gd = distance_graph(Tin, d)
    pri = priorities_level0(n, seed)[inner]
    rank = np.empty(inner.size, dtype=np.int64)
    rank[np.argsort(pri)] = np.arange(inner.size)
    mis = mis_greedy(Gd, rank) if method == "greedy" else mis_rounds(Gd, rank)
    C = interface.copy()
    C[inner[mis]] = True
    return C


def coarsen_standard(A: sp.csr_matrix, level: int, theta: float, seed: int,
                     method: str = "rounds") -> np.ndarray:
    """Levels below the reduction: C = MIS of T (distance 1)."""
    S = strength(A, theta)
    T = symmetrise(S)
    rank = priorities_coarse(S, level, seed)
    return mis_greedy(T, rank) if method == "greedy" else mis_rounds(T, rank)


# ---------------------------------------------------------------------------
# interpolation, P = [W; I] (eq. (3.13))
# ---------------------------------------------------------------------------

def interpolation(A: sp.csr_matrix, C: np.ndarray, steps: int, trunc: float = 0.0,
                  keep_pattern: Optional[sp.csr_matrix] = None) -> sp.csr_matrix:
    """Jacobi-truncated ideal interpolation (parity reading of the cited long
    distance schemes): W1 = -D^{-1} A_FC, W_{t+1} = -D^{-1}(A_FC + O W_t) with
    D = diag(A_FF), O = A_FF - D, symbolic patterns.  With trunc > 0 every F
    row keeps only the weights with |w| >= trunc * max |w| of the row (the
    others leave the pattern); with ``keep_pattern`` (an n x n_c matrix, the
    P of an earlier setup) every F row keeps exactly the weights on that
    pattern instead.  Each F row with nonzero sum is then rescaled to
    rho_i = -sum_{l != i} a_il / a_ii.  Returns P (n x n_c), coarse unknowns
    numbered by increasing fine index."""
    A = A.tocsr()
    n = A.shape[0]
    F = ~C
    fidx = np.flatnonzero(F)
    cidx = np.flatnonzero(C)
    nc = cidx.size
    AF = A[fidx].tocsr()
    AFF = AF[:, fidx].tocsr()
    AFC = AF[:, cidx].tocsr()
    AFF.sort_indices()
    AFC.sort_indices()
    Dv = AFF.diagonal()
    Dinv = sp.diags(1.0 / Dv)
    # O = A_FF without its diagonal (structure of the off-diagonal part)
    rows = np.repeat(np.arange(fidx.size), np.diff(AFF.indptr))
    keep = AFF.indices != rows
    O = sp.csr_matrix((AFF.data[keep], (rows[keep], AFF.indices[keep])), shape=AFF.shape)
    O.sort_indices()
    W = embed(-(Dinv @ AFC), AFC)
    for _ in range(steps - 1):
        inner = sym_add(AFC, sym_matmul(O, W))
        W = embed(-(Dinv @ inner), inner)
    if keep_pattern is not None:
        Kp = keep_pattern.tocsr()[fidx].tocsr()
        nrow = np.diff(W.indptr)
        rows_w = np.repeat(np.arange(W.shape[0]), nrow)
        rows_k = np.repeat(np.arange(Kp.shape[0]), np.diff(Kp.indptr))
        keep = np.isin(rows_w * nc + W.indices, rows_k * nc + Kp.indices)
        kept = np.bincount(rows_w[keep], minlength=W.shape[0])
        W = sp.csr_matrix((W.data[keep], W.indices[keep], np.concatenate([[0], np.cumsum(kept)])), shape=W.shape)
    elif trunc > 0.0:
        nrow = np.diff(W.indptr)
        rmax = np.zeros(W.shape[0])
        np.maximum.at(rmax, np.repeat(np.arange(W.shape[0]), nrow), np.abs(W.data))
        keep = np.abs(W.data) >= trunc * np.repeat(rmax, nrow)
        rows_w = np.repeat(np.arange(W.shape[0]), nrow)
        kept = np.bincount(rows_w[keep], minlength=W.shape[0])
        W = sp.csr_matrix((W.data[keep], W.indices[keep], np.concatenate([[0], np.cumsum(kept)])), shape=W.shape)
    # row rescaling to the direct-interpolation row sum
    diagA = A.diagonal()
    rowsA = np.repeat(np.arange(n), np.diff(A.indptr))
    offsum = np.zeros(n)
    np.add.at(offsum, rowsA[A.indices != rowsA], A.data[A.indices != rowsA])
    rho = -offsum[fidx] / diagA[fidx]
    wsum = np.asarray(W.sum(axis=1)).ravel()
    scale = np.where(wsum != 0.0, rho / np.where(wsum != 0.0, wsum, 1.0), 1.0)
    W = sp.csr_matrix((W.data * np.repeat(scale, np.diff(W.indptr)), W.indices, W.indptr), shape=W.shape)
    # assemble P in fine-row order
    cnum = -np.ones(n, dtype=np.int64)
    cnum[cidx] = np.arange(nc)
    prow = []
    pcol = []
    pval = []
    Wr = np.repeat(fidx, np.diff(W.indptr))
    prow.append(Wr)
    pcol.append(W.indices.astype(np.int64))
    pval.append(W.data)
    prow.append(cidx)
    pcol.append(np.arange(nc))
    pval.append(np.ones(nc))
    prow = np.concatenate(prow)
    pcol = np.concatenate(pcol)
    pval = np.concatenate(pval)
    order = np.lexsort((pcol, prow))
    counts = np.bincount(prow, minlength=n)
    indptr = np.concatenate([[0], np.cumsum(counts)])
    P = sp.csr_matrix((pval[order], pcol[order], indptr), shape=(n, nc))
    return P


def galerkin(A: sp.csr_matrix, P: sp.csr_matrix) -> sp.csr_matrix:
    """Reduced operator A_c = P^T A P (eq. (3.15)), symbolic pattern,
    computed as R (A P) with R = P^T."""
    R = P.T.tocsr()
    R.sort_indices()
    AP = sym_matmul(A, P)
    return sym_matmul(R, AP)


# ---------------------------------------------------------------------------
# FSAI smoother (eq. (2.17) factor; block form eq. (3.14))
# ---------------------------------------------------------------------------

def fsai_pattern(S: sp.csr_matrix, block: np.ndarray):
    """Row patterns J_i = {j < i : j in S_i, block_j == block_i} + [i], sorted."""
    n = S.shape[0]
    pats = []
    for i in range(n):
        nb = S.indices[S.indptr[i]:S.indptr[i + 1]]
        nb = nb[(nb < i) & (block[nb] == block[i])]
        pats.append(np.concatenate([np.sort(nb), [i]]).astype(np.int64))
    return pats


def fsai(A: sp.csr_matrix, S: sp.csr_matrix, block: np.ndarray) -> sp.csr_matrix:
    """Static-pattern factorised sparse approximate inverse: for each row i,
    solve A[J_i, J_i] g = e_last and scale g by 1/sqrt(g_last), so that
    G A G^T has unit diagonal and G^T G ~ A^{-1}.  Rows are grouped by
    pattern size and solved with batched dense solves."""
    A = A.tocsr()
    A.sort_indices()
    n = A.shape[0]
    # vectorised pattern construction
    rows = np.repeat(np.arange(n), np.diff(S.indptr))
    cols = S.indices
    keep = (cols < rows) & (block[cols] == block[rows])
    pr = np.concatenate([rows[keep], np.arange(n)])
    pc = np.concatenate([cols[keep], np.arange(n)])
    order = np.lexsort((pc, pr))
    pr, pc = pr[order], pc[order]
    counts = np.bincount(pr, minlength=n)
    indptr = np.concatenate([[0], np.cumsum(counts)])
    gval = np.empty(pr.size)
    for k in np.unique(counts):
        rws = np.flatnonzero(counts == k)
        J = pc[indptr[rws][:, None] + np.arange(k)[None, :]]       # (nr, k), last = i
        M = lookup(A, np.repeat(J, k, axis=1).ravel(), np.tile(J, (1, k)).ravel()).reshape(-1, k, k)
        e = np.zeros((rws.size, k))
        e[:, -1] = 1.0
        g = np.linalg.solve(M, e[:, :, None])[:, :, 0]
        g = g / np.sqrt(g[:, -1:])
        gval[indptr[rws][:, None] + np.arange(k)[None, :]] = g
    G = sp.csr_matrix((gval, pc, indptr), shape=(n, n))
    return G


# Scores within this relative distance of the best are ties (broken by the
# smaller column), so that rounding differences between implementations do
# not change the pattern.
AFSAI_TIE = 1e-10


def afsai_pattern(A: sp.csr_matrix, block: np.ndarray, nnz_max: int) -> sp.csr_matrix:
    """Adaptive FSAI pattern (greedy pattern search of adaptive FSAI).  Row i
    starts from P_i = {i}.  Each step takes the row g with g_i = 1 and support
    P_i that minimises g^T A g, forms r = A g, and adds the candidate
    j < i outside P_i with block_j == block_i and r_j != 0 whose score
    r_j^2 / a_jj is largest: the decrease of g^T A g that a step along e_j
    alone achieves, a lower bound of the decrease after re-minimising.  Scores
    within AFSAI_TIE of the best tie to the smaller column.  A row stops at
    nnz_max entries or when no candidate has a positive score.  All rows take
    their steps together: r for every row is one sparse product (rows of the
    current g's times A, A symmetric), and the rows still growing all hold
    the same number of entries, so their re-minimisations are one batched
    solve.  Returns the lower pattern (diagonal included) as a CSR matrix of
    ones."""
    A = A.tocsr()
    A.sort_indices()
    n = A.shape[0]
    d = A.diagonal()
    pat = np.full((n, max(nnz_max, 1)), -1, dtype=np.int64)    # entries in the order they joined
    pat[:, 0] = np.arange(n)
    g = np.zeros((n, max(nnz_max, 1)))
    g[:, 0] = 1.0
    active = np.arange(n)
    for t in range(1, nnz_max):
        if active.size == 0:
            break
        # r = (rows of g) A for the active rows
        Gr = sp.csr_matrix((g[active, :t].ravel(), pat[active, :t].ravel(),
                            np.arange(0, (active.size + 1) * t, t)), shape=(active.size, n))
        R = (Gr @ A).tocsr()
        R.sort_indices()
        rr = np.repeat(np.arange(active.size), np.diff(R.indptr))
        rows = active[rr]
        cols = R.indices
        inpat = np.zeros(cols.size, dtype=bool)
        for q in range(t):
            inpat |= pat[rows, q] == cols
        ok = (cols < rows) & (block[cols] == block[rows]) & ~inpat & (R.data != 0.0)
        score = np.where(ok, R.data * R.data / d[cols], -1.0)
        best = np.full(active.size, -1.0)
        np.maximum.at(best, rr, score)
        pick = np.full(active.size, -1, dtype=np.int64)
        take = ok & (score >= best[rr] * (1.0 - AFSAI_TIE)) & (best[rr] > 0.0)
        # columns of a row are ascending: the first qualifying entry is the smallest column
        first = np.flatnonzero(take)
        first = first[np.concatenate([[True], rr[first][1:] != rr[first][:-1]])] if first.size else first
        pick[rr[first]] = cols[first]
        grow = pick >= 0
        active = active[grow]
        if active.size == 0:
            break
        pat[active, t] = pick[grow]
        # re-minimise on Q = P \ {i}: A[Q, Q] y = -A[Q, i]
        Q = pat[active, 1:t + 1]
        M = lookup(A, np.repeat(Q, t, axis=1).ravel(), np.tile(Q, (1, t)).ravel()).reshape(-1, t, t)
        rhs = -lookup(A, Q.ravel(), np.repeat(active, t)).reshape(-1, t)
        y = np.linalg.solve(M, rhs[:, :, None])[:, :, 0]
        g[active, 0] = 1.0
        g[active, 1:t + 1] = y
    keep = pat >= 0
    S = sp.csr_matrix((np.ones(int(keep.sum())), (np.repeat(np.arange(n), keep.sum(axis=1)), pat[keep])),
                      shape=(n, n))
    S.sort_indices()
    return S


def emin(A: sp.csr_matrix, C: np.ndarray, P: sp.csr_matrix, steps: int) -> sp.csr_matrix:
    """Energy-minimising interpolation: minimise tr(P^T A P) over the F rows W
    of P = [W; I] on W's pattern with every row sum of W kept (P keeps what it
    gives for the coarse constant), by `steps` conjugate-gradient steps
    started at W.  The objective's half gradient is A_FF W + A_FC on the
    pattern; the constraint's tangent space is {D : every row of D sums to
    0} (orthogonal projection: subtract the row mean over the row's pattern);
    the preconditioner divides row f by a_ff, which maps that space to
    itself."""
    A = A.tocsr()
    A.sort_indices()
    n = A.shape[0]
    fidx = np.flatnonzero(~C)
    cidx = np.flatnonzero(C)
    AF = A[fidx].tocsr()
    AFF = AF[:, fidx].tocsr()
    AFC = AF[:, cidx].tocsr()
    W = P.tocsr()[fidx].tocsr()
    W.sort_indices()
    cnt = np.diff(W.indptr)
    wr = np.repeat(np.arange(fidx.size), cnt)
    wc = W.indices
    dinv = 1.0 / AFF.diagonal()[wr]

    def on_pattern(M):
        M = M.tocsr()
        M.sort_indices()
        return lookup(M, wr, wc)

    def project(v):
        s = np.zeros(fidx.size)
        np.add.at(s, wr, v)
        return v - (s / np.maximum(cnt, 1))[wr]

    def mat(v):
        return sp.csr_matrix((v, wc, W.indptr), shape=W.shape)

    w = W.data.copy()
    r = -project(on_pattern(AFF @ mat(w) + AFC))
    z = dinv * r
    p = z.copy()
    rz = float(r @ z)
    for _ in range(steps):
        if not rz > 0.0:
            break
        q = project(on_pattern(AFF @ mat(p)))
        pq = float(p @ q)
        if not pq > 0.0:
            break
        alpha = rz / pq
        w = w + alpha * p
        r = r - alpha * q
        z = dinv * r
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    Pn = P.tocsr().copy()
    Pn.sort_indices()
    frows = np.repeat(np.arange(n), np.diff(Pn.indptr))
    isf = ~C[frows]
    Pn.data[isf] = w        # F entries of P in fine-row order are W's entries in order
    return Pn


def damping(A: sp.csr_matrix, G: sp.csr_matrix, seed: int, iters: int = 20) -> float:
    """omega = 4 / (3 lam), lam from `iters` power iterations on G A G^T started
    at v_i = splitmix64(seed xor i)/2^64 - 1/2; lam is the Rayleigh quotient
    v^T (G A G^T) v of the last normalised iterate."""
    n = A.shape[0]
    v = unit_centered(np.uint64(seed) ^ np.arange(n, dtype=np.uint64))
    v = v / np.linalg.norm(v)
    lam = 0.0
    GT = G.T.tocsr()
    for _ in range(iters):
        w = G @ (A @ (GT @ v))
        lam = float(v @ w)
        v = w / np.linalg.norm(w)
    return 4.0 / (3.0 * lam)


# ---------------------------------------------------------------------------
# hierarchy and V-cycle (Alg. 3)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Level:
    A: sp.csr_matrix
    C: Optional[np.ndarray] = None
    P: Optional[sp.csr_matrix] = None
    R: Optional[sp.csr_matrix] = None
    G: Optional[sp.csr_matrix] = None
    omega: float = 0.0


@dataclasses.dataclass
class Hierarchy:
    levels: List[Level]
    coarse_factor: tuple = None        # cho_factor of the coarsest matrix
    nu1: int = 1                       # pre- and post-smoothing sweeps of Alg. 3
    nu2: int = 1

    @property
    def nlev(self):
        return len(self.levels)

    def stats(self):
        rows = [L.A.shape[0] for L in self.levels]
        nnz = [L.A.nnz for L in self.levels]
        return dict(rows=rows, nnz=nnz, op_complexity=sum(nnz) / nnz[0],
                    c_rat=(rows[1] / rows[0]) if len(rows) > 1 else 1.0,
                    avg_nnzr=(nnz[1] / rows[1]) if len(rows) > 1 else nnz[0] / rows[0])


@dataclasses.dataclass
class AMGOptions:
    theta: float = 0.25
    dist: int = 2
    jacobi0: int = 3          # interpolation steps at the reduction level
    trunc0: float = 0.05      # relative weight truncation at the reduction level (0 = none)
    jacobi: int = 1           # interpolation steps below it
    coarse_max: int = 2560
    max_levels: int = 20
    max_ratio: float = 0.8
    seed: int = 240705930
    mis_method: str = "rounds"
    nu1: int = 1              # smoothing sweeps before and after the coarse correction (Alg. 3)
    nu2: int = 1
    afsai_nnz: int = 0        # > 0: adaptive FSAI pattern with at most this many entries per row
    emin_steps: int = 0       # > 0: energy minimisation of every interpolation, this many CG steps


def build_hierarchy(Ainn: sp.csr_matrix, interface: np.ndarray, opt: AMGOptions,
                    coarse0: Optional[np.ndarray] = None) -> Hierarchy:
    """AMGR on the shared inner block: level 0 is the multigrid reduction of
    Sec. 3.2 (Alg. 2 coarsening with the interface forced coarse, P = [W; I],
    block-FSAI smoother), levels below are standard AMG on the reduced
    operator, the last level is solved densely.  ``coarse0``: a level-0
    coarse set computed elsewhere (the populated interface of a domain of
    copies), used instead of Alg. 2 on this matrix."""
    A = Ainn.tocsr()
    A.sort_indices()
    return _levels_from([], A, 0, interface, opt, coarse0)


def build_hierarchy_below(H: Hierarchy, opt: AMGOptions) -> Hierarchy:
    """H's reduction level as it is (split, patterns, values), and every level
    below it built afresh from H's level-1 operator exactly as build_hierarchy
    builds the levels below the reduction level."""
    if H.nlev < 2:
        raise ValueError("no level below the reduction level")
    return _levels_from([H.levels[0]], H.levels[1].A, 1, None, opt, None)


def _levels_from(levels: list, A: sp.csr_matrix, lev: int, interface, opt: AMGOptions,
                 coarse0: Optional[np.ndarray]) -> Hierarchy:
    """The loop of build_hierarchy from level ``lev`` (operator A) down,
    appended to ``levels``."""
    while True:
        L = Level(A=A)
        levels.append(L)
        n = A.shape[0]
        if n <= opt.coarse_max or lev == opt.max_levels - 1:
            break
        if lev == 0 and coarse0 is not None:
            C = np.asarray(coarse0, dtype=bool).copy()
            steps, trunc = opt.jacobi0, opt.trunc0
        elif lev == 0:
            C = coarsen_level0(A, interface, opt.theta, opt.dist, opt.seed, opt.mis_method)
            steps, trunc = opt.jacobi0, opt.trunc0
        else:
            C = coarsen_standard(A, lev, opt.theta, opt.seed, opt.mis_method)
            steps, trunc = opt.jacobi, 0.0
        nc = int(C.sum())
        if nc == 0 or nc > opt.max_ratio * n:
            break
        S = strength(A, opt.theta)
        block = C.astype(np.int64) if lev == 0 else np.zeros(n, dtype=np.int64)
        L.C = C
        L.G = fsai(A, afsai_pattern(A, block, opt.afsai_nnz) if opt.afsai_nnz > 0 else S, block)
        L.omega = damping(A, L.G, opt.seed)
        L.P = interpolation(A, C, steps, trunc)
        if opt.emin_steps > 0:
            L.P = emin(A, C, L.P, opt.emin_steps)
        L.R = L.P.T.tocsr()
        L.R.sort_indices()
        A = galerkin(A, L.P)
        lev += 1
    Ad = levels[-1].A.toarray()
    factor = sla.cho_factor(Ad, lower=True)
    return Hierarchy(levels=levels, coarse_factor=factor, nu1=opt.nu1, nu2=opt.nu2)


def vcycle(H: Hierarchy, y: np.ndarray, lev: int = 0) -> np.ndarray:
    """Alg. 3 with smoother M = omega G^T G and nu1 / nu2 sweeps (H.nu1,
    H.nu2) on every level: s = M y, then nu1 - 1 times s += M (y - A s);
    r = y - A s; h_c = V(R r); s += P h_c; then nu2 times s += M (y - A s).
    ``y`` may hold several columns."""
    if lev == H.nlev - 1:
        return sla.cho_solve(H.coarse_factor, y)
    L = H.levels[lev]
    GT = L.G.T
    s = L.omega * (GT @ (L.G @ y))
    for _ in range(H.nu1 - 1):
        s = s + L.omega * (GT @ (L.G @ (y - L.A @ s)))
    r = y - L.A @ s
    hc = vcycle(H, L.R @ r, lev + 1)
    s = s + L.P @ hc
    for _ in range(H.nu2):
        s = s + L.omega * (GT @ (L.G @ (y - L.A @ s)))
    return s


# ---------------------------------------------------------------------------
# AMGR on the decoupled subsystems (Sec. 3.2 applied in the Q_s basis)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SubHierarchy:
    """Level 0 (the reduction) is shared by every subsystem: its C/F split
    forces the interface coarse, so P_0 = [W; I] is the same for all
    A_a = A_inn + diag(sigma_a) (sigma_a lives on interface rows only).  The
    reduced operators differ only on the interface diagonal:
    A_1,a = P_0^T A_a P_0 = A_1,inn + diag(sigma_a[C]).  Levels below are
    built for every subsystem from its own A_1,a, with the C/F splits and
    smoother patterns of the shared hierarchy on A_inn (so all subsystems
    share one sparsity pattern per level) and each subsystem's own values."""
    level0: Level
    subs: List[Hierarchy]          # per subsystem: levels 1.. (coarsest dense)
    nu1: int = 1
    nu2: int = 1


def sub_level_values(A: sp.csr_matrix, shared: Level, steps: int, seed: int, level0: bool,
                     pattern: sp.csr_matrix | None = None, emin_steps: int = 0) -> Level:
    """One level for a subsystem operator A with the shared level's C/F split
    and FSAI pattern (the shared factor's, or the given lower-triangular
    ``pattern``: a kept one)."""
    n = A.shape[0]
    C = shared.C
    S = shared.G if pattern is None else pattern
    block = C.astype(np.int64) if level0 else np.zeros(n, dtype=np.int64)
    G = fsai(A, S, block)
    om = damping(A, G, seed)
    P = interpolation(A, C, steps)
    if emin_steps > 0:
        P = emin(A, C, P, emin_steps)
    R = P.T.tocsr()
    R.sort_indices()
    return Level(A=A, C=C, P=P, R=R, G=G, omega=om)


def build_sub_hierarchy(hier: Hierarchy, sigma: np.ndarray, opt: AMGOptions,
                        patterns: list | None = None) -> SubHierarchy:
    """sigma: (n_b, 2^s) outer diagonal.  hier: the shared AMGR hierarchy on
    A_inn (provides level 0 and the C/F splits and patterns below).
    ``patterns[lev]``: a kept FSAI pattern for level lev (None: from the
    strength of the shared level)."""
    L0 = hier.levels[0]
    cidx = np.flatnonzero(L0.C)
    subs = []
    for a in range(sigma.shape[1]):
        A = (hier.levels[1].A + sp.diags(sigma[cidx, a])).tocsr()
        A.sort_indices()
        levels = []
        for lev in range(1, hier.nlev):
            if lev == hier.nlev - 1:
                levels.append(Level(A=A))
                break
            Lv = sub_level_values(A, hier.levels[lev], opt.jacobi, opt.seed, False,
                                  None if patterns is None else patterns[lev], opt.emin_steps)
            levels.append(Lv)
            A = galerkin(A, Lv.P)
        fac = sla.cho_factor(levels[-1].A.toarray(), lower=True)
        subs.append(Hierarchy(levels=levels, coarse_factor=fac, nu1=opt.nu1, nu2=opt.nu2))
    return SubHierarchy(level0=L0, subs=subs, nu1=opt.nu1, nu2=opt.nu2)


def vcycle_sub(SH: SubHierarchy, Ahat_a: sp.csr_matrix, a: int, y: np.ndarray) -> np.ndarray:
    """Alg. 3 for subsystem a: level-0 smoother and transfers shared, the
    residual with the subsystem's own operator, the coarse correction by the
    subsystem's hierarchy."""
    L = SH.level0
    GT = L.G.T
    s = L.omega * (GT @ (L.G @ y))
    for _ in range(SH.nu1 - 1):
        s = s + L.omega * (GT @ (L.G @ (y - Ahat_a @ s)))
    r = y - Ahat_a @ s
    hc = vcycle(SH.subs[a], L.R @ r, 0)
    s = s + L.P @ hc
    for _ in range(SH.nu2):
        s = s + L.omega * (GT @ (L.G @ (y - Ahat_a @ s)))
    return s
