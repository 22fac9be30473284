"""Sec. 2 of the paper: mirrored ordering, base blocks, the change of basis
Q_s and the decoupled subsystems; Alg. 1.

Conventions: ``img[i, a]`` is the row (in the caller's ordering) of image a of
base cell i; bit t of ``a`` means "reflected about mirror plane t", so images
compose by XOR.  The mirrored ordering puts image a's cells in block a
(rows a*n_b .. a*n_b + n_b - 1), as in eqs. (2.1) and (2.4)-(2.5).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def popcount(x):
    x = np.asarray(x, dtype=np.int64)
    c = np.zeros_like(x)
    while np.any(x):
        c += x & 1
        x = x >> 1
    return c


def hadamard(S: int) -> np.ndarray:
    """Sylvester Hadamard matrix, entries (-1)^popcount(a & b)."""
    a = np.arange(S)
    return np.where(popcount(a[:, None] & a[None, :]) % 2 == 0, 1.0, -1.0)


def mirrored_permutation(img: np.ndarray) -> np.ndarray:
    """perm[g_m] = caller row of mirrored row g_m = a*n_b + i."""
    n_b, S = img.shape
    return img.T.reshape(-1).astype(np.int64)


def to_mirrored(A: sp.csr_matrix, img: np.ndarray) -> sp.csr_matrix:
    """The matrix in mirrored ordering, A_m = A[perm][:, perm]."""
    perm = mirrored_permutation(img)
    Am = A[perm][:, perm].tocsr()
    Am.sort_indices()
    return Am


def check_map(img: np.ndarray, n: int) -> None:
    """The symmetry map must be a permutation of 0..n-1."""
    flat = np.sort(img.reshape(-1))
    if flat.size != n or not np.array_equal(flat, np.arange(n)):
        raise ValueError("symmetry map is not a permutation")


def base_blocks(A: sp.csr_matrix, img: np.ndarray):
    """Blocks H_j (eqs. (2.4)-(2.5) generalised): H_j couples the base mesh (image 0)
    with image j.  Checks, exactly, that block (a, b) of the mirrored matrix
    equals H_{a xor b} and that A is symmetric.  Exact zeros are dropped.
    Returns {j: csr (n_b x n_b)}."""
    n_b, S = img.shape
    check_map(img, A.shape[0])
    Am = to_mirrored(A, img)
    Am.eliminate_zeros()
    if (Am != Am.T).nnz:
        raise ValueError("matrix is not symmetric")
    H = {}
    for j in range(S):
        H[j] = Am[0:n_b, j * n_b:(j + 1) * n_b].tocsr()
        H[j].sort_indices()
    for a in range(S):
        for b in range(S):
            blk = Am[a * n_b:(a + 1) * n_b, b * n_b:(b + 1) * n_b].tocsr()
            if (blk != H[a ^ b]).nnz:
                raise ValueError(f"block ({a},{b}) differs from H_{a ^ b}")
    return H


def q_matrix(s: int, n_b: int) -> sp.csr_matrix:
    """Q_s of eq. (2.12): the product over i = 1..s of
    I_{2^{i-1}} (x) (1/sqrt2)[[1,1],[1,-1]] (x) I_{n/2^i}.  Written out as
    that product of sparse factors."""
    n = n_b << s
    Q = sp.identity(n, format="csr")
    h2 = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)
    for i in range(1, s + 1):
        F = sp.kron(sp.kron(sp.identity(1 << (i - 1)), sp.csr_matrix(h2)),
                    sp.identity(n >> i), format="csr")
        Q = (Q @ F).tocsr()
    return Q


def subsystem(H: dict, a: int) -> sp.csr_matrix:
    """Diagonal block a of Q_s A Q_s^{-1}: sum_j (-1)^popcount(a & j) H_j.
    (Block (a, b) of A is H_{a xor b}; Q_s = 2^{-s/2} Had (x) I.)"""
    out = None
    for j, Hj in H.items():
        sign = -1.0 if popcount(a & j) % 2 else 1.0
        term = sign * Hj
        out = term if out is None else out + term
    out = out.tocsr()
    out.sort_indices()
    return out


def inner_outer(H: dict):
    """Splitting of eq. (2.14): A_inn = H_0 shared by all subsystems and the
    per-subsystem outer parts A_out,a = sum_{j != 0} (-1)^popcount(a&j) H_j.
    Returns (A_inn, [A_out,a for a in 0..2^s-1])."""
    S = len(H)
    Ainn = H[0].tocsr()
    outs = []
    for a in range(S):
        acc = sp.csr_matrix(Ainn.shape)
        for j in range(1, S):
            sign = -1.0 if popcount(a & j) % 2 else 1.0
            acc = acc + sign * H[j]
        outs.append(acc.tocsr())
    return Ainn, outs


def interface_rows(H: dict) -> np.ndarray:
    """Boolean mask of base cells coupled to another subdomain (Sec. 3: the
    interface unknowns): rows with a nonzero entry in some H_j, j != 0."""
    n_b = H[0].shape[0]
    mask = np.zeros(n_b, dtype=bool)
    for j, Hj in H.items():
        if j == 0:
            continue
        nz = np.diff(Hj.indptr) > 0
        mask |= nz
    return mask


def forward_transform(b: np.ndarray, img: np.ndarray) -> np.ndarray:
    """Alg. 1, first step: bhat = Q_s b, returned as (2^s, n_b, m): bhat[a]
    is the right-hand side of subsystem a.  Uses the explicit Q_s."""
    n_b, S = img.shape
    s = S.bit_length() - 1
    perm = mirrored_permutation(img)
    bm = b[perm]
    Q = q_matrix(s, n_b)
    return (Q @ bm).reshape(S, n_b, -1)


def backward_transform(xhat: np.ndarray, img: np.ndarray) -> np.ndarray:
    """Alg. 1, last step: x = Q_s xhat, back in the caller's ordering."""
    S, n_b, m = xhat.shape
    s = S.bit_length() - 1
    Q = q_matrix(s, n_b)
    xm = Q @ xhat.reshape(S * n_b, m)
    x = np.empty_like(xm)
    x[mirrored_permutation(img)] = xm
    return x
