"""AMGR in the original basis, for a domain made of copies of one subdomain.

TEST INFRASTRUCTURE ONLY: see oracle/__init__.py.

The paper's final preconditioner works on the system in its own ordering
(Sec. 3: inner-interface ordering, eq. (3.1); Sec. 3.2: Alg. 2, eqs.
(3.13)-(3.15), Alg. 3).  Nothing here needs the change of basis Q_s, so it
covers what Q_s cannot: translated (repeated) copies, any number of them, and
boundary conditions that differ between copies.  The domain is described by
sub[i, a], the row of unknown i of the base copy in copy a.

  * Interface (Sec. 3): an unknown coupled to an unknown of another copy.
    A base unknown whose row is not the same in every copy (a boundary
    condition that differs) is put on the interface too: that is how the
    interface frees the boundary conditions.  Both are decided per base
    unknown, so every copy has the same inner set, and the inner-inner block
    of every copy is the base copy's: K-bar = I (x) K.
  * Alg. 2 on the base copy: strength, T, T^d, the maximal independent set of
    the inner nodes under the hash priorities of the base indices (the
    reduction level of amg.py, run on the base copy's block with its
    interface); the set is replicated to every copy and joined with the
    whole interface: the populated interface.
  * Level 0 with that coarse set (amg.build_hierarchy): P = [W-bar; I]
    (eq. (3.13)), block FSAI over the F/C blocks (eq. (3.14); on the block-
    diagonal A_FF = I (x) K_FF it is I (x) FSAI(K_FF)), A_c = P^T A P
    (eq. (3.15)), then standard AMG levels and the V-cycle of Alg. 3.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import scipy.sparse as sp

from . import amg, krylov


def _index_maps(sub: np.ndarray):
    n_b, ns = sub.shape
    n = n_b * ns
    copy_of = np.empty(n, dtype=np.int64)
    base_of = np.empty(n, dtype=np.int64)
    copy_of[sub] = np.arange(ns)[None, :]
    base_of[sub] = np.arange(n_b)[:, None]
    return copy_of, base_of


def copy_block(A: sp.csr_matrix, sub: np.ndarray, a: int) -> sp.csr_matrix:
    """Block of copy a in base numbering: B[i, j] = A[sub[i, a], sub[j, a]]."""
    B = A.tocsr()[sub[:, a]][:, sub[:, a]].tocsr()
    B.sort_indices()
    return B


def interface_of_copies(A: sp.csr_matrix, sub: np.ndarray) -> np.ndarray:
    """Boolean mask over base unknowns: coupled to another copy in some copy,
    or with a row that differs (pattern or a value) from the base copy's row
    in some copy."""
    A = A.tocsr()
    n_b, ns = sub.shape
    copy_of, base_of = _index_maps(sub)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    cross = copy_of[rows] != copy_of[A.indices]
    iface = np.zeros(n_b, dtype=bool)
    iface[base_of[rows[cross]]] = True
    B0 = copy_block(A, sub, 0)
    for a in range(1, ns):
        Ba = copy_block(A, sub, a)
        for i in range(n_b):
            s0, e0 = B0.indptr[i], B0.indptr[i + 1]
            s1, e1 = Ba.indptr[i], Ba.indptr[i + 1]
            if e0 - s0 != e1 - s1 or np.any(B0.indices[s0:e0] != Ba.indices[s1:e1]) or \
                    np.any(B0.data[s0:e0] != Ba.data[s1:e1]):
                iface[i] = True
    return iface


def coarse_set(A: sp.csr_matrix, sub: np.ndarray, iface_base: np.ndarray, opt: amg.AMGOptions) -> np.ndarray:
    """The populated interface over all n unknowns: Alg. 2 on the base copy's
    block (MIS of T^d over its inner unknowns), replicated to every copy,
    joined with the interface of every copy."""
    C_base = amg.coarsen_level0(copy_block(A, sub, 0), iface_base, opt.theta, opt.dist, opt.seed, opt.mis_method)
    C = np.zeros(A.shape[0], dtype=bool)
    C[sub] = C_base[:, None]
    return C


def setup(A: sp.csr_matrix, sub: np.ndarray, opt: Optional[amg.AMGOptions] = None) -> dict:
    """Interface, populated coarse set and the AMGR hierarchy on the whole
    matrix in its own ordering."""
    opt = opt or amg.AMGOptions()
    A = A.tocsr()
    A.sort_indices()
    iface_base = interface_of_copies(A, sub)
    iface = np.zeros(A.shape[0], dtype=bool)
    iface[sub] = iface_base[:, None]
    C = coarse_set(A, sub, iface_base, opt)
    hier = amg.build_hierarchy(A, iface, opt, coarse0=C)
    return dict(A=A, sub=sub, interface_base=iface_base, interface=iface, C=C, hier=hier, opt=opt)


def solve(ctx: dict, b: np.ndarray, tol: float = 1e-10, maxit: int = 1000) -> krylov.PCGResult:
    """PCG on the whole system, one column per right-hand side, with the
    V-cycle of Alg. 3; column j stops once ||r_j|| <= tol ||b_j||."""
    A, H = ctx["A"], ctx["hier"]
    b = b.reshape(b.shape[0], -1)
    thresh = tol * np.linalg.norm(b, axis=0)
    return krylov.pcg_columns(lambda X: A @ X, lambda R: amg.vcycle(H, R), b, thresh, maxit)
