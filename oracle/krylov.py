"""Alg. 1 with per-column preconditioned CG on the decoupled subsystems.

Each column (subsystem a, right-hand side j) runs its own Hestenes-Stiefel
PCG from zero, with its own step lengths (the decoupled solves of Alg. 1).
A column stops ("freezes") once ||r_hat|| <= tol * ||b_j|| / sqrt(2^s); since
Q_s is orthogonal this bounds the true relative residual of right-hand side
j by tol.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np
import scipy.sparse as sp

from . import symmetry
from . import lrc as lrcmod
from .amg import AMGOptions, Hierarchy, build_hierarchy, build_sub_hierarchy, vcycle, vcycle_sub


class Breakdown(RuntimeError):
    pass


@dataclasses.dataclass
class PCGResult:
    x: np.ndarray                 # (n_rows, ncols)
    iters: np.ndarray             # per column
    converged: np.ndarray         # per column
    history: List[np.ndarray]     # residual norms per iteration


def pcg_columns(apply_A: Callable, apply_M: Callable, B: np.ndarray, thresh: np.ndarray,
                maxit: int, flexible: bool = False) -> PCGResult:
    """PCG on every column of B at once, with per-column alpha and beta.

    apply_A(X), apply_M(R) act column-wise on (n, k) blocks.  Column c stops
    once ||r_c|| <= thresh[c]; columns already below their threshold at
    the start (including zero columns) do no iteration.  Standard beta is
    <r_new, z_new> / <r_old, z_old>.  ``flexible`` selects the flexible CG of
    Notay (SIAM J. Sci. Comput. 22, 2000) with one kept direction:
    beta = -<z_new, A p> / <p, A p>, which makes every new direction
    A-orthogonal to the previous one whatever the preconditioner does (a
    preconditioner that changes between iterations, such as a V-cycle run in
    reduced precision); for a fixed SPD preconditioner it equals the standard
    beta in exact arithmetic.  Breakdown (p^T A p <= 0 or not finite in an
    active column) raises."""
    n, k = B.shape
    X = np.zeros((n, k))
    R = B.copy()
    active = np.linalg.norm(R, axis=0) > thresh
    iters = np.zeros(k, dtype=np.int64)
    P = apply_M(R)
    rho = np.einsum("ij,ij->j", R, P)
    hist = [np.linalg.norm(R, axis=0)]
    it = 0
    while active.any() and it < maxit:
        Q = apply_A(P)
        pq = np.einsum("ij,ij->j", P, Q)
        bad = active & ~(np.isfinite(pq) & (pq > 0))
        if bad.any():
            raise Breakdown(f"p^T A p <= 0 or not finite in columns {np.flatnonzero(bad)}")
        alpha = np.where(active, rho / np.where(active, pq, 1.0), 0.0)
        X += alpha * P
        R -= alpha * Q
        it += 1
        iters[active] = it
        rn = np.linalg.norm(R, axis=0)
        hist.append(rn)
        active = active & (rn > thresh)
        if not active.any():
            break
        Znew = apply_M(R)
        rho_new = np.einsum("ij,ij->j", R, Znew)
        if flexible:
            beta = np.where(active, -np.einsum("ij,ij->j", Znew, Q) / np.where(active, pq, 1.0), 0.0)
        else:
            beta = np.where(active, rho_new / np.where(active, rho, 1.0), 0.0)
        P = np.where(active[None, :], Znew + beta * P, P)
        rho = np.where(active, rho_new, rho)
    return PCGResult(x=X, iters=iters, converged=~active, history=hist)


@dataclasses.dataclass
class SolveResult:
    x: np.ndarray
    iters: np.ndarray            # (2^s, m)
    relres: np.ndarray           # true relative residual per RHS
    hierarchy: Optional[Hierarchy]


def setup(A: sp.csr_matrix, img: np.ndarray, opt: Optional[AMGOptions] = None,
          precond: str = "amgr", k: int = 0):
    """Setup of Alg. 1: base blocks, shared A_inn, per-subsystem outer parts,
    interface set, and the preconditioner: "amgr" (AMGR hierarchy on A_inn
    shared by every subsystem, LRCAMG(k) when k > 0), "amgr_sub" (the shared
    reduction level, then every subsystem's own reduced operator and levels
    below it; LRCAMG(k) on top when k > 0), "fsai" (FSAI of A_inn,
    LRCFSAI(k) when k > 0) or "none"."""
    opt = opt or AMGOptions()
    H = symmetry.base_blocks(A, img)
    Ainn, outs = symmetry.inner_outer(H)
    iface = symmetry.interface_rows(H)
    hier = build_hierarchy(Ainn, iface, opt) if precond in ("amgr", "amgr_sub") else None
    sub = None
    if precond == "amgr_sub" and hier.nlev > 1:
        sigma = np.stack([o.diagonal() for o in outs], axis=1)
        sub = build_sub_hierarchy(hier, sigma, opt)
    G = lrcmod.fsai_inner(Ainn) if precond == "fsai" else None
    low = None
    if k > 0 and precond == "amgr":
        low = lrcmod.build_lrcamg(hier, Ainn, outs, k, opt.seed)
    elif k > 0 and precond == "amgr_sub":
        Ahat = [(Ainn + o).tocsr() for o in outs]
        if sub is None:
            low = lrcmod.build_lrcamg(hier, Ainn, outs, k, opt.seed)
        else:
            low = lrcmod.build_lrcamg(hier, Ainn, outs, k, opt.seed,
                                      apply_Minv=lambda a, x: vcycle_sub(sub, Ahat[a], a, x))
    elif k > 0 and precond == "fsai":
        low = lrcmod.build_lrcfsai(G, Ainn, outs, k, opt.seed)
    return dict(H=H, Ainn=Ainn, outs=outs, interface=iface, hier=hier, G=G, lrc=low, img=img,
                opt=opt, precond=precond, sub=sub)


def solve(ctx: dict, b: np.ndarray, tol: float = 1e-10, maxit: int = 1000,
          flexible: bool = False) -> SolveResult:
    """Alg. 1: bhat = Q_s b; decoupled PCG on A_inn + A_out,a for every a with
    the shared preconditioner (I (x) M_inn^{-1}, optionally low-rank corrected
    per subsystem); x = Q_s xhat."""
    precond, lrc = ctx["precond"], ctx["lrc"]
    img = ctx["img"]
    n_b, S = img.shape
    b = b.reshape(b.shape[0], -1)
    m = b.shape[1]
    bhat = symmetry.forward_transform(b, img)           # (S, n_b, m)
    Ainn, outs, hier = ctx["Ainn"], ctx["outs"], ctx["hier"]
    Ahat = [(Ainn + outs[a]).tocsr() for a in range(S)]
    Bc = np.concatenate([bhat[a] for a in range(S)], axis=1)   # (n_b, S*m), column a*m+j
    bn = np.linalg.norm(b, axis=0)
    thresh = np.tile(tol * bn / np.sqrt(S), S)

    def apply_A(X):
        Y = np.empty_like(X)
        for a in range(S):
            Y[:, a * m:(a + 1) * m] = Ahat[a] @ X[:, a * m:(a + 1) * m]
        return Y

    if precond == "amgr":
        def apply_M(R):
            Z = vcycle(hier, R)
            if lrc is not None:
                Z = Z + lrc.apply(R, m)
            return Z
    elif precond == "amgr_sub":
        def apply_M(R):
            if ctx["sub"] is None:
                Z = vcycle(hier, R)
            else:
                Z = np.empty_like(R)
                for a in range(S):
                    Z[:, a * m:(a + 1) * m] = vcycle_sub(ctx["sub"], Ahat[a], a, R[:, a * m:(a + 1) * m])
            if lrc is not None:
                Z = Z + lrc.apply(R, m)
            return Z
    elif precond == "fsai":
        def apply_M(R):
            Z = lrcmod.fsai_apply(ctx["G"], R)
            if lrc is not None:
                Z = Z + lrc.apply(R, m)
            return Z
    elif precond == "none":
        def apply_M(R):
            return R.copy()
    else:
        raise ValueError(precond)
    res = pcg_columns(apply_A, apply_M, Bc, thresh, maxit, flexible=flexible)
    xhat = np.stack([res.x[:, a * m:(a + 1) * m] for a in range(S)])
    x = symmetry.backward_transform(xhat, img)
    # true residual in the caller's ordering, from the full matrix
    return SolveResult(x=x, iters=res.iters.reshape(S, m), relres=None, hierarchy=hier)


def true_relres(A: sp.csr_matrix, x: np.ndarray, b: np.ndarray) -> np.ndarray:
    b = b.reshape(b.shape[0], -1)
    x = x.reshape(x.shape[0], -1)
    return np.linalg.norm(b - A @ x, axis=0) / np.linalg.norm(b, axis=0)
