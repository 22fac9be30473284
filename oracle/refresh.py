"""Numeric re-setup of the AMGR hierarchy for a new matrix with the sparsity
of an earlier one (the per-coefficient rebuild of an adjoint or a time loop;
Sec. 6 names a device-side setup as future work).

TEST INFRASTRUCTURE ONLY: see oracle/__init__.py.

The structure of the earlier setup is kept: the interface, every level's C/F
split, the smoother patterns, and at the reduction level the truncated
interpolation pattern.  Every value is recomputed from the new matrix with
the same formulas as a fresh setup:
  * A_inn and the outer diagonal sigma from the new matrix (Sec. 2);
  * interpolation: the Jacobi steps of amg.interpolation on their symbolic
    patterns (which depend on the sparsity only), restricted at the reduction
    level to the kept pattern instead of the value-based truncation, then the
    row-sum rescaling (eq. (3.13));
  * with energy minimisation, the same steps on every interpolation;
  * FSAI on the kept pattern (block FSAI at level 0, eq. (3.14)) and its
    damping; the Galerkin products (eq. (3.15)) on patterns that the
    unchanged sparsity reproduces;
  * the per-subsystem levels on the shared splits and interpolation
    patterns and on the kept FSAI patterns, and the low-rank corrections, as
    krylov.setup builds them.
For a matrix whose fresh setup makes the same structural decisions (the same
matrix, or one scaled by a positive constant: strength, MIS and truncation
decisions are scale invariant) the re-setup equals the fresh setup.

rebuild_below keeps a context's reduction level as it stands and builds every
level below it afresh from its level-1 operator (the remedy when the kept
coarser splits cost iterations); when the kept reduction level is also what a
fresh setup would build, the result is the fresh setup.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import amg, krylov, lrc as lrcmod, symmetry


def refresh_hierarchy(old: amg.Hierarchy, Ainn: sp.csr_matrix, opt: amg.AMGOptions) -> amg.Hierarchy:
    A = Ainn.tocsr()
    A.sort_indices()
    levels = []
    for lev, Lo in enumerate(old.levels):
        if A.shape != Lo.A.shape or not (np.array_equal(A.indptr, Lo.A.indptr) and
                                         np.array_equal(A.indices, Lo.A.indices)):
            raise ValueError(f"level {lev}: sparsity differs from the earlier setup")
        L = amg.Level(A=A)
        levels.append(L)
        if Lo.C is None:
            break
        L.C = Lo.C.copy()
        n = A.shape[0]
        # FSAI on the earlier pattern: its lower entries are the pattern itself
        L.G = amg.fsai(A, Lo.G, np.zeros(n, dtype=np.int64))
        L.omega = amg.damping(A, L.G, opt.seed)
        if lev == 0:
            L.P = amg.interpolation(A, L.C, opt.jacobi0, keep_pattern=Lo.P if opt.trunc0 > 0.0 else None)
        else:
            L.P = amg.interpolation(A, L.C, opt.jacobi)
        if opt.emin_steps > 0:
            L.P = amg.emin(A, L.C, L.P, opt.emin_steps)
        L.R = L.P.T.tocsr()
        L.R.sort_indices()
        A = amg.galerkin(A, L.P)
    factor = sla.cho_factor(levels[-1].A.toarray(), lower=True)
    return amg.Hierarchy(levels=levels, coarse_factor=factor, nu1=old.nu1, nu2=old.nu2)


def refresh(ctx: dict, A_new: sp.csr_matrix) -> dict:
    """krylov.setup's context for A_new, built on ctx's structure."""
    img, opt, precond = ctx["img"], ctx["opt"], ctx["precond"]
    H = symmetry.base_blocks(A_new, img)
    Ainn, outs = symmetry.inner_outer(H)
    iface = symmetry.interface_rows(H)
    if not np.array_equal(iface, ctx["interface"]):
        raise ValueError("interface differs from the earlier setup")
    if precond not in ("amgr", "amgr_sub"):
        raise ValueError(precond)
    hier = refresh_hierarchy(ctx["hier"], Ainn, opt)
    sub = None
    if precond == "amgr_sub" and hier.nlev > 1:
        sigma = np.stack([o.diagonal() for o in outs], axis=1)
        # the subsystem levels keep the earlier setup's FSAI patterns too (a fresh
        # setup takes them from the strength of the shared values)
        sub = amg.build_sub_hierarchy(hier, sigma, opt, patterns=[L.G for L in ctx["hier"].levels])
    low = _corrections(ctx, hier, sub, Ainn, outs)
    return dict(ctx, H=H, Ainn=Ainn, outs=outs, interface=iface, hier=hier, sub=sub, lrc=low)


def _corrections(ctx: dict, hier, sub, Ainn, outs):
    """LRCAMG corrections of the rank ctx was set up with, for a new hierarchy."""
    opt = ctx["opt"]
    k = 0 if ctx["lrc"] is None else max(len(r) for r in ctx["lrc"].ritz)
    if k == 0:
        return None
    if sub is None:
        return lrcmod.build_lrcamg(hier, Ainn, outs, k, opt.seed)
    Ahat = [(Ainn + o).tocsr() for o in outs]
    return lrcmod.build_lrcamg(hier, Ainn, outs, k, opt.seed,
                               apply_Minv=lambda a, x: amg.vcycle_sub(sub, Ahat[a], a, x))


def rebuild_below(ctx: dict) -> dict:
    """ctx with its reduction level kept as it stands (split, patterns and
    values) and every level below it built afresh from its level-1 operator,
    as krylov.setup builds them: fresh standard splits, patterns and
    per-subsystem values, then new low-rank corrections."""
    opt, precond = ctx["opt"], ctx["precond"]
    if precond not in ("amgr", "amgr_sub"):
        raise ValueError(precond)
    hier = amg.build_hierarchy_below(ctx["hier"], opt)
    sub = None
    if precond == "amgr_sub":
        sigma = np.stack([o.diagonal() for o in ctx["outs"]], axis=1)
        sub = amg.build_sub_hierarchy(hier, sigma, opt)
    low = _corrections(ctx, hier, sub, ctx["Ainn"], ctx["outs"])
    return dict(ctx, hier=hier, sub=sub, lrc=low)
