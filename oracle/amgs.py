"""AMGS, the Schur-complement AMG of Sec. 3.1, on the decoupled subsystems.

TEST INFRASTRUCTURE ONLY: see oracle/__init__.py.

Inner-interface ordering (eq. (3.1)) of the base mesh: K = A_inn[I, I],
B = A_inn[I, G], C_1 = A_inn[G, G] (I inner, G interface rows of the base
mesh, each in increasing base index).  In the Q_s basis every subsystem is
A_a = [K B; B^T C_1 + Sigma_a] with Sigma_a = diag(sigma_a) on the interface
(eqs. (2.13)-(2.14)): K and B are shared (K-bar = I (x) K, B-bar = I (x) B),
and the Schur complement of K in A_a is S_a = C_1 + Sigma_a - B^T K^{-1} B,
the decoupled block of eq. (3.7) (for one symmetry, S_1 +- C_2).

Preconditioner (eq. (3.12)), per subsystem a and residual r = [r_I; r_G]:
    t_I = AMG_K r_I                       (the AMG of K, Sec. 3.1)
    q   = r_G - B^T t_I
    z_G = S_a^{-1} q                      (approximation below)
    z_I = t_I - K^{-1} B z_G              (K^{-1} = AMG_K again: the symmetric
                                           form; or G_K^T G_K: the light form
                                           the paper times last in Table 3)
Schur approximation (eqs. (3.4), (3.9)-(3.11)): G_K = FSAI(K);
S_G1 = C_1 - B^T G_K^T G_K B ~ C_1 - B^T K^{-1} B; G_S1 = FSAI(S_G1); then
S_a^{-1} ~ G_S1^T G_S1 + Z_a Theta_a Z_a^T, the low-rank correction of
Thm. 2.2 per subsystem toward S_AMG,a = C_1 + Sigma_a - B^T AMG_K B
(eq. (3.8)), computed as LRCFSAI: Lanczos on G_S1 S_AMG,a G_S1^T, the k
smallest Ritz pairs below one, Z = G_S1^T V, Theta = 1/lambda - 1.

Readings (the paper cites adaptive FSAI with a pre-filter tau = 0.01 and
100 / 50 entries per row, and PMIS + ExtI for the AMG of K, without
defining them):
  * AMG of K: this package's hierarchy builder with an empty interface
    (Alg. 2 degenerates to an aggressive distance-d MIS coarsening at level
    0, standard levels below).
  * FSAI of K: static pattern = lower triangle of the pattern of K_f^2, K_f
    being K without the off-diagonal entries |k_ij| < tau sqrt(k_ii k_jj).
  * S_G1 = C_1 - (X + X^T) / 2 with X = B^T (G_K^T (G_K B)) (symmetrised so
    that both sides' FSAI sees an exactly symmetric matrix).
  * FSAI of S_G1: lower triangle of the pattern of S_f^3, S_f = S_G1
    without the entries |s_ij| < tau sqrt(s_ii s_jj); values from S_G1.  At
    64^3, s = 3, k = 8 (tol 1e-10) the filtered pattern's powers 2, 3, 4, 6
    keep 7, 13, 21, 41 entries per row and take 40, 32, 31, 30 iterations;
    the power of K's pattern changes nothing (square or cube: 40).
The outer solver is PCG (standard beta) for the symmetric form and Notay's
flexible CG for the light form, whose preconditioner is not symmetric; the
paper runs GMRES.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np
import scipy.sparse as sp

from . import amg, krylov, lrc as lrcmod, symmetry


@dataclasses.dataclass
class AMGSOptions:
    amg: amg.AMGOptions = dataclasses.field(default_factory=amg.AMGOptions)
    k: int = 0                # low-rank correction rank of the Schur approximation, per subsystem
    light: bool = False       # K^{-1} = G_K^T G_K in the first factor (else AMG_K: symmetric)
    tau: float = 0.01         # pre-filter of the FSAI patterns


def split(Ainn: sp.csr_matrix, iface: np.ndarray):
    """Inner and interface index lists and the blocks K, B, C_1 (eq. (3.1))."""
    inner = np.flatnonzero(~iface)
    ifc = np.flatnonzero(iface)
    A = Ainn.tocsr()
    K = A[inner][:, inner].tocsr()
    B = A[inner][:, ifc].tocsr()
    C1 = A[ifc][:, ifc].tocsr()
    for M in (K, B, C1):
        M.sort_indices()
    return inner, ifc, K, B, C1


def filtered_pattern(M: sp.csr_matrix, tau: float) -> sp.csr_matrix:
    """Pattern of M without the off-diagonal entries |m_ij| < tau sqrt(|m_ii m_jj|)
    (the diagonal always kept); values 1."""
    M = M.tocsr()
    d = np.abs(M.diagonal())
    rows = np.repeat(np.arange(M.shape[0]), np.diff(M.indptr))
    cols = M.indices
    keep = (rows == cols) | (np.abs(M.data) >= tau * np.sqrt(d[rows] * d[cols]))
    P = sp.csr_matrix((np.ones(int(keep.sum())), (rows[keep], cols[keep])), shape=M.shape)
    P.sort_indices()
    return P


def fsai_filtered_power(M: sp.csr_matrix, tau: float, power: int) -> sp.csr_matrix:
    """FSAI of M on the lower triangle of the pattern of M_f^power, M_f the
    tau-filtered M."""
    P = filtered_pattern(M, tau)
    Q = P
    for _ in range(power - 1):
        Q = (Q @ P).tocsr()
    Q.data[:] = 1.0
    return amg.fsai(M, Q, np.zeros(M.shape[0], dtype=np.int64))


def fsai_k(K: sp.csr_matrix, tau: float) -> sp.csr_matrix:
    """G_K: FSAI of K on the lower triangle of the pattern of K_f^2."""
    return fsai_filtered_power(K, tau, 2)


def schur_g(C1: sp.csr_matrix, B: sp.csr_matrix, G: sp.csr_matrix) -> sp.csr_matrix:
    """S_G1 = C_1 - (X + X^T) / 2, X = B^T (G^T (G B)) (eq. (3.4) on the base mesh)."""
    W1 = (G @ B).tocsr()
    W2 = (G.T.tocsr() @ W1).tocsr()
    X = (B.T.tocsr() @ W2).tocsr()
    Xs = (0.5 * (X + X.T)).tocsr()
    S = (C1 - Xs).tocsr()
    S.sort_indices()
    return S


def fsai_s(S: sp.csr_matrix, tau: float) -> sp.csr_matrix:
    """G_S1: FSAI of S_G1 on the lower triangle of the pattern of S_f^3."""
    return fsai_filtered_power(S, tau, 3)


def setup(A: sp.csr_matrix, img: np.ndarray, opt: Optional[AMGSOptions] = None) -> dict:
    opt = opt or AMGSOptions()
    H = symmetry.base_blocks(A, img)
    Ainn, outs = symmetry.inner_outer(H)
    iface = symmetry.interface_rows(H)
    inner, ifc, K, B, C1 = split(Ainn, iface)
    S = len(outs)
    sigma = np.stack([o.diagonal() for o in outs], axis=1)       # (n_b, S)
    HK = amg.build_hierarchy(K, np.zeros(K.shape[0], dtype=bool), opt.amg)
    GK = fsai_k(K, opt.tau)
    SG1 = schur_g(C1, B, GK)
    GS1 = fsai_s(SG1, opt.tau)
    ctx = dict(H=H, Ainn=Ainn, outs=outs, img=img, iface=iface, inner=inner, ifc=ifc, K=K, B=B, C1=C1,
               BT=B.T.tocsr(), sigma_g=sigma[ifc], HK=HK, GK=GK, SG1=SG1, GS1=GS1, opt=opt, low=None)
    if opt.k > 0:
        ctx["low"] = build_schur_lrc(ctx, opt.k, opt.amg.seed)
    return ctx


def schur_amg(ctx: dict, a: int, X: np.ndarray) -> np.ndarray:
    """S_AMG,a X = C_1 X + sigma_a X - B^T AMG_K (B X) (eq. (3.8), decoupled)."""
    return ctx["C1"] @ X + ctx["sigma_g"][:, a:a + 1] * X - ctx["BT"] @ amg.vcycle(ctx["HK"], ctx["B"] @ X)


def build_schur_lrc(ctx: dict, k: int, seed: int, keep_all: bool = False, steps: int = None):
    """LRCFSAI(k) of every decoupled Schur block toward S_AMG,a (eq. (3.11))."""
    G = ctx["GS1"]
    GT = G.T.tocsr()
    n = G.shape[0]
    steps = steps or lrcmod.lanczos_steps(k, n)
    v0 = lrcmod.start_vector(n, seed)
    Us, cs, rs = [], [], []
    for a in range(len(ctx["outs"])):
        op = lambda v, Bv, a=a: G @ schur_amg(ctx, a, (GT @ v)[:, None])[:, 0]  # noqa: E731
        V, al, be = lrcmod.lanczos(op, lambda x: x, v0, steps)
        th, Vk = lrcmod.ritz(V, al, be, k)
        keep = np.ones(th.size, dtype=bool) if keep_all else th < 1.0
        Us.append(GT @ Vk[:, keep])
        cs.append(1.0 / th[keep] - 1.0)
        rs.append(th)
    return lrcmod.LowRank(U=Us, coef=cs, ritz=rs)


def apply_with(ctx: dict, R: np.ndarray, m: int, K1: Callable, S_inv: Callable, K2: Callable) -> np.ndarray:
    """Eq. (3.12) on every column of R (n_b x S*m, column a*m + j): K1 and K2
    approximate K^{-1} in the middle and first factors, S_inv(a, Q) the
    decoupled Schur complement of subsystem a."""
    inner, ifc = ctx["inner"], ctx["ifc"]
    T = K1(R[inner])
    Q = R[ifc] - ctx["BT"] @ T
    ZG = np.empty_like(Q)
    for a in range(R.shape[1] // m):
        ZG[:, a * m:(a + 1) * m] = S_inv(a, Q[:, a * m:(a + 1) * m])
    ZI = T - K2(ctx["B"] @ ZG)
    Z = np.empty_like(R)
    Z[inner] = ZI
    Z[ifc] = ZG
    return Z


def apply(ctx: dict, R: np.ndarray, m: int) -> np.ndarray:
    """AMGS(S_LRC^{-1}, AMG_K) (symmetric) or AMGS(S_LRC^{-1}, G_K) (light)."""
    HK, GK, GS1, low = ctx["HK"], ctx["GK"], ctx["GS1"], ctx["low"]
    GS1T, GKT = GS1.T.tocsr(), GK.T.tocsr()

    def s_inv(a, Q):
        Z = GS1T @ (GS1 @ Q)
        if low is not None and low.U[a].shape[1]:
            U = low.U[a]
            Z = Z + U @ (low.coef[a][:, None] * (U.T @ Q))
        return Z

    k1 = lambda X: amg.vcycle(HK, X)  # noqa: E731
    k2 = (lambda X: GKT @ (GK @ X)) if ctx["opt"].light else k1
    return apply_with(ctx, R, m, k1, s_inv, k2)


def solve(ctx: dict, b: np.ndarray, tol: float = 1e-10, maxit: int = 1000) -> krylov.SolveResult:
    """Alg. 1 with AMGS on every decoupled subsystem: PCG for the symmetric
    form, flexible CG for the light form."""
    img = ctx["img"]
    n_b, S = img.shape
    b = b.reshape(b.shape[0], -1)
    m = b.shape[1]
    bhat = symmetry.forward_transform(b, img)
    Ainn, outs = ctx["Ainn"], ctx["outs"]
    Ahat = [(Ainn + outs[a]).tocsr() for a in range(S)]
    Bc = np.concatenate([bhat[a] for a in range(S)], axis=1)
    thresh = np.tile(tol * np.linalg.norm(b, axis=0) / np.sqrt(S), S)

    def apply_A(X):
        Y = np.empty_like(X)
        for a in range(S):
            Y[:, a * m:(a + 1) * m] = Ahat[a] @ X[:, a * m:(a + 1) * m]
        return Y

    res = krylov.pcg_columns(apply_A, lambda R: apply(ctx, R, m), Bc, thresh, maxit, flexible=ctx["opt"].light)
    xhat = np.stack([res.x[:, a * m:(a + 1) * m] for a in range(S)])
    x = symmetry.backward_transform(xhat, img)
    return krylov.SolveResult(x=x, iters=res.iters.reshape(S, m), relres=None, hierarchy=ctx["HK"])
