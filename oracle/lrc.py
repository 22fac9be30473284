"""Low-rank corrections of Sec. 2.1 (LRCFSAI(k), eq. (2.24)) and Sec. 2.2
(LRCAMG(k), eq. (2.32)), per decoupled subsystem.

LRCAMG in symmetric form.  With M^{-1} the shared V-cycle and
X_a = M^{-1} A_a (self-adjoint in the A_a inner product), let (lam_j, u_j)
be eigenpairs of X_a with U^T A_a U = I.  For exact eigenpairs the paper's
correction (I + U Theta V^T) M^{-1} with biorthonormal left vectors
V = M U and Theta = Lambda^{-1} - I (Sigma = I - Lambda) equals
M^{-1} + U diag(1 - lam) U^T, which maps every corrected eigenvalue to 1
and leaves the rest of the spectrum alone.  Only pairs with lam_j < 1 (the
small eigenvalues that slow PCG) are kept, so the correction is positive
semidefinite and the preconditioner stays SPD for approximate pairs.

LRCFSAI.  z = G^T G r + Z Theta Z^T r with Z = G^T V_k and
Theta = Lambda^{-1} - I, V_k orthonormal eigenvectors of G A_a G^T for its k
smallest eigenvalues; G = FSAI(A_inn) on the lower pattern of A_inn.

Eigenpairs.  The paper only asks for rough approximations; the reading
here is Lanczos with full reorthogonalisation (classical Gram-Schmidt
applied twice), max(4k, 40) steps, deterministic start vector
v_i = splitmix64(seed xor i xor 0x1CC)/2^64 - 1/2 shared by all subsystems,
Ritz pairs from the tridiagonal matrix.  Ritz *vectors* inside degenerate
eigenspaces are not unique: parity unpinned for them; Ritz values and final
solutions are compared instead.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .amg import fsai, vcycle
from .splitmix import unit_centered

LANCZOS_TAG = 0x1CC


def lanczos_steps(k: int, n: int) -> int:
    return int(min(max(4 * k, 40), n))


def start_vector(n: int, seed: int) -> np.ndarray:
    return unit_centered(np.uint64(seed) ^ np.arange(n, dtype=np.uint64) ^ np.uint64(LANCZOS_TAG))


def lanczos(op: Callable, apply_B: Callable, v0: np.ndarray, steps: int):
    """Lanczos for an operator self-adjoint in <x, y>_B = x^T B y, with full
    reorthogonalisation (two classical Gram-Schmidt passes against all
    previous basis vectors).  Returns (V, alpha, beta): V's columns are
    B-orthonormal, T = tridiag(beta, alpha, beta)."""
    n = v0.size
    Bv = apply_B(v0)
    nrm = np.sqrt(v0 @ Bv)
    V = [v0 / nrm]
    BV = [Bv / nrm]
    alpha, beta = [], []
    for j in range(steps):
        w = op(V[j], BV[j])
        alpha.append(float(w @ BV[j]))
        Vm = np.column_stack(V)
        BVm = np.column_stack(BV)
        for _ in range(2):
            w = w - Vm @ (BVm.T @ w)
        Bw = apply_B(w)
        b = float(np.sqrt(max(w @ Bw, 0.0)))
        if j == steps - 1 or b <= 1e-13 * abs(alpha[-1]):
            break
        beta.append(b)
        V.append(w / b)
        BV.append(Bw / b)
    m = len(alpha)
    return np.column_stack(V[:m]), np.array(alpha), np.array(beta[:m - 1])


def ritz(V, alpha, beta, k):
    """The k smallest Ritz pairs (values ascending)."""
    theta, S = sla.eigh_tridiagonal(alpha, beta)
    order = np.argsort(theta)[:k]
    return theta[order], V @ S[:, order]


@dataclasses.dataclass
class LowRank:
    """Per-subsystem correction z_a += U_a diag(coef_a) U_a^T r_a."""
    U: List[np.ndarray]          # per subsystem, (n_b, k_a)
    coef: List[np.ndarray]       # per subsystem, (k_a,)
    ritz: List[np.ndarray]       # per subsystem, all k Ritz values kept from Lanczos

    def apply(self, R: np.ndarray, m: int) -> np.ndarray:
        Z = np.zeros_like(R)
        for a, (U, c) in enumerate(zip(self.U, self.coef)):
            cols = slice(a * m, (a + 1) * m)
            if U.shape[1]:
                Z[:, cols] = U @ (c[:, None] * (U.T @ R[:, cols]))
        return Z


def build_lrcamg(hier, Ainn: sp.csr_matrix, outs, k: int, seed: int,
                 keep_all: bool = False, steps: int = None, apply_Minv=None) -> LowRank:
    """LRCAMG(k) in symmetric form for every subsystem a: Lanczos on
    M^{-1} A_a in the A_a inner product; keep the k smallest Ritz pairs
    and, of those, the ones below 1; coefficient 1 - lam.  ``keep_all`` keeps
    every pair (the full-rank statement of Thm. 2.2).  M^{-1} is the shared
    V-cycle of ``hier``, or ``apply_Minv(a, x)`` when given (a preconditioner
    of its own per subsystem)."""
    n = Ainn.shape[0]
    steps = steps or lanczos_steps(k, n)
    v0 = start_vector(n, seed)
    Us, cs, rs = [], [], []
    for a, Ao in enumerate(outs):
        Ah = (Ainn + Ao).tocsr()
        if apply_Minv is None:
            op = lambda v, Bv: vcycle(hier, Bv)
        else:
            op = lambda v, Bv, a=a: apply_Minv(a, Bv)
        V, al, be = lanczos(op, lambda x: Ah @ x, v0, steps)
        th, U = ritz(V, al, be, k)
        keep = np.ones(th.size, dtype=bool) if keep_all else th < 1.0
        Us.append(U[:, keep])
        cs.append(1.0 - th[keep])
        rs.append(th)
    return LowRank(U=Us, coef=cs, ritz=rs)


def fsai_inner(Ainn: sp.csr_matrix) -> sp.csr_matrix:
    """FSAI of A_inn on the full lower pattern of A_inn (every stored
    neighbour, not only strong ones)."""
    n = Ainn.shape[0]
    pat = Ainn.copy().tocsr()
    pat.data[:] = 1.0
    return fsai(Ainn, pat, np.zeros(n, dtype=np.int64))


def build_lrcfsai(G: sp.csr_matrix, Ainn: sp.csr_matrix, outs, k: int, seed: int,
                  keep_all: bool = False, steps: int = None) -> LowRank:
    """LRCFSAI(k) per subsystem (eqs. (2.18)-(2.24)): Lanczos on X_a = G A_a G^T
    (Euclidean), k smallest Ritz pairs (lam, v); Z = G^T v, coefficient
    Theta = 1/lam - 1 (pairs with lam >= 1 carry a non-positive coefficient
    and are dropped, keeping the correction positive semidefinite)."""
    n = Ainn.shape[0]
    steps = steps or lanczos_steps(k, n)
    v0 = start_vector(n, seed)
    GT = G.T.tocsr()
    Us, cs, rs = [], [], []
    for a, Ao in enumerate(outs):
        Ah = (Ainn + Ao).tocsr()
        V, al, be = lanczos(lambda v, Bv: G @ (Ah @ (GT @ v)), lambda x: x, v0, steps)
        th, Vk = ritz(V, al, be, k)
        keep = np.ones(th.size, dtype=bool) if keep_all else th < 1.0
        Us.append(GT @ Vk[:, keep])
        cs.append(1.0 / th[keep] - 1.0)
        rs.append(th)
    return LowRank(U=Us, coef=cs, ritz=rs)


def fsai_apply(G: sp.csr_matrix, R: np.ndarray) -> np.ndarray:
    """z = G^T G r (the FSAI preconditioner of eq. (2.17))."""
    return G.T @ (G @ R)
