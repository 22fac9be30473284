"""Pins of the oracle's adjoint gradient: central finite differences, dL/df =
lambda, and agreement of two independent assemblies of the matrix."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gen import make_problem
from oracle import adjoint


def _loss(faces, img, kappa, f, ps):
    A = adjoint.assemble(faces, kappa, img).tocsc()
    p = spla.spsolve(A, f)
    return 0.5 * float(np.sum((p - ps) ** 2))


@pytest.mark.parametrize("N,s", [((8, 8, 8), 3), ((10, 8, 6), 2), ((12, 10), 1)])
def test_oracle_assembly_matches_generator(N, s):
    p = make_problem(N, s=s, seed=3, kappa="lognormal", jitter=0.2 if len(N) == 3 else None)
    A = adjoint.assemble(p.faces, p.kappa_base, p.img)
    assert (A - p.A).nnz == 0 or np.abs((A - p.A).data).max() <= 1e-14 * np.abs(p.A.data).max()


@pytest.mark.parametrize("kw", [dict(), dict(jitter=0.2)])
def test_kappa_gradient_central_differences(kw):
    pr = make_problem((8, 8, 8), s=3, m=1, seed=5, kappa="lognormal", with_target=True, **kw)
    f = pr.b[:, 0]
    ps = pr.p_target
    L, lam, g, _ = adjoint.loss_and_gradients(pr.faces, pr.img, pr.kappa_base, f, ps)
    rng = np.random.default_rng(0)
    for i in rng.choice(pr.n_b, size=20, replace=False):
        eps = 1e-6 * pr.kappa_base[i]
        kp = pr.kappa_base.copy()
        km = pr.kappa_base.copy()
        kp[i] += eps
        km[i] -= eps
        fd = (_loss(pr.faces, pr.img, kp, f, ps) - _loss(pr.faces, pr.img, km, f, ps)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g).max())


def test_rhs_gradient_is_lambda():
    pr = make_problem((6, 6, 6), s=2, m=1, seed=2, kappa="lognormal", with_target=True)
    f = pr.b[:, 0]
    L, lam, g, _ = adjoint.loss_and_gradients(pr.faces, pr.img, pr.kappa_base, f, pr.p_target)
    rng = np.random.default_rng(1)
    for i in rng.choice(pr.n, size=10, replace=False):
        e = np.zeros(pr.n)
        e[i] = 1e-6
        fd = (_loss(pr.faces, pr.img, pr.kappa_base, f + e, pr.p_target)
              - _loss(pr.faces, pr.img, pr.kappa_base, f - e, pr.p_target)) / 2e-6
        assert abs(fd - lam[i, 0]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(lam).max())
