"""Pins of the problem generator and of the Sec. 2 part of the oracle
(base blocks, Q_s, decoupled subsystems, Alg. 1) against closed forms,
invariants and dense direct solves."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from gen import make_problem
from oracle import symmetry
from oracle.splitmix import splitmix64

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vectors():
    rows = []
    for line in open(os.path.join(GOLDEN, "splitmix64.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        st, out = line.split()
        rows.append((int(st, 16), int(out)))
    got = splitmix64(np.array([r[0] for r in rows], dtype=np.uint64))
    assert [int(v) for v in got] == [r[1] for r in rows]


def _dirichlet_1d(N):
    k = np.arange(1, N + 1)
    return 4.0 * np.sin(k * np.pi / (2 * N)) ** 2


@pytest.mark.parametrize("N,s", [((8, 6), 1), ((6, 8), 2), ((8, 6, 4), 2), ((4, 4, 4), 3)])
def test_uniform_spectrum_closed_form(N, s):
    """Uniform grid, kappa = 1, Dirichlet walls: the two-point-flux matrix is a
    Kronecker sum of 1-D factors tridiag(-1, 2, -1) with end diagonals 3,
    eigenvalues 4 sin^2(k pi / (2N)), weighted by face area / spacing."""
    p = make_problem(N, s=s, seed=1)
    h = [1.0 / v for v in N]
    lam = 0
    for t in range(len(N)):
        w = np.prod([h[q] for q in range(len(N)) if q != t]) / h[t]
        shape = [1] * len(N)
        shape[t] = N[t]
        lam = lam + w * _dirichlet_1d(N[t]).reshape(shape)
    ex = np.sort(np.asarray(lam).ravel())
    ev = np.linalg.eigvalsh(p.A.toarray())
    assert np.max(np.abs(ev - ex)) < 1e-12 * ex.max()


@pytest.mark.parametrize("ordering", ["natural", "mirrored"])
@pytest.mark.parametrize("kw", [dict(), dict(y_stretch=1.5), dict(jitter=0.2, kappa="lognormal")])
def test_block_structure_exact(ordering, kw):
    """Block (a, b) of the mirrored matrix equals H_{a xor b} bit for bit
    (eqs. (2.4)-(2.5)); A is symmetric."""
    p = make_problem((8, 8, 8), s=3, seed=5, ordering=ordering, **kw)
    H = symmetry.base_blocks(p.A, p.img)
    assert (p.A != p.A.T).nnz == 0
    # for a two-point stencil only H_0 and the single-plane blocks are nonzero
    for j, Hj in H.items():
        if j and (j & (j - 1)):
            assert Hj.nnz == 0
        elif j:
            assert np.all(Hj.indices == np.repeat(np.arange(Hj.shape[0]), np.diff(Hj.indptr)))


def test_block_structure_rejects_asymmetric_map():
    p = make_problem((8, 8), s=1, seed=2, y_stretch=1.5, ordering="mirrored")
    img = p.img.copy()
    img[[0, 1], 1] = img[[1, 0], 1]        # swap two images: breaks the mirror map
    with pytest.raises(ValueError):
        symmetry.base_blocks(p.A, img)


@pytest.mark.parametrize("N", [8, 12, 16])
def test_interface_count_closed_form(N):
    """s = 3 cube: interface = cells touching one of the three mid-planes,
    3 (N/2)^2 - 3 (N/2) + 1."""
    p = make_problem((N, N, N), s=3, seed=1)
    H = symmetry.base_blocks(p.A, p.img)
    h = N // 2
    assert symmetry.interface_rows(H).sum() == 3 * h * h - 3 * h + 1


@pytest.mark.parametrize("s", [1, 2, 3])
def test_q_orthogonal_involution(s):
    Q = symmetry.q_matrix(s, 5).toarray()
    I = np.eye(Q.shape[0])
    assert np.abs(Q.T @ Q - I).max() < 1e-15
    assert np.abs(Q @ Q - I).max() < 1e-15
    assert np.abs(Q - Q.T).max() == 0.0
    # equals 2^{-s/2} Hadamard (x) I
    Hd = symmetry.hadamard(1 << s) / np.sqrt(1 << s)
    assert np.abs(Q - np.kron(Hd, np.eye(5))).max() < 1e-15


@pytest.mark.parametrize("kw", [dict(), dict(y_stretch=1.5), dict(jitter=0.2, kappa="lognormal")])
def test_qaq_block_diagonal_and_spectrum(kw):
    """Q_s A Q_s^{-1} is block diagonal with blocks sum_j (-1)^{|a&j|} H_j
    (eqs. (2.12)-(2.13)); its blocks' eigenvalues are A's."""
    p = make_problem((8, 6, 4), s=2, seed=7, **kw)
    H = symmetry.base_blocks(p.A, p.img)
    n_b, S = p.img.shape
    Am = symmetry.to_mirrored(p.A, p.img).toarray()
    Q = symmetry.q_matrix(S.bit_length() - 1, n_b).toarray()
    Ah = Q @ Am @ Q
    scale = np.abs(Am).max()
    evs = []
    for a in range(S):
        for b in range(S):
            blk = Ah[a * n_b:(a + 1) * n_b, b * n_b:(b + 1) * n_b]
            if a != b:
                assert np.abs(blk).max() <= 1e-14 * scale
        sub = symmetry.subsystem(H, a).toarray()
        assert np.abs(Ah[a * n_b:(a + 1) * n_b, a * n_b:(a + 1) * n_b] - sub).max() <= 1e-14 * scale
        Ainn, outs = symmetry.inner_outer(H)
        assert np.abs((Ainn + outs[a]).toarray() - sub).max() <= 1e-15 * scale
        evs.append(np.linalg.eigvalsh(sub))
    ev_all = np.sort(np.concatenate(evs))
    assert np.abs(ev_all - np.linalg.eigvalsh(Am)).max() < 1e-12 * scale


def test_subsystem_modes_closed_form():
    """Uniform cube, s = 3: subsystem a owns exactly the Dirichlet modes with
    k_t even (antisymmetric about plane t) iff bit t of a is set."""
    N = 6
    p = make_problem((N, N, N), s=3, seed=3)
    H = symmetry.base_blocks(p.A, p.img)
    h = 1.0 / N
    l1 = _dirichlet_1d(N)
    ks = np.arange(1, N + 1)
    for a in range(8):
        sel = [ks[(ks % 2 == 0) == bool((a >> t) & 1)] for t in range(3)]
        lam = (l1[sel[0] - 1][:, None, None] + l1[sel[1] - 1][None, :, None]
               + l1[sel[2] - 1][None, None, :]) * h
        ev = np.linalg.eigvalsh(symmetry.subsystem(H, a).toarray())
        assert np.abs(np.sort(lam.ravel()) - ev).max() < 1e-13


@pytest.mark.parametrize("kw", [dict(), dict(y_stretch=1.5), dict(jitter=0.2, kappa="lognormal")])
def test_reduced_solve_matches_direct(kw):
    """Alg. 1 with exact decoupled solves reproduces a dense direct solve of
    A x = b to 1e-12."""
    p = make_problem((8, 8, 6), s=2, m=3, seed=11, **kw)
    H = symmetry.base_blocks(p.A, p.img)
    n_b, S = p.img.shape
    bh = symmetry.forward_transform(p.b, p.img)
    xh = np.stack([np.linalg.solve(symmetry.subsystem(H, a).toarray(), bh[a]) for a in range(S)])
    x = symmetry.backward_transform(xh, p.img)
    xd = np.linalg.solve(p.A.toarray(), p.b)
    assert np.abs(x - xd).max() <= 1e-12 * np.abs(xd).max()


def test_mirror_symmetric_rhs_has_one_nonzero_subsystem():
    """A right-hand side symmetric about every plane transforms to zero in
    every subsystem but a = 0."""
    p = make_problem((8, 8, 8), s=3, seed=1)
    base = np.random.default_rng(0).standard_normal(p.n_b)
    b = np.zeros(p.n)
    for a in range(8):
        b[p.img[:, a]] = base
    bh = symmetry.forward_transform(b[:, None], p.img)
    assert np.abs(bh[1:]).max() < 1e-15 * np.abs(bh[0]).max()
