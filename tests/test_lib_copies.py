"""Host-side parity of the library's setup for domains made of copies
(msp_setup_copies) with the oracle's AMGR in the original basis
(oracle/copies.py): the interface of the copies, the replicated populated
interface of Alg. 2, and every level of the hierarchy (P = [W; I] of
eq. (3.13), the block FSAI of eq. (3.14), the reduced operator of eq. (3.15)
and the standard levels below), bit for bit in the patterns and splits; plus
input validation.  No GPU needed."""
import numpy as np
import pytest

from gen import make_problem, make_repeated_problem
from oracle import amg, copies

CASES = [
    dict(N=(8, 7, 6), copies=4, mirror=False, walls="mixed", opt=dict(coarse_max=40)),
    dict(N=(10, 9, 7), copies=2, mirror=True, walls="mixed", opt=dict(coarse_max=40)),
    dict(N=(24, 20), copies=5, mirror=False, walls="dirichlet", opt=dict(coarse_max=40)),
    dict(N=(16, 12, 10), copies=3, mirror=True, walls="dirichlet", opt=dict(coarse_max=64, dist=3, jacobi0=2)),
    dict(N=(24, 20, 16), copies=4, mirror=False, walls="mixed", opt=dict()),
    dict(N=(8, 7, 6), copies=4, mirror=False, walls="mixed", opt=dict(coarse_max=40, afsai_nnz=5, emin_steps=4)),
    dict(N=(10, 9, 7), copies=2, mirror=True, walls="mixed", opt=dict(coarse_max=40, afsai_nnz=5, emin_steps=4)),
]
IDS = ["repeated4_mixed", "mirrored2_mixed", "2d_repeated5", "mirrored3_d3", "repeated4_default",
       "repeated4_mixed_afsai_emin", "mirrored2_mixed_afsai_emin"]


def _setup(p, **kw):
    from paper_2407_05930_amd import Solver
    return Solver.from_copies(p.A, p.sub, device=-1, **kw)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_copies_hierarchy_bit_exact_with_oracle(case):
    p = make_repeated_problem(case["N"], case["copies"], seed=3, mirror=case["mirror"], walls=case["walls"])
    sv = _setup(p, **case["opt"])
    ctx = copies.setup(p.A, p.sub, amg.AMGOptions(**case["opt"]))
    sigma, iface = sv.export_outer()
    assert np.array_equal(iface, ctx["interface"])
    assert iface.any() and not iface.all()
    assert sigma.shape == (p.n, 1) and not sigma.any()
    H = ctx["hier"]
    assert sv.num_levels() == H.nlev >= 3
    for lev in range(H.nlev):
        e = sv.export_level(lev)
        L = H.levels[lev]
        assert np.array_equal(e["A"].indptr, L.A.indptr)
        assert np.array_equal(e["A"].indices, L.A.indices)
        assert np.abs(e["A"].data - L.A.data).max() <= 1e-12 * np.abs(L.A.data).max()
        if L.C is not None:
            assert np.array_equal(e["cf"], L.C)
            for key in ("P", "G"):
                M1, M2 = e[key], getattr(L, key)
                assert np.array_equal(M1.indptr, M2.indptr) and np.array_equal(M1.indices, M2.indices)
                assert np.abs(M1.data - M2.data).max() <= 1e-12 * np.abs(M2.data).max()
            assert abs(e["omega"] - L.omega) <= 1e-10 * L.omega
    assert np.array_equal(sv.export_level(0)["cf"], ctx["C"])
    assert abs(sv.stats.op_complexity - H.stats()["op_complexity"]) < 1e-12


def test_one_copy_matches_the_plain_reduction_level():
    """One copy: no interface, and the hierarchy is the msp_setup one of the
    same matrix with s = 0 (identity map)."""
    from paper_2407_05930_amd import Solver
    p = make_problem((12, 10, 8), s=0, seed=3, y_stretch=1.5)
    sub = np.arange(p.n, dtype=np.int64)[:, None]
    a = Solver.from_copies(p.A, sub, device=-1, coarse_max=40)
    b = Solver(p.A, p.img, device=-1, coarse_max=40)
    assert not a.export_outer()[1].any()
    assert a.num_levels() == b.num_levels()
    for lev in range(a.num_levels()):
        ea, eb = a.export_level(lev), b.export_level(lev)
        assert (ea["A"] != eb["A"]).nnz == 0
        if "cf" in eb:
            assert np.array_equal(ea["cf"], eb["cf"]) and (ea["P"] != eb["P"]).nnz == 0


def test_copies_setup_rejects_bad_inputs():
    from paper_2407_05930_amd import MspError, Solver
    p = make_repeated_problem((6, 5, 4), 3, seed=4)
    sub = p.sub.copy()
    sub[0, 1] = sub[1, 1]                                    # not a permutation
    with pytest.raises(MspError) as e:
        Solver.from_copies(p.A, sub, device=-1)
    assert e.value.status == -3
    with pytest.raises(MspError) as e:                       # n != n_b * copies
        Solver.from_copies(p.A, p.sub[:-1], device=-1)
    assert e.value.status == -1
    with pytest.raises(MspError) as e:                       # per-subsystem cycle needs Q_s
        Solver.from_copies(p.A, p.sub, device=-1, pc="amgr_sub")
    assert e.value.status == -1
    A = p.A.tolil()
    A[0, 1] += 1e-3                                          # breaks exact symmetry
    with pytest.raises(MspError) as e:
        Solver.from_copies(A.tocsr(), p.sub, device=-1)
    assert e.value.status == -2


def test_copies_setup_takes_fsai_and_no_preconditioner():
    p = make_repeated_problem((6, 5, 4), 3, seed=5, walls="mixed")
    for pc in ("fsai", "none"):
        sv = _setup(p, pc=pc)
        assert sv.num_levels() == 1
