"""Host-side parity of the library's AMGS setup (pc="amgs", Sec. 3.1) with the
oracle (oracle/amgs.py): the inner-first order of the base cells, the blocks
K, B, C_1 (eq. (3.1)), the AMG of K level by level, the FSAI of K, the
approximate Schur complement S_G1 (eq. (3.4)) and its FSAI (eq. (3.9)).
No GPU needed."""
import numpy as np
import pytest

from gen import make_problem
from oracle import amg, amgs

CASES = [
    dict(N=(16, 14, 12), s=2, kw=dict(y_stretch=1.5), opt=dict(coarse_max=40)),
    dict(N=(12, 12, 10), s=3, kw=dict(jitter=0.2, kappa="lognormal"), opt=dict(coarse_max=40)),
    dict(N=(48, 40), s=1, kw=dict(), opt=dict(coarse_max=40)),
    dict(N=(24, 24, 24), s=3, kw=dict(y_stretch=1.5), opt=dict()),
]
IDS = ["3d_s2_stretched", "3d_s3_jitter", "2d_s1", "24cube_s3"]


def _same(M1, M2, rel=1e-12, exact=False):
    M1, M2 = M1.tocsr(), M2.tocsr()
    M1.eliminate_zeros()
    M2.eliminate_zeros()
    M1.sort_indices()
    M2.sort_indices()
    assert M1.shape == M2.shape
    assert np.array_equal(M1.indptr, M2.indptr) and np.array_equal(M1.indices, M2.indices)
    if exact:
        assert np.array_equal(M1.data, M2.data)
    else:
        assert np.abs(M1.data - M2.data).max() <= rel * np.abs(M2.data).max()


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_amgs_setup_matches_oracle(case):
    from paper_2407_05930_amd import Solver
    p = make_problem(case["N"], s=case["s"], seed=11, **case["kw"])
    sv = Solver(p.A, p.img, device=-1, pc="amgs", **case["opt"])
    ctx = amgs.setup(p.A, p.img, amgs.AMGSOptions(amg=amg.AMGOptions(**case["opt"])))
    inner, ifc = ctx["inner"], ctx["ifc"]
    perm = np.concatenate([inner, ifc])
    sigma, iface = sv.export_outer()
    assert np.array_equal(iface, np.arange(p.n_b) >= inner.size)
    S = 1 << p.s
    ref_sigma = np.stack([o.diagonal() for o in ctx["outs"]], axis=1)[perm]
    assert np.abs(sigma - ref_sigma).max() <= 1e-15 * np.abs(p.A.data).max()
    _same(sv.export_amgs("B"), ctx["B"], exact=True)
    _same(sv.export_amgs("C1"), ctx["C1"], exact=True)
    _same(sv.export_amgs("GK"), ctx["GK"])
    _same(sv.export_amgs("SG1"), ctx["SG1"])
    _same(sv.export_amgs("GS1"), ctx["GS1"])
    H = ctx["HK"]
    assert sv.num_levels() == H.nlev
    for lev in range(H.nlev):
        e = sv.export_level(lev)
        L = H.levels[lev]
        _same(e["A"], L.A)
        if L.C is not None:
            assert np.array_equal(e["cf"], L.C)
            _same(e["P"], L.P)
            _same(e["G"], L.G)
            assert abs(e["omega"] - L.omega) <= 1e-10 * L.omega
    assert S == sigma.shape[1]


def test_amgs_options_are_validated():
    from paper_2407_05930_amd import MspError, Solver
    p = make_problem((8, 8, 6), s=1, seed=2)
    for kw, status in ((dict(pc="amgs", precision="mixed"), -8), (dict(pc="amgs", amgs_light=2), -1),
                       (dict(pc="amgs", schur_tau=-1.0), -1)):
        with pytest.raises(MspError) as e:
            Solver(p.A, p.img, device=-1, **kw)
        assert e.value.status == status, kw
    Solver(p.A, p.img, device=-1, pc="amgs", amgs_light=1, schur_tau=0.05)
