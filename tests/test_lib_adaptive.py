"""Host setup with the adaptive FSAI pattern and energy-minimising
interpolation options against the oracle: every level's C/F split and
patterns bit for bit (the adaptive patterns included), values to 1e-12 times
the interpolation's row-sum cancellation factor, per-subsystem values too."""
import numpy as np
import pytest

from gen import make_problem
from oracle import amg, krylov


def _cancel(P):
    W = abs(P)
    return float((np.asarray(W.sum(axis=1)).ravel() /
                  np.maximum(np.abs(np.asarray(P.sum(axis=1)).ravel()), 1e-300)).max())


def _close(M1, M2, tol):
    assert np.array_equal(M1.indptr, M2.indptr) and np.array_equal(M1.indices, M2.indices)
    assert np.abs(M1.data - M2.data).max() <= tol * np.abs(M2.data).max()


CASES = [
    dict(name="afsai5_emin4_s3", N=(20, 16, 12), s=3, kw=dict(y_stretch=1.5), af=5, em=4),
    dict(name="afsai5_s2_jitter", N=(24, 20, 16), s=2, kw=dict(jitter=0.2, kappa="lognormal"), af=5, em=0),
    dict(name="emin6_s1_lognormal", N=(24, 20, 16), s=1, kw=dict(kappa="lognormal"), af=0, em=6),
    dict(name="afsai3_emin2_2d", N=(64, 48), s=1, kw=dict(), af=3, em=2),
]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
@pytest.mark.parametrize("pc", ["amgr", "amgr_sub"])
def test_adaptive_hierarchy_matches_oracle(case, pc):
    from paper_2407_05930_amd import Solver
    p = make_problem(case["N"], s=case["s"], seed=3, **case["kw"])
    opt = dict(coarse_max=48, afsai_nnz=case["af"], emin_steps=case["em"])
    sv = Solver(p.A, p.img, device=-1, pc=pc, **opt)
    ctx = krylov.setup(p.A, p.img, amg.AMGOptions(**opt), precond=pc)
    H = ctx["hier"]
    assert sv.num_levels() == H.nlev >= 3
    amp = 1.0
    for lev in range(H.nlev):
        e = sv.export_level(lev)
        L = H.levels[lev]
        _close(e["A"], L.A, 1e-12 * amp)
        if L.C is None:
            continue
        assert np.array_equal(e["cf"], L.C)
        if case["af"]:
            assert np.all(np.diff(L.G.indptr) <= case["af"])
        amp = max(amp, _cancel(L.P))
        _close(e["P"], L.P, 1e-12 * amp)
        _close(e["G"], L.G, 1e-12 * amp)
        assert abs(e["omega"] - L.omega) <= 1e-10 * L.omega
    if pc == "amgr_sub":
        for a, SH in enumerate(ctx["sub"].subs):
            amp_a = amp
            for lev in range(1, H.nlev):
                e = sv.export_sub_level(lev, a)
                L = SH.levels[lev - 1]
                _close(e["A"], L.A, 1e-12 * amp_a)
                if L.P is not None:
                    amp_a = max(amp_a, _cancel(L.P))
                    _close(e["P"], L.P, 1e-12 * amp_a)
                    _close(e["G"], L.G, 1e-12 * amp_a)
                    assert abs(e["omega"] - L.omega) <= 1e-10 * L.omega


def test_adaptive_options_are_validated():
    from paper_2407_05930_amd import MspError, Solver
    p = make_problem((12, 10, 8), s=2, seed=4)
    for kw in (dict(afsai_nnz=65), dict(afsai_nnz=-1), dict(emin_steps=101), dict(emin_steps=-2)):
        with pytest.raises(MspError) as e:
            Solver(p.A, p.img, device=-1, coarse_max=32, **kw)
        assert e.value.status == -1
    for kw in (dict(afsai_nnz=5), dict(emin_steps=3)):
        with pytest.raises(MspError) as e:
            Solver(p.A, p.img, device=-1, coarse_max=32, pc="amgs", **kw)
        assert e.value.status == -8
