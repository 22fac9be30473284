"""msp_rebuild_below on host-only contexts (CPU): rebuilding a setup below
its reduction level reproduces it bit for bit (every level of the shared
hierarchy, every subsystem's values), for the symmetric-domain setup and for
a domain of copies; the hierarchy also equals the oracle's rebuild; the
argument checks."""
import numpy as np
import pytest

from gen import make_problem, make_repeated_problem
from oracle import amg, krylov, refresh


def _exports(sv, sub):
    out = [sv.export_level(lev) for lev in range(sv.num_levels())]
    if sub:
        out += [sv.export_sub_level(lev, a) for lev in range(1, sv.num_levels()) for a in range(1 << sv.s)]
    return out


def _identical(e0, e1):
    assert len(e0) == len(e1)
    for a, b in zip(e0, e1):
        assert a.keys() == b.keys()
        for k in a:
            x, y = a[k], b[k]
            if hasattr(x, "indptr"):
                assert np.array_equal(x.indptr, y.indptr) and np.array_equal(x.indices, y.indices), k
                assert np.array_equal(x.data, y.data), k
            else:
                assert np.array_equal(np.asarray(x), np.asarray(y)), k


@pytest.mark.parametrize("pc", ["amgr", "amgr_sub"])
@pytest.mark.parametrize("f3", [False, True], ids=["static", "afsai_emin"])
def test_rebuild_of_a_setup_reproduces_it(pc, f3):
    from paper_2407_05930_amd import Solver
    p = make_problem((24, 20, 16), s=3, m=1, seed=63, y_stretch=1.5, kappa="lognormal")
    opt = dict(coarse_max=48, afsai_nnz=5 if f3 else 0, emin_steps=4 if f3 else 0)
    sv = Solver(p.A, p.img, device=-1, pc=pc, **opt)
    assert sv.num_levels() >= 4
    e0 = _exports(sv, pc == "amgr_sub")
    sv.rebuild_below()
    assert sv.version == 1
    _identical(e0, _exports(sv, pc == "amgr_sub"))
    # and the oracle's rebuild of its own setup is that same hierarchy
    ctx = refresh.rebuild_below(krylov.setup(p.A, p.img, amg.AMGOptions(**opt), precond=pc))
    for lev, L in enumerate(ctx["hier"].levels):
        e = sv.export_level(lev)
        assert np.array_equal(e["A"].indices, L.A.indices)
        if L.C is not None:
            assert np.array_equal(e["cf"].astype(bool), L.C)
            assert np.array_equal(e["P"].indices, L.P.indices) and np.array_equal(e["G"].indices, L.G.indices)


def test_rebuild_of_a_domain_of_copies_reproduces_it():
    from paper_2407_05930_amd import Solver
    p = make_repeated_problem((12, 10, 8), 3, m=1, seed=64, walls="mixed")
    sv = Solver.from_copies(p.A, p.sub, device=-1, coarse_max=40)
    assert sv.num_levels() >= 3
    e0 = _exports(sv, False)
    sv.rebuild_below()
    _identical(e0, _exports(sv, False))


@pytest.mark.parametrize("pc", ["amgr", "amgr_sub"])
def test_rebuild_of_a_two_level_setup_reproduces_it(pc):
    """With two levels the level below the reduction level is the coarsest
    one, which the rebuild only recomputes (its dense inverses too)."""
    from paper_2407_05930_amd import Solver
    p = make_problem((12, 10, 8), s=2, m=1, seed=67, kappa="lognormal")
    sv = Solver(p.A, p.img, device=-1, pc=pc, coarse_max=200)
    assert sv.num_levels() == 2
    e0 = _exports(sv, pc == "amgr_sub")
    sv.rebuild_below()
    assert sv.num_levels() == 2
    _identical(e0, _exports(sv, pc == "amgr_sub"))


def test_rebuild_with_device_values_needs_a_device_context():
    import ctypes
    from paper_2407_05930_amd import Solver, _lib
    p = make_problem((12, 10, 8), s=2, m=1, seed=66)
    sv = Solver(p.A, p.img, device=-1, coarse_max=32)
    out = ctypes.c_void_p()
    assert _lib.lib.msp_rebuild_below(sv._ctx, ctypes.c_void_p(16), None, ctypes.byref(out)) == -1
    assert "device" in _lib.lib.msp_last_error().decode() and not out.value
    assert _lib.lib.msp_rebuild_below(sv._ctx, None, None, None) == -1


def test_rebuild_rejects_what_it_cannot_rebuild():
    from paper_2407_05930_amd import MspError, Solver
    p = make_problem((12, 10, 8), s=2, m=1, seed=65)
    for kw, status in ((dict(pc="fsai"), -8), (dict(pc="none"), -8), (dict(pc="amgs", coarse_max=32), -8),
                       (dict(coarse_max=100000), -1)):
        sv = Solver(p.A, p.img, device=-1, **kw)
        with pytest.raises(MspError) as e:
            sv.rebuild_below()
        assert e.value.status == status, kw
        assert sv.version == 0
