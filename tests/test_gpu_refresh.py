"""GPU parity of the numeric re-setup on the device (msp_refresh) against the
oracle's re-setup (oracle/refresh.py) and against fresh setups: every level's
values, the dampings, the low-rank corrections and the solves that follow."""
import sys

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gen import make_problem
from oracle import amg, krylov, refresh

pytestmark = pytest.mark.gpu

TOL = 1e-13


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cancel(P):
    """sum |w| / |sum w| over P's rows: the factor by which the row rescaling
    of eq. (3.13) amplifies rounding differences in the weights."""
    W = abs(P)
    return float((np.asarray(W.sum(axis=1)).ravel() /
                  np.maximum(np.abs(np.asarray(P.sum(axis=1)).ravel()), 1e-300)).max())


def _close(M1, M2, tol):
    assert np.array_equal(M1.indptr, M2.indptr) and np.array_equal(M1.indices, M2.indices)
    assert np.abs(M1.data - M2.data).max() <= tol * np.abs(M2.data).max()


def _check_levels(sv, H, sub=None, base=1e-12):
    """Library levels (shared, then per subsystem) against the oracle's
    hierarchy H (and its subsystem hierarchies), patterns bit for bit."""
    assert sv.num_levels() == H.nlev
    amp = 1.0
    shared = H.nlev if sub is None else 1
    for lev in range(H.nlev):
        if lev >= shared and lev > 0:
            break
        e = sv.export_level(lev)
        L = H.levels[lev]
        _close(e["A"], L.A, base * amp)
        if L.C is not None:
            assert np.array_equal(e["cf"], L.C)
            amp = max(amp, _cancel(L.P))
            _close(e["P"], L.P, base * amp)
            _close(e["G"], L.G, base * amp)
            assert abs(e["omega"] - L.omega) <= 1e-10 * L.omega
    if sub is None:
        return
    for a, SH in enumerate(sub.subs):
        amp_a = amp
        for lev in range(1, H.nlev):
            e = sv.export_sub_level(lev, a)
            L = SH.levels[lev - 1]
            _close(e["A"], L.A, base * amp_a)
            if L.P is not None:
                amp_a = max(amp_a, _cancel(L.P))
                _close(e["P"], L.P, base * amp_a)
                _close(e["G"], L.G, base * amp_a)
                assert abs(e["omega"] - L.omega) <= 1e-10 * L.omega


def _snapshot(sv, nlev, sub):
    out = [sv.export_level(lev) for lev in range(nlev)]
    if sub:
        out += [sv.export_sub_level(lev, a) for a in range(sub) for lev in range(1, nlev)]
    return out


def _same(s1, s2, tol):
    assert len(s1) == len(s2)
    for e1, e2 in zip(s1, s2):
        for key in ("A", "P", "G"):
            if key in e2:
                _close(e1[key], e2[key], tol)
        assert abs(e1["omega"] - e2["omega"]) <= 1e-10 * max(abs(e2["omega"]), 1e-300)


@pytest.mark.parametrize("pc,k,f3", [("amgr", 0, False), ("amgr_sub", 0, False), ("amgr", 4, False),
                                     ("amgr_sub", 4, False), ("amgr_sub", 4, True)])
def test_refresh_with_the_setup_values_reproduces_the_setup(pc, k, f3):
    """The re-setup from the setup matrix's own values gives the setup's
    hierarchy again, and the solve afterwards takes the same iterations (also
    with adaptive FSAI patterns and energy minimisation)."""
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("refresh same values", pc, k, f3)
    p = make_problem((24, 20, 16), s=3, m=2, seed=31, y_stretch=1.5, kappa="lognormal")
    opt = dict(coarse_max=48, **(dict(afsai_nnz=5, emin_steps=4) if f3 else {}))
    sv = Solver(p.A, p.img, tol=TOL, pc=pc, k=k, **opt)
    nlev = sv.num_levels()
    S = 8 if pc == "amgr_sub" else 0
    before = _snapshot(sv, nlev, S)
    kept0, ritz0 = sv.export_lrc() if k else (None, None)
    b = torch.from_numpy(p.b).cuda()
    x0 = sv.solve(b).cpu().numpy()
    it0 = sv.last.iters
    sv.refresh(torch.from_numpy(p.A.data).cuda())
    torch.cuda.synchronize()
    _same(_snapshot(sv, nlev, S), before, 1e-12)
    if k:
        kept, ritz = sv.export_lrc()
        assert np.array_equal(kept, kept0)
        assert np.abs(ritz - ritz0).max() <= 1e-8 * max(1.0, np.abs(ritz0).max())
    x = sv.solve(b).cpu().numpy()
    _say("its before", it0, "after", sv.last.iters)
    assert abs(sv.last.iters - it0) <= (1 if k else 0)
    assert np.linalg.norm(x - x0) <= 1e-9 * np.linalg.norm(x0)


NEW_CASES = [
    dict(name="amgr_s3", pc="amgr", k=0, N=(24, 20, 16), s=3, m=2, kw=dict(y_stretch=1.5)),
    dict(name="amgr_sub_s3", pc="amgr_sub", k=0, N=(24, 20, 16), s=3, m=2, kw=dict(y_stretch=1.5)),
    dict(name="amgr_s2_jitter", pc="amgr", k=0, N=(28, 24, 20), s=2, m=1, kw=dict(jitter=0.2)),
    dict(name="amgr_sub_s2_lrc", pc="amgr_sub", k=4, N=(20, 16, 16), s=2, m=3, kw=dict(y_stretch=1.5)),
    dict(name="amgr_s3_lrc", pc="amgr", k=8, N=(16, 16, 16), s=3, m=2, kw=dict(y_stretch=1.5)),
    dict(name="amgr_2d_s1", pc="amgr", k=0, N=(64, 48), s=1, m=2, kw=dict()),
]


@pytest.mark.parametrize("case", NEW_CASES, ids=[c["name"] for c in NEW_CASES])
def test_refresh_for_a_new_coefficient_matches_the_oracle(case):
    """A new lognormal kappa on the same mesh: every level, damping and Ritz
    value of the device re-setup equals the oracle's re-setup on the kept
    structure, and the solve matches the oracle's (iterations equal, or within
    one with low-rank corrections; x within 1e-9) and the direct solution."""
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("refresh new kappa", case["name"])
    kw = dict(case["kw"], kappa="lognormal")
    p0 = make_problem(case["N"], s=case["s"], m=case["m"], seed=41, **kw)
    p1 = make_problem(case["N"], s=case["s"], m=case["m"], seed=42, **kw)
    assert np.array_equal(p0.A.indices, p1.A.indices) and np.array_equal(p0.A.indptr, p1.A.indptr)
    opt = dict(coarse_max=48)
    pc, k = case["pc"], case["k"]
    ctx0 = krylov.setup(p0.A, p0.img, amg.AMGOptions(**opt), precond=pc, k=k)
    ctx1 = refresh.refresh(ctx0, p1.A)
    ref = krylov.solve(ctx1, p1.b, tol=TOL)
    sv = Solver(p0.A, p0.img, tol=TOL, pc=pc, k=k, **opt)
    sv.refresh(torch.from_numpy(p1.A.data).cuda())
    torch.cuda.synchronize()
    _check_levels(sv, ctx1["hier"], ctx1["sub"])
    if k:
        kept, ritz = sv.export_lrc()
        for a in range(1 << p1.s):
            r_or = np.asarray(ctx1["lrc"].ritz[a])
            assert np.abs(ritz[a][:r_or.size] - r_or).max() <= 1e-8 * max(1.0, np.abs(r_or).max())
            assert kept[a] == ctx1["lrc"].U[a].shape[1]
    x = sv.solve(torch.from_numpy(p1.b).cuda()).cpu().numpy()
    _say("its gpu", sv.last.iters, "oracle", ref.iters.max())
    assert abs(sv.last.iters - int(ref.iters.max())) <= (1 if k else 0)
    xr = ref.x.reshape(p1.n, -1)
    x = x.reshape(p1.n, -1)
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)
    assert np.all(np.abs(x - xr).max(axis=0) <= 1e-9 * np.abs(xr).max(axis=0))
    lu = spla.splu(p1.A.tocsc())
    xd = np.stack([lu.solve(p1.b.reshape(p1.n, -1)[:, j]) for j in range(xr.shape[1])], axis=1)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


@pytest.mark.parametrize("pc", ["amgr", "amgr_sub"])
def test_refresh_of_a_scaled_matrix_is_its_fresh_setup(pc):
    """2A makes the fresh setup's structural decisions again (they are scale
    invariant): the re-setup equals the library's fresh setup of 2A."""
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("refresh scaled", pc)
    p = make_problem((20, 16, 16), s=3, m=1, seed=33, jitter=0.2, kappa="lognormal")
    opt = dict(coarse_max=48)
    A2 = (2.0 * p.A).tocsr()
    sv = Solver(p.A, p.img, tol=TOL, pc=pc, **opt)
    fresh = Solver(A2, p.img, tol=TOL, pc=pc, **opt)
    nlev = fresh.num_levels()
    S = 8 if pc == "amgr_sub" else 0
    sv.refresh(torch.from_numpy(A2.data).cuda())
    torch.cuda.synchronize()
    _same(_snapshot(sv, nlev, S), _snapshot(fresh, nlev, S), 1e-12)
    b = torch.from_numpy(p.b).cuda()
    x1 = sv.solve(b).cpu().numpy()
    it1 = sv.last.iters
    x2 = fresh.solve(b).cpu().numpy()
    assert it1 == fresh.last.iters
    assert np.linalg.norm(x1 - x2) <= 1e-10 * np.linalg.norm(x2)


def test_refresh_with_fsai_matches_the_oracle():
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("refresh fsai")
    p0 = make_problem((20, 16, 16), s=3, m=2, seed=51, kappa="lognormal")
    p1 = make_problem((20, 16, 16), s=3, m=2, seed=52, kappa="lognormal")
    ctx = krylov.setup(p1.A, p1.img, precond="fsai")
    ref = krylov.solve(ctx, p1.b, tol=TOL)
    sv = Solver(p0.A, p0.img, tol=TOL, pc="fsai")
    sv.refresh(torch.from_numpy(p1.A.data).cuda())
    x = sv.solve(torch.from_numpy(p1.b).cuda()).cpu().numpy()
    _say("fsai its gpu", sv.last.iters, "oracle", ref.iters.max())
    assert sv.last.iters == int(ref.iters.max())
    assert np.linalg.norm(x - ref.x) <= 1e-9 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("prec,pc", [("mixed", "amgr"), ("mixed_bf16", "amgr_sub"), ("mixed", "amgr_sub")])
def test_refresh_in_mixed_precision_reaches_tolerance(prec, pc):
    """The single- and half-precision copies of the values follow the
    re-setup: after it, the mixed-precision solves reach the tolerance on the
    new matrix and agree with the FP64 oracle's re-setup solve."""
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("refresh mixed", prec, pc)
    p0 = make_problem((24, 24, 24), s=3, m=2, seed=61, y_stretch=1.5, kappa="lognormal")
    p1 = make_problem((24, 24, 24), s=3, m=2, seed=62, y_stretch=1.5, kappa="lognormal")
    opt = dict(coarse_max=64)
    ctx1 = refresh.refresh(krylov.setup(p0.A, p0.img, amg.AMGOptions(**opt), precond=pc), p1.A)
    ref = krylov.solve(ctx1, p1.b, tol=1e-12)
    sv = Solver(p0.A, p0.img, tol=1e-10, precision=prec, pc=pc, **opt)
    sv.refresh(torch.from_numpy(p1.A.data).cuda())
    x = sv.solve(torch.from_numpy(p1.b).cuda()).cpu().numpy()
    rr = krylov.true_relres(p1.A, x, p1.b)
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    _say("its", sv.last.iters, "oracle", ref.iters.max(), "relres", rr, "err", err)
    assert np.all(rr <= 1.5e-10)
    assert err <= 1e-7
    assert sv.last.iters <= int(ref.iters.max()) + 3


def test_refresh_of_a_domain_of_copies_solves_the_new_matrix():
    """AMGR in the original basis (a domain of copies): the re-setup from the
    setup values equals the setup, and for new values the solve reaches the
    direct solution."""
    torch = _torch()
    from gen import make_repeated_problem
    from paper_2407_05930_amd import Solver
    _say("refresh copies")
    p0 = make_repeated_problem((12, 10, 8), 3, m=1, seed=71, walls="mixed")
    p1 = make_repeated_problem((12, 10, 8), 3, m=1, seed=72, walls="mixed")
    assert np.array_equal(p0.A.indices, p1.A.indices) and not np.array_equal(p0.A.data, p1.A.data)
    sv = Solver.from_copies(p0.A, p0.sub, tol=TOL, coarse_max=48)
    nlev = sv.num_levels()
    before = _snapshot(sv, nlev, 0)
    sv.refresh(torch.from_numpy(p0.A.data).cuda())
    torch.cuda.synchronize()
    _same(_snapshot(sv, nlev, 0), before, 1e-12)
    sv.refresh(torch.from_numpy(p1.A.data).cuda())
    b = p1.b.reshape(p1.A.shape[0], -1)[:, 0].copy()
    x = sv.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    xd = spla.splu(p1.A.tocsc()).solve(b)
    _say("copies its", sv.last.iters)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


def test_refresh_rejects_what_it_does_not_rebuild():
    torch = _torch()
    from paper_2407_05930_amd import MspError, Solver
    p = make_problem((12, 10, 8), s=2, m=1, seed=81)
    v = torch.from_numpy(p.A.data).cuda()
    for kw in (dict(pc="amgs"), dict(pc="amgr", precision="mixed_bf16g")):
        _say("refresh rejects", kw)
        sv = Solver(p.A, p.img, coarse_max=32, **kw)
        with pytest.raises(MspError) as e:
            sv.refresh(v)
        assert e.value.status == -8
    with pytest.raises(ValueError):
        Solver(p.A, p.img, coarse_max=32).refresh(v.float())
    host = Solver(p.A, p.img, coarse_max=32, device=-1)
    with pytest.raises(MspError):
        host.refresh(v)


@pytest.mark.parametrize("pc", ["amgr", "amgr_sub"])
def test_two_refreshes_then_a_new_column_count_and_exports(pc):
    """The host copy of the values is fetched lazily: after two re-setups in a
    row, a solve with a column count not seen before (its kernel choices are
    tuned then, and sliced forms built from the host copy) and the exports
    all see the second matrix, as the oracle's re-setup gives it."""
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("refresh twice", pc)
    kw = dict(y_stretch=1.5, kappa="lognormal")
    p0 = make_problem((24, 20, 16), s=3, m=2, seed=91, **kw)
    p1 = make_problem((24, 20, 16), s=3, m=2, seed=92, **kw)
    p2 = make_problem((24, 20, 16), s=3, m=5, seed=93, **kw)
    opt = dict(coarse_max=48)
    sv = Solver(p0.A, p0.img, tol=TOL, pc=pc, **opt)
    sv.solve(torch.from_numpy(p0.b).cuda())
    sv.refresh(torch.from_numpy(p1.A.data).cuda())
    sv.refresh(torch.from_numpy(p2.A.data).cuda())
    ctx2 = refresh.refresh(krylov.setup(p0.A, p0.img, amg.AMGOptions(**opt), precond=pc), p2.A)
    ref = krylov.solve(ctx2, p2.b, tol=TOL)
    x = sv.solve(torch.from_numpy(p2.b).cuda()).cpu().numpy()
    _say("its gpu", sv.last.iters, "oracle", ref.iters.max())
    assert sv.last.iters == int(ref.iters.max())
    assert np.linalg.norm(x - ref.x) <= 1e-9 * np.linalg.norm(ref.x)
    _check_levels(sv, ctx2["hier"], ctx2["sub"])
    sigma, _ = sv.export_outer()
    for a in range(8):
        assert np.abs(sigma[:, a] - ctx2["outs"][a].diagonal()).max() <= 1e-15 * np.abs(p2.A.data).max()


@pytest.mark.parametrize("f3", [False, True], ids=["static_fsai", "afsai5_emin4"])
def test_refresh_of_a_deep_hierarchy_matches_the_oracle(f3):
    """Five or more levels (a small coarsest size): every level of every
    subsystem after the device re-setup equals the oracle's re-setup, and so
    do the iteration counts."""
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("refresh deep", f3)
    kw = dict(y_stretch=1.5, kappa="lognormal")
    p0 = make_problem((32, 28, 24), s=3, m=1, seed=95, **kw)
    p1 = make_problem((32, 28, 24), s=3, m=1, seed=96, **kw)
    opt = dict(coarse_max=12, **(dict(afsai_nnz=5, emin_steps=4) if f3 else {}))
    ctx0 = krylov.setup(p0.A, p0.img, amg.AMGOptions(**opt), precond="amgr_sub")
    assert ctx0["hier"].nlev >= 5
    ctx1 = refresh.refresh(ctx0, p1.A)
    ref = krylov.solve(ctx1, p1.b, tol=TOL)
    sv = Solver(p0.A, p0.img, tol=TOL, pc="amgr_sub", **opt)
    sv.refresh(torch.from_numpy(p1.A.data).cuda())
    _check_levels(sv, ctx1["hier"], ctx1["sub"])
    x = sv.solve(torch.from_numpy(p1.b).cuda()).cpu().numpy()
    _say("levels", sv.num_levels(), "its gpu", sv.last.iters, "oracle", ref.iters.max())
    assert sv.last.iters == int(ref.iters.max())
    assert np.linalg.norm(x - ref.x) <= 1e-9 * np.linalg.norm(ref.x)


def test_refresh_of_a_matrix_that_is_not_positive_definite_is_refused():
    """Negated values make every FSAI pivot non-positive: the row kernels
    flag it and finish, and msp_refresh returns MSP_ERR_NOT_SPD."""
    torch = _torch()
    from paper_2407_05930_amd import MspError, Solver
    _say("refresh not SPD")
    p = make_problem((12, 10, 8), s=2, m=1, seed=97)
    sv = Solver(p.A, p.img, coarse_max=32, pc="amgr_sub")
    with pytest.raises(MspError) as e:
        sv.refresh(torch.from_numpy(-p.A.data).cuda())
    assert e.value.status == -7
    with pytest.raises(MspError) as e:                # no solve on the half-updated values
        sv.solve(torch.from_numpy(p.b).cuda())
    assert e.value.status == -1
    sv.refresh(torch.from_numpy(p.A.data).cuda())     # a successful re-setup makes it usable again
    x = sv.solve(torch.from_numpy(p.b).cuda()).cpu().numpy()
    assert np.all(krylov.true_relres(p.A, x, p.b) <= 1e-9)


# "moves": the new kappa changes the split (True), leaves it (False), or either
# (None: on the uniform grid the lognormal kappa leaves every connection strong,
# and at distance 1 this draw moves no decision)
SPLIT_CASES = [
    dict(name="s3_d2", N=(24, 20, 16), s=3, kw=dict(y_stretch=1.5), dist=2, moves=True),
    dict(name="s2_d3_jitter", N=(28, 24, 20), s=2, kw=dict(jitter=0.2), dist=3, moves=True),
    dict(name="s3_d1_jitter", N=(20, 16, 16), s=3, kw=dict(jitter=0.2), dist=1, moves=None),
    dict(name="2d_s1_d2", N=(64, 48), s=1, kw=dict(), dist=2, moves=None),
]


@pytest.mark.parametrize("case", SPLIT_CASES, ids=[c["name"] for c in SPLIT_CASES])
def test_refresh_reports_how_far_the_kept_split_is_from_a_fresh_one(case):
    """msp_stats.split_drift: the device redoes Alg. 2 for the new values
    (strength, distance-d independent set under the setup's priorities) and
    counts the points whose C/F decision differs from the kept split.  Zero
    for the setup values and for 2A; for a new kappa exactly the points where
    a fresh host setup's split differs."""
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("split drift", case["name"])
    kw = dict(case["kw"], kappa="lognormal")
    p0 = make_problem(case["N"], s=case["s"], m=1, seed=98, **kw)
    p1 = make_problem(case["N"], s=case["s"], m=1, seed=99, **kw)
    opt = dict(coarse_max=48, dist=case["dist"])
    sv = Solver(p0.A, p0.img, pc="amgr_sub", **opt)
    assert sv.stats.split_drift == -1
    sv.refresh(torch.from_numpy(p0.A.data).cuda())
    assert sv.stats.split_drift == 0
    sv.refresh(torch.from_numpy(2.0 * p0.A.data).cuda())
    assert sv.stats.split_drift == 0
    sv.refresh(torch.from_numpy(p1.A.data).cuda())
    fresh = Solver(p1.A, p1.img, device=-1, pc="amgr_sub", **opt)
    want = int(np.sum(fresh.export_level(0)["cf"] != sv.export_level(0)["cf"]))
    _say("drift", sv.stats.split_drift, "fresh host split differs at", want, "of", p1.n_b)
    assert sv.stats.split_drift == want
    if case["moves"] is not None:
        assert (want > 0) == case["moves"]


@pytest.mark.parametrize("pc", ["amgr", "amgr_sub"])
@pytest.mark.parametrize("f3", [False, True], ids=["static", "afsai_emin"])
def test_refresh_reports_the_level_one_split_drift(pc, f3):
    """msp_stats.split_drift1: the device redoes the standard split of the
    new shared A_1 (strength, distance-1 independent set with the number of
    strong dependants, then the hash, as priority) and counts the points
    whose decision differs from the kept level-1 split; the count must equal
    the oracle's standard coarsening of the exported A_1 against the kept
    split.  Zero for the setup values and for 2A."""
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("level-1 drift", pc, f3)
    kw = dict(y_stretch=1.5, kappa="lognormal")
    p0 = make_problem((28, 24, 20), s=2, m=1, seed=101, **kw)
    p1 = make_problem((28, 24, 20), s=2, m=1, seed=102, **kw)
    opt = dict(coarse_max=48)
    if f3:
        opt.update(afsai_nnz=5, emin_steps=4)
    sv = Solver(p0.A, p0.img, pc=pc, **opt)
    assert sv.num_levels() >= 3
    assert sv.stats.split_drift1 == -1
    sv.refresh(torch.from_numpy(p0.A.data).cuda())
    assert sv.stats.split_drift1 == 0
    sv.refresh(torch.from_numpy(2.0 * p0.A.data).cuda())
    assert sv.stats.split_drift1 == 0
    sv.refresh(torch.from_numpy(p1.A.data).cuda())
    e1 = sv.export_level(1)
    o = amg.AMGOptions()
    C1 = amg.coarsen_standard(e1["A"], 1, o.theta, o.seed)
    want = int(np.sum(C1 != e1["cf"].astype(bool)))
    _say("level-1 drift", sv.stats.split_drift1, "oracle", want, "of", e1["A"].shape[0])
    assert sv.stats.split_drift1 == want
    assert want > 0


def test_level_one_drift_is_not_reported_for_two_levels():
    torch = _torch()
    from paper_2407_05930_amd import Solver
    p = make_problem((12, 10, 8), s=2, m=1, seed=103)
    sv = Solver(p.A, p.img, coarse_max=200, pc="amgr_sub")
    assert sv.num_levels() == 2
    sv.refresh(torch.from_numpy(p.A.data).cuda())
    assert sv.stats.split_drift == 0 and sv.stats.split_drift1 == -1


def test_split_drift_is_not_reported_for_domains_of_copies():
    torch = _torch()
    from gen import make_repeated_problem
    from paper_2407_05930_amd import Solver
    p = make_repeated_problem((8, 7, 6), 3, m=1, seed=100, walls="mixed")
    sv = Solver.from_copies(p.A, p.sub, coarse_max=40)
    sv.refresh(torch.from_numpy(p.A.data).cuda())
    assert sv.stats.split_drift == -1


@pytest.mark.parametrize("pc,k,f3,dev", [("amgr", 0, False, False), ("amgr_sub", 0, False, False),
                                         ("amgr_sub", 4, True, False), ("amgr_sub", 0, False, True),
                                         ("amgr_sub", 4, True, True)])
def test_rebuild_below_after_a_refresh_matches_the_oracle(pc, k, f3, dev):
    """Device re-setup for a new kappa, then msp_rebuild_below: the reduction
    level is the re-set-up one and every level below is built afresh from its
    A_1, as the oracle's rebuild_below of its re-setup does (patterns and
    splits bit for bit, values to the tolerance of the re-setup tests); the
    solve then has the oracle's iteration count with x within 1e-9, and a
    re-setup with the same values finds level 1's split where the rebuild put
    it (split_drift1 = 0).  dev: the per-subsystem values and corrections are
    computed by a device re-setup from the matrix values instead of the host."""
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("rebuild below", pc, k, f3, dev)
    kw = dict(y_stretch=1.5, kappa="lognormal")
    p0 = make_problem((28, 24, 20), s=2, m=1, seed=101, **kw)
    p1 = make_problem((28, 24, 20), s=2, m=1, seed=102, **kw)
    opt = dict(coarse_max=48)
    if f3:
        opt.update(afsai_nnz=5, emin_steps=4)
    sv = Solver(p0.A, p0.img, tol=TOL, pc=pc, k=k, **opt)
    vals = torch.from_numpy(p1.A.data).cuda()
    sv.refresh(vals)
    assert sv.stats.split_drift1 > 0
    sv.rebuild_below(vals if dev else None)
    if dev:
        assert sv.stats.split_drift1 == 0     # the rebuilt split is that of these values
    else:
        assert sv.stats.split_drift == -1 and sv.stats.split_drift1 == -1
    ctx0 = krylov.setup(p0.A, p0.img, amg.AMGOptions(**opt), precond=pc, k=k)
    ref = refresh.rebuild_below(refresh.refresh(ctx0, p1.A))
    _check_levels(sv, ref["hier"], ref["sub"], base=1e-11)
    x = sv.solve(torch.from_numpy(p1.b).cuda()).cpu().numpy()
    r = krylov.solve(ref, p1.b, tol=TOL)
    _say("its gpu", sv.last.iters, "oracle", r.iters.max())
    assert abs(sv.last.iters - int(r.iters.max())) <= (1 if k else 0)
    assert np.linalg.norm(x - r.x) <= 1e-9 * np.linalg.norm(r.x)
    sv.refresh(vals)
    assert sv.stats.split_drift1 == 0
    x2 = sv.solve(torch.from_numpy(p1.b).cuda()).cpu().numpy()
    assert np.linalg.norm(x2 - r.x) <= 1e-9 * np.linalg.norm(r.x)


def test_rebuild_below_of_copies_and_in_mixed_precision():
    """The rebuild after a re-setup for a domain of copies (FP64: the direct
    solution to 1e-9) and for a bfloat16-multivector solver with low-rank
    corrections (the FP64 oracle's rebuild solution to 1e-7, true residual
    to the tolerance); both find level 1's split unmoved on a second
    re-setup with the same values."""
    torch = _torch()
    from gen import make_repeated_problem
    from paper_2407_05930_amd import Solver
    _say("rebuild copies")
    p0 = make_repeated_problem((12, 10, 8), 3, m=1, seed=71, walls="mixed")
    p1 = make_repeated_problem((12, 10, 8), 3, m=1, seed=72, walls="mixed")
    sv = Solver.from_copies(p0.A, p0.sub, tol=TOL, coarse_max=48)
    assert sv.num_levels() >= 3
    vals = torch.from_numpy(p1.A.data).cuda()
    sv.refresh(vals)
    sv.rebuild_below()
    b = p1.b.reshape(p1.A.shape[0], -1)[:, 0].copy()
    x = sv.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    xd = spla.splu(p1.A.tocsc()).solve(b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    sv.refresh(vals)
    assert sv.stats.split_drift1 == 0
    sv.close()
    _say("rebuild mixed_bf16")
    kw = dict(y_stretch=1.5, kappa="lognormal")
    q0 = make_problem((28, 24, 20), s=3, m=2, seed=103, **kw)
    q1 = make_problem((28, 24, 20), s=3, m=2, seed=104, **kw)
    opt = dict(coarse_max=48, afsai_nnz=5, emin_steps=4)
    sm = Solver(q0.A, q0.img, tol=1e-10, pc="amgr_sub", k=4, precision="mixed_bf16", **opt)
    vq = torch.from_numpy(q1.A.data).cuda()
    sm.refresh(vq)
    sm.rebuild_below(vq)
    y = sm.solve(torch.from_numpy(q1.b).cuda()).cpu().numpy()
    ref = krylov.solve(refresh.rebuild_below(refresh.refresh(
        krylov.setup(q0.A, q0.img, amg.AMGOptions(**opt), precond="amgr_sub"), q1.A)), q1.b, tol=1e-12)
    _say("its", sm.last.iters, "oracle (k = 0)", ref.iters.max())
    assert np.all(krylov.true_relres(q1.A, y, q1.b) <= 1.5e-10)
    assert np.linalg.norm(y - ref.x) <= 1e-7 * np.linalg.norm(ref.x)
    sm.refresh(vq)
    assert sm.stats.split_drift1 == 0


@pytest.mark.parametrize("dev", [False, True])
def test_rebuild_below_of_a_two_level_hierarchy(dev):
    """Two levels: the rebuild only recomputes the coarsest operators and
    their inverses; the solve after a re-setup and a rebuild reaches the
    direct solution."""
    torch = _torch()
    from paper_2407_05930_amd import Solver
    _say("rebuild two levels", dev)
    kw = dict(kappa="lognormal")
    p0 = make_problem((12, 10, 8), s=2, m=1, seed=105, **kw)
    p1 = make_problem((12, 10, 8), s=2, m=1, seed=106, **kw)
    sv = Solver(p0.A, p0.img, tol=TOL, pc="amgr_sub", coarse_max=200, k=2)
    assert sv.num_levels() == 2
    vals = torch.from_numpy(p1.A.data).cuda()
    sv.refresh(vals)
    sv.rebuild_below(vals if dev else None)
    assert sv.num_levels() == 2
    x = sv.solve(torch.from_numpy(p1.b).cuda()).cpu().numpy()
    xd = spla.splu(p1.A.tocsc()).solve(p1.b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
