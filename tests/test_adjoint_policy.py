"""The re-setup policies of DifferentiablePoisson (device mode) on the CPU:
the device calls are replaced by a recording stand-in solver whose
msp_stats fields the test sets, so that every branch of the decision runs
without a GPU -- a re-setup that stays, a fresh host setup on reduction-level
drift, a fresh setup or a rebuild below the reduction level on level-1
drift, and a fresh setup after iteration growth.  The fresh setups are real
host-only solvers."""
import numpy as np
import pytest

from gen import make_problem


class _Stats:
    def __init__(self, nb, n1):
        self.split_drift = 0
        self.split_drift1 = 0
        self.nlev = 4
        self.rows = [nb, n1, 0, 0]


class _Solver:
    """Stands for a device solver after its first setup."""

    def __init__(self, nb, n1):
        self.stats = _Stats(nb, n1)
        self.version = 0
        self.calls = []

    def refresh(self, values):
        self.calls.append(("refresh", values))
        self.version += 1

    def rebuild_below(self, values=None):
        self.calls.append(("rebuild_below", values))
        self.version += 1


def _setup(**policy):
    import torch
    from paper_2407_05930_amd.adjoint import DifferentiablePoisson
    p = make_problem((12, 10, 8), s=2, m=1, seed=5, kappa="lognormal")
    dp = DifferentiablePoisson(p.faces, p.img, device=-1, resetup="device", coarse_max=32, **policy)
    k0 = torch.from_numpy(p.kappa_base)
    dp.solver_for(k0)                                   # a real host-only fresh setup
    assert dp.fresh_setups == 1
    fake = _Solver(p.n_b, 100)
    dp.solver = fake
    dp.op.assemble_device = lambda kap, out=None: "values"
    return dp, fake, p, k0


def _step(p, k0, i):
    import torch
    return k0 * torch.exp(torch.full((p.n_b,), 0.01 * (i + 1), dtype=torch.float64))


def test_small_drift_keeps_the_re_set_up_solver():
    dp, fake, p, k0 = _setup(max_split_drift=0.1, max_split_drift1=0.2)
    fake.stats.split_drift, fake.stats.split_drift1 = int(0.1 * p.n_b), 20
    assert dp.solver_for(_step(p, k0, 0)) is fake
    assert fake.calls == [("refresh", "values")] and dp.fresh_setups == 1 and dp.rebuilds == 0
    assert dp.solver_for(_step(p, k0, 0)) is fake and len(fake.calls) == 1     # same kappa: nothing redone


def test_reduction_level_drift_takes_a_fresh_setup():
    from paper_2407_05930_amd import Solver
    dp, fake, p, k0 = _setup(max_split_drift=0.1, max_split_drift1=0.2, drift1_action="rebuild_below")
    fake.stats.split_drift, fake.stats.split_drift1 = int(0.1 * p.n_b) + 1, 50
    sv = dp.solver_for(_step(p, k0, 0))
    assert isinstance(sv, Solver) and sv is not fake
    assert dp.fresh_setups == 2 and dp.rebuilds == 0
    assert fake.calls == [("refresh", "values")]       # level-1 drift too, but the fresh setup covers it


@pytest.mark.parametrize("action", ["fresh", "rebuild_below"])
def test_level_one_drift_takes_the_chosen_action(action):
    from paper_2407_05930_amd import Solver
    dp, fake, p, k0 = _setup(max_split_drift1=0.2, drift1_action=action)
    fake.stats.split_drift1 = 21
    sv = dp.solver_for(_step(p, k0, 0))
    if action == "fresh":
        assert isinstance(sv, Solver) and dp.fresh_setups == 2 and dp.rebuilds == 0
    else:
        assert sv is fake and dp.fresh_setups == 1 and dp.rebuilds == 1
        assert fake.calls == [("refresh", "values"), ("rebuild_below", "values")]
        assert dp._base_version == fake.version == 2


def test_level_one_bound_ignores_two_level_hierarchies():
    dp, fake, p, k0 = _setup(max_split_drift1=0.0)
    fake.stats.nlev, fake.stats.split_drift1 = 2, -1
    assert dp.solver_for(_step(p, k0, 0)) is fake and dp.fresh_setups == 1


def test_iteration_growth_takes_a_fresh_setup_for_the_next_kappa():
    from paper_2407_05930_amd import Solver

    class _Last:
        iters = 10

    dp, fake, p, k0 = _setup(max_iteration_growth=1.5)
    fake.last = _Last()
    dp._base_version = 0
    dp._observe(fake)                                   # the first solve after the fresh setup: 10
    assert dp._fresh_iters == 10
    dp.solver_for(_step(p, k0, 0))                     # re-set up (version 1)
    fake.last.iters = 16
    dp._observe(fake)                                   # 16 > 1.5 * 10
    assert dp._grown
    sv = dp.solver_for(_step(p, k0, 1))
    assert isinstance(sv, Solver) and dp.fresh_setups == 2 and not dp._grown
    assert fake.calls == [("refresh", "values")]       # no re-setup for the grown step
