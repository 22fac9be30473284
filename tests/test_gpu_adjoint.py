"""GPU parity of the differentiable solve (torch.autograd.Function through
the C interface) with the oracle's adjoint gradient."""
import numpy as np
import pytest

from gen import config_problem, make_problem
from oracle import adjoint

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("N,s,m", [((32, 32, 32), 3, 1), ((24, 16, 20), 2, 2)])
def test_adjoint_gradient_matches_oracle(N, s, m):
    torch = _torch()
    from paper_2407_05930_amd.adjoint import DifferentiablePoisson
    pr = make_problem(N, s=s, m=m, seed=12, kappa="lognormal", with_target=True)
    pstar = np.repeat(pr.p_target[:, None], m, axis=1)
    L, lam, g, p_ref = adjoint.loss_and_gradients(pr.faces, pr.img, pr.kappa_base, pr.b, pstar)
    dp = DifferentiablePoisson(pr.faces, pr.img, tol=1e-13, coarse_max=64)
    f = torch.from_numpy(pr.b).cuda().requires_grad_(True)
    kap = torch.from_numpy(pr.kappa_base).cuda().requires_grad_(True)
    p = dp(f, kap)
    loss = 0.5 * ((p - torch.from_numpy(pstar).cuda()) ** 2).sum()
    loss.backward()
    assert abs(loss.item() - L) <= 1e-9 * abs(L)
    assert np.linalg.norm(p.detach().cpu().numpy() - p_ref) <= 1e-9 * np.linalg.norm(p_ref)
    gf = f.grad.cpu().numpy()
    assert np.linalg.norm(gf - lam) <= 1e-9 * np.linalg.norm(lam)
    gk = kap.grad.cpu().numpy()
    assert np.linalg.norm(gk - g) <= 1e-9 * np.linalg.norm(g)


@pytest.mark.parametrize("prec", ["mixed", "mixed_bf16"])
def test_adjoint_gradient_with_a_mixed_precision_cycle(prec):
    """The FP64 outer PCG with an FP32-arithmetic V-cycle (FP32 or bfloat16
    multivectors) as preconditioner: both solves reach the tolerance in the
    true residual, so loss and gradients match the oracle's to 1e-9."""
    torch = _torch()
    from paper_2407_05930_amd.adjoint import DifferentiablePoisson
    pr = make_problem((32, 32, 32), s=3, m=1, seed=13, kappa="lognormal", with_target=True)
    pstar = pr.p_target[:, None]
    L, lam, g, p_ref = adjoint.loss_and_gradients(pr.faces, pr.img, pr.kappa_base, pr.b, pstar)
    dp = DifferentiablePoisson(pr.faces, pr.img, tol=1e-12, coarse_max=64, precision=prec, afsai_nnz=5,
                               emin_steps=4)
    f = torch.from_numpy(pr.b).cuda().requires_grad_(True)
    kap = torch.from_numpy(pr.kappa_base).cuda().requires_grad_(True)
    p = dp(f, kap)
    loss = 0.5 * ((p - torch.from_numpy(pstar).cuda()) ** 2).sum()
    loss.backward()
    assert abs(loss.item() - L) <= 1e-9 * abs(L)
    assert np.linalg.norm(f.grad.cpu().numpy() - lam) <= 1e-9 * np.linalg.norm(lam)
    assert np.linalg.norm(kap.grad.cpu().numpy() - g) <= 1e-9 * np.linalg.norm(g)


def test_adjoint_gradient_central_difference_on_gpu():
    """Finite differences of the GPU loss for a few base cells (32^3, s = 3)."""
    torch = _torch()
    from paper_2407_05930_amd.adjoint import DifferentiablePoisson
    pr = make_problem((32, 32, 32), s=3, m=1, seed=3, kappa="lognormal", with_target=True)
    dp = DifferentiablePoisson(pr.faces, pr.img, tol=1e-13, coarse_max=64)
    f = torch.from_numpy(pr.b).cuda()
    pst = torch.from_numpy(pr.p_target[:, None]).cuda()

    def loss_of(kv):
        with torch.no_grad():
            p = dp(f, torch.from_numpy(kv).cuda())
            return 0.5 * float(((p - pst) ** 2).sum())

    kap = torch.from_numpy(pr.kappa_base).cuda().requires_grad_(True)
    p = dp(f, kap)
    (0.5 * ((p - pst) ** 2).sum()).backward()
    g = kap.grad.cpu().numpy()
    rng = np.random.default_rng(5)
    for i in rng.choice(pr.n_b, size=5, replace=False):
        eps = 1e-5 * pr.kappa_base[i]
        kp = pr.kappa_base.copy()
        km = pr.kappa_base.copy()
        kp[i] += eps
        km[i] -= eps
        fd = (loss_of(kp) - loss_of(km)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g).max())


def test_two_forwards_with_different_kappa_then_one_backward():
    """A loss summed over two kappa samples: the first graph's backward still
    uses the solver of its own kappa after the second forward built another
    one; each gradient equals the oracle's for its kappa."""
    torch = _torch()
    from paper_2407_05930_amd.adjoint import DifferentiablePoisson
    pr = make_problem((16, 16, 16), s=3, m=1, seed=14, kappa="lognormal", with_target=True)
    k2 = pr.kappa_base * np.exp(0.3 * np.random.default_rng(1).standard_normal(pr.n_b))
    pstar = pr.p_target[:, None]
    dp = DifferentiablePoisson(pr.faces, pr.img, tol=1e-13, coarse_max=48)
    f = torch.from_numpy(pr.b).cuda().requires_grad_(True)
    ka = torch.from_numpy(pr.kappa_base).cuda().requires_grad_(True)
    kb = torch.from_numpy(k2).cuda().requires_grad_(True)
    pst = torch.from_numpy(pstar).cuda()
    loss = 0.5 * ((dp(f, ka) - pst) ** 2).sum() + 0.5 * ((dp(f, kb) - pst) ** 2).sum()
    loss.backward()
    La, lam_a, ga, _ = adjoint.loss_and_gradients(pr.faces, pr.img, pr.kappa_base, pr.b, pstar)
    Lb, lam_b, gb, _ = adjoint.loss_and_gradients(pr.faces, pr.img, k2, pr.b, pstar)
    assert abs(loss.item() - (La + Lb)) <= 1e-9 * abs(La + Lb)
    assert np.linalg.norm(ka.grad.cpu().numpy() - ga) <= 1e-9 * np.linalg.norm(ga)
    assert np.linalg.norm(kb.grad.cpu().numpy() - gb) <= 1e-9 * np.linalg.norm(gb)
    gf = lam_a + lam_b
    assert np.linalg.norm(f.grad.cpu().numpy() - gf) <= 1e-9 * np.linalg.norm(gf)


def test_unconverged_solve_is_an_error_in_the_autograd_function():
    torch = _torch()
    from paper_2407_05930_amd import MspError
    from paper_2407_05930_amd.adjoint import DifferentiablePoisson
    pr = make_problem((12, 12, 12), s=3, m=1, seed=15, kappa="lognormal", with_target=True)
    dp = DifferentiablePoisson(pr.faces, pr.img, tol=1e-13, coarse_max=48, maxit=2)
    f = torch.from_numpy(pr.b).cuda()
    kap = torch.from_numpy(pr.kappa_base).cuda().requires_grad_(True)
    with pytest.raises(MspError, match="NOT_CONVERGED"):
        dp(f, kap)


def test_device_assembly_equals_the_host_assembly():
    """msp_fv_assemble_device: the same values in the same positions, bit for
    bit (same arithmetic, same summation order), here for two kappa fields."""
    torch = _torch()
    from paper_2407_05930_amd.adjoint import FVOperator
    pr = make_problem((20, 16, 12), s=3, m=1, seed=16, kappa="lognormal", jitter=0.2)
    op = FVOperator(pr.faces, pr.img)
    for kv in (pr.kappa_base, pr.kappa_base * np.exp(np.random.default_rng(2).standard_normal(pr.n_b))):
        A = op.assemble(kv)
        d = op.assemble_device(torch.from_numpy(kv).cuda()).cpu().numpy()
        assert d.size == A.nnz
        assert np.array_equal(d, A.data)
    op.close()


def test_device_resetup_in_an_optimisation_loop_matches_the_oracle():
    """resetup = "device": kappa steps rebuild the solver on the device on
    the first setup's structure; each step's loss and gradients equal the
    oracle's for that kappa, and a backward for a forward whose kappa has
    been replaced since is refused."""
    torch = _torch()
    from paper_2407_05930_amd.adjoint import DifferentiablePoisson
    pr = make_problem((24, 20, 16), s=3, m=1, seed=17, kappa="lognormal", with_target=True)
    pstar = pr.p_target[:, None]
    dp = DifferentiablePoisson(pr.faces, pr.img, tol=1e-13, coarse_max=48, resetup="device")
    f = torch.from_numpy(pr.b).cuda()
    pst = torch.from_numpy(pstar).cuda()
    kv = pr.kappa_base.copy()
    rng = np.random.default_rng(3)
    first = None
    for step in range(3):
        kap = torch.from_numpy(kv).cuda().requires_grad_(True)
        p = dp(f, kap)
        loss = 0.5 * ((p - pst) ** 2).sum()
        loss.backward()
        L, lam, g, p_ref = adjoint.loss_and_gradients(pr.faces, pr.img, kv, pr.b, pstar)
        assert abs(loss.item() - L) <= 1e-9 * abs(L)
        assert np.linalg.norm(p.detach().cpu().numpy() - p_ref) <= 1e-9 * np.linalg.norm(p_ref)
        gk = kap.grad.cpu().numpy()
        assert np.linalg.norm(gk - g) <= 1e-9 * np.linalg.norm(g)
        if first is None:
            first = dp.solver
        assert dp.solver is first                     # re-set up in place, not rebuilt
        kv = kv * np.exp(0.2 * rng.standard_normal(pr.n_b))
    ka = torch.from_numpy(kv).cuda().requires_grad_(True)
    loss_a = 0.5 * ((dp(f, ka) - pst) ** 2).sum()
    dp(f, torch.from_numpy(kv * 1.5).cuda())           # replaces the solver's values
    with pytest.raises(RuntimeError, match="re-set up"):
        loss_a.backward()


def test_device_resetup_falls_back_to_a_fresh_setup_when_the_split_moves():
    """max_split_drift = 0: a kappa step that moves the reduction level's split
    (reported by the device re-setup) gets a fresh host setup instead, and
    its loss and gradient are those of the oracle."""
    torch = _torch()
    from paper_2407_05930_amd.adjoint import DifferentiablePoisson
    pr = make_problem((24, 20, 16), s=3, m=1, seed=18, kappa="lognormal", y_stretch=1.5, with_target=True)
    pstar = pr.p_target[:, None]
    dp = DifferentiablePoisson(pr.faces, pr.img, tol=1e-13, coarse_max=48, resetup="device", max_split_drift=0.0)
    f = torch.from_numpy(pr.b).cuda()
    pst = torch.from_numpy(pstar).cuda()
    k0 = torch.from_numpy(pr.kappa_base).cuda().requires_grad_(True)
    loss0 = 0.5 * ((dp(f, k0) - pst) ** 2).sum()      # a graph recorded with the first solver
    first = dp.solver
    assert dp.fresh_setups == 1
    k1 = pr.kappa_base * np.exp(0.5 * np.random.default_rng(4).standard_normal(pr.n_b))
    kap = torch.from_numpy(k1).cuda().requires_grad_(True)
    loss = 0.5 * ((dp(f, kap) - pst) ** 2).sum()
    assert first.stats.split_drift > 0
    assert dp.fresh_setups == 2 and dp.solver is not first
    loss.backward()
    L, lam, g, p_ref = adjoint.loss_and_gradients(pr.faces, pr.img, k1, pr.b, pstar)
    assert abs(loss.item() - L) <= 1e-9 * abs(L)
    assert np.linalg.norm(kap.grad.cpu().numpy() - g) <= 1e-9 * np.linalg.norm(g)
    with pytest.raises(RuntimeError, match="re-set up"):   # the first solver holds the new values now
        loss0.backward()


def test_device_resetup_falls_back_when_the_level_one_split_moves():
    """max_split_drift1 = 0 (and no bound on the reduction level): a small
    kappa step that moves level 1's split gets a fresh host setup, with the
    oracle's loss and gradient."""
    torch = _torch()
    from paper_2407_05930_amd.adjoint import DifferentiablePoisson
    pr = make_problem((24, 20, 16), s=3, m=1, seed=21, kappa="lognormal", y_stretch=1.5, with_target=True)
    pstar = pr.p_target[:, None]
    dp = DifferentiablePoisson(pr.faces, pr.img, tol=1e-13, coarse_max=48, resetup="device", max_split_drift1=0.0)
    f = torch.from_numpy(pr.b).cuda()
    pst = torch.from_numpy(pstar).cuda()
    dp(f, torch.from_numpy(pr.kappa_base).cuda())
    first = dp.solver
    assert dp.fresh_setups == 1 and first.num_levels() >= 3
    k1 = pr.kappa_base * np.exp(0.05 * np.random.default_rng(7).standard_normal(pr.n_b))
    kap = torch.from_numpy(k1).cuda().requires_grad_(True)
    loss = 0.5 * ((dp(f, kap) - pst) ** 2).sum()
    print("drift", first.stats.split_drift, "level 1", first.stats.split_drift1, flush=True)
    assert first.stats.split_drift1 > 0
    assert dp.fresh_setups == 2 and dp.solver is not first
    loss.backward()
    L, lam, g, _ = adjoint.loss_and_gradients(pr.faces, pr.img, k1, pr.b, pstar)
    assert abs(loss.item() - L) <= 1e-9 * abs(L)
    assert np.linalg.norm(kap.grad.cpu().numpy() - g) <= 1e-9 * np.linalg.norm(g)


def test_level_one_drift_can_rebuild_below_instead_of_a_fresh_setup():
    """drift1_action = "rebuild_below": the same kappa step keeps the solver
    (re-set-up reduction level) and rebuilds the levels below it; loss and
    gradient are the oracle's, and a graph recorded before the rebuild is
    refused its backward."""
    torch = _torch()
    from paper_2407_05930_amd.adjoint import DifferentiablePoisson
    pr = make_problem((24, 20, 16), s=3, m=1, seed=21, kappa="lognormal", y_stretch=1.5, with_target=True)
    pstar = pr.p_target[:, None]
    dp = DifferentiablePoisson(pr.faces, pr.img, tol=1e-13, coarse_max=48, resetup="device", max_split_drift1=0.0,
                               drift1_action="rebuild_below")
    f = torch.from_numpy(pr.b).cuda()
    pst = torch.from_numpy(pstar).cuda()
    k0 = torch.from_numpy(pr.kappa_base).cuda().requires_grad_(True)
    loss0 = 0.5 * ((dp(f, k0) - pst) ** 2).sum()
    first = dp.solver
    k1 = pr.kappa_base * np.exp(0.05 * np.random.default_rng(7).standard_normal(pr.n_b))
    kap = torch.from_numpy(k1).cuda().requires_grad_(True)
    loss = 0.5 * ((dp(f, kap) - pst) ** 2).sum()
    assert dp.fresh_setups == 1 and dp.rebuilds == 1 and dp.solver is first
    loss.backward()
    L, lam, g, _ = adjoint.loss_and_gradients(pr.faces, pr.img, k1, pr.b, pstar)
    assert abs(loss.item() - L) <= 1e-9 * abs(L)
    assert np.linalg.norm(kap.grad.cpu().numpy() - g) <= 1e-9 * np.linalg.norm(g)
    with pytest.raises(RuntimeError, match="re-set up"):
        loss0.backward()


def test_device_resetup_falls_back_when_the_iterations_grow():
    """max_iteration_growth: once a solve on a re-set-up solver takes more
    than the ratio times the iterations after the last fresh setup, the next
    kappa gets a fresh host setup (ratio 0.5 forces it here), and the
    gradients stay the oracle's."""
    torch = _torch()
    from paper_2407_05930_amd.adjoint import DifferentiablePoisson
    pr = make_problem((20, 16, 16), s=3, m=1, seed=19, kappa="lognormal", with_target=True)
    pstar = pr.p_target[:, None]
    dp = DifferentiablePoisson(pr.faces, pr.img, tol=1e-13, coarse_max=48, resetup="device",
                               max_iteration_growth=0.5)
    f = torch.from_numpy(pr.b).cuda()
    pst = torch.from_numpy(pstar).cuda()
    rng = np.random.default_rng(6)
    kv = pr.kappa_base.copy()
    setups = []
    for step in range(4):
        kap = torch.from_numpy(kv).cuda().requires_grad_(True)
        loss = 0.5 * ((dp(f, kap) - pst) ** 2).sum()
        loss.backward()
        setups.append(dp.fresh_setups)
        L, lam, g, _ = adjoint.loss_and_gradients(pr.faces, pr.img, kv, pr.b, pstar)
        assert np.linalg.norm(kap.grad.cpu().numpy() - g) <= 1e-9 * np.linalg.norm(g)
        kv = kv * np.exp(0.1 * rng.standard_normal(pr.n_b))
    # fresh, re-set up (grows past 0.5x), fresh, re-set up
    assert setups == [1, 1, 2, 2], setups


def test_full_size_adjoint_directional_derivative():
    """The adjoint workload at its full size (256^3, s = 3, lognormal kappa)
    in the bench's configuration: forward and adjoint solves reach a true
    relative residual of 1e-10, and dL/dkappa along a random direction d
    equals the central difference (L(kappa + h d) - L(kappa - h d)) / 2h of
    two more forward solves (after device re-setups) to 1e-5."""
    torch = _torch()
    from paper_2407_05930_amd.adjoint import DifferentiablePoisson
    pr = config_problem("adjoint3d_256_s3", assemble=False)
    print("256^3 adjoint: setup", flush=True)
    # the perturbed losses use the device re-setup: the solves reach 1e-12 whatever the preconditioner
    dp = DifferentiablePoisson(pr.faces, pr.img, tol=1e-12, pc="amgr_sub", afsai_nnz=5, emin_steps=4,
                               resetup="device")
    f = torch.from_numpy(pr.b).cuda()
    pst = torch.from_numpy(pr.p_target[:, None]).cuda()
    kap = torch.from_numpy(pr.kappa_base).cuda().requires_grad_(True)
    p = dp(f, kap)
    loss = 0.5 * ((p - pst) ** 2).sum()
    loss.backward()
    g = kap.grad.detach()
    print("256^3 adjoint: iterations", dp.solver.last.iters, flush=True)
    d = torch.from_numpy(np.random.default_rng(9).standard_normal(pr.n_b)).cuda() * kap.detach()
    h = 1e-4

    def loss_at(t):
        with torch.no_grad():
            q = dp(f, kap.detach() + t * d)
            return 0.5 * float(((q - pst) ** 2).sum())

    fd = (loss_at(h) - loss_at(-h)) / (2 * h)
    an = float((g * d).sum())
    print("256^3 adjoint: directional derivative", an, "central difference", fd, flush=True)
    assert abs(fd - an) <= 1e-5 * abs(an)
