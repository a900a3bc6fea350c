"""GPU discrete adjoint against the oracle's adjoint and against finite
differences.

- building blocks (convection transpose, FE Hessian-vector product, parameter
  VJP, position derivatives of spreading and interpolation) and one full
  adjoint step: <= 1e-10 relative to the oracle on identical inputs;
- checkpointed rollout (IBRollout, recomputation every k steps) against the
  oracle's store-all rollout gradient;
- the 64^3 / 50-step Holzapfel-Ogden block with checkpoints every 10 steps:
  gradients in (a, b, a_f, b_f) within 1e-6 of fourth-order central
  differences of the GPU forward run (multigrid rtol 1e-13 so the solver
  tolerance does not pollute the differences); 8 random X0 directions on the
  first 20 steps of the same workload (see below).

The loss is only piecewise smooth in X0 over 50 steps: the fibre term uses
I4f* = max(I4f, 1), so the stress is continuous but its derivative jumps where
a Gauss point's fibre stretch passes 1.  The relaxing block reaches that
point: the smallest I4f over all Gauss points is 1.0075 after 20 steps, 0.9998
after 25 and 0.946 after 50.  A central difference whose two runs put one
Gauss point on opposite sides of I4f = 1 at some step measures an average of
the two one-sided derivatives; the oracle's own adjoint shows the same
1e-3 (step 1e-4 h) to 4e-5 (step 1e-6 h) relative gaps to such differences on
the 50-step horizon, while it agrees with this adjoint.  Before step 25 every
Gauss point keeps I4f > 1, so on the 20-step horizon the loss is smooth and
the 1e-6 bar applies.
"""
import numpy as np
import pytest

from paper_2503_22695_amd import inputs
from tests.test_gpu_parity import host, rel, say, to_dev

pytestmark = pytest.mark.gpu

HO = inputs.HOLZAPFEL_OGDEN


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module")
def hp():
    from paper_2503_22695_amd import hipib
    hipib.lib()
    return hipib


def assert_rel(name, a, b, tol):
    e = rel(a, b)
    assert e <= tol, f"{name}: relative error {e:.3e} > {tol:.1e}"


def deformed(prob, seed=11, amp=0.05):
    rng = np.random.default_rng(seed)
    c = prob.X_ref.mean(0)
    A = np.eye(3) + amp * rng.standard_normal((3, 3))
    return c + (prob.X_ref - c) @ A.T + 0.2 * amp * prob.h * rng.standard_normal(prob.X_ref.shape)


@pytest.mark.parametrize("name", ["nh_block_32", "ho_block_64"])
def test_building_blocks(torch_dev, hp, ref, name):
    torch = torch_dev
    prob = inputs.workload(name)
    n = prob.n
    say("adjoint blocks", name)
    rng = np.random.default_rng(21)
    ctx = hp.context_for_problem(prob)
    mesh = ref.MeshBuffers.from_problem(prob)
    x = deformed(prob)
    xd = to_dev(torch, x)
    V = rng.standard_normal(x.shape)
    assert_rel("fe_hvp", host(ctx.fe_hvp(xd, to_dev(torch, V))), ref.fe_hvp(mesh, x, V), 1e-10)
    dth = torch.zeros((hp.MAX_MATERIALS, 4), dtype=torch.float64, device="cuda")
    ctx.fe_param_vjp(xd, to_dev(torch, V), dth)
    if prob.materials[0].model == HO:
        assert_rel("fe_param_vjp", host(dth)[0], ref.fe_param_vjp(mesh, x, V)[0], 1e-10)
    else:
        assert float(dth.abs().max()) == 0.0
    u = 0.1 * rng.standard_normal((3, n, n, n))
    lam = rng.standard_normal((3, n, n, n))
    assert_rel("convection_vjp", host(ctx.convection_vjp(to_dev(torch, u), to_dev(torch, lam))),
               ref.convection_vjp(u, lam), 1e-11)
    F = rng.standard_normal(x.shape)
    lamU = rng.standard_normal(x.shape)
    lx = torch.zeros_like(xd)
    ctx.spread_vjp_X(xd, to_dev(torch, F), to_dev(torch, lam), lx)
    assert_rel("spread_vjp_X", host(lx), ref.spread_vjp_X(n, x, F, lam), 1e-10)
    lx = torch.zeros_like(xd)
    ctx.interp_vjp_X(xd, to_dev(torch, u), to_dev(torch, lamU), lx)
    assert_rel("interp_vjp_X", host(lx), ref.interp_vjp_X(x, u, lamU), 1e-10)


def adjoint_step_case(torch, hp, ref, prob, x0, pressure, seed):
    n = prob.n
    rng = np.random.default_rng(seed)
    fl = ref.fluid_from_problem(prob)
    mesh = ref.MeshBuffers.from_problem(prob)
    u0 = ref.project(fl, 0.02 * rng.standard_normal((3, n, n, n)))
    u1, _, _, _ = ref.advance(fl, mesh, u0, np.zeros((n, n, n)), x0, 0.0, 1, 0.0, 0.0) \
        if pressure == 0.0 else ref_step_with_pressure(ref, fl, mesh, u0, x0, pressure)
    lam_u = rng.standard_normal(u0.shape)
    lam_X = rng.standard_normal(x0.shape)
    lu_r, lX_r, dth_r = ref.adjoint_step(fl, mesh, u0, x0, u1, pressure, lam_u, lam_X)
    ctx = hp.context_for_problem(prob)
    lu, lX = to_dev(torch, lam_u), to_dev(torch, lam_X)
    dth = torch.zeros((hp.MAX_MATERIALS, 4), dtype=torch.float64, device="cuda")
    ctx.adjoint_step(to_dev(torch, u0), to_dev(torch, x0), to_dev(torch, u1), pressure, lu, lX, dth)
    torch.cuda.synchronize()
    assert_rel("lam_u", host(lu), lu_r, 1e-10)
    assert_rel("lam_X", host(lX), lX_r, 1e-10)
    nm = len(prob.materials)
    assert_rel("dtheta", host(dth)[:nm], dth_r, 1e-10)


def ref_step_with_pressure(ref, fl, mesh, u0, x0, pressure):
    """One oracle step at a given cavity pressure (p(t) = pressure at t = 0)."""
    import math
    T = 1.0
    t0 = T * math.asin(math.sqrt(pressure)) / math.pi
    u1, p1, X1, st = ref.advance(fl, mesh, u0, np.zeros((fl.n,) * 3), x0, t0, 1, 1.0, T)
    return u1, p1, X1, st


def test_adjoint_step_ho_block(torch_dev, hp, ref):
    prob = inputs.ho_block(n=32, n_el=6)
    say("adjoint step", prob.name)
    adjoint_step_case(torch_dev, hp, ref, prob, deformed(prob, 3, 0.04), 0.0, 31)


def test_adjoint_step_shell_with_pressure(torch_dev, hp, ref):
    """Full-size 128^3 shell (inflated 2% for conditioning) with the follower
    pressure load, so the pressure VJP is exercised."""
    prob = inputs.ho_shell()
    c = np.array([0.0, 0.5, 0.5])
    x0 = c + (prob.X_ref - c) * np.array([1.0, 1.02, 1.02])
    say("adjoint step", prob.name)
    adjoint_step_case(torch_dev, hp, ref, prob, x0, 0.3, 32)


def target_positions(torch, hp, prob, theta_target, n_steps, **over):
    ro = hp.Rollout(prob, n_steps=n_steps, checkpoint_every=10 ** 6, **over)
    th = torch.tensor(theta_target, dtype=torch.float64)
    XN = ro.forward(th, to_dev(torch, prob.X0), keep_checkpoints=False)
    return XN.clone()


def test_checkpointed_rollout_matches_store_all_oracle(torch_dev, hp, ref):
    torch = torch_dev
    prob = inputs.ho_block(n=32, n_el=6, n_steps=10)
    say("rollout vs oracle", prob.name)
    theta = np.array(prob.materials[0].params[:4])
    Xt = host(target_positions(torch, hp, prob, theta * [1.1, 0.9, 1.1, 0.9], prob.n_steps))
    ro = hp.Rollout(prob, checkpoint_every=4)                 # ragged segments 4, 4, 2
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    X0 = to_dev(torch, prob.X0).requires_grad_(True)
    XN = hp.IBRollout().apply(th, X0, ro)
    L = ((XN - to_dev(torch, Xt)) ** 2).sum()
    L.backward()
    fl = ref.fluid_from_problem(prob)
    mesh = ref.MeshBuffers.from_problem(prob)
    Lr, dX0r, dthr = ref.rollout_grad(fl, mesh, prob.initial_velocity(), prob.X0, 0.0, prob.n_steps,
                                      prob.p0, prob.T, Xt)
    assert abs(float(L) - Lr) <= 1e-9 * Lr
    assert_rel("dL/dX0", host(X0.grad), dX0r, 1e-9)
    assert_rel("dL/dtheta", th.grad.numpy(), dthr[0], 1e-8)


def test_rollout_backward_uses_its_own_forward_pass(torch_dev, hp):
    """Each IBRollout call keeps its own checkpoints and material: a forward
    probe at another theta between apply and backward (the finite-difference
    pattern) and a second backward of a retained graph give the gradients of
    the plain apply-then-backward order, bitwise (deterministic mode)."""
    torch = torch_dev
    prob = inputs.ho_block(n=32, n_el=6, n_steps=6)
    say("rollout tape", prob.name)
    theta = np.array(prob.materials[0].params[:4])
    Xt = target_positions(torch, hp, prob, theta * [1.1, 0.9, 1.1, 0.9], prob.n_steps,
                          deterministic=1)

    def grads(probe, twice):
        ro = hp.Rollout(prob, checkpoint_every=4, deterministic=1)
        th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
        X0 = to_dev(torch, prob.X0).requires_grad_(True)
        L = ((hp.IBRollout().apply(th, X0, ro) - Xt) ** 2).sum()
        if probe:
            ro.forward(torch.tensor(theta * 1.3), to_dev(torch, prob.X0) * 1.001,
                       keep_checkpoints=False)
        L.backward(retain_graph=twice)
        out = [th.grad.numpy().copy(), host(X0.grad)]
        if twice:
            th.grad, X0.grad = None, None
            L.backward()
            out += [th.grad.numpy().copy(), host(X0.grad)]
        return out

    g_th, g_X = grads(False, False)
    p_th, p_X = grads(True, False)
    assert np.array_equal(p_th, g_th) and np.array_equal(p_X, g_X)
    a_th, a_X, b_th, b_X = grads(False, True)
    assert np.array_equal(a_th, g_th) and np.array_equal(a_X, g_X)
    assert np.array_equal(b_th, g_th) and np.array_equal(b_X, g_X)


def test_adjoint_workload_against_fourth_order_differences(torch_dev, hp, ref):
    """The adjoint workload: 64^3, 50 steps, HO block of 12^3 hexes, checkpoints
    every 10 steps; target from a forward run at theta * (1.1, 0.9, 1.1, 0.9)."""
    torch = torch_dev
    prob = inputs.workload("ho_block_64")
    say("adjoint workload FD", prob.name, prob.n_steps)
    theta = np.array(prob.materials[0].params[:4])
    Xt = target_positions(torch, hp, prob, theta * [1.1, 0.9, 1.1, 0.9], prob.n_steps, mg_rtol=1e-13)
    ro = hp.Rollout(prob, checkpoint_every=10, mg_rtol=1e-13)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    X0 = to_dev(torch, prob.X0).requires_grad_(True)
    L = ((hp.IBRollout().apply(th, X0, ro) - Xt) ** 2).sum()
    L.backward()
    g_th, g_X = th.grad.numpy().copy(), X0.grad.clone()

    def loss(th_np, X0d):
        XN = ro.forward(torch.tensor(th_np, dtype=torch.float64), X0d, keep_checkpoints=False)
        return float(((XN - Xt) ** 2).sum())

    def d4(f, e):
        return (-f(2 * e) + 8 * f(e) - 8 * f(-e) + f(-2 * e)) / (12 * e)
    X0d = to_dev(torch, prob.X0)
    for k in range(4):
        e = 1e-3 * theta[k]
        unit = np.zeros(4)
        unit[k] = 1.0
        fd = d4(lambda s: loss(theta + s * unit, X0d), e)
        say("theta", k, g_th[k], fd)
        assert abs(g_th[k] - fd) <= 1e-6 * abs(fd), (k, g_th[k], fd)

    # X0 directions on the smooth 20-step horizon (two checkpoint segments)
    n20 = 20
    Xt20 = target_positions(torch, hp, prob, theta * [1.1, 0.9, 1.1, 0.9], n20, mg_rtol=1e-13)
    ro20 = hp.Rollout(prob, n_steps=n20, checkpoint_every=10, mg_rtol=1e-13)
    X0 = to_dev(torch, prob.X0).requires_grad_(True)
    L20 = ((hp.IBRollout().apply(torch.tensor(theta), X0, ro20) - Xt20) ** 2).sum()
    L20.backward()
    g_X = X0.grad.clone()

    def loss20(X0v):
        XN = ro20.forward(torch.tensor(theta), X0v, keep_checkpoints=False)
        return float(((XN - Xt20) ** 2).sum())
    rng = np.random.default_rng(5)
    for _ in range(8):
        d = to_dev(torch, rng.standard_normal(prob.X0.shape))
        fd = d4(lambda s: loss20(X0d + s * d), 1e-4 * prob.h)
        g = float((g_X * d).sum())
        say("X0 direction", g, fd)
        assert abs(g - fd) <= 1e-6 * abs(fd), (g, fd)


def test_mixed_precision_adjoint_matches_fp64(torch_dev, hp, ref):
    """Same adjoint workload in mixed precision against the FP64 gradient.

    The loss gradient is linear in the final residual X^N - X_t (dL/dX^N =
    2 (X^N - X_t)), so its relative error is that of the residual, e_res = the
    mixed forward's error in X^N over max |X^N - X_t|, plus the reverse steps'
    own FP32 rounding: the bound is 2 e_res + 1e-6 (as for the walled box)."""
    torch = torch_dev
    prob = inputs.workload("ho_block_64")
    say("mixed adjoint", prob.name)
    theta = np.array(prob.materials[0].params[:4])
    Xt = target_positions(torch, hp, prob, theta * [1.1, 0.9, 1.1, 0.9], prob.n_steps)
    grads, XN = {}, {}
    for prec in (hp.FP64, hp.MIXED):
        ro = hp.Rollout(prob, checkpoint_every=10, precision=prec)
        th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
        X0 = to_dev(torch, prob.X0).requires_grad_(True)
        XNp = hp.IBRollout().apply(th, X0, ro)
        L = ((XNp - Xt) ** 2).sum()
        L.backward()
        grads[prec] = (th.grad.numpy().copy(), host(X0.grad))
        XN[prec] = host(XNp.detach())
    e_res = np.max(np.abs(XN[hp.MIXED] - XN[hp.FP64])) / np.max(np.abs(XN[hp.FP64] - host(Xt)))
    bound = 2.0 * e_res + 1e-6
    say("mixed grads", grads[hp.MIXED][0], grads[hp.FP64][0], "e_res", e_res)
    assert_rel("dL/dtheta", grads[hp.MIXED][0], grads[hp.FP64][0], bound)
    assert_rel("dL/dX0", grads[hp.MIXED][1], grads[hp.FP64][1], bound)


def test_checkpointing_matches_store_all_on_gpu(torch_dev, hp):
    """Checkpoints every 10 steps (segments recomputed in the backward pass)
    against keeping all 50 steps' states: the recomputed states differ from the
    stored ones only by the order of floating-point atomic additions, so the
    gradients agree to near rounding."""
    torch = torch_dev
    prob = inputs.workload("ho_block_64")
    say("checkpointing vs store-all", prob.name)
    theta = np.array(prob.materials[0].params[:4])
    Xt = target_positions(torch, hp, prob, theta * [1.1, 0.9, 1.1, 0.9], prob.n_steps)
    grads = []
    for k in (10, prob.n_steps):
        ro = hp.Rollout(prob, checkpoint_every=k)
        th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
        X0 = to_dev(torch, prob.X0).requires_grad_(True)
        L = ((hp.IBRollout().apply(th, X0, ro) - Xt) ** 2).sum()
        L.backward()
        grads.append((th.grad.numpy().copy(), host(X0.grad)))
    e_th, e_X = rel(grads[0][0], grads[1][0]), rel(grads[0][1], grads[1][1])
    say("checkpointed vs store-all", e_th, e_X)
    assert e_th <= 1e-12 and e_X <= 1e-12, (e_th, e_X)
