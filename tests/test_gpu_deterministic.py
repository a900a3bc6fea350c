"""Deterministic mode (hipib_config.deterministic = 1): spreading by sorted
segments, element and face scatters gathered per node in element order, the
parameter gradient reduced in a fixed order.  Every result must be bitwise the
same from run to run (fresh contexts, same inputs), and still match the oracle
to the FP64 bar of the atomic mode; checkpointed and store-all adjoint
rollouts must give bitwise the same gradients."""
import numpy as np
import pytest

from paper_2503_22695_amd import inputs
from tests.test_gpu_parity import TOL, assert_close, deformed, host, plain_ctx, say, to_dev

pytestmark = pytest.mark.gpu


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


def same(torch, a, b):
    return bool(torch.equal(a, b))


def test_spread_random_nodes_bitwise_and_oracle(torch_dev, hp, ref):
    torch = torch_dev
    n, nn = 48, 2000
    say("det spread random", n, nn)
    rng = np.random.default_rng(4)
    X = rng.uniform(-0.3, 1.3, (nn, 3))
    X[:500] = 0.5 + 0.01 * rng.standard_normal((500, 3))   # a crowded cluster
    F = rng.standard_normal((nn, 3))
    f0 = rng.standard_normal((3, n, n, n))
    outs = []
    for _ in range(2):
        ctx = plain_ctx(hp, n, deterministic=1)
        ctx.set_mesh(X, np.zeros((0, 8)), np.zeros((0, 3)), np.zeros(0))
        fd = to_dev(torch, f0)
        ctx.spread(to_dev(torch, X), to_dev(torch, F), fd)
        torch.cuda.synchronize()
        outs.append(fd)
    assert same(torch, outs[0], outs[1])
    assert_close("f", host(outs[0]), ref.spread(n, X, F, f0))


@pytest.mark.parametrize("n,nn", [(8, 300), (12, 400), (16, 600), (24, 700)])
def test_spread_small_grids_bitwise_and_oracle(torch_dev, hp, ref, n, nn):
    """Grids of one tile per axis (n = 8: every tile box wraps onto itself),
    4^3-cell tiles (n = 12), two tiles per axis (n = 16: the tile below and
    above a tile are the same one) and three (n = 24), with half of the nodes in
    one crowded cluster (more than one work item in its tile)."""
    torch = torch_dev
    say("det spread small grid", n, nn)
    rng = np.random.default_rng(n)
    X = rng.uniform(-0.3, 1.3, (nn, 3))
    X[: nn // 2] = 0.5 + 0.01 * rng.standard_normal((nn // 2, 3))
    F = rng.standard_normal((nn, 3))
    f0 = rng.standard_normal((3, n, n, n))
    outs = []
    for _ in range(2):
        ctx = plain_ctx(hp, n, deterministic=1)
        ctx.set_mesh(X, np.zeros((0, 8)), np.zeros((0, 3)), np.zeros(0))
        fd = to_dev(torch, f0)
        ctx.spread(to_dev(torch, X), to_dev(torch, F), fd)
        torch.cuda.synchronize()
        outs.append(fd)
    assert same(torch, outs[0], outs[1])
    assert_close("f", host(outs[0]), ref.spread(n, X, F, f0))


def test_spread_shell_bitwise(torch_dev, hp, ref):
    torch = torch_dev
    prob = inputs.ho_shell()
    say("det spread shell", prob.n_nodes)
    rng = np.random.default_rng(3)
    F = to_dev(torch, rng.standard_normal((prob.n_nodes, 3)))
    outs = []
    for _ in range(2):
        ctx = hp.context_for_problem(prob, deterministic=1)
        fd = torch.zeros((3, prob.n, prob.n, prob.n), dtype=torch.float64, device="cuda")
        ctx.spread(to_dev(torch, prob.X0), F, fd)
        torch.cuda.synchronize()
        outs.append(fd)
    assert same(torch, outs[0], outs[1])
    assert_close("f", host(outs[0]), ref.spread(prob.n, prob.X0, host(F)))


def test_fe_force_shell_bitwise(torch_dev, hp, ref):
    torch = torch_dev
    prob = inputs.ho_shell()
    say("det fe_force shell", prob.n_elems)
    x = deformed(prob, 11, 0.03)
    outs = []
    for _ in range(2):
        ctx = hp.context_for_problem(prob, deterministic=1)
        outs.append(ctx.fe_force(to_dev(torch, x), 0.7))
        torch.cuda.synchronize()
    assert same(torch, outs[0], outs[1])
    Fr, _, _ = ref.fe_force(ref.MeshBuffers.from_problem(prob), x)
    Fr = ref.pressure_load(prob.faces, x, 0.7, Fr)
    assert_close("F", host(outs[0]), Fr)


@pytest.mark.parametrize("name,steps", [("nh_block_32", 10), ("ho_shell_128", 3)])
def test_advance_bitwise_and_oracle(torch_dev, hp, ref, name, steps):
    torch = torch_dev
    prob = inputs.workload(name)
    t0 = 0.0
    if prob.n_faces:   # the conditioned shell start of the FP64 parity test
        c = np.array([0.0, 0.5, 0.5])
        prob.X0 = c + (prob.X_ref - c) * np.array([1.0, 1.02, 1.02])
        t0 = prob.dt
    say("det advance", name, steps)
    sims = []
    for _ in range(2):
        sim = hp.Simulation(prob, deterministic=1)
        sim.t = t0
        sim.advance(steps)
        torch.cuda.synchronize()
        sims.append(sim)
    for f in ("u", "p", "X"):
        assert same(torch, getattr(sims[0], f), getattr(sims[1], f)), f
    ur, pr, Xr, st = ref.run_problem(prob, n_steps=steps, t0=t0)
    cyc, _ = sims[0].ctx.step_stats()
    assert [list(c) for c in cyc] == [list(s.cycles) for s in st]
    assert_close("u", host(sims[0].u), ur, TOL)
    assert_close("p", host(sims[0].p), pr, TOL)
    assert_close("X - X0", host(sims[0].X) - prob.X0, Xr - prob.X0, TOL)


def test_adjoint_checkpointed_equals_store_all_bitwise(torch_dev, hp):
    """64^3 / 50-step HO block: checkpoints every 10 steps (segments recomputed
    on the second context) and every state kept give bitwise the same
    gradients, and a repeated run gives bitwise the same gradients again."""
    torch = torch_dev
    prob = inputs.workload("ho_block_64")
    say("det adjoint", prob.name)
    theta = np.array(prob.materials[0].params[:4])
    ro_t = hp.Rollout(prob, checkpoint_every=10 ** 6, deterministic=1)
    Xt = ro_t.forward(torch.tensor(theta * [1.1, 0.9, 1.1, 0.9]), to_dev(torch, prob.X0),
                      keep_checkpoints=False).clone()
    grads = []
    for k in (10, prob.n_steps, 10):
        ro = hp.Rollout(prob, checkpoint_every=k, deterministic=1)
        th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
        X0 = to_dev(torch, prob.X0).requires_grad_(True)
        L = ((hp.IBRollout().apply(th, X0, ro) - Xt) ** 2).sum()
        L.backward()
        grads.append((th.grad.clone(), X0.grad.clone(), L.detach().clone()))
    for g in grads[1:]:
        assert same(torch, grads[0][2], g[2])
        assert same(torch, grads[0][0], g[0])
        assert same(torch, grads[0][1], g[1])


def test_run_on_a_user_stream_equals_the_default_stream_bitwise(torch_dev, hp):
    """A context created on a user stream (its element forces forked to the
    context's side stream and joined back by events, as on the default
    stream) gives bitwise the same deterministic run as one on the default
    stream: the 64^3 HO block, 20 steps."""
    torch = torch_dev
    prob = inputs.workload("ho_block_64")
    say("user stream vs default stream", prob.name)
    a = hp.Simulation(prob, deterministic=1)
    a.advance(20)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = hp.Simulation(prob, deterministic=1)
        b.advance(20)
    s.synchronize()
    torch.cuda.synchronize()
    for f in ("u", "p", "X"):
        assert same(torch, getattr(a, f), getattr(b, f)), f
