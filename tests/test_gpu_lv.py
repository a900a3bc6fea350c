"""GPU parity for the full Holzapfel-Ogden law (sheet and fibre-sheet terms)
and the left-ventricle active stress: nodal forces, Hessian products, whole
steps with the activation waveform and the adjoint rollout, each against the
FP64 oracle on the same seeded inputs (1e-11 relative for the forward
operators and steps, as for the passive law; 1e-10 / 1e-9 for the adjoint
pieces, as in the passive adjoint tests)."""
import numpy as np
import pytest

from paper_2503_22695_amd import inputs
from tests.test_gpu_parity import TOL, assert_close, deformed, host, say, to_dev

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


def fibre_and_sheet_stretch(prob, seed, amp):
    """Positions whose elements stretch along their fibres and sheets (both I4
    terms active in many elements, compressed in others)."""
    x = deformed(prob, seed, amp)
    c = prob.X_ref.mean(0)
    f = prob.fibre.mean(0)
    f /= max(np.linalg.norm(f), 1e-12)
    return x + 0.04 * np.outer((prob.X_ref - c) @ f, f)


@pytest.mark.parametrize("name,Ta,det", [("lv_block_32", 0.0, 0), ("lv_block_32", 2.0, 0),
                                         ("lv_shell_128", 4.0, 0), ("lv_shell_128", 4.0, 1)])
def test_fe_force_full_law(torch_dev, hp, ref, name, Ta, det):
    torch = torch_dev
    prob = inputs.workload(name)
    say("lv fe_force", name, Ta, det)
    x = fibre_and_sheet_stretch(prob, 7, 0.03)
    ctx = hp.context_for_problem(prob, deterministic=det)
    ctx.set_active_tension(Ta)
    F = ctx.fe_force(to_dev(torch, x), 0.6)
    torch.cuda.synchronize()
    mesh = ref.MeshBuffers.from_problem(prob, active_tension=Ta)
    Fr, _, _ = ref.fe_force(mesh, x)
    if prob.n_faces:
        Fr = ref.pressure_load(prob.faces, x, 0.6, Fr)
    assert_close("F", host(F), Fr)


def test_active_tension_only_on_holzapfel_ogden(torch_dev, hp, ref):
    """The shell with leaflets: the active stress acts on the HO shell, not on
    the neo-Hookean leaflets."""
    torch = torch_dev
    prob = inputs.shell_with_leaflets(n=96)
    say("lv active on HO only", prob.name)
    x = deformed(prob, 5, 0.02)
    ctx = hp.context_for_problem(prob)
    ctx.set_active_tension(3.0)
    F = host(ctx.fe_force(to_dev(torch, x), 0.0))
    Fr, _, _ = ref.fe_force(ref.MeshBuffers.from_problem(prob, active_tension=3.0), x)
    assert_close("F", F, Fr)
    F0, _, _ = ref.fe_force(ref.MeshBuffers.from_problem(prob), x)
    leaf = np.unique(prob.conn[prob.mat_id == 1])
    shell = np.unique(prob.conn[prob.mat_id == 0])
    assert np.array_equal(F[leaf], F0[leaf]) or np.max(np.abs(F[leaf] - F0[leaf])) <= 1e-12 * np.max(np.abs(F0))
    assert np.max(np.abs(F[shell] - F0[shell])) > 1e-3 * np.max(np.abs(F0[shell]))


@pytest.mark.parametrize("Ta", [0.0, 2.0])
def test_fe_hvp_full_law(torch_dev, hp, ref, Ta):
    torch = torch_dev
    prob = inputs.lv_block()
    say("lv fe_hvp", Ta)
    x = fibre_and_sheet_stretch(prob, 8, 0.04)
    rng = np.random.default_rng(9)
    V = rng.standard_normal(x.shape)
    ctx = hp.context_for_problem(prob)
    ctx.set_active_tension(Ta)
    HV = host(ctx.fe_hvp(to_dev(torch, x), to_dev(torch, V)))
    mesh = ref.MeshBuffers.from_problem(prob, active_tension=Ta)
    assert_close("HV", HV, ref.fe_hvp(mesh, x, V), 1e-10)


def test_advance_lv_block_full_run(torch_dev, hp, ref):
    """20 steps with the activation pulse across the run: same stop decisions
    and the same fields as the oracle."""
    torch = torch_dev
    prob = inputs.lv_block()
    say("lv advance", prob.name, prob.n_steps)
    sim = hp.Simulation(prob)
    sim.advance(prob.n_steps)
    torch.cuda.synchronize()
    cyc, _ = sim.ctx.step_stats()
    ur, pr, Xr, st = ref.run_problem(prob)
    assert [list(c) for c in cyc] == [list(s.cycles) for s in st]
    assert_close("u", host(sim.u), ur, TOL)
    assert_close("p", host(sim.p), pr, TOL)
    assert_close("X - X0", host(sim.X) - prob.X0, Xr - prob.X0, TOL)


def test_advance_lv_shell_near_peak_activation(torch_dev, hp, ref):
    """The 128^3 LV shell for 3 steps starting at 40% of the run (activation
    and cavity pressure near their peaks)."""
    torch = torch_dev
    prob = inputs.lv_shell()
    t0 = 40 * prob.dt
    say("lv advance shell", prob.name, t0)
    sim = hp.Simulation(prob)
    sim.t = t0
    sim.advance(3)
    torch.cuda.synchronize()
    cyc, _ = sim.ctx.step_stats()
    ur, pr, Xr, st = ref.run_problem(prob, n_steps=3, t0=t0)
    assert [list(c) for c in cyc] == [list(s.cycles) for s in st]
    assert_close("u", host(sim.u), ur, TOL)
    assert_close("p", host(sim.p), pr, TOL)
    assert_close("X - X0", host(sim.X) - prob.X0, Xr - prob.X0, TOL)


def test_lv_adjoint_step(torch_dev, hp, ref):
    torch = torch_dev
    prob = inputs.lv_block()
    say("lv adjoint step", prob.name)
    n = prob.n
    Ta = 1.5
    x0 = fibre_and_sheet_stretch(prob, 10, 0.03)
    rng = np.random.default_rng(33)
    fl = ref.fluid_from_problem(prob)
    mesh = ref.MeshBuffers.from_problem(prob, active_tension=Ta)
    u0 = ref.project(fl, 0.02 * rng.standard_normal((3, n, n, n)))
    mesh_step = ref.MeshBuffers(prob.X_ref, prob.conn, prob.fibre, prob.mat_id, [HO],
                                [prob.materials[0].params], sheet=prob.sheet, active_tension=Ta)
    u1, _, _, _ = ref.advance(fl, mesh_step, u0, np.zeros((n, n, n)), x0, 0.0, 1)
    lam_u = rng.standard_normal(u0.shape)
    lam_X = rng.standard_normal(x0.shape)
    lu_r, lX_r, dth_r = ref.adjoint_step(fl, mesh, u0, x0, u1, 0.0, lam_u, lam_X)
    ctx = hp.context_for_problem(prob)
    ctx.set_active_tension(Ta)
    lu, lX = to_dev(torch, lam_u), to_dev(torch, lam_X)
    dth = torch.zeros((hp.MAX_MATERIALS, 4), dtype=torch.float64, device="cuda")
    ctx.adjoint_step(to_dev(torch, u0), to_dev(torch, x0), to_dev(torch, u1), 0.0, lu, lX, dth)
    torch.cuda.synchronize()
    assert_close("lam_u", host(lu), lu_r, 1e-10)
    assert_close("lam_X", host(lX), lX_r, 1e-10)
    assert_close("dtheta", host(dth)[:1], dth_r, 1e-10)


def test_lv_checkpointed_rollout_matches_oracle(torch_dev, hp, ref):
    """Rollout with checkpoints (ragged segments 4, 4, 2 over 10 steps) through
    the activation pulse: loss and gradients against the oracle's store-all
    reverse sweep."""
    torch = torch_dev
    prob = inputs.lv_block(n_steps=10)
    say("lv rollout", prob.name)
    theta = np.array(prob.materials[0].params[:4])
    ro_t = hp.Rollout(prob, checkpoint_every=10 ** 6)
    Xt = host(ro_t.forward(torch.tensor(theta * [1.1, 0.9, 1.1, 0.9]), to_dev(torch, prob.X0),
                           keep_checkpoints=False).clone())
    ro = hp.Rollout(prob, checkpoint_every=4)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    X0 = to_dev(torch, prob.X0).requires_grad_(True)
    L = ((hp.IBRollout().apply(th, X0, ro) - to_dev(torch, Xt)) ** 2).sum()
    L.backward()
    fl = ref.fluid_from_problem(prob)
    mesh = ref.MeshBuffers.from_problem(prob)
    Lr, dX0r, dthr = ref.rollout_grad(fl, mesh, prob.initial_velocity(), prob.X0, 0.0,
                                      prob.n_steps, prob.p0, prob.T, Xt)
    assert abs(float(L.detach()) - Lr) <= 1e-9 * Lr
    assert_close("dL/dX0", host(X0.grad), dX0r, 1e-9)
    assert_close("dL/dtheta", th.grad.numpy(), dthr[0], 1e-8)


def test_sheet_state_and_argument_errors(torch_dev, hp, ref):
    prob = inputs.lv_block()
    say("lv errors")
    ctx = hp.Context(hp.config_for_problem(prob))
    ctx.set_mesh(prob.X_ref, prob.conn, prob.fibre, prob.mat_id)
    ctx.set_material(0, HO, prob.materials[0].params)
    import torch
    Xd = to_dev(torch, prob.X0)
    with pytest.raises(hp.HipIBError) as ei:
        ctx.fe_force(Xd, 0.0)
    assert ei.value.status == 6            # HIPIB_E_STATE: sheets missing
    with pytest.raises(hp.HipIBError) as ei:
        ctx.set_sheets(prob.sheet[:-1])
    assert ei.value.status == 1            # wrong element count
    bad = list(prob.materials[0].params)
    bad[6] = 0.0                           # a_s > 0 with b_s = 0
    with pytest.raises(hp.HipIBError):
        ctx.set_material(0, HO, bad)
    with pytest.raises(hp.HipIBError):
        ctx.set_active_tension(float("nan"))
    with pytest.raises(hp.HipIBError):
        ctx.set_active_waveform(1.0, 0.0, -1.0)
    ctx.set_sheets(prob.sheet)
    ctx.fe_force(Xd, 0.0)
    torch.cuda.synchronize()
    # the library's waveform and the oracle's agree at a few times
    for t in (0.0, 0.004, 0.01, 0.013, 0.02, 0.03):
        assert hp.active_tension(2.0, 0.0, 0.02, t) == ref.active_tension(2.0, 0.0, 0.02, t)


@pytest.mark.parametrize("det", [0, 1])
def test_tethers_force_and_hessian(torch_dev, hp, ref, det):
    """Random symmetric positive definite tethers on a third of the nodes of a
    HO block (with its elements): force and Hessian product against the oracle,
    in atomic and deterministic mode."""
    torch = torch_dev
    prob = inputs.ho_block(n=32, n_el=6)
    say("tethers", det)
    rng = np.random.default_rng(41)
    node = rng.choice(prob.n_nodes, size=prob.n_nodes // 3, replace=False).astype(np.int32)
    A = rng.standard_normal((node.size, 3, 3))
    Km = np.einsum("tij,tkj->tik", A, A) + 0.5 * np.eye(3)
    K = np.stack([Km[:, 0, 0], Km[:, 1, 1], Km[:, 2, 2], Km[:, 0, 1], Km[:, 0, 2], Km[:, 1, 2]], 1)
    Y = prob.X_ref[node] + 0.01 * prob.h * rng.standard_normal((node.size, 3))
    prob.tethers = (node, Y, K)
    x = deformed(prob, 12, 0.03)
    ctx = hp.context_for_problem(prob, deterministic=det)
    mesh = ref.MeshBuffers.from_problem(prob)
    F = host(ctx.fe_force(to_dev(torch, x), 0.0))
    assert_close("F", F, ref.fe_force(mesh, x)[0])
    V = rng.standard_normal(x.shape)
    HV = host(ctx.fe_hvp(to_dev(torch, x), to_dev(torch, V)))
    assert_close("HV", HV, ref.fe_hvp(mesh, x, V), 1e-10)
    bad = node.copy()
    bad[1] = bad[0]
    with pytest.raises(hp.HipIBError) as ei:
        ctx.set_tethers(bad, Y, K)
    assert ei.value.status == 1
    bad[1] = prob.n_nodes
    with pytest.raises(hp.HipIBError):
        ctx.set_tethers(bad, Y, K)
    ctx.set_tethers(node[:0], Y[:0], K[:0])          # no tethers: elastic force only
    F0 = host(ctx.fe_force(to_dev(torch, x), 0.0))
    mesh0 = ref.MeshBuffers.from_problem(prob)
    mesh0.s.n_tethers = 0
    assert_close("F (no tethers)", F0, ref.fe_force(mesh0, x)[0])
