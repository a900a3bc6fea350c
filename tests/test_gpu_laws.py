"""GPU parity for the other constitutive laws ("Constitutive laws"): the
modified standard reinforcing law Psi_1 and the fibre-reinforced models Psi_2
and Psi_3, in the force kernel, its Hessian product, whole steps and the
adjoint step, against the FP64 oracle (1e-11 relative for forward operators
and steps, 1e-10 for the derivative operators)."""
import numpy as np
import pytest

from paper_2503_22695_amd import inputs
from tests.test_gpu_parity import TOL, assert_close, deformed, host, say, to_dev

pytestmark = pytest.mark.gpu

LAWS = [inputs.STANDARD_REINFORCING, inputs.FIBRE_REINFORCED_1, inputs.FIBRE_REINFORCED_2]


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


@pytest.mark.parametrize("model", LAWS)
@pytest.mark.parametrize("det", [0, 1])
def test_force_and_hessian(torch_dev, hp, ref, model, det):
    torch = torch_dev
    prob = inputs.law_block(model)
    say("law force/hvp", model, det)
    # stretched along the fibre in part of the block, compressed elsewhere
    x = deformed(prob, 60 + model, 0.06)
    ctx = hp.context_for_problem(prob, deterministic=det)
    mesh = ref.MeshBuffers.from_problem(prob)
    xd = to_dev(torch, x)
    assert_close("F", host(ctx.fe_force(xd, 0.0)), ref.fe_force(mesh, x)[0])
    V = np.random.default_rng(70 + model).standard_normal(x.shape)
    assert_close("HV", host(ctx.fe_hvp(xd, to_dev(torch, V))), ref.fe_hvp(mesh, x, V), 1e-10)


@pytest.mark.parametrize("model", LAWS)
def test_advance_block(torch_dev, hp, ref, model):
    torch = torch_dev
    prob = inputs.law_block(model)
    say("law advance", model, prob.n_steps)
    sim = hp.Simulation(prob)
    sim.advance(prob.n_steps)
    torch.cuda.synchronize()
    cyc, _ = sim.ctx.step_stats()
    ur, pr, Xr, st = ref.run_problem(prob)
    assert [list(c) for c in cyc] == [list(s.cycles) for s in st]
    assert_close("u", host(sim.u), ur, TOL)
    assert_close("p", host(sim.p), pr, TOL)
    assert_close("X - X0", host(sim.X) - prob.X0, Xr - prob.X0, TOL)


def test_adjoint_step_standard_reinforcing(torch_dev, hp, ref):
    torch = torch_dev
    prob = inputs.law_block(inputs.STANDARD_REINFORCING)
    say("law adjoint step")
    n = prob.n
    rng = np.random.default_rng(81)
    fl = ref.fluid_from_problem(prob)
    mesh = ref.MeshBuffers.from_problem(prob)
    x0 = deformed(prob, 82, 0.04)
    u0 = ref.project(fl, 0.02 * rng.standard_normal((3, n, n, n)))
    u1, _, _, _ = ref.advance(fl, mesh, u0, np.zeros((n, n, n)), x0, 0.0, 1)
    lam_u = rng.standard_normal(u0.shape)
    lam_X = rng.standard_normal(x0.shape)
    lu_r, lX_r, _ = ref.adjoint_step(fl, mesh, u0, x0, u1, 0.0, lam_u, lam_X)
    ctx = hp.context_for_problem(prob)
    lu, lX = to_dev(torch, lam_u), to_dev(torch, lam_X)
    dth = torch.zeros((hp.MAX_MATERIALS, 4), dtype=torch.float64, device="cuda")
    ctx.adjoint_step(to_dev(torch, u0), to_dev(torch, x0), to_dev(torch, u1), 0.0, lu, lX, dth)
    torch.cuda.synchronize()
    assert_close("lam_u", host(lu), lu_r, 1e-10)
    assert_close("lam_X", host(lX), lX_r, 1e-10)
    assert float(dth.abs().max()) == 0.0      # gradients are taken in HO parameters only


def test_law_parameter_errors(torch_dev, hp):
    prob = inputs.law_block(inputs.STANDARD_REINFORCING)
    say("law errors")
    ctx = hp.context_for_problem(prob)
    for model, params in ((inputs.STANDARD_REINFORCING, (1.0, 2.0, 3.0)),
                          (inputs.FIBRE_REINFORCED_1, (1.0, 2.0, 0.0, 1.0)),
                          (inputs.FIBRE_REINFORCED_2, (1.0, 0.0, 1.0, 1.0, 1.0)),
                          (7, (1.0, 1.0))):
        with pytest.raises(hp.HipIBError) as ei:
            ctx.set_material(0, model, params)
        assert ei.value.status == 1
