"""Full-horizon parity of the benchmarked workloads against the FP64 oracle.

- The 128^3 Holzapfel-Ogden shell exactly as the benchmark runs it (X0 = X_ref,
  fluid at rest, t0 = 0, cavity pressure p0 sin^2(pi t / T) with T = 100 dt,
  100 steps), in FP64 and in the mixed-precision form, against one oracle
  run of the same 100 steps.
- The 192^3 shell with leaflets over its full 50 steps from the generated
  start (shell at X_ref, the seeded divergence-free flow).

Errors are stated in both the relative l2 norm and the relative max norm
(||a - b||_inf / ||b||_inf, so that an error confined to small-magnitude
regions, such as the pressure far from the solid, is not diluted).

Tolerance of the FP64 runs.  The elastic force is computed from positions, so
its relative rounding is about eps |X| / d at a displacement scale d.  From the
stress-free start d is zero: the first step (t = 0, no cavity pressure) spreads
a force that is pure rounding (~1e-13 of the later forces), and the two
implementations agree on nothing but its size.  That noise is a velocity
perturbation of ~eps |F_elastic| dt / rho, which the viscous and elastic
dynamics carry along without growth over 100 steps; the pressure-driven motion
that follows reaches displacements of 2.3e-3 after 100 steps, so the noise
is ~1e-13 relative to it.  The bar is therefore the target's 1e-11 in both
norms.  Measured on MI355X (l2 / max norm): u 8.0e-15 / 1.7e-14, p 8.3e-13 /
1.5e-12, X - X0 6.9e-14 / 2.4e-13 on the 128^3 shell after 100 steps.

Tolerance of the mixed-precision run: 1e-6 relative for u and p and for X
relative to the displacement (e_X = ||X - X_ref||_inf / ||X_ref - X0||_inf),
as the target states, and for u in the max norm.  Measured with FP32 element
forces: e_u 3.4e-9, e_p 3.9e-7, e_X 6.5e-8, u max norm 1.2e-8.  The
pressure's max-norm error, 1.3e-6 (4.1e-7 with FP64 element forces), is held
to 1e-5: it sits where the spread FP32 element forces are largest.
"""
import numpy as np
import pytest

from paper_2503_22695_amd import inputs
from tests.test_gpu_parity import host, rel, say

pytestmark = pytest.mark.gpu

TOL = 1e-11


def rel_inf(a, b):
    a, b = np.asarray(a), np.asarray(b)
    nb = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (nb if nb > 0 else 1.0))


def mean_free(p):
    return p - p.mean()


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


def oracle_run(ref, prob, n_steps, piece=10):
    """The oracle's run of n_steps from the generated start at t0 = 0, taken in
    pieces (identical to the one-call run) so each piece reports progress."""
    fl = ref.fluid_from_problem(prob)
    mesh = ref.MeshBuffers.from_problem(prob)
    u, p, X = prob.initial_velocity(), np.zeros((prob.n,) * 3), prob.X0.copy()
    stats = []
    for s in range(0, n_steps, piece):
        m = min(piece, n_steps - s)
        u, p, X, st = ref.advance(fl, mesh, u, p, X, 0.0, m, prob.p0, prob.T, first_step=s)
        stats += st
        say("oracle", prob.name, "steps", s + m, "of", n_steps)
    return u, p, X, stats


@pytest.fixture(scope="module")
def shell_128(ref):
    prob = inputs.workload("ho_shell_128")
    assert prob.n_steps == 100 and np.array_equal(prob.X0, prob.X_ref)
    return prob, oracle_run(ref, prob, prob.n_steps)


def errors(sim, prob, ur, pr, Xr):
    u, p, X = host(sim.u), host(sim.p), host(sim.X)
    return {
        "u_l2": rel(u, ur), "u_inf": rel_inf(u, ur),
        "p_l2": rel(mean_free(p), mean_free(pr)), "p_inf": rel_inf(mean_free(p), mean_free(pr)),
        "dX_l2": rel(X - prob.X0, Xr - prob.X0), "dX_inf": rel_inf(X - prob.X0, Xr - prob.X0),
    }


@pytest.mark.timeout(600)
def test_shell_128_benchmarked_run_fp64(torch_dev, hp, shell_128):
    torch = torch_dev
    prob, (ur, pr, Xr, st) = shell_128
    say("horizon FP64", prob.name, prob.n_steps)
    sim = hp.Simulation(prob)
    sim.advance(prob.n_steps)
    torch.cuda.synchronize()
    cyc, _ = sim.ctx.step_stats()
    assert [list(c) for c in cyc] == [list(s.cycles) for s in st]
    e = errors(sim, prob, ur, pr, Xr)
    say("FP64 errors", e, "max |X - X0|", float(np.max(np.abs(Xr - prob.X0))))
    bad = {k: v for k, v in e.items() if not v <= TOL}
    assert not bad, f"FP64 100-step shell errors above {TOL}: {bad}"


@pytest.mark.timeout(600)
def test_shell_128_benchmarked_run_mixed(torch_dev, hp, shell_128):
    torch = torch_dev
    prob, (ur, pr, Xr, st) = shell_128
    say("horizon mixed", prob.name, prob.n_steps)
    sim = hp.Simulation(prob, precision=hp.MIXED)
    sim.advance(prob.n_steps)
    torch.cuda.synchronize()
    u, p, X = host(sim.u), host(sim.p), host(sim.X)
    e_u = rel(u, ur)
    e_p = rel(mean_free(p), mean_free(pr))
    e_X = float(np.max(np.abs(X - Xr)) / np.max(np.abs(Xr - prob.X0)))
    e = dict(e_u=e_u, e_p=e_p, e_X=e_X, u_inf=rel_inf(u, ur))
    p_inf = rel_inf(mean_free(p), mean_free(pr))
    say("mixed errors vs the FP64 oracle", e, "p_inf", p_inf)
    bad = {k: v for k, v in e.items() if not v <= 1e-6}
    assert not bad, f"mixed-precision 100-step shell errors above 1e-6: {bad}"
    # the pressure's largest pointwise error sits where the spread FP32 element
    # forces are largest: their rounding, relative to the element contributions,
    # survives the cancellation between neighbouring elements at a node
    assert p_inf <= 1e-5


@pytest.mark.timeout(600)
def test_shell_leaflets_192_generated_start(torch_dev, hp, ref):
    torch = torch_dev
    prob = inputs.workload("shell_leaflets_192")
    n_steps = prob.n_steps
    assert n_steps == 50
    say("horizon", prob.name, n_steps)
    ur, pr, Xr, st = oracle_run(ref, prob, n_steps)
    sim = hp.Simulation(prob)
    sim.advance(n_steps)
    torch.cuda.synchronize()
    cyc, _ = sim.ctx.step_stats()
    assert [list(c) for c in cyc] == [list(s.cycles) for s in st]
    e = errors(sim, prob, ur, pr, Xr)
    say("192^3 errors", e)
    bad = {k: v for k, v in e.items() if not v <= TOL}
    assert not bad, f"192^3 errors above {TOL}: {bad}"
