"""hipib_get_stats and the phase timing, through the C-ABI.

- the records of the last step call (cycles, residuals) equal the per-step
  records;
- kinetic energy, momentum and the largest discrete divergence of u equal
  their numpy sums over the same array;
- the solid's volume equals the volume its boundary quads enclose (a surface
  integral, divergence theorem, from numpy), and J_min / J_max are the extreme
  det F over the 2x2x2 Gauss points written out with numpy;
- a run from rest keeps the momentum at rounding level (the elastic forces
  sum to zero) and u divergence-free to the Poisson tolerance;
- phase timing counts the timed steps, every phase takes time, and the
  phases of a step do not exceed its wall time.
"""
import time

import numpy as np
import pytest

from paper_2503_22695_amd import inputs
from tests.test_gpu_parity import host, say, to_dev

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


GP = 1.0 / np.sqrt(3.0)


def hex_dN(xi):
    """dN_a/dxi of the trilinear hex, node a at ((a & 1), (a >> 1) & 1, (a >> 2) & 1)."""
    out = np.zeros((8, 3))
    for a in range(8):
        s = np.array([(a & 1) * 2 - 1, ((a >> 1) & 1) * 2 - 1, ((a >> 2) & 1) * 2 - 1], float)
        f = (1 + s * xi) / 2
        out[a] = [s[0] / 2 * f[1] * f[2], f[0] * s[1] / 2 * f[2], f[0] * f[1] * s[2] / 2]
    return out


def jacobians(X, Xref, conn):
    Js = []
    for e in conn:
        for g in range(8):
            xi = np.array([GP if g & 1 else -GP, GP if g & 2 else -GP, GP if g & 4 else -GP])
            dN = hex_dN(xi)
            Jx, Jr = X[e].T @ dN, Xref[e].T @ dN
            Js.append(np.linalg.det(Jx @ np.linalg.inv(Jr)))
    return np.array(Js)


HEX_FACES = [(0, 2, 6, 4), (1, 3, 7, 5), (0, 1, 5, 4), (2, 3, 7, 6), (0, 1, 3, 2), (4, 5, 7, 6)]


def enclosed_volume_of_hexes(X, conn):
    """(1/3) surface integral of x.n over the faces that belong to one hex only,
    each oriented away from its hex's centroid; 5x5 Gauss-Legendre per face."""
    count = {}
    for e, c in enumerate(conn):
        for f in HEX_FACES:
            key = tuple(sorted(int(c[a]) for a in f))
            count.setdefault(key, []).append((e, f))
    g, w = np.polynomial.legendre.leggauss(5)
    V = 0.0
    for key, owners in count.items():
        if len(owners) != 1:
            continue
        e, f = owners[0]
        P = X[conn[e][list(f)]]
        centre = X[conn[e]].mean(0)
        sign = 1.0 if np.dot(np.cross(P[1] - P[0], P[3] - P[0]), P.mean(0) - centre) > 0 else -1.0
        for s, ws in zip(g, w):
            for t, wt in zip(g, w):
                # bilinear face through P0 (s,t = -1,-1), P1 (1,-1), P2 (1,1), P3 (-1,1)
                N = np.array([(1 - s) * (1 - t), (1 + s) * (1 - t), (1 + s) * (1 + t), (1 - s) * (1 + t)]) / 4
                dNs = np.array([-(1 - t), (1 - t), (1 + t), -(1 + t)]) / 4
                dNt = np.array([-(1 - s), -(1 + s), (1 + s), (1 - s)]) / 4
                x = N @ P
                nA = np.cross(dNs @ P, dNt @ P)
                V += sign * ws * wt * np.dot(x, nA) / 3.0
    return V


def test_stats_match_their_definitions(torch_dev, hp):
    torch = torch_dev
    prob = inputs.neo_hookean_block()
    say("stats", prob.name)
    sim = hp.Simulation(prob)
    sim.advance(prob.n_steps)
    torch.cuda.synchronize()
    st = sim.ctx.get_stats(sim.u, sim.X)
    cyc, rr = sim.ctx.step_stats()
    assert st["steps"] == prob.n_steps == len(cyc)
    assert st["cycles_last"] == list(cyc[-1])
    assert np.allclose(st["relres_last"], rr[-1], rtol=0, atol=0)
    assert np.allclose(st["cycles_mean"], cyc.mean(0), rtol=1e-15)
    u, X = host(sim.u), host(sim.X)
    h3 = prob.h ** 3
    ke = 0.5 * prob.rho * h3 * np.sum(u * u)
    mom = prob.rho * h3 * u.reshape(3, -1).sum(1)
    div = (np.roll(u[0], -1, 2) - u[0] + np.roll(u[1], -1, 1) - u[1] + np.roll(u[2], -1, 0) - u[2]) / prob.h
    assert abs(st["kinetic_energy"] - ke) <= 1e-12 * ke
    assert np.max(np.abs(np.array(st["momentum"]) - mom)) <= 1e-12 * prob.rho * h3 * np.sum(np.abs(u))
    # (each divergence is a difference of O(|u|) values: rounding relative to |u| / h)
    assert abs(st["max_abs_div"] - np.max(np.abs(div))) <= 1e-12 * np.max(np.abs(u)) / prob.h
    # the run from rest: momentum stays at rounding level, u divergence-free
    assert np.max(np.abs(st["momentum"])) <= 1e-12 * prob.rho * h3 * np.sum(np.abs(u))
    assert st["max_abs_div"] <= 1e-6 * np.max(np.abs(u)) / prob.h
    V = enclosed_volume_of_hexes(X, prob.conn)
    say("volume", st["volume"], V, "J", st["J_min"], st["J_max"])
    assert abs(st["volume"] - V) <= 1e-12 * V
    J = jacobians(X, prob.X_ref, prob.conn)
    assert abs(st["J_min"] - J.min()) <= 1e-12 and abs(st["J_max"] - J.max()) <= 1e-12
    # no arrays: records and times only
    st0 = sim.ctx.get_stats()
    assert st0["kinetic_energy"] == 0.0 and st0["volume"] == 0.0 and st0["steps"] == prob.n_steps


def test_phase_timing(torch_dev, hp):
    torch = torch_dev
    prob = inputs.workload("ho_block_64")
    say("phase timing", prob.name)
    sim = hp.Simulation(prob)
    sim.advance(2)
    sim.ctx.set_phase_timing(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    sim.advance(3)
    torch.cuda.synchronize()
    wall_ms = 1e3 * (time.perf_counter() - t)
    st = sim.ctx.get_stats()
    ph = st["phase_ms"]
    say("phases", ph, "wall", wall_ms)
    assert st["timed_steps"] == 3
    assert all(v > 0.0 for v in ph.values())
    main = sum(v for k, v in ph.items() if k != "forces")
    assert main <= wall_ms
    sim.ctx.set_phase_timing(False)
    sim.advance(1)
    assert sim.ctx.get_stats()["timed_steps"] == 0
