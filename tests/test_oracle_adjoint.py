"""Pins of the oracle's discrete adjoint: every reverse-mode piece against a
finite difference of the corresponding forward oracle function (or an exact
identity), then one adjoint step and a whole rollout gradient against central
differences of the forward step.

C(u) is quadratic, so its central difference is exact up to rounding; the
other pieces are C^1 and checked at ~1e-7 relative."""
import math

import numpy as np
import pytest

from paper_2503_22695_amd import inputs

NH, HO = inputs.NEO_HOOKEAN, inputs.HOLZAPFEL_OGDEN
HO_PAR = (0.5, 5.0, 1.5, 8.0, 7.0)


def test_convection_transpose_dot_product(ref):
    rng = np.random.default_rng(0)
    n = 8
    u = rng.standard_normal((3, n, n, n))
    v = rng.standard_normal((3, n, n, n))
    lam = rng.standard_normal((3, n, n, n))
    eps = 1e-3
    jv = (ref.convection(u + eps * v) - ref.convection(u - eps * v)) / (2 * eps)
    lhs = np.sum(jv * lam)
    rhs = np.sum(v * ref.convection_vjp(u, lam))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_dphi_matches_difference_quotient(ref):
    for r in np.linspace(-2.3, 2.3, 97):
        e = 1e-6
        fd = (ref.phi(r + e) - ref.phi(r - e)) / (2 * e)
        assert abs(ref.dphi(r) - fd) < 1e-8, r
    assert ref.dphi(0.0) == 0.0 and ref.dphi(2.0) == 0.0
    assert abs(ref.dphi(1.0 - 1e-12) - ref.dphi(1.0 + 1e-12)) < 1e-9   # C^1 at |r| = 1


def test_spread_and_interp_position_derivatives(ref):
    n = 8
    rng = np.random.default_rng(1)
    X = rng.uniform(-0.2, 1.2, (7, 3))
    F = rng.standard_normal((7, 3))
    lam_f = rng.standard_normal((3, n, n, n))
    u = rng.standard_normal((3, n, n, n))
    lamU = rng.standard_normal((7, 3))
    gS = ref.spread_vjp_X(n, X, F, lam_f)
    gJ = ref.interp_vjp_X(X, u, lamU)
    eps = 1e-7
    for q in range(7):
        for e in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[q, e] += eps
            Xm[q, e] -= eps
            fdS = (np.sum(ref.spread(n, Xp, F) * lam_f) - np.sum(ref.spread(n, Xm, F) * lam_f)) / (2 * eps)
            fdJ = (np.sum(ref.interpolate(Xp, u) * lamU) - np.sum(ref.interpolate(Xm, u) * lamU)) / (2 * eps)
            assert abs(gS[q, e] - fdS) <= 1e-6 * max(1.0, abs(fdS)), (q, e)
            assert abs(gJ[q, e] - fdJ) <= 1e-6 * max(1.0, abs(fdJ)), (q, e)


@pytest.mark.parametrize("model,par", [(NH, (10.0, 100.0)), (HO, HO_PAR)])
def test_pk1_tangent_matches_difference_quotient(ref, model, par):
    rng = np.random.default_rng(2)
    ef = np.array([0.6, 0.8, 0.0])
    for _ in range(5):
        Fm = np.eye(3) + 0.15 * rng.standard_normal((3, 3)) + 0.2 * np.outer(ef, ef)
        dF = rng.standard_normal((3, 3))
        dP = ref.pk1_tangent(model, par, Fm, dF, ef)
        e = 1e-6
        fd = (ref.pk1(model, par, Fm + e * dF, ef)[0] - ref.pk1(model, par, Fm - e * dF, ef)[0]) / (2 * e)
        assert np.max(np.abs(dP - fd)) <= 1e-7 * max(1.0, np.max(np.abs(dP)))


def small_mesh(ref, model=HO, par=HO_PAR, n_el=2, seed=3):
    X, conn = inputs.block_mesh(n_el, 0.3)
    rng = np.random.default_rng(seed)
    g = rng.uniform(-0.7, 0.7, conn.shape[0])
    fib = np.stack([np.cos(g), np.sin(g), 0 * g], 1)
    mesh = ref.MeshBuffers(X, conn, fib, np.zeros(conn.shape[0]), [model], [list(par) + [0] * (5 - len(par))])
    x = X * np.array([1.1, 0.96, 0.98]) + 0.004 * rng.standard_normal(X.shape)
    return mesh, X, x


def test_fe_hvp_matches_force_difference_and_is_symmetric(ref):
    mesh, X, x = small_mesh(ref)
    rng = np.random.default_rng(4)
    V1, V2 = rng.standard_normal(x.shape), rng.standard_normal(x.shape)
    H1 = ref.fe_hvp(mesh, x, V1)
    e = 1e-6
    fd = (ref.fe_force(mesh, x + e * V1)[0] - ref.fe_force(mesh, x - e * V1)[0]) / (2 * e)
    assert np.max(np.abs(H1 - fd)) <= 1e-6 * np.max(np.abs(H1))
    H2 = ref.fe_hvp(mesh, x, V2)
    assert abs(np.sum(V2 * H1) - np.sum(V1 * H2)) <= 1e-11 * np.sum(np.abs(V2 * H1))


def test_fe_param_vjp_matches_parameter_difference(ref):
    mesh, X, x = small_mesh(ref)
    rng = np.random.default_rng(5)
    lam = rng.standard_normal(x.shape)
    g = ref.fe_param_vjp(mesh, x, lam)[0]
    for k in range(4):
        par = np.array(HO_PAR)
        e = 1e-6 * par[k]
        pp, pm = par.copy(), par.copy()
        pp[k] += e
        pm[k] -= e
        mp = ref.MeshBuffers(mesh.X_ref, mesh.conn, mesh.fibre, mesh.mat_id, [HO], [pp])
        mm = ref.MeshBuffers(mesh.X_ref, mesh.conn, mesh.fibre, mesh.mat_id, [HO], [pm])
        fd = (np.sum(ref.fe_force(mp, x)[0] * lam) - np.sum(ref.fe_force(mm, x)[0] * lam)) / (2 * e)
        assert abs(g[k] - fd) <= 1e-6 * max(1e-8, abs(fd)), (k, g[k], fd)


def test_pressure_vjp_matches_difference(ref):
    from tests.test_oracle_fe import closed_box_surface
    x, quads = closed_box_surface(m=2, jitter=0.03, seed=2)
    rng = np.random.default_rng(6)
    lam = rng.standard_normal(x.shape)
    g = ref.pressure_vjp(quads, x, 1.3, lam)
    e = 1e-7
    for q in range(0, len(x), 2):
        for r in range(3):
            xp, xm = x.copy(), x.copy()
            xp[q, r] += e
            xm[q, r] -= e
            fd = (np.sum(ref.pressure_load(quads, xp, 1.3) * lam) -
                  np.sum(ref.pressure_load(quads, xm, 1.3) * lam)) / (2 * e)
            assert abs(g[q, r] - fd) <= 1e-7 * max(1.0, abs(fd))


def test_projection_is_symmetric_idempotent_and_solenoidal(ref):
    n = 16
    fl = ref.fluid(n, rtol=1e-13)
    rng = np.random.default_rng(7)
    v, w = rng.standard_normal((3, n, n, n)), rng.standard_normal((3, n, n, n))
    Pv, Pw = ref.project(fl, v), ref.project(fl, w)
    assert abs(np.sum(Pv * w) - np.sum(v * Pw)) <= 1e-11 * np.sum(np.abs(Pv * w))
    assert np.max(np.abs(ref.project(fl, Pv) - Pv)) <= 1e-10 * np.max(np.abs(Pv))
    assert np.max(np.abs(ref.divergence(Pv))) <= 1e-9 * np.max(np.abs(ref.divergence(v)))
    p = rng.standard_normal((n, n, n))
    assert np.max(np.abs(ref.project(fl, ref.gradient(p)))) <= 1e-9 * np.max(np.abs(ref.gradient(p)))


def step_problem(ref, n=16, convection=1, with_pressure=False):
    prob = inputs.ho_block(n=n, n_el=3, n_steps=4)
    fl = ref.fluid_from_problem(prob, rtol=1e-14, convection=convection)
    mesh = ref.MeshBuffers.from_problem(prob)
    rng = np.random.default_rng(8)
    u0 = 0.05 * rng.standard_normal((3, n, n, n))
    u0 = ref.project(ref.fluid(n, rtol=1e-14), u0)
    return prob, fl, mesh, u0



@pytest.mark.parametrize("convection", [1, 0])
def test_adjoint_step_against_central_difference(ref, convection):
    prob, fl, mesh, u0 = step_problem(ref, convection=convection)
    n = prob.n
    rng = np.random.default_rng(9)
    X0 = prob.X0

    def fwd(u, X):
        uu, pp, XX, _ = ref.advance(fl, mesh, u, np.zeros((n, n, n)), X, 0.0, 1)
        return uu, XX
    u1, X1 = fwd(u0, X0)
    lam_u1 = rng.standard_normal(u1.shape)
    lam_X1 = rng.standard_normal(X1.shape)
    lu0, lX0, dth = ref.adjoint_step(fl, mesh, u0, X0, u1, 0.0, lam_u1, lam_X1)
    du = ref.project(ref.fluid(n, rtol=1e-14), rng.standard_normal(u0.shape))
    dX = rng.standard_normal(X0.shape)
    for (a, b, pred) in [(du, 0 * dX, np.sum(lu0 * du)), (0 * du, dX, np.sum(lX0 * dX))]:
        e = 1e-6
        up, Xp = fwd(u0 + e * a, X0 + e * b)
        um, Xm = fwd(u0 - e * a, X0 - e * b)
        fd = (np.sum((up - um) * lam_u1) + np.sum((Xp - Xm) * lam_X1)) / (2 * e)
        assert abs(pred - fd) <= 2e-6 * max(abs(fd), 1e-12), (pred, fd)


def test_rollout_gradient_against_central_difference(ref):
    """Gradient of L = sum |X^N - X_target|^2 over 3 steps with respect to the
    four Holzapfel-Ogden parameters and to X0.  The theta-sensitivity over 3
    steps is ~1e-9, so the theta differences use a 1e-3 relative step (the
    rounding of L dominates smaller steps); the X0 directions also check that
    the central-difference error falls as eps^2 (Taylor remainder)."""
    prob, fl, mesh, u0 = step_problem(ref)
    n_steps = 3
    Xt = prob.X0 + 0.01 * prob.h
    L, dX0, dth = ref.rollout_grad(fl, mesh, u0, prob.X0, 0.0, n_steps, 0.0, 1.0, Xt)

    def loss(par, X0):
        m = ref.MeshBuffers(prob.X_ref, prob.conn, prob.fibre, prob.mat_id, [HO], [par])
        _, _, XN, _ = ref.advance(fl, m, u0, np.zeros((prob.n,) * 3), X0, 0.0, n_steps)
        return float(np.sum((XN - Xt) ** 2))
    assert abs(L - loss(list(HO_PAR), prob.X0)) <= 1e-14 * abs(L) + 1e-300
    for k in range(4):
        par = np.array(HO_PAR)
        e = 1e-3 * par[k]
        pp, pm = par.copy(), par.copy()
        pp[k] += e
        pm[k] -= e
        fd = (loss(pp, prob.X0) - loss(pm, prob.X0)) / (2 * e)
        assert abs(dth[0, k] - fd) <= 2e-6 * abs(fd), (k, dth[0, k], fd)
    rng = np.random.default_rng(10)
    for _ in range(2):
        d = rng.standard_normal(prob.X0.shape)
        g = np.sum(dX0 * d)
        errs = []
        for e in (1e-4, 1e-5, 1e-6):
            fd = (loss(list(HO_PAR), prob.X0 + e * d) - loss(list(HO_PAR), prob.X0 - e * d)) / (2 * e)
            errs.append(abs(g - fd))
        assert errs[2] <= 1e-8 * abs(g)
        assert 30 < errs[0] / errs[1] < 300          # second-order remainder
