"""Pins of the oracle's walled box (boundary conditions u* = 0 and u.n = 0 on
the box faces, "Spatial Discretization"), computed on the box's mirror image.

The walled MAC operators are written out here independently with explicit
ghost values (tangential ghost = minus the interior value, wall-normal face
values zero, pressure ghost = the interior value) and the oracle is checked
against them: Dirichlet and Neumann solves (also on exact discrete
eigenvectors), ext / fold / restrict identities, a whole Stokes step
(Helmholtz, Poisson and projection equations of the step hold with the
walled operators, no penetration, zero divergence), spreading and
interpolation as transposes, and spreading away from the walls equal to the
periodic spreading."""
import numpy as np
import pytest

from paper_2503_22695_amd import inputs


def lap_walled_scalar(q, h, neumann):
    """Cell-centred 7-point Laplacian, ghost = +q (Neumann) or -q (Dirichlet)."""
    s = 1.0 if neumann else -1.0
    out = -6.0 * q
    for ax in range(3):
        qp = np.roll(q, -1, axis=ax)
        qm = np.roll(q, 1, axis=ax)
        idx_hi = [slice(None)] * 3
        idx_lo = [slice(None)] * 3
        idx_hi[ax] = -1
        idx_lo[ax] = 0
        qp[tuple(idx_hi)] = s * q[tuple(idx_hi)]
        qm[tuple(idx_lo)] = s * q[tuple(idx_lo)]
        out = out + qp + qm
    return out / h ** 2


def lap_walled_velocity(u, h):
    """Component d of u (array axes (k, j, i) = (z, y, x)): face-centred along its
    own axis with the wall faces (index 0) held at zero, Dirichlet ghosts
    (minus the interior value) across the other axes."""
    out = np.empty_like(u)
    for d in range(3):
        q = u[d].copy()
        ax_own = 2 - d
        res = -6.0 * q
        for ax in range(3):
            qp = np.roll(q, -1, axis=ax)
            qm = np.roll(q, 1, axis=ax)
            if ax != ax_own:
                hi = [slice(None)] * 3
                lo = [slice(None)] * 3
                hi[ax] = -1
                lo[ax] = 0
                qp[tuple(hi)] = -q[tuple(hi)]
                qm[tuple(lo)] = -q[tuple(lo)]
            res = res + qp + qm            # own axis: wrap to face 0, which is zero
        w = [slice(None)] * 3
        w[ax_own] = 0
        res[tuple(w)] = 0.0
        out[d] = res / h ** 2
    return out


def div_walled(u, h):
    return sum(np.roll(u[d], -1, axis=2 - d) - u[d] for d in range(3)) / h


def grad_walled(p, h):
    g = np.empty((3,) + p.shape)
    for d in range(3):
        ax = 2 - d
        g[d] = (p - np.roll(p, 1, axis=ax)) / h
        w = [slice(None)] * 3
        w[ax] = 0
        g[d][tuple(w)] = 0.0
    return g


def wall_faces_zero(u):
    for d in range(3):
        w = [slice(None)] * 3
        w[2 - d] = 0
        u[d][tuple(w)] = 0.0
    return u


@pytest.mark.parametrize("n", [8, 12])
def test_walled_poisson_and_helmholtz_solves(ref, n):
    rng = np.random.default_rng(n)
    h = 1.0 / n
    fl = ref.fluid(n, rtol=1e-13, walls=1)
    b = rng.standard_normal((n, n, n))
    b -= b.mean()
    p, cyc, rr = ref.walled_solve(fl, 0.0, 1.0, True, b)
    r = b + lap_walled_scalar(p, h, True)
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b), cyc
    sigma, nu = 50.0, 0.3
    x, cyc, rr = ref.walled_solve(fl, sigma, nu, False, b)
    r = b - (sigma * x - nu * lap_walled_scalar(x, h, False))
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b), cyc


def test_walled_eigenvectors(ref):
    """cos(pi k (i+1/2)/n) (Neumann) and sin(pi k (i+1/2)/n) (Dirichlet with the
    odd ghost) are exact eigenvectors of the walled Laplacian, eigenvalue
    -(4/h^2) sum sin^2(pi k_a / 2n)."""
    n = 8
    h = 1.0 / n
    fl = ref.fluid(n, rtol=1e-13, walls=1)
    c = np.arange(n) + 0.5
    kx, ky, kz = 1, 3, 2
    lam = -(4 / h ** 2) * sum(np.sin(np.pi * k / (2 * n)) ** 2 for k in (kx, ky, kz))
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    e = np.cos(np.pi * kx * X / n) * np.cos(np.pi * ky * Y / n) * np.cos(np.pi * kz * Z / n)
    p, _, _ = ref.walled_solve(fl, 0.0, 1.0, True, e)
    assert np.max(np.abs(p - e / (-lam))) <= 1e-10 * np.max(np.abs(e / lam))
    e = np.sin(np.pi * kx * X / n) * np.sin(np.pi * ky * Y / n) * np.sin(np.pi * kz * Z / n)
    x, _, _ = ref.walled_solve(fl, 0.0 + 10.0, 1.0, False, e)
    assert np.max(np.abs(x - e / (10.0 - lam))) <= 1e-10 * np.max(np.abs(e / (10.0 - lam)))


def test_extend_fold_restrict(ref):
    n = 6
    rng = np.random.default_rng(3)
    a = rng.standard_normal((3, n, n, n))
    bimg = rng.standard_normal((3, 2 * n, 2 * n, 2 * n))
    ea = ref.wall_extend(a, True)
    fb = ref.wall_fold(bimg)
    assert abs(np.sum(ea * bimg) - np.sum(a * fb)) <= 1e-12 * np.sum(np.abs(ea * bimg))
    assert np.array_equal(ref.wall_restrict(ea, True), wall_faces_zero(a.copy()))
    s = rng.standard_normal((n, n, n))
    es = ref.wall_extend(s, False)
    assert np.array_equal(ref.wall_restrict(es, False), s)
    # symmetry of the images: even for scalars, odd for velocity, wall faces zero
    assert np.array_equal(es, es[::-1][:, :, :])
    assert np.array_equal(ea[1], -ea[1][:, :, ::-1])     # u^y mirrored across x walls
    assert np.all(ea[0][:, :, 0] == 0) and np.all(ea[0][:, :, n] == 0)


def test_walled_stokes_step_satisfies_the_walled_equations(ref):
    """One walled Stokes step: with u* recovered as u^{n+1} + (dt/rho) G p, the
    Helmholtz, Poisson and projection equations hold with the walled operators;
    no flow through the walls, zero divergence."""
    n = 12
    h = 1.0 / n
    rho, mu, dt = 1.0, 0.05, 2e-3
    fl = ref.fluid(n, rho=rho, mu=mu, dt=dt, rtol=1e-13, convection=0, walls=1)
    rng = np.random.default_rng(5)
    u0 = wall_faces_zero(0.1 * rng.standard_normal((3, n, n, n)))
    f = wall_faces_zero(rng.standard_normal((3, n, n, n)))
    p0 = np.zeros((n, n, n))
    u1, p1, _ = ref.ns_step(fl, f, u0, p0)
    for d in range(3):
        w = [slice(None)] * 3
        w[2 - d] = 0
        assert np.all(u1[d][tuple(w)] == 0.0)
    assert np.max(np.abs(div_walled(u1, h))) <= 1e-9 * np.max(np.abs(div_walled(u0, h)) + 1)
    us = u1 + dt / rho * grad_walled(p1, h)
    res_h = rho / dt * (us - u0) - mu * lap_walled_velocity(us, h) - f
    res_h = wall_faces_zero(res_h)
    assert np.max(np.abs(res_h)) <= 1e-8 * np.max(np.abs(f))
    rhs_p = rho / dt * div_walled(us, h)
    res_p = lap_walled_scalar(p1, h, True) - rhs_p
    assert np.max(np.abs(res_p)) <= 1e-8 * np.max(np.abs(rhs_p))


def test_walled_spread_interp_transpose_and_interior_agreement(ref):
    n = 16
    h = 1.0 / n
    rng = np.random.default_rng(7)
    X = rng.uniform(0.02, 0.98, (40, 3))            # some within 2h of a wall
    F = rng.standard_normal((40, 3))
    u = wall_faces_zero(rng.standard_normal((3, n, n, n)))
    f = ref.walled_spread(n, X, F)
    U = ref.walled_interpolate(X, u)
    assert abs(np.sum(f * u) * h ** 3 - np.sum(F * U)) <= 1e-12 * np.sum(np.abs(F * U))
    Xi = rng.uniform(2.5 * h, 1 - 2.5 * h, (30, 3))   # away from the walls
    Fi = rng.standard_normal((30, 3))
    fw = ref.walled_spread(n, Xi, Fi)
    fp = ref.spread(n, Xi, Fi)
    assert np.max(np.abs(fw - fp)) <= 1e-13 * np.max(np.abs(fp))
    assert np.max(np.abs(ref.walled_interpolate(Xi, u) - ref.interpolate(Xi, u))) <= 1e-13


def test_walled_ib_run_keeps_the_walls(ref):
    """A NH block in a walled 16^3 box: ten steps with convection; every step
    keeps zero wall-normal velocity and a divergence-free field, and the block
    stays inside."""
    prob = inputs.neo_hookean_block(n=16, n_steps=10)
    prob.walls = 1
    u, p, X, st = ref.run_problem(prob)
    h = prob.h
    for d in range(3):
        w = [slice(None)] * 3
        w[2 - d] = 0
        assert np.all(u[d][tuple(w)] == 0.0)
    assert np.max(np.abs(div_walled(u, h))) <= 1e-7 * np.max(np.abs(u)) / h
    assert np.all((X > 0) & (X < 1))
    assert all(s.cycles[3] > 0 for s in st)
