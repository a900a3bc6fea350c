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


def test_pad_is_the_transpose_of_restrict(ref):
    n = 6
    rng = np.random.default_rng(11)
    for vector in (True, False):
        shp = ((3,) if vector else ()) + (2 * n,) * 3
        img = rng.standard_normal(shp)
        box = rng.standard_normal(shp[:-3] + (n,) * 3)
        lhs = np.sum(ref.wall_restrict(img, vector) * box)
        rhs = np.sum(img * ref.wall_pad(box, vector))
        assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(img)), vector


def walled_step_problem(ref, n=12, convection=1):
    prob = inputs.ho_block(n=n, n_el=3, n_steps=4)
    prob.walls = 1
    fl = ref.fluid_from_problem(prob, rtol=1e-14, convection=convection)
    mesh = ref.MeshBuffers.from_problem(prob)
    rng = np.random.default_rng(8)
    u0 = wall_faces_zero(0.05 * rng.standard_normal((3, n, n, n)))
    return prob, fl, mesh, u0


@pytest.mark.parametrize("convection", [1, 0])
def test_walled_adjoint_step_against_central_difference(ref, convection):
    """The reverse of one walled IB step against central differences of the
    forward step, along a random velocity direction (wall faces included: the
    step ignores them, so their adjoint is zero) and a random node direction."""
    prob, fl, mesh, u0 = walled_step_problem(ref, convection=convection)
    n = prob.n
    rng = np.random.default_rng(9)
    X0 = prob.X0

    def fwd(u, X):
        uu, _, XX, _ = ref.advance(fl, mesh, u, np.zeros((n, n, n)), X, 0.0, 1)
        return uu, XX
    u1, X1 = fwd(u0, X0)
    lam_u1 = rng.standard_normal(u1.shape)
    lam_X1 = rng.standard_normal(X1.shape)
    lu0, lX0, _ = ref.adjoint_step(fl, mesh, u0, X0, u1, 0.0, lam_u1, lam_X1)
    assert np.array_equal(wall_faces_zero(lu0.copy()), lu0)
    du = rng.standard_normal(u0.shape)
    dX = rng.standard_normal(X0.shape)
    for (a, b, pred) in [(du, 0 * dX, np.sum(lu0 * du)), (0 * du, dX, np.sum(lX0 * dX))]:
        e = 1e-6
        up, Xp = fwd(u0 + e * a, X0 + e * b)
        um, Xm = fwd(u0 - e * a, X0 - e * b)
        fd = (np.sum((up - um) * lam_u1) + np.sum((Xp - Xm) * lam_X1)) / (2 * e)
        assert abs(pred - fd) <= 2e-6 * max(abs(fd), 1e-12), (pred, fd)


def test_walled_rollout_gradient_against_central_difference(ref):
    """Gradient of L = sum |X^N - X_target|^2 over 3 walled steps with respect
    to X0 (two directions, second-order remainder) and the first parameter."""
    prob, fl, mesh, u0 = walled_step_problem(ref)
    n_steps = 3
    Xt = prob.X0 + 0.01 * prob.h
    L, dX0, dth = ref.rollout_grad(fl, mesh, u0, prob.X0, 0.0, n_steps, 0.0, 1.0, Xt)
    par0 = list(prob.materials[0].params)

    def loss(par, X0):
        m = ref.MeshBuffers(prob.X_ref, prob.conn, prob.fibre, prob.mat_id,
                            [prob.materials[0].model], [par])
        _, _, XN, _ = ref.advance(fl, m, u0, np.zeros((prob.n,) * 3), X0, 0.0, n_steps)
        return float(np.sum((XN - Xt) ** 2))
    assert abs(L - loss(par0, prob.X0)) <= 1e-14 * abs(L) + 1e-300
    par = np.array(par0)
    e = 1e-3 * par[0]
    pp, pm = par.copy(), par.copy()
    pp[0] += e
    pm[0] -= e
    fd = (loss(pp, prob.X0) - loss(pm, prob.X0)) / (2 * e)
    assert abs(dth[0, 0] - fd) <= 2e-6 * abs(fd), (dth[0, 0], fd)
    rng = np.random.default_rng(10)
    d = rng.standard_normal(prob.X0.shape)
    g = np.sum(dX0 * d)
    errs = []
    for e in (1e-4, 1e-5, 1e-6):
        fd = (loss(par0, prob.X0 + e * d) - loss(par0, prob.X0 - e * d)) / (2 * e)
        errs.append(abs(g - fd))
    assert errs[2] <= 1e-8 * abs(g)
    assert 30 < errs[0] / errs[1] < 300


def test_walled_adjoint_step_shell_with_pressure(ref):
    """The reverse of a walled step of a Holzapfel-Ogden shell under the
    follower cavity pressure, against a central difference along a random node
    direction.  The shell is inflated 2% across its axis: at the reference
    configuration the fibre invariant sits exactly on the kink of the fibres'
    tension-only switch, where the force is not differentiable."""
    import math
    n = 32
    prob = inputs.walled_shell(n=n, n_theta=112, n_psi=40, n_tau=3)
    fl = ref.fluid_from_problem(prob, rtol=1e-13)
    mesh = ref.MeshBuffers.from_problem(prob)
    rng = np.random.default_rng(42)
    u0 = 0.02 * rng.standard_normal((3, n, n, n))
    t0 = 0.3 * prob.T
    pressure = prob.p0 * math.sin(math.pi * t0 / prob.T) ** 2
    c = np.array([0.5, 0.5, 0.5])
    x0 = c + (prob.X_ref - c) * np.array([1.0, 1.02, 1.02])

    def fwd(u, X):
        uu, _, XX, _ = ref.advance(fl, mesh, u, np.zeros((n, n, n)), X, t0, 1, prob.p0, prob.T)
        return uu, XX
    u1, _ = fwd(u0, x0)
    lam_u = rng.standard_normal(u0.shape)
    lam_X = rng.standard_normal(x0.shape)
    _, lX, _ = ref.adjoint_step(fl, mesh, u0, x0, u1, pressure, lam_u, lam_X)
    dX = rng.standard_normal(x0.shape)
    e = 1e-6
    up, Xp = fwd(u0, x0 + e * dX)
    um, Xm = fwd(u0, x0 - e * dX)
    fd = (np.sum((up - um) * lam_u) + np.sum((Xp - Xm) * lam_X)) / (2 * e)
    assert abs(np.sum(lX * dX) - fd) <= 2e-6 * abs(fd), (np.sum(lX * dX), fd)


@pytest.mark.parametrize("convection", [1, 0])
def test_walled_adjoint_step_nodes_at_the_walls(ref, convection):
    """Tethered free nodes, half of them within 2h of a wall: the reverse step
    against central differences along random velocity and node directions,
    so the position derivatives of spreading and interpolation are checked
    where their stencils reach across the walls."""
    prob = inputs.wall_nodes()
    n = prob.n
    fl = ref.fluid_from_problem(prob, rtol=1e-14, convection=convection)
    mesh = ref.MeshBuffers.from_problem(prob)
    rng = np.random.default_rng(12)
    u0 = wall_faces_zero(0.05 * rng.standard_normal((3, n, n, n)))
    X0 = prob.X0

    def fwd(u, X):
        uu, _, XX, _ = ref.advance(fl, mesh, u, np.zeros((n, n, n)), X, 0.0, 1)
        return uu, XX
    u1, X1 = fwd(u0, X0)
    lam_u1 = rng.standard_normal(u1.shape)
    lam_X1 = rng.standard_normal(X1.shape)
    lu0, lX0, _ = ref.adjoint_step(fl, mesh, u0, X0, u1, 0.0, lam_u1, lam_X1)
    du = rng.standard_normal(u0.shape)
    dX = rng.standard_normal(X0.shape)
    for (a, b, pred) in [(du, 0 * dX, np.sum(lu0 * du)), (0 * du, dX, np.sum(lX0 * dX))]:
        e = 1e-6
        up, Xp = fwd(u0 + e * a, X0 + e * b)
        um, Xm = fwd(u0 - e * a, X0 - e * b)
        fd = (np.sum((up - um) * lam_u1) + np.sum((Xp - Xm) * lam_X1)) / (2 * e)
        assert abs(pred - fd) <= 2e-6 * max(abs(fd), 1e-12), (pred, fd)


def test_wall_nodes_workload_reaches_the_walls():
    """The near-wall workload places half its nodes within 2h of a wall (so the
    stencils of the pins above cross the walls) and keeps every node inside
    the box, each tethered once."""
    prob = inputs.wall_nodes()
    h = prob.h
    X = prob.X0
    dist = np.minimum(X, 1.0 - X).min(axis=1)
    assert np.all((X > 0) & (X < 1))
    assert np.sum(dist < 2 * h) >= len(X) // 2
    node, target, K = prob.tethers
    assert sorted(node.tolist()) == list(range(len(X)))
    assert np.all(K[:, :3] > 0) and np.all(K[:, 3:] == 0)
