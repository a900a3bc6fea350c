"""Pins of the oracle's geometric multigrid solver (the paper's abstract names a
geometric multigrid for the fluid solves; the V-cycle itself is this
implementation's reading).  Checked against closed-form eigen-solutions and an
independent FFT diagonalisation of the periodic 7-point operator."""
import math

import numpy as np
import pytest

from tests.test_oracle_grid import centre_coords


def fft_solve(b, sigma, nu):
    """Solve (sigma - nu Lap_h) x = b on the periodic grid with numpy.fft, using
    the textbook symbol of the 7-point Laplacian."""
    n = b.shape[-1]
    h = 1.0 / n
    k = np.fft.fftfreq(n) * n
    s = (4.0 / h ** 2) * np.sin(np.pi * k / n) ** 2
    lam = s[None, None, :] + s[None, :, None] + s[:, None, None]     # -symbol >= 0
    den = sigma + nu * lam
    bh = np.fft.fftn(b)
    with np.errstate(divide="ignore", invalid="ignore"):
        xh = np.where(den == 0, 0.0, bh / den)
    return np.real(np.fft.ifftn(xh))


@pytest.mark.parametrize("n", [16, 24, 32])
def test_poisson_manufactured_eigenmode(ref, n):
    fl = ref.fluid(n, rtol=1e-12)
    X, Y, Z = centre_coords(n)
    mode = np.sin(2 * math.pi * X) * np.sin(2 * math.pi * Y) * np.sin(2 * math.pi * Z)
    h = 1.0 / n
    lam = -3 * (4 / h ** 2) * math.sin(math.pi * h) ** 2
    x, cyc, rr = ref.mg_solve(fl, 0.0, 1.0, True, -lam * mode)
    assert rr <= 1e-12 and cyc <= 25
    assert np.max(np.abs(x - mode)) < 1e-10


def test_helmholtz_single_mode_factor(ref):
    n = 32
    fl = ref.fluid(n, rtol=1e-13)
    X, Y, Z = centre_coords(n)
    mode = np.cos(2 * math.pi * (X + 2 * Y)) * np.sin(2 * math.pi * Z)
    h = 1.0 / n
    lam = -(4 / h ** 2) * (math.sin(math.pi * h) ** 2 + math.sin(2 * math.pi * h) ** 2
                           + math.sin(math.pi * h) ** 2)
    sigma, nu = 1000.0, 0.01
    x, cyc, rr = ref.mg_solve(fl, sigma, nu, False, mode)
    assert np.max(np.abs(x - mode / (sigma - nu * lam))) < 1e-15 * 1e3


@pytest.mark.parametrize("n,sigma,nu,poisson,krylov", [
    (32, 0.0, 1.0, True, 1), (32, 0.0, 1.0, True, 0), (24, 0.0, 1.0, True, 1),
    (24, 0.0, 1.0, True, 0), (32, 2000.0, 0.01, False, 1), (16, 5.0, 1.0, False, 0)])
def test_matches_fft_solution(ref, n, sigma, nu, poisson, krylov):
    rng = np.random.default_rng(n)
    b = rng.standard_normal((n, n, n))
    if poisson:
        b -= b.mean()
    fl = ref.fluid(n, rtol=1e-10, krylov=krylov)
    x, cyc, rr = ref.mg_solve(fl, sigma, nu, poisson, b)
    xf = fft_solve(b, sigma, nu)
    assert rr <= 1e-10
    assert np.max(np.abs(x - xf)) <= 1e-8 * np.max(np.abs(xf))
    if poisson:
        assert abs(x.mean()) < 1e-14 * np.abs(x).max()


def test_vcycle_contraction(ref):
    """Residual reduction per V(2,2) cycle on a rough right-hand side (64^3:
    one level above the exactly solved 32^3)."""
    n = 64
    rng = np.random.default_rng(0)
    b = rng.standard_normal((n, n, n))
    b -= b.mean()
    rr = []
    for k in (1, 2, 3, 4):
        fl = ref.fluid(n, fixed_cycles=k, krylov=0)
        _, cyc, r = ref.mg_solve(fl, 0.0, 1.0, True, b)
        assert cyc == k
        rr.append(r)
    rates = [rr[i + 1] / rr[i] for i in range(3)]
    assert max(rates) < 0.25, rates   # asymptotic rate of this cycle is about 0.21


def test_zero_rhs_and_error_paths(ref):
    import oracle
    n = 16
    fl = ref.fluid(n)
    x, cyc, rr = ref.mg_solve(fl, 0.0, 1.0, True, np.zeros((n, n, n)), np.ones((n, n, n)))
    assert cyc == 0 and np.all(x == 0)
    m = 64   # (a 32^3 grid is its own coarsest level, solved exactly in one cycle)
    b = np.random.default_rng(1).standard_normal((m, m, m))
    b -= b.mean()
    with pytest.raises(oracle.OracleError) as e:
        ref.mg_solve(ref.fluid(m, max_cycles=1), 0.0, 1.0, True, b)
    assert e.value.rc == oracle.E_NOCONV
    b = np.random.default_rng(1).standard_normal((n, n, n))
    b -= b.mean()
    b[3, 2, 1] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        ref.mg_solve(fl, 0.0, 1.0, True, b)
    assert e.value.rc == oracle.E_NUMERIC
    with pytest.raises(oracle.OracleError) as e:
        ref.mg_solve(ref.fluid(20), 0.0, 1.0, True, np.ones((20, 20, 20)))
    assert e.value.rc == oracle.E_INVAL   # 20 -> 10 -> 5: odd level breaks red-black


def test_initial_guess_at_solution_needs_no_cycle(ref):
    n = 16
    rng = np.random.default_rng(3)
    b = rng.standard_normal((n, n, n))
    xs = fft_solve(b, 50.0, 1.0)
    x, cyc, rr = ref.mg_solve(ref.fluid(n), 50.0, 1.0, False, b, xs)
    assert cyc == 0 and np.array_equal(x, xs)


def neg_lap(x):
    """-Lap_h on the periodic grid (h = 1/n), written with numpy shifts."""
    n = x.shape[0]
    s = sum(np.roll(x, sh, ax) for ax in range(3) for sh in (1, -1))
    return -(s - 6.0 * x) * n * n


def test_krylov_first_step_is_energy_optimal_multiple_of_the_vcycle(ref):
    """One preconditioned-CG iteration from x = 0 is alpha z with z one V-cycle
    applied to b and alpha = (b.z)/(z.Az), the energy-minimising step (on 64^3:
    a 32^3 grid is its own coarsest level, solved exactly, so alpha would be 1)."""
    n = 64
    rng = np.random.default_rng(3)
    b = rng.standard_normal((n, n, n))
    b -= b.mean()
    z, cyc, _ = ref.mg_solve(ref.fluid(n, fixed_cycles=1, krylov=0), 0.0, 1.0, True, b)
    x1, cyc1, _ = ref.mg_solve(ref.fluid(n, fixed_cycles=1, krylov=1), 0.0, 1.0, True, b)
    assert cyc == 1 and cyc1 == 1
    alpha = np.sum(b * z) / np.sum(z * neg_lap(z))
    want = alpha * z
    want -= want.mean()
    assert np.max(np.abs(x1 - want)) <= 1e-12 * np.max(np.abs(want))
    assert abs(alpha - 1.0) > 1e-3      # the step is not the plain V-cycle's


def test_krylov_needs_fewer_cycles_than_the_plain_iteration(ref):
    n = 64
    rng = np.random.default_rng(5)
    b = rng.standard_normal((n, n, n))
    b -= b.mean()
    _, k_plain, _ = ref.mg_solve(ref.fluid(n, krylov=0), 0.0, 1.0, True, b)
    x, k_cg, rr = ref.mg_solve(ref.fluid(n, krylov=1), 0.0, 1.0, True, b)
    assert rr <= 1e-10
    assert k_cg <= 0.7 * k_plain, (k_cg, k_plain)


def young_omega(n, sigma, nu):
    c = nu * n * n
    rho = 6 * c / (sigma + 6 * c)
    return rho, 2.0 / (1.0 + math.sqrt(1.0 - rho * rho))


def test_helmholtz_relaxation_rate_is_youngs():
    """Where the Helmholtz operator's Jacobi radius rho = 6c / (sigma + 6c) is at
    most 1/2, its cycle is the red-black relaxation over-relaxed by Young's
    omega, which contracts the error by omega - 1 per sweep (up to a factor
    linear in the sweep count: the optimal SOR matrix is defective).  A cycle
    here is V(2,2) without coarse levels: four sweeps.  The ratio of 128^3 at
    dt = 5e-4 (sigma / 6c = 2.03) on a 64^3 grid (above the exactly solved
    32^3)."""
    import oracle
    n, nu = 64, 0.01
    sigma = 2000.0 / 983.04 * 6 * nu * n * n
    rho, w = young_omega(n, sigma, nu)
    assert rho <= 0.5
    rng = np.random.default_rng(7)
    b = rng.standard_normal((n, n, n))
    for k in (1, 2):
        _, cyc, r = oracle.mg_solve(oracle.fluid(n, fixed_cycles=k, krylov=0), sigma, nu, False, b)
        assert cyc == k
        sweeps = 4 * k
        assert r <= 2.0 * sweeps * (w - 1.0) ** sweeps, (k, r, (w - 1.0) ** sweeps)
    # plain Gauss-Seidel (omega = 1) could not do this: its rate is rho^2 per sweep
    assert 2.0 * 8 * (w - 1.0) ** 8 < (rho * rho) ** 8 * 1e-2


def test_helmholtz_relaxation_matches_numpy_sor():
    """One cycle at a level-0 stop equals red-black SOR written with numpy:
    four sweeps (V(2,2): pre + post), each red then black, each colour
    x += omega ((b + c * neighbour sum) / diag - x)."""
    import oracle
    n, nu, sigma = 64, 0.01, 400.0
    rho, w = young_omega(n, sigma, nu)
    assert rho <= 0.5
    rng = np.random.default_rng(8)
    b = rng.standard_normal((n, n, n))
    x0 = rng.standard_normal((n, n, n))
    x, cyc, _ = oracle.mg_solve(oracle.fluid(n, fixed_cycles=1, krylov=0), sigma, nu, False, b, x0)
    assert cyc == 1
    c = nu * n * n
    diag = sigma + 6 * c
    I, J, K = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    red = (I + J + K) % 2 == 0
    y = x0.copy()
    for mask in (red, ~red) * 4:
        s = sum(np.roll(y, sh, ax) for ax in range(3) for sh in (1, -1))
        g = (b + c * s) / diag
        y[mask] = y[mask] + w * (g[mask] - y[mask])
    assert np.max(np.abs(x - y)) <= 1e-13 * np.max(np.abs(y))


def test_coarsest_level_is_solved_exactly():
    """With mg_coarse_sweeps = 0 a grid of at most 32 cells per side is its own
    coarsest level, solved by its Fourier diagonalisation: one cycle reaches the
    FFT solution (numpy.fft) to rounding, for Poisson (mean-free) and
    Helmholtz, at 32^3, 24^3, 16^3, 12^3 and 8^3; with coarse sweeps the old
    hierarchy (down to 4^3 or 6^3) is kept."""
    import oracle
    for n in (32, 24, 16, 12, 8):
        rng = np.random.default_rng(40 + n)
        b = rng.standard_normal((n, n, n))
        for sigma, nu, poisson in ((0.0, 1.0, True), (3.0, 0.7, False)):
            bb = b - b.mean() if poisson else b
            fl = oracle.fluid(n, fixed_cycles=1, krylov=0)
            x, cyc, rr = oracle.mg_solve(fl, sigma, nu, poisson, bb)
            xf = fft_solve(bb, sigma, nu)
            assert cyc == 1 and rr <= 1e-13, (n, sigma, rr)
            assert np.max(np.abs(x - xf)) <= 1e-13 * np.max(np.abs(xf)), (n, sigma)
    # the sweep-based coarsest level needs several cycles on 16^3
    b = np.random.default_rng(7).standard_normal((16, 16, 16))
    b -= b.mean()
    _, cyc, _ = oracle.mg_solve(oracle.fluid(16, coarse_sweeps=16, krylov=0), 0.0, 1.0, True, b)
    assert cyc > 3
