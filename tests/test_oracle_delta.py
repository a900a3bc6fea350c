"""Pins of the regularized delta and the spreading / interpolation operators.

delta_h is Peskin's four-point kernel (the paper cites Peskin's review for
delta_h); spreading and interpolation follow the section "Eulerian-Lagrangian
coupling operators", which also states that the two are discretely adjoint
when evaluated with the same quadrature.
"""
import math

import numpy as np
import pytest

from tests.test_oracle_grid import face_coords


def stencil_sums(ref, r):
    b = math.floor(r)
    m = np.arange(b - 1, b + 3)
    w = np.array([ref.phi(r - mm) for mm in m])
    return m, w


def test_phi_moment_conditions(ref):
    """The conditions that define the four-point kernel: partition of unity,
    even/odd split, zero first moment and sum of squares 3/8."""
    rng = np.random.default_rng(0)
    for r in rng.uniform(-50, 50, 2000):
        m, w = stencil_sums(ref, r)
        assert abs(w.sum() - 1.0) < 1e-15
        even = w[(m % 2) == 0].sum()
        assert abs(even - 0.5) < 1e-15
        assert abs(np.sum((r - m) * w)) < 1e-14
        assert abs(np.sum(w * w) - 3.0 / 8.0) < 1e-15
        # support: nothing outside b-1..b+2
        b = math.floor(r)
        assert ref.phi(r - (b - 2)) == 0.0 and ref.phi(r - (b + 3)) == 0.0


def test_phi_special_values(ref):
    assert ref.phi(0.0) == 0.5
    assert abs(ref.phi(1.0) - 0.25) < 1e-16 and abs(ref.phi(1.0 - 1e-13) - 0.25) < 1e-12
    assert ref.phi(2.0) == 0.0 and abs(ref.phi(2.0 - 1e-12)) < 1e-6
    assert ref.phi(-0.3) == ref.phi(0.3)


def face_positions(n, d):
    X, Y, Z = face_coords(n, d)
    return X, Y, Z


def test_spread_total_force_and_first_moment(ref):
    """sum_idx h^3 f^d = sum_q F^d_q ; sum_idx h^3 x_e f^d = sum_q X_qe F^d_q
    (nodes kept away from the periodic seam so x is unambiguous)."""
    n = 16
    h = 1.0 / n
    rng = np.random.default_rng(5)
    X = rng.uniform(0.3, 0.7, (40, 3))
    F = rng.standard_normal((40, 3))
    f = ref.spread(n, X, F)
    for d in range(3):
        assert abs(h ** 3 * f[d].sum() - F[:, d].sum()) < 1e-12
        coords = face_positions(n, d)
        for e in range(3):
            lhs = h ** 3 * np.sum(coords[e] * f[d])
            rhs = np.sum(X[:, e] * F[:, d])
            assert abs(lhs - rhs) < 1e-12, (d, e)


def test_spread_periodic_wrap_preserves_total(ref):
    n = 8
    h = 1.0 / n
    X = np.array([[0.01, 0.99, 0.5], [-0.2, 1.3, 2.05]])
    F = np.array([[1.0, 2.0, 3.0], [-0.5, 0.25, 4.0]])
    f = ref.spread(n, X, F)
    for d in range(3):
        assert abs(h ** 3 * f[d].sum() - F[:, d].sum()) < 1e-12


def test_interpolation_reproduces_constants_and_linears(ref):
    n = 16
    rng = np.random.default_rng(6)
    X = rng.uniform(0.35, 0.65, (30, 3))
    u = np.empty((3, n, n, n))
    const = np.array([0.7, -1.1, 2.5])
    for d in range(3):
        u[d] = const[d]
    U = ref.interpolate(X, u)
    assert np.max(np.abs(U - const)) < 1e-14
    # locally linear field (the stencil of nodes in [0.35, 0.65] never wraps)
    A = rng.standard_normal((3, 3))
    c0 = rng.standard_normal(3)
    for d in range(3):
        xs = face_positions(n, d)
        u[d] = c0[d] + A[d, 0] * xs[0] + A[d, 1] * xs[1] + A[d, 2] * xs[2]
    U = ref.interpolate(X, u)
    assert np.max(np.abs(U - (c0 + X @ A.T))) < 1e-13


@pytest.mark.parametrize("n", [8, 16])
def test_spread_interp_adjoint(ref, n):
    """<S F, u>_h = <F, J u> (the discrete adjointness the paper states)."""
    h = 1.0 / n
    rng = np.random.default_rng(7 + n)
    X = rng.uniform(-0.5, 1.5, (25, 3))      # unwrapped, crosses the seam
    F = rng.standard_normal((25, 3))
    u = rng.standard_normal((3, n, n, n))
    lhs = h ** 3 * np.sum(ref.spread(n, X, F) * u)
    rhs = np.sum(F * ref.interpolate(X, u))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1e-300) + 1e-13


def test_spread_matches_periodic_images(ref):
    """Shifting a node by a whole period leaves the spread field unchanged."""
    n = 8
    rng = np.random.default_rng(9)
    X = rng.uniform(0, 1, (6, 3))
    F = rng.standard_normal((6, 3))
    f1 = ref.spread(n, X, F)
    f2 = ref.spread(n, X + np.array([1.0, -2.0, 3.0]), F)
    assert np.max(np.abs(f1 - f2)) < 1e-10 * np.max(np.abs(f1))
