"""Pins of the oracle's MAC-grid operators against identities and closed forms.

MAC layout (section "Discretization of the Navier-Stokes equations"): u^d on
faces at i*h along d and (.+1/2)h elsewhere; p at cell centres.
"""
import math

import numpy as np
import pytest


def face_coords(n, d):
    """Coordinates (x, y, z) arrays [k, j, i] of the face lattice of component d."""
    h = 1.0 / n
    idx = np.arange(n)
    c = [(idx + (0.0 if e == d else 0.5)) * h for e in range(3)]
    Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    return X, Y, Z


def centre_coords(n):
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    return X, Y, Z


def test_div_grad_is_laplacian(ref):
    rng = np.random.default_rng(1)
    p = rng.standard_normal((12, 12, 12))
    lhs = ref.divergence(ref.gradient(p))
    rhs = ref.laplacian(p)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(rhs))


def test_summation_by_parts(ref):
    rng = np.random.default_rng(2)
    n = 10
    u = rng.standard_normal((3, n, n, n))
    p = rng.standard_normal((n, n, n))
    a = np.sum(ref.divergence(u) * p)
    b = -np.sum(u * ref.gradient(p))
    assert abs(a - b) <= 1e-12 * np.sum(np.abs(ref.divergence(u) * p))


@pytest.mark.parametrize("k", [(1, 0, 0), (2, 3, 1), (0, 5, 7)])
def test_laplacian_fourier_symbol(ref, k):
    """Lap_h exp(i 2 pi k.x) = -(4/h^2) sum_d sin^2(pi k_d h) exp(...)."""
    n = 16
    h = 1.0 / n
    X, Y, Z = centre_coords(n)
    ph = 2 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z)
    lam = -(4.0 / h ** 2) * sum(math.sin(math.pi * kd * h) ** 2 for kd in k)
    for q in (np.cos(ph), np.sin(ph)):
        out = ref.laplacian(q)
        assert np.max(np.abs(out - lam * q)) <= 1e-10 * max(1.0, abs(lam))


def taylor_green(n):
    X, Y, _ = face_coords(n, 0)
    ux = np.sin(2 * math.pi * X) * np.cos(2 * math.pi * Y)
    X, Y, _ = face_coords(n, 1)
    uy = -np.cos(2 * math.pi * X) * np.sin(2 * math.pi * Y)
    return np.stack([ux, uy, np.zeros_like(ux)])


def test_taylor_green_discretely_solenoidal(ref):
    for n in (8, 16, 32):
        u = taylor_green(n)
        assert np.max(np.abs(ref.divergence(u))) <= 1e-12 * n


def test_convection_conservative_and_constant(ref):
    rng = np.random.default_rng(3)
    n = 12
    u = rng.standard_normal((3, n, n, n))
    C = ref.convection(u)
    for d in range(3):
        assert abs(C[d].sum()) <= 1e-11 * np.abs(C[d]).sum()
    const = np.ones((3, n, n, n)) * np.array([0.3, -1.2, 2.0])[:, None, None, None]
    assert np.max(np.abs(ref.convection(const))) <= 1e-12


def abc_flow(n, A=1.0, B=0.7, Cc=0.4):
    """Arnold-Beltrami-Childress field (curl u = 2 pi u), sampled on faces, and the
    closed form of div(u u) = grad(|u|^2 / 2) on the same faces."""
    k = 2 * math.pi

    def u_at(X, Y, Z):
        return (A * np.sin(k * Z) + Cc * np.cos(k * Y),
                B * np.sin(k * X) + A * np.cos(k * Z),
                Cc * np.sin(k * Y) + B * np.cos(k * X))

    def grad_half_sq(X, Y, Z):
        ux, uy, uz = u_at(X, Y, Z)
        gx = uy * B * k * np.cos(k * X) - uz * B * k * np.sin(k * X)
        gy = -ux * Cc * k * np.sin(k * Y) + uz * Cc * k * np.cos(k * Y)
        gz = ux * A * k * np.cos(k * Z) - uy * A * k * np.sin(k * Z)
        return gx, gy, gz
    u = np.empty((3, n, n, n))
    c = np.empty((3, n, n, n))
    for d in range(3):
        X, Y, Z = face_coords(n, d)
        u[d] = u_at(X, Y, Z)[d]
        c[d] = grad_half_sq(X, Y, Z)[d]
    return u, c


def test_convection_second_order_against_closed_form(ref):
    """A dropped/mis-indexed flux gives O(1) or O(h) error; the centred flux form
    converges at O(h^2) to the continuum div(u u)."""
    errs = []
    for n in (16, 32, 64):
        u, c = abc_flow(n)
        errs.append(np.max(np.abs(ref.convection(u) - c)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, errs
    assert errs[2] < 2e-2 * np.max(np.abs(c))
