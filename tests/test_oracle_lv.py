"""Pins of the oracle's full Holzapfel-Ogden law (sheet and fibre-sheet terms)
and of the left-ventricle active stress ("Constitutive laws"; the
left-ventricle model's active tension and its waveform), at the law, the
element and the rollout level.

What fixes each check independently of the oracle's own formulas:
  - P = dPsi/dF by central differences of the energy (the active stress has the
    potential W_a at frozen T_a, so the same check covers it);
  - balance of angular momentum: P F^T is symmetric for every frame-invariant
    law (the printed fibre-sheet stress, 2 a_fs I8 e^{..} (F e_f) (x) e_s,
    fails it; the derivative of the printed energy passes);
  - the reference state, objectivity, the fibre/sheet exchange symmetry and
    the sign of e_s;
  - the invariants of a simple shear in the fibre-sheet plane, whose energy
    has a closed form in gamma;
  - the activation waveform's values, symmetry and support;
  - element forces as minus the energy gradient, force and torque balance,
    the Hessian product against force differences, and a rollout gradient
    against central differences of the loss."""
import math

import numpy as np
import pytest

from paper_2503_22695_amd import inputs

HO = inputs.HOLZAPFEL_OGDEN
LV = inputs.LV_PARAMS


def frame(rng):
    f = rng.standard_normal(3)
    f /= np.linalg.norm(f)
    s = rng.standard_normal(3)
    s -= (s @ f) * f
    s /= np.linalg.norm(s)
    return f, s


def rand_F(rng, f, s, scale=0.15):
    # stretch along the fibre and the sheet so both I4 terms are active
    return np.eye(3) + scale * rng.standard_normal((3, 3)) + 0.2 * np.outer(f, f) + 0.15 * np.outer(s, s)


@pytest.mark.parametrize("Ta", [0.0, 2.5])
def test_full_ho_pk1_is_energy_derivative(ref, Ta):
    rng = np.random.default_rng(11)
    for trial in range(6):
        f, s = frame(rng)
        Fm = rand_F(rng, f, s, 0.1 if trial % 2 else 0.2)
        P, _ = ref.pk1(HO, LV, Fm, f, s, Ta)
        eps = 1e-6
        Pfd = np.zeros((3, 3))
        for r in range(3):
            for c in range(3):
                Fp, Fq = Fm.copy(), Fm.copy()
                Fp[r, c] += eps
                Fq[r, c] -= eps
                Pfd[r, c] = (ref.pk1(HO, LV, Fp, f, s, Ta)[1] - ref.pk1(HO, LV, Fq, f, s, Ta)[1]) / (2 * eps)
        assert np.max(np.abs(P - Pfd)) <= 1e-7 * max(1.0, np.max(np.abs(P))), trial


@pytest.mark.parametrize("Ta", [0.0, 2.5])
def test_full_ho_cauchy_stress_is_symmetric(ref, Ta):
    rng = np.random.default_rng(12)
    for _ in range(8):
        f, s = frame(rng)
        Fm = rand_F(rng, f, s, 0.25)
        P, _ = ref.pk1(HO, LV, Fm, f, s, Ta)
        K = P @ Fm.T
        assert np.max(np.abs(K - K.T)) <= 1e-13 * np.max(np.abs(K))


def test_full_ho_reference_state_and_active_stress_at_rest(ref):
    rng = np.random.default_rng(13)
    f, s = frame(rng)
    P, psi = ref.pk1(HO, LV, np.eye(3), f, s, 0.0)
    assert np.max(np.abs(P)) <= 1e-15 and abs(psi) <= 1e-15
    # at rest I4f = 1, so T = T_a and P_a = T_a e_f (x) e_f
    P, psi = ref.pk1(HO, LV, np.eye(3), f, s, 3.0)
    assert np.max(np.abs(P - 3.0 * np.outer(f, f))) <= 1e-14 and abs(psi) <= 1e-15


def test_full_ho_objectivity(ref):
    rng = np.random.default_rng(14)
    for Ta in (0.0, 1.7):
        f, s = frame(rng)
        Fm = rand_F(rng, f, s)
        Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        P, psi = ref.pk1(HO, LV, Fm, f, s, Ta)
        P2, psi2 = ref.pk1(HO, LV, Q @ Fm, f, s, Ta)
        assert np.max(np.abs(P2 - Q @ P)) <= 1e-13 * np.max(np.abs(P))
        assert abs(psi2 - psi) <= 1e-13 * abs(psi)


def test_full_ho_fibre_sheet_exchange_and_sign(ref):
    """With equal fibre and sheet constants the law is symmetric in (e_f, e_s);
    flipping either direction changes nothing."""
    par = list(LV)
    par[5], par[6] = par[2], par[3]      # a_s = a_f, b_s = b_f
    rng = np.random.default_rng(15)
    f, s = frame(rng)
    Fm = rand_F(rng, f, s)
    P1, e1 = ref.pk1(HO, par, Fm, f, s)
    P2, e2 = ref.pk1(HO, par, Fm, s, f)
    assert np.max(np.abs(P1 - P2)) <= 1e-13 * np.max(np.abs(P1)) and abs(e1 - e2) <= 1e-13 * abs(e1)
    for ff, ss in ((-f, s), (f, -s), (-f, -s)):
        P3, e3 = ref.pk1(HO, LV, Fm, ff, ss, 1.3)
        P4, e4 = ref.pk1(HO, LV, Fm, f, s, 1.3)
        assert np.max(np.abs(P3 - P4)) <= 1e-14 * np.max(np.abs(P4)) and e3 == e4


def test_full_ho_simple_shear_energy(ref):
    """F = I + g e_f (x) e_s: J = 1, I1bar = 3 + g^2, I4f = 1 (fibre inactive),
    I4s = 1 + g^2, I8fs = g, so
    Psi = a/(2b)(e^{b g^2} - 1) + a_s/(2 b_s)(e^{b_s g^4} - 1) + a_fs/(2 b_fs)(e^{b_fs g^2} - 1)."""
    a, b, af, bf, kap, as_, bs, afs, bfs = LV
    rng = np.random.default_rng(16)
    f, s = frame(rng)
    for g in (0.05, 0.2, 0.4):
        Fm = np.eye(3) + g * np.outer(f, s)
        _, psi = ref.pk1(HO, LV, Fm, f, s)
        want = (a / (2 * b) * math.expm1(b * g * g) + as_ / (2 * bs) * math.expm1(bs * g ** 4)
                + afs / (2 * bfs) * math.expm1(bfs * g * g))
        assert abs(psi - want) <= 1e-13 * want, g


def test_active_stress_uniaxial_fibre_stretch(ref):
    """Along e_f = x with F = diag(lam, lam^-1/2, lam^-1/2): I4f = lam^2, so the
    active part of P is T_a (1 + 4.9 (lam - 1)) lam in entry (x, x) only."""
    f, s = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
    for lam in (0.9, 1.0, 1.15):
        Fm = np.diag([lam, lam ** -0.5, lam ** -0.5])
        P1, _ = ref.pk1(HO, LV, Fm, f, s, 2.0)
        P0, _ = ref.pk1(HO, LV, Fm, f, s, 0.0)
        want = np.zeros((3, 3))
        want[0, 0] = 2.0 * (1.0 + 4.9 * (lam - 1.0)) * lam
        assert np.max(np.abs(P1 - P0 - want)) <= 1e-14 * 10


def test_active_tension_waveform(ref):
    """Shape (0.5, 0.8) mapped onto [t_on, t_on + d]: zero outside, rises as
    1 - exp(-(s-0.5)^2/0.005), falls as 1 - exp(-(0.8-s)^2/0.005), continuous
    and symmetric about s = 0.65."""
    tm, t_on, d = 5.8, 0.01, 0.05

    def at(s):
        return ref.active_tension(tm, t_on, d, t_on + (s - 0.5) / 0.3 * d)
    for s in (0.0, 0.3, 0.5, 0.8, 0.81, 1.2):
        assert at(s) == 0.0, s
    assert abs(at(0.575) - tm * -math.expm1(-0.075 ** 2 / 0.005)) <= 1e-14 * tm
    assert abs(at(0.65) - tm * -math.expm1(-4.5)) <= 1e-14 * tm
    for ds in (0.01, 0.07, 0.149):
        assert abs(at(0.65 - ds) - at(0.65 + ds)) <= 1e-12 * tm, ds
    assert abs(at(0.65 - 1e-9) - at(0.65 + 1e-9)) <= 1e-9
    assert ref.active_tension(0.0, t_on, d, t_on + d / 2) == 0.0
    assert ref.active_tension(tm, t_on, 0.0, t_on) == 0.0


def lv_mesh(ref, Ta, n_el=2, seed=17):
    X, conn = inputs.block_mesh(n_el, 0.3)
    rng = np.random.default_rng(seed)
    ne = conn.shape[0]
    fr = [frame(rng) for _ in range(ne)]
    fib = np.array([a for a, _ in fr])
    sh = np.array([b for _, b in fr])
    mesh = ref.MeshBuffers(X, conn, fib, np.zeros(ne), [HO], [LV], sheet=sh, active_tension=Ta)
    x = X * np.array([1.1, 0.96, 0.98]) + 0.006 * rng.standard_normal(X.shape)
    return mesh, X, x


@pytest.mark.parametrize("Ta", [0.0, 2.0])
def test_lv_element_force_is_minus_energy_gradient_and_balanced(ref, Ta):
    mesh, X, x = lv_mesh(ref, Ta)
    F, E, _ = ref.fe_force(mesh, x)
    eps = 1e-6
    for q in range(0, len(x), 3):
        for r in range(3):
            xp, xm = x.copy(), x.copy()
            xp[q, r] += eps
            xm[q, r] -= eps
            fd = -(ref.fe_force(mesh, xp)[1] - ref.fe_force(mesh, xm)[1]) / (2 * eps)
            assert abs(F[q, r] - fd) <= 1e-7 * max(1.0, np.max(np.abs(F))), (q, r)
    scale = np.max(np.abs(F))
    assert np.max(np.abs(F.sum(0))) <= 1e-13 * scale * len(x)
    assert np.max(np.abs(np.cross(x, F).sum(0))) <= 1e-13 * scale * len(x)


def test_lv_sheet_terms_need_sheets(ref):
    X, conn = inputs.block_mesh(1, 0.3)
    fib = np.tile([1.0, 0.0, 0.0], (1, 1))
    mesh = ref.MeshBuffers(X, conn, fib, np.zeros(1), [HO], [LV])
    with pytest.raises(ref.OracleError):
        ref.fe_force(mesh, X)
    passive_f_only = list(LV[:5])
    mesh = ref.MeshBuffers(X, conn, fib, np.zeros(1), [HO], [passive_f_only], active_tension=1.0)
    ref.fe_force(mesh, X * 1.01)     # fibre, isotropic and active terms need no sheet


@pytest.mark.parametrize("Ta", [0.0, 2.0])
def test_lv_hvp_and_tangent_match_differences(ref, Ta):
    rng = np.random.default_rng(18)
    for _ in range(4):
        f, s = frame(rng)
        Fm = rand_F(rng, f, s)
        dF = rng.standard_normal((3, 3))
        dP = ref.pk1_tangent(HO, LV, Fm, dF, f, s, Ta)
        e = 1e-6
        fd = (ref.pk1(HO, LV, Fm + e * dF, f, s, Ta)[0] - ref.pk1(HO, LV, Fm - e * dF, f, s, Ta)[0]) / (2 * e)
        assert np.max(np.abs(dP - fd)) <= 1e-7 * max(1.0, np.max(np.abs(dP)))
    mesh, X, x = lv_mesh(ref, Ta)
    V1, V2 = rng.standard_normal(x.shape), rng.standard_normal(x.shape)
    H1 = ref.fe_hvp(mesh, x, V1)
    e = 1e-6
    fd = (ref.fe_force(mesh, x + e * V1)[0] - ref.fe_force(mesh, x - e * V1)[0]) / (2 * e)
    assert np.max(np.abs(H1 - fd)) <= 1e-6 * np.max(np.abs(H1))
    H2 = ref.fe_hvp(mesh, x, V2)
    assert abs(np.sum(V2 * H1) - np.sum(V1 * H2)) <= 1e-11 * np.sum(np.abs(V2 * H1))


def test_lv_rollout_gradient_against_central_difference(ref):
    """Full law, active pulse over the run, tethered face: gradient of
    L = sum |X^N - X_t|^2 over 3 steps with respect to (a, b, a_f, b_f) and X0.  The parameter
    sensitivities are ~1e-10 against L ~ 1e-4, so the multigrid's stopping noise
    in L dominates steps below ~1e-2 relative; the Taylor remainder at 1e-2 is
    ~1e-8 relative."""
    n, n_steps = 16, 3
    prob = inputs.lv_block(n=n, n_el=3, n_steps=n_steps)
    fl = ref.fluid_from_problem(prob, rtol=1e-14)
    rng = np.random.default_rng(19)
    u0 = ref.project(ref.fluid(n, rtol=1e-14), 0.05 * rng.standard_normal((3, n, n, n)))
    mesh = ref.MeshBuffers.from_problem(prob)
    Xt = prob.X0 + 0.01 * prob.h
    L, dX0, dth = ref.rollout_grad(fl, mesh, u0, prob.X0, 0.0, n_steps, 0.0, 1.0, Xt)

    def loss(par, X0):
        m = ref.MeshBuffers(prob.X_ref, prob.conn, prob.fibre, prob.mat_id, [HO], [par],
                            sheet=prob.sheet, active=(prob.ta_max, prob.ta_t_on, prob.ta_duration),
                            tethers=prob.tethers)
        _, _, XN, _ = ref.advance(fl, m, u0, np.zeros((n,) * 3), X0, 0.0, n_steps)
        return float(np.sum((XN - Xt) ** 2))
    assert abs(L - loss(list(LV), prob.X0)) <= 1e-14 * abs(L)
    for k in range(4):
        par = np.array(LV)
        e = 1e-2 * par[k]
        pp, pm = par.copy(), par.copy()
        pp[k] += e
        pm[k] -= e
        fd = (loss(pp, prob.X0) - loss(pm, prob.X0)) / (2 * e)
        assert abs(dth[0, k] - fd) <= 2e-6 * abs(fd), (k, dth[0, k], fd)
    for _ in range(2):
        d = rng.standard_normal(prob.X0.shape)
        g = np.sum(dX0 * d)
        e = 1e-6
        fd = (loss(list(LV), prob.X0 + e * d) - loss(list(LV), prob.X0 - e * d)) / (2 * e)
        assert abs(g - fd) <= 1e-7 * abs(g)


def test_lv_active_pulse_changes_the_run(ref):
    """The waveform enters the steps: with the pulse the block ends elsewhere than
    without it, and a pulse that starts after the run changes nothing."""
    n, n_steps = 16, 3
    prob = inputs.lv_block(n=n, n_el=3, n_steps=n_steps)
    fl = ref.fluid_from_problem(prob)
    z = np.zeros((n,) * 3)
    u = prob.initial_velocity()

    def run(active):
        m = ref.MeshBuffers(prob.X_ref, prob.conn, prob.fibre, prob.mat_id, [HO], [LV],
                            sheet=prob.sheet, active=active, tethers=prob.tethers)
        return ref.advance(fl, m, u, z, prob.X0, 0.0, n_steps)[2]
    X_on = run((prob.ta_max, 0.0, prob.ta_duration))
    X_off = run((0.0, 0.0, 0.0))
    X_late = run((prob.ta_max, 1.0, prob.ta_duration))
    assert np.max(np.abs(X_on - X_off)) > 1e-9
    assert np.array_equal(X_late, X_off)
