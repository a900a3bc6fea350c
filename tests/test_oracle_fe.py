"""Pins of the oracle's constitutive laws and matrix-free nodal forces.

Laws: section "Constitutive laws" (volumetric U(J) = (kappa/2)(ln J)^2, modified
invariant I1bar = J^{-2/3} I1, Holzapfel-Ogden Psi_4) and the neo-Hookean law
of the mitral-valve chordae.  Nodal force: F_i = -sum_q P : grad N_i w_q
("Eulerian-Lagrangian coupling operators").
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2503_22695_amd import inputs

NH, HO = inputs.NEO_HOOKEAN, inputs.HOLZAPFEL_OGDEN
NH_PAR = (10.0, 100.0)
HO_PAR = (0.5, 5.0, 1.5, 8.0, 7.0)
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def rand_F(rng, scale=0.15):
    while True:
        Fm = np.eye(3) + scale * rng.standard_normal((3, 3))
        if np.linalg.det(Fm) > 0.3:
            return Fm


def rot(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


@pytest.mark.parametrize("model,par", [(NH, NH_PAR), (HO, HO_PAR)])
def test_stress_free_reference(ref, model, par):
    P, psi = ref.pk1(model, par, np.eye(3), (0.6, 0.8, 0.0))
    assert np.max(np.abs(P)) < 1e-14 and abs(psi) < 1e-15


@pytest.mark.parametrize("model,par", [(NH, NH_PAR), (HO, HO_PAR)])
def test_pk1_is_energy_derivative(ref, model, par):
    rng = np.random.default_rng(11 + model)
    ef = np.array([0.48, 0.6, 0.64])
    ef /= np.linalg.norm(ef)
    for _ in range(6):
        Fm = rand_F(rng)
        if model == HO:   # make sure the fibre is stretched so the fibre term is active
            Fm = Fm + 0.2 * np.outer(Fm @ ef, ef)
        P, _ = ref.pk1(model, par, Fm, ef)
        eps = 1e-6
        Pfd = np.empty((3, 3))
        for r in range(3):
            for c in range(3):
                Fp, Fmn = Fm.copy(), Fm.copy()
                Fp[r, c] += eps
                Fmn[r, c] -= eps
                Pfd[r, c] = (ref.pk1(model, par, Fp, ef)[1] - ref.pk1(model, par, Fmn, ef)[1]) / (2 * eps)
        assert np.max(np.abs(P - Pfd)) < 1e-7 * max(1.0, np.max(np.abs(P)))


@pytest.mark.parametrize("model,par", [(NH, NH_PAR), (HO, HO_PAR)])
def test_objectivity(ref, model, par):
    rng = np.random.default_rng(21)
    ef = np.array([1.0, 0.0, 0.0])
    for _ in range(5):
        Fm, Q = rand_F(rng), rot(rng)
        P, psi = ref.pk1(model, par, Fm, ef)
        P2, psi2 = ref.pk1(model, par, Q @ Fm, ef)
        assert np.max(np.abs(P2 - Q @ P)) < 1e-12 * max(1, np.abs(P).max())
        assert abs(psi2 - psi) < 1e-12 * max(1, abs(psi))


def test_uniaxial_closed_forms(ref):
    g = GOLDEN["uniaxial_isochoric"]
    lam, mu = g["lambda"], g["mu_s"]
    Fm = np.diag([lam, lam ** -0.5, lam ** -0.5])
    P, _ = ref.pk1(NH, (mu, 100.0), Fm)
    assert abs(P[0, 0] - g["nh_P11"]) < 1e-13
    assert abs(P[1, 1] - g["nh_P22"]) < 1e-13
    assert abs(P[0, 0] - 2 * mu / 3 * (lam - lam ** -2)) < 1e-13
    # Holzapfel-Ogden with the fibre along the stretch: closed form of P11
    a, b, af, bf, kap = HO_PAR
    I1b = lam ** 2 + 2 / lam
    P11 = a * math.exp(b * (I1b - 3)) * 2 / 3 * (lam - lam ** -2) \
        + 2 * af * (lam ** 2 - 1) * math.exp(bf * (lam ** 2 - 1) ** 2) * lam
    P, _ = ref.pk1(HO, HO_PAR, Fm, (1.0, 0.0, 0.0))
    assert abs(P[0, 0] - P11) < 1e-12 * abs(P11)
    assert abs(P[0, 0] - g["ho_P11"]) < 1e-12 * abs(P11)
    # compressed fibre: the fibre term is inactive (I4f* = 1)
    Fc = np.diag([1 / lam, lam ** 0.5, lam ** 0.5])
    P_ho, _ = ref.pk1(HO, (a, b, af, bf, kap), Fc, (1.0, 0.0, 0.0))
    P_iso, _ = ref.pk1(HO, (a, b, 0.0, bf, kap), Fc, (1.0, 0.0, 0.0))
    assert np.max(np.abs(P_ho - P_iso)) == 0.0


def test_volumetric_closed_form(ref):
    """Pure dilation F = s I: the isochoric parts vanish, P = kappa ln(J) / s I."""
    s = 1.07
    for model, par in [(NH, NH_PAR), (HO, (0.5, 5.0, 0.0, 8.0, 7.0))]:
        P, psi = ref.pk1(model, par, s * np.eye(3), (1.0, 0.0, 0.0))
        kap = par[-1] if model == HO else par[1]
        lnJ = 3 * math.log(s)
        assert np.max(np.abs(P - kap * lnJ / s * np.eye(3))) < 1e-12 * kap
        assert abs(psi - 0.5 * kap * lnJ ** 2) < 1e-12 * kap


def test_ho_small_b_limit_is_neo_hookean(ref):
    """a/(2b)(exp(b x) - 1) -> (a/2) x as b -> 0: HO without fibres -> NH, mu_s = a."""
    rng = np.random.default_rng(4)
    Fm = rand_F(rng)
    P_ho, _ = ref.pk1(HO, (0.5, 1e-9, 0.0, 8.0, 7.0), Fm)
    P_nh, _ = ref.pk1(NH, (0.5, 7.0), Fm)
    assert np.max(np.abs(P_ho - P_nh)) < 1e-8


def test_fibre_sign_irrelevant(ref):
    rng = np.random.default_rng(8)
    ef = np.array([0.6, 0.0, 0.8])
    Fm = rand_F(rng) + 0.3 * np.outer(ef, ef)
    P1, _ = ref.pk1(HO, HO_PAR, Fm, ef)
    P2, _ = ref.pk1(HO, HO_PAR, Fm, -ef)
    assert np.max(np.abs(P1 - P2)) == 0.0


def test_inverted_element_is_an_error(ref):
    import oracle
    with pytest.raises(oracle.OracleError) as e:
        ref.pk1(NH, NH_PAR, np.diag([1.0, 1.0, -1.0]))
    assert e.value.rc == oracle.E_NUMERIC


# --------------------------------------------------------------------------
# nodal forces on meshes
# --------------------------------------------------------------------------

def block(model, par, n_el=3, jitter=0.0, seed=0):
    import oracle
    X, conn = inputs.block_mesh(n_el, 0.3)
    if jitter:
        rng = np.random.default_rng(seed)
        X = X + rng.uniform(-jitter, jitter, X.shape)
    ne = conn.shape[0]
    fib = np.tile([0.8, 0.6, 0.0], (ne, 1))
    mesh = oracle.MeshBuffers(X, conn, fib, np.zeros(ne), [model], [list(par) + [0] * (5 - len(par))])
    return mesh, X


@pytest.mark.parametrize("model,par", [(NH, NH_PAR), (HO, HO_PAR)])
def test_zero_force_at_reference_and_rigid_motion(ref, model, par):
    mesh, X = block(model, par, jitter=0.004)
    F, E, Jmin = ref.fe_force(mesh, X)
    assert np.max(np.abs(F)) < 1e-12 and abs(E) < 1e-14 and abs(Jmin - 1) < 1e-12
    Q = rot(np.random.default_rng(3))
    x = (X - 0.5) @ Q.T + np.array([0.1, -0.3, 2.0])
    F, E, _ = ref.fe_force(mesh, x)
    assert np.max(np.abs(F)) < 1e-11 and abs(E) < 1e-12


@pytest.mark.parametrize("model,par", [(NH, NH_PAR), (HO, HO_PAR)])
def test_force_balance_for_any_deformation(ref, model, par):
    """Translation and rotation invariance of the energy give sum F = 0 and
    sum x x F = 0 for any configuration."""
    mesh, X = block(model, par)
    rng = np.random.default_rng(12)
    x = X * np.array([1.1, 0.95, 1.0]) + 0.01 * rng.standard_normal(X.shape)
    F, _, _ = ref.fe_force(mesh, x)
    scale = np.abs(F).max()
    assert np.max(np.abs(F.sum(0))) < 1e-12 * scale * len(F)
    assert np.max(np.abs(np.cross(x, F).sum(0))) < 1e-12 * scale * len(F)


@pytest.mark.parametrize("model,par", [(NH, NH_PAR), (HO, HO_PAR)])
def test_force_is_minus_energy_gradient(ref, model, par):
    mesh, X = block(model, par, n_el=2, jitter=0.003, seed=2)
    rng = np.random.default_rng(13)
    x = X * np.array([1.08, 0.97, 1.0]) + 0.005 * rng.standard_normal(X.shape)
    F, _, _ = ref.fe_force(mesh, x)
    eps = 1e-7
    for q in rng.choice(len(X), 6, replace=False):
        for r in range(3):
            xp, xm = x.copy(), x.copy()
            xp[q, r] += eps
            xm[q, r] -= eps
            dE = (ref.fe_force(mesh, xp)[1] - ref.fe_force(mesh, xm)[1]) / (2 * eps)
            assert abs(F[q, r] + dE) < 1e-6 * max(1.0, np.abs(F).max()), (q, r)


def test_patch_test_and_affine_energy(ref):
    """Affine motion x = A X + c: constant F in every element, so interior nodal
    forces vanish and the energy is Psi(A) times the block volume 0.3^3."""
    mesh, X = block(HO, HO_PAR, n_el=4, jitter=0.005, seed=5)
    A = np.array([[1.1, 0.05, 0.0], [0.02, 0.96, 0.01], [0.0, -0.03, 1.02]])
    x = X @ A.T + 0.2
    F, E, _ = ref.fe_force(mesh, x)
    m = 5
    ii = np.arange(m ** 3)
    i, j, k = ii % m, (ii // m) % m, ii // (m * m)
    interior = (i > 0) & (i < m - 1) & (j > 0) & (j < m - 1) & (k > 0) & (k < m - 1)
    assert np.max(np.abs(F[interior])) < 1e-12 * np.abs(F).max()
    # energy: jittered reference nodes change the volume, so use the unjittered block
    mesh0, X0 = block(HO, HO_PAR, n_el=4)
    F0, E0, _ = ref.fe_force(mesh0, X0 @ A.T)
    _, psi = ref.pk1(HO, HO_PAR, A, (0.8, 0.6, 0.0))
    assert abs(E0 - psi * 0.3 ** 3) < 1e-13


def test_shell_mesh_reference_is_valid_and_stress_free(ref):
    import oracle
    prob = inputs.ho_shell(n=32, n_theta=48, n_psi=16, n_tau=2)
    mesh = oracle.MeshBuffers.from_problem(prob)
    F, E, Jmin = ref.fe_force(mesh, prob.X_ref)      # raises if any det J0 <= 0
    assert np.max(np.abs(F)) < 1e-12 and abs(Jmin - 1.0) < 1e-12


# --------------------------------------------------------------------------
# pressure load
# --------------------------------------------------------------------------

def closed_box_surface(m=3, jitter=0.0, seed=0):
    """Quad surface of the unit cube [0,1]^3 split m x m per face, oriented with
    dx/dxi x dx/deta pointing INTO the box (the box plays the cavity)."""
    pts = {}
    quads = []

    def nid(p):
        key = tuple(np.round(np.asarray(p) * m).astype(int))
        if key not in pts:
            pts[key] = len(pts)
        return pts[key]
    t = np.linspace(0, 1, m + 1)
    for axis in range(3):
        for side in (0.0, 1.0):
            a1, a2 = [ax for ax in range(3) if ax != axis]
            for i in range(m):
                for j in range(m):
                    corner = []
                    for (di, dj) in ((0, 0), (1, 0), (0, 1), (1, 1)):
                        p = [0.0, 0.0, 0.0]
                        p[axis] = side
                        p[a1] = t[i + di]
                        p[a2] = t[j + dj]
                        corner.append(nid(p))
                    # normal of (a1, a2) ordering is +axis (right-handed) or -axis
                    e = np.zeros(3); e[a1] = 1
                    f = np.zeros(3); f[a2] = 1
                    nrm = np.cross(e, f)[axis]
                    inward = 1.0 if side == 0.0 else -1.0
                    if nrm * inward < 0:
                        corner = [corner[0], corner[2], corner[1], corner[3]]
                    quads.append(corner)
    X = np.zeros((len(pts), 3))
    for key, idx in pts.items():
        X[idx] = np.array(key) / m
    if jitter:
        X = X + np.random.default_rng(seed).uniform(-jitter, jitter, X.shape)
    return X, np.array(quads, dtype=np.int32)


def enclosed_volume(X, quads):
    """Volume enclosed by bilinear quads (normals pointing inward), via
    V = -(1/3) integral x . n da with a 5x5 Gauss-Legendre rule from numpy."""
    g, w = np.polynomial.legendre.leggauss(5)
    V = 0.0
    for q in quads:
        P = X[q]
        for s, ws in zip(g, w):
            for t, wt in zip(g, w):
                N = np.array([(1 - s) * (1 - t), (1 + s) * (1 - t), (1 - s) * (1 + t), (1 + s) * (1 + t)]) / 4
                dNs = np.array([-(1 - t), (1 - t), -(1 + t), (1 + t)]) / 4
                dNt = np.array([-(1 - s), -(1 + s), (1 - s), (1 + s)]) / 4
                x = N @ P
                nA = np.cross(dNs @ P, dNt @ P)
                V -= ws * wt * np.dot(x, nA) / 3.0
    return V


def test_pressure_load_is_volume_gradient(ref):
    """For a closed surface the follower pressure load is p dV/dx (pressure
    pushes the walls so as to enlarge the cavity)."""
    X, quads = closed_box_surface(m=2, jitter=0.03, seed=1)
    p = 1.7
    F = ref.pressure_load(quads, X, p)
    assert np.max(np.abs(F.sum(0))) < 1e-13
    eps = 1e-6
    for q in range(0, len(X), 3):
        for r in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[q, r] += eps
            Xm[q, r] -= eps
            dV = (enclosed_volume(Xp, quads) - enclosed_volume(Xm, quads)) / (2 * eps)
            assert abs(F[q, r] - p * dV) < 1e-8, (q, r)
    assert abs(enclosed_volume(*closed_box_surface(m=2)) - 1.0) < 1e-13
    F2 = ref.pressure_load(quads, X, 2 * p)
    assert np.max(np.abs(F2 - 2 * F)) < 1e-14


def test_shell_endocardial_load_net_force(ref):
    """The endocardium is open at the base (radius 0.21) and the apex hole
    (radius 2h): the net load is p times the difference of the two regular
    polygon areas, along +x (towards the apex)."""
    g = GOLDEN["shell_net_pressure_force"]
    prob = inputs.ho_shell(n=128)
    F = ref.pressure_load(prob.faces, prob.X_ref, 1.0)
    tot = F.sum(0)
    assert abs(tot[0] - g["Fx_per_unit_p"]) < 1e-12
    assert abs(tot[1]) < 1e-13 and abs(tot[2]) < 1e-13
