"""Pins of the oracle's tetrahedral elements (P1: 4 nodes, one-point rule; P2:
10 nodes, the symmetric 4-point rule of degree 2).

Independent checks: for one straight-sided tet under an affine deformation
(constant stress P) the nodal forces are -P times the integral of grad N_a,
which the divergence theorem turns into face-area vectors computed here by
cross products: P1 vertex a gets P (A n)_opposite / 3; P2 vertices get
nothing and edge node (i, j) gets -P [(A n) of the two faces holding the
edge] / 3.  Then: the patch test (affine deformation of a whole mesh leaves
interior nodes force-free), the energy of a uniform dilation equal to
volume x Psi, force and torque balance for any x, forces as minus the energy
gradient, and Hessian products by differences."""
import numpy as np
import pytest

from paper_2503_22695_amd import inputs

NH, SR = inputs.NEO_HOOKEAN, inputs.STANDARD_REINFORCING
NH_PAR = (10.0, 100.0)


def mesh_of(ref, X, conn, model=NH, par=NH_PAR, ef=(1.0, 0.0, 0.0)):
    ne = conn.shape[0]
    return ref.MeshBuffers(X, conn, np.tile(ef, (ne, 1)), np.zeros(ne), [model], [par])


def one_tet(order, rng):
    V = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.1], [0.1, 0.2, 1.1]]) * 0.3
    V = V + 0.02 * rng.standard_normal((4, 3))
    conn = np.arange(4)[None, :]
    if order == 2:
        mids = np.array([0.5 * (V[i] + V[j]) for i, j in inputs.TET_EDGES])
        V = np.concatenate([V, mids])
        conn = np.arange(10)[None, :]
    return V, conn.astype(np.int32)


def face_area_vectors(V):
    """(A n) of the face opposite each vertex, n pointing out of the tet."""
    out = []
    for a in range(4):
        i, j, k = [b for b in range(4) if b != a]
        An = 0.5 * np.cross(V[j] - V[i], V[k] - V[i])
        if np.dot(An, V[a] - V[i]) > 0:
            An = -An
        out.append(An)
    return np.array(out)


@pytest.mark.parametrize("order", [1, 2])
def test_single_tet_affine_forces_closed_form(ref, order):
    rng = np.random.default_rng(order)
    Xr, conn = one_tet(order, rng)
    A = np.eye(3) + 0.1 * rng.standard_normal((3, 3))
    x = Xr @ A.T + np.array([0.3, -0.1, 0.2])
    mesh = mesh_of(ref, Xr, conn)
    F, E, _ = ref.fe_force(mesh, x)
    P, psi = ref.pk1(NH, NH_PAR, A)
    S = face_area_vectors(Xr[:4])
    vol = abs(np.dot(Xr[1] - Xr[0], np.cross(Xr[2] - Xr[0], Xr[3] - Xr[0]))) / 6
    scale = np.max(np.abs(P)) * np.max(np.linalg.norm(S, axis=1))
    assert abs(E - psi * vol) <= 1e-13 * abs(psi * vol)
    if order == 1:
        want = np.array([P @ S[a] / 3.0 for a in range(4)])
        assert np.max(np.abs(F - want)) <= 1e-13 * scale
    else:
        assert np.max(np.abs(F[:4])) <= 1e-13 * scale
        for t, (i, j) in enumerate(inputs.TET_EDGES):
            k, l = [b for b in range(4) if b not in (i, j)]
            want = -P @ (S[k] + S[l]) / 3.0
            assert np.max(np.abs(F[4 + t] - want)) <= 1e-13 * scale, (i, j)


@pytest.mark.parametrize("order", [1, 2])
def test_patch_test_and_dilation_energy(ref, order):
    X, conn = inputs.tet_block_mesh(3, 0.3, order)
    mesh = mesh_of(ref, X, conn)
    rng = np.random.default_rng(10 + order)
    A = np.eye(3) + 0.08 * rng.standard_normal((3, 3))
    F, _, _ = ref.fe_force(mesh, X @ A.T)
    lo, hi = X.min(0), X.max(0)
    interior = np.all((X > lo + 1e-9) & (X < hi - 1e-9), axis=1)
    assert interior.sum() > 0
    assert np.max(np.abs(F[interior])) <= 1e-12 * np.max(np.abs(F))
    s = 1.07
    _, E, _ = ref.fe_force(mesh, 0.5 + (X - 0.5) * s)
    want = 0.3 ** 3 * 0.5 * NH_PAR[1] * (3 * np.log(s)) ** 2
    assert abs(E - want) <= 1e-12 * want


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("model,par", [(NH, NH_PAR), (SR, inputs.LAW_PARAMS[SR])])
def test_tet_forces_balanced_gradient_and_hessian(ref, order, model, par):
    X, conn = inputs.tet_block_mesh(2, 0.3, order)
    rng = np.random.default_rng(20 + order)
    mesh = mesh_of(ref, X, conn, model, par, ef=np.ones(3) / np.sqrt(3))
    x = X * np.array([1.06, 0.97, 0.99]) + 0.004 * rng.standard_normal(X.shape)
    F, E, _ = ref.fe_force(mesh, x)
    scale = np.max(np.abs(F))
    assert np.max(np.abs(F.sum(0))) <= 1e-12 * scale * len(x)
    assert np.max(np.abs(np.cross(x, F).sum(0))) <= 1e-12 * scale * len(x)
    eps = 1e-7
    for q in range(0, len(x), max(1, len(x) // 12)):
        for r in range(3):
            xp, xm = x.copy(), x.copy()
            xp[q, r] += eps
            xm[q, r] -= eps
            fd = -(ref.fe_force(mesh, xp)[1] - ref.fe_force(mesh, xm)[1]) / (2 * eps)
            assert abs(F[q, r] - fd) <= 1e-6 * scale, (q, r)
    V = rng.standard_normal(x.shape)
    H = ref.fe_hvp(mesh, x, V)
    e = 1e-6
    fd = (ref.fe_force(mesh, x + e * V)[0] - ref.fe_force(mesh, x - e * V)[0]) / (2 * e)
    assert np.max(np.abs(H - fd)) <= 1e-6 * np.max(np.abs(H))
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q = -Q
    F0, _, _ = ref.fe_force(mesh, X @ Q.T + 0.1)
    if model == NH:   # rigid motion: no force
        assert np.max(np.abs(F0)) <= 1e-12 * scale
