"""Pins of the oracle's penalty tethers (constrained solid faces and the
left-ventricle base constraint, enforced with a penalty parameter): each
tethered node feels the linear spring force -K (X - Y).

Independent checks: the force against numpy's product with the 3x3 matrix
assembled from the documented (xx, yy, zz, xy, xz, yz) layout, minus the
energy gradient by differences, zero force at the targets, the Hessian
product (exact for a linear force), and the base constraint's projector
(radial motion in the base plane is free, axial and circumferential motion
is restored with stiffness kappa)."""
import numpy as np

from paper_2503_22695_amd import inputs

HO = inputs.HOLZAPFEL_OGDEN


def K_matrix(k6):
    xx, yy, zz, xy, xz, yz = k6
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def tethered_block(ref, seed=0, n_el=2, with_elements=True):
    X, conn = inputs.block_mesh(n_el, 0.3)
    rng = np.random.default_rng(seed)
    node = rng.choice(len(X), size=7, replace=False).astype(np.int32)
    target = X[node] + 0.01 * rng.standard_normal((7, 3))
    A = rng.standard_normal((7, 3, 3))
    Km = np.einsum("tij,tkj->tik", A, A) + 0.5 * np.eye(3)       # symmetric positive definite
    K = np.stack([Km[:, 0, 0], Km[:, 1, 1], Km[:, 2, 2], Km[:, 0, 1], Km[:, 0, 2], Km[:, 1, 2]], 1)
    if not with_elements:
        conn = np.zeros((0, 8), dtype=np.int32)
    ne = conn.shape[0]
    fib = np.tile([1.0, 0.0, 0.0], (ne, 1))
    mesh = ref.MeshBuffers(X, conn, fib, np.zeros(ne), [HO], [inputs.HO_PARAMS],
                           tethers=(node, target, K))
    x = X + 0.02 * rng.standard_normal(X.shape)
    return mesh, X, x, node, target, K


def test_tether_force_is_the_spring_law(ref):
    mesh, X, x, node, target, K = tethered_block(ref, with_elements=False)
    F, E, _ = ref.fe_force(mesh, x)
    want = np.zeros_like(x)
    Ew = 0.0
    for t, a in enumerate(node):
        d = x[a] - target[t]
        want[a] = -K_matrix(K[t]) @ d
        Ew += 0.5 * d @ K_matrix(K[t]) @ d
    assert np.max(np.abs(F - want)) <= 1e-15 * np.max(np.abs(want)) * 10
    assert abs(E - Ew) <= 1e-14 * Ew
    # zero at the targets
    x0 = x.copy()
    x0[node] = target
    F0, E0, _ = ref.fe_force(mesh, x0)
    assert np.max(np.abs(F0)) == 0.0 and E0 == 0.0


def test_tethered_block_force_is_minus_energy_gradient(ref):
    mesh, X, x, node, target, K = tethered_block(ref, seed=1)
    F, E, _ = ref.fe_force(mesh, x)
    eps = 1e-6
    for a in list(node) + [0, len(x) - 1]:
        for r in range(3):
            xp, xm = x.copy(), x.copy()
            xp[a, r] += eps
            xm[a, r] -= eps
            fd = -(ref.fe_force(mesh, xp)[1] - ref.fe_force(mesh, xm)[1]) / (2 * eps)
            assert abs(F[a, r] - fd) <= 1e-7 * max(1.0, np.max(np.abs(F))), (a, r)


def test_tether_hessian_product(ref):
    mesh, X, x, node, target, K = tethered_block(ref, seed=2)
    rng = np.random.default_rng(3)
    V = rng.standard_normal(x.shape)
    H = ref.fe_hvp(mesh, x, V)
    e = 1e-6
    fd = (ref.fe_force(mesh, x + e * V)[0] - ref.fe_force(mesh, x - e * V)[0]) / (2 * e)
    assert np.max(np.abs(H - fd)) <= 1e-6 * np.max(np.abs(H))
    # the tether part alone is exactly -K V
    m0 = ref.MeshBuffers(mesh.X_ref, np.zeros((0, 8)), np.zeros((0, 3)), np.zeros(0), [HO],
                         [inputs.HO_PARAMS], tethers=(node, target, K))
    Ht = ref.fe_hvp(m0, x, V)
    for t, a in enumerate(node):
        assert np.max(np.abs(Ht[a] + K_matrix(K[t]) @ V[a])) <= 1e-14 * np.max(np.abs(Ht))


def test_base_constraint_leaves_radial_motion_free(ref):
    prob = inputs.lv_shell(n=64, n_theta=32, n_psi=8, n_tau=2)
    node, target, K = prob.tethers
    kap = inputs.LV_BASE_KAPPA
    m = ref.MeshBuffers(prob.X_ref, np.zeros((0, 8)), np.zeros((0, 3)), np.zeros(0), [HO],
                        [inputs.HO_PARAMS], tethers=prob.tethers)
    th = np.arctan2(target[:, 2] - 0.5, target[:, 1] - 0.5)
    radial = np.stack([0 * th, np.cos(th), np.sin(th)], 1)
    circ = np.stack([0 * th, -np.sin(th), np.cos(th)], 1)
    axial = np.tile([1.0, 0.0, 0.0], (len(th), 1))
    for direction, expect in ((radial, 0.0), (axial, 1.0), (circ, 1.0)):
        x = prob.X_ref.copy()
        x[node] += 0.003 * direction
        F, _, _ = ref.fe_force(m, x)
        want = -expect * kap * 0.003 * direction
        assert np.max(np.abs(F[node] - want)) <= 1e-15 + 1e-12 * kap * 0.003
