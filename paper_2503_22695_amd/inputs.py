"""Seeded synthetic inputs for the immersed-boundary timestep.

This module builds problem descriptions only: grid size and fluid constants,
hexahedral Lagrangian meshes, fibre fields, material records, endocardial
pressure faces and initial velocity fields.  It contains none of the method's
arithmetic (no delta kernel, no finite-element force, no solver), so both the
GPU library and the independent CPU oracle can take their inputs from here.

Geometry follows the paper's cardiac workloads in shape and size only (the
image-based left ventricle and valve meshes are not available):

* ``block``  -- a cube of trilinear hexes, stretched 1.1x in x and jittered;
* ``shell``  -- a truncated ellipsoidal shell (left-ventricle stand-in) with a
  transmural fibre rotation from -60 deg (epicardium) to +60 deg (endocardium)
  and an endocardial pressure surface;
* ``leaflets`` -- two one-element-thick half-annular sheets across the shell
  base (valve stand-in);
* ``lv`` -- the shell (or a block) with the full Holzapfel-Ogden law of the
  left-ventricle model (sheet and fibre-sheet terms, parameter ratios of its
  table), transmural sheet directions and an active-tension pulse.

Hex local node ``a = i + 2 j + 4 k`` sits at reference coordinates
``(xi, eta, zeta) = (2i-1, 2j-1, 2k-1)``; every element is oriented so its
reference Jacobian is positive.  Quad local node ``a = i + 2 j`` sits at
``(2i-1, 2j-1)``; every pressure quad is oriented so that
``dx/dxi x dx/deta`` points out of the solid, into the cavity.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# material model ids (shared convention of the C interfaces)
NEO_HOOKEAN = 0                # (mu_s, kappa)
HOLZAPFEL_OGDEN = 1            # (a, b, a_f, b_f, kappa[, a_s, b_s, a_fs, b_fs])
STANDARD_REINFORCING = 2       # Psi_1: (G_T, G_L, E_L, kappa)
FIBRE_REINFORCED_1 = 3         # Psi_2: (C_1, a_f, b_f, kappa)
FIBRE_REINFORCED_2 = 4         # Psi_3: (C_10, C_01, a_f, b_f, kappa)

MAT_PARAMS = 9   # parameter slots per material

HEX_CORNERS = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)],
                       dtype=np.int64)  # a = i + 2j + 4k


@dataclasses.dataclass
class Material:
    model: int
    params: Tuple[float, ...]  # NH: (mu_s, kappa); HO: (a, b, a_f, b_f, kappa[, a_s, b_s, a_fs, b_fs])

    def padded(self) -> List[float]:
        p = list(self.params) + [0.0] * (MAT_PARAMS - len(self.params))
        return p[:MAT_PARAMS]


@dataclasses.dataclass
class Problem:
    """One immersed-boundary workload: fluid box, solid mesh and run length."""
    name: str
    n: int
    rho: float
    mu: float
    dt: float
    n_steps: int
    X_ref: np.ndarray          # [n_nodes, 3] float64, reference configuration
    X0: np.ndarray             # [n_nodes, 3] float64, initial positions (unwrapped)
    conn: np.ndarray           # [n_elems, 8] int32
    fibre: np.ndarray          # [n_elems, 3] float64, unit, reference configuration
    mat_id: np.ndarray         # [n_elems] int32
    materials: List[Material]
    faces: np.ndarray          # [n_faces, 4] int32 endocardial quads (may be empty)
    p0: float = 0.0            # endocardial pressure amplitude
    T: float = 1.0             # pressure pulse period: p(t) = p0 sin^2(pi t / T)
    u0: Optional[np.ndarray] = None   # [3, n, n, n] float64 initial velocity (None = rest)
    sheet: Optional[np.ndarray] = None  # [n_elems, 3] unit sheet e_s (orthogonal to e_f)
    ta_max: float = 0.0        # active tension amplitude (0: passive)
    ta_t_on: float = 0.0       # the activation window [ta_t_on, ta_t_on + ta_duration]
    ta_duration: float = 0.0
    # penalty tethers (node [t] int32, target [t, 3], symmetric K [t, 6] as
    # xx, yy, zz, xy, xz, yz) or None
    tethers: Optional[Tuple[np.ndarray, np.ndarray, np.ndarray]] = None
    mg_rtol: float = 1e-10
    mg_pre: int = 2
    mg_post: int = 2
    mg_max_cycles: int = 50
    mg_krylov: int = 1          # Poisson by V-cycle-preconditioned conjugate gradients
    walls: int = 0              # 1: walled box (no slip, no penetration) instead of periodic
    convection: int = 1
    precision: str = "fp64"

    @property
    def h(self) -> float:
        return 1.0 / self.n

    @property
    def n_nodes(self) -> int:
        return int(self.X_ref.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.conn.shape[0])

    @property
    def n_faces(self) -> int:
        return int(self.faces.shape[0])

    def initial_velocity(self) -> np.ndarray:
        if self.u0 is None:
            return np.zeros((3, self.n, self.n, self.n), dtype=np.float64)
        return self.u0.copy()

    def material_arrays(self) -> Tuple[np.ndarray, np.ndarray]:
        models = np.array([m.model for m in self.materials], dtype=np.int32)
        params = np.array([m.padded() for m in self.materials], dtype=np.float64)
        return models, params


# ----------------------------------------------------------------------------
# structured hex meshing helpers
# ----------------------------------------------------------------------------

def _signed_volume_at_centre(P: np.ndarray) -> np.ndarray:
    """Triple product of the three mean edge vectors of each hex ([e, 8, 3])."""
    ex = (P[:, 1] - P[:, 0] + P[:, 3] - P[:, 2] + P[:, 5] - P[:, 4] + P[:, 7] - P[:, 6])
    ey = (P[:, 2] - P[:, 0] + P[:, 3] - P[:, 1] + P[:, 6] - P[:, 4] + P[:, 7] - P[:, 5])
    ez = (P[:, 4] - P[:, 0] + P[:, 5] - P[:, 1] + P[:, 6] - P[:, 2] + P[:, 7] - P[:, 3])
    return np.einsum("ei,ei->e", ex, np.cross(ey, ez))


def _swap_ij(conn: np.ndarray) -> np.ndarray:
    """Exchange local axes xi and eta (mirrors the element, flips orientation)."""
    perm = [0, 2, 1, 3, 4, 6, 5, 7]
    return conn[:, perm]


def _orient(conn: np.ndarray, X: np.ndarray) -> np.ndarray:
    vol = _signed_volume_at_centre(X[conn])
    conn = conn.copy()
    neg = vol < 0
    conn[neg] = _swap_ij(conn[neg])
    vol2 = _signed_volume_at_centre(X[conn])
    assert np.all(vol2 > 0), "degenerate hex in generated mesh"
    return conn


def _structured_conn(node_id, ne: Tuple[int, int, int]) -> np.ndarray:
    """Connectivity of an (ne0, ne1, ne2) block; node_id(i0, i1, i2) -> int arrays."""
    e0, e1, e2 = np.meshgrid(np.arange(ne[0]), np.arange(ne[1]), np.arange(ne[2]),
                             indexing="ij")
    e0, e1, e2 = e0.ravel(order="F"), e1.ravel(order="F"), e2.ravel(order="F")
    conn = np.empty((e0.size, 8), dtype=np.int64)
    for a, (i, j, k) in enumerate(HEX_CORNERS):
        conn[:, a] = node_id(e0 + i, e1 + j, e2 + k)
    return conn


# ----------------------------------------------------------------------------
# shapes
# ----------------------------------------------------------------------------

def block_mesh(n_el: int, side: float, centre=(0.5, 0.5, 0.5)):
    """Regular cube of n_el^3 hexes; returns X_ref [(n_el+1)^3, 3], conn [n_el^3, 8]."""
    m = n_el + 1
    t = np.linspace(-0.5 * side, 0.5 * side, m)
    gx, gy, gz = np.meshgrid(t, t, t, indexing="ij")
    # node id = i + m (j + m k), x fastest
    X = np.stack([gx.ravel(order="F"), gy.ravel(order="F"), gz.ravel(order="F")], axis=1)
    X = X + np.asarray(centre, dtype=np.float64)[None, :]

    def nid(i, j, k):
        return i + m * (j + m * k)
    conn = _structured_conn(nid, (n_el, n_el, n_el))
    return X, _orient(conn, X)


# edge nodes of the 10-node tetrahedron, in local order 4..9
TET_EDGES = ((0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3))


def tet_block_mesh(n_el: int, side: float, order: int = 1, centre=(0.5, 0.5, 0.5)):
    """Cube of n_el^3 cells, each split into 6 tetrahedra around its main
    diagonal (Kuhn's subdivision: conforming on the grid), positively oriented.
    order 1: 4-node tets on the (n_el+1)^3 grid nodes; order 2: 10-node tets
    with one node per edge (at its midpoint), vertices first.  Returns X_ref
    [n_nodes, 3] and conn [6 n_el^3, 4 or 10]."""
    X, _ = block_mesh(n_el, side, centre)
    m = n_el + 1
    e0, e1, e2 = np.meshgrid(np.arange(n_el), np.arange(n_el), np.arange(n_el), indexing="ij")
    base = np.stack([e0.ravel(order="F"), e1.ravel(order="F"), e2.ravel(order="F")], axis=1)
    tets = []
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        corner = np.zeros(3, dtype=np.int64)
        verts = [base + corner]
        for ax in perm:
            corner = corner.copy()
            corner[ax] = 1
            verts.append(base + corner)
        tets.append(np.stack([v[:, 0] + m * (v[:, 1] + m * v[:, 2]) for v in verts], axis=1))
    conn = np.concatenate(tets)
    P = X[conn]
    vol = np.einsum("ei,ei->e", P[:, 1] - P[:, 0], np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]))
    neg = vol < 0
    conn[neg] = conn[neg][:, [0, 2, 1, 3]]
    if order == 1:
        return X, conn.astype(np.int32)
    pairs = np.concatenate([np.sort(conn[:, [i, j]], axis=1) for i, j in TET_EDGES])
    uniq, inv = np.unique(pairs, axis=0, return_inverse=True)
    mid = 0.5 * (X[uniq[:, 0]] + X[uniq[:, 1]])
    edge_node = X.shape[0] + inv.reshape(len(TET_EDGES), -1).T
    conn10 = np.concatenate([conn, edge_node], axis=1)
    return np.concatenate([X, mid]), conn10.astype(np.int32)


def shell_mesh(n_theta: int, n_psi: int, n_tau: int, h: float, cx: float = 0.325,
               with_sheet: bool = False):
    """Truncated ellipsoidal shell.

    Node (it, ip, iq) with theta = 2 pi it / n_theta, psi linear in ip from the
    apex-hole angle psi_a to pi/2, tau = iq / n_tau (0 = endocardium):
        X = (cx + A cos psi, 0.5 + B sin psi cos theta, 0.5 + B sin psi sin theta)
        A = 0.31 + 0.04 tau,  B = 0.21 + 0.04 tau.
    The apex hole has endocardial radius 2h.  Returns X_ref, conn, fibre, faces
    (and the transmural sheet field when with_sheet).
    """
    psi_a = math.asin(2.0 * h / 0.21)
    th = 2.0 * math.pi * np.arange(n_theta) / n_theta
    ps = psi_a + (0.5 * math.pi - psi_a) * np.arange(n_psi + 1) / n_psi
    ta = np.arange(n_tau + 1) / n_tau
    T3, P3, Q3 = np.meshgrid(th, ps, ta, indexing="ij")
    A = 0.31 + 0.04 * Q3
    B = 0.21 + 0.04 * Q3
    X = np.stack([cx + A * np.cos(P3),
                  0.5 + B * np.sin(P3) * np.cos(T3),
                  0.5 + B * np.sin(P3) * np.sin(T3)], axis=-1)
    X = X.reshape(-1, 3, order="F")
    nt, npn = n_theta, n_psi + 1

    def nid(it, ip, iq):
        return (it % nt) + nt * (ip + npn * iq)
    conn = _structured_conn(nid, (n_theta, n_psi, n_tau))
    conn = _orient(conn, X)

    # fibre at each element centroid in parameter space
    e0, e1, e2 = np.meshgrid(np.arange(n_theta), np.arange(n_psi), np.arange(n_tau),
                             indexing="ij")
    e0, e1, e2 = e0.ravel(order="F"), e1.ravel(order="F"), e2.ravel(order="F")
    thc = 2.0 * math.pi * (e0 + 0.5) / n_theta
    psc = psi_a + (0.5 * math.pi - psi_a) * (e1 + 0.5) / n_psi
    tac = (e2 + 0.5) / n_tau
    Ac, Bc = 0.31 + 0.04 * tac, 0.21 + 0.04 * tac
    d_theta = np.stack([np.zeros_like(thc), -Bc * np.sin(psc) * np.sin(thc),
                        Bc * np.sin(psc) * np.cos(thc)], axis=1)
    d_psi = np.stack([-Ac * np.sin(psc), Bc * np.cos(psc) * np.cos(thc),
                      Bc * np.cos(psc) * np.sin(thc)], axis=1)
    e_th = d_theta / np.linalg.norm(d_theta, axis=1, keepdims=True)
    e_ps = d_psi / np.linalg.norm(d_psi, axis=1, keepdims=True)
    alpha = np.deg2rad(60.0 - 120.0 * tac)        # +60 endo (tau=0) .. -60 epi (tau=1)
    fibre = np.cos(alpha)[:, None] * e_th + np.sin(alpha)[:, None] * e_ps
    fibre /= np.linalg.norm(fibre, axis=1, keepdims=True)
    # transmural sheet direction: normal to the wall, Gram-Schmidt against the fibre
    sheet = np.cross(e_th, e_ps)
    sheet -= np.einsum("ei,ei->e", sheet, fibre)[:, None] * fibre
    sheet /= np.linalg.norm(sheet, axis=1, keepdims=True)

    # endocardial quads (iq = 0), oriented to point into the cavity (towards -d/dtau)
    f0, f1 = np.meshgrid(np.arange(n_theta), np.arange(n_psi), indexing="ij")
    f0, f1 = f0.ravel(order="F"), f1.ravel(order="F")
    faces = np.stack([nid(f0, f1, 0), nid(f0 + 1, f1, 0), nid(f0, f1 + 1, 0),
                      nid(f0 + 1, f1 + 1, 0)], axis=1)
    faces = _orient_faces(faces, X, inward_ref=nid(f0, f1, 1))
    if with_sheet:
        return X, conn, fibre, faces, np.ascontiguousarray(sheet)
    return X, conn, fibre, faces


def _orient_faces(faces: np.ndarray, X: np.ndarray, inward_ref: np.ndarray) -> np.ndarray:
    """Orient quads so (x1-x0 + x3-x2) x (x2-x0 + x3-x1) points away from inward_ref."""
    P = X[faces]
    exi = P[:, 1] - P[:, 0] + P[:, 3] - P[:, 2]
    eet = P[:, 2] - P[:, 0] + P[:, 3] - P[:, 1]
    nrm = np.cross(exi, eet)
    into_solid = X[inward_ref] - P.mean(axis=1)
    flip = np.einsum("fi,fi->f", nrm, into_solid) > 0
    faces = faces.copy()
    faces[flip] = faces[flip][:, [0, 2, 1, 3]]
    return faces


def leaflet_mesh(k: int, n_theta: int = 64, n_r: int = 32, cx: float = 0.325,
                 r0: float = 0.03, r1: float = 0.21, thick: float = 0.01):
    """Half-annular sheet theta in [k pi, (k+1) pi], r in [r0, r1], x in [cx-thick, cx]."""
    th = math.pi * (k + np.arange(n_theta + 1) / n_theta)
    rr = r0 + (r1 - r0) * np.arange(n_r + 1) / n_r
    xx = np.array([cx - thick, cx])
    T3, R3, X3 = np.meshgrid(th, rr, xx, indexing="ij")
    X = np.stack([X3, 0.5 + R3 * np.cos(T3), 0.5 + R3 * np.sin(T3)], axis=-1)
    X = X.reshape(-1, 3, order="F")
    m0, m1 = n_theta + 1, n_r + 1

    def nid(i, j, q):
        return i + m0 * (j + m1 * q)
    conn = _structured_conn(nid, (n_theta, n_r, 1))
    conn = _orient(conn, X)
    e0, e1 = np.meshgrid(np.arange(n_theta), np.arange(n_r), indexing="ij")
    thc = math.pi * (k + (e0.ravel(order="F") + 0.5) / n_theta)
    fibre = np.stack([np.zeros_like(thc), -np.sin(thc), np.cos(thc)], axis=1)
    return X, conn, fibre


def solenoidal_velocity(n: int, seed: int, amplitude: float, kmax: int = 4) -> np.ndarray:
    """Random divergence-free MAC velocity [3, n, n, n] (index [d, k, j, i]).

    A smooth random vector potential A (Fourier modes with |k_i| <= kmax,
    amplitudes 1 / (1 + |k|^2)) is sampled on cell edges and u = curl A is
    taken with one-sided differences along the edges, which makes every cell's
    net face flux vanish identically.  Scaled so max |u| = amplitude.  The
    Fourier sums are evaluated as separable contractions over the three axes.
    """
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    ks = np.arange(-kmax, kmax + 1)
    K = ks.size
    ka, kb, kc = np.meshgrid(ks, ks, ks, indexing="ij")
    weight = 1.0 / (1.0 + ka ** 2 + kb ** 2 + kc ** 2)
    weight[kmax, kmax, kmax] = 0.0                      # no mean mode
    idx = np.arange(n)
    Apot = []
    for e in range(3):
        coef = (rng.standard_normal((K, K, K)) + 1j * rng.standard_normal((K, K, K))) * weight
        # edge e carries A_e at: coordinate e at the cell centre, the others at faces
        off = [0.0, 0.0, 0.0]
        off[e] = 0.5
        E = [np.exp(2j * math.pi * np.outer(ks, (idx + off[ax]) * h)) for ax in range(3)]
        t1 = np.einsum("abc,ai->bci", coef, E[0])
        t2 = np.einsum("bci,bj->cji", t1, E[1])
        Apot.append(np.real(np.einsum("cji,ck->kji", t2, E[2])))
    Ax, Ay, Az = Apot

    def dfw(q, axis):  # forward difference along array axis (0=z, 1=y, 2=x)
        return (np.roll(q, -1, axis=axis) - q) / h
    # u_x at (i h, (j+1/2) h, (k+1/2) h) = dAz/dy - dAy/dz
    ux = dfw(Az, 1) - dfw(Ay, 0)
    uy = dfw(Ax, 0) - dfw(Az, 2)
    uz = dfw(Ay, 2) - dfw(Ax, 1)
    u = np.stack([ux, uy, uz])
    u *= amplitude / np.max(np.abs(u))
    return np.ascontiguousarray(u)


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

HO_PARAMS = (0.5, 5.0, 1.5, 8.0, 7.0)      # a, b, a_f, b_f, kappa (kappa = 14 a)
NH_BLOCK = (10.0, 100.0)                   # mu_s, kappa

# Left-ventricle table (a, b, a_f, b_f, a_s, b_s, a_fs, b_fs in dyn/cm^2 and 1),
# scaled so that a matches HO_PARAMS; kappa = 14 a as for HO_PARAMS.
_LV_TABLE = dict(a=2244.87, b=1.6215, af=24267.0, bf=1.8268, as_=5562.38, bs=0.7746,
                 afs=3905.16, bfs=1.695)
_LV_SCALE = HO_PARAMS[0] / _LV_TABLE["a"]
LV_PARAMS = (HO_PARAMS[0], _LV_TABLE["b"], _LV_TABLE["af"] * _LV_SCALE, _LV_TABLE["bf"],
             14.0 * HO_PARAMS[0], _LV_TABLE["as_"] * _LV_SCALE, _LV_TABLE["bs"],
             _LV_TABLE["afs"] * _LV_SCALE, _LV_TABLE["bfs"])
# active tension amplitude relative to the peak cavity pressure: 84260 Pa against
# the 14530 Pa systolic maximum of the left-ventricle model
LV_TA_OVER_P = 84260.0 / 14530.0


def _block_problem(name, n, n_el, dt, n_steps, material, fibre_seed=None,
                   seed=0) -> Problem:
    h = 1.0 / n
    X_ref, conn = block_mesh(n_el, 0.3)
    c = np.array([0.5, 0.5, 0.5])
    rng = np.random.default_rng(seed)
    X0 = c + (X_ref - c) * np.array([1.1, 1.0, 1.0])
    X0 = X0 + rng.uniform(-0.05 * h, 0.05 * h, size=X0.shape)
    ne = conn.shape[0]
    if fibre_seed is None:
        fibre = np.tile([1.0, 0.0, 0.0], (ne, 1))
    else:
        g = np.random.default_rng(fibre_seed).uniform(-0.25 * math.pi, 0.25 * math.pi, ne)
        fibre = np.stack([np.cos(g), np.sin(g), np.zeros(ne)], axis=1)
    return Problem(name=name, n=n, rho=1.0, mu=0.01, dt=dt, n_steps=n_steps,
                   X_ref=X_ref, X0=X0, conn=conn.astype(np.int32),
                   fibre=np.ascontiguousarray(fibre, dtype=np.float64),
                   mat_id=np.zeros(ne, dtype=np.int32), materials=[material],
                   faces=np.zeros((0, 4), dtype=np.int32))


def neo_hookean_block(n: int = 32, n_steps: int = 10, seed: int = 0) -> Problem:
    """Neo-Hookean 6^3-hex block (343 nodes), side 0.3, 1.1x x-stretch, rest fluid."""
    return _block_problem("nh_block_32", n, 6, 1e-3, n_steps,
                          Material(NEO_HOOKEAN, NH_BLOCK), seed=seed)


def ho_block(n: int = 64, n_el: int = 12, n_steps: int = 50, seed: int = 0,
             fibre_seed: int = 1, params=HO_PARAMS) -> Problem:
    """Holzapfel-Ogden block with fibres (cos g, sin g, 0), g ~ U(-pi/4, pi/4)."""
    return _block_problem(f"ho_block_{n}", n, n_el, 1e-3, n_steps,
                          Material(HOLZAPFEL_OGDEN, tuple(params)),
                          fibre_seed=fibre_seed, seed=seed)


# the other laws' table constants (Cook's membrane divided by 16; the valve
# laws' Pa values times 1e-4), kappa = 14 times the small-strain shear modulus
LAW_PARAMS = {
    STANDARD_REINFORCING: (0.5, 10.0, 75.0, 7.0),           # G_T, G_L, E_L, kappa
    FIBRE_REINFORCED_1: (1.74, 3.13, 55.93, 48.7),          # C_1, a_f, b_f, kappa
    FIBRE_REINFORCED_2: (0.121, 7.99, 2.423, 57.62, 27.1),  # C_10, C_01, a_f, b_f, kappa
}


def law_block(model: int, n: int = 32, n_steps: int = 10, seed: int = 0) -> Problem:
    """The 6^3-hex block (stretched 1.1x in x, jittered) with one of the other
    laws and the Cook's-membrane fibre (1, 1, 1)/sqrt(3) in every element."""
    p = _block_problem(f"law{model}_block_{n}", n, 6, 1e-3, n_steps,
                       Material(model, LAW_PARAMS[model]), seed=seed)
    p.fibre = np.ascontiguousarray(np.tile(np.ones(3) / math.sqrt(3.0), (p.n_elems, 1)))
    return p


def tet_block(order: int, model: int = STANDARD_REINFORCING, n: int = 32, n_el: int = 4,
              n_steps: int = 10, dt: float = 1e-3, seed: int = 0, kappa_tether: float = 1.0) -> Problem:
    """Tetrahedral block (order 1: P1, order 2: P2), side 0.3, stretched 1.1x in
    x and jittered, with one of the laws, the Cook's-membrane fibre (1, 1, 1)/sqrt(3),
    and its x-min face held at its initial position by penalty tethers (the
    benchmark's fixed face)."""
    h = 1.0 / n
    X_ref, conn = tet_block_mesh(n_el, 0.3, order)
    c = np.array([0.5, 0.5, 0.5])
    rng = np.random.default_rng(seed)
    X0 = c + (X_ref - c) * np.array([1.1, 1.0, 1.0])
    X0 = X0 + rng.uniform(-0.05 * h, 0.05 * h, size=X0.shape)
    ne = conn.shape[0]
    node = np.flatnonzero(X_ref[:, 0] <= X_ref[:, 0].min() + 1e-12).astype(np.int32)
    K = np.tile([kappa_tether, kappa_tether, kappa_tether, 0.0, 0.0, 0.0], (node.size, 1))
    params = HO_PARAMS if model == HOLZAPFEL_OGDEN else (NH_BLOCK if model == NEO_HOOKEAN
                                                          else LAW_PARAMS[model])
    return Problem(name=f"tet{4 if order == 1 else 10}_block_{n}", n=n, rho=1.0, mu=0.01, dt=dt,
                   n_steps=n_steps, X_ref=X_ref, X0=X0, conn=conn,
                   fibre=np.ascontiguousarray(np.tile(np.ones(3) / math.sqrt(3.0), (ne, 1))),
                   mat_id=np.zeros(ne, dtype=np.int32), materials=[Material(model, params)],
                   faces=np.zeros((0, 4), dtype=np.int32), tethers=(node, X0[node].copy(), K))


def ho_shell(n: int = 128, n_theta: int = 224, n_psi: int = 80, n_tau: int = 6,
             n_steps: int = 100, dt: float = 5e-4) -> Problem:
    """Holzapfel-Ogden truncated-ellipsoid shell with endocardial pressure pulse."""
    h = 1.0 / n
    X, conn, fibre, faces = shell_mesh(n_theta, n_psi, n_tau, h)
    ne = conn.shape[0]
    return Problem(name=f"ho_shell_{n}", n=n, rho=1.0, mu=0.01, dt=dt, n_steps=n_steps,
                   X_ref=X, X0=X.copy(), conn=conn.astype(np.int32),
                   fibre=np.ascontiguousarray(fibre), mat_id=np.zeros(ne, dtype=np.int32),
                   materials=[Material(HOLZAPFEL_OGDEN, HO_PARAMS)],
                   faces=faces.astype(np.int32), p0=1.0, T=n_steps * dt)


def shell_base_tethers(X: np.ndarray, n_theta: int, n_psi: int, n_tau: int, kappa: float):
    """Base constraint of the left-ventricle model on the shell's base ring
    (psi = pi/2, every wall layer): zero axial and circumferential displacement,
    radial motion in the base plane free.  K = kappa (e_x e_x^T + c c^T) with
    the circumferential c = (0, -sin theta, cos theta); target = X."""
    npn = n_psi + 1
    it, iq = np.meshgrid(np.arange(n_theta), np.arange(n_tau + 1), indexing="ij")
    node = (it + n_theta * (n_psi + npn * iq)).ravel().astype(np.int32)
    th = np.arctan2(X[node, 2] - 0.5, X[node, 1] - 0.5)
    s, c = np.sin(th), np.cos(th)
    z = np.zeros_like(th)
    K = kappa * np.stack([1.0 + z, s * s, c * c, z, z, -s * c], axis=1)
    return node, np.ascontiguousarray(X[node]), np.ascontiguousarray(K)


LV_BASE_KAPPA = 1.0   # nodal penalty stiffness of the base constraint


def wall_nodes(n: int = 12, n_nodes: int = 60, seed: int = 5, k: float = 50.0,
               n_steps: int = 3, dt: float = 1e-3) -> Problem:
    """Free nodes (no elements) in a walled box, half of them within 2h of a
    wall, each tethered (isotropic stiffness k) to a target 0.3h away: a
    workload whose spreading and interpolation stencils cross the walls."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    X = rng.uniform(2.5 * h, 1.0 - 2.5 * h, (n_nodes, 3))
    near = rng.integers(0, 3, n_nodes // 2)
    side = rng.integers(0, 2, n_nodes // 2)
    off = rng.uniform(0.1 * h, 1.9 * h, n_nodes // 2)
    for q in range(n_nodes // 2):
        X[q, near[q]] = off[q] if side[q] == 0 else 1.0 - off[q]
    target = X + 0.3 * h * rng.standard_normal(X.shape) / np.sqrt(3.0)
    K = np.tile([k, k, k, 0.0, 0.0, 0.0], (n_nodes, 1))
    return Problem(name=f"wall_nodes_{n}", n=n, rho=1.0, mu=0.01, dt=dt, n_steps=n_steps,
                   X_ref=X, X0=X.copy(), conn=np.zeros((0, 8), dtype=np.int32),
                   fibre=np.zeros((0, 3)), mat_id=np.zeros(0, dtype=np.int32),
                   materials=[Material(NEO_HOOKEAN, (1.0, 10.0))],
                   faces=np.zeros((0, 4), dtype=np.int32),
                   tethers=(np.arange(n_nodes, dtype=np.int32), target, K), walls=1)


def walled_shell(n: int = 64, n_theta: int = 224, n_psi: int = 80, n_tau: int = 6,
                 n_steps: int = 50, dt: float = 5e-4) -> Problem:
    """The Holzapfel-Ogden shell in a walled box (no slip, no penetration),
    centred at c_x = 0.5 so that the apex keeps clear of the walls."""
    h = 1.0 / n
    X, conn, fibre, faces = shell_mesh(n_theta, n_psi, n_tau, h, cx=0.5)
    ne = conn.shape[0]
    return Problem(name=f"walled_shell_{n}", n=n, rho=1.0, mu=0.01, dt=dt, n_steps=n_steps,
                   X_ref=X, X0=X.copy(), conn=conn.astype(np.int32),
                   fibre=np.ascontiguousarray(fibre), mat_id=np.zeros(ne, dtype=np.int32),
                   materials=[Material(HOLZAPFEL_OGDEN, HO_PARAMS)],
                   faces=faces.astype(np.int32), p0=1.0, T=n_steps * dt, walls=1)


def lv_shell(n: int = 128, n_theta: int = 224, n_psi: int = 80, n_tau: int = 6,
             n_steps: int = 100, dt: float = 5e-4) -> Problem:
    """The shell with the full Holzapfel-Ogden law (LV_PARAMS), transmural
    sheets, one active-tension pulse over the run (peak at mid-run like the
    cavity pressure pulse) and the base constraint as penalty tethers."""
    h = 1.0 / n
    X, conn, fibre, faces, sheet = shell_mesh(n_theta, n_psi, n_tau, h, with_sheet=True)
    ne = conn.shape[0]
    p0 = 1.0
    tethers = shell_base_tethers(X, n_theta, n_psi, n_tau, LV_BASE_KAPPA)
    return Problem(name=f"lv_shell_{n}", n=n, rho=1.0, mu=0.01, dt=dt, n_steps=n_steps,
                   X_ref=X, X0=X.copy(), conn=conn.astype(np.int32),
                   fibre=np.ascontiguousarray(fibre), mat_id=np.zeros(ne, dtype=np.int32),
                   materials=[Material(HOLZAPFEL_OGDEN, LV_PARAMS)],
                   faces=faces.astype(np.int32), p0=p0, T=n_steps * dt, sheet=sheet,
                   ta_max=LV_TA_OVER_P * p0, ta_t_on=0.0, ta_duration=n_steps * dt,
                   tethers=tethers)


def lv_block(n: int = 32, n_el: int = 6, n_steps: int = 20, seed: int = 0,
             frame_seed: int = 2) -> Problem:
    """Block with the full Holzapfel-Ogden law (LV_PARAMS), a random orthonormal
    fibre / sheet pair per element, an active-tension pulse over the run and
    its x-min face tethered (kappa = 1) at its initial position."""
    p = _block_problem(f"lv_block_{n}", n, n_el, 1e-3, n_steps,
                       Material(HOLZAPFEL_OGDEN, LV_PARAMS), seed=seed)
    rng = np.random.default_rng(frame_seed)
    ne = p.n_elems
    f = rng.standard_normal((ne, 3))
    f /= np.linalg.norm(f, axis=1, keepdims=True)
    s = rng.standard_normal((ne, 3))
    s -= np.einsum("ei,ei->e", s, f)[:, None] * f
    s /= np.linalg.norm(s, axis=1, keepdims=True)
    p.fibre, p.sheet = np.ascontiguousarray(f), np.ascontiguousarray(s)
    p.ta_max, p.ta_t_on, p.ta_duration = 2.0, 0.0, n_steps * p.dt
    # the face of smallest x held at its initial position (kappa I tethers)
    node = np.flatnonzero(p.X_ref[:, 0] <= p.X_ref[:, 0].min() + 1e-12).astype(np.int32)
    K = np.tile([1.0, 1.0, 1.0, 0.0, 0.0, 0.0], (node.size, 1))
    p.tethers = (node, np.ascontiguousarray(p.X0[node]), K)
    return p


def shell_with_leaflets(n: int = 192, n_steps: int = 50, dt: float = 5e-4,
                        seed: int = 0) -> Problem:
    """The shell (288 x 104 x 8 hexes) plus two neo-Hookean leaflets and a random
    divergence-free initial velocity of max amplitude 0.1."""
    h = 1.0 / n
    Xs, cs, fs, faces = shell_mesh(288, 104, 8, h)
    parts_X, parts_c, parts_f, parts_m = [Xs], [cs], [fs], [np.zeros(cs.shape[0], np.int32)]
    off = Xs.shape[0]
    for k in (0, 1):
        Xl, cl, fl = leaflet_mesh(k)
        parts_X.append(Xl)
        parts_c.append(cl + off)
        parts_f.append(fl)
        parts_m.append(np.ones(cl.shape[0], np.int32))
        off += Xl.shape[0]
    X = np.concatenate(parts_X)
    conn = np.concatenate(parts_c).astype(np.int32)
    return Problem(name=f"shell_leaflets_{n}", n=n, rho=1.0, mu=0.01, dt=dt,
                   n_steps=n_steps, X_ref=X, X0=X.copy(), conn=conn,
                   fibre=np.ascontiguousarray(np.concatenate(parts_f)),
                   mat_id=np.concatenate(parts_m),
                   materials=[Material(HOLZAPFEL_OGDEN, HO_PARAMS),
                              Material(NEO_HOOKEAN, NH_BLOCK)],
                   faces=faces.astype(np.int32), p0=1.0, T=n_steps * dt,
                   u0=solenoidal_velocity(n, seed, 0.1))


def workload(name: str) -> Problem:
    """The five named workloads (sizes as in the benchmark table)."""
    if name == "nh_block_32":        # FP64, 32^3, 10 steps
        return neo_hookean_block()
    if name == "ho_shell_128":       # FP64, 128^3, 100 steps (headline)
        return ho_shell()
    if name == "shell_leaflets_192":  # FP64, 192^3, 50 steps
        return shell_with_leaflets()
    if name == "nh_block_32_mixed":  # mixed precision, 32^3, 100 steps
        p = neo_hookean_block(n_steps=100)
        p.name, p.precision = "nh_block_32_mixed", "mixed"
        return p
    if name == "ho_block_64":        # adjoint workload, 64^3, 50 steps
        return ho_block()
    if name == "lv_shell_128":       # full HO + active tension, 128^3, 100 steps
        return lv_shell()
    if name == "lv_block_32":        # full HO + active tension, 32^3, 20 steps
        return lv_block()
    if name == "walled_block_32":    # walled box, NH block, 32^3, 10 steps
        p = neo_hookean_block()
        p.name, p.walls = "walled_block_32", 1
        return p
    if name == "walled_shell_64":    # walled box, HO shell, 64^3 (128^3 image grid), 50 steps
        return walled_shell()
    if name == "walled_ho_block_64":  # the adjoint workload in a walled box (128^3 image grid)
        p = ho_block()
        p.name, p.walls = "walled_ho_block_64", 1
        return p
    if name == "tet10_block_64":     # P2 tets, Psi_1, tethered face: the benchmark's settings
        p = tet_block(2, n=64, n_el=10, n_steps=20)
        return p
    raise KeyError(name)


WORKLOADS = ("nh_block_32", "ho_shell_128", "shell_leaflets_192",
             "nh_block_32_mixed", "ho_block_64", "lv_shell_128", "lv_block_32", "tet10_block_64",
             "walled_block_32", "walled_shell_64", "walled_ho_block_64")
