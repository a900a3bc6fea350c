/*
 * ibref.c -- plain FP64 CPU oracle of the matrix-free immersed-boundary step.
 *
 * TEST INFRASTRUCTURE ONLY (see ibref.h): loaded by the tests, the smoke check
 * and the CPU-baseline leg of the benchmark, never by the product path.
 *
 * Written from the paper's equations, loop by loop, in FP64, with no blocking
 * or fusion.  Build with -ffp-contract=off so every product and sum is rounded
 * as written.  OpenMP (optional) only parallelises independent grid loops;
 * reductions and scatters are serial so results do not depend on threads.
 *
 * Paper sections followed:
 *   "Temporal Discretization"    backward Euler with explicit coupling
 *   "Spatial Discretization"     Chorin split: Helmholtz solve, Poisson solve,
 *                                velocity correction, weak-form nodal force,
 *                                spreading at X^n, interpolation of u^{n+1}
 *   "Discretization of the Navier-Stokes equations"   MAC staggered grid
 *   "Eulerian-Lagrangian coupling operators"          spreading, interpolation,
 *                                nodal quadrature rule, nodal force formula
 *   "Constitutive laws"          Psi = W + U(J), U = (kappa/2)(ln J)^2,
 *                                modified invariant I1bar, the laws Psi_1 to
 *                                Psi_3 and the HO model Psi_4 with its sheet
 *                                and fibre-sheet terms
 *   "Mitral valve model"         neo-Hookean chordae law; tetrahedral meshes
 *                                (P1 and P2 elements) of the valve set-ups
 *   "Dynamic left ventricle model"   active fibre stress and its waveform,
 *                                endocardial pressure, base constraint
 *   Cook's membrane and aortic valve set-ups   penalty tethers
 *   "Spatial Discretization"     the walled box's boundary conditions,
 *                                solved on the box's mirror image
 *   Abstract                     geometric multigrid for the fluid solves
 * The reverse step and the rollout gradient are not in the paper: they are the
 * transposes of the steps above.  Every function is pinned by the tests
 * against closed forms, brute force, invariants or central differences.
 */
#include "ibref.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* grid helpers                                                              */
/* ------------------------------------------------------------------------- */

static inline int wrap(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }
static inline long gidx(int i, int j, int k, int n) {
    return (long)wrap(i, n) + (long)n * ((long)wrap(j, n) + (long)n * (long)wrap(k, n));
}
/* shift (i,j,k) by s along axis d */
static inline long gidx_s(int i, int j, int k, int n, int d, int s) {
    if (d == 0) i += s; else if (d == 1) j += s; else k += s;
    return gidx(i, j, k, n);
}

/* MAC discrete Laplacian, the 7-point second difference on each lattice. */
void ibref_laplacian(int32_t n, const double* q, double* out) {
    const double h = 1.0 / n, ih2 = 1.0 / (h * h);
#pragma omp parallel for
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double c = q[gidx(i, j, k, n)];
                double s = 0.0;
                for (int d = 0; d < 3; ++d)
                    s += (q[gidx_s(i, j, k, n, d, 1)] - 2.0 * c + q[gidx_s(i, j, k, n, d, -1)]) * ih2;
                out[gidx(i, j, k, n)] = s;
            }
}

/* (D u)[c] = sum_d (u^d[c + e_d] - u^d[c]) / h : divergence at cell centres. */
void ibref_divergence(int32_t n, const double* u, double* out) {
    const double h = 1.0 / n;
    const long N3 = (long)n * n * n;
#pragma omp parallel for
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double s = 0.0;
                for (int d = 0; d < 3; ++d)
                    s += (u[d * N3 + gidx_s(i, j, k, n, d, 1)] - u[d * N3 + gidx(i, j, k, n)]) / h;
                out[gidx(i, j, k, n)] = s;
            }
}

/* (G p)^d[c] = (p[c] - p[c - e_d]) / h : gradient on the faces. */
void ibref_gradient(int32_t n, const double* p, double* out) {
    const double h = 1.0 / n;
    const long N3 = (long)n * n * n;
#pragma omp parallel for
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                for (int d = 0; d < 3; ++d)
                    out[d * N3 + gidx(i, j, k, n)] =
                        (p[gidx(i, j, k, n)] - p[gidx_s(i, j, k, n, d, -1)]) / h;
}

/*
 * Convective term C(u) = div(u (x) u) in conservative (flux) form on the MAC
 * grid, centred.  The paper times a separate "convective term" but does not
 * print its discretisation; this is the standard Harlow-Welch flux form.
 * For component d at its face c:
 *   normal flux   Fdd at the cell centre c:   ((u^d[c] + u^d[c+e_d]) / 2)^2
 *   tangential    Ede at the edge below c:    ((u^d[c-e_e] + u^d[c]) / 2)
 *                                           * ((u^e[c-e_d] + u^e[c]) / 2)
 *   C^d[c] = (Fdd[c] - Fdd[c-e_d]) / h + sum_{e != d} (Ede[c+e_e] - Ede[c]) / h
 */
static double conv_normal_flux(const double* ud, int n, int i, int j, int k, int d) {
    double a = 0.5 * (ud[gidx(i, j, k, n)] + ud[gidx_s(i, j, k, n, d, 1)]);
    return a * a;
}
static double conv_edge_flux(const double* ud, const double* ue, int n, int i, int j, int k,
                             int d, int e) {
    double ad = 0.5 * (ud[gidx_s(i, j, k, n, e, -1)] + ud[gidx(i, j, k, n)]);
    double ae = 0.5 * (ue[gidx_s(i, j, k, n, d, -1)] + ue[gidx(i, j, k, n)]);
    return ad * ae;
}
void ibref_convection(int32_t n, const double* u, double* out) {
    const double h = 1.0 / n;
    const long N3 = (long)n * n * n;
#pragma omp parallel for
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                for (int d = 0; d < 3; ++d) {
                    const double* ud = u + d * N3;
                    int im[3] = {i, j, k};
                    im[d] -= 1;
                    double s = (conv_normal_flux(ud, n, i, j, k, d) -
                                conv_normal_flux(ud, n, im[0], im[1], im[2], d)) / h;
                    for (int e = 0; e < 3; ++e) {
                        if (e == d) continue;
                        const double* ue = u + e * N3;
                        int ip[3] = {i, j, k};
                        ip[e] += 1;
                        s += (conv_edge_flux(ud, ue, n, ip[0], ip[1], ip[2], d, e) -
                              conv_edge_flux(ud, ue, n, i, j, k, d, e)) / h;
                    }
                    out[d * N3 + gidx(i, j, k, n)] = s;
                }
}

/* ------------------------------------------------------------------------- */
/* regularized delta function and the coupling operators                     */
/* ------------------------------------------------------------------------- */

/* Peskin's four-point kernel phi(r) (the paper cites Peskin 2002 for delta_h);
 * delta_h(x) = prod_d phi(x_d / h) / h^3. */
double ibref_phi(double r) {
    double a = fabs(r);
    if (a < 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
    if (a < 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
    return 0.0;
}

/* Lattice coordinate of position x along axis e for the lattice of component d:
 * the face lattice d has points at i*h along d and (i+1/2)*h along the others. */
static inline double lattice_coord(double x, double h, int d, int e) {
    return x / h - (e == d ? 0.0 : 0.5);
}

/* The four lattice indices b-1..b+2 (b = floor(r)) carry all of phi's support. */
static void stencil_1d(double r, int* first, double w[4]) {
    int b = (int)floor(r);
    *first = b - 1;
    for (int m = 0; m < 4; ++m) w[m] = ibref_phi(r - (double)(b - 1 + m));
}

/*
 * Spreading ("Eulerian-Lagrangian coupling operators"):
 *   f^d[idx] += sum_q F^d_q delta_h(x^d_idx - X_q)
 * F_q is the nodal force already integrated against the basis (the nodal
 * quadrature rule carries the weights), so no extra w_q appears.
 */
void ibref_spread(int32_t n, int32_t n_nodes, const double* X, const double* F, double* f) {
    const double h = 1.0 / n, ih3 = 1.0 / (h * h * h);
    const long N3 = (long)n * n * n;
    for (int q = 0; q < n_nodes; ++q) {
        for (int d = 0; d < 3; ++d) {
            int s0[3];
            double w[3][4];
            for (int e = 0; e < 3; ++e) stencil_1d(lattice_coord(X[3 * q + e], h, d, e), &s0[e], w[e]);
            for (int c = 0; c < 4; ++c)
                for (int b = 0; b < 4; ++b)
                    for (int a = 0; a < 4; ++a) {
                        double wt = w[0][a] * w[1][b] * w[2][c] * ih3;
                        f[d * N3 + gidx(s0[0] + a, s0[1] + b, s0[2] + c, n)] += F[3 * q + d] * wt;
                    }
        }
    }
}

/*
 * Interpolation: U^d_q = sum_idx u^d[idx] delta_h(x^d_idx - X_q) h^3.  With the
 * nodal quadrature rule the L2 projection onto the nodal space is the identity
 * at the nodes, so U_q is the nodal velocity.
 */
void ibref_interpolate(int32_t n, int32_t n_nodes, const double* X, const double* u, double* U) {
    const double h = 1.0 / n;
    const long N3 = (long)n * n * n;
    for (int q = 0; q < n_nodes; ++q) {
        for (int d = 0; d < 3; ++d) {
            int s0[3];
            double w[3][4];
            for (int e = 0; e < 3; ++e) stencil_1d(lattice_coord(X[3 * q + e], h, d, e), &s0[e], w[e]);
            double acc = 0.0;
            for (int c = 0; c < 4; ++c)
                for (int b = 0; b < 4; ++b)
                    for (int a = 0; a < 4; ++a)
                        acc += u[d * N3 + gidx(s0[0] + a, s0[1] + b, s0[2] + c, n)] *
                               (w[0][a] * w[1][b] * w[2][c]);
            U[3 * q + d] = acc;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* constitutive laws ("Constitutive laws")                                   */
/* ------------------------------------------------------------------------- */

static double det3(const double* A) {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}
/* cofactor matrix: cof(A) = det(A) A^{-T} */
static void cof3(const double* A, double* C) {
    C[0] = A[4] * A[8] - A[5] * A[7];
    C[1] = A[5] * A[6] - A[3] * A[8];
    C[2] = A[3] * A[7] - A[4] * A[6];
    C[3] = A[2] * A[7] - A[1] * A[8];
    C[4] = A[0] * A[8] - A[2] * A[6];
    C[5] = A[1] * A[6] - A[0] * A[7];
    C[6] = A[1] * A[5] - A[2] * A[4];
    C[7] = A[2] * A[3] - A[0] * A[5];
    C[8] = A[0] * A[4] - A[1] * A[3];
}

/*
 * First Piola-Kirchhoff stress P = dPsi/dF and the energy density Psi
 * ("Constitutive laws").
 *   common:  J = det F, I1 = tr(F^T F), I1bar = J^{-2/3} I1,
 *            volumetric U(J) = (kappa/2)(ln J)^2 -> kappa ln J F^{-T}
 *   neo-Hookean (params mu_s, kappa), the chordae law of the mitral-valve model
 *            with coefficient a = mu_s / 2:
 *            Psi = (mu_s/2)(I1bar - 3) + U(J)
 *            P   = mu_s J^{-2/3} (F - (I1/3) F^{-T}) + kappa ln J F^{-T}
 *   Holzapfel-Ogden Psi_4 (params a, b, a_f, b_f, kappa, a_s, b_s, a_fs, b_fs),
 *   I4i = e_i . C e_i (i = f, s), I4i* = max(I4i, 1), I8fs = e_f . C e_s:
 *            Psi = a/(2b) (exp(b (I1bar - 3)) - 1)
 *                + sum_i a_i/(2 b_i) (exp(b_i (I4i* - 1)^2) - 1)
 *                + a_fs/(2 b_fs) (exp(b_fs I8fs^2) - 1) + U(J)
 *            P   = a exp(b (I1bar-3)) J^{-2/3} (F - (I1/3) F^{-T})
 *                + sum_i 2 a_i (I4i* - 1) exp(b_i (I4i* - 1)^2) (F e_i) (x) e_i
 *                + a_fs I8fs exp(b_fs I8fs^2) ((F e_f) (x) e_s + (F e_s) (x) e_f)
 *                + kappa ln J F^{-T}
 *   (the printed P_4 has F^T in the isotropic bracket where F^{-T} is the
 *   derivative of Psi_4, its isotropic energy lacks the -1 offset, and its
 *   fibre-sheet term 2 a_fs I8 e^{..} (F e_f) (x) e_s is not the derivative of
 *   the printed energy, whose dI8fs/dF = (F e_f) (x) e_s + (F e_s) (x) e_f; all
 *   three are read as corrected here.)
 *   modified standard reinforcing Psi_1 (params G_T, G_L, E_L, kappa),
 *   I5f = e_f . C^2 e_f = |C e_f|^2:
 *            Psi = (G_T/2)(I1bar - 3) + ((G_T - G_L)/2)(2 I4f - I5f - 1)
 *                + ((E_L + G_T - 4 G_L)/8)(I4f - 1)^2 + U(J)
 *            P   = G_T J^{-2/3}(F - (I1/3) F^{-T})
 *                + (2 (G_T - G_L) + ((E_L + G_T - 4 G_L)/2)(I4f - 1)) (F e_f) (x) e_f
 *                - (G_T - G_L)((F e_f) (x) (C e_f) + (F C e_f) (x) e_f) + kappa ln J F^{-T}
 *   fibre-reinforced model 1, Psi_2 (params C_1, a_f, b_f, kappa):
 *            Psi = C_1 (I1bar - 3) + a_f/(2 b_f)(exp(b_f (I4f* - 1)^2) - 1) + U(J)
 *   fibre-reinforced model 2, Psi_3 (params C_10, C_01, a_f, b_f, kappa), with the
 *   plain I4f as printed (the fibre also resists compression):
 *            Psi = C_10 (exp(C_01 (I1bar - 3)) - 1) + a_f/(2 b_f)(exp(b_f (I4f - 1)^2) - 1) + U(J)
 *            P   = 2 C_10 C_01 exp(C_01 (I1bar - 3)) J^{-2/3}(F - (I1/3) F^{-T}) + ...
 *   (the printed P_3 has C_10 in the exponent where the energy has C_01; the
 *   derivative of the energy is taken).
 *   Active stress of the myocardium (left-ventricle model): the second
 *   Piola-Kirchhoff stress S_a = T e_f (x) e_f with T = T_a (1 + 4.9 (sqrt(I4f) - 1))
 *   is added to HO materials as P_a = F S_a = T (F e_f) (x) e_f (the model
 *   introduces S_a and then adds it as a first Piola-Kirchhoff stress; the
 *   push-forward by F is the reading taken).  At frozen T_a it has the potential
 *   W_a = (T_a/2) ((1 - 4.9)(I4f - 1) + (2/3) 4.9 (I4f^{3/2} - 1)), which is added
 *   to Psi so that the nodal force stays minus the energy gradient.
 * Returns IBREF_E_NUMERIC when J <= 0, IBREF_E_INVAL for an unknown model or a
 * sheet term without es.
 */
int ibref_pk1(int32_t model, const double* par, const double* Fm, const double* ef,
              const double* es, double Ta, double* P, double* psi) {
    double J = det3(Fm);
    if (!(J > 0.0)) return IBREF_E_NUMERIC;
    double cof[9], FiT[9];
    cof3(Fm, cof);
    for (int r = 0; r < 9; ++r) FiT[r] = cof[r] / J;
    double I1 = 0.0;
    for (int r = 0; r < 9; ++r) I1 += Fm[r] * Fm[r];
    double Jm23 = pow(J, -2.0 / 3.0);
    double lnJ = log(J);
    double kappa, iso_coef, energy;
    double fib_coef = 0.0, sh_coef = 0.0, fs_coef = 0.0, i5_coef = 0.0;
    double Fe[3] = {0.0, 0.0, 0.0}, Fs[3] = {0.0, 0.0, 0.0};
    double esv[3] = {0.0, 0.0, 0.0}, Ce[3] = {0.0, 0.0, 0.0}, FCe[3] = {0.0, 0.0, 0.0};
    if (model != IBREF_NEO_HOOKEAN)
        for (int r = 0; r < 3; ++r) Fe[r] = Fm[3 * r] * ef[0] + Fm[3 * r + 1] * ef[1] + Fm[3 * r + 2] * ef[2];
    const double I4 = Fe[0] * Fe[0] + Fe[1] * Fe[1] + Fe[2] * Fe[2];
    if (model == IBREF_NEO_HOOKEAN) {
        double mu_s = par[0];
        kappa = par[1];
        iso_coef = mu_s;
        energy = 0.5 * mu_s * (Jm23 * I1 - 3.0);
    } else if (model == IBREF_HOLZAPFEL_OGDEN) {
        double a = par[0], b = par[1], af = par[2], bf = par[3];
        double as = par[5], bs = par[6], afs = par[7], bfs = par[8];
        kappa = par[4];
        double E1 = exp(b * (Jm23 * I1 - 3.0));
        iso_coef = a * E1;
        energy = a / (2.0 * b) * (E1 - 1.0);
        double I4s = I4 > 1.0 ? I4 : 1.0;
        double Ef = exp(bf * (I4s - 1.0) * (I4s - 1.0));
        fib_coef = 2.0 * af * (I4s - 1.0) * Ef;
        if (af != 0.0) energy += af / (2.0 * bf) * (Ef - 1.0);
        if (as != 0.0 || afs != 0.0) {
            if (!es) return IBREF_E_INVAL;
            for (int r = 0; r < 3; ++r) {
                esv[r] = es[r];
                Fs[r] = Fm[3 * r] * es[0] + Fm[3 * r + 1] * es[1] + Fm[3 * r + 2] * es[2];
            }
            double I4sh = Fs[0] * Fs[0] + Fs[1] * Fs[1] + Fs[2] * Fs[2];
            double I4shs = I4sh > 1.0 ? I4sh : 1.0;
            double Es = exp(bs * (I4shs - 1.0) * (I4shs - 1.0));
            sh_coef = 2.0 * as * (I4shs - 1.0) * Es;
            if (as != 0.0) energy += as / (2.0 * bs) * (Es - 1.0);
            double I8 = Fe[0] * Fs[0] + Fe[1] * Fs[1] + Fe[2] * Fs[2];
            double Efs = exp(bfs * I8 * I8);
            fs_coef = afs * I8 * Efs;
            if (afs != 0.0) energy += afs / (2.0 * bfs) * (Efs - 1.0);
        }
        if (Ta != 0.0) {
            double r4 = sqrt(I4);
            fib_coef += Ta * (1.0 + 4.9 * (r4 - 1.0));
            energy += 0.5 * Ta * ((1.0 - 4.9) * (I4 - 1.0) + (2.0 / 3.0) * 4.9 * (I4 * r4 - 1.0));
        }
    } else if (model == IBREF_STANDARD_REINFORCING) {
        double GT = par[0], GL = par[1], EL = par[2];
        kappa = par[3];
        /* C e_f = F^T (F e_f), I5f = |C e_f|^2, and F C e_f */
        for (int c = 0; c < 3; ++c) Ce[c] = Fm[c] * Fe[0] + Fm[3 + c] * Fe[1] + Fm[6 + c] * Fe[2];
        for (int r = 0; r < 3; ++r) FCe[r] = Fm[3 * r] * Ce[0] + Fm[3 * r + 1] * Ce[1] + Fm[3 * r + 2] * Ce[2];
        double I5 = Ce[0] * Ce[0] + Ce[1] * Ce[1] + Ce[2] * Ce[2];
        double cL = EL + GT - 4.0 * GL;
        iso_coef = GT;
        energy = 0.5 * GT * (Jm23 * I1 - 3.0) + 0.5 * (GT - GL) * (2.0 * I4 - I5 - 1.0) +
                 cL / 8.0 * (I4 - 1.0) * (I4 - 1.0);
        fib_coef = 2.0 * (GT - GL) + 0.5 * cL * (I4 - 1.0);
        i5_coef = -(GT - GL);
    } else if (model == IBREF_FIBRE_REINFORCED_1) {
        double C1 = par[0], af = par[1], bf = par[2];
        kappa = par[3];
        iso_coef = 2.0 * C1;
        energy = C1 * (Jm23 * I1 - 3.0);
        double I4s = I4 > 1.0 ? I4 : 1.0;
        double Ef = exp(bf * (I4s - 1.0) * (I4s - 1.0));
        fib_coef = 2.0 * af * (I4s - 1.0) * Ef;
        if (af != 0.0) energy += af / (2.0 * bf) * (Ef - 1.0);
    } else if (model == IBREF_FIBRE_REINFORCED_2) {
        double C10 = par[0], C01 = par[1], af = par[2], bf = par[3];
        kappa = par[4];
        double E1 = exp(C01 * (Jm23 * I1 - 3.0));
        iso_coef = 2.0 * C10 * C01 * E1;
        energy = C10 * (E1 - 1.0);
        double Ef = exp(bf * (I4 - 1.0) * (I4 - 1.0));
        fib_coef = 2.0 * af * (I4 - 1.0) * Ef;
        if (af != 0.0) energy += af / (2.0 * bf) * (Ef - 1.0);
    } else {
        return IBREF_E_INVAL;
    }
    energy += 0.5 * kappa * lnJ * lnJ;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            P[3 * r + c] = iso_coef * Jm23 * (Fm[3 * r + c] - I1 / 3.0 * FiT[3 * r + c]) +
                           fib_coef * Fe[r] * ef[c] + sh_coef * Fs[r] * esv[c] +
                           fs_coef * (Fe[r] * esv[c] + Fs[r] * ef[c]) +
                           i5_coef * (Fe[r] * Ce[c] + FCe[r] * ef[c]) +
                           kappa * lnJ * FiT[3 * r + c];
    if (psi) *psi = energy;
    return IBREF_OK;
}

/*
 * Active tension waveform of the left-ventricle model: T_a = ta_max (1 -
 * exp(-(s - 0.5)^2 / 0.005)) for 0.5 < s < 0.65, ta_max (1 - exp(-(0.8 - s)^2 /
 * 0.005)) for 0.65 <= s < 0.8 (both branches agree at 0.65), 0 otherwise, in
 * the model's time s (seconds).  Here s = 0.5 + 0.3 (t - t_on) / duration maps
 * the active window onto [t_on, t_on + duration] of the simulation clock.
 */
double ibref_active_tension(double ta_max, double t_on, double duration, double t) {
    if (ta_max == 0.0 || !(duration > 0.0)) return 0.0;
    double s = 0.5 + 0.3 * (t - t_on) / duration;
    if (s > 0.5 && s < 0.65) return ta_max * (1.0 - exp(-(s - 0.5) * (s - 0.5) / 0.005));
    if (s >= 0.65 && s < 0.8) return ta_max * (1.0 - exp(-(0.8 - s) * (0.8 - s) / 0.005));
    return 0.0;
}

/* ------------------------------------------------------------------------- */
/* matrix-free nodal forces                                                  */
/* ------------------------------------------------------------------------- */

/* trilinear hex: local node a = i + 2j + 4k at reference (2i-1, 2j-1, 2k-1) */
static void hex_dshape(const double xi[3], double dN[][3]) {
    for (int a = 0; a < 8; ++a) {
        double s0 = (a & 1) ? 1.0 : -1.0, s1 = (a & 2) ? 1.0 : -1.0, s2 = (a & 4) ? 1.0 : -1.0;
        double f0 = 1.0 + s0 * xi[0], f1 = 1.0 + s1 * xi[1], f2 = 1.0 + s2 * xi[2];
        dN[a][0] = s0 * f1 * f2 / 8.0;
        dN[a][1] = f0 * s1 * f2 / 8.0;
        dN[a][2] = f0 * f1 * s2 / 8.0;
    }
}

/*
 * Tetrahedra on the reference simplex xi, eta, zeta >= 0, xi + eta + zeta <= 1
 * with barycentric l0 = 1 - xi - eta - zeta, l1 = xi, l2 = eta, l3 = zeta:
 *   P1 (4 nodes): N_a = l_a;
 *   P2 (10 nodes): vertices N_a = l_a (2 l_a - 1) (a < 4), edge nodes
 *   N = 4 l_i l_j for (i, j) = (0,1), (1,2), (0,2), (0,3), (1,3), (2,3) (nodes 4..9).
 */
static const int tet_edge[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};

static void tet_dshape(int npe, const double l[4], double dN[][3]) {
    static const double gl[4][3] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int a = 0; a < 4; ++a)
        for (int k = 0; k < 3; ++k) dN[a][k] = npe == 4 ? gl[a][k] : (4.0 * l[a] - 1.0) * gl[a][k];
    if (npe == 10)
        for (int t = 0; t < 6; ++t) {
            int i = tet_edge[t][0], j = tet_edge[t][1];
            for (int k = 0; k < 3; ++k) dN[4 + t][k] = 4.0 * (l[j] * gl[i][k] + l[i] * gl[j][k]);
        }
}

/* quadrature points of each element type */
static int elem_nq(int npe) { return npe == 8 ? 8 : (npe == 4 ? 1 : 4); }

/*
 * Element rule H_q (left unspecified by the paper): hexes 2x2x2 Gauss points at
 * +-1/sqrt(3) with unit weights; P1 tets one point at the centroid (exact: the
 * deformation gradient is constant) with weight 1/6; P2 tets the symmetric
 * 4-point rule of degree 2, barycentric (a, b, b, b) and permutations with
 * a = (5 + 3 sqrt 5)/20, b = (5 - sqrt 5)/20, weights 1/24.  Returns the
 * shape-function derivatives at point g and its weight on the reference cell.
 */
static double elem_rule(int npe, int g, double dN[][3]) {
    if (npe == 8) {
        const double gp = 1.0 / sqrt(3.0);
        double xi[3] = {(g & 1) ? gp : -gp, (g & 2) ? gp : -gp, (g & 4) ? gp : -gp};
        hex_dshape(xi, dN);
        return 1.0;
    }
    double l[4];
    if (npe == 4) {
        for (int a = 0; a < 4; ++a) l[a] = 0.25;
        tet_dshape(4, l, dN);
        return 1.0 / 6.0;
    }
    const double qa = (5.0 + 3.0 * sqrt(5.0)) / 20.0, qb = (5.0 - sqrt(5.0)) / 20.0;
    for (int a = 0; a < 4; ++a) l[a] = a == g ? qa : qb;
    tet_dshape(10, l, dN);
    return 1.0 / 24.0;
}

static int mesh_npe(const ibref_mesh* m) { return m->nodes_per_elem ? m->nodes_per_elem : 8; }

/*
 * Penalty tethers (the constrained faces of the benchmark and valve models and
 * the base constraint of the left-ventricle model are enforced with a penalty
 * parameter; the force law is not printed): a linear spring on each tethered
 * node, F_a += -K (X_a - Y) with a symmetric K, energy (1/2)(X_a - Y).K(X_a - Y).
 * With hvp set, V takes the place of X - Y (the force derivative along V).
 */
static int tether_apply(const ibref_mesh* m, const double* x, const double* V, double* F,
                        double* energy) {
    double E = 0.0;
    for (int t = 0; t < m->n_tethers; ++t)
        if (m->tether_node[t] < 0 || m->tether_node[t] >= m->n_nodes) return IBREF_E_INVAL;
    for (int t = 0; t < m->n_tethers; ++t) {
        long a = m->tether_node[t];
        const double* K = m->tether_K + 6L * t;
        double Km[3][3] = {{K[0], K[3], K[4]}, {K[3], K[1], K[5]}, {K[4], K[5], K[2]}};
        double d[3];
        for (int r = 0; r < 3; ++r) d[r] = V ? V[3 * a + r] : x[3 * a + r] - m->tether_target[3L * t + r];
        for (int r = 0; r < 3; ++r) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += Km[r][c] * d[c];
            F[3 * a + r] -= s;
            E += 0.5 * d[r] * s;
        }
    }
    if (energy) *energy += E;
    return IBREF_OK;
}

/*
 * Nodal force from the weak form ("Spatial Discretization" and the mean force
 * contribution formula of the coupling section):
 *   F_a = - sum_e sum_g P(F_g) : grad_X N_a(g) w_g
 * with the element rules of elem_rule (trilinear hexes, P1 or P2 tetrahedra),
 * w_g = det(dX/dxi) at the point times the rule's weight.
 * F_g = sum_a x_a (x) grad_X N_a(g).  Also returns E = sum_e sum_g Psi w_g and
 * the smallest J.  F is overwritten.
 */
int ibref_fe_force(const ibref_mesh* m, const double* x, double* F, double* energy,
                   double* min_J) {
    const int npe = mesh_npe(m);
    if (npe != 8 && npe != 4 && npe != 10) return IBREF_E_INVAL;
    double E = 0.0, Jmin = INFINITY;
    for (long r = 0; r < 3L * m->n_nodes; ++r) F[r] = 0.0;
    for (int e = 0; e < m->n_elems; ++e) {
        const int32_t* cn = m->conn + (long)npe * e;
        int mid = m->mat_id[e];
        if (mid < 0 || mid >= m->n_mats) return IBREF_E_INVAL;
        const double* par = m->mat_params + (long)IBREF_MAT_PARAMS * mid;
        int model = m->mat_model[mid];
        const double* ef = m->fibre + 3L * e;
        const double* es = m->sheet ? m->sheet + 3L * e : NULL;
        double Xe[10][3], xe[10][3], Fe[10][3];
        for (int a = 0; a < npe; ++a) {
            if (cn[a] < 0 || cn[a] >= m->n_nodes) return IBREF_E_INVAL;
            for (int r = 0; r < 3; ++r) {
                Xe[a][r] = m->X_ref[3L * cn[a] + r];
                xe[a][r] = x[3L * cn[a] + r];
                Fe[a][r] = 0.0;
            }
        }
        for (int g = 0; g < elem_nq(npe); ++g) {
            double dN[10][3];
            const double wq = elem_rule(npe, g, dN);
            double J0[9] = {0};
            for (int a = 0; a < npe; ++a)
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) J0[3 * r + c] += Xe[a][r] * dN[a][c];
            double w = det3(J0);
            if (!(w > 0.0)) return IBREF_E_NUMERIC;
            double cof[9], J0inv[9];
            cof3(J0, cof); /* cof = w J0^{-T}  ->  J0^{-1}[r][c] = cof[c][r] / w */
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) J0inv[3 * r + c] = cof[3 * c + r] / w;
            const double wg = w * wq;   /* quadrature weight in the reference configuration */
            double gN[10][3];
            for (int a = 0; a < npe; ++a)
                for (int c = 0; c < 3; ++c) {
                    double s = 0.0;
                    for (int r = 0; r < 3; ++r) s += dN[a][r] * J0inv[3 * r + c];
                    gN[a][c] = s;
                }
            double Fm[9] = {0};
            for (int a = 0; a < npe; ++a)
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) Fm[3 * r + c] += xe[a][r] * gN[a][c];
            double J = det3(Fm);
            if (J < Jmin) Jmin = J;
            double P[9], psi;
            int rc = ibref_pk1(model, par, Fm, ef, es, m->active_tension, P, &psi);
            if (rc) return rc;
            E += psi * wg;
            for (int a = 0; a < npe; ++a)
                for (int r = 0; r < 3; ++r) {
                    double s = 0.0;
                    for (int c = 0; c < 3; ++c) s += P[3 * r + c] * gN[a][c];
                    Fe[a][r] -= s * wg;
                }
        }
        for (int a = 0; a < npe; ++a)
            for (int r = 0; r < 3; ++r) F[3L * cn[a] + r] += Fe[a][r];
    }
    int rc = tether_apply(m, x, NULL, F, &E);
    if (rc) return rc;
    if (energy) *energy = E;
    if (min_J) *min_J = Jmin;
    return IBREF_OK;
}

/*
 * Uniform pressure on a surface (the left-ventricle model loads its
 * endocardium with a spatially uniform pressure), as a follower load on the
 * current configuration:
 *   F_a += -p * integral over the quad of N_a (dx/dxi x dx/deta) dxi deta
 * with 2x2 Gauss points (exact for the bilinear integrand).  The quads are
 * oriented so dx/dxi x dx/deta points out of the solid into the cavity; the
 * load therefore pushes the wall away from the cavity.
 */
void ibref_pressure_load(int32_t n_faces, const int32_t* faces, const double* x, double p,
                         double* F) {
    const double gp = 1.0 / sqrt(3.0);
    for (int f = 0; f < n_faces; ++f) {
        const int32_t* fn = faces + 4L * f;
        for (int g = 0; g < 4; ++g) {
            double s = (g & 1) ? gp : -gp, t = (g & 2) ? gp : -gp;
            double N[4], dNs[4], dNt[4];
            for (int a = 0; a < 4; ++a) {
                double sa = (a & 1) ? 1.0 : -1.0, ta = (a & 2) ? 1.0 : -1.0;
                N[a] = (1.0 + sa * s) * (1.0 + ta * t) / 4.0;
                dNs[a] = sa * (1.0 + ta * t) / 4.0;
                dNt[a] = (1.0 + sa * s) * ta / 4.0;
            }
            double xs[3] = {0, 0, 0}, xt[3] = {0, 0, 0};
            for (int a = 0; a < 4; ++a)
                for (int r = 0; r < 3; ++r) {
                    xs[r] += x[3L * fn[a] + r] * dNs[a];
                    xt[r] += x[3L * fn[a] + r] * dNt[a];
                }
            double nA[3] = {xs[1] * xt[2] - xs[2] * xt[1], xs[2] * xt[0] - xs[0] * xt[2],
                            xs[0] * xt[1] - xs[1] * xt[0]};
            for (int a = 0; a < 4; ++a)
                for (int r = 0; r < 3; ++r) F[3L * fn[a] + r] -= p * N[a] * nA[r];
        }
    }
}

/* ------------------------------------------------------------------------- */
/* geometric multigrid for (sigma I - nu Lap_h) x = b, periodic              */
/* ------------------------------------------------------------------------- */
/*
 * The paper names a geometric multigrid solver but gives no details; the
 * algorithm below is this implementation's reading (cell-centred, symmetric):
 *   V(pre, post) cycle; in-place red-black Gauss-Seidel, red = (i+j+k) even;
 *   pre-smoothing red then black, post-smoothing black then red;
 *   restriction: per axis weights (1,3,3,1)/8 over fine cells 2I-1 .. 2I+2;
 *   prolongation: cell-centred trilinear (3/4, 1/4 per axis), added to x;
 *   coarse operators rediscretised at 2h; the coarsest level is the first
 *   with at most 32 cells per side, solved exactly (mg_coarse_sweeps = 0: the
 *   periodic operator is diagonalised by the discrete Fourier modes, with
 *   eigenvalues sigma + nu (4/h^2) sum_d sin^2(pi k_d / n); Poisson drops the
 *   k = 0 mode), or the first with fewer than 8 cells, solved by
 *   mg_coarse_sweeps red+black sweeps (mg_coarse_sweeps > 0);
 *   Poisson (sigma = 0): the mean is removed after the coarse solve
 *   and once from the final solution (the residual and the sweeps are
 *   invariant to adding a constant, so the iterates need no mean removal).
 * The Helmholtz operator (sigma > 0): on a level of spacing h its Jacobi
 * iteration matrix has spectral radius rho = 6c / (sigma + 6c), c = nu / h^2
 * (the constant mode; the periodic operator is symmetric with a constant
 * diagonal, so the Jacobi eigenvalues are real in [-rho, rho]), and red-black
 * ordering is consistently ordered, so over-relaxation by Young's factor
 * omega = 2 / (1 + sqrt(1 - rho^2)) contracts every error component by
 * omega - 1 per red+black sweep.  Where rho <= 1/2 (sigma >= 6 nu / h^2) that
 * is at most 0.072 per sweep, and a coarse-grid correction adds nothing (a
 * two-level cycle contracts less per sweep than the sweeps alone).  So the
 * Helmholtz hierarchy stops at the first level l >= 0 with rho_l <= 1/2 (or
 * at the coarsest), and that level is relaxed by red+black sweeps
 * over-relaxed by its omega_l:
 *   l = 0: the cycle is mg_pre + mg_post sweeps on the current iterate, each
 *     red then black (one ordering throughout: reversing it, as the V-cycle's
 *     post-smoothing does, repeats a colour and loses the SOR rate);
 *   0 < l < coarsest: max(mg_pre, 1) sweeps (red, black) from zero;
 *   the coarsest: its exact solve, or mg_coarse_sweeps sweeps from zero.
 * The other Helmholtz levels and every Poisson level keep plain Gauss-Seidel
 * (omega = 1).
 * Stop rule: ||b - A x||_2 <= max(rtol, 1e3 eps) ||b||_2, tested before the
 * first cycle and after every cycle; ||b|| = 0 gives x = 0.
 */

/* one colour of red-black Gauss-Seidel, over-relaxed by omega when omega != 1:
 * x <- x + omega ((b + c * neighbour sum) / diag - x) */
static void gs_colour(int n, double sigma, double nu, const double* b, double* x, int colour,
                      double omega) {
    const double h = 1.0 / n, c = nu / (h * h), diag = sigma + 6.0 * c;
#pragma omp parallel for
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = ((j + k + colour) & 1); i < n; i += 2) {
                double s = x[gidx(i + 1, j, k, n)] + x[gidx(i - 1, j, k, n)] +
                           x[gidx(i, j + 1, k, n)] + x[gidx(i, j - 1, k, n)] +
                           x[gidx(i, j, k + 1, n)] + x[gidx(i, j, k - 1, n)];
                const double xg = (b[gidx(i, j, k, n)] + c * s) / diag;
                if (omega == 1.0) {
                    x[gidx(i, j, k, n)] = xg;
                } else {
                    const double xo = x[gidx(i, j, k, n)];
                    x[gidx(i, j, k, n)] = xo + omega * (xg - xo);
                }
            }
}

/* Young's over-relaxation factor of a Helmholtz level (1 for Poisson) */
static double level_omega(int n, double sigma, double nu) {
    if (!(sigma > 0.0)) return 1.0;
    const double h = 1.0 / n, c = nu / (h * h);
    const double rho = 6.0 * c / (sigma + 6.0 * c);
    return 2.0 / (1.0 + sqrt(1.0 - rho * rho));
}

/* r = b - (sigma x - nu Lap_h x) */
static void residual(int n, double sigma, double nu, const double* b, const double* x, double* r) {
    const double h = 1.0 / n, c = nu / (h * h);
#pragma omp parallel for
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double xc = x[gidx(i, j, k, n)];
                double s = x[gidx(i + 1, j, k, n)] + x[gidx(i - 1, j, k, n)] +
                           x[gidx(i, j + 1, k, n)] + x[gidx(i, j - 1, k, n)] +
                           x[gidx(i, j, k + 1, n)] + x[gidx(i, j, k - 1, n)];
                double Ax = sigma * xc - c * (s - 6.0 * xc);
                r[gidx(i, j, k, n)] = b[gidx(i, j, k, n)] - Ax;
            }
}

static double norm2(long N, const double* v) {
    double s = 0.0;
    for (long i = 0; i < N; ++i) s += v[i] * v[i];
    return sqrt(s);
}
static void remove_mean(long N, double* v) {
    double s = 0.0;
    for (long i = 0; i < N; ++i) s += v[i];
    double m = s / (double)N;
    for (long i = 0; i < N; ++i) v[i] -= m;
}

/* coarse[I,J,K] = sum of (w_a w_b w_c / 512) fine[2I-1+a, 2J-1+b, 2K-1+c], w = 1,3,3,1 */
static void restrict_fw(int nf, const double* fine, double* coarse) {
    const int nc = nf / 2;
    static const double w[4] = {1.0, 3.0, 3.0, 1.0};
#pragma omp parallel for
    for (int K = 0; K < nc; ++K)
        for (int J = 0; J < nc; ++J)
            for (int I = 0; I < nc; ++I) {
                double s = 0.0;
                for (int c = 0; c < 4; ++c)
                    for (int b = 0; b < 4; ++b)
                        for (int a = 0; a < 4; ++a)
                            s += w[a] * w[b] * w[c] / 512.0 *
                                 fine[gidx(2 * I - 1 + a, 2 * J - 1 + b, 2 * K - 1 + c, nf)];
                coarse[gidx(I, J, K, nc)] = s;
            }
}

/* fine[i] += trilinear interpolation of coarse; fine cell i = 2I + s takes
 * 3/4 of coarse I and 1/4 of coarse I-1 (s = 0) or I+1 (s = 1), per axis. */
static void prolong_add(int nf, const double* coarse, double* fine) {
    const int nc = nf / 2;
#pragma omp parallel for
    for (int k = 0; k < nf; ++k)
        for (int j = 0; j < nf; ++j)
            for (int i = 0; i < nf; ++i) {
                int ijk[3] = {i, j, k};
                int base[3][2];
                double wt[3][2];
                for (int d = 0; d < 3; ++d) {
                    int I = ijk[d] >> 1, s = ijk[d] & 1;
                    base[d][0] = I;
                    wt[d][0] = 0.75;
                    base[d][1] = s ? I + 1 : I - 1;
                    wt[d][1] = 0.25;
                }
                double v = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a)
                            v += wt[0][a] * wt[1][b] * wt[2][c] *
                                 coarse[gidx(base[0][a], base[1][b], base[2][c], nc)];
                fine[gidx(i, j, k, nf)] += v;
            }
}

typedef struct {
    int L;            /* number of levels */
    int n[32];
    double* x[32];
    double* b[32];
    double* r[32];
} mg_levels;

static int mg_alloc(int n, mg_levels* lv) {
    memset(lv, 0, sizeof(*lv));
    int m = n, L = 0;
    while (1) {
        if (m % 2) return IBREF_E_INVAL; /* red-black colouring needs even sizes */
        lv->n[L] = m;
        long N3 = (long)m * m * m;
        lv->x[L] = (double*)calloc((size_t)N3, sizeof(double));
        lv->b[L] = (double*)calloc((size_t)N3, sizeof(double));
        lv->r[L] = (double*)calloc((size_t)N3, sizeof(double));
        ++L;
        lv->L = L;
        if (m < 8) break;
        m /= 2;
    }
    lv->L = L;
    return IBREF_OK;
}
static void mg_free(mg_levels* lv) {
    for (int l = 0; l < lv->L; ++l) { free(lv->x[l]); free(lv->b[l]); free(lv->r[l]); }
}

/* the coarsest level of the hierarchy (see above) */
static int hierarchy_bottom(const ibref_fluid* fl, const mg_levels* lv) {
    if (fl->mg_coarse_sweeps > 0) return lv->L - 1;
    for (int l = 0; l < lv->L; ++l)
        if (lv->n[l] <= 32) return l;
    return lv->L - 1;
}

/* the level at which the cycle stops descending (see above) */
static int coarsest_level(const ibref_fluid* fl, const mg_levels* lv, double sigma, double nu) {
    const int bottom = hierarchy_bottom(fl, lv);
    if (sigma > 0.0)
        for (int l = 0; l < bottom; ++l) {
            const double h = 1.0 / lv->n[l];
            if (sigma >= 6.0 * nu / (h * h)) return l;
        }
    return bottom;
}

/* Exact solve of (sigma - nu Lap_h) x = b on the periodic n^3 grid by its
 * discrete Fourier diagonalisation: bhat = F b (F_kj = e^{-2 pi i k.j / n},
 * one axis after another), xhat = bhat / lambda_k with
 * lambda_k = sigma + nu (4/h^2) sum_d sin^2(pi k_d / n), x = Re F^{-1} xhat;
 * for Poisson (sigma = 0) the k = 0 mode (lambda = 0) is dropped, so x has zero
 * mean.  Plain O(n^4) transforms. */
static void coarse_exact(int n, double sigma, double nu, const double* b, double* x) {
    const double pi = 3.14159265358979323846;
    const long N3 = (long)n * n * n;
    double* re = (double*)malloc(sizeof(double) * (size_t)N3);
    double* im = (double*)malloc(sizeof(double) * (size_t)N3);
    /* e^{2 pi i m / n}, m = 0 .. n-1: the exponent k j only matters mod n */
    double* cw = (double*)malloc(sizeof(double) * (size_t)n);
    double* sw = (double*)malloc(sizeof(double) * (size_t)n);
    for (int m = 0; m < n; ++m) {
        cw[m] = cos(2.0 * pi * (double)m / n);
        sw[m] = sin(2.0 * pi * (double)m / n);
    }
    for (long t = 0; t < N3; ++t) { re[t] = b[t]; im[t] = 0.0; }
    for (int dir = -1; dir <= 1; dir += 2) {          /* forward, then inverse */
        for (int ax = 0; ax < 3; ++ax) {
            const long stride = ax == 0 ? 1 : (ax == 1 ? n : (long)n * n);
#pragma omp parallel
            {
                double* tr = (double*)malloc(sizeof(double) * (size_t)n);
                double* ti = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp for
                for (long line = 0; line < (long)n * n; ++line) {
                    /* first cell of the line: the other two indices from `line` */
                    const long a = line % n, c = line / n;
                    long base;
                    if (ax == 0) base = n * (a + (long)n * c);
                    else if (ax == 1) base = a + (long)n * n * c;
                    else base = a + (long)n * c;
                    for (int k = 0; k < n; ++k) {
                        double sr = 0.0, si = 0.0;
                        for (int j = 0; j < n; ++j) {
                            const int m = (int)((long)k * j % n);
                            const double cr = cw[m], ci = dir * sw[m];
                            const double vr = re[base + j * stride], vi = im[base + j * stride];
                            sr += vr * cr - vi * ci;
                            si += vr * ci + vi * cr;
                        }
                        tr[k] = sr;
                        ti[k] = si;
                    }
                    for (int k = 0; k < n; ++k) { re[base + k * stride] = tr[k]; im[base + k * stride] = ti[k]; }
                }
                free(tr);
                free(ti);
            }
        }
        if (dir == -1) {
            const double h = 1.0 / n;
            for (int k3 = 0; k3 < n; ++k3)
                for (int k2 = 0; k2 < n; ++k2)
                    for (int k1 = 0; k1 < n; ++k1) {
                        const double s1 = sin(pi * k1 / n), s2 = sin(pi * k2 / n), s3 = sin(pi * k3 / n);
                        const double lam = sigma + nu * (4.0 / (h * h)) * (s1 * s1 + s2 * s2 + s3 * s3);
                        const long t = gidx(k1, k2, k3, n);
                        if (lam == 0.0) { re[t] = 0.0; im[t] = 0.0; }
                        else { re[t] /= lam * (double)N3; im[t] /= lam * (double)N3; }
                    }
        }
    }
    for (long t = 0; t < N3; ++t) x[t] = re[t];
    free(re); free(im); free(cw); free(sw);
}

static void vcycle(const ibref_fluid* fl, mg_levels* lv, int l, double sigma, double nu,
                   int poisson, const double* b, double* x) {
    int n = lv->n[l];
    long N3 = (long)n * n * n;
    const int bottom = hierarchy_bottom(fl, lv);
    const int lc = coarsest_level(fl, lv, sigma, nu);
    if (l == lc && lc == bottom && fl->mg_coarse_sweeps == 0) {
        coarse_exact(n, sigma, nu, b, x);
        if (poisson) remove_mean(N3, x);
        return;
    }
    if (l == lc) {
        const double w = level_omega(n, sigma, nu);
        if (l == 0 && lc < bottom) {
            for (int s = 0; s < fl->mg_pre + fl->mg_post; ++s) {
                gs_colour(n, sigma, nu, b, x, 0, w);
                gs_colour(n, sigma, nu, b, x, 1, w);
            }
            return;
        }
        const int sweeps = lc == bottom ? fl->mg_coarse_sweeps : (fl->mg_pre > 1 ? fl->mg_pre : 1);
        for (int s = 0; s < sweeps; ++s) {
            gs_colour(n, sigma, nu, b, x, 0, w);
            gs_colour(n, sigma, nu, b, x, 1, w);
        }
        if (poisson) remove_mean(N3, x);
        return;
    }
    for (int s = 0; s < fl->mg_pre; ++s) {
        gs_colour(n, sigma, nu, b, x, 0, 1.0);
        gs_colour(n, sigma, nu, b, x, 1, 1.0);
    }
    residual(n, sigma, nu, b, x, lv->r[l]);
    restrict_fw(n, lv->r[l], lv->b[l + 1]);
    int nc = lv->n[l + 1];
    memset(lv->x[l + 1], 0, sizeof(double) * (size_t)nc * nc * nc);
    vcycle(fl, lv, l + 1, sigma, nu, poisson, lv->b[l + 1], lv->x[l + 1]);
    prolong_add(n, lv->x[l + 1], x);
    for (int s = 0; s < fl->mg_post; ++s) {
        gs_colour(n, sigma, nu, b, x, 1, 1.0);
        gs_colour(n, sigma, nu, b, x, 0, 1.0);
    }
}

static double dot(long N, const double* a, const double* b) {
    double s = 0.0;
    for (long i = 0; i < N; ++i) s += a[i] * b[i];
    return s;
}

/* q = A p = sigma p - nu Lap_h p, written through the residual of a zero
 * right-hand side so the stencil is the smoother's */
static void apply_op(int n, double sigma, double nu, const double* p, double* zero, double* q) {
    const long N3 = (long)n * n * n;
    residual(n, sigma, nu, zero, p, q);
    for (long i = 0; i < N3; ++i) q[i] = -q[i];
}

/*
 * The "combined" multigrid reading for the Poisson equation (the paper names
 * a combined geometric multigrid solver and gives no algorithm): conjugate
 * gradients on A x = b preconditioned with z = M r, one V-cycle from a zero
 * guess.  The search direction uses the flexible (Polak-Ribiere) update, which
 * tolerates a preconditioner that is not exactly symmetric or linear:
 *   r = b - A x, z = M r, p = z, rz = r.z
 *   repeat:  q = A p,  alpha = rz / (p.q),  x += alpha p,  r -= alpha q,
 *            stop test on ||r|| (as the plain iteration, one iteration = one cycle),
 *            z = M r,  beta = z.(r_new - r_old) / rz = -alpha (z.q) / rz,
 *            rz = r.z,  p = z + beta p
 */
static int pcg_solve(const ibref_fluid* fl, mg_levels* lv, double sigma, double nu,
                     const double* b, double* x, double bn, int* kout, double* rnout) {
    const int n = fl->n;
    const long N3 = (long)n * n * n;
    double* r = (double*)malloc(sizeof(double) * (size_t)N3);
    double* z = (double*)malloc(sizeof(double) * (size_t)N3);
    double* p = (double*)malloc(sizeof(double) * (size_t)N3);
    double* q = (double*)malloc(sizeof(double) * (size_t)N3);
    double* zero = (double*)calloc((size_t)N3, sizeof(double));
    int rc = IBREF_OK, k = 0;
    if (!r || !z || !p || !q || !zero) rc = IBREF_E_INVAL;
    double tol = (fl->mg_rtol > 1e3 * DBL_EPSILON ? fl->mg_rtol : 1e3 * DBL_EPSILON) * bn;
    double rn = 0.0, rz = 0.0, alpha = 0.0;
    if (!rc) {
        residual(n, sigma, nu, b, x, r);
        rn = norm2(N3, r);
    }
    while (!rc) {
        if (!isfinite(rn)) { rc = IBREF_E_NUMERIC; break; }
        if (fl->mg_fixed_cycles > 0) {
            if (k == fl->mg_fixed_cycles) break;
        } else {
            if (rn <= tol) break;
            if (k == fl->mg_max_cycles) { rc = IBREF_E_NOCONV; break; }
        }
        memset(z, 0, sizeof(double) * (size_t)N3);
        vcycle(fl, lv, 0, sigma, nu, 1, r, z);
        if (k == 0) {
            rz = dot(N3, r, z);
            memcpy(p, z, sizeof(double) * (size_t)N3);
        } else {
            /* q and alpha are still those of the previous iteration */
            double beta = -alpha * dot(N3, z, q) / rz;
            rz = dot(N3, r, z);
            for (long i = 0; i < N3; ++i) p[i] = z[i] + beta * p[i];
        }
        apply_op(n, sigma, nu, p, zero, q);
        alpha = rz / dot(N3, p, q);
        for (long i = 0; i < N3; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        ++k;
        rn = norm2(N3, r);
    }
    free(r); free(z); free(p); free(q); free(zero);
    *kout = k;
    *rnout = rn;
    return rc;
}

int ibref_mg_solve(const ibref_fluid* fl, double sigma, double nu, int32_t poisson,
                   const double* b, double* x, int32_t* cycles, double* relres) {
    const int n = fl->n;
    const long N3 = (long)n * n * n;
    mg_levels lv;
    int rc = mg_alloc(n, &lv);
    if (rc) { mg_free(&lv); return rc; }
    double bn = norm2(N3, b);
    int k = 0;
    double rn = 0.0;
    if (!isfinite(bn)) { mg_free(&lv); return IBREF_E_NUMERIC; }
    if (bn == 0.0) {
        for (long i = 0; i < N3; ++i) x[i] = 0.0;
    } else if (poisson && fl->mg_krylov) {
        rc = pcg_solve(fl, &lv, sigma, nu, b, x, bn, &k, &rn);
        rn /= bn;
        remove_mean(N3, x);
    } else {
        double tol = (fl->mg_rtol > 1e3 * DBL_EPSILON ? fl->mg_rtol : 1e3 * DBL_EPSILON) * bn;
        residual(n, sigma, nu, b, x, lv.r[0]);
        rn = norm2(N3, lv.r[0]);
        while (1) {
            if (!isfinite(rn)) { rc = IBREF_E_NUMERIC; break; }
            if (fl->mg_fixed_cycles > 0) {
                if (k == fl->mg_fixed_cycles) break;
            } else {
                if (rn <= tol) break;
                if (k == fl->mg_max_cycles) { rc = IBREF_E_NOCONV; break; }
            }
            vcycle(fl, &lv, 0, sigma, nu, poisson, b, x);
            ++k;
            residual(n, sigma, nu, b, x, lv.r[0]);
            rn = norm2(N3, lv.r[0]);
        }
        rn /= bn;
        if (poisson) remove_mean(N3, x);
    }
    if (cycles) *cycles = k;
    if (relres) *relres = rn;
    mg_free(&lv);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* time step ("Temporal Discretization", "Spatial Discretization")           */
/* ------------------------------------------------------------------------- */

/*
 * Chorin projection step with explicit convection:
 *   g   = (rho/dt) u^n - rho C(u^n) + f
 *   ((rho/dt) I - mu Lap_h) u* = g               (per component, guess u^n)
 *   Lap_h p = (rho/dt) D u*                      (mean-free, guess p^{n-1})
 *   u^{n+1} = u* - (dt/rho) G p
 * The Poisson equation is solved as (-Lap_h) p = -(rho/dt) D u*, with the
 * discrete mean of the right-hand side removed (periodic null space).
 */
/* ------------------------------------------------------------------------- */
/* walled box through its mirror image                                        */
/* ------------------------------------------------------------------------- */

/*
 * The boundary conditions u* = 0 and u^{n+1}.n = 0 on the box faces, with the
 * MAC ghost-cell convention (tangential ghost = minus the interior value, the
 * wall-normal component stored on the wall faces and held at zero), make the
 * walled operators the restrictions of the periodic ones on the (2n)^3 grid
 * of the box and its mirror images: pressure (Neumann) is mirrored evenly,
 * every velocity component oddly.  On the image grid the spacing is the box's
 * h; the routines below work on the unit-box image grid (spacing h/2), so
 * every derivative carries its factor: Lap_h = Lap_{h/2} / 4, D_h, G_h and the
 * convection C_h are half their h/2 versions, spreading at X/2 is 8 times the
 * box's (delta_h scales as h^-3) and interpolation is unchanged.
 *
 * Index maps of the image grid (per axis, i' in 0..2n-1): a cell-centred
 * axis maps i' >= n to 2n-1-i' (mirrored); the wall-normal axis of a velocity
 * component is face-centred: faces 0 and n are the walls (value 0), i' > n
 * maps to 2n-i' (mirrored).  A mirrored axis contributes a factor -1 for
 * velocity (odd) and +1 for pressure (even).
 */
static int wall_map(int n, int ip, int face, int* src) {
    if (face) {
        if (ip == 0 || ip == n) return 0;        /* wall face */
        if (ip < n) { *src = ip; return 1; }
        *src = 2 * n - ip;
        return -1;
    }
    if (ip < n) { *src = ip; return 1; }
    *src = 2 * n - 1 - ip;
    return -1;
}

void ibref_wall_extend(int32_t n, int32_t vector, const double* box, double* img) {
    const int m = 2 * n;
    const long M3 = (long)m * m * m, N3 = (long)n * n * n;
    for (int d = 0; d < (vector ? 3 : 1); ++d)
        for (int kp = 0; kp < m; ++kp)
            for (int jp = 0; jp < m; ++jp)
                for (int ip = 0; ip < m; ++ip) {
                    int i = 0, j = 0, k = 0;
                    int si = wall_map(n, ip, vector && d == 0, &i);
                    int sj = wall_map(n, jp, vector && d == 1, &j);
                    int sk = wall_map(n, kp, vector && d == 2, &k);
                    double v = 0.0;
                    if (si && sj && sk) {
                        double sg = vector ? (double)(si * sj * sk) : 1.0;
                        v = sg * box[d * N3 + i + (long)n * (j + (long)n * k)];
                    }
                    img[d * M3 + ip + (long)m * (jp + (long)m * kp)] = v;
                }
}

/* the transpose of ibref_wall_extend: each box value collects its images */
static void wall_fold(int32_t n, int vector, const double* img, double* box) {
    const int m = 2 * n;
    const long M3 = (long)m * m * m, N3 = (long)n * n * n;
    const int nc = vector ? 3 : 1;
    for (long r = 0; r < nc * N3; ++r) box[r] = 0.0;
    for (int d = 0; d < nc; ++d)
        for (int kp = 0; kp < m; ++kp)
            for (int jp = 0; jp < m; ++jp)
                for (int ip = 0; ip < m; ++ip) {
                    int i = 0, j = 0, k = 0;
                    int si = wall_map(n, ip, vector && d == 0, &i);
                    int sj = wall_map(n, jp, vector && d == 1, &j);
                    int sk = wall_map(n, kp, vector && d == 2, &k);
                    if (si && sj && sk) {
                        double sg = vector ? (double)(si * sj * sk) : 1.0;
                        box[d * N3 + i + (long)n * (j + (long)n * k)] +=
                            sg * img[d * M3 + ip + (long)m * (jp + (long)m * kp)];
                    }
                }
}

void ibref_wall_fold(int32_t n, const double* img, double* box) { wall_fold(n, 1, img, box); }

/* the transpose of ibref_wall_restrict: the box values in the box part of the
 * image grid (wall faces of velocity zero), zero elsewhere */
void ibref_wall_pad(int32_t n, int32_t vector, const double* box, double* img) {
    const int m = 2 * n;
    const long M3 = (long)m * m * m, N3 = (long)n * n * n;
    const int nc = vector ? 3 : 1;
    for (long r = 0; r < nc * M3; ++r) img[r] = 0.0;
    for (int d = 0; d < nc; ++d)
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    int wall = vector && ((d == 0 && i == 0) || (d == 1 && j == 0) || (d == 2 && k == 0));
                    img[d * M3 + i + (long)m * (j + (long)m * k)] =
                        wall ? 0.0 : box[d * N3 + i + (long)n * (j + (long)n * k)];
                }
}

void ibref_wall_restrict(int32_t n, int32_t vector, const double* img, double* box) {
    const int m = 2 * n;
    const long M3 = (long)m * m * m, N3 = (long)n * n * n;
    for (int d = 0; d < (vector ? 3 : 1); ++d)
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    int wall = vector && ((d == 0 && i == 0) || (d == 1 && j == 0) || (d == 2 && k == 0));
                    box[d * N3 + i + (long)n * (j + (long)n * k)] =
                        wall ? 0.0 : img[d * M3 + i + (long)m * (j + (long)m * k)];
                }
}

void ibref_walled_spread(int32_t n, int32_t n_nodes, const double* X, const double* F, double* f) {
    const long M3 = 8L * n * n * n, N3 = (long)n * n * n;
    double* Xh = (double*)malloc(sizeof(double) * 3 * (size_t)(n_nodes > 0 ? n_nodes : 1));
    double* fi = (double*)calloc(3 * (size_t)M3, sizeof(double));
    double* fb = (double*)malloc(sizeof(double) * 3 * (size_t)N3);
    for (long r = 0; r < 3L * n_nodes; ++r) Xh[r] = 0.5 * X[r];
    ibref_spread(2 * n, n_nodes, Xh, F, fi);
    ibref_wall_fold(n, fi, fb);
    for (long r = 0; r < 3 * N3; ++r) f[r] += 0.125 * fb[r];
    free(Xh); free(fi); free(fb);
}

void ibref_walled_interpolate(int32_t n, int32_t n_nodes, const double* X, const double* u, double* U) {
    const long M3 = 8L * n * n * n;
    double* Xh = (double*)malloc(sizeof(double) * 3 * (size_t)(n_nodes > 0 ? n_nodes : 1));
    double* ui = (double*)malloc(sizeof(double) * 3 * (size_t)M3);
    for (long r = 0; r < 3L * n_nodes; ++r) Xh[r] = 0.5 * X[r];
    ibref_wall_extend(n, 1, u, ui);
    ibref_interpolate(2 * n, n_nodes, Xh, ui, U);
    free(Xh); free(ui);
}

/* the image grid's fluid: 2n cells on the unit box, the Helmholtz viscosity
 * scaled by (h/2 / h)^2 */
static ibref_fluid image_fluid(const ibref_fluid* fl) {
    ibref_fluid f2 = *fl;
    f2.n = 2 * fl->n;
    f2.mu = 0.25 * fl->mu;
    f2.walls = 0;
    return f2;
}

int ibref_walled_solve(const ibref_fluid* fl, double sigma, double nu, int32_t poisson,
                       const double* b, double* x, int32_t* cycles, double* relres) {
    /* one cell-centred scalar field: mirrored evenly for Poisson (Neumann), oddly
     * otherwise (Dirichlet with the ghost value minus the interior one); on the
     * image grid the Helmholtz viscosity is nu/4 and the Poisson right-hand side
     * is 4b for the unit-coefficient operator */
    const int n = fl->n, m = 2 * n;
    const long M3 = (long)m * m * m;
    ibref_fluid f2 = image_fluid(fl);
    double* bi = (double*)malloc(sizeof(double) * (size_t)M3);
    double* xi = (double*)malloc(sizeof(double) * (size_t)M3);
    for (int kp = 0; kp < m; ++kp)
        for (int jp = 0; jp < m; ++jp)
            for (int ip = 0; ip < m; ++ip) {
                int i = 0, j = 0, k = 0;
                int s = wall_map(n, ip, 0, &i) * wall_map(n, jp, 0, &j) * wall_map(n, kp, 0, &k);
                long o = i + (long)n * (j + (long)n * k), oi = ip + (long)m * (jp + (long)m * kp);
                double sg = poisson ? 1.0 : (double)s;
                bi[oi] = sg * (poisson ? 4.0 : 1.0) * b[o];
                xi[oi] = sg * x[o];
            }
    int rc = ibref_mg_solve(&f2, sigma, poisson ? 1.0 : 0.25 * nu, poisson, bi, xi, cycles, relres);
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) x[i + (long)n * (j + (long)n * k)] = xi[i + (long)m * (j + (long)m * k)];
    free(bi); free(xi);
    return rc;
}

/*
 * One fluid step in the walled box (the periodic step's equations with the
 * walls' boundary conditions), on the image grid:
 *   g = (rho/dt) u - rho C_h(u) + f, restricted to the box (wall faces 0) and
 *   mirrored back; Helmholtz on the image grid (viscosity mu/4 there) from the
 *   mirrored u; u* restricted and mirrored; b = -(rho/dt) D_h u* on the box
 *   (times 4 for the image grid's unit-coefficient Poisson operator), mirrored
 *   evenly, mean removed; Poisson from the mirrored p; u = u* - (dt/rho) G_h p;
 *   u and p restricted (the projection leaves the tangential velocity free at
 *   the walls, as u^{n+1}.n = 0 asks).
 */
static int walled_ns_step(const ibref_fluid* fl, const double* f, double* u, double* p,
                          ibref_step_stats* st) {
    const int n = fl->n, m = 2 * n;
    const long M3 = (long)m * m * m;
    const double rho = fl->rho, dt = fl->dt;
    ibref_fluid f2 = image_fluid(fl);
    double* ui = (double*)malloc(sizeof(double) * 3 * (size_t)M3);
    double* fi = (double*)malloc(sizeof(double) * 3 * (size_t)M3);
    double* gi = (double*)malloc(sizeof(double) * 3 * (size_t)M3);
    double* ci = (double*)calloc(3 * (size_t)M3, sizeof(double));
    double* pi = (double*)malloc(sizeof(double) * (size_t)M3);
    double* bi = (double*)malloc(sizeof(double) * (size_t)M3);
    double* box = (double*)malloc(sizeof(double) * 3 * (size_t)fl->n * fl->n * fl->n);
    int rc = IBREF_OK;
    ibref_wall_extend(n, 1, u, ui);
    ibref_wall_extend(n, 1, f, fi);
    ibref_wall_extend(n, 0, p, pi);
    if (fl->convection) ibref_convection(m, ui, ci);
    for (long i = 0; i < 3 * M3; ++i) gi[i] = rho / dt * ui[i] - 0.5 * rho * ci[i] + fi[i];
    ibref_wall_restrict(n, 1, gi, box);
    ibref_wall_extend(n, 1, box, gi);
    for (int d = 0; d < 3 && !rc; ++d) {
        int32_t cyc = 0;
        double rr = 0.0;
        rc = ibref_mg_solve(&f2, rho / dt, f2.mu, 0, gi + d * M3, ui + d * M3, &cyc, &rr);
        if (st) { st->cycles[d] = cyc; st->relres[d] = rr; }
    }
    if (!rc) {
        ibref_wall_restrict(n, 1, ui, box);
        ibref_wall_extend(n, 1, box, ui);
        /* the box divergence (wall faces zero), mirrored evenly: the velocity
         * images are odd in every component (no slip for u*), so the image
         * divergence itself is not even across the walls */
        ibref_divergence(m, ui, bi);
        for (long i = 0; i < M3; ++i) bi[i] = -2.0 * (rho / dt) * bi[i];
        ibref_wall_restrict(n, 0, bi, box);
        ibref_wall_extend(n, 0, box, bi);
        remove_mean(M3, bi);
        int32_t cyc = 0;
        double rr = 0.0;
        rc = ibref_mg_solve(&f2, 0.0, 1.0, 1, bi, pi, &cyc, &rr);
        if (st) { st->cycles[3] = cyc; st->relres[3] = rr; }
    }
    if (!rc) {
        ibref_gradient(m, pi, gi);
        for (long i = 0; i < 3 * M3; ++i) ui[i] = ui[i] - 0.5 * (dt / rho) * gi[i];
        ibref_wall_restrict(n, 1, ui, u);
        ibref_wall_restrict(n, 0, pi, p);
    }
    free(ui); free(fi); free(gi); free(ci); free(pi); free(bi); free(box);
    return rc;
}

int ibref_ns_step(const ibref_fluid* fl, const double* f, double* u, double* p,
                  ibref_step_stats* st) {
    if (fl->walls) return walled_ns_step(fl, f, u, p, st);
    const int n = fl->n;
    const long N3 = (long)n * n * n;
    const double rho = fl->rho, dt = fl->dt, mu = fl->mu;
    double* g = (double*)malloc(sizeof(double) * 3 * (size_t)N3);
    double* c = (double*)calloc(3 * (size_t)N3, sizeof(double));
    double* b = (double*)malloc(sizeof(double) * (size_t)N3);
    double* gp = (double*)malloc(sizeof(double) * 3 * (size_t)N3);
    int rc = IBREF_OK;
    if (fl->convection) ibref_convection(n, u, c);
    for (long i = 0; i < 3 * N3; ++i) g[i] = rho / dt * u[i] - rho * c[i] + f[i];
    for (int d = 0; d < 3 && !rc; ++d) {
        int32_t cyc = 0;
        double rr = 0.0;
        rc = ibref_mg_solve(fl, rho / dt, mu, 0, g + d * N3, u + d * N3, &cyc, &rr);
        if (st) { st->cycles[d] = cyc; st->relres[d] = rr; }
    }
    if (!rc) {
        ibref_divergence(n, u, b);
        for (long i = 0; i < N3; ++i) b[i] = -(rho / dt) * b[i];
        remove_mean(N3, b);
        int32_t cyc = 0;
        double rr = 0.0;
        rc = ibref_mg_solve(fl, 0.0, 1.0, 1, b, p, &cyc, &rr);
        if (st) { st->cycles[3] = cyc; st->relres[3] = rr; }
    }
    if (!rc) {
        ibref_gradient(n, p, gp);
        for (long i = 0; i < 3 * N3; ++i) u[i] = u[i] - dt / rho * gp[i];
    }
    free(g); free(c); free(b); free(gp);
    return rc;
}

/*
 * One immersed-boundary step with explicit coupling:
 *   F = F_el(X^n) + F_pressure(X^n)          (force for the step n -> n+1)
 *   f = S(X^n) F ;  NS step -> u^{n+1}, p^{n+1}
 *   X^{n+1} = X^n + dt J(X^n) u^{n+1}
 * The fully discrete scheme interpolates u^{n+1} (the semi-discrete display
 * writes u^n; the fully discrete statement is followed).
 */
int ibref_ib_step(const ibref_fluid* fl, const ibref_mesh* m, double* u, double* p, double* X,
                  double pressure, ibref_step_stats* st) {
    const int n = fl->n;
    const long N3 = (long)n * n * n;
    double* F = (double*)malloc(sizeof(double) * 3 * (size_t)m->n_nodes);
    double* U = (double*)malloc(sizeof(double) * 3 * (size_t)m->n_nodes);
    double* f = (double*)calloc(3 * (size_t)N3, sizeof(double));
    double E = 0.0, Jmin = 0.0;
    int rc = ibref_fe_force(m, X, F, &E, &Jmin);
    if (!rc) {
        if (m->n_faces > 0 && pressure != 0.0) ibref_pressure_load(m->n_faces, m->faces, X, pressure, F);
        if (fl->walls) ibref_walled_spread(n, m->n_nodes, X, F, f);
        else ibref_spread(n, m->n_nodes, X, F, f);
        rc = ibref_ns_step(fl, f, u, p, st);
    }
    if (!rc) {
        if (fl->walls) ibref_walled_interpolate(n, m->n_nodes, X, u, U);
        else ibref_interpolate(n, m->n_nodes, X, u, U);
        for (long r = 0; r < 3L * m->n_nodes; ++r) X[r] = X[r] + fl->dt * U[r];
    }
    if (st) { st->min_J = Jmin; st->energy = E; }
    free(F); free(U); free(f);
    return rc;
}

/* the solid at time t: the active tension follows the waveform when one is set */
static ibref_mesh mesh_at(const ibref_mesh* m, double t) {
    ibref_mesh ms = *m;
    if (m->ta_max != 0.0) ms.active_tension = ibref_active_tension(m->ta_max, m->ta_t_on, m->ta_duration, t);
    return ms;
}

int ibref_advance(const ibref_fluid* fl, const ibref_mesh* m, double* u, double* p, double* X,
                  double t0, int32_t n_steps, double p0, double T, ibref_step_stats* stats) {
    return ibref_advance_steps(fl, m, u, p, X, t0, 0, n_steps, p0, T, stats);
}

int ibref_advance_steps(const ibref_fluid* fl, const ibref_mesh* m, double* u, double* p, double* X,
                        double t0, int32_t first_step, int32_t n_steps, double p0, double T,
                        ibref_step_stats* stats) {
    const double pi = 3.14159265358979323846;
    for (int s = 0; s < n_steps; ++s) {
        double t = t0 + (first_step + s) * fl->dt;
        double pr = 0.0;
        if (p0 != 0.0 && T > 0.0) {
            double sn = sin(pi * t / T);
            pr = p0 * sn * sn;
        }
        ibref_mesh ms = mesh_at(m, t);
        int rc = ibref_ib_step(fl, &ms, u, p, X, pr, stats ? stats + s : NULL);
        if (rc) return rc;
    }
    return IBREF_OK;
}

/* ------------------------------------------------------------------------- */
/* discrete adjoint                                                          */
/* ------------------------------------------------------------------------- */
/*
 * Reverse mode of the step above, written as the transpose of each linear map
 * and the chain rule through each nonlinear one.  lam denotes dL/d(entry).
 * With Xn+1 = Xn + dt J(Xn) u^{n+1},  u^{n+1} = P H^{-1} g,
 * g = (rho/dt) u^n - rho C(u^n) + S(Xn) F(Xn; theta):
 *   lam_tot = lam_u' + dt J(Xn)^T lam_X'            (J^T = h^3 S)
 *   lam_X   = lam_X' + dt [d_X J(X)u^{n+1}]^T lam_X'
 *   lam_*   = P lam_tot                              (P symmetric)
 *   lam_g   = H^{-1} lam_*                           (H symmetric)
 *   lam_u^n = (rho/dt) lam_g - rho C'(u^n)^T lam_g
 *   lam_F   = S(Xn)^T lam_g = J(Xn) lam_g / h^3
 *   lam_X  += [d_X S(X)F]^T lam_g + (dF/dX)^T lam_F   ((dF_el/dX) is symmetric)
 *   dtheta += (dF/dtheta)^T lam_F
 */

/* reverse of ibref_convection: the same loops with every product differentiated */
void ibref_convection_vjp(int32_t n, const double* u, const double* lam, double* out) {
    const double h = 1.0 / n;
    const long N3 = (long)n * n * n;
    for (long t = 0; t < 3 * N3; ++t) out[t] = 0.0;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                for (int d = 0; d < 3; ++d) {
                    const double* ud = u + d * N3;
                    double* od = out + d * N3;
                    const double lc = lam[d * N3 + gidx(i, j, k, n)] / h;
                    int p[3] = {i, j, k};
                    /* normal flux at c (+) and at c - e_d (-) */
                    for (int sgn = 1; sgn >= -1; sgn -= 2) {
                        int c0[3] = {p[0], p[1], p[2]};
                        if (sgn < 0) c0[d] -= 1;
                        int c1[3] = {c0[0], c0[1], c0[2]};
                        c1[d] += 1;
                        long a0 = gidx(c0[0], c0[1], c0[2], n), a1 = gidx(c1[0], c1[1], c1[2], n);
                        double A = 0.5 * (ud[a0] + ud[a1]);
                        double gA = sgn * 2.0 * A * lc;
                        od[a0] += 0.5 * gA;
                        od[a1] += 0.5 * gA;
                    }
                    for (int e = 0; e < 3; ++e) {
                        if (e == d) continue;
                        const double* ue = u + e * N3;
                        double* oe = out + e * N3;
                        /* edge flux at c + e_e (+) and at c (-) */
                        for (int sgn = 1; sgn >= -1; sgn -= 2) {
                            int cc[3] = {p[0], p[1], p[2]};
                            if (sgn > 0) cc[e] += 1;
                            int me[3] = {cc[0], cc[1], cc[2]};
                            me[e] -= 1;
                            int md[3] = {cc[0], cc[1], cc[2]};
                            md[d] -= 1;
                            long ic = gidx(cc[0], cc[1], cc[2], n);
                            long ime = gidx(me[0], me[1], me[2], n);
                            long imd = gidx(md[0], md[1], md[2], n);
                            double a = 0.5 * (ud[ime] + ud[ic]);
                            double b = 0.5 * (ue[imd] + ue[ic]);
                            double gE = sgn * lc;
                            od[ime] += 0.5 * gE * b;
                            od[ic] += 0.5 * gE * b;
                            oe[imd] += 0.5 * gE * a;
                            oe[ic] += 0.5 * gE * a;
                        }
                    }
                }
}

/* derivative of Peskin's four-point kernel (phi is C^1) */
double ibref_dphi(double r) {
    double a = fabs(r), s = r < 0.0 ? -1.0 : 1.0;
    if (a < 1.0) return s * (-2.0 + (2.0 - 4.0 * a) / sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
    if (a < 2.0) return s * (-2.0 - (6.0 - 4.0 * a) / sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
    return 0.0;
}

static void stencil_1d_d(double r, int* first, double w[4], double dw[4]) {
    int b = (int)floor(r);
    *first = b - 1;
    for (int m = 0; m < 4; ++m) {
        w[m] = ibref_phi(r - (double)(b - 1 + m));
        dw[m] = ibref_dphi(r - (double)(b - 1 + m));
    }
}

/* lamX_q,e += sum_d F^d_q sum_idx lam_f^d[idx] d/dX_e delta_h(x_idx - X_q)
 * with d/dX_e prod phi = phi'(r_e)/h prod_{other} phi */
void ibref_spread_vjp_X(int32_t n, int32_t n_nodes, const double* X, const double* F,
                        const double* lam_f, double* lamX) {
    const double h = 1.0 / n, ih3 = 1.0 / (h * h * h);
    const long N3 = (long)n * n * n;
    for (int q = 0; q < n_nodes; ++q)
        for (int d = 0; d < 3; ++d) {
            int s0[3];
            double w[3][4], dw[3][4];
            for (int e = 0; e < 3; ++e)
                stencil_1d_d(lattice_coord(X[3 * q + e], h, d, e), &s0[e], w[e], dw[e]);
            double g[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < 4; ++c)
                for (int b = 0; b < 4; ++b)
                    for (int a = 0; a < 4; ++a) {
                        double l = lam_f[d * N3 + gidx(s0[0] + a, s0[1] + b, s0[2] + c, n)];
                        g[0] += l * dw[0][a] * w[1][b] * w[2][c];
                        g[1] += l * w[0][a] * dw[1][b] * w[2][c];
                        g[2] += l * w[0][a] * w[1][b] * dw[2][c];
                    }
            for (int e = 0; e < 3; ++e) lamX[3 * q + e] += F[3 * q + d] * ih3 * g[e] / h;
        }
}

/* lamX_q,e += sum_d lamU_q,d sum_idx u^d[idx] d/dX_e (prod phi) */
void ibref_interp_vjp_X(int32_t n, int32_t n_nodes, const double* X, const double* u,
                        const double* lamU, double* lamX) {
    const double h = 1.0 / n;
    const long N3 = (long)n * n * n;
    for (int q = 0; q < n_nodes; ++q)
        for (int d = 0; d < 3; ++d) {
            int s0[3];
            double w[3][4], dw[3][4];
            for (int e = 0; e < 3; ++e)
                stencil_1d_d(lattice_coord(X[3 * q + e], h, d, e), &s0[e], w[e], dw[e]);
            double g[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < 4; ++c)
                for (int b = 0; b < 4; ++b)
                    for (int a = 0; a < 4; ++a) {
                        double v = u[d * N3 + gidx(s0[0] + a, s0[1] + b, s0[2] + c, n)];
                        g[0] += v * dw[0][a] * w[1][b] * w[2][c];
                        g[1] += v * w[0][a] * dw[1][b] * w[2][c];
                        g[2] += v * w[0][a] * w[1][b] * dw[2][c];
                    }
            for (int e = 0; e < 3; ++e) lamX[3 * q + e] += lamU[3 * q + d] * g[e] / h;
        }
}

/*
 * Directional derivative of P (the laws of ibref_pk1) along dF:
 *   d(F^{-T}) = -F^{-T} dF^T F^{-T},  d ln J = F^{-T} : dF,
 *   dI1 = 2 F : dF,  d J^{-2/3} = -(2/3) J^{-2/3} d ln J,  dI4i = 2 (F e_i) . (dF e_i),
 *   dI8fs = (dF e_f) . (F e_s) + (F e_f) . (dF e_s),
 *   iso coefficient alpha = mu_s (NH) or a exp(b (I1bar - 3)) (HO),
 *   fibre / sheet coefficient f_i(I4) = 2 a_i (I4-1) exp(b_i (I4-1)^2) for I4 > 1,
 *   f_i'(I4) = 2 a_i exp(b_i (I4-1)^2) (1 + 2 b_i (I4-1)^2),
 *   fibre-sheet coefficient g(I8) = a_fs I8 exp(b_fs I8^2),
 *   g'(I8) = a_fs exp(b_fs I8^2) (1 + 2 b_fs I8^2),
 *   active coefficient T_a (1 + 4.9 (sqrt(I4f) - 1)), derivative T_a 4.9 / (2 sqrt(I4f));
 *   Psi_1: fibre coefficient 2 (G_T - G_L) + ((E_L + G_T - 4 G_L)/2)(I4f - 1) and the
 *   I5 term c5 ((F e) (x) (C e) + (F C e) (x) e), c5 = -(G_T - G_L), with
 *   d(C e) = dF^T (F e) + F^T (dF e) and d(F C e) = dF (C e) + F d(C e);
 *   Psi_2: iso 2 C_1, fibre as HO; Psi_3: iso 2 C_10 C_01 exp(C_01 (I1bar - 3)) with
 *   derivative C_01 alpha dI1bar, fibre without the max.
 */
int ibref_pk1_tangent(int32_t model, const double* par, const double* Fm, const double* ef,
                      const double* es, double Ta, const double* dFm, double* dP) {
    double J = det3(Fm);
    if (!(J > 0.0)) return IBREF_E_NUMERIC;
    double cof[9], FiT[9], dFiT[9];
    cof3(Fm, cof);
    for (int r = 0; r < 9; ++r) FiT[r] = cof[r] / J;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) s += FiT[3 * r + a] * dFm[3 * b + a] * FiT[3 * b + c];
            dFiT[3 * r + c] = -s;
        }
    double I1 = 0.0, dI1 = 0.0, dlnJ = 0.0;
    for (int r = 0; r < 9; ++r) {
        I1 += Fm[r] * Fm[r];
        dI1 += 2.0 * Fm[r] * dFm[r];
        dlnJ += FiT[r] * dFm[r];
    }
    double Jm23 = pow(J, -2.0 / 3.0), dJm23 = -2.0 / 3.0 * Jm23 * dlnJ;
    double lnJ = log(J);
    double alpha, dalpha, kappa;
    double fib = 0.0, dfib = 0.0, Fe[3] = {0, 0, 0}, dFe[3] = {0, 0, 0};
    double sh = 0.0, dsh = 0.0, Fs[3] = {0, 0, 0}, dFs[3] = {0, 0, 0};
    double fs = 0.0, dfs = 0.0, esv[3] = {0, 0, 0};
    double c5 = 0.0, Ce[3] = {0, 0, 0}, dCe[3] = {0, 0, 0}, dFCe[3] = {0, 0, 0};
    const double dI1bar = dJm23 * I1 + Jm23 * dI1;
    if (model != IBREF_NEO_HOOKEAN)
        for (int r = 0; r < 3; ++r) {
            Fe[r] = Fm[3 * r] * ef[0] + Fm[3 * r + 1] * ef[1] + Fm[3 * r + 2] * ef[2];
            dFe[r] = dFm[3 * r] * ef[0] + dFm[3 * r + 1] * ef[1] + dFm[3 * r + 2] * ef[2];
        }
    const double I4 = Fe[0] * Fe[0] + Fe[1] * Fe[1] + Fe[2] * Fe[2];
    const double dI4 = 2.0 * (Fe[0] * dFe[0] + Fe[1] * dFe[1] + Fe[2] * dFe[2]);
    if (model == IBREF_NEO_HOOKEAN) {
        alpha = par[0];
        dalpha = 0.0;
        kappa = par[1];
    } else if (model == IBREF_STANDARD_REINFORCING) {
        double GT = par[0], GL = par[1], EL = par[2], cL = EL + GT - 4.0 * GL;
        kappa = par[3];
        alpha = GT;
        dalpha = 0.0;
        fib = 2.0 * (GT - GL) + 0.5 * cL * (I4 - 1.0);
        dfib = 0.5 * cL * dI4;
        c5 = -(GT - GL);
        for (int c = 0; c < 3; ++c) {
            Ce[c] = Fm[c] * Fe[0] + Fm[3 + c] * Fe[1] + Fm[6 + c] * Fe[2];
            dCe[c] = dFm[c] * Fe[0] + dFm[3 + c] * Fe[1] + dFm[6 + c] * Fe[2] +
                     Fm[c] * dFe[0] + Fm[3 + c] * dFe[1] + Fm[6 + c] * dFe[2];
        }
        for (int r = 0; r < 3; ++r) {
            dFCe[r] = dFm[3 * r] * Ce[0] + dFm[3 * r + 1] * Ce[1] + dFm[3 * r + 2] * Ce[2] +
                      Fm[3 * r] * dCe[0] + Fm[3 * r + 1] * dCe[1] + Fm[3 * r + 2] * dCe[2];
        }
    } else if (model == IBREF_FIBRE_REINFORCED_1) {
        double C1 = par[0], af = par[1], bf = par[2];
        kappa = par[3];
        alpha = 2.0 * C1;
        dalpha = 0.0;
        if (I4 > 1.0) {
            double q = I4 - 1.0, Ef = exp(bf * q * q);
            fib = 2.0 * af * q * Ef;
            dfib = 2.0 * af * Ef * (1.0 + 2.0 * bf * q * q) * dI4;
        }
    } else if (model == IBREF_FIBRE_REINFORCED_2) {
        double C10 = par[0], C01 = par[1], af = par[2], bf = par[3];
        kappa = par[4];
        alpha = 2.0 * C10 * C01 * exp(C01 * (Jm23 * I1 - 3.0));
        dalpha = alpha * C01 * dI1bar;
        double q = I4 - 1.0, Ef = exp(bf * q * q);
        fib = 2.0 * af * q * Ef;
        dfib = 2.0 * af * Ef * (1.0 + 2.0 * bf * q * q) * dI4;
    } else if (model == IBREF_HOLZAPFEL_OGDEN) {
        double a = par[0], b = par[1], af = par[2], bf = par[3];
        double as = par[5], bs = par[6], afs = par[7], bfs = par[8];
        kappa = par[4];
        double E1 = exp(b * (Jm23 * I1 - 3.0));
        alpha = a * E1;
        dalpha = a * E1 * b * dI1bar;
        if (I4 > 1.0) {
            double Ef = exp(bf * (I4 - 1.0) * (I4 - 1.0));
            fib = 2.0 * af * (I4 - 1.0) * Ef;
            dfib = 2.0 * af * Ef * (1.0 + 2.0 * bf * (I4 - 1.0) * (I4 - 1.0)) * dI4;
        }
        if (as != 0.0 || afs != 0.0) {
            if (!es) return IBREF_E_INVAL;
            for (int r = 0; r < 3; ++r) {
                esv[r] = es[r];
                Fs[r] = Fm[3 * r] * es[0] + Fm[3 * r + 1] * es[1] + Fm[3 * r + 2] * es[2];
                dFs[r] = dFm[3 * r] * es[0] + dFm[3 * r + 1] * es[1] + dFm[3 * r + 2] * es[2];
            }
            double I4s = Fs[0] * Fs[0] + Fs[1] * Fs[1] + Fs[2] * Fs[2];
            if (I4s > 1.0) {
                double dI4s = 2.0 * (Fs[0] * dFs[0] + Fs[1] * dFs[1] + Fs[2] * dFs[2]);
                double Es = exp(bs * (I4s - 1.0) * (I4s - 1.0));
                sh = 2.0 * as * (I4s - 1.0) * Es;
                dsh = 2.0 * as * Es * (1.0 + 2.0 * bs * (I4s - 1.0) * (I4s - 1.0)) * dI4s;
            }
            double I8 = Fe[0] * Fs[0] + Fe[1] * Fs[1] + Fe[2] * Fs[2];
            double dI8 = dFe[0] * Fs[0] + dFe[1] * Fs[1] + dFe[2] * Fs[2] +
                         Fe[0] * dFs[0] + Fe[1] * dFs[1] + Fe[2] * dFs[2];
            double Efs = exp(bfs * I8 * I8);
            fs = afs * I8 * Efs;
            dfs = afs * Efs * (1.0 + 2.0 * bfs * I8 * I8) * dI8;
        }
        if (Ta != 0.0) {
            double r4 = sqrt(I4);
            fib += Ta * (1.0 + 4.9 * (r4 - 1.0));
            dfib += Ta * 4.9 / (2.0 * r4) * dI4;
        }
    } else {
        return IBREF_E_INVAL;
    }
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            int o = 3 * r + c;
            double M = Fm[o] - I1 / 3.0 * FiT[o];
            double dM = dFm[o] - dI1 / 3.0 * FiT[o] - I1 / 3.0 * dFiT[o];
            dP[o] = (dalpha * Jm23 + alpha * dJm23) * M + alpha * Jm23 * dM +
                    dfib * Fe[r] * ef[c] + fib * dFe[r] * ef[c] +
                    dsh * Fs[r] * esv[c] + sh * dFs[r] * esv[c] +
                    dfs * (Fe[r] * esv[c] + Fs[r] * ef[c]) + fs * (dFe[r] * esv[c] + dFs[r] * ef[c]) +
                    c5 * (dFe[r] * Ce[c] + Fe[r] * dCe[c] + dFCe[r] * ef[c]) +
                    kappa * dlnJ * FiT[o] + kappa * lnJ * dFiT[o];
        }
    return IBREF_OK;
}

/* shared element loop for the force derivatives: per Gauss point returns the
 * shape gradients, the weight and F; mode 0: HV -= dP grad N w; mode 1:
 * dtheta += -w dP/dtheta : (sum_a lam_a (x) grad N_a) */
static int fe_derivative_loop(const ibref_mesh* m, const double* x, const double* V, double* out,
                              int mode) {
    const int npe = mesh_npe(m);
    if (npe != 8 && npe != 4 && npe != 10) return IBREF_E_INVAL;
    for (int e = 0; e < m->n_elems; ++e) {
        const int32_t* cn = m->conn + (long)npe * e;
        int mid = m->mat_id[e];
        if (mid < 0 || mid >= m->n_mats) return IBREF_E_INVAL;
        const double* par = m->mat_params + (long)IBREF_MAT_PARAMS * mid;
        int model = m->mat_model[mid];
        const double* ef = m->fibre + 3L * e;
        const double* es = m->sheet ? m->sheet + 3L * e : NULL;
        double Xe[10][3], xe[10][3], ve[10][3], He[10][3];
        for (int a = 0; a < npe; ++a)
            for (int r = 0; r < 3; ++r) {
                Xe[a][r] = m->X_ref[3L * cn[a] + r];
                xe[a][r] = x[3L * cn[a] + r];
                ve[a][r] = V[3L * cn[a] + r];
                He[a][r] = 0.0;
            }
        for (int g = 0; g < elem_nq(npe); ++g) {
            double dN[10][3];
            const double wq = elem_rule(npe, g, dN);
            double J0[9] = {0};
            for (int a = 0; a < npe; ++a)
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) J0[3 * r + c] += Xe[a][r] * dN[a][c];
            double w = det3(J0);
            if (!(w > 0.0)) return IBREF_E_NUMERIC;
            double cof[9], J0inv[9];
            cof3(J0, cof);
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) J0inv[3 * r + c] = cof[3 * c + r] / w;
            const double wg = w * wq;
            double gN[10][3];
            for (int a = 0; a < npe; ++a)
                for (int c = 0; c < 3; ++c) {
                    double s = 0.0;
                    for (int r = 0; r < 3; ++r) s += dN[a][r] * J0inv[3 * r + c];
                    gN[a][c] = s;
                }
            double Fm[9] = {0}, dF[9] = {0};
            for (int a = 0; a < npe; ++a)
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) {
                        Fm[3 * r + c] += xe[a][r] * gN[a][c];
                        dF[3 * r + c] += ve[a][r] * gN[a][c];
                    }
            if (mode == 0) {
                double dP[9];
                int rc = ibref_pk1_tangent(model, par, Fm, ef, es, m->active_tension, dF, dP);
                if (rc) return rc;
                for (int a = 0; a < npe; ++a)
                    for (int r = 0; r < 3; ++r) {
                        double s = 0.0;
                        for (int c = 0; c < 3; ++c) s += dP[3 * r + c] * gN[a][c];
                        He[a][r] -= s * wg;
                    }
            } else if (model == IBREF_HOLZAPFEL_OGDEN) {
                /* dP/da, dP/db (isotropic), dP/da_f, dP/db_f (fibre), contracted with dF */
                double J = det3(Fm);
                if (!(J > 0.0)) return IBREF_E_NUMERIC;
                double cofF[9];
                cof3(Fm, cofF);
                double I1 = 0.0;
                for (int r = 0; r < 9; ++r) I1 += Fm[r] * Fm[r];
                double Jm23 = pow(J, -2.0 / 3.0);
                double b = par[1], af = par[2], bf = par[3], a0 = par[0];
                double E1 = exp(b * (Jm23 * I1 - 3.0));
                double Miso = 0.0, Mfib = 0.0;
                double Fe[3];
                for (int r = 0; r < 3; ++r)
                    Fe[r] = Fm[3 * r] * ef[0] + Fm[3 * r + 1] * ef[1] + Fm[3 * r + 2] * ef[2];
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) {
                        int o = 3 * r + c;
                        Miso += Jm23 * (Fm[o] - I1 / 3.0 * cofF[o] / J) * dF[o];
                        Mfib += Fe[r] * ef[c] * dF[o];
                    }
                double I4 = Fe[0] * Fe[0] + Fe[1] * Fe[1] + Fe[2] * Fe[2];
                double* dt = out + 4L * mid;
                dt[0] += -wg * E1 * Miso;
                dt[1] += -wg * a0 * (Jm23 * I1 - 3.0) * E1 * Miso;
                if (I4 > 1.0) {
                    double Ef = exp(bf * (I4 - 1.0) * (I4 - 1.0));
                    dt[2] += -wg * 2.0 * (I4 - 1.0) * Ef * Mfib;
                    dt[3] += -wg * 2.0 * af * (I4 - 1.0) * (I4 - 1.0) * (I4 - 1.0) * Ef * Mfib;
                }
                (void)af;
            }
        }
        if (mode == 0)
            for (int a = 0; a < npe; ++a)
                for (int r = 0; r < 3; ++r) out[3L * cn[a] + r] += He[a][r];
    }
    return IBREF_OK;
}

int ibref_fe_hvp(const ibref_mesh* m, const double* x, const double* V, double* HV) {
    for (long r = 0; r < 3L * m->n_nodes; ++r) HV[r] = 0.0;
    int rc = fe_derivative_loop(m, x, V, HV, 0);
    if (!rc) rc = tether_apply(m, x, V, HV, NULL);
    return rc;
}

int ibref_fe_param_vjp(const ibref_mesh* m, const double* x, const double* lamF, double* dtheta) {
    return fe_derivative_loop(m, x, lamF, dtheta, 1);
}

/* lamX_b += -p sum_g [dN_b/dxi (x_eta x mu) + dN_b/deta (mu x x_xi)],  mu = sum_a N_a lamF_a */
void ibref_pressure_vjp(int32_t n_faces, const int32_t* faces, const double* x, double p,
                        const double* lamF, double* lamX) {
    const double gp = 1.0 / sqrt(3.0);
    for (int f = 0; f < n_faces; ++f) {
        const int32_t* fn = faces + 4L * f;
        for (int g = 0; g < 4; ++g) {
            double s = (g & 1) ? gp : -gp, t = (g & 2) ? gp : -gp;
            double N[4], dNs[4], dNt[4];
            for (int a = 0; a < 4; ++a) {
                double sa = (a & 1) ? 1.0 : -1.0, ta = (a & 2) ? 1.0 : -1.0;
                N[a] = (1.0 + sa * s) * (1.0 + ta * t) / 4.0;
                dNs[a] = sa * (1.0 + ta * t) / 4.0;
                dNt[a] = (1.0 + sa * s) * ta / 4.0;
            }
            double xs[3] = {0, 0, 0}, xt[3] = {0, 0, 0}, mu[3] = {0, 0, 0};
            for (int a = 0; a < 4; ++a)
                for (int r = 0; r < 3; ++r) {
                    xs[r] += x[3L * fn[a] + r] * dNs[a];
                    xt[r] += x[3L * fn[a] + r] * dNt[a];
                    mu[r] += N[a] * lamF[3L * fn[a] + r];
                }
            double A[3] = {xt[1] * mu[2] - xt[2] * mu[1], xt[2] * mu[0] - xt[0] * mu[2],
                           xt[0] * mu[1] - xt[1] * mu[0]};          /* x_eta x mu */
            double B[3] = {mu[1] * xs[2] - mu[2] * xs[1], mu[2] * xs[0] - mu[0] * xs[2],
                           mu[0] * xs[1] - mu[1] * xs[0]};          /* mu x x_xi */
            for (int b = 0; b < 4; ++b)
                for (int r = 0; r < 3; ++r) lamX[3L * fn[b] + r] -= p * (dNs[b] * A[r] + dNt[b] * B[r]);
        }
    }
}

/* the projection of ibref_ns_step applied to v (b = -(rho/dt) D v, Poisson,
 * v -= (dt/rho) G p): the result is P v for any positive scale rho/dt */
int ibref_project(const ibref_fluid* fl, double* v) {
    const int n = fl->n;
    const long N3 = (long)n * n * n;
    const double rho = fl->rho, dt = fl->dt;
    double* b = (double*)malloc(sizeof(double) * (size_t)N3);
    double* p = (double*)calloc((size_t)N3, sizeof(double));
    double* gp = (double*)malloc(sizeof(double) * 3 * (size_t)N3);
    ibref_divergence(n, v, b);
    for (long i = 0; i < N3; ++i) b[i] = -(rho / dt) * b[i];
    remove_mean(N3, b);
    int32_t cyc;
    double rr;
    int rc = ibref_mg_solve(fl, 0.0, 1.0, 1, b, p, &cyc, &rr);
    if (!rc) {
        ibref_gradient(n, p, gp);
        for (long i = 0; i < 3 * N3; ++i) v[i] = v[i] - dt / rho * gp[i];
    }
    free(b); free(p); free(gp);
    return rc;
}

/*
 * Reverse of one walled IB step (the walled step of walled_ns_step and the
 * image spreading / interpolation of ibref_ib_step), given lam_u = dL/du^{n+1}
 * (box) and lam_X = dL/dX^{n+1}.  Every mirror map contributes its transpose
 * (extend -> fold, restrict -> pad), the periodic operators theirs
 * (G^T = -D, D^T = -G, the solves are symmetric, C'(u)^T from
 * ibref_convection_vjp), spreading at X/2 the interpolation (S^T = J / h'^3)
 * and positions the factor 1/2 of X/2.  The adjoint solves start from zero.
 */
static int walled_adjoint_step(const ibref_fluid* fl, const ibref_mesh* m, const double* u_n,
                               const double* X_n, const double* u_np1, double pressure, double* lam_u,
                               double* lam_X, double* dtheta) {
    const int n = fl->n, m2 = 2 * n, nn = m->n_nodes;
    const long M3 = (long)m2 * m2 * m2, N3 = (long)n * n * n, nn3 = 3L * nn;
    const double hi = 1.0 / m2, hi3 = hi * hi * hi;
    const double rho = fl->rho, dt = fl->dt;
    const double a = rho / dt, b = 0.5 * rho, c = 0.5 * (dt / rho);
    ibref_fluid f2 = image_fluid(fl);
    const size_t nb = (size_t)(nn3 > 0 ? nn3 : 1);
    double* Xh = (double*)malloc(sizeof(double) * nb);
    double* sX = (double*)malloc(sizeof(double) * nb);
    double* tmpX = (double*)malloc(sizeof(double) * nb);
    double* lamXn = (double*)malloc(sizeof(double) * nb);
    double* F = (double*)malloc(sizeof(double) * nb);
    double* lamF = (double*)malloc(sizeof(double) * nb);
    double* HV = (double*)malloc(sizeof(double) * nb);
    double* vi = (double*)calloc(3 * (size_t)M3, sizeof(double));   /* image vector scratch */
    double* wi = (double*)calloc(3 * (size_t)M3, sizeof(double));
    double* zi = (double*)calloc(3 * (size_t)M3, sizeof(double));
    double* si = (double*)calloc((size_t)M3, sizeof(double));       /* image scalar scratch */
    double* ti = (double*)calloc((size_t)M3, sizeof(double));
    double* vb = (double*)malloc(sizeof(double) * 3 * (size_t)N3);  /* box scratch */
    int rc = IBREF_OK;
    for (long r = 0; r < nn3; ++r) {
        Xh[r] = 0.5 * X_n[r];
        sX[r] = dt * lam_X[r];
        lamXn[r] = lam_X[r];
    }
    /* X^{n+1} = X^n + dt J(X^n/2) E u^{n+1} */
    ibref_spread(m2, nn, Xh, sX, vi);                 /* J^T = h'^3 S */
    for (long i = 0; i < 3 * M3; ++i) vi[i] *= hi3;
    wall_fold(n, 1, vi, vb);
    for (long i = 0; i < 3 * N3; ++i) vb[i] += lam_u[i];           /* dL/du^{n+1}, box */
    ibref_wall_extend(n, 1, u_np1, wi);
    for (long r = 0; r < nn3; ++r) tmpX[r] = 0.0;
    ibref_interp_vjp_X(m2, nn, Xh, wi, sX, tmpX);
    for (long r = 0; r < nn3; ++r) lamXn[r] += 0.5 * tmpX[r];
    /* u^{n+1} = R(us - c G p),  p = L^{-1} M E_s R_s (-2a D us) */
    ibref_wall_pad(n, 1, vb, vi);                     /* lam of the image u^{n+1} */
    ibref_divergence(m2, vi, si);                     /* lam_p = c D lam (G^T = -D) */
    for (long i = 0; i < M3; ++i) si[i] *= c;
    remove_mean(M3, si);
    {
        int32_t cyc;
        double rr;
        rc = ibref_mg_solve(&f2, 0.0, 1.0, 1, si, ti, &cyc, &rr);   /* lam_b = L^{-1} lam_p */
        remove_mean(M3, ti);   /* the transpose of the mean removal before the solve */
    }
    if (!rc) {
        wall_fold(n, 0, ti, vb);                      /* D^T R_s^T E_s^T (x -2a): + 2a G */
        ibref_wall_pad(n, 0, vb, si);
        ibref_gradient(m2, si, wi);
        for (long i = 0; i < 3 * M3; ++i) vi[i] += 2.0 * a * wi[i];   /* lam_us */
        wall_fold(n, 1, vi, vb);                      /* us = E R u* */
        ibref_wall_pad(n, 1, vb, wi);
        for (int d = 0; d < 3 && !rc; ++d) {          /* u* = H^{-1} g_s */
            int32_t cyc;
            double rr;
            rc = ibref_mg_solve(&f2, a, f2.mu, 0, wi + d * M3, zi + d * M3, &cyc, &rr);
        }
    }
    if (!rc) {
        wall_fold(n, 1, zi, vb);                      /* g_s = E R g */
        ibref_wall_pad(n, 1, vb, vi);                 /* lam_g (image) */
        /* g = a E u - b C(E u) + E f */
        ibref_wall_extend(n, 1, u_n, wi);
        for (long i = 0; i < 3 * M3; ++i) zi[i] = 0.0;
        if (fl->convection) ibref_convection_vjp(m2, wi, vi, zi);
        for (long i = 0; i < 3 * M3; ++i) wi[i] = a * vi[i] - b * zi[i];
        wall_fold(n, 1, wi, lam_u);                   /* dL/du^n */
        wall_fold(n, 1, vi, vb);                      /* dL/df (box) */
        ibref_wall_extend(n, 1, vb, wi);              /* E dL/df */
        /* f = (1/8) E^T S(X/2) F */
        ibref_interpolate(m2, nn, Xh, wi, lamF);
        for (long r = 0; r < nn3; ++r) lamF[r] *= 0.125 / hi3;
        rc = ibref_fe_force(m, X_n, F, NULL, NULL);
    }
    if (!rc) {
        if (m->n_faces > 0 && pressure != 0.0) ibref_pressure_load(m->n_faces, m->faces, X_n, pressure, F);
        for (long r = 0; r < nn3; ++r) tmpX[r] = 0.0;
        ibref_spread_vjp_X(m2, nn, Xh, F, wi, tmpX);
        for (long r = 0; r < nn3; ++r) lamXn[r] += 0.0625 * tmpX[r];
        rc = ibref_fe_hvp(m, X_n, lamF, HV);
    }
    if (!rc) {
        for (long r = 0; r < nn3; ++r) lamXn[r] += HV[r];
        if (m->n_faces > 0 && pressure != 0.0)
            ibref_pressure_vjp(m->n_faces, m->faces, X_n, pressure, lamF, lamXn);
        if (dtheta) rc = ibref_fe_param_vjp(m, X_n, lamF, dtheta);
        for (long r = 0; r < nn3; ++r) lam_X[r] = lamXn[r];
    }
    free(Xh); free(sX); free(tmpX); free(lamXn); free(F); free(lamF); free(HV);
    free(vi); free(wi); free(zi); free(si); free(ti); free(vb);
    return rc;
}

int ibref_adjoint_step(const ibref_fluid* fl, const ibref_mesh* m, const double* u_n,
                       const double* X_n, const double* u_np1, double pressure, double* lam_u,
                       double* lam_X, double* dtheta) {
    if (fl->walls) return walled_adjoint_step(fl, m, u_n, X_n, u_np1, pressure, lam_u, lam_X, dtheta);
    const int n = fl->n;
    const long N3 = (long)n * n * n;
    const long nn3 = 3L * m->n_nodes;
    const double h = 1.0 / n, h3 = h * h * h, rho = fl->rho, dt = fl->dt, mu = fl->mu;
    double* tot = (double*)calloc(3 * (size_t)N3, sizeof(double));
    double* lg = (double*)calloc(3 * (size_t)N3, sizeof(double));
    double* cv = (double*)calloc(3 * (size_t)N3, sizeof(double));
    double* lamXn = (double*)malloc(sizeof(double) * (size_t)(nn3 > 0 ? nn3 : 1));
    double* sX = (double*)malloc(sizeof(double) * (size_t)(nn3 > 0 ? nn3 : 1));
    double* F = (double*)malloc(sizeof(double) * (size_t)(nn3 > 0 ? nn3 : 1));
    double* lamF = (double*)malloc(sizeof(double) * (size_t)(nn3 > 0 ? nn3 : 1));
    double* HV = (double*)malloc(sizeof(double) * (size_t)(nn3 > 0 ? nn3 : 1));
    int rc = IBREF_OK;
    /* X^{n+1} = X^n + dt J(X^n) u^{n+1} */
    for (long r = 0; r < nn3; ++r) {
        lamXn[r] = lam_X[r];
        sX[r] = dt * lam_X[r];
    }
    ibref_spread(n, m->n_nodes, X_n, sX, tot);               /* tot = S(X^n) (dt lam_X') */
    for (long i = 0; i < 3 * N3; ++i) tot[i] = lam_u[i] + h3 * tot[i];
    ibref_interp_vjp_X(n, m->n_nodes, X_n, u_np1, sX, lamXn);
    /* u^{n+1} = P u*,  u* = H^{-1} g */
    rc = ibref_project(fl, tot);
    for (int d = 0; d < 3 && !rc; ++d) {
        int32_t cyc;
        double rr;
        rc = ibref_mg_solve(fl, rho / dt, mu, 0, tot + d * N3, lg + d * N3, &cyc, &rr);
    }
    if (!rc) {
        /* g = (rho/dt) u^n - rho C(u^n) + S(X^n) F */
        if (fl->convection) ibref_convection_vjp(n, u_n, lg, cv);
        for (long i = 0; i < 3 * N3; ++i) lam_u[i] = rho / dt * lg[i] - rho * cv[i];
        ibref_interpolate(n, m->n_nodes, X_n, lg, lamF);
        for (long r = 0; r < nn3; ++r) lamF[r] /= h3;
        rc = ibref_fe_force(m, X_n, F, NULL, NULL);
    }
    if (!rc) {
        if (m->n_faces > 0 && pressure != 0.0) ibref_pressure_load(m->n_faces, m->faces, X_n, pressure, F);
        ibref_spread_vjp_X(n, m->n_nodes, X_n, F, lg, lamXn);
        rc = ibref_fe_hvp(m, X_n, lamF, HV);
    }
    if (!rc) {
        for (long r = 0; r < nn3; ++r) lamXn[r] += HV[r];
        if (m->n_faces > 0 && pressure != 0.0)
            ibref_pressure_vjp(m->n_faces, m->faces, X_n, pressure, lamF, lamXn);
        if (dtheta) rc = ibref_fe_param_vjp(m, X_n, lamF, dtheta);
        for (long r = 0; r < nn3; ++r) lam_X[r] = lamXn[r];
    }
    free(tot); free(lg); free(cv); free(lamXn); free(sX); free(F); free(lamF); free(HV);
    return rc;
}

int ibref_rollout_grad(const ibref_fluid* fl, const ibref_mesh* m, const double* u0,
                       const double* X0, double t0, int32_t n_steps, double p0, double T,
                       const double* X_target, double* loss, double* dLdX0, double* dtheta) {
    const double pi = 3.14159265358979323846;
    const int n = fl->n;
    const long N3 = (long)n * n * n, nn3 = 3L * m->n_nodes;
    double* us = (double*)malloc(sizeof(double) * 3 * (size_t)N3 * (size_t)(n_steps + 1));
    double* Xs = (double*)malloc(sizeof(double) * (size_t)(nn3 > 0 ? nn3 : 1) * (size_t)(n_steps + 1));
    double* p = (double*)calloc((size_t)N3, sizeof(double));
    double* pr = (double*)malloc(sizeof(double) * (size_t)(n_steps > 0 ? n_steps : 1));
    int rc = IBREF_OK;
    memcpy(us, u0, sizeof(double) * 3 * (size_t)N3);
    memcpy(Xs, X0, sizeof(double) * (size_t)nn3);
    for (int s = 0; s < n_steps && !rc; ++s) {
        double t = t0 + s * fl->dt;
        pr[s] = 0.0;
        if (p0 != 0.0 && T > 0.0) {
            double sn = sin(pi * t / T);
            pr[s] = p0 * sn * sn;
        }
        memcpy(us + 3 * N3 * (s + 1), us + 3 * N3 * s, sizeof(double) * 3 * (size_t)N3);
        memcpy(Xs + nn3 * (s + 1), Xs + nn3 * s, sizeof(double) * (size_t)nn3);
        ibref_mesh ms = mesh_at(m, t);
        rc = ibref_ib_step(fl, &ms, us + 3 * N3 * (s + 1), p, Xs + nn3 * (s + 1), pr[s], NULL);
    }
    if (!rc) {
        const double* XN = Xs + nn3 * n_steps;
        double L = 0.0;
        for (long r = 0; r < nn3; ++r) {
            double d = XN[r] - X_target[r];
            L += d * d;
            dLdX0[r] = 2.0 * d;
        }
        *loss = L;
        double* lam_u = (double*)calloc(3 * (size_t)N3, sizeof(double));
        for (int s = n_steps - 1; s >= 0 && !rc; --s) {
            ibref_mesh ms = mesh_at(m, t0 + s * fl->dt);
            rc = ibref_adjoint_step(fl, &ms, us + 3 * N3 * s, Xs + nn3 * s, us + 3 * N3 * (s + 1),
                                    pr[s], lam_u, dLdX0, dtheta);
        }
        free(lam_u);
    }
    free(us); free(Xs); free(p); free(pr);
    return rc;
}
