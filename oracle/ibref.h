/*
 * ibref -- plain FP64 CPU implementation of the matrix-free immersed-boundary
 * timestep (Ma, Cai, Wang, Luo, Gao, "Fully GPU-Accelerated Immersed Boundary
 * Method for Fluid-Structure Interaction in Complex Cardiac Models").
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct reference the
 * GPU library is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no source with the GPU
 * library and must never be called from the product path.
 *
 * Conventions (all arrays host memory, caller-owned, C order):
 *   grid     periodic unit cube, n cells per side, h = 1/n.  Scalars are
 *            [n][n][n] with x fastest: idx = i + n*(j + n*k).  Vector fields
 *            are [3][n][n][n].  u^d[i,j,k] lives on the face at coordinate
 *            i*h along d and cell centres ((.+1/2)h) along the other axes;
 *            pressure lives at cell centres.
 *   nodes    X[n_nodes][3], unwrapped positions (only stencil indices wrap).
 *   hexes    conn[n_elems][8], local node a = i + 2j + 4k at (2i-1,2j-1,2k-1);
 *            or tetrahedra, conn[n_elems][4 or 10] (see nodes_per_elem).
 *   quads    faces[n_faces][4], local node a = i + 2j at (2i-1,2j-1).
 *
 * Return codes: 0 ok, 1 invalid argument, 4 no convergence, 5 numeric
 * (non-finite residual or J <= 0).
 */
#ifndef IBREF_H
#define IBREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { IBREF_OK = 0, IBREF_E_INVAL = 1, IBREF_E_NOCONV = 4, IBREF_E_NUMERIC = 5 };
enum {
    IBREF_NEO_HOOKEAN = 0,         /* (mu_s, kappa) */
    IBREF_HOLZAPFEL_OGDEN = 1,     /* Psi_4: (a, b, a_f, b_f, kappa, a_s, b_s, a_fs, b_fs) */
    IBREF_STANDARD_REINFORCING = 2,/* Psi_1: (G_T, G_L, E_L, kappa) */
    IBREF_FIBRE_REINFORCED_1 = 3,  /* Psi_2: (C_1, a_f, b_f, kappa) */
    IBREF_FIBRE_REINFORCED_2 = 4   /* Psi_3: (C_10, C_01, a_f, b_f, kappa) */
};
#define IBREF_MAT_PARAMS 9         /* parameter slots per material */

typedef struct {
    int32_t n;                 /* cells per side */
    double rho, mu, dt;
    int32_t mg_pre, mg_post;   /* smoothing sweeps (red+black pairs) */
    int32_t mg_max_cycles;     /* > this many V-cycles: no convergence */
    int32_t mg_fixed_cycles;   /* > 0: run exactly this many cycles, no stop test */
    int32_t mg_coarse_sweeps;  /* 0: the coarsest level is the first with at most 32 cells
                                  per side, solved exactly by its Fourier diagonalisation;
                                  > 0: the first with fewer than 8, relaxed by this many
                                  red+black sweeps */
    double mg_rtol;            /* stop when ||r|| <= rtol ||b|| */
    int32_t convection;        /* 1: explicit flux-form convection, 0: Stokes */
    int32_t mg_krylov;         /* 1: Poisson solves by conjugate gradients preconditioned
                                  with one V-cycle; 0: plain V-cycle iteration */
    int32_t walls;             /* 0: periodic box; 1: walled box (u* = 0 and u.n = 0 on
                                  every face), solved on its (2n)^3 mirror image */
} ibref_fluid;

typedef struct {
    int32_t n_nodes;
    const double* X_ref;       /* [n_nodes][3] reference configuration */
    int32_t n_elems;
    const int32_t* conn;       /* [n_elems][8] */
    const double* fibre;       /* [n_elems][3] unit fibre e_f (reference) */
    const int32_t* mat_id;     /* [n_elems] */
    int32_t n_mats;
    const int32_t* mat_model;  /* [n_mats] IBREF_NEO_HOOKEAN / IBREF_HOLZAPFEL_OGDEN */
    const double* mat_params;  /* [n_mats][IBREF_MAT_PARAMS]: NH (mu_s, kappa, 0...);
                                  HO (a, b, a_f, b_f, kappa, a_s, b_s, a_fs, b_fs) */
    int32_t n_faces;
    const int32_t* faces;      /* [n_faces][4] pressure-loaded quads */
    const double* sheet;       /* [n_elems][3] unit sheet e_s (reference, orthogonal to e_f);
                                  NULL allowed while every a_s and a_fs is 0 */
    double active_tension;     /* T_a of the active fibre stress of HO materials (force,
                                  Hessian product); ibref_advance and ibref_rollout_grad set
                                  it per step from the waveform below when ta_max != 0 */
    double ta_max, ta_t_on, ta_duration;  /* active-tension waveform (ibref_active_tension) */
    int32_t n_tethers;         /* penalty tethers: F_a += -K (X_a - Y) at node a */
    const int32_t* tether_node;     /* [n_tethers] distinct node indices */
    const double* tether_target;    /* [n_tethers][3] Y */
    const double* tether_K;         /* [n_tethers][6] symmetric K: xx, yy, zz, xy, xz, yz */
    int32_t nodes_per_elem;    /* 8 (or 0): trilinear hexes; 4: P1 tetrahedra; 10: P2
                                  tetrahedra (vertices 0-3, then edge nodes on (0,1), (1,2),
                                  (0,2), (0,3), (1,3), (2,3)); conn is [n_elems][this] */
} ibref_mesh;

typedef struct {
    int32_t cycles[4];         /* Helmholtz x, y, z, Poisson */
    double relres[4];
    double min_J;              /* smallest Jacobian over all Gauss points */
    double energy;             /* elastic energy at X^n */
} ibref_step_stats;

/* --- discrete operators on the MAC grid --- */
void ibref_laplacian(int32_t n, const double* q, double* out);        /* out = Lap_h q */
void ibref_divergence(int32_t n, const double* u, double* out);       /* out = D u */
void ibref_gradient(int32_t n, const double* p, double* out);         /* out = G p */
void ibref_convection(int32_t n, const double* u, double* out);       /* out = C(u) */

/* --- regularized delta and coupling --- */
double ibref_phi(double r);                                            /* 4-point Peskin kernel */
void ibref_spread(int32_t n, int32_t n_nodes, const double* X, const double* F, double* f); /* f += S(X)F */
void ibref_interpolate(int32_t n, int32_t n_nodes, const double* X, const double* u, double* U); /* U = J(X)u */

/* --- solid mechanics --- */
/* P = dPsi/dF (+ the active stress for HO) and Psi (+ the active potential);
 * es may be NULL when a_s = a_fs = 0; Ta is the active tension T_a(t) */
int ibref_pk1(int32_t model, const double* params, const double* Fm /*[3][3] row-major*/,
              const double* ef, const double* es, double Ta, double* P /*[3][3]*/, double* psi);
/* T_a(t): ta_max times the left-ventricle activation shape, whose window
 * (0.5, 0.8) is mapped onto [t_on, t_on + duration] */
double ibref_active_tension(double ta_max, double t_on, double duration, double t);
int ibref_fe_force(const ibref_mesh* m, const double* x, double* F /*[n_nodes][3], :=*/,
                   double* energy, double* min_J);
void ibref_pressure_load(int32_t n_faces, const int32_t* faces, const double* x, double p,
                         double* F /* += */);

/* --- multigrid: solves (sigma I - nu Lap_h) x = b on the periodic grid; with
 * mg_krylov the Poisson case (poisson = 1) runs preconditioned conjugate
 * gradients, counting one iteration as one cycle --- */
int ibref_mg_solve(const ibref_fluid* fl, double sigma, double nu, int32_t poisson,
                   const double* b, double* x /* guess -> solution */,
                   int32_t* cycles, double* relres);

/* --- walled box: the image construction (n = cells per side of the box) ---
 * A walled box is the (2n)^3 periodic box holding its mirror images: scalars
 * (pressure) are even across every wall; velocity components are odd across
 * every wall (the wall-normal face values vanish, the tangential ghost values
 * are minus the interior ones: no slip).  ext: box -> image grid; fold: the
 * transpose of ext; restrict: the box part of an image field, wall faces 0. */
void ibref_wall_extend(int32_t n, int32_t vector, const double* box, double* img);
void ibref_wall_fold(int32_t n, const double* img, double* box /* := */);
void ibref_wall_restrict(int32_t n, int32_t vector, const double* img, double* box);
void ibref_wall_pad(int32_t n, int32_t vector, const double* box, double* img); /* restrict^T */
/* f += S(X) F and U = J(X) u on the walled box, through the image grid */
void ibref_walled_spread(int32_t n, int32_t n_nodes, const double* X, const double* F, double* f);
void ibref_walled_interpolate(int32_t n, int32_t n_nodes, const double* X, const double* u, double* U);
/* (sigma I - nu Lap_h) x = b for one cell-centred field on the walled box:
 * Poisson (sigma = 0) with Neumann walls, else Dirichlet walls */
int ibref_walled_solve(const ibref_fluid* fl, double sigma, double nu, int32_t poisson,
                       const double* b, double* x, int32_t* cycles, double* relres);

/* --- one fluid step (given the Eulerian force density f) and one IB step --- */
int ibref_ns_step(const ibref_fluid* fl, const double* f, double* u, double* p,
                  ibref_step_stats* st);
int ibref_ib_step(const ibref_fluid* fl, const ibref_mesh* m, double* u, double* p, double* X,
                  double pressure, ibref_step_stats* st);
/* n_steps IB steps from t0; endocardial pressure p0 sin^2(pi t_n / T) at t_n = t0 + n dt.
 * stats (may be NULL) receives one record per step. */
int ibref_advance(const ibref_fluid* fl, const ibref_mesh* m, double* u, double* p, double* X,
                  double t0, int32_t n_steps, double p0, double T, ibref_step_stats* stats);
/* Steps first_step .. first_step + n_steps - 1 of a run started at t0 (step s at
 * t0 + s dt): a long run taken in pieces gives exactly the unsplit run. */
int ibref_advance_steps(const ibref_fluid* fl, const ibref_mesh* m, double* u, double* p, double* X,
                        double t0, int32_t first_step, int32_t n_steps, double p0, double T,
                        ibref_step_stats* stats);

/* --- discrete adjoint (reverse mode of one IB step) ---------------------
 * Gradients are taken with respect to the plain entries of the arrays
 * (lam = dL/d(array)).  The multigrid solves are treated as exact inverses of
 * their symmetric operators. */
void ibref_convection_vjp(int32_t n, const double* u, const double* lam, double* out); /* out = C'(u)^T lam */
double ibref_dphi(double r);                                           /* d phi / d r */
/* lamX += [d/dX (S(X) F)]^T lam_f */
void ibref_spread_vjp_X(int32_t n, int32_t n_nodes, const double* X, const double* F,
                        const double* lam_f, double* lamX);
/* lamX += [d/dX (J(X) u)]^T lamU */
void ibref_interp_vjp_X(int32_t n, int32_t n_nodes, const double* X, const double* u,
                        const double* lamU, double* lamX);
/* dP = dP/dF : dF (directional derivative of the first Piola-Kirchhoff stress) */
int ibref_pk1_tangent(int32_t model, const double* params, const double* Fm, const double* ef,
                      const double* es, double Ta, const double* dFm, double* dP);
/* HV = (dF/dx) V, the directional derivative of the elastic nodal force
 * (minus the strain-energy Hessian times V); overwritten */
int ibref_fe_hvp(const ibref_mesh* m, const double* x, const double* V, double* HV);
/* dtheta[m][0..3] += lamF . dF/d(a, b, a_f, b_f) for Holzapfel-Ogden materials */
int ibref_fe_param_vjp(const ibref_mesh* m, const double* x, const double* lamF, double* dtheta);
/* lamX += [d/dx F_pressure(x)]^T lamF */
void ibref_pressure_vjp(int32_t n_faces, const int32_t* faces, const double* x, double p,
                        const double* lamF, double* lamX);
/* v := P v, the discrete projection onto solenoidal fields (Poisson solve) */
int ibref_project(const ibref_fluid* fl, double* v);
/* Reverse of one ibref_ib_step from (u_n, X_n) to u_np1:
 * in: lam_u = dL/du^{n+1}, lam_X = dL/dX^{n+1};  out: lam_u = dL/du^n,
 * lam_X = dL/dX^n;  dtheta[n_mats][4] += dL/d(a, b, a_f, b_f) of this step.
 * On a walled box the step is reversed on the image grid, each mirror map by
 * its transpose (extension by the fold, restriction by ibref_wall_pad). */
int ibref_adjoint_step(const ibref_fluid* fl, const ibref_mesh* m, const double* u_n,
                       const double* X_n, const double* u_np1, double pressure, double* lam_u,
                       double* lam_X, double* dtheta);
/* Loss L = sum_q |X^N_q - X_target_q|^2 after n_steps from (u0, X0) at t0 (p0 sin^2
 * pressure as ibref_advance), its gradient with respect to X0 and the HO
 * parameters, by storing every state and running ibref_adjoint_step backwards. */
int ibref_rollout_grad(const ibref_fluid* fl, const ibref_mesh* m, const double* u0,
                       const double* X0, double t0, int32_t n_steps, double p0, double T,
                       const double* X_target, double* loss, double* dLdX0, double* dtheta);

#ifdef __cplusplus
}
#endif
#endif
