/*
 * hipib -- matrix-free immersed-boundary timestep on AMD Instinct MI355X (gfx950).
 *
 * Implements the fully discrete scheme of Ma, Cai, Wang, Luo and Gao, "Fully
 * GPU-Accelerated Immersed Boundary Method for Fluid-Structure Interaction in
 * Complex Cardiac Models": given u^n and X^n, find u^{n+1}, p^{n+1}, X^{n+1}
 * (section "Spatial Discretization") with
 *   - nodal forces F_i = -sum_q P(X_q) : grad N_i(X_q) w_q, evaluated element by
 *     element without any assembled matrix ("Eulerian-Lagrangian coupling
 *     operators"; laws from "Constitutive laws");
 *   - spreading f = S(X^n) F and interpolation U = J(X^n) u^{n+1} through the
 *     4-point Peskin delta on the staggered (MAC) grid;
 *   - a Chorin projection step (Helmholtz solve, Poisson solve, velocity
 *     correction) whose solves use geometric multigrid (named in the abstract).
 *
 * Layout (all device arrays contiguous, FP64, caller-owned):
 *   grid     periodic unit cube, n cells per side, h = 1/n; scalars [n][n][n]
 *            with x fastest (idx = i + n*(j + n*k)); vectors [3][n][n][n];
 *            u^d[i,j,k] sits at coordinate i*h along d and (.+1/2)h along the
 *            other two axes, p at cell centres.
 *   nodes    X[n_nodes][3], unwrapped positions (stencil indices wrap).
 *   hexes    conn[n_elems][8], local node a = i + 2j + 4k at (2i-1,2j-1,2k-1).
 *   quads    faces[n_faces][4], local node a = i + 2j; dx/dxi x dx/deta points
 *            out of the solid into the loaded cavity.
 *
 * Streams: every call is enqueued on the context's stream and returns without
 * waiting, except calls that return host values (hipib_mg_solve,
 * hipib_ns_step, hipib_ib_step, hipib_advance: they wait for the multigrid
 * stop decisions).  The context keeps no pointer to caller arrays after a call.
 *
 * Errors: every call returns a status and never aborts across the boundary;
 * hipib_last_error() returns a message for the calling thread's last failure.
 * Argument errors (null or misaligned pointer, bad size, index out of range)
 * return HIPIB_E_INVAL before anything is enqueued.  A HIP runtime failure
 * makes the context unusable (HIPIB_E_HIP from then on).  After any error the
 * contents of output arrays are unspecified.
 */
#ifndef HIPIB_H
#define HIPIB_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hipib_ctx hipib_ctx;

typedef enum {
    HIPIB_OK = 0,
    HIPIB_E_INVAL = 1,    /* bad argument; nothing was enqueued */
    HIPIB_E_NOMEM = 2,    /* device allocation failed */
    HIPIB_E_HIP = 3,      /* HIP runtime error; the context is unusable */
    HIPIB_E_NOCONV = 4,   /* multigrid reached mg_max_cycles */
    HIPIB_E_NUMERIC = 5,  /* non-finite residual, or J <= 0 at a Gauss point */
    HIPIB_E_STATE = 6     /* call before hipib_set_mesh / missing material */
} hipib_status;

typedef enum { HIPIB_FP64 = 0, HIPIB_MIXED = 1 } hipib_precision;
typedef enum {
    HIPIB_NEO_HOOKEAN = 0,           /* (mu_s, kappa) */
    HIPIB_HOLZAPFEL_OGDEN = 1,       /* Psi_4 (a, b, a_f, b_f, kappa[, a_s, b_s, a_fs, b_fs]) */
    HIPIB_STANDARD_REINFORCING = 2,  /* Psi_1 (G_T, G_L, E_L, kappa) */
    HIPIB_FIBRE_REINFORCED_1 = 3,    /* Psi_2 (C_1, a_f, b_f, kappa) */
    HIPIB_FIBRE_REINFORCED_2 = 4     /* Psi_3 (C_10, C_01, a_f, b_f, kappa) */
} hipib_model;
typedef enum { HIPIB_OP_HELMHOLTZ = 0, HIPIB_OP_POISSON = 1 } hipib_op;

#define HIPIB_MAX_MATERIALS 8

typedef struct {
    int32_t n;                /* cells per side: c * 2^k, c in {4, 6}, n >= 8 */
    double rho, mu, dt;       /* density, viscosity, time step (all > 0) */
    int32_t mg_pre, mg_post;  /* red+black smoothing sweeps before / after the
                                 coarse-grid correction (V(2,2): 2, 2) */
    int32_t mg_max_cycles;    /* more cycles than this: HIPIB_E_NOCONV */
    int32_t mg_fixed_cycles;  /* > 0: exactly this many cycles, no stop test */
    int32_t mg_coarse_sweeps; /* 0 (default): the coarsest level is the first with at
                                 most 32 cells per side, solved exactly by its Fourier
                                 diagonalisation; > 0: the first with fewer than 8,
                                 relaxed by this many red+black sweeps */
    double mg_rtol;           /* stop when ||b - A x||_2 <= rtol ||b||_2 */
    int32_t convection;       /* 1: explicit flux-form convection; 0: Stokes */
    int32_t precision;        /* hipib_precision */
    int32_t deterministic;    /* 1: atomic-free, bitwise run-to-run reproducible.
                                 Spreading then keeps one box per work item: about
                                 (n^3/T^3 + nodes/256) x 3 (T+4)^3 x 8 bytes of device
                                 memory (T = 8; 4 when n = 12), 190 MB at n = 128 */
    int32_t mg_krylov;        /* 1: Poisson solves by conjugate gradients preconditioned
                                 with one V-cycle (the "combined" multigrid reading of
                                 the abstract; one iteration counts as one cycle);
                                 0: plain V-cycle iteration.  Helmholtz solves always
                                 use the plain iteration. */
    int32_t walls;            /* 0: periodic box.  1: walled box with the boundary
                                 conditions u* = 0 and u^{n+1}.n = 0 on every face
                                 ("Spatial Discretization"); the wall-normal velocity
                                 of the faces at index 0 of its axis is zero (it
                                 stands for both walls of that axis), tangential
                                 ghosts are minus the interior values, pressure has
                                 Neumann walls.  Solved on the (2n)^3 periodic grid of
                                 the box and its mirror images (a second context the
                                 library owns: 8 times the grid memory and work);
                                 hipib_mg_solve takes each component as one
                                 cell-centred field (Dirichlet, or Neumann for
                                 Poisson).  hipib_adjoint_step reverses the walled
                                 step; the derivatives of single periodic operators
                                 (hipib_spread_vjp_X, hipib_interp_vjp_X,
                                 hipib_convection_vjp) return HIPIB_E_STATE. */
} hipib_config;

/* Fills cfg with the defaults: V(2,2), exact coarsest solve, rtol 1e-10, 50 cycles,
 * convection on, FP64, atomic mode, Krylov Poisson solves, periodic box;
 * n/rho/mu/dt are set to 32/1/0.01/1e-3. */
void hipib_default_config(hipib_config* cfg);

/* Creates a context for one grid on the current HIP device.  stream is a
 * hipStream_t (NULL: the null stream).  Allocates every grid workspace. */
hipib_status hipib_create(const hipib_config* cfg, void* stream, hipib_ctx** out);
hipib_status hipib_destroy(hipib_ctx* ctx);
/* Makes stream (a hipStream_t; NULL: the null stream) the context's stream for
 * every later call.  Work the context enqueued on its previous stream is
 * ordered before anything later enqueued on the new one (an event recorded on
 * the old stream is waited for by the new one); the caller's own work on the
 * old stream is not.  HIPIB_E_HIP if the event calls fail. */
hipib_status hipib_set_stream(hipib_ctx* ctx, void* stream);
const char* hipib_last_error(void);

/* --- set-up (host arrays, copied into the context) ---------------------- */
/* Lagrangian mesh: X_ref [n_nodes][3], conn [n_elems][8] (0 <= conn < n_nodes),
 * fibre [n_elems][3] (unit e_f in the reference configuration), mat_id
 * [n_elems] (0 <= mat_id < HIPIB_MAX_MATERIALS).  n_nodes may be 0. */
hipib_status hipib_set_mesh(hipib_ctx* ctx, int32_t n_nodes, const double* X_ref,
                            int32_t n_elems, const int32_t* conn, const double* fibre,
                            const int32_t* mat_id);
/* As hipib_set_mesh for any element type (the benchmark discretises its solid
 * with P2 tetrahedra): nodes_per_elem 8 = trilinear hexes (2x2x2 Gauss), 4 = P1
 * tetrahedra (one point at the centroid), 10 = P2 tetrahedra (vertices 0-3, then
 * edge nodes on (0,1), (1,2), (0,2), (0,3), (1,3), (2,3); the symmetric 4-point
 * rule of degree 2); conn [n_elems][nodes_per_elem], each element positively
 * oriented (det dX/dxi > 0 on the reference simplex xi, eta, zeta >= 0,
 * xi + eta + zeta <= 1 with vertices at the origin and the unit axes). */
hipib_status hipib_set_mesh_elements(hipib_ctx* ctx, int32_t n_nodes, const double* X_ref,
                                     int32_t n_elems, int32_t nodes_per_elem, const int32_t* conn,
                                     const double* fibre, const int32_t* mat_id);
/* Material law of one id ("Constitutive laws"), U = kappa/2 (ln J)^2 throughout:
 *   neo-Hookean (mu_s, kappa): Psi = mu_s/2 (I1bar - 3) + U;
 *   modified standard reinforcing Psi_1 (G_T, G_L, E_L, kappa):
 *     Psi = G_T/2 (I1bar - 3) + (G_T - G_L)/2 (2 I4f - I5f - 1)
 *         + (E_L + G_T - 4 G_L)/8 (I4f - 1)^2 + U,   I5f = e_f.C^2 e_f;
 *   fibre-reinforced 1, Psi_2 (C_1, a_f, b_f, kappa):
 *     Psi = C_1 (I1bar - 3) + a_f/(2b_f)(e^{b_f (I4f*-1)^2} - 1) + U;
 *   fibre-reinforced 2, Psi_3 (C_10, C_01, a_f, b_f, kappa), the plain I4f as
 *     printed: Psi = C_10 (e^{C_01 (I1bar-3)} - 1) + a_f/(2b_f)(e^{b_f (I4f-1)^2} - 1) + U
 *     (its stress is the derivative of this energy: C_01 in the exponent);
 * requires non-negative moduli and kappa, and b_f, C_01 > 0.  Holzapfel-Ogden
 * params (a, b, a_f, b_f, kappa[, a_s, b_s, a_fs, b_fs]) (n_params 5 or 9;
 * 5 means a_s = a_fs = 0):
 *   Psi = a/(2b)(e^{b(I1bar-3)} - 1) + sum_{i=f,s} a_i/(2b_i)(e^{b_i (I4i*-1)^2} - 1)
 *       + a_fs/(2b_fs)(e^{b_fs I8fs^2} - 1) + kappa/2 (ln J)^2,
 * I4i = e_i.C e_i, I4i* = max(I4i, 1), I8fs = e_f.C e_s; the fibre-sheet stress
 * is the derivative of this energy, a_fs I8 e^{b_fs I8^2} F (e_f(x)e_s + e_s(x)e_f).
 * Requires a, a_f, a_s, a_fs, kappa >= 0, b, b_f > 0, and b_s (b_fs) > 0 when
 * a_s (a_fs) > 0.  A material with a_s or a_fs > 0 needs hipib_set_sheets. */
hipib_status hipib_set_material(hipib_ctx* ctx, int32_t mat_id, int32_t model,
                                const double* params, int32_t n_params);
/* Penalty tethers (the constrained faces of the benchmark and valve models and
 * the base constraint of the left-ventricle model, enforced with a penalty
 * parameter; "Solid boundary" of the profile table): each tethered node a
 * gets the linear spring force F_a += -K_t (X_a - Y_t) in hipib_fe_force (and
 * so in every step), -K_t V_a in hipib_fe_hvp and the adjoint step.  node:
 * host [n_tethers] distinct indices < n_nodes; target Y: host [n_tethers][3];
 * K: host [n_tethers][6] symmetric stiffness (xx, yy, zz, xy, xz, yz), e.g.
 * kappa (1,1,1,0,0,0) to fix a node, kappa (n n^T + c c^T) to hold only the
 * normal and circumferential displacement.  Replaces earlier tethers;
 * dropped by the next hipib_set_mesh. */
hipib_status hipib_set_tethers(hipib_ctx* ctx, int32_t n_tethers, const int32_t* node,
                               const double* target, const double* K);
/* Sheet directions e_s of the elements (host [n_elems][3], unit, orthogonal to
 * the fibre, reference configuration; n_elems must equal the mesh's).  Dropped
 * by the next hipib_set_mesh. */
hipib_status hipib_set_sheets(hipib_ctx* ctx, int32_t n_elems, const double* sheet);
/* Active stress of the myocardium (the left-ventricle model): Holzapfel-Ogden
 * materials get P_a = T (F e_f) (x) e_f, the push-forward of the second
 * Piola-Kirchhoff stress S_a = T e_f (x) e_f, with T = T_a (1 + 4.9 (sqrt(I4f) - 1)).
 * hipib_set_active_tension sets the T_a used by hipib_fe_force, hipib_ib_step,
 * hipib_adjoint_step and hipib_fe_hvp (0 on creation; must be finite). */
hipib_status hipib_set_active_tension(hipib_ctx* ctx, double Ta);
/* T_a(t) of the left-ventricle model's activation, ta_max (1 - e^{-(s-0.5)^2/0.005})
 * for 0.5 < s < 0.65 and ta_max (1 - e^{-(0.8-s)^2/0.005}) for 0.65 <= s < 0.8,
 * 0 otherwise, with its window mapped onto the simulation clock by
 * s = 0.5 + 0.3 (t - t_on) / duration (0 when duration <= 0). */
double hipib_active_tension(double ta_max, double t_on, double duration, double t);
/* Activation followed by hipib_advance: with ta_max != 0 each step n sets the
 * active tension to hipib_active_tension(ta_max, t_on, duration, t_n) before it
 * runs (the last step's value stays set).  ta_max = 0 switches this off. */
hipib_status hipib_set_active_waveform(hipib_ctx* ctx, double ta_max, double t_on, double duration);
/* Quads loaded by the uniform cavity pressure (host [n_faces][4]). */
hipib_status hipib_set_pressure_faces(hipib_ctx* ctx, int32_t n_faces, const int32_t* faces);

/* --- hot path (device arrays) -------------------------------------------- */
/* F := -sum_e sum_g P(F_g) : grad N_a w_g  (2x2x2 Gauss)  +  the follower load
 * -pressure * integral N_a (dx/dxi x dx/deta) over the pressure faces.
 * X, F: [n_nodes][3]. */
hipib_status hipib_fe_force(hipib_ctx* ctx, const double* X, double pressure, double* F);
/* f += S(X) F:  f^d[idx] += sum_q F^d_q delta_h(x^d_idx - X_q).  f: [3][n^3].
 * ("Eulerian-Lagrangian coupling operators", spreading.)  Waits for
 * completion; HIPIB_E_NUMERIC if a position is non-finite or 1e9 cells or more
 * from the origin (such a node is spread at the origin). */
hipib_status hipib_spread(hipib_ctx* ctx, const double* X, const double* F, double* f);
/* hipib_spread without a context and without allocating, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): f += S(X) F on the periodic n^3
 * grid in FP64, with the kernels of hipib_spread on an FP64 context, atomic
 * mode.  X, F: device [n_nodes][3]; f: device [3][n^3], accumulated; stream: a
 * hipStream_t (NULL: the null stream); nothing waits for completion.  The node
 * bins live in a static device workspace of 13.1 MB per GPU (held until the
 * process ends): n must be 4*2^k or 6*2^k in [8, 256] and n_nodes at most
 * 1048576, else HIPIB_E_INVAL.  Positions are not checked (the call does not
 * wait): a non-finite one is spread at the origin.  Calls that overlap on one GPU (other streams,
 * other threads) share that workspace and race: order them.  The first call on
 * a device looks the workspace up (HIPIB_E_HIP if that fails). */
hipib_status hipib_spread_noalloc(int32_t n, int32_t n_nodes, const double* X, const double* F,
                                  double* f, void* stream);
/* U := J(X) u:  U^d_q = sum_idx u^d[idx] delta_h(x^d_idx - X_q) h^3
 * ("Eulerian-Lagrangian coupling operators", interpolation).  Waits for
 * completion; HIPIB_E_NUMERIC for a non-finite or out-of-range position, as
 * hipib_spread. */
hipib_status hipib_interpolate(hipib_ctx* ctx, const double* X, const double* u, double* U);
/* Solves (sigma I - nu Lap_h) x = b for ncomp independent components
 * (component stride n^3): Helmholtz sigma = rho/dt, nu = mu; Poisson sigma = 0,
 * nu = 1 (right-hand side must have zero mean; x is returned mean-free).  The
 * two elliptic solves of "Spatial Discretization" (first and second
 * equations) by the geometric multigrid the Abstract names: Poisson by
 * conjugate gradients preconditioned with one V(pre, post) cycle (mg_krylov),
 * Helmholtz by cycles whose hierarchy stops where the operator's Jacobi radius
 * is at most 1/2, relaxed there by red-black SOR with Young's factor.
 * x holds the initial guess on entry.  cycles/relres: host arrays [ncomp]
 * (may be NULL).  Waits for completion.  HIPIB_E_NOCONV after mg_max_cycles
 * cycles, HIPIB_E_NUMERIC for a non-finite residual. */
hipib_status hipib_mg_solve(hipib_ctx* ctx, int32_t op, int32_t ncomp, const double* b,
                            double* x, int32_t* cycles, double* relres);
/* One fluid step ("Spatial Discretization": the Chorin split with explicit
 * convection, "Temporal Discretization") with force density f ([3][n^3], may
 * be NULL = 0):
 *   ((rho/dt) I - mu Lap_h) u* = (rho/dt) u - rho C(u) + f   (guess u)
 *   (-Lap_h) p = -(rho/dt) D u* (mean removed)                 (guess p)
 *   u := u* - (dt/rho) G p.        u: [3][n^3] in/out, p: [n^3] in/out. */
hipib_status hipib_ns_step(hipib_ctx* ctx, const double* f, double* u, double* p);
/* One immersed-boundary step with explicit coupling ("Spatial
 * Discretization", last equation; "Eulerian-Lagrangian coupling operators"):
 * F(X^n) incl. pressure, f = S(X^n)F, ns_step, X += dt J(X^n) u^{n+1}.
 * X: [n_nodes][3] in/out.  HIPIB_E_NUMERIC for an inverted element (J <= 0 at
 * a Gauss point) or a non-finite or out-of-range position. */
hipib_status hipib_ib_step(hipib_ctx* ctx, double* u, double* p, double* X, double pressure);
/* n_steps IB steps (hipib_ib_step) from time t0 with cavity pressure
 * hipib_cavity_pressure(p0, T, t_n) (p0 sin^2(pi t_n / T), 0 when T <= 0),
 * t_n = t0 + n dt, and the active tension of hipib_set_active_waveform when
 * one is set (the left-ventricle model's loading, "Dynamic left ventricle
 * model"). */
hipib_status hipib_advance(hipib_ctx* ctx, double* u, double* p, double* X, double t0,
                           int32_t n_steps, double p0, double T);

/* Per-step records of the last hipib_advance / hipib_ib_step / hipib_ns_step
 * call: cycles[s][4] and relres[s][4] (Helmholtz x, y, z, Poisson) for
 * s < min(max_steps, steps recorded).  Returns the number of records. */
int32_t hipib_get_step_stats(hipib_ctx* ctx, int32_t* cycles, double* relres,
                             int32_t max_steps);

/* Phases of an immersed-boundary step, timed by hipib_set_phase_timing. */
typedef enum {
    HIPIB_PHASE_FORCES = 0,    /* element forces, pressure load, tethers (side stream) */
    HIPIB_PHASE_RHS = 1,       /* node binning and the fluid right-hand side */
    HIPIB_PHASE_SPREAD = 2,    /* spreading, after waiting for the forces */
    HIPIB_PHASE_HELMHOLTZ = 3, /* the three Helmholtz solves */
    HIPIB_PHASE_POISSON = 4,   /* divergence, mean removal, Poisson solve */
    HIPIB_PHASE_PROJECT = 5,   /* velocity correction */
    HIPIB_PHASE_INTERP = 6,    /* interpolation and position update */
    HIPIB_N_PHASES = 7
} hipib_phase;

typedef struct {
    /* the last hipib_advance / hipib_ib_step / hipib_ns_step call */
    int32_t steps;              /* steps it recorded */
    int32_t cycles_last[4];     /* multigrid cycles of its last step (Helmholtz x, y, z, Poisson) */
    double relres_last[4];      /* their final relative residuals */
    double cycles_mean[4];      /* mean cycles over its steps */
    /* phase timing (hipib_set_phase_timing) */
    int32_t timed_steps;        /* steps timed since timing was switched on */
    double phase_ms[HIPIB_N_PHASES];  /* their accumulated milliseconds per phase */
    /* of the positions X passed to hipib_get_stats (0 when X is NULL or there
     * are no elements): det F over all quadrature points, and the solid's
     * volume sum_e sum_q w_q det(dx/dxi) (its change is the paper's volume
     * conservation measure, "Benchmarks") */
    double J_min, J_max, volume;
    /* of the velocity u passed (0 when u is NULL): (rho/2) h^3 sum |u|^2 over the
     * face lattices, rho h^3 sum u^d, max over cells of |D u| (the discrete
     * divergence, sum_d (u^d[c + e_d] - u^d[c]) / h) */
    double kinetic_energy, momentum[3], max_abs_div;
} hipib_stats;

/* Run diagnostics: the records of the last step call, the phase times, and
 * the quantities above computed on the device from u ([3][n^3], may be NULL)
 * and X ([n_nodes][3], may be NULL; needs hipib_set_mesh).  out: host.
 * Waits for completion.  The per-workgroup partials are summed on the host in
 * a fixed order. */
hipib_status hipib_get_stats(hipib_ctx* ctx, const double* u, const double* X, hipib_stats* out);
/* enable != 0: every later hipib_ib_step / hipib_advance step of a periodic box
 * records HIP events at its phase boundaries and adds the phase durations
 * into the hipib_stats phase times (one extra wait per step); the counts
 * restart at zero.  enable = 0 switches it off.  Walled steps are not timed
 * by phase. */
hipib_status hipib_set_phase_timing(hipib_ctx* ctx, int32_t enable);
/* The cavity pressure p0 sin^2(pi t / T) of hipib_advance at time t (0 when
 * p0 = 0 or T <= 0): the load of the left-ventricle model's endocardium over
 * one beat ("Dynamic left ventricle model"); callers reversing an advance
 * (the adjoint rollout) take the same values from here. */
double hipib_cavity_pressure(double p0, double T, double t);

/* --- discrete adjoint ----------------------------------------------------
 * Reverse mode of hipib_ib_step for gradients of a loss L with respect to the
 * node positions and the Holzapfel-Ogden parameters (a, b, a_f, b_f) of each
 * material.  lam_* are dL/d(array entry) in the layout of the array.  The
 * multigrid solves are treated as exact inverses of their symmetric operators
 * (H = (rho/dt) I - mu Lap_h, and the projection P = I - G Lap_h^+ D), so the
 * transposed step runs the same solvers: interpolation is the transpose of
 * spreading, the force's transpose product is the strain-energy Hessian-vector
 * product, the projection's adjoint is the projection.  dtheta is a device
 * array [HIPIB_MAX_MATERIALS][4] that is accumulated into (+=); entries of
 * neo-Hookean materials stay unchanged.  The sheet, fibre-sheet and active
 * terms enter the Hessian products (so lam_X and lam_u are exact for the full
 * law) but their constants get no gradient. */
/* Reverse of one hipib_ib_step from (u_n, X_n) at cavity pressure `pressure`,
 * whose result velocity was u_np1.  lam_u in: dL/du^{n+1}, out: dL/du^n;
 * lam_X in: dL/dX^{n+1}, out: dL/dX^n.  The adjoint Poisson and Helmholtz
 * solves start from the previous call's solutions (zero on a context's first
 * call), as the forward solves start from the previous step's; results depend
 * on that start only within the multigrid tolerance.  On a walled box
 * (config walls = 1) the step is reversed on the mirror-image grid, each mirror
 * map by its transpose (extension by the fold onto the box, restriction by
 * zero padding); its adjoint solves also start from the previous call's
 * solutions.  The first call on a context allocates the reverse step's
 * workspaces (HIPIB_E_NOMEM if that fails).  Waits for completion. */
hipib_status hipib_adjoint_step(hipib_ctx* ctx, const double* u_n, const double* X_n,
                                const double* u_np1, double pressure, double* lam_u,
                                double* lam_X, double* dtheta);
/* Zeroes the starting points of the reverse step's adjoint solves (each
 * hipib_adjoint_step starts them from the previous call's solutions), so a
 * backward pass that calls this first gives the same gradients whatever
 * passes ran on the context before it.  Nothing to do before the first
 * hipib_adjoint_step.  Enqueued on the context's stream. */
hipib_status hipib_adjoint_reset(hipib_ctx* ctx);
/* HV := (dF_el/dX) V, the directional derivative of the elastic nodal force
 * (minus the strain-energy Hessian times V). */
hipib_status hipib_fe_hvp(hipib_ctx* ctx, const double* X, const double* V, double* HV);
/* dtheta += (dF_el/dtheta)^T lamF. */
hipib_status hipib_fe_param_vjp(hipib_ctx* ctx, const double* X, const double* lamF,
                                double* dtheta);
/* lamX += [d/dX (S(X) F)]^T lam_f   (lam_f: [3][n^3]). */
hipib_status hipib_spread_vjp_X(hipib_ctx* ctx, const double* X, const double* F,
                                const double* lam_f, double* lamX);
/* lamX += [d/dX (J(X) u)]^T lamU. */
hipib_status hipib_interp_vjp_X(hipib_ctx* ctx, const double* X, const double* u,
                                const double* lamU, double* lamX);
/* out := C'(u)^T lam, the transpose of the convection Jacobian ([3][n^3]). */
hipib_status hipib_convection_vjp(hipib_ctx* ctx, const double* u, const double* lam, double* out);

/* --- measurement -------------------------------------------------------- */
/* Kernel classes that can be timed with HIP events: each timed launch goes
 * through hipExtLaunchKernel with a start and a stop event, which take the
 * dispatch's own start and end timestamps on the stream it is launched on.
 * The algorithmic bytes of a launch are counted per cell of the level it works
 * on (FP64; n^3 cells, times the components the launch covers): */
typedef enum {
    HIPIB_TIMER_OFF = 0,
    /* red or black Gauss-Seidel half-sweep on the finest level of a Poisson
     * solve (not the first one from a zero guess): 12 B (read the other
     * colour's half of x and this colour's half of b, write this colour's x) */
    HIPIB_TIMER_SMOOTH_FINE_POISSON = 1,
    /* over-relaxed red or black half-sweep on the finest level of a Helmholtz
     * solve (on the iterate): 16 B per cell and component (also reads the
     * colour's own old x) */
    HIPIB_TIMER_SMOOTH_FINE_HELMHOLTZ = 2,
    /* finest-level red residual and its restriction: 13 B (x, red b, coarse b) */
    HIPIB_TIMER_RESID_RESTRICT = 3,
    /* finest-level coarse-grid correction: with at least two post-smoothing
     * sweeps folded into the first (black) post-smoothing half-sweep, 13 B
     * (that half-sweep's 12 B and the coarse correction); otherwise the
     * prolongation added to the red cells, 9 B */
    HIPIB_TIMER_PROLONG = 4,
    /* fused first coarse level, down half (four half-sweeps from zero,
     * residual, restriction): 17 B per cell of that level */
    HIPIB_TIMER_LEVEL_DOWN = 5,
    /* fused first coarse level, up half (prolongation, four half-sweeps): 21 B */
    HIPIB_TIMER_LEVEL_UP = 6,
    /* the coarsest level: its exact solve (one workgroup per component at
     * most 16^3; three plane-parallel passes at 24^3 and 32^3), or with
     * mg_coarse_sweeps > 0 the levels of at most 16^3 cells in one workgroup:
     * 16 B per cell of that level and pass (b read, x written) */
    HIPIB_TIMER_SMALL_VCYCLE = 7,
    /* residual norm of the finest level: 16 B per cell and component */
    HIPIB_TIMER_RESID_NORM = 8,
    /* conjugate-gradient passes: r.z and z.q (the preconditioner's last two
     * finest-level half-sweeps, which sum them: 16 B per cell in FP64; where
     * the finest level is the exactly solved one, a separate 24 B pass);
     * p, q = A z + beta q and p.q, 40 B; x, r updates and ||r||^2, 48 B */
    HIPIB_TIMER_CG_DOTS = 9,
    HIPIB_TIMER_CG_DIR = 10,
    HIPIB_TIMER_CG_UPDATE = 11,
    /* single-workgroup reductions of partials (stop tests, CG scalars): their
     * partials, 8 B each */
    HIPIB_TIMER_REDUCE = 12,
    /* fluid right-hand side 48 B (72 B with u^n packed as the Helmholtz guess
     * inside a step), divergence 32 B, velocity correction 56 B (64 B from the
     * packed u* and p inside a step), layout conversions 16 B per cell and
     * component */
    HIPIB_TIMER_RHS = 13,
    HIPIB_TIMER_DIVERGENCE = 14,
    HIPIB_TIMER_PROJECT = 15,
    HIPIB_TIMER_PACK = 16,
    /* spreading, interpolation (with the position update), element forces:
     * their bytes depend on the node positions and are not counted here
     * (reported as 0) */
    HIPIB_TIMER_SPREAD = 17,
    HIPIB_TIMER_INTERP = 18,
    HIPIB_TIMER_FE_FORCE = 19,
    HIPIB_N_TIMERS = 20
} hipib_timer;
/* Selects the timed kernel class and clears earlier timings. */
hipib_status hipib_timer_enable(hipib_ctx* ctx, int32_t which);
/* Waits for the stream, then returns the number of timed launches, their total
 * duration in milliseconds and the mean algorithmic bytes per launch; clears
 * the accumulated timings. */
hipib_status hipib_timer_read(hipib_ctx* ctx, int32_t* launches, double* total_ms,
                              double* bytes_per_launch);

#ifdef __cplusplus
}
#endif
#endif
