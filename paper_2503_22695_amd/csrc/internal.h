// Internal declarations of the hipib library (gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "hipib.h"

namespace hipib {

constexpr int kMaxLevels = 16;
constexpr int kSmallMax = 16;       // levels with n <= 16 run in one workgroup (LDS)
constexpr int kReduceBlock = 256;
constexpr int kSpreadChunk = 256;   // nodes per spreading work item (= its threads)

// upper bound on the number of spreading work items
inline int64_t spread_list_cap(int64_t ntiles, int64_t nn) {
    return ntiles + (nn + kSpreadChunk - 1) / kSpreadChunk + 1;
}

constexpr int kMatParams = 9;       // (a, b, a_f, b_f, kappa, a_s, b_s, a_fs, b_fs)

// Material table passed by value to the force kernels.
struct MatTable {
    int32_t model[HIPIB_MAX_MATERIALS];
    int32_t sheet[HIPIB_MAX_MATERIALS];   // 1: Holzapfel-Ogden with a_s or a_fs > 0
    double p[HIPIB_MAX_MATERIALS][kMatParams];
};

// Multigrid stop-decision state, kept on the device and mirrored to pinned host
// memory at each synchronisation point.
struct MGState {
    double bn[3];       // ||b||_2 per component
    double rn[3];       // ||r||_2 per component after the latest cycle
    double mean[3];     // Poisson: mean removed by the latest mean step
    int32_t active[3];  // 1 while the component still needs cycles
    int32_t cycles[3];  // cycles done
    int32_t zero_req[3];// ||b|| = 0: the solution is x = 0
    int32_t status;     // HIPIB_OK / HIPIB_E_NOCONV / HIPIB_E_NUMERIC
    int32_t numeric;    // set by the force kernel when J <= 0
    int32_t bad_position;  // set by the node binning for a non-finite or out-of-range position
    int32_t pad[2];
    // conjugate gradients (component 0): r.z, step alpha, direction update beta
    double rz, alpha, beta;
};

struct Level {
    int n = 0;
    int64_t n3 = 0;
    void* x = nullptr;     // [3][n3] packed, l >= 1, element type of the V-cycle
    void* b = nullptr;
    void* x2 = nullptr;    // [3][n3] x after pre-smoothing (levels run as fused halves)
};

struct StepRecord {
    int32_t cycles[4];
    double relres[4];
};

}  // namespace hipib

struct hipib_ctx {
    hipib_config cfg{};
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;         // element forces of ib_step, overlapping the fluid right-hand side
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int device = 0;
    int n = 0;
    int64_t n3 = 0;
    double h = 0.0;

    // multigrid hierarchy
    int L = 0;              // number of levels
    int small_start = 0;    // first level run by the single-workgroup kernel
    size_t small_lds = 0;   // its dynamic LDS bytes
    // exact solve of the coarsest level (mg_coarse_sweeps = 0): the level's real
    // Fourier basis Q [N][N] and eigenvalue factors s [N], FP64 and FP32 copies
    // set by a conjugate-gradient iteration around its preconditioner: r and q
    // for the dots fused into the finest level's last half-sweeps (parts: the
    // partials those wrote, 0 if none)
    struct CgDotsReq {
        const double* r = nullptr;
        const double* q = nullptr;
        int64_t parts = 0;
    } cg_dots;
    int exact_level = 0;    // first level with at most 32 cells per side (the exact coarsest level)
    void* coarse_work = nullptr;   // its transform array (24^3 and 32^3), 3 components
    double* coarse_tab = nullptr;
    float* coarse_tab32 = nullptr;
    hipib::Level lv[hipib::kMaxLevels];
    void* r0 = nullptr;     // [3][n3] residual scratch of the V-cycle type (any level)
    double* xp = nullptr;   // [3][n3] packed FP64 solution of the current solve
    double* sx = nullptr;   // the packed solution array the running solve iterates on (xp or bp)
    double* kv[4] = {nullptr, nullptr, nullptr, nullptr};  // [n3] packed CG vectors r, z, p, q
    double* bpk = nullptr;  // [3][n3] packed FP64 right-hand side
    float* e32 = nullptr;   // [3][n3] packed FP32 correction (mixed precision)
    float* r32 = nullptr;   // [3][n3] packed FP32 scaled residual (mixed precision)
    double* bp = nullptr;   // [n3] Poisson right-hand side (natural), or p packed during a step
    double* part = nullptr; // reduction partials
    int64_t part_cap = 0;
    hipib::MGState* st = nullptr;       // device
    hipib::MGState* st_host = nullptr;  // pinned host mirror
    int predicted[2] = {1, 1};          // cycles enqueued before the first check

    // Lagrangian mesh
    int32_t nn = 0, ne = 0, nf = 0;
    int npe = 8;              // nodes per element: 8 hexes, 4 P1 tets, 10 P2 tets
    bool mesh_set = false;
    double* Xref = nullptr;
    int32_t* conn = nullptr;  // [ne][npe]
    double* fibre = nullptr;
    int32_t* mat_id = nullptr;
    int32_t* faces = nullptr;
    double* F = nullptr;      // [nn][3] nodal force scratch

    // Eulerian tile bins of the nodes (counting sort by tile of T^3 cells)
    int tile = 8;             // T: 8 when n % 8 == 0, else 4
    int tiles_axis = 0;       // n / T
    int64_t ntiles = 0;
    int32_t* bin_count = nullptr;   // [ntiles] (kept zero between uses)
    int32_t* bin_off = nullptr;     // [ntiles + 1]
    int32_t* tile_list = nullptr;   // [spread_list_cap][2] spreading work items (tile, first rank)
    int32_t* n_list = nullptr;      // [1] number of work items
    int32_t* node_tile = nullptr;   // [nn]
    int32_t* node_rank = nullptr;   // [nn]
    int32_t* perm = nullptr;        // [nn] nodes grouped by tile
    uint32_t mat_used = 0;    // bit m: some element uses material m
    uint32_t mat_set = 0;     // bit m: material m defined
    hipib::MatTable mats{};
    double* sheet = nullptr;  // [ne][3] sheet directions (hipib_set_sheets), else null
    double active_ta = 0.0;   // T_a of the active fibre stress (Holzapfel-Ogden materials)
    double ta_max = 0.0, ta_t_on = 0.0, ta_duration = 0.0;  // waveform followed by advance
    // walled box (cfg.walls): the (2n)^3 periodic image context and its fields
    hipib_ctx* img = nullptr;
    double* w_u = nullptr;    // [3][M3] velocity image
    double* w_f = nullptr;    // [3][M3] force image
    double* w_g = nullptr;    // [3][M3] Helmholtz right-hand side image
    double* w_p = nullptr;    // [M3] pressure image
    double* w_b = nullptr;    // [M3] Poisson right-hand side image
    double* w_box = nullptr;  // [3][n3] box scratch
    double* w_fbox = nullptr; // [3][n3] folded force
    double* w_Xh = nullptr;   // [nn][3] positions on the image grid's unit box (X / 2)
    double* w_U = nullptr;    // [nn][3] interpolated velocity
    int32_t w_nn = -1;        // node count the node buffers are sized for
    double* w_ap = nullptr;   // [m^3] adjoint pressure of the walled reverse step (its solves' start)
    double* w_ah = nullptr;   // [3][m^3] adjoint Helmholtz solution of the walled reverse step
    int32_t nt = 0;                  // penalty tethers (hipib_set_tethers)
    int32_t* tether_node = nullptr;  // [nt] distinct node indices
    double* tether_Y = nullptr;      // [nt][3] targets
    double* tether_K = nullptr;      // [nt][6] symmetric stiffness xx, yy, zz, xy, xz, yz

    std::vector<hipib::StepRecord> recs;
    bool broken = false;

    // deterministic mode (allocated by set_mesh / set_pressure_faces)
    int32_t* det_node_off = nullptr;   // [nn + 1] CSR: node -> (element, local node) in element order
    int32_t* det_node_inc = nullptr;   // [npe ne] entries e * npe + a
    double* det_contrib = nullptr;     // [ne][npe][3] per-element nodal contributions
    double* det_param = nullptr;       // [ne][4] per-element parameter-gradient terms
    int32_t* det_face_off = nullptr;   // [nn + 1] CSR: node -> (face, local node)
    int32_t* det_face_inc = nullptr;   // [4 nf] entries f * 4 + a
    double* det_face_contrib = nullptr;  // [nf][4][3]
    uint32_t* det_key[2] = {nullptr, nullptr};  // node sort keys (cell index, tile-major)
    int32_t* det_idx[2] = {nullptr, nullptr};   // node numbers in key order
    int32_t* det_hist = nullptr;       // [256][det_nblk] digit counts, then offsets
    int32_t* det_lfirst = nullptr;     // [ntiles] work-list index of each tile's first item
    int32_t* det_active = nullptr;     // [ntiles] tiles some item's box reaches; then their count
    int32_t* det_nactive = nullptr;    // det_active + ntiles
    double* det_buf = nullptr;         // [spread_list_cap][3][(T + 4)^3] per-item spreading boxes
    int det_nblk = 0;                  // radix-sort workgroups
    int det_bits = 0;                  // bits of the largest cell key

    // adjoint workspaces (allocated on the first adjoint call)
    double* adj_tot = nullptr;   // [3][n3]
    double* adj_lg = nullptr;    // [3][n3]
    double* adj_p = nullptr;     // [n3]
    double* adj_sX = nullptr;    // [nn][3]
    double* adj_lamF = nullptr;  // [nn][3]
    int32_t adj_ready_nn = -1;

    // phase timing of ib_step (hipib_set_phase_timing): events on the context's
    // stream at the phase boundaries, and around the element forces on the side stream
    bool phase_timing = false;
    hipEvent_t ph_ev[8] = {};
    hipEvent_t ph_force[2] = {};
    double phase_ms[HIPIB_N_PHASES] = {};
    int64_t phase_steps = 0;

    // event timing of one kernel class (hipib_timer)
    int timer_which = 0;
    std::vector<hipEvent_t> ev_pool;   // pairs: start 2i, stop 2i+1
    size_t ev_used = 0;                // pairs recorded since the last read
    double timer_bytes = 0.0;          // algorithmic bytes of the timed launches
    int64_t timer_launches = 0;        // launches timed since the last read
};

namespace hipib {

// ---- error reporting (thread-local message) --------------------------------
hipib_status fail(hipib_status s, const char* fmt, ...);
hipib_status hip_fail(hipib_ctx* ctx, hipError_t e, const char* what, const char* file, int line);

#define HIPIB_HIP(call)                                                          \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) return ::hipib::hip_fail(ctx, e_, #call, __FILE__, __LINE__); \
    } while (0)

#define HIPIB_TRY(call)                      \
    do {                                     \
        hipib_status s_ = (call);            \
        if (s_ != HIPIB_OK) return s_;       \
    } while (0)

// stats.hip: the on-demand diagnostics of hipib_get_stats (u, X may be null)
hipib_status compute_stats(hipib_ctx* ctx, const double* u, const double* X, hipib_stats* out);

// ---- launchers (each file owns its kernels) ---------------------------------
// grid.hip
// g_packed: g is written in the packed red-black layout (pk) instead of the natural one
hipib_status launch_rhs_build(hipib_ctx* ctx, const double* u, const double* f, double* g,
                              double* upk = nullptr, bool g_packed = false);
// the fluid part of a step on the packed layout (g built and spread packed in
// bpk, u^n packed in xp): Helmholtz, divergence, Poisson, projection into u and p;
// mark(ctx, k) (optional) after each of the three phases, k = 3, 4, 5
hipib_status fluid_step_packed(hipib_ctx* ctx, double* u, double* p, int32_t* cyc, double* rr,
                               hipib_status (*mark)(hipib_ctx*, int));
hipib_status launch_divergence_rhs(hipib_ctx* ctx, const double* u, double* b);
hipib_status launch_project(hipib_ctx* ctx, double* u, const double* p);
hipib_status launch_zero(hipib_ctx* ctx, double* p, int64_t count);
// with explicit coefficients: g = rho_dt u - rho_conv C(u) + f; b = -coef D u; u -= coef G p
hipib_status launch_rhs_build_coef(hipib_ctx* ctx, const double* u, const double* f, double* g,
                                   double rho_dt, double rho_conv, double* upk = nullptr,
                                   bool g_packed = false);
hipib_status launch_divergence_rhs_coef(hipib_ctx* ctx, const double* u, double* b, double coef);
hipib_status launch_project_coef(hipib_ctx* ctx, double* u, const double* p, double coef);
// walls.hip (walled box through its mirror image)
hipib_status walled_create(hipib_ctx* ctx);
void walled_free(hipib_ctx* ctx);
hipib_status walled_set_nodes(hipib_ctx* ctx, const double* X_ref_host);
hipib_status walled_ns_step(hipib_ctx* ctx, const double* f, double* u, double* p);
hipib_status walled_ib_step(hipib_ctx* ctx, double* u, double* p, double* X, double pressure);
hipib_status walled_spread(hipib_ctx* ctx, const double* X, const double* F, double* f);
hipib_status walled_interpolate(hipib_ctx* ctx, const double* X, const double* u, double* U);
hipib_status walled_solve(hipib_ctx* ctx, int op, int ncomp, const double* b, double* x,
                          int32_t* cycles, double* relres);
hipib_status walled_adjoint_step(hipib_ctx* ctx, const double* u_n, const double* X_n,
                                 const double* u_np1, double pressure, double* lam_u, double* lam_X,
                                 double* dtheta);
// mg.hip
hipib_status mg_solve(hipib_ctx* ctx, int op, int ncomp, const double* b, double* x,
                      int32_t* cycles, double* relres);
hipib_status mg_remove_mean(hipib_ctx* ctx, double* v, int slot);
hipib_status mg_prepare(hipib_ctx* ctx);
size_t mg_level_elem_size(const hipib_ctx* ctx);
int64_t mg_partials_needed(int n);
hipib_status sync_state(hipib_ctx* ctx);
// after a binning of node positions and a synchronisation: HIPIB_E_NUMERIC if
// a position was non-finite or out of range (it was binned at the origin)
inline hipib_status position_status(const hipib_ctx* ctx) {
    if (ctx->st_host->bad_position)
        return fail(HIPIB_E_NUMERIC, "non-finite or out-of-range node position");
    return HIPIB_OK;
}
// ib.hip
hipib_status launch_bin(hipib_ctx* ctx, const double* X);
// f_packed: f is in the packed red-black layout (pk) instead of the natural one
hipib_status launch_spread(hipib_ctx* ctx, const double* X, const double* F, double* f,
                           bool f_packed = false);
hipib_status launch_interpolate(hipib_ctx* ctx, const double* X, const double* u, double* U,
                                double* Xupd, double dt);
// fe.hip
hipib_status launch_fe_force(hipib_ctx* ctx, const double* X, double pressure, double* F);
// tethers: out_a -= K (X_a - Y) (V null), or out_a -= K V_a (their force derivative along V)
hipib_status launch_tethers(hipib_ctx* ctx, const double* X, const double* V, double* out);
// det.hip (deterministic mode)
hipib_status det_prepare_mesh(hipib_ctx* ctx, const int32_t* conn);
hipib_status det_prepare_faces(hipib_ctx* ctx, const int32_t* faces, int nf);
hipib_status det_spread(hipib_ctx* ctx, const double* X, const double* F, double* f, bool f_packed);
// out (= or +=) per-node sums of det_contrib (faces: det_face_contrib) in element order
hipib_status det_gather_nodes(hipib_ctx* ctx, bool faces, bool accumulate, double* out);
hipib_status det_param_reduce(hipib_ctx* ctx, double* dtheta);
void det_free(hipib_ctx* ctx);
void det_free_faces(hipib_ctx* ctx);
// adjoint.hip
hipib_status adjoint_step(hipib_ctx* ctx, const double* u_n, const double* X_n, const double* u_np1,
                          double pressure, double* lam_u, double* lam_X, double* dtheta);
hipib_status launch_conv_vjp(hipib_ctx* ctx, const double* u, const double* lam, double* out,
                             double a, double b);
hipib_status adjoint_scratch(hipib_ctx* ctx);
hipib_status adjoint_forces(hipib_ctx* ctx, const double* X_n, double pressure, const double* lamF,
                            double* lam_X, double* dtheta);
hipib_status launch_fe_hvp(hipib_ctx* ctx, const double* X, const double* V, double* out);
hipib_status launch_fe_param_vjp(hipib_ctx* ctx, const double* X, const double* lamF, double* dtheta);
hipib_status launch_vjp_X(hipib_ctx* ctx, const double* X, const double* field, const double* coef,
                          double* lamX, double scale);

// ---- event timing --------------------------------------------------------------
// When launches of `kind` are being timed: takes the next event pair from the
// pool (the caller launches with hipExtLaunchKernelGGL, which stamps the
// dispatch's own start and end into them), counts the launch and returns true.
bool timer_events(hipib_ctx* ctx, int kind, double bytes, hipEvent_t* start, hipEvent_t* stop);

// Launches kernel k on the context's stream; when the timer is on for `kind`
// (a hipib_timer; 0: never timed), through hipExtLaunchKernel with the
// dispatch-stamped start and stop events of timer_events.  The arguments are
// converted to the kernel's parameter types.
template <typename... KArgs, typename... Args>
hipib_status launch_k(hipib_ctx* ctx, int kind, double bytes, void (*k)(KArgs...), dim3 grid,
                      dim3 block, size_t shmem, Args... args) {
    hipEvent_t t0, t1;
    if (kind != 0 && timer_events(ctx, kind, bytes, &t0, &t1))
        hipExtLaunchKernelGGL(k, grid, block, (uint32_t)shmem, ctx->stream, t0, t1, 0,
                              static_cast<KArgs>(args)...);
    else
        hipLaunchKernelGGL(k, grid, block, (uint32_t)shmem, ctx->stream, static_cast<KArgs>(args)...);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch", __FILE__, __LINE__);
    return HIPIB_OK;
}

// ---- small device helpers ----------------------------------------------------
__device__ __forceinline__ int wrap_idx(int i, int n) {
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// offset of cell (i,j,k) of an n^3 component in the packed red-black layout:
// the red cells ((i+j+k) even) first, then the black ones, each colour as
// rows of n/2 cells (i >> 1) ordered by j, then k
__device__ __forceinline__ int64_t pk(int i, int j, int k, int n) {
    const int q = (i + j + k) & 1;
    const int H = n >> 1;
    return (int64_t)q * ((int64_t)H * n * n) + (i >> 1) + (int64_t)H * ((int64_t)j + (int64_t)n * k);
}

// Sum over a workgroup of blockDim.x (multiple of 64, <= 1024) threads.
// Deterministic: fixed shuffle tree within each wavefront, fixed order across waves.
__device__ __forceinline__ double block_sum(double v, double* lds /*[16]*/) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) s += lds[w];
    }
    __syncthreads();
    return s;  // valid in thread 0
}

}  // namespace hipib
