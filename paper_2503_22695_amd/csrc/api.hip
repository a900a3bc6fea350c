// C-ABI entry points of libhipib: argument validation, context lifetime and
// the order of one immersed-boundary step ("Spatial Discretization"):
//   F = F_el(X^n) + F_pressure(X^n);  g = (rho/dt) u^n - rho C(u^n) + S(X^n) F;
//   ((rho/dt) - mu Lap_h) u* = g;  (-Lap_h) p = -(rho/dt) D u*;
//   u^{n+1} = u* - (dt/rho) G p;  X^{n+1} = X^n + dt J(X^n) u^{n+1}.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "internal.h"

namespace hipib {

static thread_local char g_err[512] = "";

hipib_status fail(hipib_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

hipib_status hip_fail(hipib_ctx* ctx, hipError_t e, const char* what, const char* file, int line) {
    if (ctx) ctx->broken = true;
    return fail(HIPIB_E_HIP, "HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e), what,
                file, line);
}

}  // namespace hipib

using namespace hipib;

namespace {

bool aligned8(const void* p) { return p != nullptr && (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

hipib_status check_ctx(hipib_ctx* ctx) {
    if (!ctx) return fail(HIPIB_E_INVAL, "null context");
    if (ctx->broken) return fail(HIPIB_E_HIP, "context unusable after an earlier HIP error");
    return HIPIB_OK;
}

hipib_status check_mesh_ready(hipib_ctx* ctx) {
    if (!ctx->mesh_set) return fail(HIPIB_E_STATE, "hipib_set_mesh has not been called");
    const uint32_t missing = ctx->mat_used & ~ctx->mat_set;
    if (missing) {
        for (int m = 0; m < HIPIB_MAX_MATERIALS; ++m)
            if (missing & (1u << m)) return fail(HIPIB_E_STATE, "material %d is used but not set", m);
    }
    if (!ctx->sheet && ctx->ne > 0)
        for (int m = 0; m < HIPIB_MAX_MATERIALS; ++m)
            if ((ctx->mat_used & (1u << m)) && ctx->mats.sheet[m])
                return fail(HIPIB_E_STATE, "material %d has sheet terms but no sheets are set", m);
    return HIPIB_OK;
}

template <typename T>
hipib_status dev_alloc(hipib_ctx* ctx, T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(HIPIB_E_NOMEM, "hipMalloc of %zu bytes failed", count * sizeof(T));
    }
    (void)ctx;
    return HIPIB_OK;
}

void free_mesh(hipib_ctx* ctx) {
    (void)hipFree(ctx->Xref);
    (void)hipFree(ctx->conn);
    (void)hipFree(ctx->fibre);
    (void)hipFree(ctx->sheet);
    (void)hipFree(ctx->tether_node);
    (void)hipFree(ctx->tether_Y);
    (void)hipFree(ctx->tether_K);
    ctx->tether_node = nullptr;
    ctx->tether_Y = ctx->tether_K = nullptr;
    ctx->nt = 0;
    (void)hipFree(ctx->mat_id);
    (void)hipFree(ctx->F);
    (void)hipFree(ctx->node_tile);
    (void)hipFree(ctx->node_rank);
    (void)hipFree(ctx->perm);
    ctx->node_tile = ctx->node_rank = ctx->perm = nullptr;
    det_free(ctx);
    det_free_faces(ctx);
    ctx->Xref = nullptr;
    ctx->conn = nullptr;
    ctx->fibre = nullptr;
    ctx->sheet = nullptr;
    ctx->mat_id = nullptr;
    ctx->F = nullptr;
    ctx->mesh_set = false;
    ctx->nn = ctx->ne = 0;
    ctx->mat_used = 0;
}

void free_all(hipib_ctx* ctx) {
    // the side stream's work is joined into the context's stream by every
    // ib_step; wait for it anyway before anything is freed
    if (ctx->side) {
        (void)hipStreamSynchronize(ctx->side);
        (void)hipStreamDestroy(ctx->side);
    }
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    ctx->side = nullptr;
    ctx->ev_fork = ctx->ev_join = nullptr;
    walled_free(ctx);
    free_mesh(ctx);
    (void)hipFree(ctx->faces);
    for (int l = 0; l < kMaxLevels; ++l) {
        (void)hipFree(ctx->lv[l].x);
        (void)hipFree(ctx->lv[l].b);
        (void)hipFree(ctx->lv[l].x2);
    }
    (void)hipFree(ctx->r0);
    (void)hipFree(ctx->xp);
    (void)hipFree(ctx->bpk);
    (void)hipFree(ctx->e32);
    for (int v = 0; v < 4; ++v) (void)hipFree(ctx->kv[v]);
    (void)hipFree(ctx->r32);
    (void)hipFree(ctx->bp);
    (void)hipFree(ctx->part);
    (void)hipFree(ctx->bin_count);
    (void)hipFree(ctx->bin_off);
    (void)hipFree(ctx->tile_list);
    (void)hipFree(ctx->n_list);
    (void)hipFree(ctx->st);
    if (ctx->st_host) (void)hipHostFree(ctx->st_host);
    (void)hipFree(ctx->adj_tot);
    (void)hipFree(ctx->adj_lg);
    (void)hipFree(ctx->adj_p);
    (void)hipFree(ctx->adj_sX);
    (void)hipFree(ctx->adj_lamF);
    (void)hipFree(ctx->coarse_tab);
    (void)hipFree(ctx->coarse_work);
    (void)hipFree(ctx->coarse_tab32);
    for (hipEvent_t e : ctx->ph_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->ph_force)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    ctx->ev_pool.clear();
}

void record_step(hipib_ctx* ctx, const int32_t* cyc, const double* rr) {
    StepRecord r;
    for (int t = 0; t < 4; ++t) {
        r.cycles[t] = cyc[t];
        r.relres[t] = rr[t];
    }
    ctx->recs.push_back(r);
}

// phase boundary k of a timed step (event on the context's stream)
hipib_status phase_mark(hipib_ctx* ctx, bool timed, int k) {
    if (timed) HIPIB_HIP(hipEventRecord(ctx->ph_ev[k], ctx->stream));
    return HIPIB_OK;
}

// fluid part of a step: g holds the Helmholtz right-hand side on entry;
// timed: phase events 3, 4, 5 after the Helmholtz solves, the Poisson solve
// and the projection
hipib_status mark_timed(hipib_ctx* ctx, int k) { return phase_mark(ctx, true, k); }

// (u^n packed into xp by the right-hand side builder)
hipib_status fluid_solves(hipib_ctx* ctx, double* u, double* p, bool timed = false) {
    int32_t cyc[4] = {0, 0, 0, 0};
    double rr[4] = {0, 0, 0, 0};
    HIPIB_TRY(fluid_step_packed(ctx, u, p, cyc, rr, timed ? mark_timed : nullptr));
    record_step(ctx, cyc, rr);
    return HIPIB_OK;
}

// adds the phase durations of a timed step (waits for its last event)
hipib_status phase_accumulate(hipib_ctx* ctx) {
    HIPIB_HIP(hipEventSynchronize(ctx->ph_ev[6]));
    float ms = 0.0f;
    HIPIB_HIP(hipEventElapsedTime(&ms, ctx->ph_force[0], ctx->ph_force[1]));
    ctx->phase_ms[HIPIB_PHASE_FORCES] += ms;
    for (int k = 1; k < HIPIB_N_PHASES; ++k) {
        HIPIB_HIP(hipEventElapsedTime(&ms, ctx->ph_ev[k - 1], ctx->ph_ev[k]));
        ctx->phase_ms[k] += ms;
    }
    ctx->phase_steps += 1;
    return HIPIB_OK;
}

hipib_status ib_step(hipib_ctx* ctx, double* u, double* p, double* X, double pressure) {
    if (ctx->cfg.walls) return walled_ib_step(ctx, u, p, X, pressure);
    // the element forces run on the side stream while the context's stream bins
    // the nodes and builds the fluid right-hand side (disjoint buffers); the
    // spreading waits for both
    const bool timed = ctx->phase_timing;
    HIPIB_TRY(phase_mark(ctx, timed, 0));
    HIPIB_HIP(hipEventRecord(ctx->ev_fork, ctx->stream));
    HIPIB_HIP(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
    if (timed) HIPIB_HIP(hipEventRecord(ctx->ph_force[0], ctx->side));
    hipStream_t own = ctx->stream;
    ctx->stream = ctx->side;
    const hipib_status fs = launch_fe_force(ctx, X, pressure, ctx->F);
    ctx->stream = own;
    HIPIB_TRY(fs);
    if (timed) HIPIB_HIP(hipEventRecord(ctx->ph_force[1], ctx->side));
    HIPIB_HIP(hipEventRecord(ctx->ev_join, ctx->side));
    HIPIB_TRY(launch_bin(ctx, X));
    HIPIB_TRY(launch_rhs_build(ctx, u, nullptr, ctx->bpk, ctx->xp, true));
    HIPIB_TRY(phase_mark(ctx, timed, 1));
    HIPIB_HIP(hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0));
    HIPIB_TRY(launch_spread(ctx, X, ctx->F, ctx->bpk, true));
    HIPIB_TRY(phase_mark(ctx, timed, 2));
    HIPIB_TRY(fluid_solves(ctx, u, p, timed));
    HIPIB_TRY(position_status(ctx));
    if (ctx->st_host->numeric)
        return fail(HIPIB_E_NUMERIC, "non-positive Jacobian at a Gauss point (inverted element)");
    HIPIB_TRY(launch_interpolate(ctx, X, u, nullptr, X, ctx->cfg.dt));
    HIPIB_TRY(phase_mark(ctx, timed, 6));
    if (timed) HIPIB_TRY(phase_accumulate(ctx));
    return HIPIB_OK;
}

}  // namespace

extern "C" {

void hipib_default_config(hipib_config* cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->n = 32;
    cfg->rho = 1.0;
    cfg->mu = 0.01;
    cfg->dt = 1e-3;
    cfg->mg_pre = 2;
    cfg->mg_post = 2;
    cfg->mg_max_cycles = 50;
    cfg->mg_fixed_cycles = 0;
    cfg->mg_coarse_sweeps = 0;
    cfg->mg_rtol = 1e-10;
    cfg->convection = 1;
    cfg->precision = HIPIB_FP64;
    cfg->deterministic = 0;
    cfg->mg_krylov = 1;
    cfg->walls = 0;
}

const char* hipib_last_error(void) { return g_err; }

hipib_status hipib_create(const hipib_config* cfg, void* stream, hipib_ctx** out) {
    if (!cfg || !out) return fail(HIPIB_E_INVAL, "null argument");
    *out = nullptr;
    const int n = cfg->n;
    if (n < 8 || n > 1024) return fail(HIPIB_E_INVAL, "n = %d outside [8, 1024]", n);
    {
        int m = n;
        while (m >= 8) {
            if (m % 2) return fail(HIPIB_E_INVAL, "n = %d: a multigrid level has odd size %d", n, m);
            m /= 2;
        }
        if (m != 4 && m != 6) return fail(HIPIB_E_INVAL, "n = %d is not 4*2^k or 6*2^k", n);
    }
    if (!(cfg->rho > 0) || !(cfg->mu > 0) || !(cfg->dt > 0))
        return fail(HIPIB_E_INVAL, "rho, mu and dt must be positive");
    if (cfg->mg_pre < 0 || cfg->mg_post < 0 || cfg->mg_max_cycles < 1 || cfg->mg_fixed_cycles < 0 ||
        cfg->mg_coarse_sweeps < 0 || !(cfg->mg_rtol >= 0))
        return fail(HIPIB_E_INVAL, "invalid multigrid parameters");
    if (cfg->precision != HIPIB_FP64 && cfg->precision != HIPIB_MIXED)
        return fail(HIPIB_E_INVAL, "unknown precision %d", cfg->precision);
    if (cfg->deterministic != 0 && cfg->deterministic != 1)
        return fail(HIPIB_E_INVAL, "deterministic must be 0 or 1");
    if (cfg->mg_krylov != 0 && cfg->mg_krylov != 1)
        return fail(HIPIB_E_INVAL, "mg_krylov must be 0 or 1");
    if (cfg->walls != 0 && cfg->walls != 1) return fail(HIPIB_E_INVAL, "walls must be 0 or 1");
    if (cfg->walls && 2 * n > 1024) return fail(HIPIB_E_INVAL, "walled box: 2n = %d > 1024", 2 * n);

    hipib_ctx* ctx = new hipib_ctx();
    ctx->cfg = *cfg;
    ctx->stream = static_cast<hipStream_t>(stream);
    (void)hipGetDevice(&ctx->device);
    ctx->n = n;
    ctx->n3 = (int64_t)n * n * n;
    ctx->h = 1.0 / n;
    int L = 0, m = n;
    while (true) {
        ctx->lv[L].n = m;
        ctx->lv[L].n3 = (int64_t)m * m * m;
        ++L;
        if (m < 8) break;
        m /= 2;
    }
    ctx->L = L;
    ctx->small_start = L - 1;
    for (int l = 0; l < L; ++l)
        if (ctx->lv[l].n <= kSmallMax) { ctx->small_start = l; break; }
    ctx->exact_level = L - 1;
    for (int l = 0; l < L; ++l)
        if (ctx->lv[l].n <= 32) { ctx->exact_level = l; break; }
    hipib_status s = HIPIB_OK;
    const size_t esz = mg_level_elem_size(ctx);
    auto alloc_bytes = [&](void** p, size_t bytes) {
        if (s != HIPIB_OK) return;
        hipError_t e = hipMalloc(p, bytes ? bytes : 1);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            s = fail(HIPIB_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
        }
    };
    for (int l = 1; l < L; ++l) {
        alloc_bytes(&ctx->lv[l].x, 3 * (size_t)ctx->lv[l].n3 * esz);
        alloc_bytes(&ctx->lv[l].b, 3 * (size_t)ctx->lv[l].n3 * esz);
    }
    // pre-smoothing arrays of the levels run as fused down/up halves
    for (int l = 1; l < ctx->small_start; ++l)
        if (ctx->lv[l].n % 8 == 0) alloc_bytes(&ctx->lv[l].x2, 3 * (size_t)ctx->lv[l].n3 * esz);
    alloc_bytes(&ctx->r0, 3 * (size_t)ctx->n3 * esz);
    if (s == HIPIB_OK) s = dev_alloc(ctx, &ctx->xp, 3 * (size_t)ctx->n3);
    if (s == HIPIB_OK) s = dev_alloc(ctx, &ctx->bpk, 3 * (size_t)ctx->n3);
    if (cfg->precision == HIPIB_MIXED) {
        if (s == HIPIB_OK) s = dev_alloc(ctx, &ctx->e32, 3 * (size_t)ctx->n3);
        if (s == HIPIB_OK) s = dev_alloc(ctx, &ctx->r32, 3 * (size_t)ctx->n3);
    }
    if (cfg->mg_krylov)   // conjugate-gradient vectors r, z, p, q of the Poisson solve
        for (int v = 0; v < 4 && s == HIPIB_OK; ++v) s = dev_alloc(ctx, &ctx->kv[v], (size_t)ctx->n3);
    if (s == HIPIB_OK) s = dev_alloc(ctx, &ctx->bp, (size_t)ctx->n3);
    ctx->tile = (n % 8 == 0) ? 8 : 4;
    ctx->tiles_axis = n / ctx->tile;
    ctx->ntiles = (int64_t)ctx->tiles_axis * ctx->tiles_axis * ctx->tiles_axis;
    if (s == HIPIB_OK) s = dev_alloc(ctx, &ctx->bin_count, (size_t)ctx->ntiles);
    if (s == HIPIB_OK) s = dev_alloc(ctx, &ctx->bin_off, (size_t)ctx->ntiles + 1);
    if (s == HIPIB_OK) s = dev_alloc(ctx, &ctx->tile_list, 2 * (size_t)spread_list_cap(ctx->ntiles, 0));
    if (s == HIPIB_OK) s = dev_alloc(ctx, &ctx->n_list, 1);
    ctx->part_cap = mg_partials_needed(n);
    if (s == HIPIB_OK) s = dev_alloc(ctx, &ctx->part, (size_t)ctx->part_cap);
    if (s == HIPIB_OK) s = dev_alloc(ctx, &ctx->st, 1);
    if (s == HIPIB_OK) {
        hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&ctx->st_host), sizeof(MGState));
        if (e != hipSuccess) s = fail(HIPIB_E_NOMEM, "pinned host allocation failed");
        else std::memset(ctx->st_host, 0, sizeof(MGState));
    }
    if (s == HIPIB_OK) {
        // default priority, like the context's own stream
        hipError_t e = hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming);
        if (e != hipSuccess) s = fail(HIPIB_E_HIP, "HIP error %d creating the side stream", (int)e);
    }
    if (s == HIPIB_OK) s = mg_prepare(ctx);
    if (s == HIPIB_OK && cfg->walls) s = walled_create(ctx);
    if (s == HIPIB_OK) {
        hipError_t e = hipMemsetAsync(ctx->st, 0, sizeof(MGState), ctx->stream);
        if (e == hipSuccess)
            e = hipMemsetAsync(ctx->bin_count, 0, sizeof(int32_t) * (size_t)ctx->ntiles, ctx->stream);
        if (e == hipSuccess) e = hipMemsetAsync(ctx->n_list, 0, sizeof(int32_t), ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) s = fail(HIPIB_E_HIP, "HIP error %d initialising the context", (int)e);
    }
    if (s != HIPIB_OK) {
        free_all(ctx);
        delete ctx;
        return s;
    }
    *out = ctx;
    return HIPIB_OK;
}

hipib_status hipib_destroy(hipib_ctx* ctx) {
    if (!ctx) return HIPIB_OK;
    (void)hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    delete ctx;
    return HIPIB_OK;
}

hipib_status hipib_set_stream(hipib_ctx* ctx, void* stream) {
    HIPIB_TRY(check_ctx(ctx));
    hipStream_t next = static_cast<hipStream_t>(stream);
    if (next == ctx->stream) return HIPIB_OK;
    // work still enqueued on the old stream (a step's interpolation and
    // position update, for one) is ordered before anything on the new one
    HIPIB_HIP(hipEventRecord(ctx->ev_fork, ctx->stream));
    HIPIB_HIP(hipStreamWaitEvent(next, ctx->ev_fork, 0));
    ctx->stream = next;
    return HIPIB_OK;
}

hipib_status hipib_set_mesh(hipib_ctx* ctx, int32_t n_nodes, const double* X_ref, int32_t n_elems,
                            const int32_t* conn, const double* fibre, const int32_t* mat_id) {
    return hipib_set_mesh_elements(ctx, n_nodes, X_ref, n_elems, 8, conn, fibre, mat_id);
}

hipib_status hipib_set_mesh_elements(hipib_ctx* ctx, int32_t n_nodes, const double* X_ref,
                                     int32_t n_elems, int32_t nodes_per_elem, const int32_t* conn,
                                     const double* fibre, const int32_t* mat_id) {
    HIPIB_TRY(check_ctx(ctx));
    const int npe = nodes_per_elem;
    if (npe != 8 && npe != 4 && npe != 10)
        return fail(HIPIB_E_INVAL, "nodes_per_elem = %d (8, 4 or 10)", npe);
    if (n_nodes < 0 || n_elems < 0) return fail(HIPIB_E_INVAL, "negative mesh size");
    if (n_elems > 0 && n_nodes == 0) return fail(HIPIB_E_INVAL, "elements without nodes");
    if (n_nodes > 0 && !X_ref) return fail(HIPIB_E_INVAL, "null X_ref");
    if (n_elems > 0 && (!conn || !fibre || !mat_id)) return fail(HIPIB_E_INVAL, "null element array");
    uint32_t used = 0;
    for (int64_t t = 0; t < npe * (int64_t)n_elems; ++t)
        if (conn[t] < 0 || conn[t] >= n_nodes)
            return fail(HIPIB_E_INVAL, "conn[%lld] = %d out of range", (long long)t, conn[t]);
    for (int32_t e = 0; e < n_elems; ++e) {
        if (mat_id[e] < 0 || mat_id[e] >= HIPIB_MAX_MATERIALS)
            return fail(HIPIB_E_INVAL, "mat_id[%d] = %d out of range", e, mat_id[e]);
        used |= 1u << mat_id[e];
    }
    for (int64_t t = 0; t < 3 * (int64_t)n_nodes; ++t)
        if (!std::isfinite(X_ref[t])) return fail(HIPIB_E_INVAL, "non-finite X_ref");
    for (int64_t t = 0; t < 3 * (int64_t)n_elems; ++t)
        if (!std::isfinite(fibre[t])) return fail(HIPIB_E_INVAL, "non-finite fibre");
    HIPIB_HIP(hipStreamSynchronize(ctx->stream));
    free_mesh(ctx);
    // pressure faces refer to the previous mesh's nodes: drop them
    (void)hipFree(ctx->faces);
    ctx->faces = nullptr;
    ctx->nf = 0;
    HIPIB_TRY(dev_alloc(ctx, &ctx->Xref, 3 * (size_t)n_nodes));
    HIPIB_TRY(dev_alloc(ctx, &ctx->F, 3 * (size_t)n_nodes));
    HIPIB_TRY(dev_alloc(ctx, &ctx->conn, npe * (size_t)n_elems));
    HIPIB_TRY(dev_alloc(ctx, &ctx->fibre, 3 * (size_t)n_elems));
    HIPIB_TRY(dev_alloc(ctx, &ctx->mat_id, (size_t)n_elems));
    HIPIB_TRY(dev_alloc(ctx, &ctx->node_tile, (size_t)n_nodes));
    HIPIB_TRY(dev_alloc(ctx, &ctx->node_rank, (size_t)n_nodes));
    HIPIB_TRY(dev_alloc(ctx, &ctx->perm, (size_t)n_nodes));
    (void)hipFree(ctx->tile_list);
    ctx->tile_list = nullptr;
    HIPIB_TRY(dev_alloc(ctx, &ctx->tile_list, 2 * (size_t)spread_list_cap(ctx->ntiles, n_nodes)));
    if (n_nodes > 0)
        HIPIB_HIP(hipMemcpy(ctx->Xref, X_ref, 3 * sizeof(double) * n_nodes, hipMemcpyHostToDevice));
    if (n_elems > 0) {
        HIPIB_HIP(hipMemcpy(ctx->conn, conn, npe * sizeof(int32_t) * n_elems, hipMemcpyHostToDevice));
        HIPIB_HIP(hipMemcpy(ctx->fibre, fibre, 3 * sizeof(double) * n_elems, hipMemcpyHostToDevice));
        HIPIB_HIP(hipMemcpy(ctx->mat_id, mat_id, sizeof(int32_t) * n_elems, hipMemcpyHostToDevice));
    }
    ctx->nn = n_nodes;
    ctx->ne = n_elems;
    ctx->npe = npe;
    ctx->mat_used = used;
    if (ctx->cfg.walls) {
        hipib_status sw = walled_set_nodes(ctx, X_ref);
        if (sw != HIPIB_OK) {
            free_mesh(ctx);
            return sw;
        }
    }
    if (ctx->cfg.deterministic) {
        hipib_status sd = det_prepare_mesh(ctx, conn);
        if (sd == HIPIB_OK) sd = det_prepare_faces(ctx, nullptr, 0);
        if (sd != HIPIB_OK) {
            free_mesh(ctx);
            return sd;
        }
    }
    ctx->mesh_set = true;
    return HIPIB_OK;
}

hipib_status hipib_set_material(hipib_ctx* ctx, int32_t mat_id, int32_t model, const double* params,
                                int32_t n_params) {
    HIPIB_TRY(check_ctx(ctx));
    if (mat_id < 0 || mat_id >= HIPIB_MAX_MATERIALS) return fail(HIPIB_E_INVAL, "mat_id out of range");
    if (!params) return fail(HIPIB_E_INVAL, "null params");
    double p[kMatParams] = {};
    if (model == HIPIB_NEO_HOOKEAN) {
        if (n_params != 2) return fail(HIPIB_E_INVAL, "neo-Hookean takes (mu_s, kappa)");
    } else if (model == HIPIB_STANDARD_REINFORCING) {
        if (n_params != 4) return fail(HIPIB_E_INVAL, "standard reinforcing takes (G_T, G_L, E_L, kappa)");
    } else if (model == HIPIB_FIBRE_REINFORCED_1) {
        if (n_params != 4) return fail(HIPIB_E_INVAL, "fibre-reinforced 1 takes (C_1, a_f, b_f, kappa)");
    } else if (model == HIPIB_FIBRE_REINFORCED_2) {
        if (n_params != 5)
            return fail(HIPIB_E_INVAL, "fibre-reinforced 2 takes (C_10, C_01, a_f, b_f, kappa)");
    } else if (model == HIPIB_HOLZAPFEL_OGDEN) {
        if (n_params != 5 && n_params != kMatParams)
            return fail(HIPIB_E_INVAL,
                        "Holzapfel-Ogden takes (a, b, a_f, b_f, kappa[, a_s, b_s, a_fs, b_fs])");
    } else {
        return fail(HIPIB_E_INVAL, "unknown material model %d", model);
    }
    for (int t = 0; t < n_params; ++t) {
        if (!std::isfinite(params[t])) return fail(HIPIB_E_INVAL, "non-finite parameter");
        p[t] = params[t];
    }
    if (model == HIPIB_NEO_HOOKEAN) {
        if (!(p[0] >= 0) || !(p[1] >= 0)) return fail(HIPIB_E_INVAL, "negative modulus");
    } else if (model == HIPIB_STANDARD_REINFORCING) {
        if (!(p[0] >= 0) || !(p[1] >= 0) || !(p[2] >= 0) || !(p[3] >= 0))
            return fail(HIPIB_E_INVAL, "negative modulus");
    } else if (model == HIPIB_FIBRE_REINFORCED_1) {
        if (!(p[0] >= 0) || !(p[1] >= 0) || !(p[2] > 0) || !(p[3] >= 0))
            return fail(HIPIB_E_INVAL, "fibre-reinforced 1 needs C_1, a_f, kappa >= 0 and b_f > 0");
    } else if (model == HIPIB_FIBRE_REINFORCED_2) {
        if (!(p[0] >= 0) || !(p[1] > 0) || !(p[2] >= 0) || !(p[3] > 0) || !(p[4] >= 0))
            return fail(HIPIB_E_INVAL, "fibre-reinforced 2 needs C_10, a_f, kappa >= 0 and C_01, b_f > 0");
    } else {
        if (!(p[0] >= 0) || !(p[1] > 0) || !(p[2] >= 0) || !(p[3] > 0) || !(p[4] >= 0))
            return fail(HIPIB_E_INVAL, "Holzapfel-Ogden needs a, a_f, kappa >= 0 and b, b_f > 0");
        if (!(p[5] >= 0) || !(p[6] >= 0) || !(p[7] >= 0) || !(p[8] >= 0) ||
            (p[5] > 0 && !(p[6] > 0)) || (p[7] > 0 && !(p[8] > 0)))
            return fail(HIPIB_E_INVAL, "sheet terms need a_s, a_fs >= 0 and b_s, b_fs > 0 where used");
    }
    ctx->mats.model[mat_id] = model;
    ctx->mats.sheet[mat_id] = (model == HIPIB_HOLZAPFEL_OGDEN && (p[5] > 0 || p[7] > 0)) ? 1 : 0;
    for (int t = 0; t < kMatParams; ++t) ctx->mats.p[mat_id][t] = p[t];
    ctx->mat_set |= 1u << mat_id;
    return HIPIB_OK;
}

hipib_status hipib_set_sheets(hipib_ctx* ctx, int32_t n_elems, const double* sheet) {
    HIPIB_TRY(check_ctx(ctx));
    if (!ctx->mesh_set) return fail(HIPIB_E_STATE, "hipib_set_mesh has not been called");
    if (n_elems != ctx->ne) return fail(HIPIB_E_INVAL, "n_elems %d != mesh's %d", n_elems, ctx->ne);
    if (n_elems > 0 && !sheet) return fail(HIPIB_E_INVAL, "null sheet");
    for (int64_t t = 0; t < 3 * (int64_t)n_elems; ++t)
        if (!std::isfinite(sheet[t])) return fail(HIPIB_E_INVAL, "non-finite sheet");
    HIPIB_HIP(hipStreamSynchronize(ctx->stream));
    (void)hipFree(ctx->sheet);
    ctx->sheet = nullptr;
    double* d = nullptr;
    HIPIB_TRY(dev_alloc(ctx, &d, 3 * (size_t)n_elems));
    if (n_elems > 0) {
        hipError_t e = hipMemcpy(d, sheet, 3 * sizeof(double) * n_elems, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            return hip_fail(ctx, e, "hipMemcpy(sheet)", __FILE__, __LINE__);
        }
    }
    ctx->sheet = d;
    return HIPIB_OK;
}

hipib_status hipib_set_tethers(hipib_ctx* ctx, int32_t n_tethers, const int32_t* node,
                               const double* target, const double* K) {
    HIPIB_TRY(check_ctx(ctx));
    if (!ctx->mesh_set) return fail(HIPIB_E_STATE, "hipib_set_mesh has not been called");
    if (n_tethers < 0 || (n_tethers > 0 && (!node || !target || !K)))
        return fail(HIPIB_E_INVAL, "bad tether arrays");
    std::vector<char> seen((size_t)ctx->nn, 0);
    for (int32_t t = 0; t < n_tethers; ++t) {
        if (node[t] < 0 || node[t] >= ctx->nn)
            return fail(HIPIB_E_INVAL, "tether node[%d] = %d out of range", t, node[t]);
        if (seen[node[t]]) return fail(HIPIB_E_INVAL, "node %d tethered twice", node[t]);
        seen[node[t]] = 1;
    }
    for (int64_t t = 0; t < 3 * (int64_t)n_tethers; ++t)
        if (!std::isfinite(target[t])) return fail(HIPIB_E_INVAL, "non-finite tether target");
    for (int64_t t = 0; t < 6 * (int64_t)n_tethers; ++t)
        if (!std::isfinite(K[t])) return fail(HIPIB_E_INVAL, "non-finite tether stiffness");
    HIPIB_HIP(hipStreamSynchronize(ctx->stream));
    (void)hipFree(ctx->tether_node);
    (void)hipFree(ctx->tether_Y);
    (void)hipFree(ctx->tether_K);
    ctx->tether_node = nullptr;
    ctx->tether_Y = ctx->tether_K = nullptr;
    ctx->nt = 0;
    if (n_tethers == 0) return HIPIB_OK;
    HIPIB_TRY(dev_alloc(ctx, &ctx->tether_node, (size_t)n_tethers));
    HIPIB_TRY(dev_alloc(ctx, &ctx->tether_Y, 3 * (size_t)n_tethers));
    HIPIB_TRY(dev_alloc(ctx, &ctx->tether_K, 6 * (size_t)n_tethers));
    HIPIB_HIP(hipMemcpy(ctx->tether_node, node, sizeof(int32_t) * n_tethers, hipMemcpyHostToDevice));
    HIPIB_HIP(hipMemcpy(ctx->tether_Y, target, 3 * sizeof(double) * n_tethers, hipMemcpyHostToDevice));
    HIPIB_HIP(hipMemcpy(ctx->tether_K, K, 6 * sizeof(double) * n_tethers, hipMemcpyHostToDevice));
    ctx->nt = n_tethers;
    return HIPIB_OK;
}

hipib_status hipib_set_active_tension(hipib_ctx* ctx, double Ta) {
    HIPIB_TRY(check_ctx(ctx));
    if (!std::isfinite(Ta)) return fail(HIPIB_E_INVAL, "non-finite active tension");
    ctx->active_ta = Ta;
    return HIPIB_OK;
}

double hipib_active_tension(double ta_max, double t_on, double duration, double t) {
    if (ta_max == 0.0 || !(duration > 0.0)) return 0.0;
    const double s = 0.5 + 0.3 * (t - t_on) / duration;
    if (s > 0.5 && s < 0.65) return ta_max * (1.0 - std::exp(-(s - 0.5) * (s - 0.5) / 0.005));
    if (s >= 0.65 && s < 0.8) return ta_max * (1.0 - std::exp(-(0.8 - s) * (0.8 - s) / 0.005));
    return 0.0;
}

hipib_status hipib_set_active_waveform(hipib_ctx* ctx, double ta_max, double t_on, double duration) {
    HIPIB_TRY(check_ctx(ctx));
    if (!std::isfinite(ta_max) || !std::isfinite(t_on) || !std::isfinite(duration) || duration < 0)
        return fail(HIPIB_E_INVAL, "bad active-tension waveform");
    ctx->ta_max = ta_max;
    ctx->ta_t_on = t_on;
    ctx->ta_duration = duration;
    return HIPIB_OK;
}

hipib_status hipib_set_pressure_faces(hipib_ctx* ctx, int32_t n_faces, const int32_t* faces) {
    HIPIB_TRY(check_ctx(ctx));
    if (!ctx->mesh_set) return fail(HIPIB_E_STATE, "hipib_set_mesh has not been called");
    if (n_faces < 0 || (n_faces > 0 && !faces)) return fail(HIPIB_E_INVAL, "bad faces");
    for (int64_t t = 0; t < 4 * (int64_t)n_faces; ++t)
        if (faces[t] < 0 || faces[t] >= ctx->nn)
            return fail(HIPIB_E_INVAL, "faces[%lld] = %d out of range", (long long)t, faces[t]);
    HIPIB_HIP(hipStreamSynchronize(ctx->stream));
    (void)hipFree(ctx->faces);
    ctx->faces = nullptr;
    ctx->nf = 0;
    HIPIB_TRY(dev_alloc(ctx, &ctx->faces, 4 * (size_t)n_faces));
    if (n_faces > 0)
        HIPIB_HIP(hipMemcpy(ctx->faces, faces, 4 * sizeof(int32_t) * n_faces, hipMemcpyHostToDevice));
    if (ctx->cfg.deterministic) HIPIB_TRY(det_prepare_faces(ctx, faces, n_faces));
    ctx->nf = n_faces;
    return HIPIB_OK;
}

hipib_status hipib_fe_force(hipib_ctx* ctx, const double* X, double pressure, double* F) {
    HIPIB_TRY(check_ctx(ctx));
    HIPIB_TRY(check_mesh_ready(ctx));
    if (ctx->nn > 0 && (!aligned8(X) || !aligned8(F))) return fail(HIPIB_E_INVAL, "bad X or F pointer");
    if (!std::isfinite(pressure)) return fail(HIPIB_E_INVAL, "non-finite pressure");
    return launch_fe_force(ctx, X, pressure, F);
}

hipib_status hipib_spread(hipib_ctx* ctx, const double* X, const double* F, double* f) {
    HIPIB_TRY(check_ctx(ctx));
    if (!ctx->mesh_set) return fail(HIPIB_E_STATE, "hipib_set_mesh has not been called");
    if (!aligned8(f) || (ctx->nn > 0 && (!aligned8(X) || !aligned8(F))))
        return fail(HIPIB_E_INVAL, "bad pointer");
    if (ctx->cfg.walls) {
        HIPIB_TRY(walled_spread(ctx, X, F, f));
        HIPIB_TRY(sync_state(ctx->img));
        return position_status(ctx->img);
    }
    HIPIB_TRY(launch_bin(ctx, X));
    HIPIB_TRY(launch_spread(ctx, X, F, f));
    HIPIB_TRY(sync_state(ctx));
    return position_status(ctx);
}

hipib_status hipib_interpolate(hipib_ctx* ctx, const double* X, const double* u, double* U) {
    HIPIB_TRY(check_ctx(ctx));
    if (!ctx->mesh_set) return fail(HIPIB_E_STATE, "hipib_set_mesh has not been called");
    if (!aligned8(u) || (ctx->nn > 0 && (!aligned8(X) || !aligned8(U))))
        return fail(HIPIB_E_INVAL, "bad pointer");
    if (ctx->cfg.walls) {
        HIPIB_TRY(walled_interpolate(ctx, X, u, U));
        HIPIB_TRY(sync_state(ctx->img));
        return position_status(ctx->img);
    }
    HIPIB_TRY(launch_bin(ctx, X));
    HIPIB_TRY(launch_interpolate(ctx, X, u, U, nullptr, 0.0));
    HIPIB_TRY(sync_state(ctx));
    return position_status(ctx);
}

hipib_status hipib_mg_solve(hipib_ctx* ctx, int32_t op, int32_t ncomp, const double* b, double* x,
                            int32_t* cycles, double* relres) {
    HIPIB_TRY(check_ctx(ctx));
    if (op != HIPIB_OP_HELMHOLTZ && op != HIPIB_OP_POISSON) return fail(HIPIB_E_INVAL, "unknown op");
    if (ncomp < 1 || ncomp > 3) return fail(HIPIB_E_INVAL, "ncomp must be 1..3");
    if (!aligned8(b) || !aligned8(x)) return fail(HIPIB_E_INVAL, "bad pointer");
    if (ctx->cfg.walls) return walled_solve(ctx, op, ncomp, b, x, cycles, relres);
    return mg_solve(ctx, op, ncomp, b, x, cycles, relres);
}

hipib_status hipib_ns_step(hipib_ctx* ctx, const double* f, double* u, double* p) {
    HIPIB_TRY(check_ctx(ctx));
    if (!aligned8(u) || !aligned8(p) || (f && !aligned8(f))) return fail(HIPIB_E_INVAL, "bad pointer");
    ctx->recs.clear();
    if (ctx->cfg.walls) return walled_ns_step(ctx, f, u, p);
    HIPIB_TRY(launch_rhs_build(ctx, u, f, ctx->bpk, ctx->xp, true));
    return fluid_solves(ctx, u, p);
}

hipib_status hipib_ib_step(hipib_ctx* ctx, double* u, double* p, double* X, double pressure) {
    HIPIB_TRY(check_ctx(ctx));
    HIPIB_TRY(check_mesh_ready(ctx));
    if (!aligned8(u) || !aligned8(p) || (ctx->nn > 0 && !aligned8(X)))
        return fail(HIPIB_E_INVAL, "bad pointer");
    if (!std::isfinite(pressure)) return fail(HIPIB_E_INVAL, "non-finite pressure");
    ctx->recs.clear();
    return ib_step(ctx, u, p, X, pressure);
}

hipib_status hipib_advance(hipib_ctx* ctx, double* u, double* p, double* X, double t0,
                           int32_t n_steps, double p0, double T) {
    HIPIB_TRY(check_ctx(ctx));
    HIPIB_TRY(check_mesh_ready(ctx));
    if (!aligned8(u) || !aligned8(p) || (ctx->nn > 0 && !aligned8(X)))
        return fail(HIPIB_E_INVAL, "bad pointer");
    if (n_steps < 0 || !std::isfinite(t0) || !std::isfinite(p0) || !std::isfinite(T))
        return fail(HIPIB_E_INVAL, "bad time arguments");
    ctx->recs.clear();
    for (int32_t s = 0; s < n_steps; ++s) {
        const double t = t0 + s * ctx->cfg.dt;
        const double pr = hipib_cavity_pressure(p0, T, t);
        if (ctx->ta_max != 0.0)
            ctx->active_ta = hipib_active_tension(ctx->ta_max, ctx->ta_t_on, ctx->ta_duration, t);
        HIPIB_TRY(ib_step(ctx, u, p, X, pr));
    }
    return HIPIB_OK;
}

hipib_status hipib_adjoint_step(hipib_ctx* ctx, const double* u_n, const double* X_n,
                                const double* u_np1, double pressure, double* lam_u,
                                double* lam_X, double* dtheta) {
    HIPIB_TRY(check_ctx(ctx));
    HIPIB_TRY(check_mesh_ready(ctx));
    if (!aligned8(u_n) || !aligned8(u_np1) || !aligned8(lam_u) || !aligned8(dtheta) ||
        (ctx->nn > 0 && (!aligned8(X_n) || !aligned8(lam_X))))
        return fail(HIPIB_E_INVAL, "bad pointer");
    if (!std::isfinite(pressure)) return fail(HIPIB_E_INVAL, "non-finite pressure");
    if (ctx->cfg.walls) return walled_adjoint_step(ctx, u_n, X_n, u_np1, pressure, lam_u, lam_X, dtheta);
    return adjoint_step(ctx, u_n, X_n, u_np1, pressure, lam_u, lam_X, dtheta);
}

hipib_status hipib_adjoint_reset(hipib_ctx* ctx) {
    HIPIB_TRY(check_ctx(ctx));
    if (ctx->adj_lg) HIPIB_TRY(launch_zero(ctx, ctx->adj_lg, 3 * ctx->n3));
    if (ctx->adj_p) HIPIB_TRY(launch_zero(ctx, ctx->adj_p, ctx->n3));
    if (ctx->cfg.walls && ctx->img) {
        if (ctx->w_ap) HIPIB_TRY(launch_zero(ctx, ctx->w_ap, ctx->img->n3));
        if (ctx->w_ah) HIPIB_TRY(launch_zero(ctx, ctx->w_ah, 3 * ctx->img->n3));
    }
    return HIPIB_OK;
}

hipib_status hipib_fe_hvp(hipib_ctx* ctx, const double* X, const double* V, double* HV) {
    HIPIB_TRY(check_ctx(ctx));
    HIPIB_TRY(check_mesh_ready(ctx));
    if (ctx->nn > 0 && (!aligned8(X) || !aligned8(V) || !aligned8(HV)))
        return fail(HIPIB_E_INVAL, "bad pointer");
    return launch_fe_hvp(ctx, X, V, HV);
}

hipib_status hipib_fe_param_vjp(hipib_ctx* ctx, const double* X, const double* lamF,
                                double* dtheta) {
    HIPIB_TRY(check_ctx(ctx));
    HIPIB_TRY(check_mesh_ready(ctx));
    if (!aligned8(dtheta) || (ctx->nn > 0 && (!aligned8(X) || !aligned8(lamF))))
        return fail(HIPIB_E_INVAL, "bad pointer");
    return launch_fe_param_vjp(ctx, X, lamF, dtheta);
}

hipib_status hipib_spread_vjp_X(hipib_ctx* ctx, const double* X, const double* F,
                                const double* lam_f, double* lamX) {
    HIPIB_TRY(check_ctx(ctx));
    if (!ctx->mesh_set) return fail(HIPIB_E_STATE, "hipib_set_mesh has not been called");
    if (!aligned8(lam_f) || (ctx->nn > 0 && (!aligned8(X) || !aligned8(F) || !aligned8(lamX))))
        return fail(HIPIB_E_INVAL, "bad pointer");
    if (ctx->cfg.walls) return fail(HIPIB_E_STATE, "the periodic operators' derivatives: not defined on a walled box");
    const double h = ctx->h;
    return launch_vjp_X(ctx, X, lam_f, F, lamX, 1.0 / (h * h * h * h));
}

hipib_status hipib_interp_vjp_X(hipib_ctx* ctx, const double* X, const double* u,
                                const double* lamU, double* lamX) {
    HIPIB_TRY(check_ctx(ctx));
    if (!ctx->mesh_set) return fail(HIPIB_E_STATE, "hipib_set_mesh has not been called");
    if (!aligned8(u) || (ctx->nn > 0 && (!aligned8(X) || !aligned8(lamU) || !aligned8(lamX))))
        return fail(HIPIB_E_INVAL, "bad pointer");
    if (ctx->cfg.walls) return fail(HIPIB_E_STATE, "the periodic operators' derivatives: not defined on a walled box");
    return launch_vjp_X(ctx, X, u, lamU, lamX, 1.0 / ctx->h);
}

hipib_status hipib_convection_vjp(hipib_ctx* ctx, const double* u, const double* lam, double* out) {
    HIPIB_TRY(check_ctx(ctx));
    if (!aligned8(u) || !aligned8(lam) || !aligned8(out)) return fail(HIPIB_E_INVAL, "bad pointer");
    if (ctx->cfg.walls) return fail(HIPIB_E_STATE, "the periodic operators' derivatives: not defined on a walled box");
    return launch_conv_vjp(ctx, u, lam, out, 0.0, 1.0);
}

hipib_status hipib_timer_enable(hipib_ctx* ctx, int32_t which) {
    HIPIB_TRY(check_ctx(ctx));
    if (which < HIPIB_TIMER_OFF || which >= HIPIB_N_TIMERS)
        return fail(HIPIB_E_INVAL, "unknown timer %d", which);
    HIPIB_HIP(hipStreamSynchronize(ctx->stream));
    ctx->timer_which = which;
    ctx->ev_used = 0;
    ctx->timer_launches = 0;
    ctx->timer_bytes = 0.0;
    return HIPIB_OK;
}

hipib_status hipib_timer_read(hipib_ctx* ctx, int32_t* launches, double* total_ms,
                              double* bytes_per_launch) {
    HIPIB_TRY(check_ctx(ctx));
    HIPIB_HIP(hipStreamSynchronize(ctx->stream));
    double tot = 0.0;
    for (size_t i = 0; i < ctx->ev_used; ++i) {
        float ms = 0.0f;
        HIPIB_HIP(hipEventElapsedTime(&ms, ctx->ev_pool[2 * i], ctx->ev_pool[2 * i + 1]));
        tot += ms;
    }
    if (launches) *launches = (int32_t)ctx->timer_launches;
    if (total_ms) *total_ms = tot;
    if (bytes_per_launch)
        *bytes_per_launch = ctx->timer_launches > 0 ? ctx->timer_bytes / (double)ctx->timer_launches : 0.0;
    ctx->ev_used = 0;
    ctx->timer_launches = 0;
    ctx->timer_bytes = 0.0;
    return HIPIB_OK;
}

double hipib_cavity_pressure(double p0, double T, double t) {
    if (p0 == 0.0 || !(T > 0.0)) return 0.0;
    const double pi = 3.14159265358979323846;
    const double sn = std::sin(pi * t / T);
    return p0 * sn * sn;
}

hipib_status hipib_get_stats(hipib_ctx* ctx, const double* u, const double* X, hipib_stats* out) {
    HIPIB_TRY(check_ctx(ctx));
    if (!out) return fail(HIPIB_E_INVAL, "null output");
    if ((u && !aligned8(u)) || (X && !aligned8(X))) return fail(HIPIB_E_INVAL, "bad pointer");
    if (X && !ctx->mesh_set) return fail(HIPIB_E_STATE, "hipib_set_mesh has not been called");
    std::memset(out, 0, sizeof(*out));
    const int32_t ns = (int32_t)ctx->recs.size();
    out->steps = ns;
    for (int t = 0; t < 4; ++t) {
        double sum = 0.0;
        for (const StepRecord& r : ctx->recs) sum += r.cycles[t];
        out->cycles_mean[t] = ns > 0 ? sum / ns : 0.0;
        if (ns > 0) {
            out->cycles_last[t] = ctx->recs.back().cycles[t];
            out->relres_last[t] = ctx->recs.back().relres[t];
        }
    }
    out->timed_steps = (int32_t)ctx->phase_steps;
    for (int k = 0; k < HIPIB_N_PHASES; ++k) out->phase_ms[k] = ctx->phase_ms[k];
    return compute_stats(ctx, u, X && ctx->nn > 0 ? X : nullptr, out);
}

hipib_status hipib_set_phase_timing(hipib_ctx* ctx, int32_t enable) {
    HIPIB_TRY(check_ctx(ctx));
    if (enable && !ctx->ph_ev[0]) {
        for (hipEvent_t& e : ctx->ph_ev) HIPIB_HIP(hipEventCreate(&e));
        for (hipEvent_t& e : ctx->ph_force) HIPIB_HIP(hipEventCreate(&e));
    }
    ctx->phase_timing = enable != 0;
    ctx->phase_steps = 0;
    for (double& v : ctx->phase_ms) v = 0.0;
    return HIPIB_OK;
}

int32_t hipib_get_step_stats(hipib_ctx* ctx, int32_t* cycles, double* relres, int32_t max_steps) {
    if (!ctx || max_steps < 0) return 0;
    const int32_t n = (int32_t)ctx->recs.size() < max_steps ? (int32_t)ctx->recs.size() : max_steps;
    for (int32_t s = 0; s < n; ++s)
        for (int t = 0; t < 4; ++t) {
            if (cycles) cycles[4 * s + t] = ctx->recs[s].cycles[t];
            if (relres) relres[4 * s + t] = ctx->recs[s].relres[t];
        }
    return n;
}

}  // extern "C"
