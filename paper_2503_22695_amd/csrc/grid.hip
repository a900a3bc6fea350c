// Pointwise MAC-grid kernels of the Chorin step ("Spatial Discretization"):
// right-hand side with explicit flux-form convection, divergence of the
// intermediate velocity, and the velocity correction.  All three stream the
// grid once; one thread per cell, 64x4 thread tiles so each wavefront reads
// 64 consecutive x-cells (512 B) per array.
#include "internal.h"

namespace hipib {
namespace {

constexpr int TX = 64, TY = 4;

struct Grid3 {
    int n;
    int64_t n3;
    __device__ __forceinline__ int64_t at(int i, int j, int k) const {
        return (int64_t)i + (int64_t)n * ((int64_t)j + (int64_t)n * k);
    }
};

// C^d at face (i,j,k) of component d, conservative centred form:
//   normal flux at cell centres ((u^d[c] + u^d[c+e_d]) / 2)^2,
//   tangential flux at edges ((u^d[c-e_e] + u^d[c]) / 2)((u^e[c-e_d] + u^e[c]) / 2).
__device__ __forceinline__ double conv_component(const double* __restrict__ u, const Grid3 g,
                                                 int d, int i, int j, int k, double inv_h) {
    const int n = g.n;
    const double* ud = u + d * g.n3;
    int p[3] = {i, j, k};
    int cm[3] = {i, j, k};
    int cp[3] = {i, j, k};
    cm[d] = wrap_idx(p[d] - 1, n);
    cp[d] = wrap_idx(p[d] + 1, n);
    const double u0 = ud[g.at(i, j, k)];
    const double ap = 0.5 * (u0 + ud[g.at(cp[0], cp[1], cp[2])]);
    const double am = 0.5 * (ud[g.at(cm[0], cm[1], cm[2])] + u0);
    double s = (ap * ap - am * am) * inv_h;
    for (int e = 0; e < 3; ++e) {
        if (e == d) continue;
        const double* ue = u + e * g.n3;
        int em[3] = {i, j, k}, ep[3] = {i, j, k}, epdm[3] = {i, j, k};
        em[e] = wrap_idx(p[e] - 1, n);
        ep[e] = wrap_idx(p[e] + 1, n);
        epdm[e] = ep[e];
        epdm[d] = cm[d];
        // edge below c (along e) and edge above c
        const double lo = 0.5 * (ud[g.at(em[0], em[1], em[2])] + u0) *
                          (0.5 * (ue[g.at(cm[0], cm[1], cm[2])] + ue[g.at(i, j, k)]));
        const double hi = 0.5 * (u0 + ud[g.at(ep[0], ep[1], ep[2])]) *
                          (0.5 * (ue[g.at(epdm[0], epdm[1], epdm[2])] + ue[g.at(ep[0], ep[1], ep[2])]));
        s += (hi - lo) * inv_h;
    }
    return s;
}

__global__ void __launch_bounds__(TX * TY)
k_rhs_build(const double* __restrict__ u, const double* __restrict__ f, double* __restrict__ g,
            Grid3 G, double rho_dt, double rho, double inv_h, int convection, double* __restrict__ upk,
            int g_packed) {
    const int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y, k = blockIdx.z;
    if (i >= G.n || j >= G.n) return;
    const int64_t c = G.at(i, j, k);
    const int64_t o = (upk || g_packed) ? pk(i, j, k, G.n) : 0;
    const int64_t og = g_packed ? o : c;
    for (int d = 0; d < 3; ++d) {
        const double cv = convection ? conv_component(u, G, d, i, j, k, inv_h) : 0.0;
        const double ud = u[d * G.n3 + c];
        double v = rho_dt * ud - rho * cv;
        if (f) v = v + f[d * G.n3 + c];
        g[d * G.n3 + og] = v;
        if (upk) upk[d * G.n3 + o] = ud;   // u^n packed: the Helmholtz guess
    }
}

// b = -(rho/dt) D u, D u = sum_d (u^d[c+e_d] - u^d[c]) / h
__global__ void __launch_bounds__(TX * TY)
k_divergence_rhs(const double* __restrict__ u, double* __restrict__ b, Grid3 G, double rho_dt,
                 double inv_h) {
    const int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y, k = blockIdx.z;
    if (i >= G.n || j >= G.n) return;
    const int n = G.n;
    const int64_t c = G.at(i, j, k);
    double s = (u[G.at(wrap_idx(i + 1, n), j, k)] - u[c]) * inv_h;
    s += (u[G.n3 + G.at(i, wrap_idx(j + 1, n), k)] - u[G.n3 + c]) * inv_h;
    s += (u[2 * G.n3 + G.at(i, j, wrap_idx(k + 1, n))] - u[2 * G.n3 + c]) * inv_h;
    b[c] = -rho_dt * s;
}

// u^d -= (dt/rho) (p[c] - p[c - e_d]) / h
__global__ void __launch_bounds__(TX * TY)
k_project(double* __restrict__ u, const double* __restrict__ p, Grid3 G, double dt_rho,
          double inv_h) {
    const int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y, k = blockIdx.z;
    if (i >= G.n || j >= G.n) return;
    const int n = G.n;
    const int64_t c = G.at(i, j, k);
    const double pc = p[c];
    const double gx = (pc - p[G.at(wrap_idx(i - 1, n), j, k)]) * inv_h;
    const double gy = (pc - p[G.at(i, wrap_idx(j - 1, n), k)]) * inv_h;
    const double gz = (pc - p[G.at(i, j, wrap_idx(k - 1, n))]) * inv_h;
    u[c] = u[c] - dt_rho * gx;
    u[G.n3 + c] = u[G.n3 + c] - dt_rho * gy;
    u[2 * G.n3 + c] = u[2 * G.n3 + c] - dt_rho * gz;
}

__global__ void k_zero(double* __restrict__ p, int64_t count) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x)
        p[t] = 0.0;
}

dim3 plane_grid(int n) { return dim3((n + TX - 1) / TX, (n + TY - 1) / TY, n); }

}  // namespace

hipib_status launch_rhs_build_coef(hipib_ctx* ctx, const double* u, const double* f, double* g,
                                   double rho_dt, double rho_conv, double* upk, bool g_packed) {
    Grid3 G{ctx->n, ctx->n3};
    const double bytes = (f ? 72.0 : 48.0) + (upk ? 24.0 : 0.0);
    return launch_k(ctx, HIPIB_TIMER_RHS, bytes * (double)ctx->n3, k_rhs_build, plane_grid(ctx->n),
                    dim3(TX, TY), 0, u, f, g, G, rho_dt, rho_conv, 1.0 / ctx->h, ctx->cfg.convection, upk,
                    g_packed ? 1 : 0);
}

hipib_status launch_rhs_build(hipib_ctx* ctx, const double* u, const double* f, double* g, double* upk,
                              bool g_packed) {
    return launch_rhs_build_coef(ctx, u, f, g, ctx->cfg.rho / ctx->cfg.dt, ctx->cfg.rho, upk, g_packed);
}

hipib_status launch_divergence_rhs_coef(hipib_ctx* ctx, const double* u, double* b, double coef) {
    Grid3 G{ctx->n, ctx->n3};
    return launch_k(ctx, HIPIB_TIMER_DIVERGENCE, 32.0 * (double)ctx->n3, k_divergence_rhs, plane_grid(ctx->n),
                    dim3(TX, TY), 0, u, b, G, coef, 1.0 / ctx->h);
}

hipib_status launch_divergence_rhs(hipib_ctx* ctx, const double* u, double* b) {
    return launch_divergence_rhs_coef(ctx, u, b, ctx->cfg.rho / ctx->cfg.dt);
}

hipib_status launch_project_coef(hipib_ctx* ctx, double* u, const double* p, double coef) {
    Grid3 G{ctx->n, ctx->n3};
    return launch_k(ctx, HIPIB_TIMER_PROJECT, 56.0 * (double)ctx->n3, k_project, plane_grid(ctx->n), dim3(TX, TY), 0,
                    u, p, G, coef, 1.0 / ctx->h);
}

hipib_status launch_project(hipib_ctx* ctx, double* u, const double* p) {
    return launch_project_coef(ctx, u, p, ctx->cfg.dt / ctx->cfg.rho);
}

hipib_status launch_zero(hipib_ctx* ctx, double* p, int64_t count) {
    if (count <= 0) return HIPIB_OK;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_zero<<<(unsigned)blocks, 256, 0, ctx->stream>>>(p, count);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

}  // namespace hipib
