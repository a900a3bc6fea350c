// Run diagnostics (hipib_get_stats): quantities the paper reports for its
// benchmarks and runs (volume change of the solid, the Jacobian of the
// deformation, "Benchmarks") and the checks of a discrete incompressible flow
// (kinetic energy, momentum, divergence of the velocity).  Computed on demand
// from the arrays the caller passes, off the hot path: each kernel writes one
// partial per workgroup and the host sums the partials in index order.
#include <algorithm>
#include <cfloat>
#include <vector>

#include "solid.h"

namespace hipib {
namespace {

constexpr int kStatBlocks = 1024, kStatThreads = 256;

// per workgroup: sum u^x, u^y, u^z, sum |u|^2 (over the three face lattices)
// and max |D u| over the cells (D u = sum_d (u^d[c+e_d] - u^d[c]) / h)
__global__ void __launch_bounds__(kStatThreads)
k_grid_stats(const double* __restrict__ u, int n, double inv_h, double* __restrict__ part) {
    __shared__ double red[5][kStatThreads / 64];
    const int64_t n3 = (int64_t)n * n * n;
    double s[4] = {0.0, 0.0, 0.0, 0.0}, dmax = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * kStatThreads + threadIdx.x; c < n3;
         c += (int64_t)gridDim.x * kStatThreads) {
        const int i = (int)(c % n), j = (int)((c / n) % n), k = (int)(c / ((int64_t)n * n));
        const double ux = u[c], uy = u[n3 + c], uz = u[2 * n3 + c];
        s[0] += ux;
        s[1] += uy;
        s[2] += uz;
        s[3] += ux * ux + uy * uy + uz * uz;
        const int ip = i + 1 < n ? i + 1 : 0, jp = j + 1 < n ? j + 1 : 0, kp = k + 1 < n ? k + 1 : 0;
        const double div = ((u[ip + (int64_t)n * (j + (int64_t)n * k)] - ux) +
                            (u[n3 + i + (int64_t)n * (jp + (int64_t)n * k)] - uy) +
                            (u[2 * n3 + i + (int64_t)n * (j + (int64_t)n * kp)] - uz)) * inv_h;
        dmax = fmax(dmax, fabs(div));
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        for (int t = 0; t < 4; ++t) s[t] += __shfl_down(s[t], o, 64);
        dmax = fmax(dmax, __shfl_down(dmax, o, 64));
    }
    if (lane == 0) {
        for (int t = 0; t < 4; ++t) red[t][w] = s[t];
        red[4][w] = dmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a[4] = {0.0, 0.0, 0.0, 0.0}, m = 0.0;
        for (int v = 0; v < kStatThreads / 64; ++v) {
            for (int t = 0; t < 4; ++t) a[t] += red[t][v];
            m = fmax(m, red[4][v]);
        }
        for (int t = 0; t < 4; ++t) part[t * gridDim.x + blockIdx.x] = a[t];
        part[4 * gridDim.x + blockIdx.x] = m;
    }
}

// per workgroup: min and max of det F over the Gauss points, and the solid's
// volume sum_e sum_q w_q det(dx/dxi); F = (dx/dxi)(dX/dxi)^{-1}
template <typename S>
__global__ void __launch_bounds__(kStatThreads)
k_solid_stats(const double* __restrict__ X, const double* __restrict__ Xref,
              const int32_t* __restrict__ conn, int ne, double* __restrict__ part) {
    constexpr int N = S::N;
    __shared__ double red[3][kStatThreads / 64];
    double jmin = DBL_MAX, jmax = -DBL_MAX, vol = 0.0;
    for (int e = blockIdx.x * kStatThreads + threadIdx.x; e < ne; e += gridDim.x * kStatThreads) {
        double xr[N][3], xc[N][3];
        for (int a = 0; a < N; ++a) {
            const int64_t q = conn[N * (int64_t)e + a];
            for (int r = 0; r < 3; ++r) {
                xr[a][r] = Xref[3 * q + r];
                xc[a][r] = X[3 * q + r];
            }
        }
        for (int g = 0; g < S::Q; ++g) {
            double dN[N][3];
            const double wq = elem_rule<S, double>(g, dN);
            double Jr[9], Jx[9];
            for (int t = 0; t < 9; ++t) Jr[t] = Jx[t] = 0.0;
            for (int a = 0; a < N; ++a)
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) {
                        Jr[3 * r + c] += xr[a][r] * dN[a][c];
                        Jx[3 * r + c] += xc[a][r] * dN[a][c];
                    }
            const double dx = det3(Jx), dX = det3(Jr);
            const double J = dx / dX;
            jmin = fmin(jmin, J);
            jmax = fmax(jmax, J);
            vol += wq * dx;
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        jmin = fmin(jmin, __shfl_down(jmin, o, 64));
        jmax = fmax(jmax, __shfl_down(jmax, o, 64));
        vol += __shfl_down(vol, o, 64);
    }
    if (lane == 0) {
        red[0][w] = jmin;
        red[1][w] = jmax;
        red[2][w] = vol;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = DBL_MAX, b = -DBL_MAX, v = 0.0;
        for (int t = 0; t < kStatThreads / 64; ++t) {
            a = fmin(a, red[0][t]);
            b = fmax(b, red[1][t]);
            v += red[2][t];
        }
        part[blockIdx.x] = a;
        part[gridDim.x + blockIdx.x] = b;
        part[2 * gridDim.x + blockIdx.x] = v;
    }
}

template <typename S>
hipib_status launch_solid_stats(hipib_ctx* ctx, const double* X, int blocks) {
    k_solid_stats<S><<<blocks, kStatThreads, 0, ctx->stream>>>(X, ctx->Xref, ctx->conn, ctx->ne, ctx->part);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

}  // namespace

hipib_status compute_stats(hipib_ctx* ctx, const double* u, const double* X, hipib_stats* out) {
    std::vector<double> h;
    if (u) {
        const int64_t n3 = ctx->n3;
        const int blocks = (int)std::min<int64_t>(std::min<int64_t>(kStatBlocks, ctx->part_cap / 5),
                                                  (n3 + kStatThreads - 1) / kStatThreads);
        k_grid_stats<<<blocks, kStatThreads, 0, ctx->stream>>>(u, ctx->n, 1.0 / ctx->h, ctx->part);
        HIPIB_HIP(hipGetLastError());
        h.assign(5 * (size_t)blocks, 0.0);
        HIPIB_HIP(hipMemcpyAsync(h.data(), ctx->part, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                                 ctx->stream));
        HIPIB_HIP(hipStreamSynchronize(ctx->stream));
        double s[4] = {0.0, 0.0, 0.0, 0.0}, dmax = 0.0;
        for (int b = 0; b < blocks; ++b) {
            for (int t = 0; t < 4; ++t) s[t] += h[t * (size_t)blocks + b];
            dmax = std::max(dmax, h[4 * (size_t)blocks + b]);
        }
        const double h3 = ctx->h * ctx->h * ctx->h, rho = ctx->cfg.rho;
        for (int d = 0; d < 3; ++d) out->momentum[d] = rho * h3 * s[d];
        out->kinetic_energy = 0.5 * rho * h3 * s[3];
        out->max_abs_div = dmax;
    }
    if (X && ctx->ne > 0) {
        const int blocks = (int)std::min<int64_t>(std::min<int64_t>(kStatBlocks, ctx->part_cap / 3),
                                                  (ctx->ne + kStatThreads - 1) / kStatThreads);
        if (ctx->npe == 4) HIPIB_TRY(launch_solid_stats<Tet4>(ctx, X, blocks));
        else if (ctx->npe == 10) HIPIB_TRY(launch_solid_stats<Tet10>(ctx, X, blocks));
        else HIPIB_TRY(launch_solid_stats<Hex8>(ctx, X, blocks));
        h.assign(3 * (size_t)blocks, 0.0);
        HIPIB_HIP(hipMemcpyAsync(h.data(), ctx->part, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                                 ctx->stream));
        HIPIB_HIP(hipStreamSynchronize(ctx->stream));
        double a = DBL_MAX, b = -DBL_MAX, v = 0.0;
        for (int k = 0; k < blocks; ++k) {
            a = std::min(a, h[k]);
            b = std::max(b, h[blocks + (size_t)k]);
            v += h[2 * (size_t)blocks + k];
        }
        out->J_min = a;
        out->J_max = b;
        out->volume = v;
    }
    return HIPIB_OK;
}

}  // namespace hipib
