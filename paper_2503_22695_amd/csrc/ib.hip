// Eulerian-Lagrangian coupling ("Eulerian-Lagrangian coupling operators"):
//   spreading      f^d[idx] += sum_q F^d_q delta_h(x^d_idx - X_q)
//   interpolation  U^d_q = sum_idx u^d[idx] delta_h(x^d_idx - X_q) h^3
// with Peskin's four-point kernel delta_h(x) = prod_e phi(x_e / h) / h^3.
// For a lattice coordinate r = X_e / h - offset (offset 0 along the face
// direction d, 1/2 along the others), the support is b-1 .. b+2 with
// b = floor(r), f = r - b, s = sqrt(1 + 4 f (1 - f)) and weights
//   ((3 - 2f - s), (3 - 2f + s), (1 + 2f + s), (1 + 2f - s)) / 8,
// which is phi evaluated at f+1, f, 1-f, 2-f.
#include "internal.h"

namespace hipib {
namespace {

struct Stencil1 {
    int i0;        // first index, wrapped into [0, n)
    double w[4];
};

__device__ __forceinline__ Stencil1 peskin4(double r, int n) {
    if (!(fabs(r) < 1.0e9)) r = 0.0;   // non-finite or absurd positions never index out of range
    const double b = floor(r);
    const double f = r - b;
    const double s = sqrt(1.0 + 4.0 * f * (1.0 - f));
    Stencil1 st;
    st.w[0] = (3.0 - 2.0 * f - s) * 0.125;
    st.w[1] = (3.0 - 2.0 * f + s) * 0.125;
    st.w[2] = (1.0 + 2.0 * f + s) * 0.125;
    st.w[3] = (1.0 + 2.0 * f - s) * 0.125;
    int i0 = ((int)b - 1) % n;
    st.i0 = i0 < 0 ? i0 + n : i0;
    return st;
}

__device__ __forceinline__ int step_wrap(int i, int n) { return i >= n ? i - n : i; }

// one thread per node; 3 x 64 atomic adds of F^d w into the face lattices
__global__ void __launch_bounds__(256)
k_spread_atomic(const double* __restrict__ X, const double* __restrict__ F, double* __restrict__ f,
                int nn, int n, int64_t n3, double inv_h, double ih3) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nn) return;
    const double x[3] = {X[3 * q] * inv_h, X[3 * q + 1] * inv_h, X[3 * q + 2] * inv_h};
    for (int d = 0; d < 3; ++d) {
        const double val = F[3 * q + d] * ih3;
        const Stencil1 sx = peskin4(x[0] - (d == 0 ? 0.0 : 0.5), n);
        const Stencil1 sy = peskin4(x[1] - (d == 1 ? 0.0 : 0.5), n);
        const Stencil1 sz = peskin4(x[2] - (d == 2 ? 0.0 : 0.5), n);
        double* fd = f + d * n3;
        for (int c = 0; c < 4; ++c) {
            const int kk = step_wrap(sz.i0 + c, n);
            for (int b = 0; b < 4; ++b) {
                const int jj = step_wrap(sy.i0 + b, n);
                const double wyz = sy.w[b] * sz.w[c];
                const int64_t row = (int64_t)n * ((int64_t)jj + (int64_t)n * kk);
                for (int a = 0; a < 4; ++a) {
                    const int ii = step_wrap(sx.i0 + a, n);
                    atomicAdd(fd + row + ii, val * (sx.w[a] * wyz));
                }
            }
        }
    }
}

// one thread per node: gather 3 x 64 values; optionally X += dt U (in place)
__global__ void __launch_bounds__(256)
k_interp(const double* X, const double* __restrict__ u, double* __restrict__ U, double* Xupd,
         double dt, int nn, int n, int64_t n3, double inv_h) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nn) return;
    const double X0 = X[3 * q], X1 = X[3 * q + 1], X2 = X[3 * q + 2];
    const double x[3] = {X0 * inv_h, X1 * inv_h, X2 * inv_h};
    double Uq[3];
    for (int d = 0; d < 3; ++d) {
        const Stencil1 sx = peskin4(x[0] - (d == 0 ? 0.0 : 0.5), n);
        const Stencil1 sy = peskin4(x[1] - (d == 1 ? 0.0 : 0.5), n);
        const Stencil1 sz = peskin4(x[2] - (d == 2 ? 0.0 : 0.5), n);
        const double* ud = u + d * n3;
        double acc = 0.0;
        for (int c = 0; c < 4; ++c) {
            const int kk = step_wrap(sz.i0 + c, n);
            for (int b = 0; b < 4; ++b) {
                const int jj = step_wrap(sy.i0 + b, n);
                const double wyz = sy.w[b] * sz.w[c];
                const int64_t row = (int64_t)n * ((int64_t)jj + (int64_t)n * kk);
                for (int a = 0; a < 4; ++a) {
                    const int ii = step_wrap(sx.i0 + a, n);
                    acc += ud[row + ii] * (sx.w[a] * wyz);
                }
            }
        }
        Uq[d] = acc;
    }
    if (U) {
        U[3 * q] = Uq[0];
        U[3 * q + 1] = Uq[1];
        U[3 * q + 2] = Uq[2];
    }
    if (Xupd) {
        Xupd[3 * q] = X0 + dt * Uq[0];
        Xupd[3 * q + 1] = X1 + dt * Uq[1];
        Xupd[3 * q + 2] = X2 + dt * Uq[2];
    }
}

}  // namespace

hipib_status launch_spread(hipib_ctx* ctx, const double* X, const double* F, double* f) {
    if (ctx->nn == 0) return HIPIB_OK;
    const double h = ctx->h;
    k_spread_atomic<<<(ctx->nn + 255) / 256, 256, 0, ctx->stream>>>(X, F, f, ctx->nn, ctx->n, ctx->n3,
                                                                    1.0 / h, 1.0 / (h * h * h));
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

hipib_status launch_interpolate(hipib_ctx* ctx, const double* X, const double* u, double* U,
                                double* Xupd, double dt) {
    if (ctx->nn == 0) return HIPIB_OK;
    k_interp<<<(ctx->nn + 255) / 256, 256, 0, ctx->stream>>>(X, u, U, Xupd, dt, ctx->nn, ctx->n,
                                                             ctx->n3, 1.0 / ctx->h);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

}  // namespace hipib
