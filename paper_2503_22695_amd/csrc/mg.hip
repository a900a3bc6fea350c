// Geometric multigrid for (sigma I - nu Lap_h) x = b on the periodic grid: the
// Helmholtz (sigma = rho/dt, nu = mu) and Poisson (sigma = 0, nu = 1) solves of
// the Chorin step.  The paper names a geometric multigrid only; the cycle here
// is a cell-centred symmetric V(pre, post) cycle:
//   red-black Gauss-Seidel in place (red = (i+j+k) even; pre: red, black;
//   post: black, red), residual, restriction by per-axis weights (1,3,3,1)/8,
//   coarse operators rediscretised at 2h, cell-centred trilinear prolongation
//   added to x, coarsest level (first with < 8 cells per side) solved by a fixed
//   number of red+black sweeps, Poisson means removed after the coarse solve
//   and after each top-level cycle.  Stop: ||r||_2 <= max(rtol, 1e3 eps) ||b||_2.
//
// GPU mapping: every fine-level stage is one bandwidth-bound stencil kernel
// (64x4 thread tiles, one thread per cell; colour sweeps one thread per cell of
// the colour).  All levels with at most 16 cells per side run inside ONE
// workgroup of 1024 threads with the level arrays in LDS (112 KB for 16^3),
// which removes ~25 tiny launches per cycle.  Up to three independent
// components (the three velocity lattices) are solved in the same launches;
// each kernel block first reads its component's `active` flag, so components
// stop independently.  Stop decisions are taken on the device; the host
// enqueues the predicted number of cycles and synchronises once to read them.
#include <cfloat>

#include "internal.h"

namespace hipib {
namespace {

constexpr int TX = 64, TY = 4;
constexpr int kSmallThreads = 1024;

enum FinalizeMode { FIN_BNORM = 0, FIN_INIT_R = 1, FIN_CYCLE_R = 2, FIN_MEAN = 3 };

struct LevelGeom {
    int n;
    int64_t cs;  // component stride
    __device__ __forceinline__ int64_t at(int i, int j, int k) const {
        return (int64_t)i + (int64_t)n * ((int64_t)j + (int64_t)n * k);
    }
};

// ---------------------------------------------------------------------------
// fine-level stencil kernels; grid (x tiles, y tiles, n * ncomp)
// ---------------------------------------------------------------------------

// TAG only separates launches in profiles: 0 coarse levels, 1 finest level of a
// Helmholtz solve, 2 finest level of a Poisson solve.
template <int TAG>
__global__ void __launch_bounds__(TX * TY)
k_gs_colour(double* __restrict__ x, const double* __restrict__ b, LevelGeom G, double c,
            double diag, int colour, const int32_t* __restrict__ active) {
    const int comp = blockIdx.z / G.n, k = blockIdx.z - comp * G.n;
    if (!active[comp]) return;
    const int n = G.n;
    const int j = blockIdx.y * TY + threadIdx.y;
    const int i = 2 * (blockIdx.x * TX + threadIdx.x) + ((j + k + colour) & 1);
    if (i >= n || j >= n) return;
    double* xc = x + comp * G.cs;
    const double* bc = b + comp * G.cs;
    const double s = xc[G.at(wrap_idx(i + 1, n), j, k)] + xc[G.at(wrap_idx(i - 1, n), j, k)] +
                     xc[G.at(i, wrap_idx(j + 1, n), k)] + xc[G.at(i, wrap_idx(j - 1, n), k)] +
                     xc[G.at(i, j, wrap_idx(k + 1, n))] + xc[G.at(i, j, wrap_idx(k - 1, n))];
    const int64_t o = G.at(i, j, k);
    xc[o] = (bc[o] + c * s) / diag;
}

__device__ __forceinline__ double residual_at(const double* __restrict__ xc,
                                              const double* __restrict__ bc, const LevelGeom& G,
                                              int i, int j, int k, double sigma, double c) {
    const int n = G.n;
    const int64_t o = G.at(i, j, k);
    const double xo = xc[o];
    const double s = xc[G.at(wrap_idx(i + 1, n), j, k)] + xc[G.at(wrap_idx(i - 1, n), j, k)] +
                     xc[G.at(i, wrap_idx(j + 1, n), k)] + xc[G.at(i, wrap_idx(j - 1, n), k)] +
                     xc[G.at(i, j, wrap_idx(k + 1, n))] + xc[G.at(i, j, wrap_idx(k - 1, n))];
    const double Ax = sigma * xo - c * (s - 6.0 * xo);
    return bc[o] - Ax;
}

__global__ void __launch_bounds__(TX * TY)
k_residual(const double* __restrict__ x, const double* __restrict__ b, double* __restrict__ r,
           LevelGeom G, int64_t rcs, double sigma, double c, const int32_t* __restrict__ active) {
    const int comp = blockIdx.z / G.n, k = blockIdx.z - comp * G.n;
    if (!active[comp]) return;
    const int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y;
    if (i >= G.n || j >= G.n) return;
    r[comp * rcs + G.at(i, j, k)] =
        residual_at(x + comp * G.cs, b + comp * G.cs, G, i, j, k, sigma, c);
}

// sum of r^2 per block (one partial per block, all threads participate)
__global__ void __launch_bounds__(TX * TY)
k_resid_norm(const double* __restrict__ x, const double* __restrict__ b, LevelGeom G,
             double sigma, double c, const int32_t* __restrict__ active,
             double* __restrict__ part, int64_t pstride) {
    __shared__ double red[16];
    const int comp = blockIdx.z / G.n, k = blockIdx.z - comp * G.n;
    if (!active[comp]) return;  // block-uniform
    const int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y;
    double v = 0.0;
    if (i < G.n && j < G.n) {
        const double r = residual_at(x + comp * G.cs, b + comp * G.cs, G, i, j, k, 0.0 + sigma, c);
        v = r * r;
    }
    const int tid = threadIdx.x + TX * threadIdx.y;
    // flatten the 2-D block for the reduction
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < (TX * TY) / 64; ++w) s += red[w];
        const int64_t blk = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * k);
        part[comp * pstride + blk] = s;
    }
}

// sum (square = 1: of squares) of a contiguous component array; fixed chunking
__global__ void __launch_bounds__(256)
k_sum_partials(const double* __restrict__ v, int64_t cs, int64_t count, int square,
               const int32_t* __restrict__ active, double* __restrict__ part, int64_t pstride) {
    __shared__ double red[16];
    const int comp = blockIdx.y;
    if (active && !active[comp]) return;
    const double* vc = v + comp * cs;
    double s = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < count; t += (int64_t)gridDim.x * 256) {
        const double a = vc[t];
        s += square ? a * a : a;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[comp * pstride + blockIdx.x] = s;
}

__global__ void __launch_bounds__(TX * TY)
k_restrict(const double* __restrict__ r, int nf, int64_t rcs, double* __restrict__ bc,
           LevelGeom C, const int32_t* __restrict__ active) {
    const int comp = blockIdx.z / C.n, K = blockIdx.z - comp * C.n;
    if (!active[comp]) return;
    const int I = blockIdx.x * TX + threadIdx.x, J = blockIdx.y * TY + threadIdx.y;
    if (I >= C.n || J >= C.n) return;
    const double w[4] = {1.0, 3.0, 3.0, 1.0};
    const double* rc = r + comp * rcs;
    double s = 0.0;
    for (int cz = 0; cz < 4; ++cz) {
        const int kk = wrap_idx(2 * K - 1 + cz, nf);
        for (int cy = 0; cy < 4; ++cy) {
            const int jj = wrap_idx(2 * J - 1 + cy, nf);
            const int64_t row = (int64_t)nf * ((int64_t)jj + (int64_t)nf * kk);
            for (int cx = 0; cx < 4; ++cx) {
                const int ii = wrap_idx(2 * I - 1 + cx, nf);
                s += w[cx] * w[cy] * w[cz] / 512.0 * rc[row + ii];
            }
        }
    }
    bc[comp * C.cs + C.at(I, J, K)] = s;
}

__global__ void __launch_bounds__(TX * TY)
k_prolong_add(double* __restrict__ x, LevelGeom F, const double* __restrict__ xc, LevelGeom C,
              const int32_t* __restrict__ active) {
    const int comp = blockIdx.z / F.n, k = blockIdx.z - comp * F.n;
    if (!active[comp]) return;
    const int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y;
    if (i >= F.n || j >= F.n) return;
    const int nc = C.n;
    const int ijk[3] = {i, j, k};
    int base[3][2];
    for (int d = 0; d < 3; ++d) {
        const int I = ijk[d] >> 1;
        base[d][0] = I;
        base[d][1] = (ijk[d] & 1) ? wrap_idx(I + 1, nc) : wrap_idx(I - 1, nc);
    }
    const double wt[2] = {0.75, 0.25};
    const double* xcc = xc + comp * C.cs;
    double v = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a)
                v += wt[a] * wt[b] * wt[c] * xcc[C.at(base[0][a], base[1][b], base[2][c])];
    const int64_t o = comp * F.cs + F.at(i, j, k);
    x[o] += v;
}

__global__ void k_sub_mean(double* __restrict__ v, int64_t cs, int64_t count,
                           const MGState* __restrict__ st) {
    const int comp = blockIdx.y;
    if (!st->active[comp]) return;
    const double m = st->mean[comp];
    double* vc = v + comp * cs;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x)
        vc[t] -= m;
}

__global__ void k_zero_requested(double* __restrict__ x, int64_t cs, int64_t count,
                                 const MGState* __restrict__ st) {
    const int comp = blockIdx.y;
    if (!st->zero_req[comp]) return;
    double* xc = x + comp * cs;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x)
        xc[t] = 0.0;
}

// Reduce the partials of each component (fixed order) and update the state.
__global__ void __launch_bounds__(1024)
k_finalize(const double* __restrict__ part, int64_t nparts, int64_t pstride, int ncomp, int mode,
           MGState* st, double rtol, int max_cycles, int fixed_cycles, double inv_count) {
    __shared__ double red[16];
    for (int comp = 0; comp < ncomp; ++comp) {
        const bool skip = (mode == FIN_CYCLE_R || mode == FIN_MEAN) && !st->active[comp];
        if (skip) continue;  // uniform across the block
        double s = 0.0;
        for (int64_t t = threadIdx.x; t < nparts; t += blockDim.x) s += part[comp * pstride + t];
        s = block_sum(s, red);
        if (threadIdx.x == 0) {
            if (mode == FIN_BNORM) {
                st->bn[comp] = sqrt(s);
            } else if (mode == FIN_MEAN) {
                st->mean[comp] = s * inv_count;
            } else {
                const double bn = st->bn[comp];
                if (mode == FIN_INIT_R) {
                    st->cycles[comp] = 0;
                    st->zero_req[comp] = 0;
                } else {
                    st->cycles[comp] += 1;
                }
                const double rn = sqrt(s);
                int act = 1;
                if (!isfinite(bn)) {
                    st->status = HIPIB_E_NUMERIC;
                    act = 0;
                } else if (bn == 0.0) {
                    st->zero_req[comp] = 1;
                    st->rn[comp] = 0.0;
                    act = 0;
                } else {
                    st->rn[comp] = rn;
                    const double tol = (rtol > 1e3 * DBL_EPSILON ? rtol : 1e3 * DBL_EPSILON) * bn;
                    const int cyc = st->cycles[comp];
                    if (!isfinite(rn)) {
                        st->status = HIPIB_E_NUMERIC;
                        act = 0;
                    } else if (fixed_cycles > 0) {
                        act = cyc < fixed_cycles;
                    } else if (rn <= tol) {
                        act = 0;
                    } else if (cyc >= max_cycles) {
                        st->status = HIPIB_E_NOCONV;
                        act = 0;
                    }
                }
                st->active[comp] = act;
            }
        }
        __syncthreads();
    }
}

__global__ void k_state_reset(MGState* st, int ncomp) {
    if (threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) {
            st->active[c] = c < ncomp ? 1 : 0;
            st->cycles[c] = 0;
            st->zero_req[c] = 0;
            st->mean[c] = 0.0;
        }
        st->status = HIPIB_OK;
    }
}

// ---------------------------------------------------------------------------
// all levels with n <= 16 in one workgroup, arrays in LDS
//
// The level chain is a compile-time constant (16-8-4, 12-6 or 8-4), so every
// index split is a multiply/shift.  Levels above the coarsest use all 1024
// threads with a workgroup barrier between stages; the coarsest level (4^3 or
// 6^3, many sweeps) runs on wavefront 0 alone: LDS operations of one wavefront
// complete in program order, so a wavefront-scope fence between half-sweeps
// replaces the barrier.
// ---------------------------------------------------------------------------

struct SmallArgs {
    int pre, post, sweeps, poisson, zero_init;
    double sigma, nu;
};

template <int N>
__device__ __forceinline__ int wrapc(int i) {
    return i < 0 ? i + N : (i >= N ? i - N : i);
}

template <int N>
__device__ __forceinline__ int at3(int i, int j, int k) {
    return i + N * (j + N * k);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// one colour of red-black Gauss-Seidel by threads t = t0, t0+nt, ...
template <int N>
__device__ __forceinline__ void s_gs(double* x, const double* b, double c, double diag, int colour,
                                     int t0, int nt) {
    constexpr int HALF = N / 2, CNT = HALF * N * N;
    for (int t = t0; t < CNT; t += nt) {
        const int ih = t % HALF, rest = t / HALF;
        const int j = rest % N, k = rest / N;
        const int i = 2 * ih + ((j + k + colour) & 1);
        const double s = x[at3<N>(wrapc<N>(i + 1), j, k)] + x[at3<N>(wrapc<N>(i - 1), j, k)] +
                         x[at3<N>(i, wrapc<N>(j + 1), k)] + x[at3<N>(i, wrapc<N>(j - 1), k)] +
                         x[at3<N>(i, j, wrapc<N>(k + 1))] + x[at3<N>(i, j, wrapc<N>(k - 1))];
        const int o = at3<N>(i, j, k);
        x[o] = (b[o] + c * s) / diag;
    }
}

template <int N>
__device__ __forceinline__ void s_residual(const double* x, const double* b, double* r, double sigma,
                                           double c) {
    constexpr int CNT = N * N * N;
    for (int o = threadIdx.x; o < CNT; o += blockDim.x) {
        const int i = o % N, j = (o / N) % N, k = o / (N * N);
        const double xo = x[o];
        const double s = x[at3<N>(wrapc<N>(i + 1), j, k)] + x[at3<N>(wrapc<N>(i - 1), j, k)] +
                         x[at3<N>(i, wrapc<N>(j + 1), k)] + x[at3<N>(i, wrapc<N>(j - 1), k)] +
                         x[at3<N>(i, j, wrapc<N>(k + 1))] + x[at3<N>(i, j, wrapc<N>(k - 1))];
        const double Ax = sigma * xo - c * (s - 6.0 * xo);
        r[o] = b[o] - Ax;
    }
}

template <int NF>
__device__ __forceinline__ void s_restrict(const double* r, double* bc) {
    constexpr int NC = NF / 2, CNT = NC * NC * NC;
    const double w[4] = {1.0, 3.0, 3.0, 1.0};
    for (int o = threadIdx.x; o < CNT; o += blockDim.x) {
        const int I = o % NC, J = (o / NC) % NC, K = o / (NC * NC);
        double s = 0.0;
        for (int cz = 0; cz < 4; ++cz)
            for (int cy = 0; cy < 4; ++cy)
                for (int cx = 0; cx < 4; ++cx)
                    s += w[cx] * w[cy] * w[cz] / 512.0 *
                         r[at3<NF>(wrapc<NF>(2 * I - 1 + cx), wrapc<NF>(2 * J - 1 + cy),
                                   wrapc<NF>(2 * K - 1 + cz))];
        bc[o] = s;
    }
}

template <int NF>
__device__ __forceinline__ void s_prolong_add(double* x, const double* xc) {
    constexpr int NC = NF / 2, CNT = NF * NF * NF;
    const double wt[2] = {0.75, 0.25};
    for (int o = threadIdx.x; o < CNT; o += blockDim.x) {
        const int ijk[3] = {o % NF, (o / NF) % NF, o / (NF * NF)};
        int base[3][2];
        for (int d = 0; d < 3; ++d) {
            const int I = ijk[d] >> 1;
            base[d][0] = I;
            base[d][1] = (ijk[d] & 1) ? wrapc<NC>(I + 1) : wrapc<NC>(I - 1);
        }
        double v = 0.0;
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a)
                    v += wt[a] * wt[b] * wt[c] * xc[at3<NC>(base[0][a], base[1][b], base[2][c])];
        x[o] += v;
    }
}

// coarsest level on wavefront 0: zero (optional), sweeps, Poisson mean removal
template <int N>
__device__ __forceinline__ void s_coarse_wave(double* x, const double* b, const SmallArgs& A,
                                              bool zero) {
    constexpr int CNT = N * N * N;
    const int lane = threadIdx.x;
    const double h = 1.0 / (double)N;
    const double c = A.nu / (h * h), diag = A.sigma + 6.0 * c;
    if (zero)
        for (int o = lane; o < CNT; o += 64) x[o] = 0.0;
    wave_sync();
    for (int s = 0; s < A.sweeps; ++s) {
        s_gs<N>(x, b, c, diag, 0, lane, 64);
        wave_sync();
        s_gs<N>(x, b, c, diag, 1, lane, 64);
        wave_sync();
    }
    if (A.poisson) {
        double v = 0.0;
        for (int o = lane; o < CNT; o += 64) v += x[o];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        const double m = v / (double)CNT;
        wave_sync();
        for (int o = lane; o < CNT; o += 64) x[o] -= m;
        wave_sync();
    }
}

// one level above the coarsest: pre-smoothing, residual and restriction (down)
template <int N>
__device__ __forceinline__ void s_down(double* x, const double* b, double* r, double* bnext,
                                       const SmallArgs& A, bool zero) {
    constexpr int CNT = N * N * N;
    const double h = 1.0 / (double)N;
    const double c = A.nu / (h * h), diag = A.sigma + 6.0 * c;
    if (zero) {
        for (int o = threadIdx.x; o < CNT; o += blockDim.x) x[o] = 0.0;
        __syncthreads();
    }
    for (int s = 0; s < A.pre; ++s) {
        s_gs<N>(x, b, c, diag, 0, threadIdx.x, blockDim.x);
        __syncthreads();
        s_gs<N>(x, b, c, diag, 1, threadIdx.x, blockDim.x);
        __syncthreads();
    }
    s_residual<N>(x, b, r, A.sigma, c);
    __syncthreads();
    s_restrict<N>(r, bnext);
    __syncthreads();
}

// prolongation and post-smoothing (up)
template <int N>
__device__ __forceinline__ void s_up(double* x, const double* b, const double* xc, const SmallArgs& A) {
    const double h = 1.0 / (double)N;
    const double c = A.nu / (h * h), diag = A.sigma + 6.0 * c;
    s_prolong_add<N>(x, xc);
    __syncthreads();
    for (int s = 0; s < A.post; ++s) {
        s_gs<N>(x, b, c, diag, 1, threadIdx.x, blockDim.x);
        __syncthreads();
        s_gs<N>(x, b, c, diag, 0, threadIdx.x, blockDim.x);
        __syncthreads();
    }
}

// One V-cycle over the levels N0 (, N0/2, ...) down to the coarsest (< 8).
// Level arrays in LDS: [x, b, r] per level, consecutive.
template <int N0>
__global__ void __launch_bounds__(kSmallThreads)
k_small_vcycle(double* __restrict__ xg, const double* __restrict__ bg, int64_t cs, SmallArgs A,
               const int32_t* __restrict__ active) {
    extern __shared__ double lds[];
    const int comp = blockIdx.x;
    if (!active[comp]) return;
    constexpr int N1 = N0 / 2;
    constexpr int C0 = N0 * N0 * N0, C1 = N1 * N1 * N1;
    double* x0 = lds;
    double* b0 = x0 + C0;
    double* r0 = b0 + C0;
    double* x1 = r0 + C0;
    double* b1 = x1 + C1;
    double* r1 = b1 + C1;
    for (int o = threadIdx.x; o < C0; o += blockDim.x) {
        b0[o] = bg[comp * cs + o];
        x0[o] = A.zero_init ? 0.0 : xg[comp * cs + o];
    }
    __syncthreads();
    s_down<N0>(x0, b0, r0, b1, A, false);
    if constexpr (N1 >= 8) {
        constexpr int N2 = N1 / 2;
        constexpr int C2 = N2 * N2 * N2;
        double* x2 = r1 + C1;
        double* b2 = x2 + C2;
        s_down<N1>(x1, b1, r1, b2, A, true);
        if (threadIdx.x < 64) s_coarse_wave<N2>(x2, b2, A, true);
        __syncthreads();
        s_up<N1>(x1, b1, x2, A);
    } else {
        (void)r1;
        if (threadIdx.x < 64) s_coarse_wave<N1>(x1, b1, A, true);
        __syncthreads();
    }
    s_up<N0>(x0, b0, x1, A);
    for (int o = threadIdx.x; o < C0; o += blockDim.x) xg[comp * cs + o] = x0[o];
}

dim3 tiles(int n, int ncomp, bool colour) {
    const int nx = colour ? n / 2 : n;
    return dim3((nx + TX - 1) / TX, (n + TY - 1) / TY, n * ncomp);
}

int64_t norm_parts(int n) {
    return (int64_t)((n + TX - 1) / TX) * ((n + TY - 1) / TY) * n;
}

struct OpCoef {
    double sigma, nu;
    int poisson;
};

OpCoef op_coef(const hipib_ctx* ctx, int op) {
    if (op == HIPIB_OP_POISSON) return {0.0, 1.0, 1};
    return {ctx->cfg.rho / ctx->cfg.dt, ctx->cfg.mu, 0};
}

hipib_status finalize(hipib_ctx* ctx, int64_t nparts, int64_t pstride, int ncomp, int mode,
                      double inv_count) {
    k_finalize<<<1, 1024, 0, ctx->stream>>>(ctx->part, nparts, pstride, ncomp, mode, ctx->st,
                                             ctx->cfg.mg_rtol, ctx->cfg.mg_max_cycles,
                                             ctx->cfg.mg_fixed_cycles, inv_count);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

// component pointers: level 0 = caller arrays (stride n3), others = workspaces
struct LevelPtr {
    double* x;
    const double* b;
    int64_t cs;
};

hipib_status small_vcycle(hipib_ctx* ctx, int l, LevelPtr p, int ncomp, const OpCoef& oc,
                          bool zero_init) {
    SmallArgs A{};
    A.pre = ctx->cfg.mg_pre;
    A.post = ctx->cfg.mg_post;
    A.sweeps = ctx->cfg.mg_coarse_sweeps;
    A.poisson = oc.poisson;
    A.zero_init = zero_init ? 1 : 0;
    A.sigma = oc.sigma;
    A.nu = oc.nu;
    const int n = ctx->lv[l].n;
    const dim3 grid(ncomp), blk(kSmallThreads);
    if (n == 16)
        k_small_vcycle<16><<<grid, blk, ctx->small_lds, ctx->stream>>>(p.x, p.b, p.cs, A, ctx->st->active);
    else if (n == 12)
        k_small_vcycle<12><<<grid, blk, ctx->small_lds, ctx->stream>>>(p.x, p.b, p.cs, A, ctx->st->active);
    else if (n == 8)
        k_small_vcycle<8><<<grid, blk, ctx->small_lds, ctx->stream>>>(p.x, p.b, p.cs, A, ctx->st->active);
    else
        return fail(HIPIB_E_INVAL, "no coarse-level kernel for n = %d", n);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

hipib_status gs_sweep(hipib_ctx* ctx, int l, LevelPtr p, int ncomp, const OpCoef& oc, double c,
                      double diag, int colour) {
    const int n = ctx->lv[l].n;
    const LevelGeom G{n, p.cs};
    const int32_t* act = ctx->st->active;
    const dim3 grid = tiles(n, ncomp, true), blk(TX, TY);
    if (l > 0) {
        k_gs_colour<0><<<grid, blk, 0, ctx->stream>>>(p.x, p.b, G, c, diag, colour, act);
    } else if (!oc.poisson) {
        k_gs_colour<1><<<grid, blk, 0, ctx->stream>>>(p.x, p.b, G, c, diag, colour, act);
    } else {
        const int pair = timer_start(ctx, HIPIB_TIMER_SMOOTH_FINE_POISSON, 12.0 * (double)ctx->n3);
        k_gs_colour<2><<<grid, blk, 0, ctx->stream>>>(p.x, p.b, G, c, diag, colour, act);
        timer_stop(ctx, pair);
    }
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

hipib_status vcycle(hipib_ctx* ctx, int l, LevelPtr p, int ncomp, const OpCoef& oc) {
    if (l == ctx->small_start) return small_vcycle(ctx, l, p, ncomp, oc, l > 0);
    const int n = ctx->lv[l].n;
    const double h = 1.0 / n, c = oc.nu / (h * h), diag = oc.sigma + 6.0 * c;
    const int32_t* act = ctx->st->active;
    const LevelGeom G{n, p.cs};
    for (int s = 0; s < ctx->cfg.mg_pre; ++s) {
        HIPIB_TRY(gs_sweep(ctx, l, p, ncomp, oc, c, diag, 0));
        HIPIB_TRY(gs_sweep(ctx, l, p, ncomp, oc, c, diag, 1));
    }
    const int64_t rcs = (int64_t)n * n * n;
    k_residual<<<tiles(n, ncomp, false), dim3(TX, TY), 0, ctx->stream>>>(p.x, p.b, ctx->r0, G, rcs,
                                                                          oc.sigma, c, act);
    hipib::Level& C = ctx->lv[l + 1];
    const LevelGeom GC{C.n, C.n3};
    k_restrict<<<tiles(C.n, ncomp, false), dim3(TX, TY), 0, ctx->stream>>>(ctx->r0, n, rcs, C.b, GC, act);
    LevelPtr pc{C.x, C.b, C.n3};
    if (l + 1 == ctx->small_start) {
        HIPIB_TRY(small_vcycle(ctx, l + 1, pc, ncomp, oc, true));
    } else {
        HIPIB_TRY(launch_zero(ctx, C.x, ncomp * C.n3));
        HIPIB_TRY(vcycle(ctx, l + 1, pc, ncomp, oc));
    }
    k_prolong_add<<<tiles(n, ncomp, false), dim3(TX, TY), 0, ctx->stream>>>(p.x, G, C.x, GC, act);
    for (int s = 0; s < ctx->cfg.mg_post; ++s) {
        HIPIB_TRY(gs_sweep(ctx, l, p, ncomp, oc, c, diag, 1));
        HIPIB_TRY(gs_sweep(ctx, l, p, ncomp, oc, c, diag, 0));
    }
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

hipib_status resid_norm(hipib_ctx* ctx, LevelPtr p, int ncomp, const OpCoef& oc, int mode) {
    const int n = ctx->n;
    const double h = 1.0 / n, c = oc.nu / (h * h);
    const int64_t np = norm_parts(n);
    k_resid_norm<<<tiles(n, ncomp, false), dim3(TX, TY), 0, ctx->stream>>>(
        p.x, p.b, LevelGeom{n, p.cs}, oc.sigma, c, ctx->st->active, ctx->part, np);
    HIPIB_HIP(hipGetLastError());
    return finalize(ctx, np, np, ncomp, mode, 0.0);
}

int sum_blocks(int64_t count) {
    int64_t b = (count + 255) / 256;
    return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

}  // namespace

int timer_start(hipib_ctx* ctx, int kind, double bytes) {
    if (ctx->timer_which != kind) return -1;
    const size_t pair = ctx->ev_used;
    while (ctx->ev_pool.size() < 2 * (pair + 1)) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        ctx->ev_pool.push_back(e);
    }
    if (hipEventRecord(ctx->ev_pool[2 * pair], ctx->stream) != hipSuccess) return -1;
    ctx->timer_bytes = bytes;
    return (int)pair;
}

void timer_stop(hipib_ctx* ctx, int pair) {
    if (pair < 0) return;
    if (hipEventRecord(ctx->ev_pool[2 * pair + 1], ctx->stream) == hipSuccess) ctx->ev_used = pair + 1;
}

hipib_status mg_prepare(hipib_ctx* ctx) {
    if (ctx->small_lds > 160 * 1024)
        return fail(HIPIB_E_INVAL, "coarse levels need %zu bytes of LDS", ctx->small_lds);
    HIPIB_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_small_vcycle<16>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)ctx->small_lds));
    HIPIB_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_small_vcycle<12>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)ctx->small_lds));
    HIPIB_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_small_vcycle<8>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)ctx->small_lds));
    return HIPIB_OK;
}

hipib_status sync_state(hipib_ctx* ctx) {
    HIPIB_HIP(hipMemcpyAsync(ctx->st_host, ctx->st, sizeof(MGState), hipMemcpyDeviceToHost,
                             ctx->stream));
    HIPIB_HIP(hipStreamSynchronize(ctx->stream));
    return HIPIB_OK;
}

// v -= mean(v) for a single field of n^3 values, unconditionally (state slot 0
// is forced active for the duration).
hipib_status mg_remove_mean(hipib_ctx* ctx, double* v, int /*slot*/) {
    k_state_reset<<<1, 64, 0, ctx->stream>>>(ctx->st, 1);
    const int nb = sum_blocks(ctx->n3);
    k_sum_partials<<<dim3(nb, 1), 256, 0, ctx->stream>>>(v, ctx->n3, ctx->n3, 0, nullptr, ctx->part, nb);
    HIPIB_HIP(hipGetLastError());
    HIPIB_TRY(finalize(ctx, nb, nb, 1, FIN_MEAN, 1.0 / (double)ctx->n3));
    k_sub_mean<<<dim3(sum_blocks(ctx->n3), 1), 256, 0, ctx->stream>>>(v, ctx->n3, ctx->n3, ctx->st);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

hipib_status mg_solve(hipib_ctx* ctx, int op, int ncomp, const double* b, double* x,
                      int32_t* cycles, double* relres) {
    const OpCoef oc = op_coef(ctx, op);
    LevelPtr p{x, b, ctx->n3};
    const int nb = sum_blocks(ctx->n3);
    k_state_reset<<<1, 64, 0, ctx->stream>>>(ctx->st, ncomp);
    k_sum_partials<<<dim3(nb, ncomp), 256, 0, ctx->stream>>>(b, ctx->n3, ctx->n3, 1, nullptr,
                                                             ctx->part, nb);
    HIPIB_HIP(hipGetLastError());
    HIPIB_TRY(finalize(ctx, nb, nb, ncomp, FIN_BNORM, 0.0));
    HIPIB_TRY(resid_norm(ctx, p, ncomp, oc, FIN_INIT_R));
    k_zero_requested<<<dim3(nb, ncomp), 256, 0, ctx->stream>>>(x, ctx->n3, ctx->n3, ctx->st);
    HIPIB_HIP(hipGetLastError());

    int enqueue = ctx->predicted[op] > 0 ? ctx->predicted[op] : 1;
    int total = 0;
    const int limit = (ctx->cfg.mg_fixed_cycles > 0 ? ctx->cfg.mg_fixed_cycles : ctx->cfg.mg_max_cycles) + 1;
    while (true) {
        for (int e = 0; e < enqueue; ++e) {
            HIPIB_TRY(vcycle(ctx, 0, p, ncomp, oc));
            if (oc.poisson) {
                k_sum_partials<<<dim3(nb, ncomp), 256, 0, ctx->stream>>>(
                    x, ctx->n3, ctx->n3, 0, ctx->st->active, ctx->part, nb);
                HIPIB_HIP(hipGetLastError());
                HIPIB_TRY(finalize(ctx, nb, nb, ncomp, FIN_MEAN, 1.0 / (double)ctx->n3));
                k_sub_mean<<<dim3(nb, ncomp), 256, 0, ctx->stream>>>(x, ctx->n3, ctx->n3, ctx->st);
                HIPIB_HIP(hipGetLastError());
            }
            HIPIB_TRY(resid_norm(ctx, p, ncomp, oc, FIN_CYCLE_R));
        }
        total += enqueue;
        HIPIB_TRY(sync_state(ctx));
        const MGState& s = *ctx->st_host;
        if (s.status != HIPIB_OK) break;
        bool any = false;
        for (int c = 0; c < ncomp; ++c) any = any || s.active[c];
        if (!any) break;
        if (total > limit) return fail(HIPIB_E_NOCONV, "multigrid: stop state did not settle");
        enqueue = 1;
    }
    const MGState& s = *ctx->st_host;
    int mx = 1;
    for (int c = 0; c < ncomp; ++c) {
        if (cycles) cycles[c] = s.cycles[c];
        if (relres) relres[c] = s.bn[c] > 0.0 ? s.rn[c] / s.bn[c] : 0.0;
        if (s.cycles[c] > mx) mx = s.cycles[c];
    }
    ctx->predicted[op] = mx;
    if (s.status == HIPIB_E_NOCONV)
        return fail(HIPIB_E_NOCONV, "multigrid did not reach rtol %g in %d cycles", ctx->cfg.mg_rtol,
                    ctx->cfg.mg_max_cycles);
    if (s.status == HIPIB_E_NUMERIC) return fail(HIPIB_E_NUMERIC, "multigrid: non-finite residual");
    return HIPIB_OK;
}

}  // namespace hipib
