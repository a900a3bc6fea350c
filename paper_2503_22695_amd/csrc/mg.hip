// Geometric multigrid for (sigma I - nu Lap_h) x = b on the periodic grid: the
// Helmholtz (sigma = rho/dt, nu = mu) and Poisson (sigma = 0, nu = 1) solves of
// the Chorin step.  The paper names a geometric multigrid only; the cycle here
// is a cell-centred symmetric V(pre, post) cycle:
//   red-black Gauss-Seidel in place (red = (i+j+k) even; pre: red, black;
//   post: black, red), residual, restriction by per-axis weights (1,3,3,1)/8,
//   coarse operators rediscretised at 2h, cell-centred trilinear prolongation
//   added to x, coarsest level (the first with at most 32 cells per side)
//   solved exactly by its discrete Fourier diagonalisation (with
//   mg_coarse_sweeps > 0: the first with fewer than 8 cells, relaxed by that
//   many red+black sweeps), Poisson means removed after the coarse solve and
//   once from the final solution (residual and sweeps are invariant to a
//   constant shift).  Stop: ||r||_2 <= max(rtol, 1e3 eps) ||b||_2.
//   The Helmholtz hierarchy stops where the operator's Jacobi radius is at most
//   1/2 (see stop_level), and that level is relaxed by red-black SOR with
//   Young's factor; when that is the finest level, a cycle is pre + post such
//   sweeps on the iterate.
//
// Storage: every solver array is kept in a packed red-black layout.  For a
// level of n cells per side (n even) and H = n/2, component c, colour
// q = (i+j+k) & 1, cell (i,j,k) sits at
//     c * n^3 + q * n^3/2 + (i >> 1) + H * (j + n * k).
// A cell's six neighbours all have the other colour; with p = i & 1 =
// (j+k+q) & 1 its x-neighbours sit at packed positions ih+p-1 and ih+p of the
// other colour's row (j,k) and its y/z neighbours at ih of rows (j+-1,k),
// (j,k+-1).  A half-sweep therefore streams exactly what it needs: the other
// colour of x, its own colour of b, its own colour of x written (12 B/cell in
// FP64), with unit-stride rows.  The caller's arrays are packed on entry to a
// solve and the solution unpacked on exit; inside a step the fluid arrays
// stay packed from the right-hand side to the projection (fluid_step_packed).
//
// Precision: in FP64 mode the V-cycles run on the FP64 solution.  In mixed
// mode the outer loop stays in FP64 (residual, norm, stop test, solution
// update, Poisson mean) and each cycle computes the correction e of the scaled
// residual r / ||b|| with one FP32 V-cycle from e = 0:  x += ||b|| e.  For a
// linear smoother this is the same cycle as the FP64 one, with the correction
// rounded to FP32 (iterative refinement with a V-cycle preconditioner).
//
// GPU mapping: one bandwidth-bound kernel per fine-level stage (64x4 thread
// tiles), with the stages that can share a pass fused (the zero-guess pair of
// half-sweeps, the coarse-grid correction in the first post-smoothing
// half-sweep, the CG dots in the last two); the first coarse levels run as
// one down and one up workgroup-blocked launch each; the exact coarsest solve
// is one workgroup per component (at most 16^3) or three plane-parallel
// launches (24^3, 32^3).  Up to three components (the three velocity
// lattices) share every launch and stop independently through per-component
// `active` flags read at block start.  Stop decisions are made on the device;
// the host enqueues the predicted number of cycles and waits once to read
// them.
#include <cfloat>
#include <cmath>
#include <vector>

#include <hip/hip_ext.h>

#include "internal.h"

namespace hipib {
namespace {

constexpr int TX = 64, TY = 4;
constexpr int kSmallThreads = 1024;

enum FinalizeMode {
    FIN_BNORM = 0, FIN_INIT_R = 1, FIN_CYCLE_R = 2, FIN_MEAN = 3, FIN_MEAN_ALL = 4,
    FIN_MEAN_BNORM = 5,  // component 0: mean of b from slot 0 (sum b), ||b - mean|| with slot 1 (sum b^2)
    FIN_BNORM_INIT_R = 6 // per component: ||b|| from the b^2 partials after ncomp * pstride, then as FIN_INIT_R
};

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }


// Sum of the six neighbours of the colour-q cell at packed (ih, j, k), read
// from the other colour's array xo, in the order i+1, i-1, j+1, j-1, k+1, k-1.
template <typename T>
__device__ __forceinline__ T nbr_sum(const T* __restrict__ xo, int ih, int j, int k, int n, int q) {
    const int H = n >> 1;
    const int p = (j + k + q) & 1;
    int ip = ih + p, im = ih + p - 1;
    if (ip >= H) ip -= H;
    if (im < 0) im += H;
    const int jp = wrapi(j + 1, n), jm = wrapi(j - 1, n), kp = wrapi(k + 1, n), km = wrapi(k - 1, n);
    const int64_t row = (int64_t)H * ((int64_t)j + (int64_t)n * k);
    return xo[row + ip] + xo[row + im] + xo[(int64_t)H * (jp + (int64_t)n * k) + ih] +
           xo[(int64_t)H * (jm + (int64_t)n * k) + ih] + xo[(int64_t)H * (j + (int64_t)n * kp) + ih] +
           xo[(int64_t)H * (j + (int64_t)n * km) + ih];
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Renumbering so that XCD x runs the x-th contiguous eighth of the grid (in
// x-fastest order: a slab of z-planes) keeps a stencil's neighbouring planes
// in the same L2.  Identity when the grid is not a multiple of 8.
__device__ __forceinline__ uint3 xcd_block() {
    const unsigned gx = gridDim.x, gy = gridDim.y;
    const unsigned nb = gx * gy * gridDim.z;
    unsigned b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    if ((nb & 7u) == 0) b = (b & 7u) * (nb >> 3) + (b >> 3);
    return make_uint3(b % gx, (b / gx) % gy, b / (gx * gy));
}

// grid for both colours: z = (comp * 2 + q) * n + k
dim3 packed_grid(int n, int ncomp) {
    return dim3((n / 2 + TX - 1) / TX, (n + TY - 1) / TY, 2 * n * ncomp);
}
// grid over natural cells: z = comp * n + k
dim3 natural_grid(int n, int ncomp) {
    return dim3((n + TX - 1) / TX, (n + TY - 1) / TY, n * ncomp);
}

// ---------------------------------------------------------------------------
// layout conversion
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(TX * TY)
k_pack(const double* __restrict__ src, double* __restrict__ dst, int n, int64_t n3) {
    const int comp = blockIdx.z / n, k = blockIdx.z - comp * n;
    const int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y;
    if (i >= n || j >= n) return;
    dst[comp * n3 + pk(i, j, k, n)] = src[comp * n3 + i + (int64_t)n * (j + (int64_t)n * k)];
}

__global__ void __launch_bounds__(TX * TY)
k_unpack(const double* __restrict__ src, double* __restrict__ dst, int n, int64_t n3,
         const double* __restrict__ mean) {
    const int comp = blockIdx.z / n, k = blockIdx.z - comp * n;
    const int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y;
    if (i >= n || j >= n) return;
    const double v = src[comp * n3 + pk(i, j, k, n)];
    dst[comp * n3 + i + (int64_t)n * (j + (int64_t)n * k)] = mean ? v - mean[comp] : v;
}

// ---------------------------------------------------------------------------
// stencil kernels on packed levels
// ---------------------------------------------------------------------------

// One colour q of red-black Gauss-Seidel: x_q = (b_q + c * sum_nbr x) / diag.
// Each thread updates a column of KPT = gs_kpt<T>() cells along z: the other colour's
// values at (ih, j) on planes k0-1 .. k0+KPT serve as the z-neighbours of the
// column and as one of each cell's two x-neighbours, and all of the thread's
// loads are issued before the first update.  Neighbours are summed in the
// order i+1, i-1, j+1, j-1, k+1, k-1.
// zg: the other colour is known to be zero (first half-sweep from a zero
// guess), so its neighbours are not read; the result is the same to the bit.
// SOR: over-relaxation, x_q += omega (x_gs - x_q), which also reads the cell's
// own old value (16 B/cell in FP64 instead of 12) unless zo says it is zero.
// TAG only separates launches in profiles: 0 coarse levels, 1 finest level of
// a Helmholtz solve, 2 finest level of a Poisson solve.
constexpr int KPT = 4;  // column length of the residual norm

// column length of a half-sweep: 2 cells in FP64, 4 in FP32 (measured best
// on the 128^3 workload)
template <typename T>
constexpr int gs_kpt() { return sizeof(T) == 8 ? 2 : 4; }

// grid of a half-sweep: (packed x tiles, y tiles, z columns * ncomp)
template <typename T>
dim3 gs_grid(int n, int ncomp) {
    constexpr int K = gs_kpt<T>();
    return dim3((n / 2 + TX - 1) / TX, (n + TY - 1) / TY, ((n + K - 1) / K) * ncomp);
}

template <typename T, int TAG, bool SOR = false>
__global__ void __launch_bounds__(TX * TY)
k_gs(T* __restrict__ x, const T* __restrict__ b, int n, int64_t cs, T c, T inv_diag, int q,
     int zg, const int32_t* __restrict__ active, T omega = T(1), int zo = 0) {
    constexpr int KPT = gs_kpt<T>();
    const uint3 bid = xcd_block();
    const int nkb = (n + KPT - 1) / KPT;
    const int comp = bid.z / nkb, k0 = (bid.z - comp * nkb) * KPT;
    if (!active[comp]) return;
    const int H = n >> 1;
    const int ih = bid.x * TX + threadIdx.x, j = bid.y * TY + threadIdx.y;
    if (ih >= H || j >= n) return;
    const int64_t half3 = (int64_t)H * n * n;
    T* xq = x + comp * cs + q * half3;
    const T* xo = x + comp * cs + (1 - q) * half3;
    const T* bq = b + comp * cs + q * half3;
    const int jp = wrapi(j + 1, n), jm = wrapi(j - 1, n);
    const int ihp = ih + 1 < H ? ih + 1 : 0, ihm = ih > 0 ? ih - 1 : H - 1;
    T col[KPT + 2], side[KPT], yp[KPT], ym[KPT], bv[KPT], xold[KPT];
    if (!zg) {
#pragma unroll
        for (int r = 0; r < KPT + 2; ++r) {
            const int kk = wrapi(k0 - 1 + r, n);
            col[r] = xo[ih + (int64_t)H * ((int64_t)j + (int64_t)n * kk)];
        }
    }
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
        const int k = k0 + r;
        if (k < n) {
            const int64_t row = (int64_t)H * ((int64_t)j + (int64_t)n * k);
            bv[r] = bq[row + ih];
            if (SOR) xold[r] = zo ? T(0) : xq[row + ih];
            if (!zg) {
                const int p = (j + k + q) & 1;
                side[r] = xo[row + (p ? ihp : ihm)];
                yp[r] = xo[(int64_t)H * ((int64_t)jp + (int64_t)n * k) + ih];
                ym[r] = xo[(int64_t)H * ((int64_t)jm + (int64_t)n * k) + ih];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
        const int k = k0 + r;
        if (k < n) {
            T s = T(0);
            if (!zg) {
                // x-neighbours: p = 1 -> (ih+1, ih), p = 0 -> (ih, ih-1)
                const int p = (j + k + q) & 1;
                const T a_ip = p ? side[r] : col[r + 1];
                const T a_im = p ? col[r + 1] : side[r];
                s = a_ip + a_im + yp[r] + ym[r] + col[r + 2] + col[r];
            }
            const T xg = (bv[r] + c * s) * inv_diag;
            xq[(int64_t)H * ((int64_t)j + (int64_t)n * k) + ih] =
                SOR ? xold[r] + omega * (xg - xold[r]) : xg;
        }
    }
}

// The first two half-sweeps of a pre-smoothing from a zero guess, in one pass:
// red x = b / diag (its neighbours are zero) and black x = (b + c * sum of those
// red values) / diag.  Each thread takes a column of black cells as k_gs does,
// forms its red neighbours from b, and also writes the red cells at the
// packed positions of its column, so every red cell is written once.  The
// values are those of the two separate half-sweeps (red ones as
// (b + c * 0) / diag).
template <typename T>
__global__ void __launch_bounds__(TX * TY)
k_gs_zero2(T* __restrict__ x, const T* __restrict__ b, int n, int64_t cs, T c, T inv_diag,
           const int32_t* __restrict__ active) {
    constexpr int KPT = gs_kpt<T>();
    const uint3 bid = xcd_block();
    const int nkb = (n + KPT - 1) / KPT;
    const int comp = bid.z / nkb, k0 = (bid.z - comp * nkb) * KPT;
    if (!active[comp]) return;
    const int H = n >> 1;
    const int ih = bid.x * TX + threadIdx.x, j = bid.y * TY + threadIdx.y;
    if (ih >= H || j >= n) return;
    const int64_t half3 = (int64_t)H * n * n;
    T* xr = x + comp * cs;            // red half
    T* xq = xr + half3;               // black half
    const T* br = b + comp * cs;
    const T* bq = br + half3;
    const int jp = wrapi(j + 1, n), jm = wrapi(j - 1, n);
    const int ihp = ih + 1 < H ? ih + 1 : 0, ihm = ih > 0 ? ih - 1 : H - 1;
    T col[KPT + 2], side[KPT], yp[KPT], ym[KPT], bv[KPT];
#pragma unroll
    for (int r = 0; r < KPT + 2; ++r) {
        const int kk = wrapi(k0 - 1 + r, n);
        col[r] = br[ih + (int64_t)H * ((int64_t)j + (int64_t)n * kk)];
    }
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
        const int k = k0 + r;
        if (k < n) {
            const int64_t row = (int64_t)H * ((int64_t)j + (int64_t)n * k);
            const int p = (j + k + 1) & 1;
            bv[r] = bq[row + ih];
            side[r] = br[row + (p ? ihp : ihm)];
            yp[r] = br[(int64_t)H * ((int64_t)jp + (int64_t)n * k) + ih];
            ym[r] = br[(int64_t)H * ((int64_t)jm + (int64_t)n * k) + ih];
        }
    }
    // red values from a zero guess
#pragma unroll
    for (int r = 0; r < KPT + 2; ++r) col[r] = (col[r] + c * T(0)) * inv_diag;
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
        const int k = k0 + r;
        if (k < n) {
            side[r] = (side[r] + c * T(0)) * inv_diag;
            yp[r] = (yp[r] + c * T(0)) * inv_diag;
            ym[r] = (ym[r] + c * T(0)) * inv_diag;
            const int p = (j + k + 1) & 1;
            const T a_ip = p ? side[r] : col[r + 1];
            const T a_im = p ? col[r + 1] : side[r];
            const T sn = a_ip + a_im + yp[r] + ym[r] + col[r + 2] + col[r];
            const int64_t row = (int64_t)H * ((int64_t)j + (int64_t)n * k);
            xq[row + ih] = (bv[r] + c * sn) * inv_diag;
            xr[row + ih] = col[r + 1];
        }
    }
}

// The first post-smoothing half-sweep (colour q, nonzero guess, no
// over-relaxation) fused with the coarse-grid correction: the other colour's
// values in its stencil are taken as x + P e, P the cell-centred trilinear
// prolongation of the coarse correction e (3/4 on the nearest coarse cell,
// 1/4 on the next, per axis).  x of the other colour is left uncorrected in
// memory: the next half-sweep, of that colour, overwrites it from this
// colour's values alone.  The workgroup stages the coarse values its stencils
// reach in LDS, interpolates them along y and z into one row per fine (j, k)
// it needs (Rw), and each neighbour's correction is the x-interpolation of two
// row values.  Grid and columns as k_gs.
constexpr int kProlongRows = 16;  // y rows of columns per k_gs_prolong workgroup (4: 14.7 us, 8: 13.5, 16: 13.0 at 128^3)

template <typename T, int PY>
__global__ void __launch_bounds__(TX * PY)
k_gs_prolong(T* __restrict__ x, const T* __restrict__ b, int n, int64_t cs, const T* __restrict__ xc, int nc,
             int64_t ccs, T c, T inv_diag, int q, const int32_t* __restrict__ active) {
    constexpr int KPT = gs_kpt<T>();
    constexpr int RI = TX + 4;                        // coarse I: ih0 - 2 .. ih0 + TX + 1
    constexpr int CJ = PY / 2 + 2, CK = KPT / 2 + 2;  // coarse J: j0/2 - 1 .. j0/2 + PY/2, K likewise
    constexpr int NRJ = PY + 2, NRK = KPT + 2;        // fine rows j0 - 1 .. j0 + PY, planes k0 - 1 .. k0 + KPT
    constexpr int NE = CK * CJ * RI, EPT = (NE + TX * PY - 1) / (TX * PY);
    __shared__ T E[CK][CJ][RI];
    __shared__ T Rw[NRK][NRJ][RI];
    const uint3 bid = xcd_block();
    const int nkb = (n + KPT - 1) / KPT;
    const int comp = bid.z / nkb, k0 = (bid.z - comp * nkb) * KPT;
    if (!active[comp]) return;  // block-uniform
    const int H = n >> 1;
    const int ih0 = bid.x * TX, j0 = bid.y * PY;
    const int tid = threadIdx.x + TX * threadIdx.y;
    const int ih = ih0 + threadIdx.x, j = j0 + threadIdx.y;
    const bool own = ih < H && j < n;
    const int64_t half3 = (int64_t)H * n * n;
    T* xq = x + comp * cs + q * half3;
    const T* xo = x + comp * cs + (1 - q) * half3;
    const T* bq = b + comp * cs + q * half3;
    const int jp = wrapi(j + 1, n), jm = wrapi(j - 1, n);
    const int ihp = ih + 1 < H ? ih + 1 : 0, ihm = ih > 0 ? ih - 1 : H - 1;
    // the half-sweep's own loads first, so their latency overlaps the staging
    T col[KPT + 2], side[KPT], yp[KPT], ym[KPT], bv[KPT];
    if (own) {
#pragma unroll
        for (int r = 0; r < KPT + 2; ++r) {
            const int kk = wrapi(k0 - 1 + r, n);
            col[r] = xo[ih + (int64_t)H * ((int64_t)j + (int64_t)n * kk)];
        }
#pragma unroll
        for (int r = 0; r < KPT; ++r) {
            const int k = k0 + r;
            if (k < n) {
                const int64_t row = (int64_t)H * ((int64_t)j + (int64_t)n * k);
                const int p = (j + k + q) & 1;
                bv[r] = bq[row + ih];
                side[r] = xo[row + (p ? ihp : ihm)];
                yp[r] = xo[(int64_t)H * ((int64_t)jp + (int64_t)n * k) + ih];
                ym[r] = xo[(int64_t)H * ((int64_t)jm + (int64_t)n * k) + ih];
            }
        }
    }
    const int I_lo = ih0 - 2, J_lo = j0 / 2 - 1, K_lo = k0 / 2 - 1;
    const T* ec = xc + comp * ccs;
    {
        T ev[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int t = tid + e * TX * PY;
            if (t < NE) {
                const int ci = t % RI, cj = (t / RI) % CJ, ck = t / (RI * CJ);
                // (I reaches ih0 + TX + 1, beyond 2 nc on small grids, where the
                // high entries are staged but never read)
                int I = I_lo + ci, J = J_lo + cj, K = K_lo + ck;   // all >= -2
                I = I < 0 ? I + nc : (I >= nc ? I % nc : I);
                J = J < 0 ? J + nc : (J >= nc ? J % nc : J);
                K = K < 0 ? K + nc : (K >= nc ? K % nc : K);
                ev[e] = ec[pk(I, J, K, nc)];
            }
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int t = tid + e * TX * PY;
            if (t < NE) (&E[0][0][0])[t] = ev[e];
        }
    }
    __syncthreads();
    const T w0 = T(0.75), w1 = T(0.25);
    for (int t = tid; t < NRK * NRJ * RI; t += TX * PY) {
        const int ri = t % RI, rj = (t / RI) % NRJ, rk = t / (RI * NRJ);
        // unwrapped fine row (j', k') and its two coarse rows per axis (arithmetic shifts floor)
        const int ju = j0 - 1 + rj, ku = k0 - 1 + rk;
        const int Jn = (ju >> 1) - J_lo, Jf = Jn + ((ju & 1) ? 1 : -1);
        const int Kn = (ku >> 1) - K_lo, Kf = Kn + ((ku & 1) ? 1 : -1);
        Rw[rk][rj][ri] = w0 * (w0 * E[Kn][Jn][ri] + w1 * E[Kn][Jf][ri]) +
                         w1 * (w0 * E[Kf][Jn][ri] + w1 * E[Kf][Jf][ri]);
    }
    __syncthreads();
    if (!own) return;
    // correction at the other-colour cell of packed half-index hu (unwrapped) in
    // row (rj, rk): its fine i = 2 hu + ((j' + k' + 1 - q) & 1)
    auto pe = [&](int hu, int rj, int rk) -> T {
        const int par = (j0 - 1 + rj + k0 - 1 + rk + 1 - q) & 1;
        const int li = hu - I_lo;                     // local index of I = hu
        const int lf = li + (par ? 1 : -1);
        return w0 * Rw[rk][rj][li] + w1 * Rw[rk][rj][lf];
    };
    const int rj0 = threadIdx.y + 1;
#pragma unroll
    for (int r = 0; r < KPT + 2; ++r) col[r] += pe(ih, rj0, r);
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
        const int k = k0 + r;
        if (k < n) {
            const int p = (j + k + q) & 1;
            side[r] += pe(p ? ih + 1 : ih - 1, rj0, r + 1);
            yp[r] += pe(ih, rj0 + 1, r + 1);
            ym[r] += pe(ih, rj0 - 1, r + 1);
            const T a_ip = p ? side[r] : col[r + 1];
            const T a_im = p ? col[r + 1] : side[r];
            const T sn = a_ip + a_im + yp[r] + ym[r] + col[r + 2] + col[r];
            xq[(int64_t)H * ((int64_t)j + (int64_t)n * k) + ih] = (bv[r] + c * sn) * inv_diag;
        }
    }
}

// A finest-level Poisson half-sweep of the conjugate-gradient preconditioner
// (one component, nonzero guess, no over-relaxation) that also sums, over the
// cells it writes, the dots r.z and z.q of the z it finishes: the last two
// half-sweeps of the post-smoothing write each colour's final z.  In FP64 r is
// the sweep's own right-hand side; in mixed mode the sweep runs on e = z / ||b||
// and reads the FP64 residual rd.  Block partials go to part[poff + block]
// (r.z) and part[pstride + poff + block] (z.q).
template <typename T>
__global__ void __launch_bounds__(TX * TY)
k_gs_dot(T* __restrict__ x, const T* __restrict__ b, int n, T c, T inv_diag, int q,
         const double* __restrict__ rd, const double* __restrict__ qd, const MGState* __restrict__ st,
         double* __restrict__ part, int64_t pstride, int64_t poff) {
    constexpr int KPT = gs_kpt<T>();
    __shared__ double red[2][(TX * TY) / 64];
    if (!st->active[0]) return;  // uniform
    const uint3 bid = xcd_block();
    const int k0 = bid.z * KPT;
    const int H = n >> 1;
    const int ih = bid.x * TX + threadIdx.x, j = bid.y * TY + threadIdx.y;
    const double zs = sizeof(T) == 4 ? st->bn[0] : 1.0;
    double a = 0.0, d = 0.0;
    if (ih < H && j < n) {
        const int64_t half3 = (int64_t)H * n * n;
        T* xq = x + q * half3;
        const T* xo = x + (1 - q) * half3;
        const T* bq = b + q * half3;
        const int jp = wrapi(j + 1, n), jm = wrapi(j - 1, n);
        const int ihp = ih + 1 < H ? ih + 1 : 0, ihm = ih > 0 ? ih - 1 : H - 1;
        T col[KPT + 2], side[KPT], yp[KPT], ym[KPT], bv[KPT];
        double rv[KPT], qv[KPT];
#pragma unroll
        for (int r = 0; r < KPT + 2; ++r)
            col[r] = xo[ih + (int64_t)H * ((int64_t)j + (int64_t)n * wrapi(k0 - 1 + r, n))];
#pragma unroll
        for (int r = 0; r < KPT; ++r) {
            const int k = k0 + r;
            if (k < n) {
                const int64_t row = (int64_t)H * ((int64_t)j + (int64_t)n * k);
                const int p = (j + k + q) & 1;
                bv[r] = bq[row + ih];
                side[r] = xo[row + (p ? ihp : ihm)];
                yp[r] = xo[(int64_t)H * ((int64_t)jp + (int64_t)n * k) + ih];
                ym[r] = xo[(int64_t)H * ((int64_t)jm + (int64_t)n * k) + ih];
                rv[r] = sizeof(T) == 8 ? (double)bv[r] : rd[q * half3 + row + ih];
                qv[r] = qd[q * half3 + row + ih];
            }
        }
#pragma unroll
        for (int r = 0; r < KPT; ++r) {
            const int k = k0 + r;
            if (k < n) {
                const int p = (j + k + q) & 1;
                const T a_ip = p ? side[r] : col[r + 1];
                const T a_im = p ? col[r + 1] : side[r];
                const T sn = a_ip + a_im + yp[r] + ym[r] + col[r + 2] + col[r];
                const T xg = (bv[r] + c * sn) * inv_diag;
                xq[(int64_t)H * ((int64_t)j + (int64_t)n * k) + ih] = xg;
                const double zv = zs * (double)xg;
                a += rv[r] * zv;
                d += zv * qv[r];
            }
        }
    }
    const int tid = threadIdx.x + TX * threadIdx.y;
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o, 64);
        d += __shfl_down(d, o, 64);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = a;
        red[1][tid >> 6] = d;
    }
    __syncthreads();
    if (tid == 0) {
        double sa = 0.0, sd = 0.0;
        for (int w = 0; w < (TX * TY) / 64; ++w) {
            sa += red[0][w];
            sd += red[1][w];
        }
        const int64_t blk = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
        part[poff + blk] = sa;
        part[pstride + poff + blk] = sd;
    }
}

// r = b - (sigma x - c (sum_nbr x - 6 x)), both colours
template <typename T>
__global__ void __launch_bounds__(TX * TY)
k_residual(const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ r, int n, int64_t cs,
           T sigma, T c, const int32_t* __restrict__ active) {
    const int z = blockIdx.z, comp = z / (2 * n), rem = z - comp * 2 * n, q = rem / n, k = rem - q * n;
    if (!active[comp]) return;
    const int H = n >> 1;
    const int ih = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y;
    if (ih >= H || j >= n) return;
    const int64_t half3 = (int64_t)H * n * n;
    const int64_t o = comp * cs + q * half3 + ih + (int64_t)H * ((int64_t)j + (int64_t)n * k);
    const T xo = x[o];
    const T s = nbr_sum(x + comp * cs + (1 - q) * half3, ih, j, k, n, q);
    const T Ax = sigma * xo - c * (s - T(6) * xo);
    r[o] = b[o] - Ax;
}

// coarse b[I,J,K] = sum_{a,b,c} (w_a w_b w_c / 512) r[2I-1+a, 2J-1+b, 2K-1+c], w = 1,3,3,1
template <typename T>
__global__ void __launch_bounds__(TX * TY)
k_restrict(const T* __restrict__ r, int nf, int64_t fcs, T* __restrict__ bc, int nc, int64_t ccs,
           const int32_t* __restrict__ active) {
    const int z = blockIdx.z, comp = z / (2 * nc), rem = z - comp * 2 * nc, Q = rem / nc, K = rem - Q * nc;
    if (!active[comp]) return;
    const int Hc = nc >> 1;
    const int IH = blockIdx.x * TX + threadIdx.x, J = blockIdx.y * TY + threadIdx.y;
    if (IH >= Hc || J >= nc) return;
    const int I = 2 * IH + ((J + K + Q) & 1);
    const T w[4] = {T(1), T(3), T(3), T(1)};
    const T* rc = r + comp * fcs;
    T s = T(0);
    for (int cz = 0; cz < 4; ++cz) {
        const int kk = wrapi(2 * K - 1 + cz, nf);
        for (int cy = 0; cy < 4; ++cy) {
            const int jj = wrapi(2 * J - 1 + cy, nf);
            for (int cx = 0; cx < 4; ++cx) {
                const int ii = wrapi(2 * I - 1 + cx, nf);
                s += w[cx] * w[cy] * w[cz] / T(512) * rc[pk(ii, jj, kk, nf)];
            }
        }
    }
    bc[comp * ccs + (int64_t)Q * ((int64_t)Hc * nc * nc) + IH + (int64_t)Hc * ((int64_t)J + (int64_t)nc * K)] = s;
}

// Restriction of the residual right after a pre-smoothing that ended with a
// black half-sweep.  There the black residual b - A x is zero in exact
// arithmetic (each black value was just set to solve its own row), so only
// red cells contribute: coarse b[I,J,K] = sum over the red cells of the
// 4x4x4 window 2I-1..2I+2 (per axis) of (w_a w_b w_c / 512) r, w = 1,3,3,1.
// One workgroup per coarse tile of RCX x RCY x RCZ cells: the red residuals
// of its fine window go to LDS once (no residual array in HBM), then each
// thread sums its window from LDS.
constexpr int RCX = 32, RCY = 8, RCZ = 4;
constexpr int RWY = 2 * RCY + 2, RWZ = 2 * RCZ + 2;  // fine window rows and planes
constexpr int RRED = RCX + 1;                        // red cells per window row
constexpr int RTHREADS = RCX * RCY * RCZ;            // one thread per coarse cell

dim3 resid_restrict_grid(int nc, int ncomp) {
    return dim3((nc + RCX - 1) / RCX, (nc + RCY - 1) / RCY, ((nc + RCZ - 1) / RCZ) * ncomp);
}

template <typename T>
__global__ void __launch_bounds__(RTHREADS)
k_resid_restrict(const T* __restrict__ x, const T* __restrict__ b, int nf, int64_t fcs,
                 T* __restrict__ bc, int nc, int64_t ccs, T sigma, T c,
                 const int32_t* __restrict__ active) {
    __shared__ T rr[RWZ][RWY][RRED];
    const int nzb = (nc + RCZ - 1) / RCZ;
    const int comp = blockIdx.z / nzb, kb = blockIdx.z - comp * nzb;
    if (!active[comp]) return;
    const int I0 = blockIdx.x * RCX, J0 = blockIdx.y * RCY, K0 = kb * RCZ;
    // window extent actually needed (partial tiles at the high edges)
    const int ni = min(RCX, nc - I0), nj = min(RCY, nc - J0), nk = min(RCZ, nc - K0);
    const int xs = 2 * I0 - 1, ys = 2 * J0 - 1, zs = 2 * K0 - 1;
    const int H = nf >> 1;
    const int64_t half3 = (int64_t)H * nf * nf;
    const T* xr = x + comp * fcs;
    const T* xb = xr + half3;
    const T* br = b + comp * fcs;
    const int rows = 2 * nj + 2, planes = 2 * nk + 2, reds = ni + 1;
    const int cnt = planes * rows * reds;
    // batches of 4 cells per thread: all their loads are issued before any use
    constexpr int RB = 4;
    for (int t0 = threadIdx.x; t0 < cnt; t0 += RB * RTHREADS) {
        T xv[RB], sv[RB], bv[RB];
        int dst[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int t = t0 + r * RTHREADS;
            dst[r] = -1;
            if (t < cnt) {
                const int m = t % reds, rest = t / reds;
                const int ly = rest % rows, lz = rest / rows;
                const int yu = ys + ly, zu = zs + lz;
                // red cells of this row sit at xs + off + 2m (parity is unchanged
                // by the periodic wrap because nf is even)
                const int off = (xs + yu + zu) & 1;
                const int i = wrapi(xs + off + 2 * m, nf), j = wrapi(yu, nf), k = wrapi(zu, nf);
                const int ih = i >> 1;
                const int64_t o = ih + (int64_t)H * ((int64_t)j + (int64_t)nf * k);
                xv[r] = xr[o];
                sv[r] = nbr_sum(xb, ih, j, k, nf, 0);
                bv[r] = br[o];
                dst[r] = m + RRED * (ly + RWY * lz);
            }
        }
#pragma unroll
        for (int r = 0; r < RB; ++r)
            if (dst[r] >= 0) (&rr[0][0][0])[dst[r]] = bv[r] - (sigma * xv[r] - c * (sv[r] - T(6) * xv[r]));
    }
    __syncthreads();
    const int col = threadIdx.x % (RCX * RCY), kk = threadIdx.x / (RCX * RCY);
    const int tx = col % RCX, ty = col / RCX;
    if (tx >= ni || ty >= nj || kk >= nk) return;
    const T w[4] = {T(1), T(3), T(3), T(1)};
    {
        T acc = T(0);
        for (int cz = 0; cz < 4; ++cz) {
            const int lz = 2 * kk + cz;
            T pl = T(0);
            for (int cy = 0; cy < 4; ++cy) {
                const int ly = 2 * ty + cy;
                const int off = (xs + ys + ly + zs + lz) & 1;
                // the thread's window 2I-1..2I+2 holds red cells at a = off, off + 2
                pl += w[cy] * (w[off] * rr[lz][ly][tx] + w[off + 2] * rr[lz][ly][tx + 1]);
            }
            acc += w[cz] * pl;
        }
        const int I = I0 + tx, J = J0 + ty, K = K0 + kk;
        bc[comp * ccs + pk(I, J, K, nc)] = acc * T(1.0 / 512.0);
    }
}

// fine x += trilinear interpolation of coarse x (3/4 nearest, 1/4 next, per
// axis) on the first nq colours: nq = 1 (red only) when the next operation is
// a black half-sweep, which overwrites the black cells without reading them
template <typename T>
__global__ void __launch_bounds__(TX * TY)
k_prolong_add(T* __restrict__ x, int nf, int64_t fcs, const T* __restrict__ xc, int nc, int64_t ccs,
              int nq, const int32_t* __restrict__ active) {
    const int z = blockIdx.z, comp = z / (nq * nf), rem = z - comp * nq * nf, q = rem / nf, k = rem - q * nf;
    if (!active[comp]) return;
    const int H = nf >> 1;
    const int ih = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y;
    if (ih >= H || j >= nf) return;
    const int i = 2 * ih + ((j + k + q) & 1);
    const int ijk[3] = {i, j, k};
    int base[3][2];
    for (int d = 0; d < 3; ++d) {
        const int I = ijk[d] >> 1;
        base[d][0] = I;
        base[d][1] = (ijk[d] & 1) ? wrapi(I + 1, nc) : wrapi(I - 1, nc);
    }
    const T wt[2] = {T(0.75), T(0.25)};
    const T* xcc = xc + comp * ccs;
    T v = T(0);
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a)
                v += wt[a] * wt[b] * wt[c] * xcc[pk(base[0][a], base[1][b], base[2][c], nc)];
    x[comp * fcs + (int64_t)q * ((int64_t)H * nf * nf) + ih + (int64_t)H * ((int64_t)j + (int64_t)nf * k)] += v;
}

template <typename T>
__global__ void k_zero_t(T* __restrict__ p, int64_t count) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x)
        p[t] = T(0);
}

// ---------------------------------------------------------------------------
// FP64 outer loop: residual norm (and FP32 scaled residual), update, means
// ---------------------------------------------------------------------------

// sum of r^2 per block (and with bsq = ncomp of b^2, after ncomp * pstride
// partials); TO32: also r32 = (float)(r / ||b||).  Grid: (packed
// x tiles, y tiles, (comp * 2 + q) * z-columns); each thread takes a column of
// KPT cells of colour q along z with the loads of k_gs.
template <bool TO32>
__global__ void __launch_bounds__(TX * TY)
k_resid_norm(const double* __restrict__ x, double* __restrict__ b, int n, int64_t cs,
             double sigma, double c, const MGState* __restrict__ st, float* __restrict__ r32,
             double* __restrict__ part, int64_t pstride, double* __restrict__ rstore, int submean, int bsq) {
    __shared__ double red[2][16];
    const int nkb = (n + KPT - 1) / KPT;
    const uint3 bid = xcd_block();
    const int z = bid.z, comp = z / (2 * nkb), rem = z - comp * 2 * nkb, q = rem / nkb;
    const int k0 = (rem - q * nkb) * KPT;
    if (!st->active[comp]) return;  // block-uniform
    const int H = n >> 1;
    const int ih = bid.x * TX + threadIdx.x, j = bid.y * TY + threadIdx.y;
    double v = 0.0, vb = 0.0;
    if (ih < H && j < n) {
        const int64_t half3 = (int64_t)H * n * n;
        const double* xq = x + comp * cs + q * half3;
        const double* xo = x + comp * cs + (1 - q) * half3;
        double* bq = b + comp * cs + q * half3;
        const double bmean = submean ? st->mean[comp] : 0.0;
        const int jp = wrapi(j + 1, n), jm = wrapi(j - 1, n);
        const int ihp = ih + 1 < H ? ih + 1 : 0, ihm = ih > 0 ? ih - 1 : H - 1;
        double col[KPT + 2], side[KPT], yp[KPT], ym[KPT], bv[KPT], xv[KPT];
#pragma unroll
        for (int r = 0; r < KPT + 2; ++r)
            col[r] = xo[ih + (int64_t)H * ((int64_t)j + (int64_t)n * wrapi(k0 - 1 + r, n))];
#pragma unroll
        for (int r = 0; r < KPT; ++r) {
            const int k = k0 + r;
            if (k < n) {
                const int64_t row = (int64_t)H * ((int64_t)j + (int64_t)n * k);
                const int p = (j + k + q) & 1;
                bv[r] = bq[row + ih];
                xv[r] = xq[row + ih];
                side[r] = xo[row + (p ? ihp : ihm)];
                yp[r] = xo[(int64_t)H * ((int64_t)jp + (int64_t)n * k) + ih];
                ym[r] = xo[(int64_t)H * ((int64_t)jm + (int64_t)n * k) + ih];
            }
        }
        const double inv_bn = TO32 ? 1.0 / st->bn[comp] : 0.0;
#pragma unroll
        for (int r = 0; r < KPT; ++r) {
            const int k = k0 + r;
            if (k < n) {
                const int p = (j + k + q) & 1;
                const double a_ip = p ? side[r] : col[r + 1];
                const double a_im = p ? col[r + 1] : side[r];
                const double s = a_ip + a_im + yp[r] + ym[r] + col[r + 2] + col[r];
                if (submean) {
                    bv[r] -= bmean;
                    bq[(int64_t)H * ((int64_t)j + (int64_t)n * k) + ih] = bv[r];
                }
                const double rr = bv[r] - (sigma * xv[r] - c * (s - 6.0 * xv[r]));
                v += rr * rr;
                vb += bv[r] * bv[r];
                if (rstore) rstore[comp * cs + q * half3 + (int64_t)H * ((int64_t)j + (int64_t)n * k) + ih] = rr;
                if (TO32)
                    r32[comp * cs + q * half3 + (int64_t)H * ((int64_t)j + (int64_t)n * k) + ih] =
                        (float)(rr * inv_bn);
            }
        }
    }
    const int tid = threadIdx.x + TX * threadIdx.y;
    for (int o = 32; o > 0; o >>= 1) {
        v += __shfl_down(v, o, 64);
        vb += __shfl_down(vb, o, 64);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = v;
        red[1][tid >> 6] = vb;
    }
    __syncthreads();
    if (tid == 0) {
        double s = 0.0, sb = 0.0;
        for (int w = 0; w < (TX * TY) / 64; ++w) {
            s += red[0][w];
            sb += red[1][w];
        }
        const int64_t blk = bid.x + (int64_t)gridDim.x * (bid.y + (int64_t)gridDim.y * rem);
        part[comp * pstride + blk] = s;
        if (bsq) part[(bsq + comp) * pstride + blk] = sb;   // bsq = ncomp: ||b||^2 after the residuals
    }
}

// ---------------------------------------------------------------------------
// Poisson by V-cycle-preconditioned conjugate gradients (mg_krylov; one
// component).  Vectors r, z, p, q are packed like x; the scalars live in the
// device state.  One iteration: z = M r (one V-cycle from a zero guess; in
// mixed mode the FP32 V-cycle of r / ||b||, z = ||b|| e), the dots r.z and
// z.q, beta = -alpha (z.q) / (r.z)_old (0 on the first iteration, the
// flexible Polak-Ribiere update), p = z + beta p together with
// q = A p = A z + beta q and p.q, alpha = (r.z) / (p.q), then x += alpha p and
// r -= alpha q with ||r||^2 for the stop test.
// ---------------------------------------------------------------------------

// per-block partial sums of r.z (slot 0) and z.q (slot 1); z = zs * z32 in mixed mode
template <typename TZ>
__global__ void __launch_bounds__(256)
k_cg_dots(const double* __restrict__ r, const TZ* __restrict__ z, const double* __restrict__ q,
          int64_t n3, const MGState* __restrict__ st, double* __restrict__ part, int64_t pstride) {
    __shared__ double red[16];
    if (!st->active[0]) return;  // uniform
    const double zs = sizeof(TZ) == 4 ? st->bn[0] : 1.0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    double a = 0.0, b = 0.0;
    for (int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x; t0 < n3; t0 += 4 * stride) {
        double rv[4], zv[4], qv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t t = t0 + u * stride;
            const bool in = t < n3;
            rv[u] = in ? r[t] : 0.0;
            zv[u] = in ? zs * (double)z[t] : 0.0;
            qv[u] = in ? q[t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a += rv[u] * zv[u];
            b += zv[u] * qv[u];
        }
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        part[pstride + blockIdx.x] = b;
    }
}

// p = z + beta p and q = A z + beta q (= A p), partial p.q per block; grid and
// columns as k_resid_norm
template <typename TZ>
__global__ void __launch_bounds__(TX * TY)
k_cg_dir(const TZ* __restrict__ z, double* __restrict__ p, double* __restrict__ q, int n,
         double sigma, double c, const MGState* __restrict__ st, double* __restrict__ part) {
    __shared__ double red[16];
    const int nkb = (n + KPT - 1) / KPT;
    const uint3 bid = xcd_block();
    const int rem = bid.z, qc = rem / nkb, k0 = (rem - qc * nkb) * KPT;
    if (!st->active[0]) return;  // uniform
    const double beta = st->beta, zs = sizeof(TZ) == 4 ? st->bn[0] : 1.0;
    const int H = n >> 1;
    const int ih = bid.x * TX + threadIdx.x, j = bid.y * TY + threadIdx.y;
    double v = 0.0;
    if (ih < H && j < n) {
        const int64_t half3 = (int64_t)H * n * n;
        const TZ* zq = z + qc * half3;
        const TZ* zo = z + (1 - qc) * half3;
        double* pq = p + qc * half3;
        double* qq = q + qc * half3;
        const int jp = wrapi(j + 1, n), jm = wrapi(j - 1, n);
        const int ihp = ih + 1 < H ? ih + 1 : 0, ihm = ih > 0 ? ih - 1 : H - 1;
        double col[KPT + 2], side[KPT], yp[KPT], ym[KPT], zv[KPT], pv[KPT], qv[KPT];
#pragma unroll
        for (int r = 0; r < KPT + 2; ++r)
            col[r] = zs * (double)zo[ih + (int64_t)H * ((int64_t)j + (int64_t)n * wrapi(k0 - 1 + r, n))];
#pragma unroll
        for (int r = 0; r < KPT; ++r) {
            const int k = k0 + r;
            if (k < n) {
                const int64_t row = (int64_t)H * ((int64_t)j + (int64_t)n * k);
                const int pp = (j + k + qc) & 1;
                zv[r] = zs * (double)zq[row + ih];
                side[r] = zs * (double)zo[row + (pp ? ihp : ihm)];
                yp[r] = zs * (double)zo[(int64_t)H * ((int64_t)jp + (int64_t)n * k) + ih];
                ym[r] = zs * (double)zo[(int64_t)H * ((int64_t)jm + (int64_t)n * k) + ih];
                pv[r] = beta != 0.0 ? pq[row + ih] : 0.0;
                qv[r] = beta != 0.0 ? qq[row + ih] : 0.0;
            }
        }
#pragma unroll
        for (int r = 0; r < KPT; ++r) {
            const int k = k0 + r;
            if (k < n) {
                const int pp = (j + k + qc) & 1;
                const double a_ip = pp ? side[r] : col[r + 1];
                const double a_im = pp ? col[r + 1] : side[r];
                const double sn = a_ip + a_im + yp[r] + ym[r] + col[r + 2] + col[r];
                const double Az = sigma * zv[r] - c * (sn - 6.0 * zv[r]);
                const double pn = zv[r] + beta * pv[r];
                const double qn = Az + beta * qv[r];
                const int64_t row = (int64_t)H * ((int64_t)j + (int64_t)n * k);
                pq[row + ih] = pn;
                qq[row + ih] = qn;
                v += pn * qn;
            }
        }
    }
    const int tid = threadIdx.x + TX * threadIdx.y;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < (TX * TY) / 64; ++w) s += red[w];
        part[bid.x + (int64_t)gridDim.x * (bid.y + (int64_t)gridDim.y * rem)] = s;
    }
}

// alpha = (r.z) / (p.q), p.q summed from the npq partials of k_cg_dir in a
// fixed order by every block (so all blocks hold the same alpha; block 0 keeps
// it in the state for the next beta); then x += alpha p, r -= alpha q, partials
// of ||r||^2 (part[block]) and of sum x (part[gridDim.x + block], for the mean
// of the converged solution); r32 (mixed) = r / ||b||
constexpr int kUpdThreads = 512, kUpdMaxBlocks = 512;   // (256 x 1024: 22.1 us at 128^3; 512 x 512: 19.7)
__global__ void __launch_bounds__(kUpdThreads)
k_cg_update(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
            const double* __restrict__ q, int64_t n3, MGState* __restrict__ st,
            float* __restrict__ r32, const double* __restrict__ pq_part, int64_t npq, double* __restrict__ part) {
    __shared__ double red[16];
    if (!st->active[0]) return;  // uniform
    double a = 0.0;
    for (int64_t t = threadIdx.x; t < npq; t += kUpdThreads) a += pq_part[t];
    a = block_sum(a, red);
    __shared__ double alpha_s;
    if (threadIdx.x == 0) {
        alpha_s = a != 0.0 ? st->rz / a : 0.0;
        if (blockIdx.x == 0) st->alpha = alpha_s;
    }
    __syncthreads();
    const double alpha = alpha_s, inv_bn = r32 ? 1.0 / st->bn[0] : 0.0;
    const int64_t stride = (int64_t)gridDim.x * kUpdThreads;
    double v = 0.0, sx = 0.0;
    for (int64_t t0 = (int64_t)blockIdx.x * kUpdThreads + threadIdx.x; t0 < n3; t0 += 4 * stride) {
        double xv[4], rv[4], pv[4], qv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t t = t0 + u * stride;
            if (t < n3) {
                xv[u] = x[t];
                rv[u] = r[t];
                pv[u] = p[t];
                qv[u] = q[t];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t t = t0 + u * stride;
            if (t < n3) {
                const double rn = rv[u] - alpha * qv[u];
                const double xn = xv[u] + alpha * pv[u];
                x[t] = xn;
                r[t] = rn;
                v += rn * rn;
                sx += xn;
                if (r32) r32[t] = (float)(rn * inv_bn);
            }
        }
    }
    v = block_sum(v, red);
    sx = block_sum(sx, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = v;
        part[gridDim.x + blockIdx.x] = sx;
    }
}

// reduce the dot partials (slot 0: r.z, slot 1: z.q) in a fixed order; beta and
// the new r.z into the state
__global__ void __launch_bounds__(1024)
k_cg_scalars(const double* __restrict__ part, int64_t nparts, int64_t pstride, MGState* st) {
    __shared__ double red[16];
    if (!st->active[0]) return;  // uniform
    double a = 0.0, b = 0.0;
    for (int64_t t = threadIdx.x; t < nparts; t += blockDim.x) {
        a += part[t];
        b += part[pstride + t];
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    if (threadIdx.x == 0) {
        // a = r.z (new), b = z.q with q = A p of the previous iteration
        st->beta = (st->cycles[0] == 0 || st->rz == 0.0) ? 0.0 : -st->alpha * b / st->rz;
        st->rz = a;
    }
}

// x += ||b|| e (mixed mode)
__global__ void k_update(double* __restrict__ x, const float* __restrict__ e, int64_t cs,
                         const MGState* __restrict__ st) {
    const int comp = blockIdx.y;
    if (!st->active[comp]) return;
    const double s = st->bn[comp];
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < cs; t += (int64_t)gridDim.x * blockDim.x)
        x[comp * cs + t] += s * (double)e[comp * cs + t];
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
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x; t0 < count; t0 += 4 * stride) {
        double v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t t = t0 + r * stride;
            v[r] = t < count ? vc[t] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) s += square ? v[r] * v[r] : v[r];
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[comp * pstride + blockIdx.x] = s;
}

__global__ void k_sub_mean(double* __restrict__ v, int64_t cs, int64_t count,
                           const MGState* __restrict__ st, int all) {
    const int comp = blockIdx.y;
    if (!all && !st->active[comp]) return;
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
    if (mode == FIN_MEAN_BNORM) {
        double s = 0.0, s2 = 0.0;
        for (int64_t t = threadIdx.x; t < nparts; t += blockDim.x) {
            s += part[t];
            s2 += part[pstride + t];
        }
        s = block_sum(s, red);
        s2 = block_sum(s2, red);
        if (threadIdx.x == 0) {
            const double m = s * inv_count;
            st->mean[0] = m;
            st->bn[0] = sqrt(fmax(s2 - s * m, 0.0));   // sum (b - m)^2 = sum b^2 - m sum b
        }
        return;
    }
    for (int comp = 0; comp < ncomp; ++comp) {
        const bool skip = (mode == FIN_CYCLE_R || mode == FIN_MEAN) && !st->active[comp];
        if (skip) continue;  // uniform across the block
        if (mode == FIN_BNORM_INIT_R) {
            double sb = 0.0;
            for (int64_t t = threadIdx.x; t < nparts; t += blockDim.x) sb += part[(ncomp + comp) * pstride + t];
            sb = block_sum(sb, red);
            if (threadIdx.x == 0) st->bn[comp] = sqrt(sb);
            __syncthreads();
        }
        double s = 0.0;
        // loads in batches of 8, summed in index order
        for (int64_t t0 = threadIdx.x; t0 < nparts; t0 += 8 * (int64_t)blockDim.x) {
            double v[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int64_t t = t0 + r * (int64_t)blockDim.x;
                v[r] = t < nparts ? part[comp * pstride + t] : 0.0;
            }
#pragma unroll
            for (int r = 0; r < 8; ++r) s += v[r];
        }
        s = block_sum(s, red);
        if (threadIdx.x == 0) {
            if (mode == FIN_BNORM) {
                st->bn[comp] = sqrt(s);
            } else if (mode == FIN_MEAN || mode == FIN_MEAN_ALL) {
                st->mean[comp] = s * inv_count;
            } else {
                const double bn = st->bn[comp];
                if (mode == FIN_INIT_R || mode == FIN_BNORM_INIT_R) {
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
// all levels with n <= 16 in one workgroup, arrays in LDS in the packed
// red-black layout of the global arrays: a half-sweep reads the other colour
// with unit stride across a wavefront's lanes, and loading or storing a level
// is a straight copy.
//
// The level chain is a compile-time constant (16-8-4, 12-6 or 8-4).  Levels
// above the coarsest use all threads with a workgroup barrier between stages;
// the coarsest level (4^3 or 6^3, many sweeps) runs on wavefront 0 alone: LDS
// operations of one wavefront complete in program order, so a wavefront-scope
// fence between half-sweeps replaces the barrier.  As on the larger levels,
// the first half-sweep from a zero guess reads no neighbours, only red
// residuals are restricted after a pre-smoothing that ends black, and the
// correction is prolongated to red cells only before a post-smoothing that
// starts black.
// ---------------------------------------------------------------------------

template <typename T>
struct SmallArgs {
    int pre, post, sweeps, poisson, zero_init;
    int depth;   // levels below N0 the cycle descends (the last one relaxed by `sweeps`)
    T sigma, nu;
    T omega;     // over-relaxation of the level the cycle stops at (1: Gauss-Seidel)
};

template <int N>
__device__ __forceinline__ int wrapc(int i) {
    return i < 0 ? i + N : (i >= N ? i - N : i);
}

// packed offset of cell (i, j, k) of a level with N cells per side
template <int N>
__device__ __forceinline__ int pkc(int i, int j, int k) {
    return ((i + j + k) & 1) * ((N / 2) * N * N) + (i >> 1) + (N / 2) * (j + N * k);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Exact solve of a coarsest level of at most 16 cells per side of the periodic
// operator sigma I - nu Lap_h, in one workgroup per component:
//   x = Q3 diag(1 / lambda) Q3^T b,  Q3 = Q (x) Q (x) Q,
// with Q the level's real orthonormal Fourier basis (columns: the constant,
// sqrt(2/N) cos(2 pi f j / N) for f = 1 .. N/2 - 1, the alternating (-1)^j,
// sqrt(2/N) sin(2 pi f j / N)) and lambda = sigma + nu (s[m1] + s[m2] + s[m3]),
// s[m] = (4 / h^2) sin^2(pi f(m) / N); lambda = 0 (the Poisson constant mode) is
// dropped.  The three forward and three inverse passes each transform the
// slowest axis of the LDS array and write its index as the fastest of the next
// layout (x, y, z -> mz, x, y -> my, mz, x -> mx, my, mz -> ... -> x, y, z), so
// a wavefront's lanes read consecutive cells; rows are padded to N + 1 values.
// A thread computes CG consecutive outputs of one line; for N = 16 a wavefront's
// output group is uniform, so its coefficients come through the scalar cache.
// ---------------------------------------------------------------------------
constexpr int kExactThreads = 1024, kExactGroup = 4;

template <int N>
constexpr int exact_lds_words() { return 2 * (N + 1) * N * N; }

template <int N, typename T>
__device__ __forceinline__ void exact_pass(const T* __restrict__ in, T* __restrict__ out,
                                           const T* __restrict__ Q, bool forward) {
    constexpr int NP = N + 1, R = N * N, G = N / kExactGroup;
    const int t = threadIdx.x;
    if (t >= R * G) return;
    int grp = t / R;
    if constexpr ((R % 64) == 0) grp = __builtin_amdgcn_readfirstlane(grp);
    const int r = t - grp * R;
    const int f = r % N, sdx = r / N;        // fastest and middle index of the input layout
    T v[N];
#pragma unroll
    for (int a = 0; a < N; ++a) v[a] = in[f + NP * sdx + NP * N * a];
#pragma unroll
    for (int u = 0; u < kExactGroup; ++u) {
        const int o = grp * kExactGroup + u;
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < N; ++a) acc += (forward ? Q[a * N + o] : Q[o * N + a]) * v[a];
        out[o + NP * f + NP * N * sdx] = acc;
    }
}

template <int N, typename T>
__global__ void __launch_bounds__(kExactThreads)
k_coarse_exact(T* __restrict__ xg, const T* __restrict__ bg, int64_t cs, const T* __restrict__ tab,
               T sigma, T nu, const int32_t* __restrict__ active) {
    extern __shared__ unsigned char lds_raw[];
    constexpr int NP = N + 1, N3 = N * N * N;
    T* A = reinterpret_cast<T*>(lds_raw);
    T* B = A + NP * N * N;
    const int comp = blockIdx.x;
    if (!active[comp]) return;
    const T* Q = tab;
    const T* sv = tab + N * N;
    for (int o = threadIdx.x; o < N3; o += kExactThreads) {
        const int i = o % N, j = (o / N) % N, k = o / (N * N);
        A[i + NP * j + NP * N * k] = bg[comp * cs + pkc<N>(i, j, k)];
    }
    __syncthreads();
    exact_pass<N>(A, B, Q, true);     // z
    __syncthreads();
    exact_pass<N>(B, A, Q, true);     // y
    __syncthreads();
    exact_pass<N>(A, B, Q, true);     // x: B holds (mx, my, mz)
    __syncthreads();
    for (int o = threadIdx.x; o < N3; o += kExactThreads) {
        const int m1 = o % N, m2 = (o / N) % N, m3 = o / (N * N);
        const T lam = sigma + nu * (sv[m1] + sv[m2] + sv[m3]);
        T* v = B + m1 + NP * m2 + NP * N * m3;
        *v = lam != T(0) ? *v / lam : T(0);
    }
    __syncthreads();
    exact_pass<N>(B, A, Q, false);    // z
    __syncthreads();
    exact_pass<N>(A, B, Q, false);    // y
    __syncthreads();
    exact_pass<N>(B, A, Q, false);    // x: A holds (x, y, z)
    __syncthreads();
    for (int o = threadIdx.x; o < N3; o += kExactThreads) {
        const int i = o % N, j = (o / N) % N, k = o / (N * N);
        xg[comp * cs + pkc<N>(i, j, k)] = A[i + NP * j + NP * N * k];
    }
}

// The same solve at 24^3 and 32^3, where a component's level no longer fits
// one workgroup's LDS, in three launches of one workgroup per plane:
//   k_exact_fwd_xy  plane k:  b -> transforms along x, then y   -> W[k][my][mx]
//   k_exact_z       plane my: transform along z, divide by lambda, inverse
//                             along z, in place in W
//   k_exact_inv_xy  plane k:  inverse along y, then x           -> x (packed)
// Every output of a pass is one thread's N-term sum over a row of LDS; the
// basis sits in LDS with rows padded to N + 1 values.  W holds N^3 values per
// component.
constexpr int kPlaneThreads = 1024;

template <int N, typename T>
__device__ __forceinline__ void exact_load_basis(T* Qs, const T* __restrict__ tab) {
    for (int t = threadIdx.x; t < N * N; t += kPlaneThreads) Qs[(t / N) * (N + 1) + t % N] = tab[t];
}

template <int N, typename T>
__global__ void __launch_bounds__(kPlaneThreads)
k_exact_fwd_xy(const T* __restrict__ bg, int64_t cs, const T* __restrict__ tab, T* __restrict__ work,
               const int32_t* __restrict__ active) {
    constexpr int NP = N + 1;
    __shared__ T Qs[N * NP], P[N * NP], U[N * NP];
    const int k = blockIdx.x, comp = blockIdx.y;
    if (!active[comp]) return;
    exact_load_basis<N>(Qs, tab);
    for (int t = threadIdx.x; t < N * N; t += kPlaneThreads) {
        const int i = t % N, j = t / N;
        P[j * NP + i] = bg[comp * cs + pkc<N>(i, j, k)];
    }
    __syncthreads();
    const int t = threadIdx.x, a = t % N, r = t / N;
    const bool on = t < N * N;
    if (on) {   // U[j][mx] = sum_i Q[i][mx] b[j][i]
        T acc = T(0);
#pragma unroll 8
        for (int i = 0; i < N; ++i) acc += Qs[i * NP + a] * P[r * NP + i];
        U[r * NP + a] = acc;
    }
    __syncthreads();
    if (on) {   // W[k][my][mx] = sum_j Q[j][my] U[j][mx]
        T acc = T(0);
#pragma unroll 8
        for (int j = 0; j < N; ++j) acc += Qs[j * NP + r] * U[j * NP + a];
        work[(int64_t)comp * N * N * N + (k * N + r) * N + a] = acc;
    }
}

template <int N, typename T>
__global__ void __launch_bounds__(kPlaneThreads)
k_exact_z(T* __restrict__ work, const T* __restrict__ tab, T sigma, T nu,
          const int32_t* __restrict__ active) {
    constexpr int NP = N + 1;
    __shared__ T Qs[N * NP], Z[N * NP], V[N * NP];
    const int my = blockIdx.x, comp = blockIdx.y;
    if (!active[comp]) return;
    const T* sv = tab + N * N;
    T* wc = work + (int64_t)comp * N * N * N;
    exact_load_basis<N>(Qs, tab);
    for (int t = threadIdx.x; t < N * N; t += kPlaneThreads) {
        const int mx = t % N, k = t / N;
        Z[k * NP + mx] = wc[(k * N + my) * N + mx];
    }
    __syncthreads();
    const int t = threadIdx.x, a = t % N, r = t / N;
    const bool on = t < N * N;
    if (on) {   // V[mz][mx] = sum_k Q[k][mz] Z[k][mx] / lambda(mx, my, mz)
        T acc = T(0);
#pragma unroll 8
        for (int k = 0; k < N; ++k) acc += Qs[k * NP + r] * Z[k * NP + a];
        const T lam = sigma + nu * (sv[a] + sv[my] + sv[r]);
        V[r * NP + a] = lam != T(0) ? acc / lam : T(0);
    }
    __syncthreads();
    if (on) {   // W[k][my][mx] = sum_mz Q[k][mz] V[mz][mx]
        T acc = T(0);
#pragma unroll 8
        for (int m = 0; m < N; ++m) acc += Qs[r * NP + m] * V[m * NP + a];
        wc[(r * N + my) * N + a] = acc;
    }
}

template <int N, typename T>
__global__ void __launch_bounds__(kPlaneThreads)
k_exact_inv_xy(T* __restrict__ xg, int64_t cs, const T* __restrict__ tab, const T* __restrict__ work,
               const int32_t* __restrict__ active) {
    constexpr int NP = N + 1;
    __shared__ T Qs[N * NP], P[N * NP], U[N * NP];
    const int k = blockIdx.x, comp = blockIdx.y;
    if (!active[comp]) return;
    const T* wc = work + (int64_t)comp * N * N * N;
    exact_load_basis<N>(Qs, tab);
    for (int t = threadIdx.x; t < N * N; t += kPlaneThreads) P[(t / N) * NP + t % N] = wc[k * N * N + t];
    __syncthreads();
    const int t = threadIdx.x, a = t % N, r = t / N;
    const bool on = t < N * N;
    if (on) {   // U[j][mx] = sum_my Q[j][my] W[k][my][mx]
        T acc = T(0);
#pragma unroll 8
        for (int m = 0; m < N; ++m) acc += Qs[r * NP + m] * P[m * NP + a];
        U[r * NP + a] = acc;
    }
    __syncthreads();
    if (on) {   // x[k][j][i] = sum_mx Q[i][mx] U[j][mx]
        T acc = T(0);
#pragma unroll 8
        for (int m = 0; m < N; ++m) acc += Qs[a * NP + m] * U[r * NP + m];
        xg[comp * cs + pkc<N>(a, r, k)] = acc;
    }
}

// sum of the six neighbours (order i+1, i-1, j+1, j-1, k+1, k-1) of the
// colour-q cell at packed position (ih, j, k), from the other colour's half xo
template <int N, typename T>
__device__ __forceinline__ T s_nbr(const T* xo, int ih, int j, int k, int q) {
    constexpr int H = N / 2;
    const int p = (j + k + q) & 1;
    int ip = ih + p, im = ih + p - 1;
    if (ip >= H) ip -= H;
    if (im < 0) im += H;
    const int row = H * (j + N * k);
    return xo[row + ip] + xo[row + im] + xo[H * (wrapc<N>(j + 1) + N * k) + ih] +
           xo[H * (wrapc<N>(j - 1) + N * k) + ih] + xo[H * (j + N * wrapc<N>(k + 1)) + ih] +
           xo[H * (j + N * wrapc<N>(k - 1)) + ih];
}

// colour-q half-sweep over packed cells t0, t0 + nt, ...; zg: the other colour
// is zero; omega != 1: over-relaxed, x += omega (x_gs - x), with the cell's own
// old value taken as zero when zo
template <int N, typename T>
__device__ __forceinline__ void s_gs(T* x, const T* b, T c, T inv_diag, int q, int t0, int nt,
                                     bool zg = false, T omega = T(1), bool zo = false) {
    constexpr int H = N / 2, HALF = H * N * N;
    const T* xo = x + (1 - q) * HALF;
    for (int t = t0; t < HALF; t += nt) {
        const int ih = t % H, rest = t / H;
        const int j = rest % N, k = rest / N;
        const T s = zg ? T(0) : s_nbr<N>(xo, ih, j, k, q);
        const T xg = (b[q * HALF + t] + c * s) * inv_diag;
        if (omega == T(1)) {
            x[q * HALF + t] = xg;
        } else {
            const T xq = zo ? T(0) : x[q * HALF + t];
            x[q * HALF + t] = xq + omega * (xg - xq);
        }
    }
}

// residual of the colour-q cells into r
template <int N, typename T>
__device__ __forceinline__ void s_residual(const T* x, const T* b, T* r, T sigma, T c, int q) {
    constexpr int H = N / 2, HALF = H * N * N;
    const T* xo = x + (1 - q) * HALF;
    for (int t = threadIdx.x; t < HALF; t += blockDim.x) {
        const int ih = t % H, rest = t / H;
        const int j = rest % N, k = rest / N;
        const T xv = x[q * HALF + t];
        const T s = s_nbr<N>(xo, ih, j, k, q);
        r[q * HALF + t] = b[q * HALF + t] - (sigma * xv - c * (s - T(6) * xv));
    }
}

// coarse b (packed order) = restriction of r; red_only: black residuals are
// zero and not read
template <int NF, typename T>
__device__ __forceinline__ void s_restrict(const T* r, T* bc, bool red_only) {
    constexpr int NC = NF / 2, HC = NC / 2, HALFC = HC * NC * NC;
    const T w[4] = {T(1), T(3), T(3), T(1)};
    for (int o = threadIdx.x; o < 2 * HALFC; o += blockDim.x) {
        const int Q = o / HALFC, t = o - Q * HALFC;
        const int Ih = t % HC, rest = t / HC;
        const int J = rest % NC, K = rest / NC;
        const int I = 2 * Ih + ((J + K + Q) & 1);
        T s = T(0);
        for (int cz = 0; cz < 4; ++cz) {
            const int k = wrapc<NF>(2 * K - 1 + cz);
            for (int cy = 0; cy < 4; ++cy) {
                const int j = wrapc<NF>(2 * J - 1 + cy);
                for (int cx = 0; cx < 4; ++cx) {
                    const int i = wrapc<NF>(2 * I - 1 + cx);
                    if (red_only && ((i + j + k) & 1)) continue;
                    s += w[cx] * w[cy] * w[cz] / T(512) * r[pkc<NF>(i, j, k)];
                }
            }
        }
        bc[o] = s;
    }
}

// fine x += trilinear prolongation of xc on the red cells (red_only) or all
template <int NF, typename T>
__device__ __forceinline__ void s_prolong_add(T* x, const T* xc, bool red_only) {
    constexpr int NC = NF / 2, H = NF / 2, HALF = H * NF * NF;
    const T wt[2] = {T(0.75), T(0.25)};
    const int cnt = red_only ? HALF : 2 * HALF;
    for (int o = threadIdx.x; o < cnt; o += blockDim.x) {
        const int q = o / HALF, t = o - q * HALF;
        const int ih = t % H, rest = t / H;
        const int j = rest % NF, k = rest / NF;
        const int ijk[3] = {2 * ih + ((j + k + q) & 1), j, k};
        int base[3][2];
        for (int d = 0; d < 3; ++d) {
            const int I = ijk[d] >> 1;
            base[d][0] = I;
            base[d][1] = (ijk[d] & 1) ? wrapc<NC>(I + 1) : wrapc<NC>(I - 1);
        }
        T v = T(0);
        for (int cz = 0; cz < 2; ++cz)
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx)
                    v += wt[cx] * wt[cy] * wt[cz] * xc[pkc<NC>(base[0][cx], base[1][cy], base[2][cz])];
        x[o] += v;
    }
}

template <int N, typename T>
__device__ __forceinline__ void level_coef(const SmallArgs<T>& A, T& c, T& inv_diag) {
    const T h = T(1) / T(N);
    c = A.nu / (h * h);
    inv_diag = T(1) / (A.sigma + T(6) * c);
}

// coarsest level on wavefront 0 from a zero guess: sweeps, Poisson mean removal
template <int N, typename T>
__device__ __forceinline__ void s_coarse_wave(T* x, const T* b, const SmallArgs<T>& A) {
    constexpr int CNT = N * N * N;
    const int lane = threadIdx.x;
    T c, inv_diag;
    level_coef<N>(A, c, inv_diag);
    if (A.sweeps <= 0)
        for (int o = lane; o < CNT; o += 64) x[o] = T(0);
    wave_sync();
    for (int s = 0; s < A.sweeps; ++s) {
        s_gs<N>(x, b, c, inv_diag, 0, lane, 64, s == 0, A.omega, s == 0);
        wave_sync();
        s_gs<N>(x, b, c, inv_diag, 1, lane, 64, false, A.omega, s == 0);
        wave_sync();
    }
    if (A.poisson) {
        T v = T(0);
        for (int o = lane; o < CNT; o += 64) v += x[o];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        const T m = v / T(CNT);
        wave_sync();
        for (int o = lane; o < CNT; o += 64) x[o] -= m;
        wave_sync();
    }
}

// one level above the coarsest: pre-smoothing, residual and restriction
// (down); zero: x is zero on entry (its contents are not read)
template <int N, typename T>
__device__ __forceinline__ void s_down(T* x, const T* b, T* r, T* bnext, const SmallArgs<T>& A, bool zero) {
    constexpr int CNT = N * N * N;
    T c, inv_diag;
    level_coef<N>(A, c, inv_diag);
    if (zero && A.pre <= 0) {
        for (int o = threadIdx.x; o < CNT; o += blockDim.x) x[o] = T(0);
        __syncthreads();
    }
    for (int s = 0; s < A.pre; ++s) {
        s_gs<N>(x, b, c, inv_diag, 0, threadIdx.x, blockDim.x, zero && s == 0);
        __syncthreads();
        s_gs<N>(x, b, c, inv_diag, 1, threadIdx.x, blockDim.x);
        __syncthreads();
    }
    const bool red_only = A.pre > 0;
    s_residual<N>(x, b, r, A.sigma, c, 0);
    if (!red_only) s_residual<N>(x, b, r, A.sigma, c, 1);
    __syncthreads();
    s_restrict<N>(r, bnext, red_only);
    __syncthreads();
}

// prolongation and post-smoothing (up)
template <int N, typename T>
__device__ __forceinline__ void s_up(T* x, const T* b, const T* xc, const SmallArgs<T>& A) {
    T c, inv_diag;
    level_coef<N>(A, c, inv_diag);
    s_prolong_add<N>(x, xc, A.post > 0);
    __syncthreads();
    for (int s = 0; s < A.post; ++s) {
        s_gs<N>(x, b, c, inv_diag, 1, threadIdx.x, blockDim.x);
        __syncthreads();
        s_gs<N>(x, b, c, inv_diag, 0, threadIdx.x, blockDim.x);
        __syncthreads();
    }
}

// the level the cycle stops at, relaxed by all threads from x (zero: x = 0 on
// entry, not read)
template <int N, typename T>
__device__ __forceinline__ void s_relax(T* x, const T* b, const SmallArgs<T>& A, bool zero) {
    T c, inv_diag;
    level_coef<N>(A, c, inv_diag);
    for (int s = 0; s < A.sweeps; ++s) {
        const bool z = zero && s == 0;
        s_gs<N>(x, b, c, inv_diag, 0, threadIdx.x, blockDim.x, z, A.omega, z);
        __syncthreads();
        s_gs<N>(x, b, c, inv_diag, 1, threadIdx.x, blockDim.x, false, A.omega, z);
        __syncthreads();
    }
}

// One V-cycle over the levels N0 (, N0/2, ...) down to the coarsest (< 8), or
// down to A.depth levels below N0 when the cycle stops earlier.
// LDS holds [x, b, r] per level, packed like the global arrays.
template <int N0, typename T>
__global__ void __launch_bounds__(kSmallThreads)
k_small_vcycle(T* __restrict__ xg, const T* __restrict__ bg, int64_t cs, SmallArgs<T> A,
               const int32_t* __restrict__ active) {
    extern __shared__ unsigned char lds_raw[];
    T* lds = reinterpret_cast<T*>(lds_raw);
    const int comp = blockIdx.x;
    if (!active[comp]) return;
    constexpr int N1 = N0 / 2;
    constexpr int C0 = N0 * N0 * N0, C1 = N1 * N1 * N1;
    T* x0 = lds;
    T* b0 = x0 + C0;
    T* r0 = b0 + C0;
    T* x1 = r0 + C0;
    T* b1 = x1 + C1;
    T* r1 = b1 + C1;
    {
        // all of a thread's loads are issued before the first LDS store
        constexpr int R = (C0 + kSmallThreads - 1) / kSmallThreads;
        const bool load_x = !A.zero_init;
        T bv[R], xv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int o = threadIdx.x + r * kSmallThreads;
            if (o < C0) {
                bv[r] = bg[comp * cs + o];
                if (load_x) xv[r] = xg[comp * cs + o];
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int o = threadIdx.x + r * kSmallThreads;
            if (o < C0) {
                b0[o] = bv[r];
                if (load_x) x0[o] = xv[r];
            }
        }
    }
    __syncthreads();
    if (A.depth == 0) {
        // N0 is the level the cycle stops at
        s_relax<N0>(x0, b0, A, A.zero_init != 0);
        for (int o = threadIdx.x; o < C0; o += blockDim.x) xg[comp * cs + o] = x0[o];
        return;
    }
    s_down<N0>(x0, b0, r0, b1, A, A.zero_init != 0);
    if constexpr (N1 >= 8) {
        constexpr int N2 = N1 / 2;
        constexpr int C2 = N2 * N2 * N2;
        T* x2 = r1 + C1;
        T* b2 = x2 + C2;
        if (A.depth == 1) {
            // N1 is the level the cycle stops at
            if (threadIdx.x < 64) s_coarse_wave<N1>(x1, b1, A);
            __syncthreads();
        } else {
            s_down<N1>(x1, b1, r1, b2, A, true);
            if (threadIdx.x < 64) s_coarse_wave<N2>(x2, b2, A);
            __syncthreads();
            s_up<N1>(x1, b1, x2, A);
        }
    } else {
        (void)r1;
        if (threadIdx.x < 64) s_coarse_wave<N1>(x1, b1, A);
        __syncthreads();
    }
    s_up<N0>(x0, b0, x1, A);
    for (int o = threadIdx.x; o < C0; o += blockDim.x) xg[comp * cs + o] = x0[o];
}

// ---------------------------------------------------------------------------
// coarse levels above the single-workgroup ones: one launch per half of the
// V-cycle on a level.  Used for V(2,2) with a zero guess (always the case
// below the finest level) on levels with n a multiple of 8.
//
// A workgroup owns an 8^3 block of the level (a 4^3 block of the next one)
// and recomputes in LDS every cell its result depends on, with the arithmetic
// of the separate kernels in the same order:
//   k_level_down: red (from x = 0), black, red, black half-sweeps on boxes
//     reaching 5, 4, 3, 2 cells beyond the block; red-cell residuals on the
//     restriction window (1 cell beyond; black residuals are zero after the
//     black half-sweep); restriction into the next level's b; the smoothed x
//     of the block is kept for k_level_up.
//   k_level_up: x_red += prolongated coarse correction on a box reaching 4
//     cells beyond the block; black, red, black, red half-sweeps on boxes
//     reaching 3, 2, 1, 0 cells; the block's x is stored.
// Blocks read neighbours' cells only from arrays no launch of the pair writes,
// so there is no ordering between workgroups.
// ---------------------------------------------------------------------------

constexpr int KB = 8;                                 // owned cells per axis
constexpr int KDH = 5, KUH = 4;                       // halos of the down / up kernels
constexpr int KDE = KB + 2 * KDH, KUE = KB + 2 * KUH; // LDS box sides (18, 16)
constexpr int KW = KB + 2;                            // restriction window side
constexpr int KTHREADS = 1024;

template <int E>
__device__ __forceinline__ int lix(int a, int b, int c) { return a + E * (b + E * c); }

// packed offset inside a component of the cell at unwrapped (gi, gj, gk)
__device__ __forceinline__ int64_t pkw(int gi, int gj, int gk, int n) {
    return pk(wrapi(gi, n), wrapi(gj, n), wrapi(gk, n), n);
}

// Colour-q cells of the box reaching D cells beyond the owned block (local
// origin: global cell (g0x, g0y, g0z) at LDS index 0, block at HH):
// x = (b + c * neighbour sum) * inv_diag; zg: neighbours are zero.  Each
// thread first loads b for all its cells (all loads in flight), then updates.
template <int E, int HH, int D, typename T>
__device__ __forceinline__ void box_gs(T* xs, const T* __restrict__ bg, int n, int g0x, int g0y,
                                       int g0z, int q, T c, T inv_diag, bool zg) {
    constexpr int lo = HH - D, S = KB + 2 * D, S2 = S / 2;
    constexpr int cnt = S2 * S * S, R = (cnt + KTHREADS - 1) / KTHREADS;
    T bv[R];
    int oo[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int u = threadIdx.x + r * KTHREADS;
        oo[r] = -1;
        if (u < cnt) {
            const int ah = u % S2, rest = u / S2;
            const int lb = lo + rest % S, lc = lo + rest / S;
            const int la = lo + 2 * ah + ((q + g0x + lo + g0y + lb + g0z + lc) & 1);
            oo[r] = lix<E>(la, lb, lc);
            bv[r] = bg[pkw(g0x + la, g0y + lb, g0z + lc, n)];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int o = oo[r];
        if (o >= 0) {
            T sum = T(0);
            if (!zg)
                sum = xs[o + 1] + xs[o - 1] + xs[o + E] + xs[o - E] + xs[o + E * E] + xs[o - E * E];
            xs[o] = (bv[r] + c * sum) * inv_diag;
        }
    }
}

__device__ __forceinline__ void level_block(int n, int& comp, int& i0, int& j0, int& k0) {
    const int nb = n / KB, nb3 = nb * nb * nb;
    comp = blockIdx.x / nb3;
    const int r = blockIdx.x - comp * nb3;
    i0 = KB * (r % nb);
    j0 = KB * ((r / nb) % nb);
    k0 = KB * (r / (nb * nb));
}

template <typename T>
__global__ void __launch_bounds__(KTHREADS)
k_level_down(const T* __restrict__ b, T* __restrict__ xpre, int n, int64_t cs, T* __restrict__ bc,
             int64_t ccs, T sigma, T c, T inv_diag, const int32_t* __restrict__ active) {
    __shared__ T xs[KDE * KDE * KDE];
    __shared__ T rw[KW * KW * KW];
    int comp, i0, j0, k0;
    level_block(n, comp, i0, j0, k0);
    if (!active[comp]) return;
    const int g0x = i0 - KDH, g0y = j0 - KDH, g0z = k0 - KDH;
    const T* bcp = b + comp * cs;
    constexpr int CW = KW * KW * KW;
    for (int u = threadIdx.x; u < CW; u += KTHREADS) rw[u] = T(0);   // black entries stay zero
    // Each thread owns up to RR red cells of the box reaching 5 cells beyond the
    // block and up to RK black cells of the one reaching 4 (the cells of the
    // first half-sweep of each colour, numbered as in box_gs); their b is
    // loaded once, and each later half-sweep updates the owned cells inside its
    // smaller box (distance from the block: the largest per-axis overhang).
    constexpr int S5 = KB + 10, CR = (S5 / 2) * S5 * S5, RR = (CR + KTHREADS - 1) / KTHREADS;
    constexpr int S4 = KB + 8, CK = (S4 / 2) * S4 * S4, RK = (CK + KTHREADS - 1) / KTHREADS;
    auto dist = [](int la, int lb, int lc) {
        const int dx = max(max(KDH - la, la - (KDH + KB - 1)), 0);
        const int dy = max(max(KDH - lb, lb - (KDH + KB - 1)), 0);
        const int dz = max(max(KDH - lc, lc - (KDH + KB - 1)), 0);
        return max(dx, max(dy, dz));
    };
    T br[RR], bk[RK];
    int orr[RR], ork[RK], dr[RR], dk[RK], wr[RR];
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int u = threadIdx.x + r * KTHREADS;
        orr[r] = -1;
        if (u < CR) {
            const int lo = KDH - 5, ah = u % (S5 / 2), rest = u / (S5 / 2);
            const int lb = lo + rest % S5, lc = lo + rest / S5;
            const int la = lo + 2 * ah + ((g0x + lo + g0y + lb + g0z + lc) & 1);
            orr[r] = lix<KDE>(la, lb, lc);
            dr[r] = dist(la, lb, lc);
            wr[r] = dr[r] <= 1 ? lix<KW>(la - (KDH - 1), lb - (KDH - 1), lc - (KDH - 1)) : -1;
            br[r] = bcp[pkw(g0x + la, g0y + lb, g0z + lc, n)];
        }
    }
#pragma unroll
    for (int r = 0; r < RK; ++r) {
        const int u = threadIdx.x + r * KTHREADS;
        ork[r] = -1;
        if (u < CK) {
            const int lo = KDH - 4, ah = u % (S4 / 2), rest = u / (S4 / 2);
            const int lb = lo + rest % S4, lc = lo + rest / S4;
            const int la = lo + 2 * ah + ((1 + g0x + lo + g0y + lb + g0z + lc) & 1);
            ork[r] = lix<KDE>(la, lb, lc);
            dk[r] = dist(la, lb, lc);
            bk[r] = bcp[pkw(g0x + la, g0y + lb, g0z + lc, n)];
        }
    }
    auto nsum = [&](int o) {
        return xs[o + 1] + xs[o - 1] + xs[o + KDE] + xs[o - KDE] + xs[o + KDE * KDE] + xs[o - KDE * KDE];
    };
    // red from x = 0, black, red, black on boxes reaching 5, 4, 3, 2 cells
#pragma unroll
    for (int r = 0; r < RR; ++r)
        if (orr[r] >= 0) xs[orr[r]] = (br[r] + c * T(0)) * inv_diag;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RK; ++r)
        if (ork[r] >= 0) xs[ork[r]] = (bk[r] + c * nsum(ork[r])) * inv_diag;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RR; ++r)
        if (orr[r] >= 0 && dr[r] <= 3) xs[orr[r]] = (br[r] + c * nsum(orr[r])) * inv_diag;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RK; ++r)
        if (ork[r] >= 0 && dk[r] <= 2) xs[ork[r]] = (bk[r] + c * nsum(ork[r])) * inv_diag;
    __syncthreads();
    // red residuals on the restriction window (1 cell beyond the block)
#pragma unroll
    for (int r = 0; r < RR; ++r)
        if (orr[r] >= 0 && wr[r] >= 0) {
            const T xo = xs[orr[r]];
            rw[wr[r]] = br[r] - (sigma * xo - c * (nsum(orr[r]) - T(6) * xo));
        }
    // the block's smoothed x
    T* xp = xpre + comp * cs;
    for (int u = threadIdx.x; u < KB * KB * KB; u += KTHREADS) {
        const int a = u % KB, bb = (u / KB) % KB, cc = u / (KB * KB);
        xp[pk(i0 + a, j0 + bb, k0 + cc, n)] = xs[lix<KDE>(KDH + a, KDH + bb, KDH + cc)];
    }
    __syncthreads();
    constexpr int KC = KB / 2;
    if (threadIdx.x < KC * KC * KC) {
        const int ci = threadIdx.x % KC, cj = (threadIdx.x / KC) % KC, ck = threadIdx.x / (KC * KC);
        const T w[4] = {T(1), T(3), T(3), T(1)};
        T sum = T(0);
        for (int cz = 0; cz < 4; ++cz)
            for (int cy = 0; cy < 4; ++cy)
                for (int cx = 0; cx < 4; ++cx)
                    sum += w[cx] * w[cy] * w[cz] / T(512) * rw[lix<KW>(2 * ci + cx, 2 * cj + cy, 2 * ck + cz)];
        bc[comp * ccs + pk(i0 / 2 + ci, j0 / 2 + cj, k0 / 2 + ck, n / 2)] = sum;
    }
}

template <typename T>
__global__ void __launch_bounds__(KTHREADS)
k_level_up(const T* __restrict__ b, const T* __restrict__ xpre, const T* __restrict__ xc,
           T* __restrict__ x, int n, int64_t cs, int64_t ccs, T c, T inv_diag,
           const int32_t* __restrict__ active) {
    __shared__ T xs[KUE * KUE * KUE];
    int comp, i0, j0, k0;
    level_block(n, comp, i0, j0, k0);
    if (!active[comp]) return;
    const int g0x = i0 - KUH, g0y = j0 - KUH, g0z = k0 - KUH;
    const int nc = n / 2;
    const T* bcp = b + comp * cs;
    const T* xpp = xpre + comp * cs;
    const T* xcc = xc + comp * ccs;
    // the coarse correction around the block (the 10^3 coarse cells the
    // trilinear prolongation reaches from the box) in LDS, read once
    constexpr int KCE = (KUE / 2) + 2;
    __shared__ T cs_[KCE * KCE * KCE];
    const int c0x = g0x / 2 - 1, c0y = g0y / 2 - 1, c0z = g0z / 2 - 1;   // (g0 even)
    for (int u = threadIdx.x; u < KCE * KCE * KCE; u += KTHREADS) {
        const int a = u % KCE, bb = (u / KCE) % KCE, cc = u / (KCE * KCE);
        cs_[u] = xcc[pk(wrapi(c0x + a, nc), wrapi(c0y + bb, nc), wrapi(c0z + cc, nc), nc)];
    }
    __syncthreads();
    // red cells of the whole box: smoothed x plus the trilinear correction
    {
        constexpr int S = KUE, S2 = S / 2, CNT = S2 * S * S;
        const T wt[2] = {T(0.75), T(0.25)};
        constexpr int R = (CNT + KTHREADS - 1) / KTHREADS;
        T xv[R];
        int oo[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int u = threadIdx.x + r * KTHREADS;
            oo[r] = -1;
            if (u < CNT) {
                const int ah = u % S2, rest = u / S2;
                const int lb = rest % S, lc = rest / S;
                const int la = 2 * ah + ((g0x + g0y + lb + g0z + lc) & 1);
                xv[r] = xpp[pkw(g0x + la, g0y + lb, g0z + lc, n)];
                oo[r] = lix<KUE>(la, lb, lc);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (oo[r] >= 0) {
                const int u = threadIdx.x + r * KTHREADS;
                const int ah = u % S2, rest = u / S2;
                const int lb = rest % S, lc = rest / S;
                const int la = 2 * ah + ((g0x + g0y + lb + g0z + lc) & 1);
                // per axis: nearest coarse cell (unwrapped fine index >> 1) and the next
                const int l3[3] = {g0x + la, g0y + lb, g0z + lc};
                const int c3[3] = {c0x, c0y, c0z};
                int base[3][2];
                for (int d = 0; d < 3; ++d) {
                    const int I = (l3[d] >> 1) - c3[d];
                    base[d][0] = I;
                    base[d][1] = (l3[d] & 1) ? I + 1 : I - 1;
                }
                T v = T(0);
                for (int cz = 0; cz < 2; ++cz)
                    for (int cy = 0; cy < 2; ++cy)
                        for (int cx = 0; cx < 2; ++cx)
                            v += wt[cx] * wt[cy] * wt[cz] * cs_[lix<KCE>(base[0][cx], base[1][cy], base[2][cz])];
                xs[oo[r]] = xv[r] + v;
            }
        }
    }
    __syncthreads();
    box_gs<KUE, KUH, 3>(xs, bcp, n, g0x, g0y, g0z, 1, c, inv_diag, false);
    __syncthreads();
    box_gs<KUE, KUH, 2>(xs, bcp, n, g0x, g0y, g0z, 0, c, inv_diag, false);
    __syncthreads();
    box_gs<KUE, KUH, 1>(xs, bcp, n, g0x, g0y, g0z, 1, c, inv_diag, false);
    __syncthreads();
    box_gs<KUE, KUH, 0>(xs, bcp, n, g0x, g0y, g0z, 0, c, inv_diag, false);
    __syncthreads();
    T* xo = x + comp * cs;
    for (int u = threadIdx.x; u < KB * KB * KB; u += KTHREADS) {
        const int a = u % KB, bb = (u / KB) % KB, cc = u / (KB * KB);
        xo[pk(i0 + a, j0 + bb, k0 + cc, n)] = xs[lix<KUE>(KUH + a, KUH + bb, KUH + cc)];
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

int64_t norm_parts(int n) {
    return (int64_t)((n / 2 + TX - 1) / TX) * ((n + TY - 1) / TY) * 2 * ((n + KPT - 1) / KPT);
}

dim3 norm_grid(int n, int ncomp) {
    return dim3((n / 2 + TX - 1) / TX, (n + TY - 1) / TY, 2 * ((n + KPT - 1) / KPT) * ncomp);
}

int sum_blocks(int64_t count) {
    int64_t b = (count + 255) / 256;
    return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

// workgroups of the conjugate-gradient update pass
int update_blocks(int64_t count) {
    int64_t b = (count + kUpdThreads - 1) / kUpdThreads;
    return (int)(b < kUpdMaxBlocks ? (b < 1 ? 1 : b) : kUpdMaxBlocks);
}

struct OpCoef {
    double sigma, nu;
    int poisson;
};

OpCoef op_coef(const hipib_ctx* ctx, int op) {
    if (op == HIPIB_OP_POISSON) return {0.0, 1.0, 1};
    return {ctx->cfg.rho / ctx->cfg.dt, ctx->cfg.mu, 0};
}

// The level at which a cycle stops descending.  On a level of spacing h the
// Helmholtz operator's Jacobi iteration has spectral radius
// rho = 6c / (sigma + 6c), c = nu / h^2 (the constant mode of the periodic
// operator, whose Jacobi spectrum is real), and red-black ordering is
// consistently ordered, so red-black SOR with Young's factor
// omega = 2 / (1 + sqrt(1 - rho^2)) contracts every error component by
// omega - 1 per sweep.  The Helmholtz hierarchy stops at the first level
// l >= 0 with rho_l <= 1/2 (sigma >= 6 nu / h_l^2: at most 0.072 per sweep;
// a coarse-grid correction adds less than its sweeps would), relaxed there
// with that level's omega.  Otherwise (and for Poisson) the coarsest level
// is the first with fewer than 8 cells per side.
// The coarsest level: with mg_coarse_sweeps = 0 the first with at most 32 cells
// per side, solved exactly (k_coarse_exact, k_exact_*); otherwise the first
// with fewer than 8, relaxed by the coarse sweeps.
bool exact_coarse(const hipib_ctx* ctx) { return ctx->cfg.mg_coarse_sweeps == 0; }
int bottom_level(const hipib_ctx* ctx) { return exact_coarse(ctx) ? ctx->exact_level : ctx->L - 1; }

int stop_level(const hipib_ctx* ctx, const OpCoef& oc) {
    const int bottom = bottom_level(ctx);
    if (oc.sigma > 0.0)
        for (int l = 0; l < bottom; ++l) {
            const double h = 1.0 / ctx->lv[l].n;
            if (oc.sigma >= 6.0 * oc.nu / (h * h)) return l;
        }
    return bottom;
}

// red+black sweeps that relax the level a cycle stops at: the coarse sweeps
// on the coarsest level, pre + post sweeps on the iterate when the finest
// level is the stop (the cycle has no coarse levels), else max(pre, 1) from
// zero
int stop_sweeps(const hipib_ctx* ctx, int lc) {
    if (lc == bottom_level(ctx)) return ctx->cfg.mg_coarse_sweeps;
    if (lc == 0) return ctx->cfg.mg_pre + ctx->cfg.mg_post;
    return ctx->cfg.mg_pre > 1 ? ctx->cfg.mg_pre : 1;
}

// Young's over-relaxation factor of a Helmholtz level (1 for Poisson)
double level_omega(int n, const OpCoef& oc) {
    if (!(oc.sigma > 0.0)) return 1.0;
    const double h = 1.0 / n, c = oc.nu / (h * h);
    const double rho = 6.0 * c / (oc.sigma + 6.0 * c);
    return 2.0 / (1.0 + std::sqrt(1.0 - rho * rho));
}

// reduce the partials at ctx->part + offset
hipib_status finalize_at(hipib_ctx* ctx, int64_t offset, int64_t nparts, int64_t pstride, int ncomp, int mode,
                         double inv_count) {
    return launch_k(ctx, HIPIB_TIMER_REDUCE, 8.0 * (double)nparts * ncomp, k_finalize, dim3(1), dim3(1024), 0,
                    ctx->part + offset, nparts, pstride, ncomp, mode, ctx->st, ctx->cfg.mg_rtol,
                    ctx->cfg.mg_max_cycles, ctx->cfg.mg_fixed_cycles, inv_count);
}

hipib_status finalize(hipib_ctx* ctx, int64_t nparts, int64_t pstride, int ncomp, int mode,
                      double inv_count) {
    return finalize_at(ctx, 0, nparts, pstride, ncomp, mode, inv_count);
}

template <typename T>
hipib_status zero_t(hipib_ctx* ctx, T* p, int64_t count) {
    if (count <= 0) return HIPIB_OK;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_zero_t<T><<<(unsigned)blocks, 256, 0, ctx->stream>>>(p, count);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

// level arrays of the V-cycle type T: level 0 given by the caller of vcycle
template <typename T>
struct LevelPtr {
    T* x;
    const T* b;
    int64_t cs;
};

template <typename T>
T* level_x(hipib_ctx* ctx, int l) { return static_cast<T*>(ctx->lv[l].x); }
template <typename T>
T* level_b(hipib_ctx* ctx, int l) { return static_cast<T*>(ctx->lv[l].b); }

template <typename T>
const T* exact_table(const hipib_ctx* ctx);
template <>
const double* exact_table<double>(const hipib_ctx* ctx) { return ctx->coarse_tab; }
template <>
const float* exact_table<float>(const hipib_ctx* ctx) { return ctx->coarse_tab32; }

// exact solve of the coarsest level l (the first with at most 32 cells per side)
template <typename T>
hipib_status coarse_exact(hipib_ctx* ctx, int l, LevelPtr<T> p, int ncomp, const OpCoef& oc) {
    const int n = ctx->lv[l].n;
    const dim3 grid(ncomp), blk(kExactThreads);
    const int32_t* act = ctx->st->active;
    const double bytes = 2.0 * sizeof(T) * (double)ctx->lv[l].n3 * ncomp;
    const T* tab = exact_table<T>(ctx);
    if (n == 16)
        return launch_k(ctx, HIPIB_TIMER_SMALL_VCYCLE, bytes, k_coarse_exact<16, T>, grid, blk,
                        exact_lds_words<16>() * sizeof(T), p.x, p.b, p.cs, tab, (T)oc.sigma, (T)oc.nu, act);
    if (n == 12)
        return launch_k(ctx, HIPIB_TIMER_SMALL_VCYCLE, bytes, k_coarse_exact<12, T>, grid, blk,
                        exact_lds_words<12>() * sizeof(T), p.x, p.b, p.cs, tab, (T)oc.sigma, (T)oc.nu, act);
    if (n == 8)
        return launch_k(ctx, HIPIB_TIMER_SMALL_VCYCLE, bytes, k_coarse_exact<8, T>, grid, blk,
                        exact_lds_words<8>() * sizeof(T), p.x, p.b, p.cs, tab, (T)oc.sigma, (T)oc.nu, act);
    T* work = static_cast<T*>(ctx->coarse_work);
    if (n == 32 || n == 24) {
        const dim3 pg(n, ncomp), pb(kPlaneThreads);
        const double wb = sizeof(T) * (double)ctx->lv[l].n3 * ncomp;
        if (n == 32) {
            HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_SMALL_VCYCLE, wb * 2, k_exact_fwd_xy<32, T>, pg, pb, 0, p.b, p.cs,
                               tab, work, act));
            HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_SMALL_VCYCLE, wb * 2, k_exact_z<32, T>, pg, pb, 0, work, tab,
                               (T)oc.sigma, (T)oc.nu, act));
            return launch_k(ctx, HIPIB_TIMER_SMALL_VCYCLE, wb * 2, k_exact_inv_xy<32, T>, pg, pb, 0, p.x, p.cs,
                            tab, work, act);
        }
        HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_SMALL_VCYCLE, wb * 2, k_exact_fwd_xy<24, T>, pg, pb, 0, p.b, p.cs,
                           tab, work, act));
        HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_SMALL_VCYCLE, wb * 2, k_exact_z<24, T>, pg, pb, 0, work, tab,
                           (T)oc.sigma, (T)oc.nu, act));
        return launch_k(ctx, HIPIB_TIMER_SMALL_VCYCLE, wb * 2, k_exact_inv_xy<24, T>, pg, pb, 0, p.x, p.cs, tab,
                        work, act);
    }
    return fail(HIPIB_E_INVAL, "no exact coarse solve for n = %d", n);
}

template <typename T>
hipib_status small_vcycle(hipib_ctx* ctx, int l, LevelPtr<T> p, int ncomp, const OpCoef& oc,
                          bool zero_init) {
    SmallArgs<T> A{};
    const int lc = stop_level(ctx, oc);
    A.pre = ctx->cfg.mg_pre;
    A.post = ctx->cfg.mg_post;
    A.sweeps = stop_sweeps(ctx, lc);
    A.depth = lc - l;
    A.omega = (T)level_omega(ctx->lv[lc].n, oc);
    A.poisson = oc.poisson;
    A.zero_init = zero_init ? 1 : 0;
    A.sigma = (T)oc.sigma;
    A.nu = (T)oc.nu;
    const int n = ctx->lv[l].n;
    const dim3 grid(ncomp), blk(kSmallThreads);
    const int32_t* act = ctx->st->active;
    const double bytes = 2.0 * sizeof(T) * (double)ctx->lv[l].n3 * ncomp;
    if (n == 16)
        return launch_k(ctx, HIPIB_TIMER_SMALL_VCYCLE, bytes, k_small_vcycle<16, T>, grid, blk, ctx->small_lds,
                        p.x, p.b, p.cs, A, act);
    if (n == 12)
        return launch_k(ctx, HIPIB_TIMER_SMALL_VCYCLE, bytes, k_small_vcycle<12, T>, grid, blk, ctx->small_lds,
                        p.x, p.b, p.cs, A, act);
    if (n == 8)
        return launch_k(ctx, HIPIB_TIMER_SMALL_VCYCLE, bytes, k_small_vcycle<8, T>, grid, blk, ctx->small_lds,
                        p.x, p.b, p.cs, A, act);
    return fail(HIPIB_E_INVAL, "no coarse-level kernel for n = %d", n);
}

// levels run as one k_level_down / k_level_up pair per V-cycle: the levels
// below the finest and above the single-workgroup ones with n a multiple of
// 8, for V(2,2) (there the guess is always zero).  On the finest level the
// blocks' recomputed halos cost more than the launches they save.
bool level_fused(const hipib_ctx* ctx, int l) {
    return l >= 1 && l < ctx->small_start && ctx->lv[l].n % KB == 0 && ctx->lv[l].x2 != nullptr &&
           ctx->cfg.mg_pre == 2 && ctx->cfg.mg_post == 2;
}

template <typename T>
hipib_status gs_sweep(hipib_ctx* ctx, int l, LevelPtr<T> p, int ncomp, const OpCoef& oc, T c,
                      T inv_diag, int colour, int zg) {
    const int n = ctx->lv[l].n;
    const int32_t* act = ctx->st->active;
    const dim3 grid = gs_grid<T>(n, ncomp), blk(TX, TY);
    hipEvent_t t0, t1;
    if (l > 0) {
        k_gs<T, 0><<<grid, blk, 0, ctx->stream>>>(p.x, p.b, n, p.cs, c, inv_diag, colour, zg, act);
    } else if (!oc.poisson) {
        k_gs<T, 1><<<grid, blk, 0, ctx->stream>>>(p.x, p.b, n, p.cs, c, inv_diag, colour, zg, act);
    } else if (!zg && timer_events(ctx, HIPIB_TIMER_SMOOTH_FINE_POISSON,
                                   1.5 * sizeof(T) * (double)ctx->n3, &t0, &t1)) {
        // (only the 12 B/cell half-sweeps; a zero-guess first half-sweep moves 8)
        // the events take the dispatch's own start and end timestamps
        hipExtLaunchKernelGGL(k_gs<T, 2>, grid, blk, 0, ctx->stream, t0, t1, 0, p.x, p.b, n, p.cs, c,
                              inv_diag, colour, zg, act, T(1), 0);
    } else {
        k_gs<T, 2><<<grid, blk, 0, ctx->stream>>>(p.x, p.b, n, p.cs, c, inv_diag, colour, zg, act);
    }
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

// `sweeps` red+black sweeps, each red then black, over-relaxed by omega: the
// relaxation of the level a Helmholtz cycle stops at.  zero_guess: x is zero
// on entry (the first red half-sweep reads neither colour, the first black
// one not its own).
template <typename T>
hipib_status relax(hipib_ctx* ctx, int l, LevelPtr<T> p, int ncomp, const OpCoef& oc, int sweeps,
                   bool zero_guess, double omega) {
    const int n = ctx->lv[l].n;
    const T h = T(1) / T(n);
    const T c = (T)oc.nu / (h * h);
    const T inv_diag = T(1) / ((T)oc.sigma + T(6) * c);
    const int32_t* act = ctx->st->active;
    const dim3 grid = gs_grid<T>(n, ncomp), blk(TX, TY);
    for (int s = 0; s < 2 * sweeps; ++s) {
        const int zg = (s == 0 && zero_guess) ? 1 : 0;
        const int zo = (s < 2 && zero_guess) ? 1 : 0;
        // timed: the finest level's half-sweeps on the iterate (16 B per cell in FP64)
        const int kind = (l == 0 && !zo) ? HIPIB_TIMER_SMOOTH_FINE_HELMHOLTZ : 0;
        if (l == 0)
            HIPIB_TRY(launch_k(ctx, kind, 2.0 * sizeof(T) * (double)ctx->lv[l].n3 * ncomp, k_gs<T, 1, true>,
                               grid, blk, 0, p.x, p.b, n, p.cs, c, inv_diag, s & 1, zg, act, (T)omega, zo));
        else
            HIPIB_TRY(launch_k(ctx, 0, 0.0, k_gs<T, 0, true>, grid, blk, 0, p.x, p.b, n, p.cs, c, inv_diag,
                               s & 1, zg, act, (T)omega, zo));
    }
    return HIPIB_OK;
}

// `sweeps` red+black sweeps starting with colour `first`; zero_guess: x is
// zero on entry (its first half-sweep reads no neighbours).  Each finest-level
// Poisson half-sweep is timed on its own when the timer is on.
template <typename T>
hipib_status smooth(hipib_ctx* ctx, int l, LevelPtr<T> p, int ncomp, const OpCoef& oc, int sweeps,
                    int first, bool zero_guess, int start = 0) {
    if (sweeps <= 0) return HIPIB_OK;
    const int n = ctx->lv[l].n;
    const T h = T(1) / T(n);
    const T c = (T)oc.nu / (h * h);
    const T inv_diag = T(1) / ((T)oc.sigma + T(6) * c);
    // the preconditioner's finest-level post-smoothing of a conjugate-gradient
    // iteration: its last two half-sweeps also sum r.z and z.q
    const bool dots = l == 0 && ctx->cg_dots.q != nullptr && !zero_guess && ncomp == 1;
    const dim3 grid = gs_grid<T>(n, 1);
    const int64_t nb = (int64_t)grid.x * grid.y * grid.z;
    if (start == 0 && zero_guess && first == 0) {
        HIPIB_TRY(launch_k(ctx, 0, 0.0, k_gs_zero2<T>, gs_grid<T>(n, ncomp), dim3(TX, TY), 0, p.x, p.b, n, p.cs, c,
                           inv_diag, ctx->st->active));
        start = 2;
    }
    for (int s = start; s < 2 * sweeps; ++s) {
        const int zg = (s == 0 && zero_guess) ? 1 : 0;
        const int colour = (s & 1) ? 1 - first : first;
        if (dots && s >= 2 * sweeps - 2) {
            const int64_t poff = s == 2 * sweeps - 2 ? 0 : nb;
            HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_CG_DOTS, (sizeof(T) * 1.5 + (sizeof(T) == 4 ? 8.0 : 4.0)) * (double)ctx->n3,
                               k_gs_dot<T>, grid, dim3(TX, TY), 0, p.x, p.b, n, c, inv_diag, colour,
                               ctx->cg_dots.r, ctx->cg_dots.q, ctx->st, ctx->part, 2 * nb, poff));
            ctx->cg_dots.parts = 2 * nb;
        } else {
            HIPIB_TRY(gs_sweep<T>(ctx, l, p, ncomp, oc, c, inv_diag, colour, zg));
        }
    }
    return HIPIB_OK;
}

// One V-cycle from level l.  zero_guess: x is taken as zero on entry (its
// contents are never read).  With at least one pre-smoothing sweep (ending
// black) the residual is restricted from the red cells only, and with at
// least one post-smoothing sweep (starting black) the correction is
// prolongated to the red cells only.
template <typename T>
hipib_status vcycle(hipib_ctx* ctx, int l, LevelPtr<T> p, int ncomp, const OpCoef& oc,
                    bool zero_guess) {
    if (exact_coarse(ctx) && l == ctx->exact_level) return coarse_exact<T>(ctx, l, p, ncomp, oc);  // (x not read)
    if (l == ctx->small_start) return small_vcycle<T>(ctx, l, p, ncomp, oc, zero_guess);
    const int n = ctx->lv[l].n;
    const int32_t* act = ctx->st->active;
    const T h = T(1) / T(n);
    const T c = (T)oc.nu / (h * h);
    const int pre = ctx->cfg.mg_pre, post = ctx->cfg.mg_post;
    const int lc = stop_level(ctx, oc);
    if (l == lc) return relax<T>(ctx, l, p, ncomp, oc, stop_sweeps(ctx, lc), zero_guess,
                                 level_omega(n, oc));
    if (zero_guess && level_fused(ctx, l)) {
        const T inv_diag = T(1) / ((T)oc.sigma + T(6) * c);
        const Level& C = ctx->lv[l + 1];
        T* xc = level_x<T>(ctx, l + 1);
        T* bc = level_b<T>(ctx, l + 1);
        T* x2 = static_cast<T*>(ctx->lv[l].x2);
        const int nb = n / KB;
        const unsigned blocks = (unsigned)(nb * nb * nb * ncomp);
        HIPIB_TRY(launch_k(ctx, l == 1 ? HIPIB_TIMER_LEVEL_DOWN : 0, 17.0 / 8.0 * sizeof(T) * (double)ctx->lv[l].n3 * ncomp,
                           k_level_down<T>, dim3(blocks), dim3(KTHREADS), 0, p.b, x2, n, p.cs, bc, C.n3,
                           (T)oc.sigma, c, inv_diag, act));
        HIPIB_TRY(vcycle<T>(ctx, l + 1, LevelPtr<T>{xc, bc, C.n3}, ncomp, oc, true));
        HIPIB_TRY(launch_k(ctx, l == 1 ? HIPIB_TIMER_LEVEL_UP : 0, 21.0 / 8.0 * sizeof(T) * (double)ctx->lv[l].n3 * ncomp,
                           k_level_up<T>, dim3(blocks), dim3(KTHREADS), 0, p.b, x2, xc, p.x, n, p.cs, C.n3, c,
                           inv_diag, act));
        return HIPIB_OK;
    }
    if (zero_guess && pre == 0) HIPIB_TRY(zero_t<T>(ctx, p.x, ncomp * p.cs));
    HIPIB_TRY(smooth<T>(ctx, l, p, ncomp, oc, pre, 0, zero_guess));
    const Level& C = ctx->lv[l + 1];
    T* xc = level_x<T>(ctx, l + 1);
    T* bc = level_b<T>(ctx, l + 1);
    if (pre > 0) {
        HIPIB_TRY(launch_k(ctx, l == 0 ? HIPIB_TIMER_RESID_RESTRICT : 0,
                           13.0 / 8.0 * sizeof(T) * (double)ctx->lv[l].n3 * ncomp, k_resid_restrict<T>,
                           resid_restrict_grid(C.n, ncomp), dim3(RTHREADS), 0, p.x, p.b, n, p.cs, bc, C.n, C.n3,
                           (T)oc.sigma, c, act));
    } else {
        T* r = static_cast<T*>(ctx->r0);
        k_residual<T><<<packed_grid(n, ncomp), dim3(TX, TY), 0, ctx->stream>>>(
            p.x, p.b, r, n, p.cs, (T)oc.sigma, c, act);
        k_restrict<T><<<packed_grid(C.n, ncomp), dim3(TX, TY), 0, ctx->stream>>>(r, n, p.cs, bc, C.n,
                                                                                   C.n3, act);
    }
    HIPIB_HIP(hipGetLastError());
    HIPIB_TRY(vcycle<T>(ctx, l + 1, LevelPtr<T>{xc, bc, C.n3}, ncomp, oc, true));
    if (post >= 2) {
        // the correction enters through the first (black) post-smoothing half-sweep
        constexpr int KP = gs_kpt<T>();
        const dim3 pg((n / 2 + TX - 1) / TX, (n + kProlongRows - 1) / kProlongRows, ((n + KP - 1) / KP) * ncomp);
        HIPIB_TRY(launch_k(ctx, l == 0 ? HIPIB_TIMER_PROLONG : 0, 13.0 / 8.0 * sizeof(T) * (double)ctx->lv[l].n3 * ncomp,
                           k_gs_prolong<T, kProlongRows>, pg, dim3(TX, kProlongRows), 0, p.x, p.b, n, p.cs, xc, C.n,
                           C.n3, c, T(1) / ((T)oc.sigma + T(6) * c), 1, act));
        return smooth<T>(ctx, l, p, ncomp, oc, post, 1, false, 1);
    }
    const int nq = post > 0 ? 1 : 2;
    HIPIB_TRY(launch_k(ctx, (l == 0 && nq == 1) ? HIPIB_TIMER_PROLONG : 0,
                       9.0 / 8.0 * sizeof(T) * (double)ctx->lv[l].n3 * ncomp, k_prolong_add<T>,
                       dim3((n / 2 + TX - 1) / TX, (n + TY - 1) / TY, nq * n * ncomp), dim3(TX, TY), 0, p.x, n,
                       p.cs, xc, C.n, C.n3, nq, act));
    HIPIB_TRY(smooth<T>(ctx, l, p, ncomp, oc, post, 1, false));
    return HIPIB_OK;
}

// ||b - A x|| per component into the state (mode FIN_INIT_R / FIN_CYCLE_R);
// in mixed mode also writes the scaled FP32 residual of every active component
hipib_status resid_norm(hipib_ctx* ctx, int ncomp, const OpCoef& oc, int mode,
                        double* rstore = nullptr, int submean = 0) {
    // FIN_BNORM_INIT_R (FP64): ||b|| from the same pass
    const int bsq = mode == FIN_BNORM_INIT_R ? ncomp : 0;
    const int n = ctx->n;
    const double h = 1.0 / n, c = oc.nu / (h * h);
    const int64_t np = norm_parts(n);
    const double bytes = 16.0 * (double)ctx->n3 * ncomp;
    if (ctx->cfg.precision == HIPIB_MIXED)
        HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_RESID_NORM, bytes, k_resid_norm<true>, norm_grid(n, ncomp), dim3(TX, TY),
                           0, ctx->sx, ctx->bpk, n, ctx->n3, oc.sigma, c, ctx->st, ctx->r32, ctx->part, np, rstore,
                           submean, 0));
    else
        HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_RESID_NORM, bytes, k_resid_norm<false>, norm_grid(n, ncomp),
                           dim3(TX, TY), 0, ctx->sx, ctx->bpk, n, ctx->n3, oc.sigma, c, ctx->st, nullptr,
                           ctx->part, np, rstore, submean, bsq));
    return finalize(ctx, np, np, ncomp, mode, 0.0);
}

// one preconditioned conjugate-gradient iteration of the Poisson solve
hipib_status cg_iteration(hipib_ctx* ctx, const OpCoef& oc) {
    const int n = ctx->n;
    const int64_t n3 = ctx->n3;
    const double h = 1.0 / n, c = oc.nu / (h * h);
    const int nb = sum_blocks(n3);
    double *r = ctx->kv[0], *z = ctx->kv[1], *p = ctx->kv[2], *q = ctx->kv[3];
    const bool mixed = ctx->cfg.precision == HIPIB_MIXED;
    const int64_t np = norm_parts(n);
    const double zb = mixed ? 4.0 : 8.0;   // bytes of a z value
    // z = M r; the preconditioner's last two half-sweeps sum r.z and z.q when
    // it post-smooths the finest level, else k_cg_dots does
    ctx->cg_dots = hipib_ctx::CgDotsReq{r, q, 0};
    hipib_status vs;
    if (mixed) vs = vcycle<float>(ctx, 0, LevelPtr<float>{ctx->e32, ctx->r32, n3}, 1, oc, true);
    else vs = vcycle<double>(ctx, 0, LevelPtr<double>{z, r, n3}, 1, oc, true);
    const int64_t fused = ctx->cg_dots.parts;
    ctx->cg_dots = hipib_ctx::CgDotsReq{};
    HIPIB_TRY(vs);
    int64_t dparts = fused;
    if (fused == 0) {
        if (mixed)
            HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_CG_DOTS, (16.0 + zb) * n3, k_cg_dots<float>, dim3(nb), dim3(256), 0,
                               r, ctx->e32, q, n3, ctx->st, ctx->part, nb));
        else
            HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_CG_DOTS, (16.0 + zb) * n3, k_cg_dots<double>, dim3(nb), dim3(256), 0,
                               r, z, q, n3, ctx->st, ctx->part, nb));
        dparts = nb;
    }
    HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_REDUCE, 16.0 * dparts, k_cg_scalars, dim3(1), dim3(1024), 0, ctx->part,
                       dparts, dparts, ctx->st));
    if (mixed)
        HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_CG_DIR, (32.0 + zb) * n3, k_cg_dir<float>, norm_grid(n, 1), dim3(TX, TY),
                           0, ctx->e32, p, q, n, oc.sigma, c, ctx->st, ctx->part));
    else
        HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_CG_DIR, (32.0 + zb) * n3, k_cg_dir<double>, norm_grid(n, 1), dim3(TX, TY),
                           0, z, p, q, n, oc.sigma, c, ctx->st, ctx->part));
    // (alpha is reduced by k_cg_update itself: its ||r||^2 partials go after p.q's)
    const int nbu = update_blocks(n3);
    HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_CG_UPDATE, (mixed ? 52.0 : 48.0) * n3, k_cg_update, dim3(nbu), dim3(kUpdThreads), 0,
                       ctx->sx, r, p, q, n3, ctx->st, mixed ? ctx->r32 : nullptr, ctx->part, np, ctx->part + np));
    return finalize_at(ctx, np, nbu, nbu, 1, FIN_CYCLE_R, 0.0);
}

bool use_cg(const hipib_ctx* ctx, const OpCoef& oc, int ncomp) {
    return oc.poisson && ncomp == 1 && ctx->cfg.mg_krylov && ctx->kv[0] != nullptr;
}

// one top-level cycle on the packed FP64 solution
hipib_status cycle(hipib_ctx* ctx, int ncomp, const OpCoef& oc) {
    if (use_cg(ctx, oc, ncomp)) return cg_iteration(ctx, oc);
    const int nb = sum_blocks(ctx->n3);
    if (ctx->cfg.precision == HIPIB_MIXED) {
        HIPIB_TRY(vcycle<float>(ctx, 0, LevelPtr<float>{ctx->e32, ctx->r32, ctx->n3}, ncomp, oc, true));
        k_update<<<dim3(nb, ncomp), 256, 0, ctx->stream>>>(ctx->sx, ctx->e32, ctx->n3, ctx->st);
        HIPIB_HIP(hipGetLastError());
    } else {
        HIPIB_TRY(vcycle<double>(ctx, 0, LevelPtr<double>{ctx->sx, ctx->bpk, ctx->n3}, ncomp, oc, false));
    }
    return resid_norm(ctx, ncomp, oc, FIN_CYCLE_R);
}

}  // namespace

bool timer_events(hipib_ctx* ctx, int kind, double bytes, hipEvent_t* start, hipEvent_t* stop) {
    if (ctx->timer_which != kind) return false;
    const size_t pair = ctx->ev_used;
    while (ctx->ev_pool.size() < 2 * (pair + 1)) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return false;
        ctx->ev_pool.push_back(e);
    }
    *start = ctx->ev_pool[2 * pair];
    *stop = ctx->ev_pool[2 * pair + 1];
    ctx->ev_used = pair + 1;
    ctx->timer_bytes += bytes;
    ctx->timer_launches += 1;
    return true;
}

hipib_status mg_prepare(hipib_ctx* ctx) {
    const size_t tsz = mg_level_elem_size(ctx);
    size_t lds = 0;
    for (int l = ctx->small_start; l < ctx->L; ++l) lds += 3 * (size_t)ctx->lv[l].n3 * tsz;
    ctx->small_lds = lds;
    if (lds > 160 * 1024) return fail(HIPIB_E_INVAL, "coarse levels need %zu bytes of LDS", lds);
    // The attribute belongs to the kernel, not to a context: each instantiation
    // gets the LDS of its own level chain ([x, b, r] per level), so contexts
    // of other sizes or precisions never lower what another one launches with.
    struct SmallKernel {
        const void* fn;
        int bytes;
    };
    auto chain = [](int n0, int esz) {
        int cells = 0;
        for (int m = n0;; m /= 2) {
            cells += m * m * m;
            if (m < 8) break;
        }
        return 3 * cells * esz;
    };
    const SmallKernel ks[] = {
        {reinterpret_cast<const void*>(&k_small_vcycle<16, double>), chain(16, 8)},
        {reinterpret_cast<const void*>(&k_small_vcycle<12, double>), chain(12, 8)},
        {reinterpret_cast<const void*>(&k_small_vcycle<8, double>), chain(8, 8)},
        {reinterpret_cast<const void*>(&k_small_vcycle<16, float>), chain(16, 4)},
        {reinterpret_cast<const void*>(&k_small_vcycle<12, float>), chain(12, 4)},
        {reinterpret_cast<const void*>(&k_small_vcycle<8, float>), chain(8, 4)}};
    for (const SmallKernel& k : ks)
        HIPIB_HIP(hipFuncSetAttribute(k.fn, hipFuncAttributeMaxDynamicSharedMemorySize, k.bytes));
    const SmallKernel ke[] = {
        {reinterpret_cast<const void*>(&k_coarse_exact<16, double>), exact_lds_words<16>() * 8},
        {reinterpret_cast<const void*>(&k_coarse_exact<12, double>), exact_lds_words<12>() * 8},
        {reinterpret_cast<const void*>(&k_coarse_exact<8, double>), exact_lds_words<8>() * 8},
        {reinterpret_cast<const void*>(&k_coarse_exact<16, float>), exact_lds_words<16>() * 4},
        {reinterpret_cast<const void*>(&k_coarse_exact<12, float>), exact_lds_words<12>() * 4},
        {reinterpret_cast<const void*>(&k_coarse_exact<8, float>), exact_lds_words<8>() * 4}};
    for (const SmallKernel& k : ke)
        HIPIB_HIP(hipFuncSetAttribute(k.fn, hipFuncAttributeMaxDynamicSharedMemorySize, k.bytes));
    if (ctx->cfg.mg_coarse_sweeps == 0) {
        // the coarsest level's real Fourier basis and eigenvalue factors
        const int N = ctx->lv[ctx->exact_level].n;
        if (N != 32 && N != 24 && N != 16 && N != 12 && N != 8)
            return fail(HIPIB_E_INVAL, "no exact coarse solve for n = %d", N);
        const double pi = 3.14159265358979323846;
        std::vector<double> tab((size_t)N * N + N);
        for (int j = 0; j < N; ++j)
            for (int m = 0; m < N; ++m) {
                double q;
                if (m == 0) q = 1.0 / std::sqrt((double)N);
                else if (m < N / 2) q = std::sqrt(2.0 / N) * std::cos(2.0 * pi * m * j / N);
                else if (m == N / 2) q = ((j & 1) ? -1.0 : 1.0) / std::sqrt((double)N);
                else q = std::sqrt(2.0 / N) * std::sin(2.0 * pi * (m - N / 2) * j / N);
                tab[(size_t)j * N + m] = q;
            }
        for (int m = 0; m < N; ++m) {
            const int f = m <= N / 2 ? m : m - N / 2;
            const double sn = std::sin(pi * f / N);
            tab[(size_t)N * N + m] = 4.0 * N * N * sn * sn;     // (4 / h^2) sin^2, h = 1 / N
        }
        std::vector<float> tab32(tab.begin(), tab.end());
        if (hipMalloc(reinterpret_cast<void**>(&ctx->coarse_tab), tab.size() * sizeof(double)) != hipSuccess ||
            hipMalloc(reinterpret_cast<void**>(&ctx->coarse_tab32), tab.size() * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(HIPIB_E_NOMEM, "coarse-level table allocation failed");
        }
        HIPIB_HIP(hipMemcpy(ctx->coarse_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
        HIPIB_HIP(hipMemcpy(ctx->coarse_tab32, tab32.data(), tab32.size() * sizeof(float), hipMemcpyHostToDevice));
        if (N > 16 && hipMalloc(&ctx->coarse_work, 3 * (size_t)N * N * N * tsz) != hipSuccess) {
            (void)hipGetLastError();
            return fail(HIPIB_E_NOMEM, "coarse-level work array allocation failed");
        }
    }
    return HIPIB_OK;
}

int64_t mg_partials_needed(int n) { return 6 * (norm_parts(n) + 1024); }

size_t mg_level_elem_size(const hipib_ctx* ctx) {
    return ctx->cfg.precision == HIPIB_MIXED ? sizeof(float) : sizeof(double);
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
    k_sub_mean<<<dim3(sum_blocks(ctx->n3), 1), 256, 0, ctx->stream>>>(v, ctx->n3, ctx->n3, ctx->st, 0);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

// The solve on packed arrays: xpk holds the initial guess, ctx->bpk the
// right-hand side.  b_ready: the state was reset and holds ||b - mean(b)|| and
// the mean of b (Poisson, component 0), which the initial residual pass then
// subtracts from b.  A converged Poisson solve leaves the solution's mean in
// the state for the caller to subtract (the null space of the periodic
// Laplacian); *mean_ok says whether it is there.
// device address of the state's mean[] (no host access to the state)
const double* state_mean(const hipib_ctx* ctx) {
    return reinterpret_cast<const double*>(reinterpret_cast<const char*>(ctx->st) + offsetof(MGState, mean));
}

hipib_status solve_packed(hipib_ctx* ctx, int op, int ncomp, double* xpk, bool b_ready, int32_t* cycles,
                          double* relres, bool* mean_ok) {
    const OpCoef oc = op_coef(ctx, op);
    const int nb = sum_blocks(ctx->n3);
    ctx->sx = xpk;
    // in FP64 ||b|| comes from the initial residual pass (mixed mode scales its
    // FP32 residual by ||b||, so it needs ||b|| first)
    const bool fused_bnorm = !b_ready && ctx->cfg.precision == HIPIB_FP64;
    if (fused_bnorm) {
        k_state_reset<<<1, 64, 0, ctx->stream>>>(ctx->st, ncomp);
        HIPIB_HIP(hipGetLastError());
    } else if (!b_ready) {
        k_state_reset<<<1, 64, 0, ctx->stream>>>(ctx->st, ncomp);
        k_sum_partials<<<dim3(nb, ncomp), 256, 0, ctx->stream>>>(ctx->bpk, ctx->n3, ctx->n3, 1, nullptr,
                                                                 ctx->part, nb);
        HIPIB_HIP(hipGetLastError());
        HIPIB_TRY(finalize(ctx, nb, nb, ncomp, FIN_BNORM, 0.0));
    }
    // (conjugate gradients keep the initial residual as their r)
    HIPIB_TRY(resid_norm(ctx, ncomp, oc, fused_bnorm ? FIN_BNORM_INIT_R : FIN_INIT_R,
                         use_cg(ctx, oc, ncomp) ? ctx->kv[0] : nullptr, b_ready && oc.poisson ? 1 : 0));
    k_zero_requested<<<dim3(nb, ncomp), 256, 0, ctx->stream>>>(xpk, ctx->n3, ctx->n3, ctx->st);
    HIPIB_HIP(hipGetLastError());

    int enqueue = ctx->predicted[op] > 0 ? ctx->predicted[op] : 1;
    int total = 0;
    const int limit =
        (ctx->cfg.mg_fixed_cycles > 0 ? ctx->cfg.mg_fixed_cycles : ctx->cfg.mg_max_cycles) + 1;
    while (true) {
        for (int e = 0; e < enqueue; ++e) HIPIB_TRY(cycle(ctx, ncomp, oc));
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
    *mean_ok = oc.poisson && ctx->st_host->status == HIPIB_OK;
    if (*mean_ok && use_cg(ctx, oc, ncomp) && ctx->st_host->cycles[0] > 0) {
        // the last conjugate-gradient update left the partial sums of x after
        // its ||r||^2 partials (later enqueued cycles were no-ops)
        const int nbu = update_blocks(ctx->n3);
        HIPIB_TRY(finalize_at(ctx, norm_parts(ctx->n) + nbu, nbu, nbu, 1, FIN_MEAN_ALL, 1.0 / (double)ctx->n3));
    } else if (*mean_ok) {
        k_sum_partials<<<dim3(nb, ncomp), 256, 0, ctx->stream>>>(xpk, ctx->n3, ctx->n3, 0, nullptr, ctx->part,
                                                                 nb);
        HIPIB_HIP(hipGetLastError());
        HIPIB_TRY(finalize(ctx, nb, nb, ncomp, FIN_MEAN_ALL, 1.0 / (double)ctx->n3));
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

hipib_status mg_solve(hipib_ctx* ctx, int op, int ncomp, const double* b, double* x,
                      int32_t* cycles, double* relres) {
    const int n = ctx->n;
    // pack the caller's b and initial guess
    HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_PACK, 16.0 * (double)ctx->n3 * ncomp, k_pack, natural_grid(n, ncomp),
                       dim3(TX, TY), 0, b, ctx->bpk, n, ctx->n3));
    HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_PACK, 16.0 * (double)ctx->n3 * ncomp, k_pack, natural_grid(n, ncomp),
                       dim3(TX, TY), 0, x, ctx->xp, n, ctx->n3));
    bool mean_ok = false;
    const hipib_status s = solve_packed(ctx, op, ncomp, ctx->xp, false, cycles, relres, &mean_ok);
    // unpack (a Poisson solution without its mean), also after a failed solve
    HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_PACK, 16.0 * (double)ctx->n3 * ncomp, k_unpack, natural_grid(n, ncomp),
                       dim3(TX, TY), 0, ctx->xp, x, n, ctx->n3,
                       mean_ok ? state_mean(ctx) : nullptr));
    return s;
}

// ---------------------------------------------------------------------------
// The fluid part of a step on the packed layout: the right-hand side builder
// packs u^n as the Helmholtz guess, u* stays packed from the Helmholtz solve
// to the projection, the divergence writes the Poisson right-hand side packed
// (with the partial sums of its mean and norm), and p is solved in place in
// its own packed array (ctx->bp).
// ---------------------------------------------------------------------------

// b = -(rho/dt) D u* on the colour-q cells of a column, from the packed u*;
// block partials of sum b (slot 0) and sum b^2 (slot 1).  Grid and columns as
// k_resid_norm (one component, both colours).
__global__ void __launch_bounds__(TX * TY)
k_divergence_packed(const double* __restrict__ u, double* __restrict__ b, int n, int64_t n3, double rho_dt,
                    double inv_h, double* __restrict__ part, int64_t pstride) {
    __shared__ double red[2][(TX * TY) / 64];
    const int nkb = (n + KPT - 1) / KPT;
    const uint3 bid = xcd_block();
    const int rem = bid.z, q = rem / nkb, k0 = (rem - q * nkb) * KPT;
    const int H = n >> 1;
    const int ih = bid.x * TX + threadIdx.x, j = bid.y * TY + threadIdx.y;
    double s1 = 0.0, s2 = 0.0;
    if (ih < H && j < n) {
        const int64_t half3 = (int64_t)H * n * n;
        const int64_t oo = (1 - q) * half3;   // the other colour: the + neighbours
        const int jp = wrapi(j + 1, n);
        const int ihp = ih + 1 < H ? ih + 1 : 0;
        double ux[KPT], uxp[KPT], uy[KPT], uyp[KPT], uz[KPT], uzp[KPT];
#pragma unroll
        for (int r = 0; r < KPT; ++r) {
            const int k = k0 + r;
            if (k < n) {
                const int64_t row = (int64_t)H * ((int64_t)j + (int64_t)n * k);
                const int64_t oq = q * half3 + row + ih;
                const int p = (j + k + q) & 1;        // i = 2 ih + p; i + 1 sits at ih + p
                ux[r] = u[oq];
                uxp[r] = u[oo + row + (p ? ihp : ih)];
                uy[r] = u[n3 + oq];
                uyp[r] = u[n3 + oo + (int64_t)H * ((int64_t)jp + (int64_t)n * k) + ih];
                uz[r] = u[2 * n3 + oq];
                uzp[r] = u[2 * n3 + oo + (int64_t)H * ((int64_t)j + (int64_t)n * wrapi(k + 1, n)) + ih];
            }
        }
#pragma unroll
        for (int r = 0; r < KPT; ++r) {
            const int k = k0 + r;
            if (k < n) {
                double sd = (uxp[r] - ux[r]) * inv_h;
                sd += (uyp[r] - uy[r]) * inv_h;
                sd += (uzp[r] - uz[r]) * inv_h;
                const double bv = -rho_dt * sd;
                b[q * half3 + (int64_t)H * ((int64_t)j + (int64_t)n * k) + ih] = bv;
                s1 += bv;
                s2 += bv * bv;
            }
        }
    }
    const int tid = threadIdx.x + TX * threadIdx.y;
    for (int o = 32; o > 0; o >>= 1) {
        s1 += __shfl_down(s1, o, 64);
        s2 += __shfl_down(s2, o, 64);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = s1;
        red[1][tid >> 6] = s2;
    }
    __syncthreads();
    if (tid == 0) {
        double a = 0.0, c = 0.0;
        for (int w = 0; w < (TX * TY) / 64; ++w) {
            a += red[0][w];
            c += red[1][w];
        }
        const int64_t blk = bid.x + (int64_t)gridDim.x * (bid.y + (int64_t)gridDim.y * rem);
        part[blk] = a;
        part[pstride + blk] = c;
    }
}

// u^{n+1}[c] = u*[c] - (dt/rho) G p and p[c] (natural) from the packed u* and
// p, with p's mean subtracted first (mean may be null)
__global__ void __launch_bounds__(TX * TY)
k_project_packed(const double* __restrict__ us, const double* __restrict__ pp, const double* __restrict__ mean,
                 double* __restrict__ u, double* __restrict__ p, int n, int64_t n3, double dt_rho, double inv_h) {
    const int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y, k = blockIdx.z;
    if (i >= n || j >= n) return;
    const double m = mean ? mean[0] : 0.0;
    const int64_t o = pk(i, j, k, n);
    const double pc = pp[o] - m;
    const double px = pp[pk(wrapi(i - 1, n), j, k, n)] - m;
    const double py = pp[pk(i, wrapi(j - 1, n), k, n)] - m;
    const double pz = pp[pk(i, j, wrapi(k - 1, n), n)] - m;
    const int64_t c = i + (int64_t)n * (j + (int64_t)n * k);
    u[c] = us[o] - dt_rho * ((pc - px) * inv_h);
    u[n3 + c] = us[n3 + o] - dt_rho * ((pc - py) * inv_h);
    u[2 * n3 + c] = us[2 * n3 + o] - dt_rho * ((pc - pz) * inv_h);
    p[c] = pc;
}

hipib_status fluid_step_packed(hipib_ctx* ctx, double* u, double* p, int32_t* cyc, double* rr,
                               hipib_status (*mark)(hipib_ctx*, int)) {
    const int n = ctx->n;
    const int64_t n3 = ctx->n3;
    // Helmholtz: its right-hand side g was built and spread packed in bpk by the
    // caller, the guess u^n packed into xp by the right-hand side builder
    bool mean_ok = false;
    HIPIB_TRY(solve_packed(ctx, HIPIB_OP_HELMHOLTZ, 3, ctx->xp, false, cyc, rr, &mean_ok));
    if (mark) HIPIB_TRY(mark(ctx, 3));
    // Poisson: guess p^{n-1} packed into bp; b = -(rho/dt) D u* packed, its mean
    // and norm reduced from the divergence pass's partials
    HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_PACK, 16.0 * (double)n3, k_pack, natural_grid(n, 1), dim3(TX, TY), 0, p,
                       ctx->bp, n, n3));
    k_state_reset<<<1, 64, 0, ctx->stream>>>(ctx->st, 1);
    HIPIB_HIP(hipGetLastError());
    const int64_t np = norm_parts(n);
    HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_DIVERGENCE, 32.0 * (double)n3, k_divergence_packed, norm_grid(n, 1),
                       dim3(TX, TY), 0, ctx->xp, ctx->bpk, n, n3, ctx->cfg.rho / ctx->cfg.dt, 1.0 / ctx->h,
                       ctx->part, np));
    HIPIB_TRY(finalize(ctx, np, np, 1, FIN_MEAN_BNORM, 1.0 / (double)n3));
    HIPIB_TRY(solve_packed(ctx, HIPIB_OP_POISSON, 1, ctx->bp, true, cyc + 3, rr + 3, &mean_ok));
    if (mark) HIPIB_TRY(mark(ctx, 4));
    HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_PROJECT, 64.0 * (double)n3, k_project_packed, natural_grid(n, 1),
                       dim3(TX, TY), 0, ctx->xp, ctx->bp,
                       mean_ok ? state_mean(ctx) : nullptr, u, p, n, n3,
                       ctx->cfg.dt / ctx->cfg.rho, 1.0 / ctx->h));
    if (mark) HIPIB_TRY(mark(ctx, 5));
    return HIPIB_OK;
}

}  // namespace hipib
