// Eulerian-Lagrangian coupling ("Eulerian-Lagrangian coupling operators"):
//   spreading      f^d[idx] += sum_q F^d_q delta_h(x^d_idx - X_q)
//   interpolation  U^d_q = sum_idx u^d[idx] delta_h(x^d_idx - X_q) h^3
// with Peskin's four-point kernel delta_h(x) = prod_e phi(x_e / h) / h^3.
// For a lattice coordinate r = X_e / h - offset (offset 0 along the face
// direction d, 1/2 along the others), the support is b-1 .. b+2 with
// b = floor(r), f = r - b, s = sqrt(1 + 4 f (1 - f)) and weights
//   ((3 - 2f - s), (3 - 2f + s), (1 + 2f + s), (1 + 2f - s)) / 8,
// which is phi evaluated at f+1, f, 1-f, 2-f.
//
// Spreading is binned: nodes are counting-sorted by the Eulerian tile (T^3
// cells) holding floor(X/h); every stencil point of a node in tile t lies in
// the (T+4)^3 box starting two cells below the tile, on all three lattices.
// One workgroup per work item (at most kSpreadChunk nodes of one tile) and
// lattice accumulates its box in LDS with FP64 LDS atomics, then adds the box
// to the grid with one coalesced pass of global atomics (boxes of
// neighbouring tiles overlap by four cells).  Interpolation
// walks the nodes in the same tile order so a wavefront gathers from a small
// neighbourhood.  Summation order is not fixed, so results agree with a serial
// sum to rounding.
#include <mutex>

#include "delta.h"

namespace hipib {
namespace {

// ---------------------------------------------------------------------------
// Workspace of hipib_spread_noalloc: the node bins live in one static device
// array instead of memory the library allocates.  Limits: grids of at most
// kNaMaxN cells per side (8^3-cell tiles: at most (kNaMaxN/8)^3 tiles; the
// one smaller valid size that is not a multiple of 8, n = 12, has 27 tiles of
// 4^3) and at most kNaMaxNodes nodes.  Layout in int32 words: tile counts
// [ntiles], offsets [ntiles + 1], work list [2 * cap], list length [1], node
// tiles [nn], node ranks [nn], node order [nn].
// ---------------------------------------------------------------------------
constexpr int kNaMaxN = 256;
constexpr int kNaMaxNodes = 1 << 20;
constexpr int64_t kNaMaxTiles = (int64_t)(kNaMaxN / 8) * (kNaMaxN / 8) * (kNaMaxN / 8);
constexpr int64_t kNaMaxList = kNaMaxTiles + (kNaMaxNodes + kSpreadChunk - 1) / kSpreadChunk + 1;
constexpr int64_t kNaWords = kNaMaxTiles + (kNaMaxTiles + 1) + 2 * kNaMaxList + 1 + 3 * (int64_t)kNaMaxNodes;

static __device__ __align__(256) int32_t scratch[kNaWords];

__global__ void __launch_bounds__(256) k_zero_i32(int32_t* __restrict__ p, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}


// tile of each node and its rank inside the tile.  Consecutive nodes of a
// mesh mostly share a tile, so the lanes of a wavefront with equal tiles are
// grouped and one lane adds the group's size to the count (one atomic per
// distinct tile per wavefront instead of one per node).
__global__ void k_clear_flag(int32_t* flag) {
    if (threadIdx.x == 0) *flag = 0;
}

// A non-finite position, or one 1e9 cells or more from the origin, sets
// `bad` (when given) and is binned (and later spread and interpolated) at the
// origin, so every index stays in range; the entry points then fail with
// HIPIB_E_NUMERIC.
__global__ void __launch_bounds__(256)
k_bin_count(const double* __restrict__ X, int nn, int n, int T, int ta, double inv_h,
            int32_t* __restrict__ node_tile, int32_t* __restrict__ node_rank,
            int32_t* __restrict__ count, int32_t* __restrict__ bad) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = q < nn;
    int tile = -1;
    if (valid) {
        int t[3];
        for (int e = 0; e < 3; ++e) {
            const double r = X[3 * q + e] * inv_h;
            if (bad && !(fabs(r) < 1.0e9)) *bad = 1;
            const int c = (int)floor(safe_coord(r));
            t[e] = wrap_mod(c, n) / T;
        }
        tile = t[0] + ta * (t[1] + ta * t[2]);
        node_tile[q] = tile;
    }
    const int lane = (int)__lane_id();
    unsigned long long pending = __ballot(valid);
    int rank = 0;
    while (pending) {  // uniform over the wavefront
        const int leader = __ffsll((long long)pending) - 1;
        const int key = __shfl(tile, leader, 64);
        const bool mine = valid && tile == key;
        const unsigned long long m = __ballot(mine);
        int base = 0;
        if (lane == leader) base = atomicAdd(count + key, __popcll(m));
        base = __shfl(base, leader, 64);
        if (mine) rank = base + __popcll(m & ((1ull << lane) - 1ull));
        pending &= ~m;
    }
    if (valid) node_rank[q] = rank;
}

// Exclusive scan of the tile counts and the list of work items: each
// occupied tile is cut into chunks of at most kSpreadChunk nodes, listed as
// (tile, first rank) pairs, so a tile crowded with nodes is spread by several
// workgroups.  Counts are reset to 0 for the next binning.  When given,
// lfirst[t] receives the list index of tile t's first work item.
__global__ void __launch_bounds__(1024)
k_bin_scan(int32_t* __restrict__ count, int64_t ntiles, int32_t* __restrict__ off,
           int32_t* __restrict__ list, int32_t* __restrict__ nlist, int32_t* __restrict__ lfirst) {
    __shared__ int32_t s_sum[1024], s_nz[1024];
    const int tid = threadIdx.x;
    const int64_t per = (ntiles + 1023) / 1024;
    const int64_t beg = tid * per < ntiles ? tid * per : ntiles;
    const int64_t end = beg + per < ntiles ? beg + per : ntiles;
    int32_t sum = 0, nz = 0;
    for (int64_t i = beg; i < end; ++i) {
        sum += count[i];
        nz += (count[i] + kSpreadChunk - 1) / kSpreadChunk;
    }
    s_sum[tid] = sum;
    s_nz[tid] = nz;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int32_t a = tid >= o ? s_sum[tid - o] : 0;
        const int32_t b = tid >= o ? s_nz[tid - o] : 0;
        __syncthreads();
        s_sum[tid] += a;
        s_nz[tid] += b;
        __syncthreads();
    }
    int32_t run = s_sum[tid] - sum, lrun = s_nz[tid] - nz;
    for (int64_t i = beg; i < end; ++i) {
        off[i] = run;
        if (lfirst) lfirst[i] = lrun;
        const int32_t c = count[i];
        run += c;
        for (int32_t r = 0; r < c; r += kSpreadChunk) {
            list[2 * lrun] = (int32_t)i;
            list[2 * lrun + 1] = r;
            ++lrun;
        }
        count[i] = 0;
    }
    if (tid == 1023) {
        off[ntiles] = s_sum[1023];
        *nlist = s_nz[1023];
    }
}

__global__ void __launch_bounds__(256)
k_bin_scatter(const int32_t* __restrict__ node_tile, const int32_t* __restrict__ node_rank,
              const int32_t* __restrict__ off, int32_t* __restrict__ perm, int nn) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nn) return;
    perm[off[node_tile[q]] + node_rank[q]] = q;
}

// one workgroup per (work item, lattice d = blockIdx.y) (grid-stride over the
// list): up to kSpreadChunk nodes of one tile, one node per thread; LDS box of
// E^3 cells of lattice d, E = T + 4, starting at T * tile - 2 (a workgroup per
// lattice: a third of the LDS atomics per thread and three times the
// workgroups of a single box of all three lattices).  Ranks inside the chunk
// are dealt to threads with an odd stride, so the lanes of a wavefront take
// nodes that are far apart in mesh order, which keeps apart the LDS addresses
// they add to in the same instruction.  TW: type of the
// weights and their products (the lattice coordinate, its floor and the
// fractional offset are always FP64); the LDS box and the grid accumulate in
// FP64, since neighbouring nodes' forces partly cancel there.
template <int T, typename TW>
__global__ void __launch_bounds__(kSpreadChunk)
k_spread_tiles(const double* __restrict__ X, const double* __restrict__ F, double* __restrict__ f,
               const int32_t* __restrict__ perm, const int32_t* __restrict__ off,
               const int32_t* __restrict__ list, const int32_t* __restrict__ nlist, int n, int ta,
               int64_t n3, double inv_h, double ih3, int f_packed) {
    constexpr int E = T + 4, E3 = E * E * E;
    __shared__ double box[E3];
    const int d = blockIdx.y;
    const int ntl = *nlist;
    for (int li = blockIdx.x; li < ntl; li += gridDim.x) {
        const int tile = list[2 * li];
        const int tb[3] = {T * (tile % ta), T * ((tile / ta) % ta), T * (tile / (ta * ta))};
        for (int e = threadIdx.x; e < E3; e += blockDim.x) box[e] = 0.0;
        __syncthreads();
        const int idx = off[tile] + list[2 * li + 1] + ((threadIdx.x * 109) & (kSpreadChunk - 1));
        if (idx < off[tile + 1]) {
            const int q = perm[idx];
            double xs[3];
            int cw[3];
            for (int e = 0; e < 3; ++e) {
                xs[e] = safe_coord(X[3 * q + e] * inv_h);
                cw[e] = wrap_mod((int)floor(xs[e]), n);
            }
            {
                const TW val = (TW)(F[3 * q + d] * ih3);
                int ls[3];
                TW w[3][4];
                for (int e = 0; e < 3; ++e) {
                    const double r = xs[e] - (e == d ? 0.0 : 0.5);
                    const double bf = floor(r);
                    const TW fr = (TW)(r - bf);
                    const TW sq = sqrt(TW(1) + TW(4) * fr * (TW(1) - fr));
                    w[e][0] = (TW(3) - TW(2) * fr - sq) * TW(0.125);
                    w[e][1] = (TW(3) - TW(2) * fr + sq) * TW(0.125);
                    w[e][2] = (TW(1) + TW(2) * fr + sq) * TW(0.125);
                    w[e][3] = (TW(1) + TW(2) * fr - sq) * TW(0.125);
                    // stencil start relative to the node's cell is -1 or -2
                    const int ds = (int)bf - 1 - (int)floor(xs[e]);
                    ls[e] = cw[e] - tb[e] + 2 + ds;
                }
                double* bd = box;
                for (int c = 0; c < 4; ++c)
                    for (int b = 0; b < 4; ++b) {
                        const TW wyz = w[1][b] * w[2][c];
                        const int row = (ls[0]) + E * ((ls[1] + b) + E * (ls[2] + c));
                        for (int a = 0; a < 4; ++a) atomicAdd(bd + row + a, (double)(val * (w[0][a] * wyz)));
                    }
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < E3; e += blockDim.x) {
            const double v = box[e];
            if (v != 0.0) {
                const int r = e;
                const int lx = r % E, ly = (r / E) % E, lz = r / (E * E);
                const int gx = wrap_mod(tb[0] - 2 + lx, n), gy = wrap_mod(tb[1] - 2 + ly, n),
                          gz = wrap_mod(tb[2] - 2 + lz, n);
                const int64_t g = f_packed ? pk(gx, gy, gz, n) : gx + (int64_t)n * (gy + (int64_t)n * gz);
                atomicAdd(f + d * n3 + g, v);
            }
        }
        __syncthreads();
    }
}

// Interpolation U = J(X) u, optionally X += dt U (in place, FP64), by the
// binning's work items: one workgroup per item (grid-stride over the list),
// up to kSpreadChunk nodes of one tile, one node per thread.  The E^3 box of
// each velocity component around the tile (E = T + 4, from T * tile - 2, the
// reach of every node's 4x4x4 stencils on all three staggered lattices) is
// staged in LDS with coalesced row loads, so the stencil values a tile's nodes
// share are fetched from L2 once; each node's 3 x 64-term sums then read LDS,
// in the same weights and order as a direct gather.  TW: type of the box, the
// weights and the accumulation.
template <int T, typename TW>
__global__ void __launch_bounds__(kSpreadChunk)
k_interp_tiles(const double* X, const double* __restrict__ u, double* __restrict__ U, double* Xupd, double dt,
               const int32_t* __restrict__ perm, const int32_t* __restrict__ off,
               const int32_t* __restrict__ list, const int32_t* __restrict__ nlist, int n, int ta,
               int64_t n3, double inv_h) {
    constexpr int E = T + 4, E3 = E * E * E;
    __shared__ TW box[3 * E3];
    const int ntl = *nlist;
    for (int li = blockIdx.x; li < ntl; li += gridDim.x) {
        const int tile = list[2 * li];
        const int tb[3] = {T * (tile % ta), T * ((tile / ta) % ta), T * (tile / (ta * ta))};
        __syncthreads();   // the previous item's reads of the box are done
        for (int e = threadIdx.x; e < 3 * E3; e += blockDim.x) {
            const int d = e / E3, r = e - d * E3;
            const int lx = r % E, ly = (r / E) % E, lz = r / (E * E);
            const int gx = wrap_mod(tb[0] - 2 + lx, n), gy = wrap_mod(tb[1] - 2 + ly, n),
                      gz = wrap_mod(tb[2] - 2 + lz, n);
            box[e] = (TW)u[d * n3 + gx + (int64_t)n * (gy + (int64_t)n * gz)];
        }
        __syncthreads();
        const int idx = off[tile] + list[2 * li + 1] + threadIdx.x;
        if (idx < off[tile + 1]) {
            const int q = perm[idx];
            const double X0 = X[3 * q], X1 = X[3 * q + 1], X2 = X[3 * q + 2];
            const double xs[3] = {safe_coord(X0 * inv_h), safe_coord(X1 * inv_h), safe_coord(X2 * inv_h)};
            int cw[3];
            for (int e = 0; e < 3; ++e) cw[e] = wrap_mod((int)floor(xs[e]), n);
            TW Uq[3];
            for (int d = 0; d < 3; ++d) {
                int ls[3];
                TW w[3][4];
                for (int e = 0; e < 3; ++e) {
                    const double r = xs[e] - (e == d ? 0.0 : 0.5);
                    const double bf = floor(r);
                    const TW fr = (TW)(r - bf);
                    const TW sq = sqrt(TW(1) + TW(4) * fr * (TW(1) - fr));
                    w[e][0] = (TW(3) - TW(2) * fr - sq) * TW(0.125);
                    w[e][1] = (TW(3) - TW(2) * fr + sq) * TW(0.125);
                    w[e][2] = (TW(1) + TW(2) * fr + sq) * TW(0.125);
                    w[e][3] = (TW(1) + TW(2) * fr - sq) * TW(0.125);
                    // stencil start relative to the node's cell is -1 or -2
                    const int ds = (int)bf - 1 - (int)floor(xs[e]);
                    ls[e] = cw[e] - tb[e] + 2 + ds;
                }
                const TW* bd = box + d * E3;
                TW acc = TW(0);
                for (int c = 0; c < 4; ++c)
                    for (int b = 0; b < 4; ++b) {
                        const TW wyz = w[1][b] * w[2][c];
                        const int row = ls[0] + E * ((ls[1] + b) + E * (ls[2] + c));
                        for (int a = 0; a < 4; ++a) acc += bd[row + a] * (w[0][a] * wyz);
                    }
                Uq[d] = acc;
            }
            if (U) {
                U[3 * q] = (double)Uq[0];
                U[3 * q + 1] = (double)Uq[1];
                U[3 * q + 2] = (double)Uq[2];
            }
            if (Xupd) {
                Xupd[3 * q] = X0 + dt * (double)Uq[0];
                Xupd[3 * q + 1] = X1 + dt * (double)Uq[1];
                Xupd[3 * q + 2] = X2 + dt * (double)Uq[2];
            }
        }
    }
}

}  // namespace

hipib_status launch_bin(hipib_ctx* ctx, const double* X) {
    if (ctx->nn == 0) return HIPIB_OK;
    const int nb = (ctx->nn + 255) / 256;
    k_clear_flag<<<1, 64, 0, ctx->stream>>>(&ctx->st->bad_position);
    k_bin_count<<<nb, 256, 0, ctx->stream>>>(X, ctx->nn, ctx->n, ctx->tile, ctx->tiles_axis,
                                             1.0 / ctx->h, ctx->node_tile, ctx->node_rank,
                                             ctx->bin_count, &ctx->st->bad_position);
    k_bin_scan<<<1, 1024, 0, ctx->stream>>>(ctx->bin_count, ctx->ntiles, ctx->bin_off,
                                            ctx->tile_list, ctx->n_list, ctx->det_lfirst);
    k_bin_scatter<<<nb, 256, 0, ctx->stream>>>(ctx->node_tile, ctx->node_rank, ctx->bin_off,
                                               ctx->perm, ctx->nn);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

// expects launch_bin(ctx, X) to have been enqueued for the same X
hipib_status launch_spread(hipib_ctx* ctx, const double* X, const double* F, double* f, bool f_packed) {
    if (ctx->nn == 0) return HIPIB_OK;
    if (ctx->cfg.deterministic) return det_spread(ctx, X, F, f, f_packed);
    const double h = ctx->h;
    const int64_t cap = spread_list_cap(ctx->ntiles, ctx->nn);
    const int blocks = (int)(cap < 8192 ? cap : 8192);
    const bool mixed = ctx->cfg.precision == HIPIB_MIXED;
#define HIPIB_SPREAD(TT, TW)                                                                       \
    HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_SPREAD, 0.0, k_spread_tiles<TT, TW>, dim3(blocks, 3), dim3(kSpreadChunk), 0,  \
                       X, F, f, ctx->perm, ctx->bin_off, ctx->tile_list, ctx->n_list, ctx->n,                 \
                       ctx->tiles_axis, ctx->n3, 1.0 / h, 1.0 / (h * h * h), f_packed ? 1 : 0))
    if (ctx->tile == 8) {
        if (mixed) HIPIB_SPREAD(8, float); else HIPIB_SPREAD(8, double);
    } else {
        if (mixed) HIPIB_SPREAD(4, float); else HIPIB_SPREAD(4, double);
    }
#undef HIPIB_SPREAD
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

// expects launch_bin(ctx, X) to have been enqueued for the same X
hipib_status launch_interpolate(hipib_ctx* ctx, const double* X, const double* u, double* U,
                                double* Xupd, double dt) {
    if (ctx->nn == 0) return HIPIB_OK;
    const int64_t cap = spread_list_cap(ctx->ntiles, ctx->nn);
    const int blocks = (int)(cap < 8192 ? cap : 8192);
    const bool mixed = ctx->cfg.precision == HIPIB_MIXED;
#define HIPIB_INTERP(TT, TW)                                                                               \
    return launch_k(ctx, HIPIB_TIMER_INTERP, 0.0, k_interp_tiles<TT, TW>, dim3(blocks), dim3(kSpreadChunk), 0, X, \
                    u, U, Xupd, dt, ctx->perm, ctx->bin_off, ctx->tile_list, ctx->n_list, ctx->n,               \
                    ctx->tiles_axis, ctx->n3, 1.0 / ctx->h)
    if (ctx->tile == 8) {
        if (mixed) HIPIB_INTERP(8, float);
        HIPIB_INTERP(8, double);
    }
    if (mixed) HIPIB_INTERP(4, float);
    HIPIB_INTERP(4, double);
#undef HIPIB_INTERP
}

}  // namespace hipib

// ---------------------------------------------------------------------------
// hipib_spread_noalloc
// ---------------------------------------------------------------------------

namespace hipib {
namespace {

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mutex;
int32_t* g_na_ptr[kNaMaxDevices] = {};   // device address of `scratch`, per device

// Device address of this device's copy of `scratch`, looked up on the first
// call on each device (with that device current).  Host code never passes the
// array's own name to a kernel: on the host it is only a stand-in.
hipib_status noalloc_scratch(int32_t** out) {
    hipib_ctx* ctx = nullptr;   // (no context to mark broken)
    int dev = 0;
    HIPIB_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) return fail(HIPIB_E_INVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_na_mutex);
    if (!g_na_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return fail(HIPIB_E_HIP, "hipGetSymbolAddress(scratch) failed on device %d: HIP error %d",
                        dev, (int)e);
        }
        g_na_ptr[dev] = static_cast<int32_t*>(p);
    }
    *out = g_na_ptr[dev];
    return HIPIB_OK;
}

}  // namespace

}  // namespace hipib

using namespace hipib;

hipib_status hipib_spread_noalloc(int32_t n, int32_t n_nodes, const double* X, const double* F,
                                  double* f, void* stream) {
    hipib_ctx* ctx = nullptr;   // (no context to mark broken)
    if (n < 8 || n > kNaMaxN)
        return fail(HIPIB_E_INVAL, "hipib_spread_noalloc: n = %d outside [8, %d]", n, kNaMaxN);
    {
        int m = n;
        while (m >= 8) {
            if (m % 2) return fail(HIPIB_E_INVAL, "hipib_spread_noalloc: n = %d is not 4*2^k or 6*2^k", n);
            m /= 2;
        }
        if (m != 4 && m != 6)
            return fail(HIPIB_E_INVAL, "hipib_spread_noalloc: n = %d is not 4*2^k or 6*2^k", n);
    }
    if (n_nodes < 0 || n_nodes > kNaMaxNodes)
        return fail(HIPIB_E_INVAL, "hipib_spread_noalloc: n_nodes = %d outside [0, %d]", n_nodes,
                    kNaMaxNodes);
    if (f == nullptr || (reinterpret_cast<uintptr_t>(f) & 7u) ||
        (n_nodes > 0 && (X == nullptr || F == nullptr || (reinterpret_cast<uintptr_t>(X) & 7u) ||
                         (reinterpret_cast<uintptr_t>(F) & 7u))))
        return fail(HIPIB_E_INVAL, "hipib_spread_noalloc: bad pointer");
    if (n_nodes == 0) return HIPIB_OK;
    int32_t* base = nullptr;
    HIPIB_TRY(noalloc_scratch(&base));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int T = (n % 8 == 0) ? 8 : 4;
    const int ta = n / T;
    const int64_t ntiles = (int64_t)ta * ta * ta;
    const int64_t cap = spread_list_cap(ntiles, n_nodes);
    int32_t* count = base;
    int32_t* off = count + ntiles;
    int32_t* list = off + ntiles + 1;
    int32_t* nlist = list + 2 * cap;
    int32_t* node_tile = nlist + 1;
    int32_t* node_rank = node_tile + n_nodes;
    int32_t* perm = node_rank + n_nodes;
    if (perm + n_nodes > base + kNaWords)
        return fail(HIPIB_E_INVAL, "hipib_spread_noalloc: workspace exceeds its %lld words",
                    (long long)kNaWords);
    const double h = 1.0 / n;
    const int nb = (n_nodes + 255) / 256;
    // the tile counts start at zero (a fill kernel, so the call can be captured in a graph)
    k_zero_i32<<<(unsigned)((ntiles + 255) / 256), 256, 0, st>>>(count, ntiles);
    k_bin_count<<<nb, 256, 0, st>>>(X, n_nodes, n, T, ta, 1.0 / h, node_tile, node_rank, count, nullptr);
    k_bin_scan<<<1, 1024, 0, st>>>(count, ntiles, off, list, nlist, nullptr);
    k_bin_scatter<<<nb, 256, 0, st>>>(node_tile, node_rank, off, perm, n_nodes);
    const int blocks = (int)(cap < 8192 ? cap : 8192);
    const int64_t n3 = (int64_t)n * n * n;
    if (T == 8)
        k_spread_tiles<8, double><<<dim3(blocks, 3), kSpreadChunk, 0, st>>>(X, F, f, perm, off, list, nlist, n, ta,
                                                                   n3, 1.0 / h, 1.0 / (h * h * h), 0);
    else
        k_spread_tiles<4, double><<<dim3(blocks, 3), kSpreadChunk, 0, st>>>(X, F, f, perm, off, list, nlist, n, ta,
                                                                   n3, 1.0 / h, 1.0 / (h * h * h), 0);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}
