// Deterministic mode (hipib_config.deterministic = 1): the parts of the step
// that otherwise add floating-point values with atomics in a run-dependent
// order are replaced by fixed-order sums, so every result is bitwise the same
// from run to run.
//
// Spreading ("Eulerian-Lagrangian coupling operators", sorted-segment form,
// atomic-free): the nodes are sorted, stably, by the cell holding floor(X/h)
// (key: tile-major cell index; a hand-written LSD radix sort of 8-bit digits),
// so each tile's bin lists its cells in order and each cell's nodes in node
// order.  The binning's work items (at most kSpreadChunk consecutive nodes of
// one tile) each sum their nodes' contributions, in that order, into a box of
// their own (lane-owned box cells, no atomics) written to a per-item buffer;
// every grid value then adds the boxes that reach it in a fixed order (its
// neighbouring tiles in z, y, x order, each tile's items in list order).
//
// Element and face scatters (FE force, pressure load and their adjoints) write
// per-element contributions; each node then sums the contributions of its
// incident (element, local node) pairs in element order (a CSR list built at
// set-up).  The Holzapfel-Ogden parameter gradient is summed per element slot
// with a fixed reduction tree.
#include "delta.h"
#include "internal.h"

namespace hipib {
namespace {

constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kRadixThreads = 256;
constexpr int kRadixPerThread = 8;
constexpr int kRadixBlock = kRadixThreads * kRadixPerThread;   // keys per workgroup
static_assert(kRadixThreads == kRadixBins, "one thread per digit in the radix passes");

// sort key of every node: tile-major index of the cell holding floor(X/h)
// (the binning's tile and cell, so the key order groups the tile bins);
// values start as the node numbers.  Thread 0 also clears the count of
// active tiles that k_det_active fills.
__global__ void __launch_bounds__(256)
k_det_keys(const double* __restrict__ X, int nn, int n, int T, int ta, double inv_h,
           uint32_t* __restrict__ key, int32_t* __restrict__ idx, int32_t* __restrict__ nactive) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) *nactive = 0;
    if (q >= nn) return;
    int c[3];
    for (int e = 0; e < 3; ++e) c[e] = wrap_mod((int)floor(safe_coord(X[3 * q + e] * inv_h)), n);
    const int64_t tile = c[0] / T + (int64_t)ta * (c[1] / T + (int64_t)ta * (c[2] / T));
    const int local = c[0] % T + T * (c[1] % T + T * (c[2] % T));
    key[q] = (uint32_t)(tile * T * T * T + local);
    idx[q] = q;
}

// digit histogram of each workgroup's kRadixBlock keys: hist[digit][block]
__global__ void __launch_bounds__(kRadixThreads)
k_radix_hist(const uint32_t* __restrict__ key, int64_t count, int shift, int32_t* __restrict__ hist,
             int nblocks) {
    __shared__ int32_t c[kRadixBins];
    c[threadIdx.x] = 0;
    __syncthreads();
    for (int r = 0; r < kRadixPerThread; ++r) {
        const int64_t i = (int64_t)blockIdx.x * kRadixBlock + r * kRadixThreads + threadIdx.x;
        if (i < count) atomicAdd(&c[(key[i] >> shift) & (kRadixBins - 1)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = c[threadIdx.x];
}

// exclusive scan of hist in place (digit-major, so a digit's blocks follow
// each other): one workgroup, in pieces of 8192 counts staged in LDS with
// coalesced loads; each thread scans 8 consecutive counts, the 1024 thread
// sums are scanned in LDS and a carry runs from piece to piece
__global__ void __launch_bounds__(1024)
k_radix_scan(int32_t* __restrict__ hist, int64_t total) {
    constexpr int PER = 8, PIECE = 1024 * PER;
    __shared__ int32_t s[PIECE];
    __shared__ int32_t ts[1024];
    const int tid = threadIdx.x;
    int32_t carry = 0;
    for (int64_t base = 0; base < total; base += PIECE) {
        for (int k = 0; k < PER; ++k) {
            const int64_t i = base + k * 1024 + tid;
            s[k * 1024 + tid] = i < total ? hist[i] : 0;
        }
        __syncthreads();
        int32_t v[PER], sum = 0;
        for (int k = 0; k < PER; ++k) {
            v[k] = s[tid * PER + k];
            sum += v[k];
        }
        ts[tid] = sum;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int32_t a = tid >= o ? ts[tid - o] : 0;
            __syncthreads();
            ts[tid] += a;
            __syncthreads();
        }
        int32_t run = carry + ts[tid] - sum;
        for (int k = 0; k < PER; ++k) {
            s[tid * PER + k] = run;
            run += v[k];
        }
        carry += ts[1023];
        __syncthreads();
        for (int k = 0; k < PER; ++k) {
            const int64_t i = base + k * 1024 + tid;
            if (i < total) hist[i] = s[k * 1024 + tid];
        }
        __syncthreads();
    }
}

// stable scatter by one digit.  With R = kRadixPerThread, wavefront w of the
// workgroup takes R rounds of 64 consecutive keys (keys [64 R w, 64 R (w + 1))
// of the block); in each round the lanes holding equal digits are found with
// one ballot per digit bit, which gives each key its rank among the round's
// equal digits and the round's count per digit.  Counts of the 4 R (wave,
// round) groups are prefix-summed per digit in group order, on top of the
// digit's offset for this block, so equal digits keep their input order.
__global__ void __launch_bounds__(kRadixThreads)
k_radix_scatter(const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin, int64_t count,
                int shift, const int32_t* __restrict__ hist, int nblocks, uint32_t* __restrict__ kout,
                int32_t* __restrict__ vout) {
    constexpr int G = (kRadixThreads / 64) * kRadixPerThread;
    __shared__ int32_t cnt[G][kRadixBins];
    for (int g = 0; g < G; ++g) cnt[g][threadIdx.x] = 0;
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    uint32_t k[kRadixPerThread];
    int32_t v[kRadixPerThread];
    int dig[kRadixPerThread], rank[kRadixPerThread];
    bool ok[kRadixPerThread];
    for (int r = 0; r < kRadixPerThread; ++r) {
        const int64_t i = (int64_t)blockIdx.x * kRadixBlock + w * (64 * kRadixPerThread) + r * 64 + lane;
        ok[r] = i < count;
        k[r] = ok[r] ? kin[i] : 0u;
        v[r] = ok[r] ? vin[i] : 0;
        dig[r] = (int)((k[r] >> shift) & (kRadixBins - 1));
        unsigned long long m = __ballot(ok[r]);
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (dig[r] >> b) & 1;
            const unsigned long long bb = __ballot(ok[r] && bit);
            m &= bit ? bb : ~bb;
        }
        rank[r] = __popcll(m & below);
        if (ok[r] && rank[r] == 0) cnt[w * kRadixPerThread + r][dig[r]] = __popcll(m);
    }
    __syncthreads();
    {
        int32_t run = hist[(int64_t)threadIdx.x * nblocks + blockIdx.x];
        for (int g = 0; g < G; ++g) {
            const int32_t c = cnt[g][threadIdx.x];
            cnt[g][threadIdx.x] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int r = 0; r < kRadixPerThread; ++r) {
        if (!ok[r]) continue;
        const int32_t pos = cnt[w * kRadixPerThread + r][dig[r]] + rank[r];
        kout[pos] = k[r];
        vout[pos] = v[r];
    }
}

// weight k (0..3) of the four-point stencil at fractional offset fr, with
// sq = sqrt(1 + 4 fr (1 - fr)): the atomic spreading's formulas and rounding
template <typename TW>
__device__ __forceinline__ TW phi4(TW fr, TW sq, int k) {
    const TW t = k < 2 ? TW(3) - TW(2) * fr : TW(1) + TW(2) * fr;
    return (k == 0 || k == 3 ? t - sq : t + sq) * TW(0.125);
}

// Ordered scatter of one work item (at most kSpreadChunk consecutive sorted
// nodes of one tile: its cells in order, each cell's nodes in node order) on
// lattice d into the item's own E^3 box (E = T + 4, from 2 cells below the
// tile, the reach of every stencil of the tile's nodes).  Each box cell is
// owned by one lane: wave w holds box planes 4 w .. 4 w + 3 and lane
// (rx, ry, rz) the cells whose (x, y, z) mod 4 is (rx, ry, rz) there.  A
// 4x4x4 stencil meets each residue class once, so for every node each lane
// adds at most one product, to a cell only it writes: the box sums are in node
// order with no atomics and no cross-lane ordering.  Each node's 1-D weights
// (TW), force and stencil start are computed once into LDS first.
template <int T, typename TW>
__global__ void __launch_bounds__((T + 4) / 4 * 64)
k_det_scatter(const double* __restrict__ X, const double* __restrict__ F, const int32_t* __restrict__ sidx,
              const int32_t* __restrict__ bin_off, const int32_t* __restrict__ list,
              const int32_t* __restrict__ nlist, int n, int ta, double inv_h, double ih3,
              double* __restrict__ buf) {
    constexpr int E = T + 4, E3 = E * E * E, NW = E / 4, NT = NW * 64, C = kSpreadChunk;
    static_assert(E % 4 == 0, "box planes in groups of four");
    __shared__ TW s_w[C][12];
    __shared__ TW s_val[C];
    __shared__ int32_t s_start[C];
    __shared__ double box[E3];
    const int d = blockIdx.y;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rx = lane & 3, ry = (lane >> 2) & 3, rz = lane >> 4;
    const int zc = 4 * w + rz;
    const int ntl = *nlist;
    for (int li = blockIdx.x; li < ntl; li += gridDim.x) {
        const int tile = list[2 * li];
        const int tb[3] = {T * (tile % ta), T * ((tile / ta) % ta), T * (tile / (ta * ta))};
        const int s0 = bin_off[tile] + list[2 * li + 1];
        const int left = bin_off[tile + 1] - s0;
        const int cnt = left < C ? left : C;
        __syncthreads();   // the previous item's reads of LDS are done
        for (int e = threadIdx.x; e < E3; e += NT) box[e] = 0.0;
        for (int i = threadIdx.x; i < cnt; i += NT) {
            const int q = sidx[s0 + i];
            int st = 0;
            for (int e = 0; e < 3; ++e) {
                const double xs = safe_coord(X[3 * q + e] * inv_h);
                const int cw = wrap_mod((int)floor(xs), n);
                const double r = xs - (e == d ? 0.0 : 0.5);
                const double bf = floor(r);
                const TW fr = (TW)(r - bf);
                const TW sq = sqrt(TW(1) + TW(4) * fr * (TW(1) - fr));
                for (int k = 0; k < 4; ++k) s_w[i][4 * e + k] = phi4(fr, sq, k);
                // stencil start in the box: the node's cell minus 1 or 2
                const int ls = cw - tb[e] + 2 + ((int)bf - 1 - (int)floor(xs));
                st |= ls << (8 * e);
            }
            s_val[i] = (TW)(F[3 * q + d] * ih3);
            s_start[i] = st;
        }
        __syncthreads();
        for (int i = 0; i < cnt; ++i) {
            const int st = s_start[i];
            const int lsx = st & 255, lsy = (st >> 8) & 255, lsz = st >> 16;
            const int c = zc - lsz;
            if ((unsigned)c > 3u) continue;
            const int a = (rx - lsx) & 3, b = (ry - lsy) & 3;
            const TW wyz = s_w[i][4 + b] * s_w[i][8 + c];
            const TW v = s_val[i] * (s_w[i][a] * wyz);
            box[(lsx + a) + E * ((lsy + b) + E * zc)] += (double)v;
        }
        __syncthreads();
        double* B = buf + ((int64_t)li * 3 + d) * E3;
        for (int e = threadIdx.x; e < E3; e += NT) B[e] = box[e];
    }
}

// tiles whose grid values some work item's box reaches (an occupied tile
// among the tile and its neighbours), listed in any order
__global__ void __launch_bounds__(256)
k_det_active(const int32_t* __restrict__ bin_off, int64_t ntiles, int ta, int32_t* __restrict__ active,
             int32_t* __restrict__ nactive) {
    const int64_t tile = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tile >= ntiles) return;
    const int t3[3] = {(int)(tile % ta), (int)((tile / ta) % ta), (int)(tile / ((int64_t)ta * ta))};
    bool on = false;
    for (int k = 0; k < 27; ++k) {   // all 27 loads issued together
        const int nt[3] = {wrap_mod(t3[0] + k % 3 - 1, ta), wrap_mod(t3[1] + (k / 3) % 3 - 1, ta),
                           wrap_mod(t3[2] + k / 9 - 1, ta)};
        const int64_t t = nt[0] + (int64_t)ta * (nt[1] + (int64_t)ta * nt[2]);
        on |= bin_off[t + 1] > bin_off[t];
    }
    if (on) active[atomicAdd(nactive, 1)] = (int32_t)tile;
}

// f^d[g] += the boxes of the work items that reach g, in a fixed order: the
// distinct neighbouring tiles (z, then y, then x offsets), each tile's items in
// list order.  Workgroups take the active tiles (grid-stride) for lattice d,
// one thread per grid value of the tile.
template <int T>
__global__ void __launch_bounds__(T * T * T)
k_det_combine(const double* __restrict__ buf, const int32_t* __restrict__ bin_off,
              const int32_t* __restrict__ lfirst, const int32_t* __restrict__ active,
              const int32_t* __restrict__ nactive, int n, int ta, int64_t n3, double* __restrict__ f,
              int f_packed) {
    constexpr int E = T + 4, E3 = E * E * E;
    __shared__ int32_t s_nch[27], s_l0[27], s_org[27][3];
    const int d = blockIdx.y;
    const int na = *nactive;
    // neighbouring tiles along an axis, each once: -1, 0, +1 (two tiles: -1, 0; one: 0)
    const int o0 = ta >= 2 ? -1 : 0, m = ta >= 3 ? 3 : ta, m3 = m * m * m;
    for (int ai = blockIdx.x; ai < na; ai += gridDim.x) {
        const int tile = active[ai];
        const int t3[3] = {tile % ta, (tile / ta) % ta, tile / (ta * ta)};
        __syncthreads();   // the previous tile's reads of the table are done
        if ((int)threadIdx.x < m3) {
            const int k = threadIdx.x;
            const int nt[3] = {wrap_mod(t3[0] + o0 + k % m, ta), wrap_mod(t3[1] + o0 + (k / m) % m, ta),
                               wrap_mod(t3[2] + o0 + k / (m * m), ta)};
            const int64_t t = nt[0] + (int64_t)ta * (nt[1] + (int64_t)ta * nt[2]);
            const int32_t cnt = bin_off[t + 1] - bin_off[t];
            s_nch[k] = (cnt + kSpreadChunk - 1) / kSpreadChunk;
            s_l0[k] = lfirst[t];
            for (int e = 0; e < 3; ++e) s_org[k][e] = T * nt[e] - 2;   // the tile's box origin
        }
        __syncthreads();
        const int g[3] = {T * t3[0] + (int)threadIdx.x % T, T * t3[1] + ((int)threadIdx.x / T) % T,
                          T * t3[2] + (int)threadIdx.x / (T * T)};
        double acc = 0.0;
        bool any = false;
        for (int k = 0; k < m3; ++k) {   // z, then y, then x offsets
            const int nch = s_nch[k];
            if (nch == 0) continue;
            const int l0 = s_l0[k];
            int rel[3];
            for (int e = 0; e < 3; ++e) {   // g - origin lies in (-n, n + 2): one wrap at most
                const int r = g[e] - s_org[k][e];
                rel[e] = r < 0 ? r + n : (r >= n ? r - n : r);
            }
            // box coordinates of g in the tile's box (a grid smaller than the box
            // meets it more than once along an axis)
            for (int bz = rel[2]; bz < E; bz += n)
                for (int by = rel[1]; by < E; by += n)
                    for (int bx = rel[0]; bx < E; bx += n) {
                        const double* B = buf + ((int64_t)l0 * 3 + d) * E3 + bx + E * (by + E * bz);
                        constexpr int64_t S = 3 * (int64_t)E3;   // stride between a tile's items
                        int ch = 0;
                        for (; ch + 8 <= nch; ch += 8) {   // eight loads in flight, added in order
                            double v[8];
                            for (int u = 0; u < 8; ++u) v[u] = B[(ch + u) * S];
                            for (int u = 0; u < 8; ++u) acc += v[u];
                        }
                        for (; ch < nch; ++ch) acc += B[ch * S];
                        any = true;
                    }
        }
        if (any)
            f[d * n3 + (f_packed ? pk(g[0], g[1], g[2], n) : g[0] + (int64_t)n * (g[1] + (int64_t)n * g[2]))] += acc;
    }
}

// out[3 i + r] (= or +=) sum over t in [off[i], off[i+1]) of contrib[3 inc[t] + r]
__global__ void __launch_bounds__(256)
k_det_gather(const double* __restrict__ contrib, const int32_t* __restrict__ off,
             const int32_t* __restrict__ inc, int count, int accumulate, double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int t = off[i]; t < off[i + 1]; ++t) {
        const int64_t c = 3 * (int64_t)inc[t];
        s0 += contrib[c];
        s1 += contrib[c + 1];
        s2 += contrib[c + 2];
    }
    if (accumulate) {
        out[3 * i] += s0;
        out[3 * i + 1] += s1;
        out[3 * i + 2] += s2;
    } else {
        out[3 * i] = s0;
        out[3 * i + 1] = s1;
        out[3 * i + 2] = s2;
    }
}

// dtheta[m][k] += sum over elements of material m of part[4 e + k]: block
// (m, k), 256 threads with strided partial sums in element order, then a
// fixed shared-memory tree
__global__ void __launch_bounds__(256)
k_det_param_reduce(const double* __restrict__ part, const int32_t* __restrict__ mat_id, int ne,
                   double* __restrict__ dtheta) {
    __shared__ double red[256];
    const int m = blockIdx.x / 4, k = blockIdx.x - 4 * m;
    double s = 0.0;
    for (int e = threadIdx.x; e < ne; e += 256)
        if (mat_id[e] == m) s += part[4 * (int64_t)e + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] != 0.0) dtheta[blockIdx.x] += red[0];
}

}  // namespace

hipib_status det_prepare_mesh(hipib_ctx* ctx, const int32_t* conn) {
    // node -> incident (element, local node) pairs in element order
    const int nn = ctx->nn, ne = ctx->ne, npe = ctx->npe;
    std::vector<int32_t> off(nn + 1, 0), inc(npe * (size_t)ne);
    for (int64_t t = 0; t < npe * (int64_t)ne; ++t) ++off[conn[t] + 1];
    for (int i = 0; i < nn; ++i) off[i + 1] += off[i];
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (int64_t t = 0; t < npe * (int64_t)ne; ++t) inc[fill[conn[t]]++] = (int32_t)t;
    auto alloc = [&](void** p, size_t bytes) -> hipib_status {
        *p = nullptr;
        if (hipMalloc(p, bytes ? bytes : 1) != hipSuccess) {
            (void)hipGetLastError();
            return fail(HIPIB_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
        }
        return HIPIB_OK;
    };
    HIPIB_TRY(alloc(reinterpret_cast<void**>(&ctx->det_node_off), sizeof(int32_t) * (nn + 1)));
    HIPIB_TRY(alloc(reinterpret_cast<void**>(&ctx->det_node_inc), sizeof(int32_t) * inc.size()));
    HIPIB_HIP(hipMemcpy(ctx->det_node_off, off.data(), sizeof(int32_t) * (nn + 1), hipMemcpyHostToDevice));
    if (!inc.empty())
        HIPIB_HIP(hipMemcpy(ctx->det_node_inc, inc.data(), sizeof(int32_t) * inc.size(), hipMemcpyHostToDevice));
    HIPIB_TRY(alloc(reinterpret_cast<void**>(&ctx->det_contrib), sizeof(double) * 3 * npe * (size_t)ne));
    HIPIB_TRY(alloc(reinterpret_cast<void**>(&ctx->det_param), sizeof(double) * 4 * (size_t)ne));
    // spreading: sort keys and values (two buffers each), digit histograms,
    // each tile's first work item, the active tiles and one box per work item
    const int nblk = (int)((nn + kRadixBlock - 1) / kRadixBlock);
    ctx->det_nblk = nblk;
    int bits = 1;
    while (((int64_t)1 << bits) < ctx->n3) ++bits;
    ctx->det_bits = bits;
    for (int b = 0; b < 2; ++b) {
        HIPIB_TRY(alloc(reinterpret_cast<void**>(&ctx->det_key[b]), sizeof(uint32_t) * (size_t)nn));
        HIPIB_TRY(alloc(reinterpret_cast<void**>(&ctx->det_idx[b]), sizeof(int32_t) * (size_t)nn));
    }
    HIPIB_TRY(alloc(reinterpret_cast<void**>(&ctx->det_hist), sizeof(int32_t) * kRadixBins * (size_t)nblk));
    const int64_t cap = spread_list_cap(ctx->ntiles, nn);
    const int64_t E = ctx->tile + 4;
    HIPIB_TRY(alloc(reinterpret_cast<void**>(&ctx->det_lfirst), sizeof(int32_t) * (size_t)ctx->ntiles));
    HIPIB_TRY(alloc(reinterpret_cast<void**>(&ctx->det_active), sizeof(int32_t) * (size_t)(ctx->ntiles + 1)));
    ctx->det_nactive = ctx->det_active + ctx->ntiles;
    HIPIB_TRY(alloc(reinterpret_cast<void**>(&ctx->det_buf), sizeof(double) * 3 * E * E * E * (size_t)cap));
    return HIPIB_OK;
}

hipib_status det_prepare_faces(hipib_ctx* ctx, const int32_t* faces, int nf) {
    std::vector<int32_t> off(ctx->nn + 1, 0), inc(4 * (size_t)nf);
    for (int64_t t = 0; t < 4 * (int64_t)nf; ++t) ++off[faces[t] + 1];
    for (int i = 0; i < ctx->nn; ++i) off[i + 1] += off[i];
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (int64_t t = 0; t < 4 * (int64_t)nf; ++t) inc[fill[faces[t]]++] = (int32_t)t;
    (void)hipFree(ctx->det_face_off);
    (void)hipFree(ctx->det_face_inc);
    (void)hipFree(ctx->det_face_contrib);
    ctx->det_face_off = ctx->det_face_inc = nullptr;
    ctx->det_face_contrib = nullptr;
    if (hipMalloc(&ctx->det_face_off, sizeof(int32_t) * (ctx->nn + 1)) != hipSuccess ||
        hipMalloc(&ctx->det_face_inc, sizeof(int32_t) * (inc.size() ? inc.size() : 1)) != hipSuccess ||
        hipMalloc(&ctx->det_face_contrib, sizeof(double) * 12 * (size_t)(nf ? nf : 1)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(HIPIB_E_NOMEM, "hipMalloc of the face lists failed");
    }
    HIPIB_HIP(hipMemcpy(ctx->det_face_off, off.data(), sizeof(int32_t) * (ctx->nn + 1), hipMemcpyHostToDevice));
    if (!inc.empty())
        HIPIB_HIP(hipMemcpy(ctx->det_face_inc, inc.data(), sizeof(int32_t) * inc.size(), hipMemcpyHostToDevice));
    return HIPIB_OK;
}

hipib_status det_spread(hipib_ctx* ctx, const double* X, const double* F, double* f, bool f_packed) {
    const int nn = ctx->nn;
    if (nn == 0) return HIPIB_OK;
    const double h = ctx->h;
    const int T = ctx->tile, ta = ctx->tiles_axis, nblk = ctx->det_nblk;
    hipStream_t st = ctx->stream;
    k_det_keys<<<(nn + 255) / 256, 256, 0, st>>>(X, nn, ctx->n, T, ta, 1.0 / h, ctx->det_key[0],
                                                ctx->det_idx[0], ctx->det_nactive);
    int cur = 0;
    for (int shift = 0; shift < ctx->det_bits; shift += kRadixBits) {
        k_radix_hist<<<nblk, kRadixThreads, 0, st>>>(ctx->det_key[cur], nn, shift, ctx->det_hist, nblk);
        k_radix_scan<<<1, 1024, 0, st>>>(ctx->det_hist, (int64_t)kRadixBins * nblk);
        k_radix_scatter<<<nblk, kRadixThreads, 0, st>>>(ctx->det_key[cur], ctx->det_idx[cur], nn, shift,
                                                        ctx->det_hist, nblk, ctx->det_key[1 - cur],
                                                        ctx->det_idx[1 - cur]);
        cur = 1 - cur;
    }
    const int64_t cap = spread_list_cap(ctx->ntiles, nn);
    const dim3 gs((unsigned)(cap < 2048 ? cap : 2048), 3);
    const dim3 gc((unsigned)(ctx->ntiles < 1024 ? ctx->ntiles : 1024), 3);
    k_det_active<<<(unsigned)((ctx->ntiles + 255) / 256), 256, 0, st>>>(ctx->bin_off, ctx->ntiles, ta,
                                                                        ctx->det_active, ctx->det_nactive);
    const bool mixed = ctx->cfg.precision == HIPIB_MIXED;
#define HIPIB_DET(TT, TW)                                                                                  \
    HIPIB_TRY(launch_k(ctx, HIPIB_TIMER_SPREAD, 0.0, k_det_scatter<TT, TW>, gs, dim3((TT + 4) / 4 * 64), 0, X, \
                       F, ctx->det_idx[cur], ctx->bin_off, ctx->tile_list, ctx->n_list, ctx->n, ta,        \
                       1.0 / h, 1.0 / (h * h * h), ctx->det_buf));                                         \
    k_det_combine<TT><<<gc, TT * TT * TT, 0, st>>>(ctx->det_buf, ctx->bin_off, ctx->det_lfirst,             \
                                                    ctx->det_active, ctx->det_nactive, ctx->n, ta, ctx->n3, f, \
                                                    f_packed ? 1 : 0)
    if (T == 8) {
        if (mixed) { HIPIB_DET(8, float); } else { HIPIB_DET(8, double); }
    } else {
        if (mixed) { HIPIB_DET(4, float); } else { HIPIB_DET(4, double); }
    }
#undef HIPIB_DET
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

hipib_status det_gather_nodes(hipib_ctx* ctx, bool faces, bool accumulate, double* out) {
    if (ctx->nn == 0) return HIPIB_OK;
    k_det_gather<<<(ctx->nn + 255) / 256, 256, 0, ctx->stream>>>(
        faces ? ctx->det_face_contrib : ctx->det_contrib, faces ? ctx->det_face_off : ctx->det_node_off,
        faces ? ctx->det_face_inc : ctx->det_node_inc, ctx->nn, accumulate ? 1 : 0, out);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

hipib_status det_param_reduce(hipib_ctx* ctx, double* dtheta) {
    if (ctx->ne == 0) return HIPIB_OK;
    k_det_param_reduce<<<HIPIB_MAX_MATERIALS * 4, 256, 0, ctx->stream>>>(ctx->det_param, ctx->mat_id,
                                                                         ctx->ne, dtheta);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

void det_free(hipib_ctx* ctx) {
    (void)hipFree(ctx->det_node_off);
    (void)hipFree(ctx->det_node_inc);
    (void)hipFree(ctx->det_contrib);
    (void)hipFree(ctx->det_param);
    for (int b = 0; b < 2; ++b) {
        (void)hipFree(ctx->det_key[b]);
        (void)hipFree(ctx->det_idx[b]);
        ctx->det_key[b] = nullptr;
        ctx->det_idx[b] = nullptr;
    }
    (void)hipFree(ctx->det_hist);
    (void)hipFree(ctx->det_lfirst);
    (void)hipFree(ctx->det_active);
    (void)hipFree(ctx->det_buf);
    ctx->det_node_off = ctx->det_node_inc = nullptr;
    ctx->det_contrib = ctx->det_param = nullptr;
    ctx->det_hist = ctx->det_lfirst = ctx->det_active = ctx->det_nactive = nullptr;
    ctx->det_buf = nullptr;
}

void det_free_faces(hipib_ctx* ctx) {
    (void)hipFree(ctx->det_face_off);
    (void)hipFree(ctx->det_face_inc);
    (void)hipFree(ctx->det_face_contrib);
    ctx->det_face_off = ctx->det_face_inc = nullptr;
    ctx->det_face_contrib = nullptr;
}

}  // namespace hipib
