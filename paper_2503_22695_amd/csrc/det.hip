// Deterministic mode (hipib_config.deterministic = 1): the parts of the step
// that otherwise add floating-point values with atomics in a run-dependent
// order are replaced by fixed-order sums, so every result is bitwise the same
// from run to run.
//
// Spreading ("Eulerian-Lagrangian coupling operators", sorted-segment form):
// every (node q, lattice d, stencil point s) contribution F^d_q w_s / h^3 is
// written as a (grid index, value) pair at position (3 q + d) 64 + s; a stable
// radix sort on the grid index groups the pairs of each grid point in node
// order; the first pair of each group sums its group in that order and adds
// the sum to the grid value (one writer per grid point).
//
// Element and face scatters (FE force, pressure load and their adjoints) write
// per-element contributions; each node then sums the contributions of its
// incident (element, local node) pairs in element order (a CSR list built at
// set-up).  The Holzapfel-Ogden parameter gradient is summed per element slot
// with a fixed reduction tree.
#include <hipcub/hipcub.hpp>

#include "delta.h"
#include "internal.h"

namespace hipib {
namespace {

// one thread per (node, lattice): 64 pairs
template <typename TW>
__global__ void __launch_bounds__(256)
k_det_pairs(const double* __restrict__ X, const double* __restrict__ F, int nn, int n, int64_t n3,
            double inv_h, double ih3, uint32_t* __restrict__ keys, double* __restrict__ vals) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * nn) return;
    const int q = t / 3, d = t - 3 * q;
    int i0[3];
    TW w[3][4];
    for (int e = 0; e < 3; ++e) {
        const double r = safe_coord(X[3 * q + e] * inv_h - (e == d ? 0.0 : 0.5));
        const double bf = floor(r);
        const TW fr = (TW)(r - bf);
        const TW sq = sqrt(TW(1) + TW(4) * fr * (TW(1) - fr));
        w[e][0] = (TW(3) - TW(2) * fr - sq) * TW(0.125);
        w[e][1] = (TW(3) - TW(2) * fr + sq) * TW(0.125);
        w[e][2] = (TW(1) + TW(2) * fr + sq) * TW(0.125);
        w[e][3] = (TW(1) + TW(2) * fr - sq) * TW(0.125);
        i0[e] = wrap_mod((int)bf - 1, n);
    }
    const TW val = (TW)(F[3 * q + d] * ih3);
    const int64_t base = (int64_t)t * 64;
    for (int c = 0; c < 4; ++c) {
        const int kk = step_wrap(i0[2] + c, n);
        for (int b = 0; b < 4; ++b) {
            const int jj = step_wrap(i0[1] + b, n);
            const TW wyz = w[1][b] * w[2][c];
            for (int a = 0; a < 4; ++a) {
                const int ii = step_wrap(i0[0] + a, n);
                const int64_t s = base + a + 4 * (b + 4 * c);
                keys[s] = (uint32_t)(d * n3 + ii + (int64_t)n * (jj + (int64_t)n * kk));
                vals[s] = (double)(val * (w[0][a] * wyz));
            }
        }
    }
}

// first pair of each run of equal keys sums the run in order into f[key]
__global__ void __launch_bounds__(256)
k_det_segsum(const uint32_t* __restrict__ keys, const double* __restrict__ vals, int64_t count,
             double* __restrict__ f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint32_t k = keys[i];
    if (i > 0 && keys[i - 1] == k) return;
    double s = 0.0;
    for (int64_t j = i; j < count && keys[j] == k; ++j) s += vals[j];
    f[k] += s;
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
    // spreading pairs and sort workspace
    const int64_t np = 192 * (int64_t)nn;
    ctx->det_pairs = np;
    for (int b = 0; b < 2; ++b) {
        HIPIB_TRY(alloc(reinterpret_cast<void**>(&ctx->det_keys[b]), sizeof(uint32_t) * (size_t)np));
        HIPIB_TRY(alloc(reinterpret_cast<void**>(&ctx->det_vals[b]), sizeof(double) * (size_t)np));
    }
    int bits = 1;
    while (((int64_t)1 << bits) < 3 * ctx->n3) ++bits;
    ctx->det_end_bit = bits;
    size_t tb = 0;
    HIPIB_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, ctx->det_keys[0], ctx->det_keys[1],
                                                 ctx->det_vals[0], ctx->det_vals[1], np > 0 ? np : 1,
                                                 0, bits, ctx->stream));
    HIPIB_TRY(alloc(&ctx->det_temp, tb));
    ctx->det_temp_bytes = tb;
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

hipib_status det_spread(hipib_ctx* ctx, const double* X, const double* F, double* f) {
    if (ctx->nn == 0) return HIPIB_OK;
    const int nb = (3 * ctx->nn + 255) / 256;
    const double h = ctx->h;
    if (ctx->cfg.precision == HIPIB_MIXED)
        k_det_pairs<float><<<nb, 256, 0, ctx->stream>>>(X, F, ctx->nn, ctx->n, ctx->n3, 1.0 / h,
                                                        1.0 / (h * h * h), ctx->det_keys[0], ctx->det_vals[0]);
    else
        k_det_pairs<double><<<nb, 256, 0, ctx->stream>>>(X, F, ctx->nn, ctx->n, ctx->n3, 1.0 / h,
                                                         1.0 / (h * h * h), ctx->det_keys[0], ctx->det_vals[0]);
    HIPIB_HIP(hipGetLastError());
    size_t tb = ctx->det_temp_bytes;
    HIPIB_HIP(hipcub::DeviceRadixSort::SortPairs(ctx->det_temp, tb, ctx->det_keys[0], ctx->det_keys[1],
                                                 ctx->det_vals[0], ctx->det_vals[1], ctx->det_pairs, 0,
                                                 ctx->det_end_bit, ctx->stream));
    const int64_t np = ctx->det_pairs;
    k_det_segsum<<<(unsigned)((np + 255) / 256), 256, 0, ctx->stream>>>(ctx->det_keys[1], ctx->det_vals[1],
                                                                        np, f);
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
    (void)hipFree(ctx->det_temp);
    for (int b = 0; b < 2; ++b) {
        (void)hipFree(ctx->det_keys[b]);
        (void)hipFree(ctx->det_vals[b]);
        ctx->det_keys[b] = nullptr;
        ctx->det_vals[b] = nullptr;
    }
    ctx->det_node_off = ctx->det_node_inc = nullptr;
    ctx->det_contrib = ctx->det_param = nullptr;
    ctx->det_temp = nullptr;
    ctx->det_pairs = 0;
}

void det_free_faces(hipib_ctx* ctx) {
    (void)hipFree(ctx->det_face_off);
    (void)hipFree(ctx->det_face_inc);
    (void)hipFree(ctx->det_face_contrib);
    ctx->det_face_off = ctx->det_face_inc = nullptr;
    ctx->det_face_contrib = nullptr;
}

}  // namespace hipib
