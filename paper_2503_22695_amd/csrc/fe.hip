// Matrix-free nodal forces on trilinear hexahedra ("Eulerian-Lagrangian
// coupling operators": F_i = -sum_q P(X_q) : grad N_i(X_q) w_q) and the
// uniform cavity pressure on quads (the left-ventricle model's endocardial
// load), as a follower load on the current configuration.  Holzapfel-Ogden
// materials may carry sheet and fibre-sheet terms (per-element sheet
// directions) and the left-ventricle model's active fibre stress; penalty
// tethers add linear springs at constrained nodes.
//
// One thread per element (trilinear hexes, or P1 / P2 tetrahedra: the kernel is
// instantiated per element type).  With Jr = dX/dxi and Jx = dx/dxi at a Gauss point,
// F = Jx Jr^{-1}, grad_X N_a = Jr^{-T} grad_xi N_a and
//   sum_c P[r][c] grad_X N_a[c] w = sum_s Q[r][s] dN_a/dxi_s,  Q = w P Jr^{-T},
// so the shape-function gradients in X are never formed: per Gauss point the
// element does two N-node gathers of 3x3 Jacobians, one 3x3 inverse, the law,
// one 3x3 product and a 3N-entry update, all in registers (rules in solid.h).
// Node accumulation uses
// hardware FP64 atomics, or in deterministic mode per-element contributions
// gathered per node in element order.
#include "solid.h"

namespace hipib {
namespace {

// T: arithmetic type of the element computation; S: element type (Hex8, Tet4,
// Tet10).  Node positions are taken relative to the element's first node in
// FP64 before rounding to T (the Jacobians only see differences), and element
// forces are accumulated into the FP64 nodal array.  DISP (the FP32 element
// forces of the mixed-precision form): the nodal displacements X - X_ref are
// formed in FP64 and rounded to T, the Gauss point works on the displacement
// gradient H = (dd/dxi) Jr^{-1} and the stress comes from pk1_disp, so the
// rounding of T is relative to the strain, not to |X| / displacement.
template <typename T, typename S, bool DISP = false>
__global__ void __launch_bounds__(128)
k_fe_force(const double* __restrict__ X, const double* __restrict__ Xref,
           const int32_t* __restrict__ conn, const double* __restrict__ fibre,
           const double* __restrict__ sheet, const int32_t* __restrict__ mat_id, MatTable mats,
           double Ta, int ne, double* __restrict__ F, MGState* st, double* __restrict__ contrib) {
    constexpr int N = S::N;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    int nd[N];
#pragma unroll
    for (int a = 0; a < N; ++a) nd[a] = conn[N * (int64_t)e + a];
    T xr[N][3], xc[N][3], fe[N][3];
    const double r0[3] = {Xref[3 * nd[0]], Xref[3 * nd[0] + 1], Xref[3 * nd[0] + 2]};
    const double c0[3] = {X[3 * nd[0]], X[3 * nd[0] + 1], X[3 * nd[0] + 2]};
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            xr[a][r] = (T)(Xref[3 * nd[a] + r] - r0[r]);
            xc[a][r] = DISP ? (T)(X[3 * nd[a] + r] - Xref[3 * nd[a] + r]) : (T)(X[3 * nd[a] + r] - c0[r]);
            fe[a][r] = T(0);
        }
    const int m = mat_id[e];
    const int model = mats.model[m];
    const bool sh = mats.sheet[m] != 0;
    T par[kMatParams];
#pragma unroll
    for (int t = 0; t < kMatParams; ++t) par[t] = (T)mats.p[m][t];
    const T ef[3] = {(T)fibre[3 * e], (T)fibre[3 * e + 1], (T)fibre[3 * e + 2]};
    T es[3] = {T(0), T(0), T(0)};
    T efes = T(0);   // e_f . e_s in FP64 (zero up to the rounding of the inputs)
    if (sh) {
        es[0] = (T)sheet[3 * e];
        es[1] = (T)sheet[3 * e + 1];
        es[2] = (T)sheet[3 * e + 2];
        efes = (T)(fibre[3 * e] * sheet[3 * e] + fibre[3 * e + 1] * sheet[3 * e + 1] +
                   fibre[3 * e + 2] * sheet[3 * e + 2]);
    }
    // the active stress acts on Holzapfel-Ogden (myocardium) materials only
    const T ta = model == HIPIB_HOLZAPFEL_OGDEN ? (T)Ta : T(0);
    bool bad = false;
    for (int g = 0; g < S::Q; ++g) {
        T dN[N][3];
        const T wq = elem_rule<S, T>(g, dN);
        T Jr[9], Jx[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) Jr[t] = Jx[t] = T(0);
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Jr[3 * r + c] += xr[a][r] * dN[a][c];
                    Jx[3 * r + c] += xc[a][r] * dN[a][c];
                }
        const T w = det3(Jr);
        if (!(w > T(0))) { bad = true; continue; }
        T cr[9], Jri[9];
        cof3(Jr, cr);
        const T iw = T(1) / w;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) Jri[3 * r + c] = cr[3 * c + r] * iw;   // Jr^{-1}
        T Fm[9];   // F, or H = F - I when DISP
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                Fm[3 * r + c] = Jx[3 * r] * Jri[c] + Jx[3 * r + 1] * Jri[3 + c] + Jx[3 * r + 2] * Jri[6 + c];
        T P[9];
        if (DISP) {
            if (!pk1_disp<T>(model, par, Fm, ef, es, efes, sh, ta, P)) { bad = true; continue; }
        } else {
            if (!pk1<T>(model, par, Fm, ef, es, sh, ta, P)) { bad = true; continue; }
        }
        const T wg = w * wq;
        T Q[9];   // wg P Jr^{-T}
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int s = 0; s < 3; ++s)
                Q[3 * r + s] = wg * (P[3 * r] * Jri[3 * s] + P[3 * r + 1] * Jri[3 * s + 1] +
                                     P[3 * r + 2] * Jri[3 * s + 2]);
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
            for (int r = 0; r < 3; ++r)
                fe[a][r] -= Q[3 * r] * dN[a][0] + Q[3 * r + 1] * dN[a][1] + Q[3 * r + 2] * dN[a][2];
    }
    if (bad) atomicOr(&st->numeric, 1);
    if (contrib) {  // deterministic mode: gathered per node in element order
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
            for (int r = 0; r < 3; ++r) contrib[3 * (N * (int64_t)e + a) + r] = (double)fe[a][r];
        return;
    }
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int r = 0; r < 3; ++r) atomicAdd(F + 3 * nd[a] + r, (double)fe[a][r]);
}

// F_a -= p * sum over 2x2 Gauss points of N_a (dx/dxi x dx/deta)
__global__ void __launch_bounds__(256)
k_pressure_load(const double* __restrict__ X, const int32_t* __restrict__ faces, int nf, double p,
                double* __restrict__ F, double* __restrict__ contrib) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    int nd[4];
    double x[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        nd[a] = faces[4 * f + a];
#pragma unroll
        for (int r = 0; r < 3; ++r) x[a][r] = X[3 * nd[a] + r];
    }
    const double gp = 0.57735026918962576451;
    double fa[4][3] = {};
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const double s = (g & 1) ? gp : -gp, t = (g & 2) ? gp : -gp;
        double N[4], dS[4], dT[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const double sa = (a & 1) ? 1.0 : -1.0, ta = (a & 2) ? 1.0 : -1.0;
            N[a] = (1.0 + sa * s) * (1.0 + ta * t) * 0.25;
            dS[a] = sa * (1.0 + ta * t) * 0.25;
            dT[a] = (1.0 + sa * s) * ta * 0.25;
        }
        double xs[3] = {0, 0, 0}, xt[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                xs[r] += x[a][r] * dS[a];
                xt[r] += x[a][r] * dT[a];
            }
        const double nA[3] = {xs[1] * xt[2] - xs[2] * xt[1], xs[2] * xt[0] - xs[0] * xt[2],
                              xs[0] * xt[1] - xs[1] * xt[0]};
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int r = 0; r < 3; ++r) fa[a][r] -= p * N[a] * nA[r];
    }
    if (contrib) {  // deterministic mode: gathered per node in face order
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int r = 0; r < 3; ++r) contrib[12 * (int64_t)f + 3 * a + r] = fa[a][r];
        return;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 3; ++r) atomicAdd(F + 3 * nd[a] + r, fa[a][r]);
}

// Penalty tethers, one thread per tether; the nodes are distinct, so the
// read-modify-write of out needs no atomic (the force kernels before it on the
// stream have finished).  V == null: d = X_a - Y_t, else d = V_a.
__global__ void __launch_bounds__(256)
k_tether(const double* __restrict__ X, const double* __restrict__ V,
         const int32_t* __restrict__ node, const double* __restrict__ Y,
         const double* __restrict__ K, int nt, double* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const int64_t a = node[t];
    double d[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) d[r] = V ? V[3 * a + r] : X[3 * a + r] - Y[3 * (int64_t)t + r];
    const double* k = K + 6 * (int64_t)t;   // xx, yy, zz, xy, xz, yz
    out[3 * a] -= k[0] * d[0] + k[3] * d[1] + k[4] * d[2];
    out[3 * a + 1] -= k[3] * d[0] + k[1] * d[1] + k[5] * d[2];
    out[3 * a + 2] -= k[4] * d[0] + k[5] * d[1] + k[2] * d[2];
}

__global__ void k_clear_numeric(MGState* st) {
    if (threadIdx.x == 0) st->numeric = 0;
}

}  // namespace

hipib_status launch_tethers(hipib_ctx* ctx, const double* X, const double* V, double* out) {
    if (ctx->nt == 0) return HIPIB_OK;
    k_tether<<<(ctx->nt + 255) / 256, 256, 0, ctx->stream>>>(X, V, ctx->tether_node, ctx->tether_Y,
                                                             ctx->tether_K, ctx->nt, out);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

namespace {
// one element kernel per element type
template <typename S>
hipib_status launch_elements(hipib_ctx* ctx, const double* X, double* F, double* contrib) {
    const dim3 grid((ctx->ne + 127) / 128);
    if (ctx->cfg.precision == HIPIB_MIXED)
        return launch_k(ctx, HIPIB_TIMER_FE_FORCE, 0.0, k_fe_force<float, S, true>, grid, dim3(128), 0, X,
                        ctx->Xref, ctx->conn, ctx->fibre, ctx->sheet, ctx->mat_id, ctx->mats, ctx->active_ta,
                        ctx->ne, F, ctx->st, contrib);
    return launch_k(ctx, HIPIB_TIMER_FE_FORCE, 0.0, k_fe_force<double, S>, grid, dim3(128), 0, X, ctx->Xref,
                    ctx->conn, ctx->fibre, ctx->sheet, ctx->mat_id, ctx->mats, ctx->active_ta, ctx->ne, F,
                    ctx->st, contrib);
}

hipib_status launch_element_forces(hipib_ctx* ctx, const double* X, double* F, double* contrib) {
    if (ctx->npe == 4) return launch_elements<Tet4>(ctx, X, F, contrib);
    if (ctx->npe == 10) return launch_elements<Tet10>(ctx, X, F, contrib);
    return launch_elements<Hex8>(ctx, X, F, contrib);
}
}  // namespace

hipib_status launch_fe_force(hipib_ctx* ctx, const double* X, double pressure, double* F) {
    k_clear_numeric<<<1, 64, 0, ctx->stream>>>(ctx->st);
    const bool det = ctx->cfg.deterministic != 0;
    if (det) {
        if (ctx->ne > 0) {
            HIPIB_TRY(launch_element_forces(ctx, X, F, ctx->det_contrib));
            HIPIB_TRY(det_gather_nodes(ctx, false, false, F));
        } else {
            HIPIB_TRY(launch_zero(ctx, F, 3 * (int64_t)ctx->nn));
        }
        if (ctx->nf > 0 && pressure != 0.0) {
            k_pressure_load<<<(ctx->nf + 255) / 256, 256, 0, ctx->stream>>>(
                X, ctx->faces, ctx->nf, pressure, F, ctx->det_face_contrib);
            HIPIB_HIP(hipGetLastError());
            HIPIB_TRY(det_gather_nodes(ctx, true, true, F));
        }
        return launch_tethers(ctx, X, nullptr, F);
    }
    HIPIB_TRY(launch_zero(ctx, F, 3 * (int64_t)ctx->nn));
    if (ctx->ne > 0) HIPIB_TRY(launch_element_forces(ctx, X, F, nullptr));
    if (ctx->nf > 0 && pressure != 0.0) {
        k_pressure_load<<<(ctx->nf + 255) / 256, 256, 0, ctx->stream>>>(X, ctx->faces, ctx->nf,
                                                                         pressure, F, nullptr);
        HIPIB_HIP(hipGetLastError());
    }
    return launch_tethers(ctx, X, nullptr, F);
}

}  // namespace hipib
