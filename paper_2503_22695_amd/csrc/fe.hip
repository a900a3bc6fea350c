// Matrix-free nodal forces on trilinear hexahedra ("Eulerian-Lagrangian
// coupling operators": F_i = -sum_q P(X_q) : grad N_i(X_q) w_q) and the
// uniform cavity pressure on quads (the left-ventricle model's endocardial
// load), as a follower load on the current configuration.
//
// One thread per element.  With Jr = dX/dxi and Jx = dx/dxi at a Gauss point,
// F = Jx Jr^{-1}, grad_X N_a = Jr^{-T} grad_xi N_a and
//   sum_c P[r][c] grad_X N_a[c] w = sum_s Q[r][s] dN_a/dxi_s,  Q = w P Jr^{-T},
// so the shape-function gradients in X are never formed: per Gauss point the
// element does two 8-node gathers of 3x3 Jacobians, one 3x3 inverse, the law,
// one 3x3 product and a 24-entry update, all in registers.  Element rule:
// 2x2x2 Gauss points at +-1/sqrt(3), unit weights.  Node accumulation uses
// hardware FP64 atomics.
#include "internal.h"

namespace hipib {
namespace {

__device__ __forceinline__ double det3(const double* A) {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

__device__ __forceinline__ void cof3(const double* A, double* C) {
    C[0] = A[4] * A[8] - A[5] * A[7];
    C[1] = A[5] * A[6] - A[3] * A[8];
    C[2] = A[3] * A[7] - A[4] * A[6];
    C[3] = A[2] * A[7] - A[1] * A[8];
    C[4] = A[0] * A[8] - A[2] * A[6];
    C[5] = A[1] * A[6] - A[0] * A[7];
    C[6] = A[1] * A[5] - A[2] * A[4];
    C[7] = A[2] * A[3] - A[0] * A[5];
    C[8] = A[0] * A[4] - A[1] * A[3];
}

// First Piola-Kirchhoff stress ("Constitutive laws"):
//   neo-Hookean (mu_s, kappa):  mu_s J^{-2/3}(F - I1/3 F^{-T}) + kappa ln J F^{-T}
//   Holzapfel-Ogden (a, b, a_f, b_f, kappa):
//     a e^{b(I1bar-3)} J^{-2/3}(F - I1/3 F^{-T})
//     + 2 a_f (I4f*-1) e^{b_f (I4f*-1)^2} (F e_f) (x) e_f + kappa ln J F^{-T}
// Returns false when J <= 0.
__device__ __forceinline__ bool pk1(int model, const double* par, const double* Fm,
                                    const double* ef, double* P) {
    const double J = det3(Fm);
    if (!(J > 0.0)) return false;
    double cof[9];
    cof3(Fm, cof);
    const double invJ = 1.0 / J;
    double I1 = 0.0;
#pragma unroll
    for (int r = 0; r < 9; ++r) I1 += Fm[r] * Fm[r];
    const double cb = cbrt(J);
    const double Jm23 = 1.0 / (cb * cb);
    const double lnJ = log(J);
    double iso, kappa, fib = 0.0;
    double Fe[3] = {0.0, 0.0, 0.0};
    if (model == HIPIB_NEO_HOOKEAN) {
        iso = par[0];
        kappa = par[1];
    } else {
        kappa = par[4];
        iso = par[0] * exp(par[1] * (Jm23 * I1 - 3.0));
#pragma unroll
        for (int r = 0; r < 3; ++r) Fe[r] = Fm[3 * r] * ef[0] + Fm[3 * r + 1] * ef[1] + Fm[3 * r + 2] * ef[2];
        const double I4 = Fe[0] * Fe[0] + Fe[1] * Fe[1] + Fe[2] * Fe[2];
        if (I4 > 1.0) fib = 2.0 * par[2] * (I4 - 1.0) * exp(par[3] * (I4 - 1.0) * (I4 - 1.0));
    }
    const double a = iso * Jm23, third = I1 / 3.0, vol = kappa * lnJ;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double FiT = cof[3 * r + c] * invJ;
            P[3 * r + c] = a * (Fm[3 * r + c] - third * FiT) + fib * Fe[r] * ef[c] + vol * FiT;
        }
    return true;
}

__global__ void __launch_bounds__(128)
k_fe_force(const double* __restrict__ X, const double* __restrict__ Xref,
           const int32_t* __restrict__ conn, const double* __restrict__ fibre,
           const int32_t* __restrict__ mat_id, MatTable mats, int ne, double* __restrict__ F,
           MGState* st) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    int nd[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) nd[a] = conn[8 * e + a];
    double xr[8][3], xc[8][3], fe[8][3];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            xr[a][r] = Xref[3 * nd[a] + r];
            xc[a][r] = X[3 * nd[a] + r];
            fe[a][r] = 0.0;
        }
    const int m = mat_id[e];
    const int model = mats.model[m];
    double par[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) par[t] = mats.p[m][t];
    const double ef[3] = {fibre[3 * e], fibre[3 * e + 1], fibre[3 * e + 2]};
    const double gp = 0.57735026918962576451;  // 1/sqrt(3)
    bool bad = false;
    for (int g = 0; g < 8; ++g) {
        const double xi[3] = {(g & 1) ? gp : -gp, (g & 2) ? gp : -gp, (g & 4) ? gp : -gp};
        double dN[8][3];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const double s0 = (a & 1) ? 1.0 : -1.0, s1 = (a & 2) ? 1.0 : -1.0, s2 = (a & 4) ? 1.0 : -1.0;
            const double f0 = 1.0 + s0 * xi[0], f1 = 1.0 + s1 * xi[1], f2 = 1.0 + s2 * xi[2];
            dN[a][0] = s0 * f1 * f2 * 0.125;
            dN[a][1] = f0 * s1 * f2 * 0.125;
            dN[a][2] = f0 * f1 * s2 * 0.125;
        }
        double Jr[9], Jx[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) Jr[t] = Jx[t] = 0.0;
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Jr[3 * r + c] += xr[a][r] * dN[a][c];
                    Jx[3 * r + c] += xc[a][r] * dN[a][c];
                }
        const double w = det3(Jr);
        if (!(w > 0.0)) { bad = true; continue; }
        double cr[9], Jri[9];
        cof3(Jr, cr);
        const double iw = 1.0 / w;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) Jri[3 * r + c] = cr[3 * c + r] * iw;   // Jr^{-1}
        double Fm[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                Fm[3 * r + c] = Jx[3 * r] * Jri[c] + Jx[3 * r + 1] * Jri[3 + c] + Jx[3 * r + 2] * Jri[6 + c];
        double P[9];
        if (!pk1(model, par, Fm, ef, P)) { bad = true; continue; }
        double Q[9];   // w P Jr^{-T}
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int s = 0; s < 3; ++s)
                Q[3 * r + s] = w * (P[3 * r] * Jri[3 * s] + P[3 * r + 1] * Jri[3 * s + 1] +
                                    P[3 * r + 2] * Jri[3 * s + 2]);
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int r = 0; r < 3; ++r)
                fe[a][r] -= Q[3 * r] * dN[a][0] + Q[3 * r + 1] * dN[a][1] + Q[3 * r + 2] * dN[a][2];
    }
    if (bad) atomicOr(&st->numeric, 1);
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int r = 0; r < 3; ++r) atomicAdd(F + 3 * nd[a] + r, fe[a][r]);
}

// F_a -= p * sum over 2x2 Gauss points of N_a (dx/dxi x dx/deta)
__global__ void __launch_bounds__(256)
k_pressure_load(const double* __restrict__ X, const int32_t* __restrict__ faces, int nf, double p,
                double* __restrict__ F) {
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
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 3; ++r) atomicAdd(F + 3 * nd[a] + r, fa[a][r]);
}

__global__ void k_clear_numeric(MGState* st) {
    if (threadIdx.x == 0) st->numeric = 0;
}

}  // namespace

hipib_status launch_fe_force(hipib_ctx* ctx, const double* X, double pressure, double* F) {
    k_clear_numeric<<<1, 64, 0, ctx->stream>>>(ctx->st);
    HIPIB_TRY(launch_zero(ctx, F, 3 * (int64_t)ctx->nn));
    if (ctx->ne > 0) {
        k_fe_force<<<(ctx->ne + 127) / 128, 128, 0, ctx->stream>>>(
            X, ctx->Xref, ctx->conn, ctx->fibre, ctx->mat_id, ctx->mats, ctx->ne, F, ctx->st);
        HIPIB_HIP(hipGetLastError());
    }
    if (ctx->nf > 0 && pressure != 0.0) {
        k_pressure_load<<<(ctx->nf + 255) / 256, 256, 0, ctx->stream>>>(X, ctx->faces, ctx->nf,
                                                                         pressure, F);
        HIPIB_HIP(hipGetLastError());
    }
    return HIPIB_OK;
}

}  // namespace hipib
