// Discrete adjoint of one immersed-boundary step (reverse mode of the step in
// api.hip), for gradients with respect to the node positions and the
// Holzapfel-Ogden parameters.  lam denotes dL/d(array entry).  With
//   X^{n+1} = X^n + dt J(X^n) u^{n+1},  u^{n+1} = P H^{-1} g,
//   g = (rho/dt) u^n - rho C(u^n) + S(X^n) F(X^n; theta),
// one reverse step is
//   lam_tot = lam_u' + dt J^T lam_X'          (J^T = h^3 S: a spread)
//   lam_X   = lam_X' + dt [d_X J(X) u^{n+1}]^T lam_X'
//   lam_*   = P lam_tot                        (P is symmetric: the forward
//                                               projection, one Poisson solve)
//   lam_g   = H^{-1} lam_*                     (H symmetric: three Helmholtz solves)
//   lam_u^n = (rho/dt) lam_g - rho C'(u^n)^T lam_g
//   lam_F   = S^T lam_g = J(X^n) lam_g / h^3   (an interpolation)
//   lam_X  += [d_X S(X) F]^T lam_g + (dF/dX) lam_F + [dF_p/dX]^T lam_F
//   dtheta += (dF/dtheta)^T lam_F
// (dF_el/dX = -Hess E is symmetric, so its transpose product is the
// directional derivative of the force: the strain-energy Hessian-vector
// product.)  The multigrid solves are treated as exact inverses.
#include "delta.h"
#include "solid.h"

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

__device__ __forceinline__ int wrapn(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// out = (rho/dt) lam - rho C'(u)^T lam, gathered per face:
//   [C'^T lam]_d[c] = (gA[c] + gA[c - e_d]) / 2
//                   + sum_{e != d} (G_de[c] b_de[c] + G_de[c + e_e] b_de[c + e_e]) / 2
// with the cell-centre normal flux adjoint gA[m] = (u_d[m] + u_d[m+e_d])
// (lam_d[m] - lam_d[m+e_d]) / h, the edge flux adjoint (an edge flux is shared by
// components d and e) G_de[c] = (lam_d[c-e_e] - lam_d[c] + lam_e[c-e_d] - lam_e[c]) / h
// and the edge average b_de[c] = (u_e[c-e_d] + u_e[c]) / 2.
__global__ void __launch_bounds__(TX * TY)
k_conv_vjp_rhs(const double* __restrict__ u, const double* __restrict__ lam, double* __restrict__ out,
               Grid3 G, double rho_dt, double rho, double inv_h, int convection) {
    const int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y, k = blockIdx.z;
    if (i >= G.n || j >= G.n) return;
    const int n = G.n;
    const int p[3] = {i, j, k};
    for (int d = 0; d < 3; ++d) {
        const double* ud = u + d * G.n3;
        const double* ld = lam + d * G.n3;
        const int64_t c = G.at(i, j, k);
        double ct = 0.0;
        if (convection) {
            int q[3] = {i, j, k};
            q[d] = wrapn(p[d] + 1, n);
            const int64_t cpd = G.at(q[0], q[1], q[2]);
            q[d] = wrapn(p[d] - 1, n);
            const int64_t cmd = G.at(q[0], q[1], q[2]);
            const double gA0 = (ud[c] + ud[cpd]) * (ld[c] - ld[cpd]) * inv_h;
            const double gA1 = (ud[cmd] + ud[c]) * (ld[cmd] - ld[c]) * inv_h;
            ct = 0.5 * (gA0 + gA1);
            for (int e = 0; e < 3; ++e) {
                if (e == d) continue;
                const double* ue = u + e * G.n3;
                const double* le = lam + e * G.n3;
                // edges at c and c + e_e
                for (int s = 0; s < 2; ++s) {
                    int cc[3] = {i, j, k};
                    if (s) cc[e] = wrapn(p[e] + 1, n);
                    int me[3] = {cc[0], cc[1], cc[2]};
                    me[e] = wrapn(cc[e] - 1, n);
                    int md[3] = {cc[0], cc[1], cc[2]};
                    md[d] = wrapn(cc[d] - 1, n);
                    const int64_t ic = G.at(cc[0], cc[1], cc[2]);
                    const int64_t ime = G.at(me[0], me[1], me[2]);
                    const int64_t imd = G.at(md[0], md[1], md[2]);
                    const double Gde = (ld[ime] - ld[ic] + le[imd] - le[ic]) * inv_h;
                    const double bde = 0.5 * (ue[imd] + ue[ic]);
                    ct += 0.5 * Gde * bde;
                }
            }
        }
        out[d * G.n3 + c] = rho_dt * ld[c] - rho * ct;
    }
}

// lamX[q][e] += scale * sum_d coef[q][d] * sum_stencil field_d[idx] d/dr_e (w_x w_y w_z)
// (the position derivative of spreading (field = lam_f, coef = F) and of
// interpolation (field = u, coef = lam_U)); one thread per node in tile order
template <typename TW>
__global__ void __launch_bounds__(256)
k_vjp_X(const double* __restrict__ X, const double* __restrict__ field,
        const double* __restrict__ coef, double* __restrict__ lamX, double scale, int nn, int n,
        int64_t n3, double inv_h, const int32_t* __restrict__ perm) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nn) return;
    const int q = perm ? perm[t] : t;
    const double xs[3] = {X[3 * q] * inv_h, X[3 * q + 1] * inv_h, X[3 * q + 2] * inv_h};
    double g[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < 3; ++d) {
        TW w[3][4], dw[3][4];
        int i0[3];
        for (int e = 0; e < 3; ++e)
            i0[e] = peskin_weights<TW, true>(xs[e] - (e == d ? 0.0 : 0.5), n, w[e], dw[e]);
        const double* fd = field + d * n3;
        TW gx = TW(0), gy = TW(0), gz = TW(0);
        for (int c = 0; c < 4; ++c) {
            const int kk = step_wrap(i0[2] + c, n);
            for (int b = 0; b < 4; ++b) {
                const int jj = step_wrap(i0[1] + b, n);
                const int64_t row = (int64_t)n * ((int64_t)jj + (int64_t)n * kk);
                const TW wyz = w[1][b] * w[2][c], dyz = dw[1][b] * w[2][c], ydz = w[1][b] * dw[2][c];
                for (int a = 0; a < 4; ++a) {
                    const TW v = (TW)fd[row + step_wrap(i0[0] + a, n)];
                    gx += v * dw[0][a] * wyz;
                    gy += v * w[0][a] * dyz;
                    gz += v * w[0][a] * ydz;
                }
            }
        }
        const double cq = coef[3 * q + d];
        g[0] += cq * (double)gx;
        g[1] += cq * (double)gy;
        g[2] += cq * (double)gz;
    }
    for (int e = 0; e < 3; ++e) lamX[3 * q + e] += scale * g[e];
}

// out += (dF/dx) V per element: dF = Jv Jr^{-1}, dP = tangent of P along dF,
// contribution -w dP grad N_a = -sum_s (w dP Jr^{-T})[r][s] dN_a/dxi_s
template <typename S>
__global__ void __launch_bounds__(128)
k_fe_hvp(const double* __restrict__ X, const double* __restrict__ Xref,
         const int32_t* __restrict__ conn, const double* __restrict__ fibre,
         const double* __restrict__ sheet, const int32_t* __restrict__ mat_id, MatTable mats,
         double Ta, int ne, const double* __restrict__ V, double* __restrict__ out, MGState* st,
         double* __restrict__ contrib) {
    constexpr int N = S::N;
    // 10-node elements re-read their node data at each point (from L1) instead of
    // holding it in registers, which would spill; the arithmetic is the same
    constexpr bool kHold = N <= 8;
    constexpr int NH = kHold ? N : 1;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    int nd[N];
    for (int a = 0; a < N; ++a) nd[a] = conn[N * (int64_t)e + a];
    double xr[NH][3], xc[NH][3], vv[NH][3], he[N][3];
    const double r0[3] = {Xref[3 * nd[0]], Xref[3 * nd[0] + 1], Xref[3 * nd[0] + 2]};
    const double c0[3] = {X[3 * nd[0]], X[3 * nd[0] + 1], X[3 * nd[0] + 2]};
    for (int a = 0; a < N; ++a)
        for (int r = 0; r < 3; ++r) {
            if constexpr (kHold) {
                xr[a][r] = Xref[3 * nd[a] + r] - r0[r];
                xc[a][r] = X[3 * nd[a] + r] - c0[r];
                vv[a][r] = V[3 * nd[a] + r];
            }
            he[a][r] = 0.0;
        }
    const int m = mat_id[e];
    const int model = mats.model[m];
    const double* par = mats.p[m];
    const double ef[3] = {fibre[3 * e], fibre[3 * e + 1], fibre[3 * e + 2]};
    const bool sh = mats.sheet[m] != 0;
    double es[3] = {0.0, 0.0, 0.0};
    if (sh) {
        es[0] = sheet[3 * e];
        es[1] = sheet[3 * e + 1];
        es[2] = sheet[3 * e + 2];
    }
    const double ta = model == HIPIB_HOLZAPFEL_OGDEN ? Ta : 0.0;
    bool bad = false;
    for (int g = 0; g < S::Q; ++g) {
        double dN[N][3];
        const double wq = elem_rule<S, double>(g, dN);
        double Jr[9], Jx[9], Jv[9];
        if constexpr (kHold) {
            gather_jac<N>(xr, dN, Jr);
            gather_jac<N>(xc, dN, Jx);
            gather_jac<N>(vv, dN, Jv);
        } else {
            for (int t = 0; t < 9; ++t) Jr[t] = Jx[t] = Jv[t] = 0.0;
            for (int a = 0; a < N; ++a)
                for (int r = 0; r < 3; ++r) {
                    const double dr = Xref[3 * nd[a] + r] - r0[r], dx = X[3 * nd[a] + r] - c0[r];
                    const double dv = V[3 * nd[a] + r];
                    for (int c = 0; c < 3; ++c) {
                        Jr[3 * r + c] += dr * dN[a][c];
                        Jx[3 * r + c] += dx * dN[a][c];
                        Jv[3 * r + c] += dv * dN[a][c];
                    }
                }
        }
        const double w = det3(Jr);
        if (!(w > 0.0)) { bad = true; continue; }
        double cr[9], Jri[9];
        cof3(Jr, cr);
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) Jri[3 * r + c] = cr[3 * c + r] / w;
        double Fm[9], dF[9], dP[9];
        matmul3(Jx, Jri, Fm);
        matmul3(Jv, Jri, dF);
        if (!pk1_tangent<double>(model, par, Fm, ef, es, sh, ta, dF, dP)) { bad = true; continue; }
        const double wg = w * wq;
        double Q[9];
        for (int r = 0; r < 3; ++r)
            for (int s = 0; s < 3; ++s)
                Q[3 * r + s] = wg * (dP[3 * r] * Jri[3 * s] + dP[3 * r + 1] * Jri[3 * s + 1] +
                                     dP[3 * r + 2] * Jri[3 * s + 2]);
        for (int a = 0; a < N; ++a)
            for (int r = 0; r < 3; ++r)
                he[a][r] -= Q[3 * r] * dN[a][0] + Q[3 * r + 1] * dN[a][1] + Q[3 * r + 2] * dN[a][2];
    }
    if (bad) atomicOr(&st->numeric, 1);
    if (contrib) {  // deterministic mode: gathered per node in element order
        for (int a = 0; a < N; ++a)
            for (int r = 0; r < 3; ++r) contrib[3 * (N * (int64_t)e + a) + r] = he[a][r];
        return;
    }
    for (int a = 0; a < N; ++a)
        for (int r = 0; r < 3; ++r) atomicAdd(out + 3 * nd[a] + r, he[a][r]);
}

// dtheta[m][k] += -sum_g w dP/dtheta_k : (sum_a lam_a (x) grad_X N_a) for the
// Holzapfel-Ogden parameters (a, b, a_f, b_f):
//   dP/da   = e^{b(I1bar-3)} J^{-2/3}(F - I1/3 F^{-T}),   dP/db = a (I1bar-3) dP/da,
//   dP/da_f = 2 (I4-1) e^{b_f (I4-1)^2} (F e)(x)e,        dP/db_f = a_f (I4-1)^2 dP/da_f
// Per-block sums in LDS, then one global atomic per block and entry; in
// deterministic mode (part != null) the per-element terms go to part[e][4]
// for a fixed-order reduction.
template <typename S>
__global__ void __launch_bounds__(128)
k_fe_param_vjp(const double* __restrict__ X, const double* __restrict__ Xref,
               const int32_t* __restrict__ conn, const double* __restrict__ fibre,
               const int32_t* __restrict__ mat_id, MatTable mats, int ne,
               const double* __restrict__ lam, double* __restrict__ dtheta,
               double* __restrict__ part) {
    __shared__ double acc[HIPIB_MAX_MATERIALS * 4];
    for (int t = threadIdx.x; t < HIPIB_MAX_MATERIALS * 4; t += blockDim.x) acc[t] = 0.0;
    __syncthreads();
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < ne && part)
        for (int k = 0; k < 4; ++k) part[4 * (int64_t)e + k] = 0.0;
    if (e < ne) {
        const int m = mat_id[e];
        if (mats.model[m] == HIPIB_HOLZAPFEL_OGDEN) {
            constexpr int N = S::N;
            int nd[N];
            for (int a = 0; a < N; ++a) nd[a] = conn[N * (int64_t)e + a];
            double xr[N][3], xc[N][3], ll[N][3];
            for (int a = 0; a < N; ++a)
                for (int r = 0; r < 3; ++r) {
                    xr[a][r] = Xref[3 * nd[a] + r] - Xref[3 * nd[0] + r];
                    xc[a][r] = X[3 * nd[a] + r] - X[3 * nd[0] + r];
                    ll[a][r] = lam[3 * nd[a] + r];
                }
            const double* par = mats.p[m];
            const double ef[3] = {fibre[3 * e], fibre[3 * e + 1], fibre[3 * e + 2]};
            double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
            for (int g = 0; g < S::Q; ++g) {
                double dN[N][3];
                const double wq = elem_rule<S, double>(g, dN);
                double Jr[9], Jx[9], Jl[9];
                gather_jac<N>(xr, dN, Jr);
                gather_jac<N>(xc, dN, Jx);
                gather_jac<N>(ll, dN, Jl);
                const double w0 = det3(Jr);
                if (!(w0 > 0.0)) continue;
                const double w = w0 * wq;
                double cr[9], Jri[9];
                cof3(Jr, cr);
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) Jri[3 * r + c] = cr[3 * c + r] / w0;
                double Fm[9], Gl[9];
                matmul3(Jx, Jri, Fm);
                matmul3(Jl, Jri, Gl);
                const double J = det3(Fm);
                if (!(J > 0.0)) continue;
                double cf[9];
                cof3(Fm, cf);
                double I1 = 0.0;
                for (int r = 0; r < 9; ++r) I1 += Fm[r] * Fm[r];
                const double cb = cbrt(J), Jm23 = 1.0 / (cb * cb);
                const double E1 = exp(par[1] * (Jm23 * I1 - 3.0));
                double Fe[3];
                for (int r = 0; r < 3; ++r) Fe[r] = Fm[3 * r] * ef[0] + Fm[3 * r + 1] * ef[1] + Fm[3 * r + 2] * ef[2];
                double Miso = 0.0, Mfib = 0.0;
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) {
                        const int o = 3 * r + c;
                        Miso += Jm23 * (Fm[o] - I1 / 3.0 * cf[o] / J) * Gl[o];
                        Mfib += Fe[r] * ef[c] * Gl[o];
                    }
                d0 -= w * E1 * Miso;
                d1 -= w * par[0] * (Jm23 * I1 - 3.0) * E1 * Miso;
                const double I4 = Fe[0] * Fe[0] + Fe[1] * Fe[1] + Fe[2] * Fe[2];
                if (I4 > 1.0) {
                    const double q = I4 - 1.0, Ef = exp(par[3] * q * q);
                    d2 -= w * 2.0 * q * Ef * Mfib;
                    d3 -= w * 2.0 * par[2] * q * q * q * Ef * Mfib;
                }
            }
            if (part) {
                part[4 * (int64_t)e + 0] = d0;
                part[4 * (int64_t)e + 1] = d1;
                part[4 * (int64_t)e + 2] = d2;
                part[4 * (int64_t)e + 3] = d3;
            } else {
                atomicAdd(&acc[4 * m + 0], d0);
                atomicAdd(&acc[4 * m + 1], d1);
                atomicAdd(&acc[4 * m + 2], d2);
                atomicAdd(&acc[4 * m + 3], d3);
            }
        }
    }
    __syncthreads();
    if (part) return;
    for (int t = threadIdx.x; t < HIPIB_MAX_MATERIALS * 4; t += blockDim.x)
        if (acc[t] != 0.0) atomicAdd(dtheta + t, acc[t]);
}

// lamX_b += -p sum_g [dN_b/dxi (x_eta x mu) + dN_b/deta (mu x x_xi)], mu = sum_a N_a lamF_a
__global__ void __launch_bounds__(256)
k_pressure_vjp(const double* __restrict__ X, const int32_t* __restrict__ faces, int nf, double p,
               const double* __restrict__ lamF, double* __restrict__ lamX, double* __restrict__ contrib) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    int nd[4];
    double x[4][3], l[4][3], out[4][3];
    for (int a = 0; a < 4; ++a) {
        nd[a] = faces[4 * f + a];
        for (int r = 0; r < 3; ++r) {
            x[a][r] = X[3 * nd[a] + r];
            l[a][r] = lamF[3 * nd[a] + r];
            out[a][r] = 0.0;
        }
    }
    const double gp = 0.57735026918962576451;
    for (int g = 0; g < 4; ++g) {
        const double s = (g & 1) ? gp : -gp, t = (g & 2) ? gp : -gp;
        double N[4], dS[4], dT[4];
        for (int a = 0; a < 4; ++a) {
            const double sa = (a & 1) ? 1.0 : -1.0, ta = (a & 2) ? 1.0 : -1.0;
            N[a] = (1.0 + sa * s) * (1.0 + ta * t) * 0.25;
            dS[a] = sa * (1.0 + ta * t) * 0.25;
            dT[a] = (1.0 + sa * s) * ta * 0.25;
        }
        double xs[3] = {0, 0, 0}, xt[3] = {0, 0, 0}, mu[3] = {0, 0, 0};
        for (int a = 0; a < 4; ++a)
            for (int r = 0; r < 3; ++r) {
                xs[r] += x[a][r] * dS[a];
                xt[r] += x[a][r] * dT[a];
                mu[r] += N[a] * l[a][r];
            }
        const double A[3] = {xt[1] * mu[2] - xt[2] * mu[1], xt[2] * mu[0] - xt[0] * mu[2],
                             xt[0] * mu[1] - xt[1] * mu[0]};
        const double B[3] = {mu[1] * xs[2] - mu[2] * xs[1], mu[2] * xs[0] - mu[0] * xs[2],
                             mu[0] * xs[1] - mu[1] * xs[0]};
        for (int b = 0; b < 4; ++b)
            for (int r = 0; r < 3; ++r) out[b][r] -= p * (dS[b] * A[r] + dT[b] * B[r]);
    }
    if (contrib) {  // deterministic mode: gathered per node in face order
        for (int a = 0; a < 4; ++a)
            for (int r = 0; r < 3; ++r) contrib[12 * (int64_t)f + 3 * a + r] = out[a][r];
        return;
    }
    for (int a = 0; a < 4; ++a)
        for (int r = 0; r < 3; ++r) atomicAdd(lamX + 3 * nd[a] + r, out[a][r]);
}

__global__ void k_axpby(double* y, const double* x, double a, double b,
                        int64_t count) {
    // y = a x + b y   (b = 0: y = a x, reading y not needed)
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x)
        y[t] = b == 0.0 ? a * x[t] : a * x[t] + b * y[t];
}

unsigned blocks_for(int64_t count) {
    int64_t b = (count + 255) / 256;
    if (b > 4096) b = 4096;
    return (unsigned)(b < 1 ? 1 : b);
}

hipib_status axpby(hipib_ctx* ctx, double* y, const double* x, double a, double b, int64_t count) {
    if (count <= 0) return HIPIB_OK;
    k_axpby<<<blocks_for(count), 256, 0, ctx->stream>>>(y, x, a, b, count);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

hipib_status vjp_X(hipib_ctx* ctx, const double* X, const double* field, const double* coef,
                   double* lamX, double scale) {
    if (ctx->nn == 0) return HIPIB_OK;
    const unsigned nb = (unsigned)((ctx->nn + 255) / 256);
    if (ctx->cfg.precision == HIPIB_MIXED)
        k_vjp_X<float><<<nb, 256, 0, ctx->stream>>>(X, field, coef, lamX, scale, ctx->nn, ctx->n,
                                                    ctx->n3, 1.0 / ctx->h, ctx->perm);
    else
        k_vjp_X<double><<<nb, 256, 0, ctx->stream>>>(X, field, coef, lamX, scale, ctx->nn, ctx->n,
                                                     ctx->n3, 1.0 / ctx->h, ctx->perm);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

hipib_status ensure_adjoint_scratch(hipib_ctx* ctx) {
    if (ctx->adj_ready_nn == ctx->nn && ctx->adj_tot) return HIPIB_OK;
    HIPIB_HIP(hipStreamSynchronize(ctx->stream));
    (void)hipFree(ctx->adj_sX);
    (void)hipFree(ctx->adj_lamF);
    ctx->adj_sX = ctx->adj_lamF = nullptr;
    auto alloc = [&](double** p, size_t count) -> hipib_status {
        if (*p) return HIPIB_OK;
        if (hipMalloc(reinterpret_cast<void**>(p), (count ? count : 1) * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return fail(HIPIB_E_NOMEM, "adjoint workspace allocation failed");
        }
        return HIPIB_OK;
    };
    const bool fresh = ctx->adj_lg == nullptr;
    HIPIB_TRY(alloc(&ctx->adj_tot, 3 * (size_t)ctx->n3));
    HIPIB_TRY(alloc(&ctx->adj_lg, 3 * (size_t)ctx->n3));
    HIPIB_TRY(alloc(&ctx->adj_p, (size_t)ctx->n3));
    if (fresh) {  // the adjoint solves' first initial guesses
        HIPIB_TRY(launch_zero(ctx, ctx->adj_lg, 3 * ctx->n3));
        HIPIB_TRY(launch_zero(ctx, ctx->adj_p, ctx->n3));
    }
    HIPIB_TRY(alloc(&ctx->adj_sX, 3 * (size_t)ctx->nn));
    HIPIB_TRY(alloc(&ctx->adj_lamF, 3 * (size_t)ctx->nn));
    ctx->adj_ready_nn = ctx->nn;
    return HIPIB_OK;
}

// element-derivative kernels, one instantiation per element type
template <typename S>
hipib_status hvp_elements_t(hipib_ctx* ctx, const double* X, const double* V, double* out,
                            double* contrib) {
    k_fe_hvp<S><<<(ctx->ne + 127) / 128, 128, 0, ctx->stream>>>(
        X, ctx->Xref, ctx->conn, ctx->fibre, ctx->sheet, ctx->mat_id, ctx->mats, ctx->active_ta,
        ctx->ne, V, out, ctx->st, contrib);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

hipib_status hvp_elements(hipib_ctx* ctx, const double* X, const double* V, double* out,
                          double* contrib) {
    if (ctx->npe == 4) return hvp_elements_t<Tet4>(ctx, X, V, out, contrib);
    if (ctx->npe == 10) return hvp_elements_t<Tet10>(ctx, X, V, out, contrib);
    return hvp_elements_t<Hex8>(ctx, X, V, out, contrib);
}

template <typename S>
hipib_status param_vjp_elements_t(hipib_ctx* ctx, const double* X, const double* lamF,
                                  double* dtheta, double* part) {
    k_fe_param_vjp<S><<<(ctx->ne + 127) / 128, 128, 0, ctx->stream>>>(
        X, ctx->Xref, ctx->conn, ctx->fibre, ctx->mat_id, ctx->mats, ctx->ne, lamF, dtheta, part);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

hipib_status param_vjp_elements(hipib_ctx* ctx, const double* X, const double* lamF,
                                double* dtheta, double* part) {
    if (ctx->npe == 4) return param_vjp_elements_t<Tet4>(ctx, X, lamF, dtheta, part);
    if (ctx->npe == 10) return param_vjp_elements_t<Tet10>(ctx, X, lamF, dtheta, part);
    return param_vjp_elements_t<Hex8>(ctx, X, lamF, dtheta, part);
}

}  // namespace

hipib_status adjoint_step(hipib_ctx* ctx, const double* u_n, const double* X_n, const double* u_np1,
                          double pressure, double* lam_u, double* lam_X, double* dtheta) {
    HIPIB_TRY(ensure_adjoint_scratch(ctx));
    const double h = ctx->h, h3 = h * h * h, rho = ctx->cfg.rho, dt = ctx->cfg.dt;
    const int64_t nn3 = 3 * (int64_t)ctx->nn, g3 = 3 * ctx->n3;
    HIPIB_TRY(launch_bin(ctx, X_n));
    // X^{n+1} = X^n + dt J(X^n) u^{n+1}
    HIPIB_TRY(axpby(ctx, ctx->adj_sX, lam_X, dt * h3, 0.0, nn3));            // sX = dt h^3 lam_X'
    HIPIB_TRY(axpby(ctx, ctx->adj_tot, lam_u, 1.0, 0.0, g3));                // tot = lam_u'
    HIPIB_TRY(launch_spread(ctx, X_n, ctx->adj_sX, ctx->adj_tot));          // tot += S sX
    HIPIB_TRY(vjp_X(ctx, X_n, u_np1, ctx->adj_sX, lam_X, 1.0 / (h * h3)));  // interpolation term
    // u^{n+1} = P u*: lam_* = P lam_tot
    HIPIB_TRY(launch_divergence_rhs(ctx, ctx->adj_tot, ctx->bp));
    HIPIB_TRY(mg_remove_mean(ctx, ctx->bp, 0));
    // warm start: the previous reverse step's adjoint pressure (zero on the first call)
    HIPIB_TRY(mg_solve(ctx, HIPIB_OP_POISSON, 1, ctx->bp, ctx->adj_p, nullptr, nullptr));
    HIPIB_TRY(launch_project(ctx, ctx->adj_tot, ctx->adj_p));
    // u* = H^{-1} g: lam_g = H^{-1} lam_*  (warm start: the previous call's lam_g)
    HIPIB_TRY(mg_solve(ctx, HIPIB_OP_HELMHOLTZ, 3, ctx->adj_tot, ctx->adj_lg, nullptr, nullptr));
    // g = (rho/dt) u^n - rho C(u^n) + S F
    {
        const int n = ctx->n;
        const dim3 grid((n + TX - 1) / TX, (n + TY - 1) / TY, n);
        k_conv_vjp_rhs<<<grid, dim3(TX, TY), 0, ctx->stream>>>(u_n, ctx->adj_lg, lam_u,
                                                               Grid3{n, ctx->n3}, rho / dt, rho,
                                                               1.0 / h, ctx->cfg.convection);
        HIPIB_HIP(hipGetLastError());
    }
    if (ctx->nn > 0) {
        HIPIB_TRY(launch_interpolate(ctx, X_n, ctx->adj_lg, ctx->adj_lamF, nullptr, 0.0));
        HIPIB_TRY(axpby(ctx, ctx->adj_lamF, ctx->adj_lamF, 1.0 / h3, 0.0, nn3));   // lam_F = J lam_g / h^3
        HIPIB_TRY(launch_fe_force(ctx, X_n, pressure, ctx->F));                    // forward force
        HIPIB_TRY(vjp_X(ctx, X_n, ctx->adj_lg, ctx->F, lam_X, 1.0 / (h * h3)));    // spreading term
        HIPIB_TRY(adjoint_forces(ctx, X_n, pressure, ctx->adj_lamF, lam_X, dtheta));
    }
    HIPIB_TRY(sync_state(ctx));
    HIPIB_TRY(position_status(ctx));
    if (ctx->st_host->numeric)
        return fail(HIPIB_E_NUMERIC, "non-positive Jacobian at a Gauss point (inverted element)");
    return HIPIB_OK;
}

hipib_status adjoint_scratch(hipib_ctx* ctx) { return ensure_adjoint_scratch(ctx); }

// lam_X += (dF/dX)^T lamF, dtheta += (dF/dtheta)^T lamF for the nodal force F
// of the elements, the tethers and the pressure load
hipib_status adjoint_forces(hipib_ctx* ctx, const double* X_n, double pressure, const double* lamF,
                            double* lam_X, double* dtheta) {
    const bool det = ctx->cfg.deterministic != 0;
    if (ctx->ne > 0) {
        HIPIB_TRY(hvp_elements(ctx, X_n, lamF, lam_X, det ? ctx->det_contrib : nullptr));
        if (det) HIPIB_TRY(det_gather_nodes(ctx, false, true, lam_X));
        HIPIB_TRY(param_vjp_elements(ctx, X_n, lamF, dtheta, det ? ctx->det_param : nullptr));
        if (det) HIPIB_TRY(det_param_reduce(ctx, dtheta));
    }
    HIPIB_TRY(launch_tethers(ctx, X_n, lamF, lam_X));   // K symmetric: K^T lamF = K lamF
    if (ctx->nf > 0 && pressure != 0.0) {
        k_pressure_vjp<<<(ctx->nf + 255) / 256, 256, 0, ctx->stream>>>(
            X_n, ctx->faces, ctx->nf, pressure, lamF, lam_X, det ? ctx->det_face_contrib : nullptr);
        HIPIB_HIP(hipGetLastError());
        if (det) HIPIB_TRY(det_gather_nodes(ctx, true, true, lam_X));
    }
    return HIPIB_OK;
}

// out = a lam + b C'(u)^T lam
hipib_status launch_conv_vjp(hipib_ctx* ctx, const double* u, const double* lam, double* out,
                             double a, double b) {
    const int n = ctx->n;
    const dim3 grid((n + TX - 1) / TX, (n + TY - 1) / TY, n);
    k_conv_vjp_rhs<<<grid, dim3(TX, TY), 0, ctx->stream>>>(u, lam, out, Grid3{n, ctx->n3}, a, -b,
                                                           1.0 / ctx->h, 1);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

hipib_status launch_fe_hvp(hipib_ctx* ctx, const double* X, const double* V, double* out) {
    HIPIB_TRY(launch_zero(ctx, out, 3 * (int64_t)ctx->nn));
    if (ctx->ne > 0) {
        const bool det = ctx->cfg.deterministic != 0;
        HIPIB_TRY(hvp_elements(ctx, X, V, out, det ? ctx->det_contrib : nullptr));
        if (det) HIPIB_TRY(det_gather_nodes(ctx, false, true, out));
    }
    return launch_tethers(ctx, X, V, out);
}

hipib_status launch_fe_param_vjp(hipib_ctx* ctx, const double* X, const double* lamF, double* dtheta) {
    if (ctx->ne == 0) return HIPIB_OK;
    const bool det = ctx->cfg.deterministic != 0;
    HIPIB_TRY(param_vjp_elements(ctx, X, lamF, dtheta, det ? ctx->det_param : nullptr));
    if (det) HIPIB_TRY(det_param_reduce(ctx, dtheta));
    return HIPIB_OK;
}

hipib_status launch_vjp_X(hipib_ctx* ctx, const double* X, const double* field, const double* coef,
                          double* lamX, double scale) {
    HIPIB_TRY(launch_bin(ctx, X));
    return vjp_X(ctx, X, field, coef, lamX, scale);
}

}  // namespace hipib
