// Device helpers for the hexahedral solid: 3x3 algebra, the first
// Piola-Kirchhoff stress of the constitutive laws ("Constitutive laws") and its
// directional derivative.  Shared by the force kernels and their adjoints.
#pragma once

#include "internal.h"

namespace hipib {

template <typename T>
__device__ __forceinline__ T det3(const T* A) {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// cofactor matrix, cof(A) = det(A) A^{-T}
template <typename T>
__device__ __forceinline__ void cof3(const T* A, T* C) {
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

// First Piola-Kirchhoff stress:
//   neo-Hookean (mu_s, kappa):  mu_s J^{-2/3}(F - I1/3 F^{-T}) + kappa ln J F^{-T}
//   Holzapfel-Ogden (a, b, a_f, b_f, kappa, a_s, b_s, a_fs, b_fs):
//     a e^{b(I1bar-3)} J^{-2/3}(F - I1/3 F^{-T})
//     + 2 a_f (I4f*-1) e^{b_f (I4f*-1)^2} (F e_f) (x) e_f
//     + 2 a_s (I4s*-1) e^{b_s (I4s*-1)^2} (F e_s) (x) e_s          (sheet materials)
//     + a_fs I8 e^{b_fs I8^2} ((F e_f) (x) e_s + (F e_s) (x) e_f)   (sheet materials)
//     + T_a (1 + 4.9 (sqrt(I4f) - 1)) (F e_f) (x) e_f               (active stress)
//     + kappa ln J F^{-T}
// The fibre-sheet term is the derivative of a_fs/(2 b_fs)(e^{b_fs I8^2} - 1).
// `sheet` selects the sheet terms (es is then read); Ta = 0 drops the active term.
//   Psi_1 (G_T, G_L, E_L, kappa): G_T J^{-2/3}(F - I1/3 F^{-T})
//     + (2 (G_T - G_L) + (E_L + G_T - 4 G_L)/2 (I4f - 1)) (F e_f) (x) e_f
//     - (G_T - G_L) ((F e_f) (x) (C e_f) + (F C e_f) (x) e_f) + kappa ln J F^{-T}
//   Psi_2 (C_1, a_f, b_f, kappa): 2 C_1 J^{-2/3}(..) + 2 a_f (I4f*-1) e^{b_f (I4f*-1)^2} (F e_f)(x)e_f + ..
//   Psi_3 (C_10, C_01, a_f, b_f, kappa): 2 C_10 C_01 e^{C_01 (I1bar-3)} J^{-2/3}(..)
//     + 2 a_f (I4f-1) e^{b_f (I4f-1)^2} (F e_f)(x)e_f + ..   (plain I4f)
// Returns false when J <= 0.
template <typename T>
__device__ __forceinline__ bool pk1(int model, const T* par, const T* Fm, const T* ef, const T* es,
                                    bool sheet, T Ta, T* P) {
    const T J = det3(Fm);
    if (!(J > T(0))) return false;
    T cof[9];
    cof3(Fm, cof);
    const T invJ = T(1) / J;
    T I1 = T(0);
#pragma unroll
    for (int r = 0; r < 9; ++r) I1 += Fm[r] * Fm[r];
    const T cb = cbrt(J);
    const T Jm23 = T(1) / (cb * cb);
    const T lnJ = log(J);
    T iso, kappa, fib = T(0), sh = T(0), fs = T(0);
    T Fe[3] = {T(0), T(0), T(0)}, Fs[3] = {T(0), T(0), T(0)};
    if (model != HIPIB_NEO_HOOKEAN) {
#pragma unroll
        for (int r = 0; r < 3; ++r) Fe[r] = Fm[3 * r] * ef[0] + Fm[3 * r + 1] * ef[1] + Fm[3 * r + 2] * ef[2];
    }
    const T I4 = Fe[0] * Fe[0] + Fe[1] * Fe[1] + Fe[2] * Fe[2];
    if (model == HIPIB_NEO_HOOKEAN) {
        iso = par[0];
        kappa = par[1];
    } else if (model == HIPIB_STANDARD_REINFORCING) {
        iso = par[0];
        kappa = par[3];
        fib = T(2) * (par[0] - par[1]) + T(0.5) * (par[2] + par[0] - T(4) * par[1]) * (I4 - T(1));
    } else if (model == HIPIB_FIBRE_REINFORCED_1) {
        iso = T(2) * par[0];
        kappa = par[3];
        if (I4 > T(1)) fib = T(2) * par[1] * (I4 - T(1)) * exp(par[2] * (I4 - T(1)) * (I4 - T(1)));
    } else if (model == HIPIB_FIBRE_REINFORCED_2) {
        iso = T(2) * par[0] * par[1] * exp(par[1] * (Jm23 * I1 - T(3)));
        kappa = par[4];
        fib = T(2) * par[2] * (I4 - T(1)) * exp(par[3] * (I4 - T(1)) * (I4 - T(1)));
    } else {
        kappa = par[4];
        iso = par[0] * exp(par[1] * (Jm23 * I1 - T(3)));
        if (I4 > T(1)) fib = T(2) * par[2] * (I4 - T(1)) * exp(par[3] * (I4 - T(1)) * (I4 - T(1)));
        if (Ta != T(0)) fib += Ta * (T(1) + T(4.9) * (sqrt(I4) - T(1)));
        if (sheet) {
#pragma unroll
            for (int r = 0; r < 3; ++r) Fs[r] = Fm[3 * r] * es[0] + Fm[3 * r + 1] * es[1] + Fm[3 * r + 2] * es[2];
            const T I4s = Fs[0] * Fs[0] + Fs[1] * Fs[1] + Fs[2] * Fs[2];
            if (I4s > T(1)) sh = T(2) * par[5] * (I4s - T(1)) * exp(par[6] * (I4s - T(1)) * (I4s - T(1)));
            const T I8 = Fe[0] * Fs[0] + Fe[1] * Fs[1] + Fe[2] * Fs[2];
            fs = par[7] * I8 * exp(par[8] * I8 * I8);
        }
    }
    const T a = iso * Jm23, third = I1 / T(3), vol = kappa * lnJ;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T FiT = cof[3 * r + c] * invJ;
            T v = a * (Fm[3 * r + c] - third * FiT) + fib * Fe[r] * ef[c] + vol * FiT;
            if (sheet) v += sh * Fs[r] * es[c] + fs * (Fe[r] * es[c] + Fs[r] * ef[c]);
            P[3 * r + c] = v;
        }
    if (model == HIPIB_STANDARD_REINFORCING) {   // the I5f term
        T Ce[3], FCe[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) Ce[c] = Fm[c] * Fe[0] + Fm[3 + c] * Fe[1] + Fm[6 + c] * Fe[2];
#pragma unroll
        for (int r = 0; r < 3; ++r) FCe[r] = Fm[3 * r] * Ce[0] + Fm[3 * r + 1] * Ce[1] + Fm[3 * r + 2] * Ce[2];
        const T c5 = par[1] - par[0];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) P[3 * r + c] += c5 * (Fe[r] * Ce[c] + FCe[r] * ef[c]);
    }
    return true;
}

// The same first Piola-Kirchhoff stress written on the displacement gradient
// H = F - I, for evaluation in FP32: every quantity that vanishes in the
// reference configuration is formed from H without subtracting O(1) terms, so
// the rounding error of P is relative to P itself (to the strain) rather than
// to |X| / displacement.
//   J - 1 = tr H + (tr(H)^2 - tr(H H)) / 2 + det H,   ln J = log1p(J - 1),
//   J^{-2/3} - 1 = expm1(-2/3 ln J),   I1 - 3 = 2 tr H + |H|^2,
//   J^{-2/3}(F - I1/3 F^{-T}) = J^{-2/3} dev(E) F^{-T},  E = B - I = H + H^T + H H^T,
//   cof F = I + tr(H) I - H^T + cof H,   F^{-T} = cof F / J,
//   I4 - 1 = 2 e.(H e) + |H e|^2,   F e = e + H e,
//   I8 = e_f.e_s + e_f.(H e_s) + (H e_f).e_s + (H e_f).(H e_s)   (efes = e_f.e_s, in FP64),
//   sqrt(I4) - 1 = (I4 - 1) / (sqrt(I4) + 1),
// and for the standard reinforcing law the fibre and I5 terms combine, at
// d = (C - I) e = (H + H^T + H^T H) e, into
//   (E_L + G_T - 4 G_L)/2 (I4 - 1) (F e)(x)e - (G_T - G_L) ((F e)(x)d + (F d)(x)e).
// Returns false when J <= 0.
template <typename T>
__device__ __forceinline__ bool pk1_disp(int model, const T* par, const T* H, const T* ef, const T* es,
                                         T efes, bool sheet, T Ta, T* P) {
    const T trH = H[0] + H[4] + H[8];
    T trHH = T(0), HsqSum = T(0);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            trHH += H[3 * r + c] * H[3 * c + r];
            HsqSum += H[3 * r + c] * H[3 * r + c];
        }
    const T jm1 = trH + T(0.5) * (trH * trH - trHH) + det3(H);   // J - 1
    if (!(jm1 > T(-1))) return false;
    const T J = T(1) + jm1;
    const T lnJ = log1p(jm1);
    const T jm = expm1(T(-2) / T(3) * lnJ);                        // J^{-2/3} - 1
    const T i1m3 = T(2) * trH + HsqSum;                             // I1 - 3
    const T i1bm3 = i1m3 + jm * (T(3) + i1m3);                      // I1bar - 3
    // G = F^{-T}
    T G[9];
    cof3(H, G);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) G[3 * r + c] -= H[3 * c + r];
    G[0] += T(1) + trH;
    G[4] += T(1) + trH;
    G[8] += T(1) + trH;
    const T invJ = T(1) / J;
#pragma unroll
    for (int r = 0; r < 9; ++r) G[r] *= invJ;
    // dev(E), E = H + H^T + H H^T
    T E[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            E[3 * r + c] = H[3 * r + c] + H[3 * c + r] +
                           (H[3 * r] * H[3 * c] + H[3 * r + 1] * H[3 * c + 1] + H[3 * r + 2] * H[3 * c + 2]);
    const T third = i1m3 / T(3);   // tr E / 3
    E[0] -= third;
    E[4] -= third;
    E[8] -= third;
    // fibre (and sheet) stretches
    T He[3] = {T(0), T(0), T(0)}, Fe[3] = {T(0), T(0), T(0)};
    T I4m1 = T(0);
    if (model != HIPIB_NEO_HOOKEAN) {
#pragma unroll
        for (int r = 0; r < 3; ++r) He[r] = H[3 * r] * ef[0] + H[3 * r + 1] * ef[1] + H[3 * r + 2] * ef[2];
        I4m1 = T(2) * (ef[0] * He[0] + ef[1] * He[1] + ef[2] * He[2]) +
               (He[0] * He[0] + He[1] * He[1] + He[2] * He[2]);
#pragma unroll
        for (int r = 0; r < 3; ++r) Fe[r] = ef[r] + He[r];
    }
    T iso, kappa, fib = T(0), sh = T(0), fs = T(0);
    T Fs[3] = {T(0), T(0), T(0)};
    if (model == HIPIB_NEO_HOOKEAN) {
        iso = par[0];
        kappa = par[1];
    } else if (model == HIPIB_STANDARD_REINFORCING) {
        iso = par[0];
        kappa = par[3];
        fib = T(0.5) * (par[2] + par[0] - T(4) * par[1]) * I4m1;
    } else if (model == HIPIB_FIBRE_REINFORCED_1) {
        iso = T(2) * par[0];
        kappa = par[3];
        if (I4m1 > T(0)) fib = T(2) * par[1] * I4m1 * exp(par[2] * I4m1 * I4m1);
    } else if (model == HIPIB_FIBRE_REINFORCED_2) {
        iso = T(2) * par[0] * par[1] * exp(par[1] * i1bm3);
        kappa = par[4];
        fib = T(2) * par[2] * I4m1 * exp(par[3] * I4m1 * I4m1);
    } else {
        kappa = par[4];
        iso = par[0] * exp(par[1] * i1bm3);
        if (I4m1 > T(0)) fib = T(2) * par[2] * I4m1 * exp(par[3] * I4m1 * I4m1);
        if (Ta != T(0)) fib += Ta * (T(1) + T(4.9) * (I4m1 / (sqrt(T(1) + I4m1) + T(1))));
        if (sheet) {
            T Hs[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) Hs[r] = H[3 * r] * es[0] + H[3 * r + 1] * es[1] + H[3 * r + 2] * es[2];
            const T I4sm1 = T(2) * (es[0] * Hs[0] + es[1] * Hs[1] + es[2] * Hs[2]) +
                            (Hs[0] * Hs[0] + Hs[1] * Hs[1] + Hs[2] * Hs[2]);
            if (I4sm1 > T(0)) sh = T(2) * par[5] * I4sm1 * exp(par[6] * I4sm1 * I4sm1);
            const T I8 = efes + (ef[0] * Hs[0] + ef[1] * Hs[1] + ef[2] * Hs[2]) +
                         (He[0] * es[0] + He[1] * es[1] + He[2] * es[2]) +
                         (He[0] * Hs[0] + He[1] * Hs[1] + He[2] * Hs[2]);
            fs = par[7] * I8 * exp(par[8] * I8 * I8);
#pragma unroll
            for (int r = 0; r < 3; ++r) Fs[r] = es[r] + Hs[r];
        }
    }
    const T a = iso * (T(1) + jm), vol = kappa * lnJ;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T devG = E[3 * r] * G[c] + E[3 * r + 1] * G[3 + c] + E[3 * r + 2] * G[6 + c];
            T v = a * devG + vol * G[3 * r + c] + fib * Fe[r] * ef[c];
            if (sheet) v += sh * Fs[r] * es[c] + fs * (Fe[r] * es[c] + Fs[r] * ef[c]);
            P[3 * r + c] = v;
        }
    if (model == HIPIB_STANDARD_REINFORCING) {
        // d = (H + H^T + H^T H) e, F d = d + H d
        T d[3], Fd[3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            d[c] = He[c] + (H[c] * ef[0] + H[3 + c] * ef[1] + H[6 + c] * ef[2]) +
                   (H[c] * He[0] + H[3 + c] * He[1] + H[6 + c] * He[2]);
#pragma unroll
        for (int r = 0; r < 3; ++r) Fd[r] = d[r] + H[3 * r] * d[0] + H[3 * r + 1] * d[1] + H[3 * r + 2] * d[2];
        const T c5 = par[1] - par[0];   // G_L - G_T
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) P[3 * r + c] += c5 * (Fe[r] * d[c] + Fd[r] * ef[c]);
    }
    return true;
}

// dP = dP/dF : dF.  With G = F^{-T}: dG = -G dF^T G, d ln J = G : dF,
// dI1 = 2 F : dF, d J^{-2/3} = -(2/3) J^{-2/3} d ln J, dI4i = 2 (F e_i).(dF e_i),
// dI8 = (dF e_f).(F e_s) + (F e_f).(dF e_s); iso coefficient alpha (mu_s, or
// a e^{b(I1bar-3)}), fibre / sheet coefficient f_i(I4) = 2 a_i (I4-1) e^{b_i (I4-1)^2}
// with f_i' = 2 a_i e^{..}(1 + 2 b_i (I4-1)^2), fibre-sheet g(I8) = a_fs I8 e^{b_fs I8^2}
// with g' = a_fs e^{..}(1 + 2 b_fs I8^2), active T_a (1 + 4.9 (sqrt(I4f) - 1)) with
// derivative T_a 4.9 / (2 sqrt(I4f)).
template <typename T>
__device__ __forceinline__ bool pk1_tangent(int model, const T* par, const T* Fm, const T* ef,
                                            const T* es, bool sheet, T Ta, const T* dF, T* dP) {
    const T J = det3(Fm);
    if (!(J > T(0))) return false;
    T G[9], dG[9];
    cof3(Fm, G);
    const T invJ = T(1) / J;
#pragma unroll
    for (int r = 0; r < 9; ++r) G[r] *= invJ;
    // dG = -G dF^T G: (dF^T G)[s][c] = sum_t dF[t][s] G[t][c]
    T M[9];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) M[3 * s + c] = dF[s] * G[c] + dF[3 + s] * G[3 + c] + dF[6 + s] * G[6 + c];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            dG[3 * r + c] = -(G[3 * r] * M[c] + G[3 * r + 1] * M[3 + c] + G[3 * r + 2] * M[6 + c]);
    T I1 = T(0), dI1 = T(0), dlnJ = T(0);
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        I1 += Fm[r] * Fm[r];
        dI1 += T(2) * Fm[r] * dF[r];
        dlnJ += G[r] * dF[r];
    }
    const T cb = cbrt(J);
    const T Jm23 = T(1) / (cb * cb);
    const T dJm23 = -T(2) / T(3) * Jm23 * dlnJ;
    const T lnJ = log(J);
    T alpha, dalpha, kappa, fib = T(0), dfib = T(0);
    T sh = T(0), dsh = T(0), fs = T(0), dfs = T(0);
    T Fe[3] = {T(0), T(0), T(0)}, dFe[3] = {T(0), T(0), T(0)};
    T Fs[3] = {T(0), T(0), T(0)}, dFs[3] = {T(0), T(0), T(0)};
    if (model != HIPIB_NEO_HOOKEAN) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            Fe[r] = Fm[3 * r] * ef[0] + Fm[3 * r + 1] * ef[1] + Fm[3 * r + 2] * ef[2];
            dFe[r] = dF[3 * r] * ef[0] + dF[3 * r + 1] * ef[1] + dF[3 * r + 2] * ef[2];
        }
    }
    const T I4 = Fe[0] * Fe[0] + Fe[1] * Fe[1] + Fe[2] * Fe[2];
    const T dI4 = T(2) * (Fe[0] * dFe[0] + Fe[1] * dFe[1] + Fe[2] * dFe[2]);
    const T dI1bar = dJm23 * I1 + Jm23 * dI1;
    if (model == HIPIB_NEO_HOOKEAN) {
        alpha = par[0];
        dalpha = T(0);
        kappa = par[1];
    } else if (model == HIPIB_STANDARD_REINFORCING) {
        alpha = par[0];
        dalpha = T(0);
        kappa = par[3];
        const T cL = par[2] + par[0] - T(4) * par[1];
        fib = T(2) * (par[0] - par[1]) + T(0.5) * cL * (I4 - T(1));
        dfib = T(0.5) * cL * dI4;
    } else if (model == HIPIB_FIBRE_REINFORCED_1) {
        alpha = T(2) * par[0];
        dalpha = T(0);
        kappa = par[3];
        if (I4 > T(1)) {
            const T q = I4 - T(1);
            const T Ef = exp(par[2] * q * q);
            fib = T(2) * par[1] * q * Ef;
            dfib = T(2) * par[1] * Ef * (T(1) + T(2) * par[2] * q * q) * dI4;
        }
    } else if (model == HIPIB_FIBRE_REINFORCED_2) {
        alpha = T(2) * par[0] * par[1] * exp(par[1] * (Jm23 * I1 - T(3)));
        dalpha = alpha * par[1] * dI1bar;
        kappa = par[4];
        const T q = I4 - T(1);
        const T Ef = exp(par[3] * q * q);
        fib = T(2) * par[2] * q * Ef;
        dfib = T(2) * par[2] * Ef * (T(1) + T(2) * par[3] * q * q) * dI4;
    } else {
        kappa = par[4];
        const T E1 = exp(par[1] * (Jm23 * I1 - T(3)));
        alpha = par[0] * E1;
        dalpha = alpha * par[1] * dI1bar;
        if (I4 > T(1)) {
            const T q = I4 - T(1);
            const T Ef = exp(par[3] * q * q);
            fib = T(2) * par[2] * q * Ef;
            dfib = T(2) * par[2] * Ef * (T(1) + T(2) * par[3] * q * q) * dI4;
        }
        if (Ta != T(0)) {
            const T r4 = sqrt(I4);
            fib += Ta * (T(1) + T(4.9) * (r4 - T(1)));
            dfib += Ta * T(4.9) / (T(2) * r4) * dI4;
        }
        if (sheet) {
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                Fs[r] = Fm[3 * r] * es[0] + Fm[3 * r + 1] * es[1] + Fm[3 * r + 2] * es[2];
                dFs[r] = dF[3 * r] * es[0] + dF[3 * r + 1] * es[1] + dF[3 * r + 2] * es[2];
            }
            const T I4s = Fs[0] * Fs[0] + Fs[1] * Fs[1] + Fs[2] * Fs[2];
            if (I4s > T(1)) {
                const T dI4s = T(2) * (Fs[0] * dFs[0] + Fs[1] * dFs[1] + Fs[2] * dFs[2]);
                const T q = I4s - T(1);
                const T Es = exp(par[6] * q * q);
                sh = T(2) * par[5] * q * Es;
                dsh = T(2) * par[5] * Es * (T(1) + T(2) * par[6] * q * q) * dI4s;
            }
            const T I8 = Fe[0] * Fs[0] + Fe[1] * Fs[1] + Fe[2] * Fs[2];
            const T dI8 = dFe[0] * Fs[0] + dFe[1] * Fs[1] + dFe[2] * Fs[2] +
                          Fe[0] * dFs[0] + Fe[1] * dFs[1] + Fe[2] * dFs[2];
            const T Efs = exp(par[8] * I8 * I8);
            fs = par[7] * I8 * Efs;
            dfs = par[7] * Efs * (T(1) + T(2) * par[8] * I8 * I8) * dI8;
        }
    }
    const T c1 = dalpha * Jm23 + alpha * dJm23, c2 = alpha * Jm23;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int o = 3 * r + c;
            const T Mo = Fm[o] - I1 / T(3) * G[o];
            const T dMo = dF[o] - dI1 / T(3) * G[o] - I1 / T(3) * dG[o];
            T v = c1 * Mo + c2 * dMo + dfib * Fe[r] * ef[c] + fib * dFe[r] * ef[c] +
                  kappa * dlnJ * G[o] + kappa * lnJ * dG[o];
            if (sheet)
                v += dsh * Fs[r] * es[c] + sh * dFs[r] * es[c] +
                     dfs * (Fe[r] * es[c] + Fs[r] * ef[c]) + fs * (dFe[r] * es[c] + dFs[r] * ef[c]);
            dP[o] = v;
        }
    if (model == HIPIB_STANDARD_REINFORCING) {
        // d[c5 ((F e)(x)(C e) + (F C e)(x)e)], d(C e) = dF^T (F e) + F^T (dF e),
        // d(F C e) = dF (C e) + F d(C e)
        T Ce[3], dCe[3], dFCe[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Ce[c] = Fm[c] * Fe[0] + Fm[3 + c] * Fe[1] + Fm[6 + c] * Fe[2];
            dCe[c] = dF[c] * Fe[0] + dF[3 + c] * Fe[1] + dF[6 + c] * Fe[2] +
                     Fm[c] * dFe[0] + Fm[3 + c] * dFe[1] + Fm[6 + c] * dFe[2];
        }
#pragma unroll
        for (int r = 0; r < 3; ++r)
            dFCe[r] = dF[3 * r] * Ce[0] + dF[3 * r + 1] * Ce[1] + dF[3 * r + 2] * Ce[2] +
                      Fm[3 * r] * dCe[0] + Fm[3 * r + 1] * dCe[1] + Fm[3 * r + 2] * dCe[2];
        const T c5 = par[1] - par[0];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                dP[3 * r + c] += c5 * (dFe[r] * Ce[c] + Fe[r] * dCe[c] + dFCe[r] * ef[c]);
    }
    return true;
}

// derivative of the trilinear shape function a = i + 2j + 4k at reference point xi
template <typename T>
__device__ __forceinline__ void hex_dN(const T* xi, T dN[8][3]) {
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const T s0 = (a & 1) ? T(1) : T(-1), s1 = (a & 2) ? T(1) : T(-1), s2 = (a & 4) ? T(1) : T(-1);
        const T f0 = T(1) + s0 * xi[0], f1 = T(1) + s1 * xi[1], f2 = T(1) + s2 * xi[2];
        dN[a][0] = s0 * f1 * f2 * T(0.125);
        dN[a][1] = f0 * s1 * f2 * T(0.125);
        dN[a][2] = f0 * f1 * s2 * T(0.125);
    }
}

// Element types: node count N, quadrature points Q, and the rule (the paper
// leaves it open): hexes 2x2x2 Gauss at +-1/sqrt(3) with unit weights; P1 tets
// one point at the centroid, weight 1/6; P2 tets (vertices 0-3, edge nodes on
// (0,1), (1,2), (0,2), (0,3), (1,3), (2,3)) the symmetric 4-point rule of degree 2,
// barycentric (a, b, b, b) and permutations, a = (5 + 3 sqrt 5)/20, b = (5 - sqrt 5)/20,
// weights 1/24.  Tets use barycentric l0 = 1 - xi - eta - zeta, l1..l3 = xi, eta, zeta.
struct Hex8 { static constexpr int N = 8, Q = 8; };
struct Tet4 { static constexpr int N = 4, Q = 1; };
struct Tet10 { static constexpr int N = 10, Q = 4; };

// dN_a/dxi at quadrature point g; returns the point's reference weight
template <typename S, typename T>
__device__ __forceinline__ T elem_rule(int g, T dN[S::N][3]) {
    if constexpr (S::N == 8) {
        const T gp = T(0.57735026918962576451);  // 1/sqrt(3)
        const T xi[3] = {(g & 1) ? gp : -gp, (g & 2) ? gp : -gp, (g & 4) ? gp : -gp};
        hex_dN(xi, dN);
        return T(1);
    } else {
        // gradients of the barycentric coordinates
        const T gl[4][3] = {{T(-1), T(-1), T(-1)}, {T(1), T(0), T(0)}, {T(0), T(1), T(0)}, {T(0), T(0), T(1)}};
        if constexpr (S::N == 4) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int k = 0; k < 3; ++k) dN[a][k] = gl[a][k];
            return T(1) / T(6);
        } else {
            const T qa = T(0.58541019662496845446), qb = T(0.13819660112501051518);
            T l[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) l[a] = a == g ? qa : qb;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int k = 0; k < 3; ++k) dN[a][k] = (T(4) * l[a] - T(1)) * gl[a][k];
            constexpr int ei[6] = {0, 1, 0, 0, 1, 2}, ej[6] = {1, 2, 2, 3, 3, 3};
#pragma unroll
            for (int t = 0; t < 6; ++t)
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    dN[4 + t][k] = T(4) * (l[ej[t]] * gl[ei[t]][k] + l[ei[t]] * gl[ej[t]][k]);
            return T(1) / T(24);
        }
    }
}

// sum_a v_a (x) dN_a  (3x3, row r = component of v, column c = reference axis)
template <int N, typename T>
__device__ __forceinline__ void gather_jac(const T v[N][3], const T dN[N][3], T* Jm) {
#pragma unroll
    for (int t = 0; t < 9; ++t) Jm[t] = T(0);
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) Jm[3 * r + c] += v[a][r] * dN[a][c];
}

// A B (3x3 row-major)
template <typename T>
__device__ __forceinline__ void matmul3(const T* A, const T* B, T* C) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}

}  // namespace hipib
