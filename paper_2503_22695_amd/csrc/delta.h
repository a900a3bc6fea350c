// Device helpers for Peskin's four-point regularized delta: for a lattice
// coordinate r with b = floor(r), f = r - b, s = sqrt(1 + 4 f (1 - f)), the
// support b-1 .. b+2 carries the weights ((3-2f-s), (3-2f+s), (1+2f+s), (1+2f-s))/8
// (phi at f+1, f, 1-f, 2-f) and their derivatives with respect to f,
// (-2-s', -2+s', 2+s', 2-s')/8 with s' = (2 - 4 f) / s (phi is C^1; s >= 1).
#pragma once

#include "internal.h"

namespace hipib {

__device__ __forceinline__ double safe_coord(double r) { return fabs(r) < 1.0e9 ? r : 0.0; }

__device__ __forceinline__ int wrap_mod(int i, int n) {
    const int r = i % n;
    return r < 0 ? r + n : r;
}

__device__ __forceinline__ int step_wrap(int i, int n) { return i >= n ? i - n : i; }

// weights (and optionally their f-derivatives) for the lattice coordinate r
// (computed in FP64 up to the fractional offset, then in TW); returns the first
// index b - 1 wrapped into [0, n)
template <typename TW, bool DERIV>
__device__ __forceinline__ int peskin_weights(double r, int n, TW* w, TW* dw) {
    r = safe_coord(r);
    const double bf = floor(r);
    const TW f = (TW)(r - bf);
    const TW s = sqrt(TW(1) + TW(4) * f * (TW(1) - f));
    w[0] = (TW(3) - TW(2) * f - s) * TW(0.125);
    w[1] = (TW(3) - TW(2) * f + s) * TW(0.125);
    w[2] = (TW(1) + TW(2) * f + s) * TW(0.125);
    w[3] = (TW(1) + TW(2) * f - s) * TW(0.125);
    if (DERIV) {
        const TW sp = (TW(2) - TW(4) * f) / s;
        dw[0] = (-TW(2) - sp) * TW(0.125);
        dw[1] = (-TW(2) + sp) * TW(0.125);
        dw[2] = (TW(2) + sp) * TW(0.125);
        dw[3] = (TW(2) - sp) * TW(0.125);
    }
    return wrap_mod((int)bf - 1, n);
}

}  // namespace hipib
