// Kaiser-Bessel window taps shared by the interpolation kernels (device code).
//
// Taps: with u = omega K / (2 pi), k_start = floor(u - J/2) + 1 and taps
// k_start + j, j < J, at distances t_j = u - k_start - j in [-J/2, J/2);
// grid indices wrap modulo K.  The window psi(t) = I0(beta sqrt(1 -
// (2t/J)^2)) / I0(beta) is evaluated per tap by a degree-10 polynomial in
// x = 2 f - 1 (f = fractional position of u - J/2), fitted on the host.
#pragma once

#include "kbn_internal.h"

namespace {

__device__ __forceinline__ void tap_origin(int J, int cell, float frac, int &start, float &f) {
    if ((J & 1) == 0) {
        start = cell - J / 2 + 1;
        f = frac;
    } else if (frac >= 0.5f) {
        start = cell - J / 2 + 1;
        f = frac - 0.5f;
    } else {
        start = cell - J / 2;
        f = frac + 0.5f;
    }
}

template <int J>
__device__ __forceinline__ void kb_weights(float f, const float *__restrict__ coef, float *w) {
    const float x = 2.f * f - 1.f;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        float acc = coef[j * KBN_NCOEF + KBN_NCOEF - 1];
#pragma unroll
        for (int k = KBN_NCOEF - 2; k >= 0; --k) acc = fmaf(acc, x, coef[j * KBN_NCOEF + k]);
        w[j] = acc;
    }
}

__device__ __forceinline__ int wrapk(int i, int K) {  // i in [-K, 2K)
    return i < 0 ? i + K : (i >= K ? i - K : i);
}

// Tap reach of a point in cell c: taps lie in [c - LO, c + HI].
template <int J>
struct Reach {
    static constexpr int LO = (J & 1) ? J / 2 : J / 2 - 1;
    static constexpr int HI = (J & 1) ? J / 2 + 1 : J / 2;
};

}  // namespace
