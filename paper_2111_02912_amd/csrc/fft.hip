// Oversampled-grid FFT passes of the NUFFT (appendix: "K-point FFT ... via
// zero-padding"), one pass per axis, each a batch of 1D transforms done in
// LDS with a mixed-radix Stockham schedule (radices 2, 3, 4, 5, 7, 8).
//
// Pass kinds:
//   first pass (forward, last axis): reads image rows, applies the scaling
//     factors s_n of every axis, an optional coil map and an optional
//     coordinate weight r^[w] (the Jacobian operand x (.) r^[d] of Sec. II-C),
//     places the N values at r mod K (zero-padding) and transforms.
//   mid pass (any other axis, strided): zero-padded input rows in, all K
//     outputs (forward), or all K inputs in and only the N kept rows out
//     (adjoint crop).
//   last adjoint pass (last axis): inverse transform, crop to N, scaling
//     factors and conj(coil map), summed over coils.
// Forward transforms use exp(-2 pi i k n / K), inverse ones exp(+...), both
// unnormalised.  Twiddles come from a host FP64 table rounded to float.
#include "kbn_internal.h"

namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
    static __device__ __forceinline__ void run(float2 *a) {
        const float2 t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    }
};

template <bool INV>
struct Dft<4, INV> {
    static __device__ __forceinline__ void run(float2 *a) {
        const float2 t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
        const float2 t2 = cadd(a[1], a[3]), t3 = rot<INV>(csub(a[1], a[3]));
        a[0] = cadd(t0, t2);
        a[2] = csub(t0, t2);
        a[1] = cadd(t1, t3);
        a[3] = csub(t1, t3);
    }
};

template <bool INV>
struct Dft<8, INV> {
    static __device__ __forceinline__ void run(float2 *a) {
        float2 e[4] = {a[0], a[2], a[4], a[6]};
        float2 o[4] = {a[1], a[3], a[5], a[7]};
        Dft<4, INV>::run(e);
        Dft<4, INV>::run(o);
        const float r = 0.70710678118654752f;
        // o[k] *= W8^k, W8 = exp(-+ 2 pi i / 8)
        float2 w1, w3;
        if (!INV) {
            w1 = make_float2(r * (o[1].x + o[1].y), r * (o[1].y - o[1].x));
            w3 = make_float2(r * (o[3].y - o[3].x), -r * (o[3].x + o[3].y));
        } else {
            w1 = make_float2(r * (o[1].x - o[1].y), r * (o[1].x + o[1].y));
            w3 = make_float2(-r * (o[3].x + o[3].y), r * (o[3].x - o[3].y));
        }
        const float2 w2 = rot<INV>(o[2]);
        a[0] = cadd(e[0], o[0]);
        a[4] = csub(e[0], o[0]);
        a[1] = cadd(e[1], w1);
        a[5] = csub(e[1], w1);
        a[2] = cadd(e[2], w2);
        a[6] = csub(e[2], w2);
        a[3] = cadd(e[3], w3);
        a[7] = csub(e[3], w3);
    }
};

// cos(2 pi i / R), sin(2 pi i / R) for the odd radices
template <int R>
struct Trig;
template <>
struct Trig<3> {
    static constexpr float c[3] = {1.0f, -0.5f, -0.5f};
    static constexpr float s[3] = {0.0f, 0.86602540378443865f, -0.86602540378443865f};
};
template <>
struct Trig<5> {
    static constexpr float c[5] = {1.0f, 0.30901699437494742f, -0.80901699437494742f,
                                   -0.80901699437494742f, 0.30901699437494742f};
    static constexpr float s[5] = {0.0f, 0.95105651629515357f, 0.58778525229247313f,
                                   -0.58778525229247313f, -0.95105651629515357f};
};
template <>
struct Trig<7> {
    static constexpr float c[7] = {1.0f,
                                   0.62348980185873353f,
                                   -0.22252093395631440f,
                                   -0.90096886790241913f,
                                   -0.90096886790241913f,
                                   -0.22252093395631440f,
                                   0.62348980185873353f};
    static constexpr float s[7] = {0.0f,
                                   0.78183148246802981f,
                                   0.97492791218182361f,
                                   0.43388373911755812f,
                                   -0.43388373911755812f,
                                   -0.97492791218182361f,
                                   -0.78183148246802981f};
};

// Direct odd-length DFT using the symmetric pairs (n, R - n).
template <int R, bool INV>
struct DftOdd {
    static __device__ __forceinline__ void run(float2 *a) {
        constexpr int H = (R - 1) / 2;
        float2 sp[H], sm[H];
#pragma unroll
        for (int n = 1; n <= H; ++n) {
            sp[n - 1] = cadd(a[n], a[R - n]);
            sm[n - 1] = csub(a[n], a[R - n]);
        }
        const float2 a0 = a[0];
        float2 sum = a0;
#pragma unroll
        for (int n = 0; n < H; ++n) sum = cadd(sum, sp[n]);
        a[0] = sum;
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            float2 A = a0, Bv = make_float2(0.f, 0.f);
#pragma unroll
            for (int n = 1; n <= H; ++n) {
                const int idx = (n * k) % R;
                const float cc = Trig<R>::c[idx], ss = Trig<R>::s[idx];
                A.x += sp[n - 1].x * cc;
                A.y += sp[n - 1].y * cc;
                Bv.x += sm[n - 1].x * ss;
                Bv.y += sm[n - 1].y * ss;
            }
            const float2 iB = make_float2(-Bv.y, Bv.x);
            a[k] = INV ? cadd(A, iB) : csub(A, iB);
            a[R - k] = INV ? csub(A, iB) : cadd(A, iB);
        }
    }
};
template <bool INV>
struct Dft<3, INV> : DftOdd<3, INV> {};
template <bool INV>
struct Dft<5, INV> : DftOdd<5, INV> {};
template <bool INV>
struct Dft<7, INV> : DftOdd<7, INV> {};

// One Stockham stage of radix R over nl lines of length L held in LDS.
// Element i of line l lives at buf[l * ls + i * es].  Each thread owns up to
// MAXE / R butterflies; all reads finish (barrier) before the in-place writes.
template <int R, int MAXE, bool INV>
__device__ __forceinline__ void fft_stage(float2 *buf, const float2 *twl, int L, int Ns, int nl,
                                          int ls, int es, bool line_fast) {
    constexpr int NB = MAXE / R;
    const int nbf = L / R;
    const int total = nl * nbf;
    const int tstride = L / (Ns * R);
    float2 v[NB][R];
    int ob[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int w = threadIdx.x + b * KBN_BLOCK;
        ob[b] = -1;
        if (w < total) {
            int l, j;
            if (line_fast) {
                j = w / nl;
                l = w - j * nl;
            } else {
                l = w / nbf;
                j = w - l * nbf;
            }
            const int k = j % Ns;
            const int base = l * ls;
#pragma unroll
            for (int q = 0; q < R; ++q) v[b][q] = buf[base + (j + q * nbf) * es];
            if (Ns > 1) {
#pragma unroll
                for (int q = 1; q < R; ++q) {
                    float2 t = twl[q * k * tstride];
                    if (INV) t.y = -t.y;
                    v[b][q] = cmul(v[b][q], t);
                }
            }
            Dft<R, INV>::run(v[b]);
            ob[b] = base + ((j - k) * R + k) * es;
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (ob[b] >= 0) {
#pragma unroll
            for (int q = 0; q < R; ++q) buf[ob[b] + q * Ns * es] = v[b][q];
        }
    }
    __syncthreads();
}

template <int MAXE, bool INV>
__device__ void fft_lds(float2 *buf, const float2 *twl, const KbnRadix &rp, int nl, int ls, int es,
                        bool line_fast) {
    const int L = rp.L;
    int Ns = 1;
    for (int s = 0; s < rp.nst; ++s) {
        const int R = rp.r[s];
        switch (R) {
            case 8: fft_stage<8, MAXE, INV>(buf, twl, L, Ns, nl, ls, es, line_fast); break;
            case 4: fft_stage<4, MAXE, INV>(buf, twl, L, Ns, nl, ls, es, line_fast); break;
            case 2: fft_stage<2, MAXE, INV>(buf, twl, L, Ns, nl, ls, es, line_fast); break;
            case 3: fft_stage<3, MAXE, INV>(buf, twl, L, Ns, nl, ls, es, line_fast); break;
            case 5: fft_stage<5, MAXE, INV>(buf, twl, L, Ns, nl, ls, es, line_fast); break;
            default: fft_stage<7, MAXE, INV>(buf, twl, L, Ns, nl, ls, es, line_fast); break;
        }
        Ns *= R;
    }
}

__device__ __forceinline__ int wrap_pos(int j, int n, int L) {  // r = j - floor(n/2), r mod L
    int p = j - n / 2;
    return p < 0 ? p + L : p;
}

// Product of the scaling factors of the leading axes (and the optional
// coordinate weight) for image row `row` (flat index over axes 0..D-2).
__device__ __forceinline__ float row_factor(int row, int D, const int *N, const float *const *deap,
                                            int wsel) {
    float f = 1.f;
    int rem = row;
    for (int d = D - 2; d >= 0; --d) {
        const int id = rem % N[d];
        rem /= N[d];
        f *= deap[d][id];
        if (wsel == d) f *= (float)(id - N[d] / 2);
    }
    return f;
}

template <int MAXE>
__global__ void __launch_bounds__(KBN_BLOCK)
k_first_pass(KbnFirstPassArgs a, KbnRadix rp, const float2 *__restrict__ tw, int nl) {
    extern __shared__ float2 smem[];
    const int L = rp.L;
    float2 *twl = smem;
    float2 *buf = smem + L;
    for (int i = threadIdx.x; i < L; i += KBN_BLOCK) twl[i] = tw[i];
    const int64_t line0 = (int64_t)blockIdx.x * nl;
    const int nlb = (int)min((int64_t)nl, a.nlines - line0);
    for (int i = threadIdx.x; i < nl * L; i += KBN_BLOCK) buf[i] = make_float2(0.f, 0.f);
    __syncthreads();
    const int Nl = a.Nl;
    const float *deap_l = a.deap[a.D - 1];
    for (int e = threadIdx.x; e < nlb * Nl; e += KBN_BLOCK) {
        const int li = e / Nl;
        const int j = e - li * Nl;
        const int64_t line = line0 + li;
        const int64_t ch = line / a.R0;
        const int row = (int)(line - ch * a.R0);
        const int w = (int)(ch % a.nw);
        const int64_t cc = ch / a.nw;
        const int c = (int)(cc % a.C);
        const int64_t bl = cc / a.C;
        const int wsel = a.weighted ? w : -1;
        float2 v = a.x[(bl * a.R0 + row) * (int64_t)Nl + j];
        float f = deap_l[j] * row_factor(row, a.D, a.N, a.deap, wsel);
        if (wsel == a.D - 1) f *= (float)(j - Nl / 2);
        if (a.smaps) v = cmul(v, a.smaps[((int64_t)c * a.R0 + row) * Nl + j]);
        buf[li * L + wrap_pos(j, Nl, L)] = make_float2(v.x * f, v.y * f);
    }
    __syncthreads();
    fft_lds<MAXE, false>(buf, twl, rp, nl, L, 1, false);
    float2 *out = a.out + line0 * L;
    for (int e = threadIdx.x; e < nlb * L; e += KBN_BLOCK) out[e] = buf[e];
}

template <int MAXE, bool INV>
__global__ void __launch_bounds__(KBN_BLOCK)
k_mid_pass(KbnMidPassArgs a, KbnRadix rp, const float2 *__restrict__ tw, int nl) {
    extern __shared__ float2 smem[];
    const int L = rp.L;
    float2 *twl = smem;
    float2 *buf = smem + L;
    for (int i = threadIdx.x; i < L; i += KBN_BLOCK) twl[i] = tw[i];
    const int ntile = (a.inner + nl - 1) / nl;
    const int64_t o = blockIdx.x / ntile;
    const int c0 = (int)(blockIdx.x - o * ntile) * nl;
    const int ncols = min(nl, a.inner - c0);
    if (a.pad_in)
        for (int i = threadIdx.x; i < nl * L; i += KBN_BLOCK) buf[i] = make_float2(0.f, 0.f);
    __syncthreads();
    const float2 *in = a.in + (o * a.nin) * (int64_t)a.inner + c0;
    for (int e = threadIdx.x; e < a.nin * ncols; e += KBN_BLOCK) {
        const int i = e / ncols;
        const int cc = e - i * ncols;
        const int p = a.pad_in ? wrap_pos(i, a.nin, L) : i;
        buf[p * nl + cc] = in[(int64_t)i * a.inner + cc];
    }
    __syncthreads();
    fft_lds<MAXE, INV>(buf, twl, rp, nl, 1, nl, true);
    float2 *out = a.out + (o * a.nout) * (int64_t)a.inner + c0;
    for (int e = threadIdx.x; e < a.nout * ncols; e += KBN_BLOCK) {
        const int i = e / ncols;
        const int cc = e - i * ncols;
        const int p = a.crop_out ? wrap_pos(i, a.nout, L) : i;
        out[(int64_t)i * a.inner + cc] = buf[p * nl + cc];
    }
}

template <int MAXE>
__global__ void __launch_bounds__(KBN_BLOCK)
k_last_adj(KbnLastAdjArgs a, KbnRadix rp, const float2 *__restrict__ tw, int nl) {
    extern __shared__ float2 smem[];
    const int L = rp.L;
    float2 *twl = smem;
    float2 *buf = smem + L;
    for (int i = threadIdx.x; i < L; i += KBN_BLOCK) twl[i] = tw[i];
    const int64_t line0 = (int64_t)blockIdx.x * nl;
    const int nlb = (int)min((int64_t)nl, a.nlines - line0);
    const int Nl = a.Nl;
    const float *deap_l = a.deap[a.D - 1];
    float2 acc[MAXE];
#pragma unroll
    for (int k = 0; k < MAXE; ++k) acc[k] = make_float2(0.f, 0.f);
    for (int c = 0; c < a.C; ++c) {
        for (int e = threadIdx.x; e < nlb * L; e += KBN_BLOCK) {
            const int li = e / L;
            const int p = e - li * L;
            const int64_t line = line0 + li;
            const int64_t bl = line / a.R0;
            const int row = (int)(line - bl * a.R0);
            buf[e] = a.in[(((bl * a.C + c) * a.R0) + row) * (int64_t)L + p];
        }
        __syncthreads();
        fft_lds<MAXE, true>(buf, twl, rp, nl, L, 1, false);
#pragma unroll
        for (int k = 0; k < MAXE; ++k) {
            const int e = threadIdx.x + k * KBN_BLOCK;
            if (e < nlb * Nl) {
                const int li = e / Nl;
                const int j = e - li * Nl;
                const int64_t line = line0 + li;
                const int64_t bl = line / a.R0;
                const int row = (int)(line - bl * a.R0);
                float2 v = buf[li * L + wrap_pos(j, Nl, L)];
                const int cm = a.cmod > 0 ? (int)(bl % a.cmod) : c;
                if (a.smaps) v = cmulc(v, a.smaps[((int64_t)cm * a.R0 + row) * Nl + j]);
                const float f = deap_l[j] * row_factor(row, a.D, a.N, a.deap, -1);
                acc[k].x += v.x * f;
                acc[k].y += v.y * f;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < MAXE; ++k) {
        const int e = threadIdx.x + k * KBN_BLOCK;
        if (e < nlb * Nl) {
            float2 *dst = a.x + line0 * Nl + e;
            if (a.accumulate) {
                const float2 o = *dst;
                *dst = make_float2(o.x + acc[k].x, o.y + acc[k].y);
            } else {
                *dst = acc[k];
            }
        }
    }
}

int min_elems(const KbnRadix &rp, int maxe) {
    int m = maxe;
    for (int s = 0; s < rp.nst; ++s) {
        const int R = rp.r[s];
        const int e = (maxe / R) * R;
        if (e < m) m = e;
    }
    return m;
}

}  // namespace

int kbn_lines_per_block(const KbnRadix &rp, int maxe) {
    int nl = KBN_BLOCK * min_elems(rp, maxe) / rp.L;
    return nl < 1 ? 1 : nl;
}

hipError_t kbn_launch_first_pass(const KbnFirstPassArgs &a, const KbnRadix &rp, const float2 *tw,
                                 int maxe, hipStream_t s) {
    int nl = kbn_lines_per_block(rp, maxe);
    if ((int64_t)nl > a.nlines) nl = (int)a.nlines;
    const int64_t blocks = (a.nlines + nl - 1) / nl;
    const size_t lds = sizeof(float2) * (size_t)rp.L * (nl + 1);
    if (maxe == 32)
        k_first_pass<32><<<dim3((unsigned)blocks), dim3(KBN_BLOCK), lds, s>>>(a, rp, tw, nl);
    else
        k_first_pass<16><<<dim3((unsigned)blocks), dim3(KBN_BLOCK), lds, s>>>(a, rp, tw, nl);
    return hipGetLastError();
}

hipError_t kbn_launch_mid_pass(const KbnMidPassArgs &a, const KbnRadix &rp, const float2 *tw,
                               int inverse, int maxe, hipStream_t s) {
    int nl = kbn_lines_per_block(rp, maxe);
    if (nl > a.inner) nl = a.inner;
    const int64_t ntile = (a.inner + nl - 1) / nl;
    const int64_t blocks = a.outer * ntile;
    const size_t lds = sizeof(float2) * (size_t)rp.L * (nl + 1);
    if (maxe == 32) {
        if (inverse)
            k_mid_pass<32, true><<<dim3((unsigned)blocks), dim3(KBN_BLOCK), lds, s>>>(a, rp, tw, nl);
        else
            k_mid_pass<32, false><<<dim3((unsigned)blocks), dim3(KBN_BLOCK), lds, s>>>(a, rp, tw, nl);
    } else {
        if (inverse)
            k_mid_pass<16, true><<<dim3((unsigned)blocks), dim3(KBN_BLOCK), lds, s>>>(a, rp, tw, nl);
        else
            k_mid_pass<16, false><<<dim3((unsigned)blocks), dim3(KBN_BLOCK), lds, s>>>(a, rp, tw, nl);
    }
    return hipGetLastError();
}

// coil sum of the per-coil images of the split last pass, in coil order
__global__ void __launch_bounds__(KBN_BLOCK)
k_coil_sum(const float2 *__restrict__ ws, int64_t nb, int C, int64_t npix, float2 *__restrict__ x,
           int accumulate) {
    const int64_t n = nb * npix;
    for (int64_t i = (int64_t)blockIdx.x * KBN_BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * KBN_BLOCK) {
        const int64_t b = i / npix;
        const int64_t j = i - b * npix;
        float2 acc = accumulate ? x[i] : make_float2(0.f, 0.f);
        for (int c = 0; c < C; ++c) {
            const float2 v = ws[(b * C + c) * npix + j];
            acc.x += v.x;
            acc.y += v.y;
        }
        x[i] = acc;
    }
}

hipError_t kbn_launch_coil_sum(const float2 *ws, int64_t nb, int C, int64_t npix, float2 *x, int accumulate,
                               hipStream_t s) {
    const int64_t n = nb * npix;
    if (n <= 0) return hipSuccess;
    const int64_t g = std::min<int64_t>((n + KBN_BLOCK - 1) / KBN_BLOCK, 65536);
    k_coil_sum<<<dim3((unsigned)g), dim3(KBN_BLOCK), 0, s>>>(ws, nb, C, npix, x, accumulate);
    return hipGetLastError();
}

hipError_t kbn_launch_last_adj(const KbnLastAdjArgs &a, const KbnRadix &rp, const float2 *tw,
                               int maxe, hipStream_t s) {
    int nl = kbn_lines_per_block(rp, maxe);
    if ((int64_t)nl > a.nlines) nl = (int)a.nlines;
    const int64_t blocks = (a.nlines + nl - 1) / nl;
    const size_t lds = sizeof(float2) * (size_t)rp.L * (nl + 1);
    if (maxe == 32)
        k_last_adj<32><<<dim3((unsigned)blocks), dim3(KBN_BLOCK), lds, s>>>(a, rp, tw, nl);
    else
        k_last_adj<16><<<dim3((unsigned)blocks), dim3(KBN_BLOCK), lds, s>>>(a, rp, tw, nl);
    return hipGetLastError();
}
