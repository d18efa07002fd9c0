// Compile-time specialised FFT passes for the common oversampled grid sizes.
//
// Same operations as the generic passes in fft.hip (forward first pass with
// the scaling / coil / coordinate-weight prologue, strided forward and
// inverse passes with zero-padding and cropping, last inverse pass with
// crop, scaling and coil sum), for L in a fixed set.  With L and the number
// E of elements per thread known at compile time, every radix, stride and
// index is a constant.  Each thread holds the inputs of its E / R
// butterflies in registers; stage 0 reads them straight from global memory
// (zero-padding rows are never read), the last stage writes straight to
// global memory (cropped rows are never written), and only the stages in
// between exchange data through LDS.
//
// Butterfly ownership (Stockham, natural order in and out): in stage s with
// radix R and span Ns, thread u of a line owns butterflies j = u + TL*b,
// b < E/R (TL = L/E threads per line); butterfly j reads elements
// j + q*L/R and writes element (j - j%Ns)*R + j%Ns + q*Ns, q < R.
#include <algorithm>
#include <climits>

#include "kbn_internal.h"

#include <hip/hip_runtime.h>

namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
template <bool INV>
__device__ __forceinline__ float2 rot(float2 a) {  // * -i (forward) or * +i (inverse)
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---- small DFTs (forward sign exp(-2 pi i / R), conjugate for INV) --------
template <int R, bool INV>
struct SDft;
template <bool INV>
struct SDft<2, INV> {
    static __device__ __forceinline__ void run(float2 *a) {
        const float2 t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    }
};
template <bool INV>
struct SDft<4, INV> {
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
struct SDft<8, INV> {
    static __device__ __forceinline__ void run(float2 *a) {
        float2 e[4] = {a[0], a[2], a[4], a[6]};
        float2 o[4] = {a[1], a[3], a[5], a[7]};
        SDft<4, INV>::run(e);
        SDft<4, INV>::run(o);
        const float r = 0.70710678118654752f;
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
template <int R>
struct STrig;
template <>
struct STrig<3> {
    static constexpr float c[3] = {1.0f, -0.5f, -0.5f};
    static constexpr float s[3] = {0.0f, 0.86602540378443865f, -0.86602540378443865f};
};
template <>
struct STrig<5> {
    static constexpr float c[5] = {1.0f, 0.30901699437494742f, -0.80901699437494742f,
                                   -0.80901699437494742f, 0.30901699437494742f};
    static constexpr float s[5] = {0.0f, 0.95105651629515357f, 0.58778525229247313f,
                                   -0.58778525229247313f, -0.95105651629515357f};
};
template <int R, bool INV>
struct SDftOdd {
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
                A.x += sp[n - 1].x * STrig<R>::c[idx];
                A.y += sp[n - 1].y * STrig<R>::c[idx];
                Bv.x += sm[n - 1].x * STrig<R>::s[idx];
                Bv.y += sm[n - 1].y * STrig<R>::s[idx];
            }
            const float2 iB = make_float2(-Bv.y, Bv.x);
            a[k] = INV ? cadd(A, iB) : csub(A, iB);
            a[R - k] = INV ? csub(A, iB) : cadd(A, iB);
        }
    }
};
template <>
struct STrig<7> {
    static constexpr float c[7] = {1.0f, 0.62348980185873353f, -0.22252093395631440f,
                                   -0.90096886790241912f, -0.90096886790241912f, -0.22252093395631440f,
                                   0.62348980185873353f};
    static constexpr float s[7] = {0.0f, 0.78183148246802981f, 0.97492791218182361f,
                                   0.43388373911755812f, -0.43388373911755812f, -0.97492791218182361f,
                                   -0.78183148246802981f};
};
template <bool INV>
struct SDft<3, INV> : SDftOdd<3, INV> {};
template <bool INV>
struct SDft<7, INV> : SDftOdd<7, INV> {};
template <bool INV>
struct SDft<5, INV> : SDftOdd<5, INV> {};

// ---- compile-time radix plan -----------------------------------------------
constexpr int pick_radix(int rem, int E) {
    return (rem % 8 == 0 && E % 8 == 0)   ? 8
           : (rem % 4 == 0 && E % 4 == 0) ? 4
           : (rem % 2 == 0 && E % 2 == 0) ? 2
           : (rem % 3 == 0 && E % 3 == 0) ? 3
           : (rem % 5 == 0 && E % 5 == 0) ? 5
           : (rem % 7 == 0 && E % 7 == 0) ? 7
                                          : 0;
}
constexpr int rem_at(int L, int E, int s) {
    int rem = L;
    for (int i = 0; i < s; ++i) rem /= pick_radix(rem, E);
    return rem;
}
constexpr int nstages(int L, int E) {
    int rem = L, n = 0;
    while (rem > 1) {
        const int r = pick_radix(rem, E);
        if (r == 0) return -1;
        rem /= r;
        ++n;
    }
    return n;
}

template <int L_, int E_, bool INV_>
struct Fft {
    static constexpr int L = L_, E = E_, TL = L_ / E_;
    static constexpr bool INV = INV_;
    static constexpr int NST = nstages(L_, E_);
    static_assert(NST > 0, "no radix plan for this (L, E)");
    template <int S>
    static constexpr int R() { return pick_radix(rem_at(L, E, S), E); }
    template <int S>
    static constexpr int Ns() { return L / rem_at(L, E, S); }
    // input position of register element i = b*R + q in stage S
    template <int S>
    static __device__ __forceinline__ int in_pos(int u, int i) {
        constexpr int Rr = R<S>();
        return u + TL * (i / Rr) + (i % Rr) * (L / Rr);
    }
    // output position of register element i after stage S
    template <int S>
    static __device__ __forceinline__ int out_pos(int u, int i) {
        constexpr int Rr = R<S>(), N = Ns<S>();
        const int j = u + TL * (i / Rr);
        const int k = j % N;
        return (j - k) * Rr + k + (i % Rr) * N;
    }
    // twiddles and butterflies of stage S on the registers
    template <int S>
    static __device__ __forceinline__ void bfly(float2 (&v)[E], int u, const float2 *__restrict__ tw) {
        constexpr int Rr = R<S>(), N = Ns<S>(), NB = E / Rr, TS = L / (N * Rr);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (N > 1) {
                const int k = (u + TL * b) % N;
#pragma unroll
                for (int q = 1; q < Rr; ++q) {
                    float2 t = tw[q * k * TS];
                    if (INV) t.y = -t.y;
                    v[b * Rr + q] = cmul(v[b * Rr + q], t);
                }
            }
            SDft<Rr, INV>::run(&v[b * Rr]);
        }
    }
};

// Runs stages S..NST-1.  `lds_idx(pos)` maps a line position to its LDS
// index; `sink(i, pos, value)` consumes the last stage's outputs.
template <class F, int S>
struct Stages {
    template <class LdsIdx, class Sink>
    static __device__ __forceinline__ void run(float2 (&v)[F::E], int u, const float2 *tw, float2 *lds,
                                               LdsIdx lds_idx, Sink sink) {
        F::template bfly<S>(v, u, tw);
        if constexpr (S + 1 < F::NST) {
            if (S > 0) __syncthreads();  // stage S's LDS reads are done everywhere
#pragma unroll
            for (int i = 0; i < F::E; ++i) lds[lds_idx(F::template out_pos<S>(u, i))] = v[i];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < F::E; ++i) v[i] = lds[lds_idx(F::template in_pos<S + 1>(u, i))];
            Stages<F, S + 1>::run(v, u, tw, lds, lds_idx, sink);
        } else {
#pragma unroll
            for (int i = 0; i < F::E; ++i) sink(i, F::template out_pos<S>(u, i), v[i]);
        }
    }
};

// image index of line position p for a line of n values centred at r = 0
// (r = j - floor(n/2) sits at p = r mod L); -1 for zero-padding positions
template <int L>
__device__ __forceinline__ int pos_to_img(int p, int n) {
    const int h = n / 2;
    if (p < n - h) return p + h;
    if (p >= L - h) return p - L + h;
    return -1;
}

// k_cols: channel of the o-th line group in processing order: input channel
// (the return value), output channel `oo` and whether it is derived (scaled
// by r^[0]).  With DER the groups run pair by pair, [unweighted, r^[0],
// r^[1], ...], so that the derived channel re-reads its source while that
// is still in cache; see KbnMidPassArgs::dsplit (k_cols_pf orders its tiles
// with der_tile instead).
template <bool DER>
__device__ __forceinline__ int64_t col_map(const KbnMidPassArgs &a, int64_t o, int64_t &oo, bool &der) {
    der = false;
    oo = o;
    if constexpr (DER) {
        const int64_t cc = o / (a.dnw + 1);
        const int k = (int)(o - cc * (a.dnw + 1));
        if (k == 0) {
            oo = cc;
            return cc;
        }
        oo = a.dsplit + cc * a.dnw + (k - 1);
        der = k == 1;
        return der ? cc : oo;
    }
    return o;
}

// Inputs of the E register elements of one column line at the stage-0
// positions.  HALF (forward passes whose input is an image axis zero-padded
// to twice its length, K = 2N as on the sigma = 2 grids, with a stage-0
// radix divisible by 4): the element index alone says which positions hold
// image rows, so the others are zero without an address, a test or a load
// (half the elements) and the row offset is a constant.  DER && der: each
// row r is scaled by r - nin / 2 (the derived r^[0] channel).
template <class F, bool HALF, bool DER>
__device__ __forceinline__ void col_load(const KbnMidPassArgs &a, const float2 *in, int u, bool col_ok, bool der,
                                         float2 (&w)[F::E]) {
    constexpr int L = F::L, E = F::E;
    if constexpr (HALF) {
        constexpr int R0 = F::template R<0>();
        static_assert(R0 % 4 == 0, "HALF needs a stage-0 radix divisible by 4");
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int q = i % R0;
            if (q < R0 / 4 || q >= 3 * R0 / 4) {
                const int p = F::template in_pos<0>(u, i);
                const int r = q < R0 / 4 ? p + L / 4 : p - 3 * L / 4;
                w[i] = col_ok ? in[(int64_t)r * a.inner] : make_float2(0.f, 0.f);
                if (DER && der) {
                    const float f = (float)(r - L / 4);
                    w[i] = make_float2(w[i].x * f, w[i].y * f);
                }
            } else {
                w[i] = make_float2(0.f, 0.f);
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int p = F::template in_pos<0>(u, i);
            const int r = a.pad_in ? pos_to_img<L>(p, a.nin) : p;
            w[i] = (col_ok && r >= 0) ? in[(int64_t)r * a.inner] : make_float2(0.f, 0.f);
            if (DER && der) {
                const float f = (float)(r - a.nin / 2);
                w[i] = make_float2(w[i].x * f, w[i].y * f);
            }
        }
    }
}

// the HALF load applies to a forward pass of length L (stage-0 radix
// divisible by 4; an inverse pass cropping its output the same way measured
// slower, 0.190 -> 0.205 ms on the 256-image step)
template <int L, int E>
constexpr bool half_ok() {
    return Fft<L, E, false>::template R<0>() % 4 == 0;
}

// ---- strided pass along a non-last axis -------------------------------------
// lines = LINES adjacent columns; LDS layout [position][column] (column fastest).
// k_cols transforms one column tile per workgroup.  k_cols_pf walks over
// column tiles with a grid stride and loads the next tile's inputs into
// registers before transforming the current one, so the loads of one tile
// overlap the LDS stages of the previous (the grid holds only as many
// workgroups as fit on the device at once); it needs about twice the
// registers, so it is used only where it measured faster.
template <int L, int E, bool INV, int NT, bool DER = false, bool HALF = false>
__global__ void __launch_bounds__(NT) k_cols(KbnMidPassArgs a, const float2 *__restrict__ tw) {
    using F = Fft<L, E, INV>;
    static_assert(!(INV && (DER || HALF)), "derived channels and the HALF load are forward forms");
    static_assert(NT % F::TL == 0, "a workgroup holds whole lines");
    constexpr int LINES = NT / F::TL;
    extern __shared__ float2 lds[];  // [L][LINES], dynamic (may exceed 64 KiB)
    const int l = threadIdx.x % LINES;
    const int u = threadIdx.x / LINES;
    const int ntile = (a.inner + LINES - 1) / LINES;
    const int64_t o = blockIdx.x / ntile;
    const int c0 = (int)(blockIdx.x - o * ntile) * LINES;
    const bool col_ok = c0 + l < a.inner;
    bool der;
    int64_t oo;
    const int64_t oi = col_map<DER>(a, o, oo, der);
    const float2 *in = a.in + (oi * a.nin) * (int64_t)a.inner + c0 + l;
    float2 *out = a.out + (oo * a.nout) * (int64_t)a.inner + c0 + l;
    float2 v[E];
    col_load<F, HALF, DER>(a, in, u, col_ok, der, v);
    auto lds_idx = [](int pos) { return pos * LINES; };
    float2 *ldsl = lds + l;
    auto sink = [&](int, int pos, float2 val) {
        const int r = a.crop_out ? pos_to_img<L>(pos, a.nout) : pos;
        if (col_ok && r >= 0) out[(int64_t)r * a.inner] = val;
    };
    Stages<F, 0>::run(v, u, tw, ldsl, lds_idx, sink);
}

// Tile t of the persistent column pass with a derived channel: input and
// output channel, first column and, for unweighted and derived tiles, the
// index q of the (pair, column tile) they share (-1 for the others).  The
// first 2P tiles (P = pairs x column tiles) come in blocks of 2G (G = grid
// size): G unweighted tiles, then the derived tiles of the same q, so that
// a workgroup striding by G meets each derived tile right after its source
// (in the last, shorter block the twin is loaded again); the weighted
// channels w = 1 .. dnw-1 follow in channel order.
// (32-bit: the launcher takes this form only below 2^31 tiles)
__device__ __forceinline__ void der_tile(const KbnMidPassArgs &a, int t, int G, int ntile, int lines, int64_t &oi,
                                         int64_t &oo, int &c0, bool &der, int &q) {
    const int P = (int)a.dsplit * ntile;
    int ct;
    if (t < 2 * P) {
        const int base = (t / (2 * G)) * G;
        const int w = t - 2 * base;
        const int rem = min(G, P - base);
        der = w >= rem;
        q = base + (der ? w - rem : w);
        const int cc = q / ntile;
        ct = q - cc * ntile;
        oi = cc;
        oo = der ? a.dsplit + (int64_t)cc * a.dnw : cc;
    } else {
        const int r = t - 2 * P;
        const int wq = r / ntile;
        ct = r - wq * ntile;
        const int cc = wq / (a.dnw - 1);
        oi = oo = a.dsplit + (int64_t)cc * a.dnw + 1 + (wq - cc * (a.dnw - 1));
        der = false;
        q = -1;
    }
    c0 = ct * lines;
}

template <int L, int E, bool INV, int NT, bool DER = false, bool HALF = false>
__global__ void __launch_bounds__(NT) k_cols_pf(KbnMidPassArgs a, const float2 *__restrict__ tw) {
    using F = Fft<L, E, INV>;
    static_assert(!(INV && (DER || HALF)), "derived channels and the HALF load are forward forms");
    static_assert(NT % F::TL == 0, "a workgroup holds whole lines");
    constexpr int LINES = NT / F::TL;
    extern __shared__ float2 lds[];  // [L][LINES], dynamic
    const int l = threadIdx.x % LINES;
    const int u = threadIdx.x / LINES;
    const int ntile = (a.inner + LINES - 1) / LINES;
    const int64_t total = a.outer * ntile;
    // tile t -> input channel oi, output channel oo, first column c0
    auto tile = [&](int64_t t, int64_t &oi, int64_t &oo, int &c0, bool &der, int &q) {
        if constexpr (DER) {
            der_tile(a, (int)t, (int)gridDim.x, ntile, LINES, oi, oo, c0, der, q);
        } else {
            oi = oo = t / ntile;
            c0 = (int)(t - oi * ntile) * LINES;
            der = false;
            q = -1;
        }
    };
    // r^[0] of the image row of register element i
    auto rweight = [&](int i) {
        const int r = pos_to_img<L>(F::template in_pos<0>(u, i), a.nin);
        return (float)(r - a.nin / 2);
    };
    auto load = [&](int64_t oi, int c0, bool der, float2 (&w)[E]) {
        const bool col_ok = c0 + l < a.inner;
        const float2 *in = a.in + (oi * a.nin) * (int64_t)a.inner + c0 + l;
        col_load<F, HALF, DER>(a, in, u, col_ok, der, w);
    };
    float2 nv[E];
    int64_t t = blockIdx.x;
    // tile t's channels and column, then the next tile's
    int64_t oi = 0, oo = 0;
    int c0 = 0, q = -1;
    bool der = false;
    if (t < total) {
        tile(t, oi, oo, c0, der, q);
        load(oi, c0, der, nv);
    }
    auto lds_idx = [](int pos) { return pos * LINES; };
    float2 *ldsl = lds + l;
    for (; t < total; t += gridDim.x) {
        float2 v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = nv[i];
        const int64_t co = oo;
        const int cc0 = c0;
        const int64_t tn = t + gridDim.x;
        if (tn < total) {
            const int pq = q;
            const bool pder = der;
            tile(tn, oi, oo, c0, der, q);
            // the next tile derived from this one: scale the values in
            // registers instead of reading them again
            const bool twin = DER && !pder && pq >= 0 && der && q == pq;
            if (twin) {
#pragma unroll
                for (int i = 0; i < E; ++i) {
                    const float f = rweight(i);
                    nv[i] = make_float2(v[i].x * f, v[i].y * f);
                }
            } else {
                load(oi, c0, der, nv);
            }
        }
        if (t != (int64_t)blockIdx.x) __syncthreads();  // the previous tile's LDS reads are done
        const bool col_ok = cc0 + l < a.inner;
        float2 *out = a.out + (co * a.nout) * (int64_t)a.inner + cc0 + l;
        auto sink = [&](int, int pos, float2 val) {
            const int r = a.crop_out ? pos_to_img<L>(pos, a.nout) : pos;
            if (col_ok && r >= 0) out[(int64_t)r * a.inner] = val;
        };
        Stages<F, 0>::run(v, u, tw, ldsl, lds_idx, sink);
    }
}

// ---- forward first pass along the last axis (with prologue) ----------------
// LDS layout [line][position]
template <int L, int E, int NT>
__global__ void __launch_bounds__(NT) k_rows_first(KbnFirstPassArgs a, const float2 *__restrict__ tw) {
    using F = Fft<L, E, false>;
    static_assert(NT % F::TL == 0, "a workgroup holds whole lines");
    constexpr int LINES = NT / F::TL;
    __shared__ float2 lds[L * LINES];
    __shared__ float2 twl[L];
    for (int i = threadIdx.x; i < L; i += NT) twl[i] = tw[i];
    const int li = threadIdx.x / F::TL;
    const int u = threadIdx.x % F::TL;
    const int64_t line = (int64_t)blockIdx.x * LINES + li;
    const bool line_ok = line < a.nlines;
    const int Nl = a.Nl;
    float2 v[E];
    // per-line constants
    int64_t xrow = 0, srow = 0;
    float lf = 0.f;
    int wsel = -1;
    int64_t oline = line;  // output line
    if (line_ok) {
        const int64_t ch = line / a.R0;
        const int row = (int)(line - ch * a.R0);
        int64_t cc;
        if (a.nplain > 0) {  // forward plus omega-Jacobian layout (D >= 2)
            if (ch < a.nplain) {
                cc = ch;
            } else {
                const int64_t q = ch - a.nplain;
                cc = q / (a.D - 1);
                wsel = 1 + (int)(q - cc * (a.D - 1));
                oline = (a.nplain + cc * a.D + wsel) * a.R0 + row;
            }
        } else {
            cc = ch / a.nw;
            wsel = a.weighted ? (int)(ch - cc * a.nw) : -1;
        }
        const int c = (int)(cc % a.C);
        const int64_t bl = cc / a.C;
        xrow = (bl * a.R0 + row) * (int64_t)Nl;
        srow = ((int64_t)c * a.R0 + row) * Nl;
        float f = 1.f;
        int rem = row;
        for (int d = a.D - 2; d >= 0; --d) {
            const int id = rem % a.N[d];
            rem /= a.N[d];
            f *= a.deap[d][id];
            if (wsel == d) f *= (float)(id - a.N[d] / 2);
        }
        lf = f;
    }
    const float *deap_l = a.deap[a.D - 1];
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int p = F::template in_pos<0>(u, i);
        const int j = pos_to_img<L>(p, Nl);
        float2 x = make_float2(0.f, 0.f);
        if (line_ok && j >= 0) {
            x = a.x[xrow + j];
            float f = lf * deap_l[j];
            if (wsel == a.D - 1) f *= (float)(j - Nl / 2);
            if (a.smaps) x = cmul(x, a.smaps[srow + j]);
            x = make_float2(x.x * f, x.y * f);
        }
        v[i] = x;
    }
    __syncthreads();  // twiddles in LDS
    float2 *out = a.out + oline * L;
    auto lds_idx = [](int pos) { return pos; };
    float2 *ldsl = lds + li * L;
    auto sink = [&](int, int pos, float2 val) {
        if (line_ok) out[pos] = val;
    };
    Stages<F, 0>::run(v, u, twl, ldsl, lds_idx, sink);
}

// ---- last inverse pass along the last axis (crop, scaling, coil sum) -------
// ONE: a single coil (C = 1, with or without a map): each value is weighted
// and stored as the last stage produces it, with no coil accumulators.
template <int L, int E, int NT, bool ONE>
__global__ void __launch_bounds__(NT) k_rows_last_adj(KbnLastAdjArgs a, const float2 *__restrict__ tw) {
    using F = Fft<L, E, true>;
    static_assert(NT % F::TL == 0, "a workgroup holds whole lines");
    constexpr int LINES = NT / F::TL;
    __shared__ float2 lds[L * LINES];
    __shared__ float2 twl[L];
    for (int i = threadIdx.x; i < L; i += NT) twl[i] = tw[i];
    const int li = threadIdx.x / F::TL;
    const int u = threadIdx.x % F::TL;
    const int64_t line = (int64_t)blockIdx.x * LINES + li;
    const bool line_ok = line < a.nlines;
    const int Nl = a.Nl;
    int64_t bl = 0;
    int row = 0;
    float lf = 0.f;
    if (line_ok) {
        bl = line / a.R0;
        row = (int)(line - bl * a.R0);
        float f = 1.f;
        int rem = row;
        for (int d = a.D - 2; d >= 0; --d) {
            const int id = rem % a.N[d];
            rem /= a.N[d];
            f *= a.deap[d][id];
        }
        lf = f;
    }
    const float *deap_l = a.deap[a.D - 1];
    if constexpr (ONE) {
        const float2 *in = a.in + line * (int64_t)L;
        float2 v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int p = F::template in_pos<0>(u, i);
            v[i] = line_ok ? in[p] : make_float2(0.f, 0.f);
        }
        __syncthreads();  // twiddles in LDS
        const int cm = a.cmod > 0 ? (int)(bl % a.cmod) : 0;
        const float2 *srow = a.smaps ? a.smaps + ((int64_t)cm * a.R0 + row) * Nl : nullptr;
        float2 *x = a.x + line * Nl;
        auto lds_idx = [](int pos) { return pos; };
        float2 *ldsl = lds + li * L;
        auto sink = [&](int, int pos, float2 val) {
            const int j = pos_to_img<L>(pos, Nl);
            if (line_ok && j >= 0) {
                if (srow) val = cmulc(val, srow[j]);
                const float f = lf * deap_l[j];
                val = make_float2(val.x * f, val.y * f);
                if (a.accumulate) {
                    const float2 o = x[j];
                    val = make_float2(o.x + val.x, o.y + val.y);
                }
                x[j] = val;
            }
        };
        Stages<F, 0>::run(v, u, twl, ldsl, lds_idx, sink);
        return;
    }
    float2 acc[E];
#pragma unroll
    for (int i = 0; i < E; ++i) acc[i] = make_float2(0.f, 0.f);
    __syncthreads();  // twiddles in LDS
    for (int c = 0; c < a.C; ++c) {
        const float2 *in = a.in + (((bl * a.C + c) * a.R0) + row) * (int64_t)L;
        float2 v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int p = F::template in_pos<0>(u, i);
            v[i] = line_ok ? in[p] : make_float2(0.f, 0.f);
        }
        if (c > 0) __syncthreads();  // previous coil's last LDS reads are done
        const int cm = a.cmod > 0 ? (int)(bl % a.cmod) : c;
        const float2 *srow = a.smaps ? a.smaps + ((int64_t)cm * a.R0 + row) * Nl : nullptr;
        auto lds_idx = [](int pos) { return pos; };
        float2 *ldsl = lds + li * L;
        auto sink = [&](int i, int pos, float2 val) {
            const int j = pos_to_img<L>(pos, Nl);
            if (line_ok && j >= 0) {
                if (srow) val = cmulc(val, srow[j]);
                const float f = lf * deap_l[j];
                acc[i].x += val.x * f;
                acc[i].y += val.y * f;
            }
        };
        Stages<F, 0>::run(v, u, twl, ldsl, lds_idx, sink);
    }
    // write: register element i of the last stage holds line position out_pos
    float2 *x = a.x + line * Nl;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int pos = F::template out_pos<F::NST - 1>(u, i);
        const int j = pos_to_img<L>(pos, Nl);
        if (line_ok && j >= 0) {
            if (a.accumulate) {
                const float2 o = x[j];
                x[j] = make_float2(o.x + acc[i].x, o.y + acc[i].y);
            } else {
                x[j] = acc[i];
            }
        }
    }
}

// Elements per thread for each specialised length: rows (last axis) and
// columns (strided axes, at most 64 KiB of LDS per workgroup).  Every radix
// of a length's plan must divide E (radices 8, 4, 2, 3, 5), L / E threads
// serve one line and a workgroup holds whole lines: 400 = 2^4 5^2 takes
// E = 20 (radices 4,4,5,5) with 20 threads per line in 320-thread
// workgroups; 480 = 2^5 3 5 takes E = 60 (4,4,2,3,5) with 128 threads.
// Per-length configuration: elements per thread of the row and column
// passes (every radix of the length's plan must divide them, so lengths with
// factors 2, 3 and 5 take 30 and those with 2, 3 and 7 take 42) and, for
// lengths whose line does not divide 256 threads, the lines (row passes) or
// columns (column passes) a workgroup holds, within 64 KB of LDS (80 KB for
// the 16 columns of 640, which read whole 128-byte row segments: 28% faster
// than 8 columns, while 768 with 16 columns, 96 KB, fits one workgroup per
// CU and loses); 0 keeps the tuned thread counts of row_nt / col_nt.  Row passes are LDS-occupancy
// bound, so they take the smaller E where a length allows two.
struct FftLen {
    int L, re, ce, rl, cl;
};
constexpr FftLen kFftLens[] = {
    {128, 8, 8, 0, 0},     {160, 10, 20, 0, 0},   {192, 12, 12, 0, 0},   {200, 20, 20, 8, 16},
    {256, 8, 16, 0, 0},    {270, 30, 30, 16, 16}, {288, 12, 24, 8, 16},  {300, 30, 30, 16, 16},
    {320, 10, 20, 0, 0},   {324, 12, 12, 8, 8},   {360, 30, 30, 16, 16}, {384, 12, 24, 0, 0},
    {392, 14, 28, 8, 16},
    {400, 10, 20, 0, 0},   {432, 12, 24, 8, 16},  {448, 28, 28, 8, 16},  {450, 30, 30, 8, 16},
    {480, 60, 60, 0, 0},   {486, 18, 18, 8, 8},   {500, 20, 20, 8, 8},   {504, 42, 42, 8, 16},
    {512, 8, 16, 0, 0},    {540, 30, 30, 8, 8},   {576, 12, 24, 8, 8},   {588, 42, 42, 8, 8},
    {600, 30, 30, 8, 8},   {640, 10, 20, 0, 16},  {648, 24, 24, 8, 8},   {672, 42, 42, 8, 8},
    {686, 14, 14, 8, 8},   {720, 30, 30, 8, 8},   {750, 30, 30, 8, 8},   {756, 42, 42, 8, 8},
    {768, 24, 24, 0, 0},   {800, 20, 20, 8, 8},   {1024, 16, 32, 0, 0},
};
constexpr FftLen fft_len(int L) {
    for (const FftLen &f : kFftLens)
        if (f.L == L) return f;
    return FftLen{L, 0, 0, 0, 0};
}
constexpr int row_e(int L) { return fft_len(L).re; }
constexpr int col_e(int L) { return fft_len(L).ce; }
// threads per row-pass workgroup (whole lines of L / E threads each)
constexpr int row_nt(int L) {
    return fft_len(L).rl ? fft_len(L).rl * (L / row_e(L)) : L == 400 ? 320 : L == 480 ? 128 : KBN_BLOCK;
}
// threads per column-pass workgroup (512 for L = 512: 16 columns of 32
// threads, 64 KB of LDS, measured faster than 256 threads with E = 32)
constexpr int col_nt(int L) {
    return fft_len(L).cl ? fft_len(L).cl * (L / col_e(L))
           : L == 512    ? 512
           : L == 400    ? 320
           : L == 480    ? 128
                         : KBN_BLOCK;
}

// workgroups of a kernel that can be resident on the current device at once
template <class K>
int64_t resident_blocks(K kernel, int nt, size_t lds) {
    int nb = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, nt, lds) != hipSuccess || nb < 1) nb = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 1;
    return (int64_t)nb * cus;
}

// column passes that load ahead (L = 512: 0.65 -> 0.45 ms forward, 0.22 ->
// 0.19 ms inverse for 256 images of 512 x 512 on MI355X; 128 and 256: 3-8%);
// the longer lengths keep more elements per thread and would spill
constexpr bool col_pf(int L) { return L == 128 || L == 256 || L == 512; }

// a kernel whose dynamic LDS exceeds the default 64 KiB opts in (once)
template <class K>
hipError_t allow_lds(K kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// one forward column-pass launch (the persistent form where col_pf(L))
template <int L, bool DER, bool HALF>
hipError_t launch_cols_fwd(const KbnMidPassArgs &a, const float2 *tw, int64_t total, hipStream_t s) {
    constexpr int E = col_e(L);
    constexpr int NT = col_nt(L);
    constexpr size_t LDS = sizeof(float2) * L * (NT / (L / E));
    if constexpr (col_pf(L)) {
        static const hipError_t ok = allow_lds(k_cols_pf<L, E, false, NT, DER, HALF>, LDS);
        if (ok != hipSuccess) return ok;
        static const int64_t cap = resident_blocks(k_cols_pf<L, E, false, NT, DER, HALF>, NT, LDS);
        k_cols_pf<L, E, false, NT, DER, HALF><<<dim3((unsigned)std::min<int64_t>(total, cap)), dim3(NT), LDS, s>>>(a, tw);
    } else {
        static const hipError_t ok = allow_lds(k_cols<L, E, false, NT, DER, HALF>, LDS);
        if (ok != hipSuccess) return ok;
        k_cols<L, E, false, NT, DER, HALF><<<dim3((unsigned)total), dim3(NT), LDS, s>>>(a, tw);
    }
    return hipGetLastError();
}

// one inverse column-pass launch
template <int L>
hipError_t launch_cols_inv(const KbnMidPassArgs &a, const float2 *tw, int64_t total, hipStream_t s) {
    constexpr int E = col_e(L);
    constexpr int NT = col_nt(L);
    constexpr size_t LDS = sizeof(float2) * L * (NT / (L / E));
    if constexpr (col_pf(L)) {
        static const hipError_t ok = allow_lds(k_cols_pf<L, E, true, NT>, LDS);
        if (ok != hipSuccess) return ok;
        static const int64_t cap = resident_blocks(k_cols_pf<L, E, true, NT>, NT, LDS);
        k_cols_pf<L, E, true, NT><<<dim3((unsigned)std::min<int64_t>(total, cap)), dim3(NT), LDS, s>>>(a, tw);
    } else {
        static const hipError_t ok = allow_lds(k_cols<L, E, true, NT>, LDS);
        if (ok != hipSuccess) return ok;
        k_cols<L, E, true, NT><<<dim3((unsigned)total), dim3(NT), LDS, s>>>(a, tw);
    }
    return hipGetLastError();
}

template <int L>
hipError_t launch_cols(const KbnMidPassArgs &a, const float2 *tw, int inverse, hipStream_t s) {
    constexpr int E = col_e(L);
    constexpr int NT = col_nt(L);
    constexpr int LINES = NT / (L / E);
    const int64_t ntile = (a.inner + LINES - 1) / LINES;
    const int64_t total = a.outer * ntile;
    if (total <= 0) return hipSuccess;
    const bool der = a.dsplit > 0;
    if (der && (inverse || !a.pad_in || a.dnw < 2 || a.outer != a.dsplit * (a.dnw + 1) || total > INT_MAX / 2))
        return hipErrorInvalidValue;
    if (!inverse) {
        if constexpr (half_ok<L, E>()) {
            if (a.pad_in && 2 * a.nin == L)
                return der ? launch_cols_fwd<L, true, true>(a, tw, total, s)
                           : launch_cols_fwd<L, false, true>(a, tw, total, s);
        }
        return der ? launch_cols_fwd<L, true, false>(a, tw, total, s) : launch_cols_fwd<L, false, false>(a, tw, total, s);
    }
    return launch_cols_inv<L>(a, tw, total, s);
}

template <int L>
hipError_t launch_rows_first(const KbnFirstPassArgs &a, const float2 *tw, hipStream_t s) {
    constexpr int E = row_e(L);
    constexpr int NT = row_nt(L);
    constexpr int LINES = NT / (L / E);
    const dim3 grid((unsigned)((a.nlines + LINES - 1) / LINES));
    k_rows_first<L, E, NT><<<grid, dim3(NT), 0, s>>>(a, tw);
    return hipGetLastError();
}

template <int L>
hipError_t launch_rows_last(const KbnLastAdjArgs &a, const float2 *tw, hipStream_t s) {
    constexpr int E = row_e(L);
    constexpr int NT = row_nt(L);
    constexpr int LINES = NT / (L / E);
    const dim3 grid((unsigned)((a.nlines + LINES - 1) / LINES));
    if (a.C == 1)
        k_rows_last_adj<L, E, NT, true><<<grid, dim3(NT), 0, s>>>(a, tw);
    else
        k_rows_last_adj<L, E, NT, false><<<grid, dim3(NT), 0, s>>>(a, tw);
    return hipGetLastError();
}

#define KBN_FAST_SIZES(X) \
    X(128) X(160) X(192) X(200) X(256) X(270) X(288) X(300) X(320) X(324) X(360) X(384) X(392) X(400) \
    X(432) X(448) X(450) X(480) X(486) X(500) X(504) X(512) X(540) X(576) X(588) X(600) X(640) X(648) \
    X(672) X(686) X(720) X(750) X(756) X(768) X(800) X(1024)
// the last adjoint pass keeps E accumulators besides the E values, which
// spills for 480 (E = 60), 504, 588, 756 (E = 42) and 800: those lengths
// take the generic last pass
#define KBN_FAST_LAST_SIZES(X) \
    X(128) X(160) X(192) X(200) X(256) X(270) X(288) X(300) X(320) X(324) X(360) X(384) X(392) X(400) \
    X(432) X(448) X(450) X(486) X(500) X(512) X(540) X(576) X(600) X(640) X(648) X(672) X(686) X(720) \
    X(750) X(768) X(1024)

}  // namespace

bool kbn_fast_fft_size(int L) {
    switch (L) {
#define KBN_CASE(n) case n:
        KBN_FAST_SIZES(KBN_CASE)
#undef KBN_CASE
        return true;
        default: return false;
    }
}

bool kbn_fast_last_size(int L) {
    switch (L) {
#define KBN_CASE(n) case n:
        KBN_FAST_LAST_SIZES(KBN_CASE)
#undef KBN_CASE
        return true;
        default: return false;
    }
}

hipError_t kbn_launch_fast_mid(const KbnMidPassArgs &a, int L, const float2 *tw, int inverse,
                               hipStream_t s) {
    switch (L) {
#define KBN_CASE(n) case n: return launch_cols<n>(a, tw, inverse, s);
        KBN_FAST_SIZES(KBN_CASE)
#undef KBN_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t kbn_launch_fast_first(const KbnFirstPassArgs &a, int L, const float2 *tw, hipStream_t s) {
    switch (L) {
#define KBN_CASE(n) case n: return launch_rows_first<n>(a, tw, s);
        KBN_FAST_SIZES(KBN_CASE)
#undef KBN_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t kbn_launch_fast_last(const KbnLastAdjArgs &a, int L, const float2 *tw, hipStream_t s) {
    switch (L) {
#define KBN_CASE(n) case n: return launch_rows_last<n>(a, tw, s);
        KBN_FAST_LAST_SIZES(KBN_CASE)
#undef KBN_CASE
        default: return hipErrorInvalidValue;
    }
}
