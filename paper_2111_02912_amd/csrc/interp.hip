// J-tap Kaiser-Bessel interpolation between the oversampled grid and the
// sample locations (appendix: a~_mn = sum_j u_j*(omega_m) s_n
// exp(-i gamma (k_m + j) n)), and its transpose.
//
// Taps: with u = omega K / (2 pi), k_start = floor(u - J/2) + 1 and taps
// k_start + j, j < J, at distances t_j = u - k_start - j in [-J/2, J/2);
// grid indices wrap modulo K.  The window psi(t) = I0(beta sqrt(1 -
// (2t/J)^2)) / I0(beta) is evaluated per tap by a degree-10 polynomial in
// x = 2 f - 1 (f = fractional position of u - J/2), fitted on the host.
//
// gather (type 2, forward operator): one thread per sorted sample, weights
// computed once and reused over all channels of its group.  Mode 1 fuses
// the omega-Jacobian epilogue of eq. (e,jac,Ax,v): for channel (b, c, d) the
// interpolated value z = [A(s_c x_b r^[d])]_m is folded into
// Im{z conj(v_{b,c,m})} and summed over the channels in registers.
//
// spread (type 1, adjoint operator): each workgroup owns one tile of the
// grid for a group of channels, accumulates every sample whose taps reach
// the tile into an LDS copy of the tile (LDS float atomics), then writes the
// tile with plain stores: every grid cell is written exactly once, so the
// grid needs neither zero-initialisation nor global atomics.
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

template <int D, int J, int MODE>
__global__ void __launch_bounds__(KBN_BLOCK) k_gather(KbnGeom g, KbnGatherArgs a, int cg) {
    const int64_t p = (int64_t)blockIdx.x * KBN_BLOCK + threadIdx.x;
    if (p >= a.M) return;
    const int q = a.order[p];
    const bool bad = p >= a.toff[g.ntiles];
    float w[D][J];
    int idx[D][J];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        int start;
        float f;
        tap_origin(J, a.cell[d * a.M + p], a.frac[d * a.M + p], start, f);
        kb_weights<J>(f, g.coef, w[d]);
#pragma unroll
        for (int j = 0; j < J; ++j) idx[d][j] = wrapk(start + j, g.K[d]);
    }
    // flatten the leading axes' strides into the index tables
    if (D >= 2) {
#pragma unroll
        for (int j = 0; j < J; ++j) idx[D - 2][j] *= g.K[D - 1];
    }
    if (D == 3) {
#pragma unroll
        for (int j = 0; j < J; ++j) idx[0][j] *= g.K[1] * g.K[2];
    }
    const int ch0 = blockIdx.y * cg;
    const int ch1 = min(ch0 + cg, a.nch);
    float jac[KBN_MAX_D] = {0.f, 0.f, 0.f};
    for (int ch = ch0; ch < ch1; ++ch) {
        const float2 *G = a.grid + (int64_t)ch * a.gsize;
        float2 acc = make_float2(0.f, 0.f);
        if (D == 1) {
#pragma unroll
            for (int j0 = 0; j0 < J; ++j0) {
                const float2 v = G[idx[0][j0]];
                acc.x = fmaf(w[0][j0], v.x, acc.x);
                acc.y = fmaf(w[0][j0], v.y, acc.y);
            }
        } else if (D == 2) {
#pragma unroll
            for (int j0 = 0; j0 < J; ++j0) {
                const float2 *row = G + idx[0][j0];
                float2 s = make_float2(0.f, 0.f);
#pragma unroll
                for (int j1 = 0; j1 < J; ++j1) {
                    const float2 v = row[idx[1][j1]];
                    s.x = fmaf(w[1][j1], v.x, s.x);
                    s.y = fmaf(w[1][j1], v.y, s.y);
                }
                acc.x = fmaf(w[0][j0], s.x, acc.x);
                acc.y = fmaf(w[0][j0], s.y, acc.y);
            }
        } else {
#pragma unroll
            for (int j0 = 0; j0 < J; ++j0) {
                float2 s1 = make_float2(0.f, 0.f);
#pragma unroll
                for (int j1 = 0; j1 < J; ++j1) {
                    const float2 *row = G + idx[0][j0] + idx[1][j1];
                    float2 s = make_float2(0.f, 0.f);
#pragma unroll
                    for (int j2 = 0; j2 < J; ++j2) {
                        const float2 v = row[idx[2][j2]];
                        s.x = fmaf(w[2][j2], v.x, s.x);
                        s.y = fmaf(w[2][j2], v.y, s.y);
                    }
                    s1.x = fmaf(w[1][j1], s.x, s1.x);
                    s1.y = fmaf(w[1][j1], s.y, s1.y);
                }
                acc.x = fmaf(w[0][j0], s1.x, acc.x);
                acc.y = fmaf(w[0][j0], s1.y, acc.y);
            }
        }
        if (MODE == 0) {
            const int64_t bc = ch;  // channel = b_local * C + c
            if (bad) acc = make_float2(__builtin_nanf(""), __builtin_nanf(""));
            a.y[bc * a.M + q] = acc;
        } else {
            const int wd = ch % a.nw;
            const int64_t bc = ch / a.nw;
            const float2 v = a.v[bc * a.M + q];
            jac[wd] += acc.y * v.x - acc.x * v.y;  // Im{acc conj(v)}
        }
    }
    if (MODE == 1) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            float val = bad ? __builtin_nanf("") : jac[d];
            atomicAdd(&a.domega[(int64_t)q * D + d], val);
        }
    }
}

// Distinct tiles along one axis whose samples can reach [a0, a0 + te).
// A sample in cell c touches cells [c - lo, c + hi] (lo = J/2 - 1 and
// hi = J/2 for even J; lo = hi = J/2 for odd J, covering both tap origins),
// so the contributing cells are [a0 - hi, a0 + te - 1 + lo], modulo K.
__device__ __forceinline__ int axis_neighbours(int a0, int te, int K, int T, int J, int *out) {
    const int lo = (J & 1) ? J / 2 : J / 2 - 1;
    const int hi = J / 2;
    int cur = a0 - hi;
    if (cur < 0) cur += K;
    int remaining = te + lo + hi;
    int n = 0;
    while (remaining > 0 && n < 4) {
        const int t = cur / T;
        bool seen = false;
        for (int i = 0; i < n; ++i) seen |= out[i] == t;
        if (!seen) out[n++] = t;
        int tend = (t + 1) * T;
        if (tend > K) tend = K;
        remaining -= tend - cur;
        cur = tend == K ? 0 : tend;
    }
    return n;
}

template <int D, int J>
__global__ void __launch_bounds__(KBN_BLOCK) k_spread(KbnGeom g, KbnSpreadArgs a, int cg) {
    extern __shared__ float lacc[];  // [cg][te_0]...[te_{D-1}] complex, interleaved
    const int tile = blockIdx.x;
    int tc[KBN_MAX_D], a0[KBN_MAX_D], te[KBN_MAX_D];
    {
        int rem = tile;
        for (int d = D - 1; d >= 0; --d) {
            tc[d] = rem % g.nt[d];
            rem /= g.nt[d];
            a0[d] = tc[d] * g.T[d];
            te[d] = min(g.T[d], g.K[d] - a0[d]);
        }
    }
    int tsize = 1;
    for (int d = 0; d < D; ++d) tsize *= te[d];
    const int ch0 = blockIdx.y * cg;
    const int nchg = min(cg, a.nch - ch0);
    for (int i = threadIdx.x; i < 2 * nchg * tsize; i += KBN_BLOCK) lacc[i] = 0.f;
    __syncthreads();

    int nb[KBN_MAX_D][4], nn[KBN_MAX_D];
    for (int d = 0; d < D; ++d) nn[d] = axis_neighbours(a0[d], te[d], g.K[d], g.T[d], J, nb[d]);
    int ncombo = 1;
    for (int d = 0; d < D; ++d) ncombo *= nn[d];
    for (int cmb = 0; cmb < ncombo; ++cmb) {
        int rem = cmb, nt_id = 0;
        for (int d = 0; d < D; ++d) {
            const int i = rem % nn[d];
            rem /= nn[d];
            nt_id = nt_id * g.nt[d] + nb[d][i];
        }
        const int pbeg = a.toff[nt_id], pend = a.toff[nt_id + 1];
        for (int p = pbeg + threadIdx.x; p < pend; p += KBN_BLOCK) {
            int loc[D][J];
            unsigned mask[D];
            float f[D];
            bool any = true;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                int start;
                tap_origin(J, a.cell[d * a.M + p], a.frac[d * a.M + p], start, f[d]);
                int l0 = start - a0[d];
                if (l0 < 0) l0 += g.K[d];
                if (l0 < 0) l0 += g.K[d];
                mask[d] = 0u;
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    int l = l0 + j;
                    if (l >= g.K[d]) l -= g.K[d];
                    loc[d][j] = l;
                    if (l < te[d]) mask[d] |= 1u << j;
                }
                any = any && mask[d] != 0u;
            }
            if (!any) continue;
            float w[D][J];
#pragma unroll
            for (int d = 0; d < D; ++d) kb_weights<J>(f[d], g.coef, w[d]);
            const int q = a.order[p];
            for (int c = 0; c < nchg; ++c) {
                const float2 yv = a.y[(int64_t)(ch0 + c) * a.M + q];
                float *base = lacc + 2 * c * tsize;
                if (D == 1) {
#pragma unroll
                    for (int j0 = 0; j0 < J; ++j0) {
                        if (!(mask[0] >> j0 & 1u)) continue;
                        float *cell = base + 2 * loc[0][j0];
                        atomicAdd(cell, w[0][j0] * yv.x);
                        atomicAdd(cell + 1, w[0][j0] * yv.y);
                    }
                } else if (D == 2) {
#pragma unroll
                    for (int j0 = 0; j0 < J; ++j0) {
                        if (!(mask[0] >> j0 & 1u)) continue;
                        const float2 r0 = make_float2(w[0][j0] * yv.x, w[0][j0] * yv.y);
                        float *rowp = base + 2 * loc[0][j0] * te[1];
#pragma unroll
                        for (int j1 = 0; j1 < J; ++j1) {
                            if (!(mask[1] >> j1 & 1u)) continue;
                            float *cell = rowp + 2 * loc[1][j1];
                            atomicAdd(cell, w[1][j1] * r0.x);
                            atomicAdd(cell + 1, w[1][j1] * r0.y);
                        }
                    }
                } else {
#pragma unroll
                    for (int j0 = 0; j0 < J; ++j0) {
                        if (!(mask[0] >> j0 & 1u)) continue;
                        const float2 r0 = make_float2(w[0][j0] * yv.x, w[0][j0] * yv.y);
#pragma unroll
                        for (int j1 = 0; j1 < J; ++j1) {
                            if (!(mask[1] >> j1 & 1u)) continue;
                            const float2 r1 = make_float2(w[1][j1] * r0.x, w[1][j1] * r0.y);
                            float *rowp = base + 2 * (loc[0][j0] * te[1] + loc[1][j1]) * te[2];
#pragma unroll
                            for (int j2 = 0; j2 < J; ++j2) {
                                if (!(mask[2] >> j2 & 1u)) continue;
                                float *cell = rowp + 2 * loc[2][j2];
                                atomicAdd(cell, w[2][j2] * r1.x);
                                atomicAdd(cell + 1, w[2][j2] * r1.y);
                            }
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    // write the owned tile of every channel in the group
    for (int c = 0; c < nchg; ++c) {
        float2 *G = a.grid + (int64_t)(ch0 + c) * a.gsize;
        const float *src = lacc + 2 * c * tsize;
        for (int i = threadIdx.x; i < tsize; i += KBN_BLOCK) {
            int rem = i;
            int64_t off = 0, stride = 1;
            for (int d = D - 1; d >= 0; --d) {
                const int l = rem % te[d];
                rem /= te[d];
                off += (int64_t)(a0[d] + l) * stride;
                stride *= g.K[d];
            }
            G[off] = make_float2(src[2 * i], src[2 * i + 1]);
        }
    }
}

__global__ void k_fill(float *p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <int D, int J>
hipError_t gather_dj(const KbnGeom &g, const KbnGatherArgs &a, int mode, hipStream_t s) {
    if (a.M == 0 || a.nch == 0) return hipSuccess;
    // channel groups: keep whole (b, c) sets of weight channels together
    int cg = a.nch;
    const int64_t pblocks = (a.M + KBN_BLOCK - 1) / KBN_BLOCK;
    const int64_t want = 2048;  // workgroups to aim for
    if (pblocks * 1 < want) {
        int groups = (int)((want + pblocks - 1) / pblocks);
        if (groups > a.nch / a.nw) groups = a.nch / a.nw;
        if (groups < 1) groups = 1;
        cg = ((a.nch / a.nw + groups - 1) / groups) * a.nw;
    } else {
        cg = a.nw * ((8 + a.nw - 1) / a.nw);
        if (cg > a.nch) cg = a.nch;
    }
    const int ng = (a.nch + cg - 1) / cg;
    dim3 grid((unsigned)pblocks, (unsigned)ng);
    if (mode == 0)
        k_gather<D, J, 0><<<grid, dim3(KBN_BLOCK), 0, s>>>(g, a, cg);
    else
        k_gather<D, J, 1><<<grid, dim3(KBN_BLOCK), 0, s>>>(g, a, cg);
    return hipGetLastError();
}

template <int D, int J>
hipError_t spread_dj(const KbnGeom &g, const KbnSpreadArgs &a, hipStream_t s) {
    if (a.nch == 0) return hipSuccess;
    int tmax = 1;
    for (int d = 0; d < D; ++d) tmax *= g.T[d] < g.K[d] ? g.T[d] : g.K[d];
    const size_t per_ch = sizeof(float2) * (size_t)tmax;
    int cg = (int)((48 * 1024) / per_ch);
    if (cg < 1) cg = 1;
    if (cg > 8) cg = 8;
    if (cg > a.nch) cg = a.nch;
    const int ng = (a.nch + cg - 1) / cg;
    dim3 grid((unsigned)g.ntiles, (unsigned)ng);
    k_spread<D, J><<<grid, dim3(KBN_BLOCK), per_ch * cg, s>>>(g, a, cg);
    return hipGetLastError();
}

template <int D>
hipError_t gather_d(const KbnGeom &g, const KbnGatherArgs &a, int mode, hipStream_t s) {
    switch (g.J) {
        case 2: return gather_dj<D, 2>(g, a, mode, s);
        case 3: return gather_dj<D, 3>(g, a, mode, s);
        case 4: return gather_dj<D, 4>(g, a, mode, s);
        case 5: return gather_dj<D, 5>(g, a, mode, s);
        case 6: return gather_dj<D, 6>(g, a, mode, s);
        case 7: return gather_dj<D, 7>(g, a, mode, s);
        default: return gather_dj<D, 8>(g, a, mode, s);
    }
}

template <int D>
hipError_t spread_d(const KbnGeom &g, const KbnSpreadArgs &a, hipStream_t s) {
    switch (g.J) {
        case 2: return spread_dj<D, 2>(g, a, s);
        case 3: return spread_dj<D, 3>(g, a, s);
        case 4: return spread_dj<D, 4>(g, a, s);
        case 5: return spread_dj<D, 5>(g, a, s);
        case 6: return spread_dj<D, 6>(g, a, s);
        case 7: return spread_dj<D, 7>(g, a, s);
        default: return spread_dj<D, 8>(g, a, s);
    }
}

}  // namespace

hipError_t kbn_launch_gather(const KbnGeom &g, const KbnGatherArgs &a, int mode, hipStream_t s) {
    switch (g.D) {
        case 1: return gather_d<1>(g, a, mode, s);
        case 2: return gather_d<2>(g, a, mode, s);
        default: return gather_d<3>(g, a, mode, s);
    }
}

hipError_t kbn_launch_spread(const KbnGeom &g, const KbnSpreadArgs &a, hipStream_t s) {
    switch (g.D) {
        case 1: return spread_d<1>(g, a, s);
        case 2: return spread_d<2>(g, a, s);
        default: return spread_d<3>(g, a, s);
    }
}

hipError_t kbn_launch_fill(float *p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + KBN_BLOCK - 1) / KBN_BLOCK;
    k_fill<<<dim3((unsigned)blocks), dim3(KBN_BLOCK), 0, s>>>(p, n, v);
    return hipGetLastError();
}
