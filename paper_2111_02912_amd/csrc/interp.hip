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
// grid for a group of channels and sums every sample whose taps reach the
// tile (see k_spread_os), then writes the tile with plain stores: every grid
// cell is written exactly once, so the grid needs neither zero-initialisation
// nor atomics.
#include "kbn_internal.h"
#include "kbn_window.h"

#include <algorithm>
#include <cstdlib>

namespace {

// Staged gather: one workgroup per subproblem (<= KBN_SUB sorted points of
// one tile).  Channels are taken CP at a time (CP = 2 or 4): their grid
// regions (tile plus the tap reach) are loaded into LDS interleaved, with
// coalesced reads, and every thread interpolates its point for all CP
// channels from LDS, one 16-byte read per tap and channel pair.  With LA the
// region of the next CP channels is loaded into registers while the current
// ones are interpolated (each thread keeps the grid offsets of its region
// cells, computed once), so the grid reads overlap the interpolation.  Subproblems
// of the extra tile id ntiles hold the flagged points, whose outputs are NaN.
// Body of one workgroup: subproblem s, channel group gy (the kernel's
// blockIdx.x and blockIdx.y), regions staged in reg4.
template <int D, int J, int MODE, int CP, bool LA>
__device__ __forceinline__ void gather_staged_wg(const KbnGeom &g, const KbnGatherArgs &a, int cg, int s, int gy,
                                                 float4 *reg4) {
    constexpr int H = CP / 2;  // float4 (channel pairs) per region cell
    if (s >= *a.nsub) return;
    const int tile = a.subs[2 * s];
    const int p0 = a.subs[2 * s + 1];
    const int ch0 = gy * cg;
    const int ch1 = min(ch0 + cg, a.nch);
    const float qnan = __builtin_nanf("");
    if (tile == g.ntiles) {  // flagged points
        const int p = p0 + threadIdx.x;
        if (p < a.M) {
            const int q = a.order[p];
            if (MODE == 0) {
                for (int ch = ch0; ch < ch1; ++ch) a.y[(int64_t)ch * a.M + q] = make_float2(qnan, qnan);
            } else {
                float *part = a.part + (int64_t)gy * a.M * D;
                for (int d = 0; d < D; ++d) part[(int64_t)q * D + d] = qnan;
            }
        }
        return;
    }
    const int p1 = min(p0 + KBN_SUB, a.toff[tile + 1]);
    int o[D], E[D];
    {
        int rem = tile;
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            const int tc = rem % g.nt[d];
            rem /= g.nt[d];
            const int a0 = tc * g.T[d];
            const int te = min(g.T[d], g.K[d] - a0);
            o[d] = a0 - Reach<J>::LO;
            E[d] = te + Reach<J>::LO + Reach<J>::HI;
        }
    }
    int R = 1;
#pragma unroll
    for (int d = 0; d < D; ++d) R *= E[d];

    const int p = p0 + (int)threadIdx.x;
    const bool act = p < p1;
    int q = 0;
    float w[D][J];
    int base = 0;  // region offset of the point's first tap
    if (act) {
        q = a.order[p];
        int stride = 1;
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            int start;
            float f;
            tap_origin(J, a.cell[d * a.M + p], a.frac[d * a.M + p], start, f);
            kb_weights<J>(f, g.coef, w[d]);
            base += (start - o[d]) * stride;
            stride *= E[d];
        }
    }
    float jac[KBN_MAX_D] = {0.f, 0.f, 0.f};
    // LA: region cells of this thread and their grid offsets (the same for
    // every channel), and the next channel group's region loaded ahead
    constexpr int MAXC = LA ? (48 * 1024 / (CP * 8) + KBN_BLOCK - 1) / KBN_BLOCK : 1;
    int goff[MAXC];
    float4 pre[MAXC][H];
    auto fetch = [&](int chb) {
        const int nc = min(CP, ch1 - chb);
#pragma unroll
        for (int k = 0; k < MAXC; ++k) {
            const int i = (int)threadIdx.x + k * KBN_BLOCK;
#pragma unroll
            for (int h = 0; h < H; ++h) {
                float2 v0 = make_float2(0.f, 0.f), v1 = v0;
                if (i < R) {
                    if (2 * h < nc) v0 = a.grid[(int64_t)(chb + 2 * h) * a.gsize + goff[k]];
                    if (2 * h + 1 < nc) v1 = a.grid[(int64_t)(chb + 2 * h + 1) * a.gsize + goff[k]];
                }
                pre[k][h] = make_float4(v0.x, v0.y, v1.x, v1.y);
            }
        }
    };
    if constexpr (LA) {
#pragma unroll
        for (int k = 0; k < MAXC; ++k) {
            const int i = (int)threadIdx.x + k * KBN_BLOCK;
            int rem = i < R ? i : 0;
            int gi = 0, gstride = 1;
#pragma unroll
            for (int d = D - 1; d >= 0; --d) {
                const int e = rem % E[d];
                rem /= E[d];
                gi += wrapk(o[d] + e, g.K[d]) * gstride;
                gstride *= g.K[d];
            }
            goff[k] = gi;
        }
        if (ch0 < ch1) fetch(ch0);
    }
    for (int ch = ch0; ch < ch1; ch += CP) {
        const int nc = min(CP, ch1 - ch);
        if constexpr (LA) {
#pragma unroll
            for (int k = 0; k < MAXC; ++k) {
                const int i = (int)threadIdx.x + k * KBN_BLOCK;
                if (i < R) {
#pragma unroll
                    for (int h = 0; h < H; ++h) reg4[i * H + h] = pre[k][h];
                }
            }
        } else {
            for (int i = threadIdx.x; i < R; i += KBN_BLOCK) {
                int rem = i;
                int64_t gi = 0, gstride = 1;
#pragma unroll
                for (int d = D - 1; d >= 0; --d) {
                    const int e = rem % E[d];
                    rem /= E[d];
                    gi += (int64_t)wrapk(o[d] + e, g.K[d]) * gstride;
                    gstride *= g.K[d];
                }
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    const float2 v0 = 2 * h < nc ? a.grid[(int64_t)(ch + 2 * h) * a.gsize + gi] : make_float2(0.f, 0.f);
                    const float2 v1 =
                        2 * h + 1 < nc ? a.grid[(int64_t)(ch + 2 * h + 1) * a.gsize + gi] : make_float2(0.f, 0.f);
                    reg4[i * H + h] = make_float4(v0.x, v0.y, v1.x, v1.y);
                }
            }
        }
        // upstream values of this group (mode 1), read before the next group's loads
        float2 vv[CP];
#pragma unroll
        for (int k = 0; k < CP; ++k)
            vv[k] = (MODE == 1 && act && k < nc) ? a.v[(int64_t)((ch + k) / a.nw) * a.M + q] : make_float2(0.f, 0.f);
        __syncthreads();
        if constexpr (LA) {
            if (ch + CP < ch1) fetch(ch + CP);
        }
        if (act) {
            float4 acc[H];
#pragma unroll
            for (int h = 0; h < H; ++h) acc[h] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (D == 1) {
#pragma unroll
                for (int j0 = 0; j0 < J; ++j0) {
                    const float w0 = w[0][j0];
#pragma unroll
                    for (int h = 0; h < H; ++h) {
                        const float4 v = reg4[(base + j0) * H + h];
                        acc[h].x = fmaf(w0, v.x, acc[h].x);
                        acc[h].y = fmaf(w0, v.y, acc[h].y);
                        acc[h].z = fmaf(w0, v.z, acc[h].z);
                        acc[h].w = fmaf(w0, v.w, acc[h].w);
                    }
                }
            } else if (D == 2) {
                // rows one at a time: only one row's taps live in registers
#pragma unroll 1
                for (int j0 = 0; j0 < J; ++j0) {
                    const float4 *row = reg4 + (base + j0 * E[D - 1]) * H;
                    float4 t[H];
#pragma unroll
                    for (int h = 0; h < H; ++h) t[h] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                    for (int j1 = 0; j1 < J; ++j1) {
                        const float w1 = w[1][j1];
#pragma unroll
                        for (int h = 0; h < H; ++h) {
                            const float4 v = row[j1 * H + h];
                            t[h].x = fmaf(w1, v.x, t[h].x);
                            t[h].y = fmaf(w1, v.y, t[h].y);
                            t[h].z = fmaf(w1, v.z, t[h].z);
                            t[h].w = fmaf(w1, v.w, t[h].w);
                        }
                    }
                    const float w0 = w[0][j0];
#pragma unroll
                    for (int h = 0; h < H; ++h) {
                        acc[h].x = fmaf(w0, t[h].x, acc[h].x);
                        acc[h].y = fmaf(w0, t[h].y, acc[h].y);
                        acc[h].z = fmaf(w0, t[h].z, acc[h].z);
                        acc[h].w = fmaf(w0, t[h].w, acc[h].w);
                    }
                }
            } else {
#pragma unroll 1
                for (int j0 = 0; j0 < J; ++j0) {
                    float4 t1[H];
#pragma unroll
                    for (int h = 0; h < H; ++h) t1[h] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                    for (int j1 = 0; j1 < J; ++j1) {
                        const float4 *row = reg4 + (base + (j0 * E[1] + j1) * E[2]) * H;
                        float4 t[H];
#pragma unroll
                        for (int h = 0; h < H; ++h) t[h] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                        for (int j2 = 0; j2 < J; ++j2) {
                            const float w2 = w[2][j2];
#pragma unroll
                            for (int h = 0; h < H; ++h) {
                                const float4 v = row[j2 * H + h];
                                t[h].x = fmaf(w2, v.x, t[h].x);
                                t[h].y = fmaf(w2, v.y, t[h].y);
                                t[h].z = fmaf(w2, v.z, t[h].z);
                                t[h].w = fmaf(w2, v.w, t[h].w);
                            }
                        }
                        const float w1 = w[1][j1];
#pragma unroll
                        for (int h = 0; h < H; ++h) {
                            t1[h].x = fmaf(w1, t[h].x, t1[h].x);
                            t1[h].y = fmaf(w1, t[h].y, t1[h].y);
                            t1[h].z = fmaf(w1, t[h].z, t1[h].z);
                            t1[h].w = fmaf(w1, t[h].w, t1[h].w);
                        }
                    }
                    const float w0 = w[0][j0];
#pragma unroll
                    for (int h = 0; h < H; ++h) {
                        acc[h].x = fmaf(w0, t1[h].x, acc[h].x);
                        acc[h].y = fmaf(w0, t1[h].y, acc[h].y);
                        acc[h].z = fmaf(w0, t1[h].z, acc[h].z);
                        acc[h].w = fmaf(w0, t1[h].w, acc[h].w);
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < CP; ++k) {
                if (k >= nc) break;
                const int c = ch + k;
                const float ax = (k & 1) ? acc[k / 2].z : acc[k / 2].x;
                const float ay = (k & 1) ? acc[k / 2].w : acc[k / 2].y;
                if (MODE == 0) {
                    a.y[(int64_t)c * a.M + q] = make_float2(ax, ay);
                } else {
                    const float im = ay * vv[k].x - ax * vv[k].y;  // Im{acc conj(v)}
                    const int wd = c % a.nw;
#pragma unroll
                    for (int d = 0; d < D; ++d)
                        if (wd == d) jac[d] += im;
                }
            }
        }
        __syncthreads();
    }
    if (MODE == 1 && act) {
        float *part = a.part + (int64_t)gy * a.M * D;
#pragma unroll
        for (int d = 0; d < D; ++d) part[(int64_t)q * D + d] = jac[d];
    }
}

template <int D, int J, int MODE, int CP, bool LA>
__global__ void __launch_bounds__(KBN_BLOCK) k_gather_staged(KbnGeom g, KbnGatherArgs a, int cg) {
    extern __shared__ float4 reg4[];
    gather_staged_wg<D, J, MODE, CP, LA>(g, a, cg, blockIdx.x, blockIdx.y, reg4);
}

// The staged gathers of several plans in one launch: workgroup w belongs to
// the job i with start[i] <= w < start[i + 1] and is that job's workgroup
// (w - start[i]) mod blocks of channel group (w - start[i]) / blocks.
template <int D, int J, int MODE, int CP, bool LA>
__global__ void __launch_bounds__(KBN_BLOCK)
k_gather_multi(const KbnGatherJob *__restrict__ jobs, const int64_t *__restrict__ start, int njobs) {
    extern __shared__ float4 reg4[];
    const int64_t w = blockIdx.x;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    const KbnGatherJob &j = jobs[lo];
    const int64_t local = w - start[lo];
    gather_staged_wg<D, J, MODE, CP, LA>(j.g, j.a, j.cg, (int)(local % j.blocks), (int)(local / j.blocks), reg4);
}

// Direct gather (no staging): one thread per sorted point reads its taps from
// the grid in global memory; used when a staged region does not fit in LDS.
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
            const float im = acc.y * v.x - acc.x * v.y;  // Im{acc conj(v)}
#pragma unroll
            for (int d = 0; d < D; ++d)
                if (wd == d) jac[d] += im;
        }
    }
    if (MODE == 1) {
        float *part = a.part + (int64_t)blockIdx.y * a.M * D;
#pragma unroll
        for (int d = 0; d < D; ++d) part[(int64_t)q * D + d] = bad ? __builtin_nanf("") : jac[d];
    }
}

// LDS accumulator pitch of a tile axis: odd for every axis but the first,
// so that lanes stepping along any axis hit distinct LDS banks.
__host__ __device__ inline int acc_pitch(int d, int te) { return d == 0 ? te : (te | 1); }

// Channel plane stride (in float2) of the spread accumulator: padded so that
// consecutive planes start 12 LDS banks apart.
__host__ __device__ inline int spread_plane(int psize) { return psize + ((6 - psize) % 32 + 32) % 32; }

// Owner-computes spread.  Workgroup = (owner tile, channel group); the
// samples reaching the tile come from a precomputed list (index pass).  For a
// batch of list entries the workgroup stages in LDS each sample's local tap
// origin, its window weights and its k-space values; then every lane of a
// wave owns one (trailing tap, channel) pair and, entry after entry, adds its
// product into the tile accumulator with a plain LDS read-modify-write.  For
// one entry all lanes touch distinct cells, and waves own disjoint channels,
// so no two lanes ever update the same cell concurrently: no atomics, and a
// fixed accumulation order.
//   A = 1: lanes = (tap along the last axis) x (64 / J channels)
//   A = 2: lanes = (taps along the last two axes) x (64 / J^2 channels)
template <int D, int J, int A>
__global__ void __launch_bounds__(KBN_BLOCK) k_spread(KbnGeom g, KbnSpreadArgs a, int cw, int nwave) {
    constexpr int EB = KBN_SPREAD_EB;
    constexpr int LANES_TAP = A == 1 ? J : J * J;
    constexpr int NEG = -(1 << 28);                // offset of a tap outside the tile
    extern __shared__ float smem[];
    const int wk = blockIdx.y;                     // work item
    if (wk >= a.scounts[0]) return;
    const int tile = a.swork[4 * wk];
    const int slot = a.swork[4 * wk + 3];
    const int ngroup = nwave * cw;                 // channels per workgroup
    const int ch0 = blockIdx.x * ngroup;
    const int nchg = min(ngroup, a.nch - ch0);
    int a0[KBN_MAX_D], te[KBN_MAX_D], pt[KBN_MAX_D];
    {
        int rem = tile;
        for (int d = D - 1; d >= 0; --d) {
            const int tc = rem % g.nto[d];
            rem /= g.nto[d];
            a0[d] = tc * g.To[d];
            te[d] = min(g.To[d], g.K[d] - a0[d]);
            pt[d] = acc_pitch(d, te[d]);
        }
    }
    int psize = 1, tsize = 1;
    int stride[KBN_MAX_D];
    for (int d = D - 1; d >= 0; --d) {
        stride[d] = psize;
        psize *= pt[d];
        tsize *= te[d];
    }
    const int plane = spread_plane(psize);         // float2 per channel plane
    float2 *acc = reinterpret_cast<float2 *>(smem);
    // per staged entry and axis tap: (offset in the tile accumulator or NEG
    // when outside the tile, as int bits; weight)
    float2 *ent_ow = reinterpret_cast<float2 *>(acc + (size_t)ngroup * plane);  // [EB][D][J]
    int *ent_p = reinterpret_cast<int *>(ent_ow + EB * D * J);
    float2 *ent_y = reinterpret_cast<float2 *>(ent_p + EB);  // [ngroup][EB + 1]
    const int nthr = nwave * 64;
    for (int i = threadIdx.x; i < nchg * plane; i += nthr) acc[i] = make_float2(0.f, 0.f);

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int cc = lane / LANES_TAP;
    const int jin = lane - cc * LANES_TAP;
    const int cl = wave * cw + cc;                 // channel of this lane within the group
    const bool lane_on = cc < cw && cl < nchg;
    const int jb = A == 1 ? jin : jin % J;         // tap along the last axis
    const int ja = A == 1 ? 0 : jin / J;           // tap along the axis before it (A == 2)

    const int e0 = a.swork[4 * wk + 1], e1 = a.swork[4 * wk + 2];
    for (int eb = e0; eb < e1; eb += EB) {
        const int n = min(EB, e1 - eb);
        __syncthreads();  // previous batch fully consumed (and acc zeroed)
        if ((int)threadIdx.x < n) {
            // stage entry t: precomputed record -> per-axis tap offsets and weights
            const int t = threadIdx.x;
            const int e = eb + t;
            ent_p[t] = a.rec_p[e];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int l = a.rec_l[(int64_t)e * D + d];
                float w[J];
                kb_weights<J>(a.rec_f[(int64_t)e * D + d], g.coef, w);
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    int loc = l + j;
                    if (loc >= g.K[d]) loc -= g.K[d];
                    const int off = loc < te[d] ? loc * stride[d] : NEG;
                    ent_ow[(t * D + d) * J + j] = make_float2(__int_as_float(off), w[j]);
                }
            }
        }
        __syncthreads();
        // k-space values of the staged entries: EB entries x channels, with
        // nthr / EB channels per pass (nthr is a multiple of EB)
        {
            const int i = threadIdx.x % EB;
            const int cstep = nthr / EB;
            if (i < n) {
                const int pi = ent_p[i];
                for (int c = threadIdx.x / EB; c < nchg; c += cstep)
                    ent_y[c * (EB + 1) + i] = a.ys[(int64_t)(ch0 + c) * a.M + pi];
            }
        }
        __syncthreads();
        if (lane_on) {
            float2 *accc = acc + (size_t)cl * plane;
            const float2 *yc = ent_y + cl * (EB + 1);
            for (int i = 0; i < n; ++i) {
                const float2 *owi = ent_ow + i * D * J;
                const float2 ib = owi[(D - 1) * J + jb];
                int inner = __float_as_int(ib.x);
                float wv = ib.y;
                if (A == 2) {
                    const float2 ia = owi[(D - 2) * J + ja];
                    inner += __float_as_int(ia.x);
                    wv *= ia.y;
                }
                const float2 yv = yc[i];
                const float2 v = make_float2(wv * yv.x, wv * yv.y);
                constexpr int NO = D - A == 0 ? 1 : (D - A == 1 ? J : J * J);  // outer taps
                float2 o[NO];
                int cidx[NO];
                float wo[NO];
#pragma unroll
                for (int t = 0; t < NO; ++t) {
                    int off = inner;
                    float wt = 1.f;
                    if (D - A >= 1) {
                        const int j0 = D - A == 1 ? t : t / J;
                        const float2 r0 = owi[j0];
                        off += __float_as_int(r0.x);
                        wt = r0.y;
                    }
                    if (D - A == 2) {
                        const int j1 = t % J;
                        const float2 r1 = owi[J + j1];
                        off += __float_as_int(r1.x);
                        wt *= r1.y;
                    }
                    cidx[t] = off;
                    wo[t] = wt;
                    if (off >= 0) o[t] = accc[off];
                }
#pragma unroll
                for (int t = 0; t < NO; ++t)
                    if (cidx[t] >= 0)
                        accc[cidx[t]] = make_float2(fmaf(wo[t], v.x, o[t].x), fmaf(wo[t], v.y, o[t].y));
            }
        }
    }
    __syncthreads();
    // write the owned tile of every channel in the group: to the grid, or
    // (tile split into several work items) to this item's partial slot.
    // Threads cover (channel, row) pairs x last-axis columns; a row is one
    // index tuple of the leading axes.
    int nrows = 1;
    for (int d = 0; d + 1 < D; ++d) nrows *= te[d];
    const int tl = te[D - 1];
    int pstride = 1;
    for (int d = 0; d < D; ++d) pstride *= g.To[d];
    for (int idx = threadIdx.x; idx < nchg * nrows * tl; idx += nthr) {
        const int cr = idx / tl;           // (channel, row) pair
        const int col = idx - cr * tl;
        const int c = cr / nrows;
        const int r = cr - c * nrows;
        int rem = r, lo = col;
        int64_t goff = 0, gstride = g.K[D - 1];
        for (int d = D - 2; d >= 0; --d) {
            const int l = D == 2 ? rem : rem % te[d];
            rem = D == 2 ? 0 : rem / te[d];
            lo += l * stride[d];
            goff += (int64_t)(a0[d] + l) * gstride;
            gstride *= g.K[d];
        }
        const float2 v = acc[(size_t)c * plane + lo];
        if (slot >= 0)
            a.partial[((int64_t)slot * a.nch + ch0 + c) * pstride + r * tl + col] = v;
        else
            a.grid[(int64_t)(ch0 + c) * a.gsize + goff + a0[D - 1] + col] = v;
    }
}

// Output-stationary spread.  Workgroup = (work item of one owner tile,
// group of CPT channels); one thread per cell of the tile (To^D threads), which
// keeps the CPT channel sums of its cell in registers.  The work item's list
// entries are staged in batches: per entry the tap origin relative to the
// tile, the window weights of each axis (evaluated once per entry) and the
// k-space values of the channel group.  Then every thread walks the batch: its
// tap index per axis is its cell minus the entry's origin (mod K), its weight
// the product of the axis weights (zero outside the J^D footprint), and it adds
// weight * y into its sums.  No thread ever writes another thread's cell, so
// there are no atomics and no read-modify-write of shared memory, and the sum
// order (list order) is fixed.  The tile is written once at the end, to the
// grid or to the work item's partial slot.
// Body of one workgroup: channel group gx, work items wy, wy + ny, ...
// (the kernel's blockIdx.x, blockIdx.y and gridDim.y).
template <int D, int J, int CPT, int EB>
__device__ __forceinline__ void spread_os_wg(const KbnGeom &g, const KbnSpreadArgs &a, int gx, int wy, int ny) {
    __shared__ float2 s_y[EB][CPT];
    __shared__ int s_p[EB];
    // 2D: per staged entry the tap origin relative to the tile and the J
    // window weights of each axis.  3D: per staged entry and axis, the
    // window weight seen by each cell coordinate of the tile along that axis
    // (zero outside the footprint), so that a thread's weight is a product
    // of table reads (measured faster in 3D, slower in 2D).
    __shared__ float s_w[D == 2 ? EB : 1][D][J];
    __shared__ int s_l[D == 2 ? EB : 1][D];
    extern __shared__ float s_t[];  // 3D: [EB][D][To_max]
    // 3D: the window polynomials' coefficients, read by every table entry
    __shared__ float s_cf[D == 3 ? KBN_MAX_J * KBN_NCOEF : 1];
    const int nwork = a.scounts[0];
    const int nthr = blockDim.x;
    if (D == 3)
        for (int i = threadIdx.x; i < J * KBN_NCOEF; i += nthr) s_cf[i] = g.coef[i];  // seen after the first barrier
    int tmax = 1;
#pragma unroll
    for (int d = 0; d < D; ++d) tmax = max(tmax, g.To[d]);
    int c[D];
    {
        int t = threadIdx.x;
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            c[d] = t % g.To[d];
            t /= g.To[d];
        }
    }
    const int ch0 = gx * CPT;
    const int nchg = min(CPT, a.nch - ch0);
    // 3D tiles of 8 x 8 cells per x-slice: a wave holds exactly one slice
    const bool slice_waves = D == 3 && EB <= 64 && CPT <= 16 && g.To[1] == 8 && g.To[D - 1] == 8;
    // work items in dispatch order (hottest tiles first); a grid smaller
    // than the work list strides over it
    for (int wk = wy; wk < nwork; wk += ny) {
        const int tile = a.swork[4 * wk];
        const int slot = a.swork[4 * wk + 3];
        int a0[D], te[D];
        {
            int rem = tile;
#pragma unroll
            for (int d = D - 1; d >= 0; --d) {
                const int tc = rem % g.nto[d];
                rem /= g.nto[d];
                a0[d] = tc * g.To[d];
                te[d] = min(g.To[d], g.K[d] - a0[d]);
            }
        }
        bool active = true;
#pragma unroll
        for (int d = 0; d < D; ++d) active = active && c[d] < te[d];
        float2 acc[CPT];
#pragma unroll
        for (int k = 0; k < CPT; ++k) acc[k] = make_float2(0.f, 0.f);
        const int e0 = a.swork[4 * wk + 1], e1 = a.swork[4 * wk + 2];
        for (int eb = e0; eb < e1; eb += EB) {
            const int n = min(EB, e1 - eb);
            __syncthreads();  // previous batch (or work item) consumed
            for (int t = threadIdx.x; t < n; t += nthr) {
                s_p[t] = a.rec_q[eb + t];
                if (D == 2) {
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        s_l[t][d] = a.rec_l[(int64_t)(eb + t) * D + d];
                        float w[J];
                        kb_weights<J>(a.rec_f[(int64_t)(eb + t) * D + d], g.coef, w);
#pragma unroll
                        for (int j = 0; j < J; ++j) s_w[t][d][j] = w[j];
                    }
                }
            }
            // 3D weight tables: entry t, axis d, cell coordinate cc
            for (int idx = threadIdx.x; D == 3 && idx < n * D * tmax; idx += nthr) {
                const int cc = idx % tmax;
                const int td = idx / tmax;
                const int d = td % D;
                const int t = td / D;
                const int64_t e = eb + t;
                int j = cc - a.rec_l[e * D + d];
                if (j < 0) j += g.K[d];
                float wv = 0.f;
                if (j < J) {
                    const float x = 2.f * a.rec_f[e * D + d] - 1.f;
                    const float *cf = s_cf + j * KBN_NCOEF;
                    float acc_w = cf[KBN_NCOEF - 1];
#pragma unroll
                    for (int k = KBN_NCOEF - 2; k >= 0; --k) acc_w = fmaf(acc_w, x, cf[k]);
                    wv = acc_w;
                }
                s_t[idx] = wv;
            }
            __syncthreads();
            // loads past the batch or the channel group re-read a valid
            // value (never used), so that they are issued without branches
            // and several are in flight at once
#pragma unroll 4
            for (int i = threadIdx.x; i < EB * CPT; i += nthr) {
                const int t = i % EB;
                const int k = i / EB;
                const bool ok = t < n && k < nchg;
                s_y[t][k] = a.y[(int64_t)(ch0 + (ok ? k : 0)) * a.M + (ok ? s_p[t] : 0)];
            }
            __syncthreads();
            if (D == 3 && slice_waves) {
                // The wave's entries: a ballot over the batch of the slice
                // weights (lane t: entry t), so that the walk below visits
                // only entries that reach the slice, KBN_SPREAD_OS_U at a time, with all
                // their table and value reads issued before the sums.  The
                // products and the order of the sums are those of the loop
                // below.
                const int t = threadIdx.x & 63;
                const float wx_t = t < n ? s_t[t * D * tmax + c[0]] : 0.f;
                unsigned long long todo = __ballot(wx_t != 0.f);
                constexpr int U = KBN_SPREAD_OS_U;  // entries per step
                while (todo) {
                    int idx[U];
                    bool has[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        has[u] = todo != 0;
                        idx[u] = has[u] ? __builtin_ctzll(todo) : idx[0];
                        if (has[u]) todo &= todo - 1;
                    }
                    float wv[U];
                    float2 yv[U][CPT];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const float *ti = s_t + idx[u] * D * tmax;
                        float w = ti[c[0]];
#pragma unroll
                        for (int d = 1; d < D; ++d) w *= ti[d * tmax + c[d]];
                        wv[u] = w;
#pragma unroll
                        for (int k = 0; k < CPT; ++k) yv[u][k] = s_y[idx[u]][k];
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (!has[u]) break;
#pragma unroll
                        for (int k = 0; k < CPT; ++k) {
                            acc[k].x = fmaf(wv[u], yv[u][k].x, acc[k].x);
                            acc[k].y = fmaf(wv[u], yv[u][k].y, acc[k].y);
                        }
                    }
                }
                continue;
            }
            for (int i = 0; i < n; ++i) {
                float w;
                if (D == 3) {
                    const float *ti = s_t + i * D * tmax;
                    w = ti[c[0]];
                    // with 8 x 8 cells per x-slice a wave holds one slice, so
                    // this skip is taken by whole waves when the footprint
                    // misses the slice
                    if (w == 0.f) continue;
#pragma unroll
                    for (int d = 1; d < D; ++d) w *= ti[d * tmax + c[d]];
                } else {
                    bool in = true;
                    w = 1.f;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        int j = c[d] - s_l[i][d];
                        if (j < 0) j += g.K[d];
                        in = in && j < J;
                        w *= s_w[i][d][j < J ? j : J - 1];
                    }
                    w = in ? w : 0.f;
                }
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    const float2 y = s_y[i][k];
                    acc[k].x = fmaf(w, y.x, acc[k].x);
                    acc[k].y = fmaf(w, y.y, acc[k].y);
                }
            }
        }
        if (active) {
            int pstride = 1, loc = 0, lstride = 1;
            int64_t goff = 0, gstride = 1;
#pragma unroll
            for (int d = D - 1; d >= 0; --d) {
                pstride *= g.To[d];
                loc += c[d] * lstride;
                lstride *= te[d];
                goff += (int64_t)(a0[d] + c[d]) * gstride;
                gstride *= g.K[d];
            }
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                if (k < nchg) {
                    if (slot >= 0)
                        a.partial[((int64_t)slot * a.nch + ch0 + k) * pstride + loc] = acc[k];
                    else
                        a.grid[(int64_t)(ch0 + k) * a.gsize + goff] = acc[k];
                }
            }
        }
    }
}

template <int D, int J, int CPT, int EB>
__global__ void __launch_bounds__(512) k_spread_os(KbnGeom g, KbnSpreadArgs a) {
    spread_os_wg<D, J, CPT, EB>(g, a, blockIdx.x, blockIdx.y, gridDim.y);
}

// The output-stationary spreads of several plans in one launch (same
// owner-tile shape, so one workgroup size): workgroup row y belongs to the
// job i with ystart[i] <= y < ystart[i + 1], which strides over its work
// items with ny rows; columns past the job's channel groups stop at once.
template <int D, int J, int CPT, int EB>
__global__ void __launch_bounds__(512)
k_spread_os_multi(const KbnSpreadJob *__restrict__ jobs, const int *__restrict__ ystart, int njobs) {
    const int y = blockIdx.y;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ystart[mid] <= y) lo = mid;
        else hi = mid - 1;
    }
    const KbnSpreadJob &j = jobs[lo];
    if ((int)blockIdx.x >= j.ngr) return;
    spread_os_wg<D, J, CPT, EB>(j.g, j.a, blockIdx.x, y - ystart[lo], j.ny);
}

// Output-stationary spread with one channel per lane, for 2D 8 x 8 owner
// tiles and at least 64 channels.  A wave owns one tile for 64 channels and
// each lane keeps the 64 cell sums of its own channel in registers.  Per
// staged list entry the lanes share the window weights of each axis,
// tabulated over the tile's 8 cell coordinates (zero outside the footprint),
// and a mask of the rows the footprint covers; the wave visits only the
// covered rows, with wave-uniform branches, and each lane adds weight * y of
// its channel to the row's cells (a zero weight adds +0 outside the
// footprint).  A cell's weight is the same product w_axis0 * w_axis1 as in
// k_spread_os and the entries are added in list order, so both kernels
// produce the same sums for finite data.  The finished tile goes
// through LDS two rows at a time, so that each store instruction writes whole
// row segments of a few channels instead of one cell of 64 channels.
template <int J, int EB>
__global__ void __launch_bounds__(64, KBN_SPREAD_CL_WAVES) k_spread_cl(KbnGeom g, KbnSpreadArgs a) {
    constexpr int T = 8;
    constexpr int NC = 64;         // channels per wave (one per lane)
    constexpr int YP = NC + 1;     // padded entry row of the staged values
    constexpr int TP = 2 * T + 1;  // padded channel row of two transposed tile rows
    constexpr int SY = EB * YP > NC * TP ? EB * YP : NC * TP;
    __shared__ float2 s_y[SY];
    __shared__ float4 s_w[EB][2][T / 4];
    __shared__ int s_m[EB];  // bit r: row r covered
    __shared__ int s_p[EB];
    // window polynomial coefficients of each tap, padded to 12 for float4
    // reads (read from a global table, the compiler keeps all 66 in vector
    // registers next to the 128 of the sums)
    constexpr int CP = 12;
    static_assert(KBN_NCOEF <= CP, "coefficient padding");
    static_assert(NC % EB == 0 && (EB * 2 * T) % NC == 0, "batch size");
    __shared__ float4 s_coef[J * CP / 4];
    const int lane = threadIdx.x;
    for (int i = lane; i < J * CP; i += NC) {
        const int j = i / CP, k = i - j * CP;
        reinterpret_cast<float *>(s_coef)[i] = k < KBN_NCOEF ? g.coef[j * KBN_NCOEF + k] : 0.f;
    }
    const int ch0 = blockIdx.x * NC;
    const int nchg = min(NC, a.nch - ch0);
    const int nwork = a.scounts[0];
    for (int wk = blockIdx.y; wk < nwork; wk += gridDim.y) {
        const int tile = a.swork[4 * wk];
        const int slot = a.swork[4 * wk + 3];
        const int e0 = a.swork[4 * wk + 1], e1 = a.swork[4 * wk + 2];
        const int tr = tile / g.nto[1];
        const int a0r = tr * T, a0c = (tile - tr * g.nto[1]) * T;
        const int ter = min(T, g.K[0] - a0r), tec = min(T, g.K[1] - a0c);
        float2 acc[T][T];
#pragma unroll
        for (int r = 0; r < T; ++r)
#pragma unroll
            for (int c = 0; c < T; ++c) acc[r][c] = make_float2(0.f, 0.f);
        for (int eb = e0; eb < e1; eb += EB) {
            const int n = min(EB, e1 - eb);
            __syncthreads();  // previous batch (or tile write-out) consumed
            if (lane < n) s_p[lane] = a.rec_q[eb + lane];
            // window weights: lane -> (entry t, axis d, cell cc), EB * 16
            // cells in passes of 64, each the tap polynomial of its cell with
            // the Horner steps of kb_weights; the row masks come from a
            // ballot over the axis-0 cells of each entry
#pragma unroll
            for (int it = 0; it < EB * 2 * T / NC; ++it) {
                const int idx = it * NC + lane;
                const int t = idx / (2 * T), d = (idx / T) & 1, cc = idx % T;
                bool in = false;
                float wv = 0.f;
                if (t < n) {
                    const int64_t e = eb + t;
                    int j = cc - a.rec_l[e * 2 + d];
                    if (j < 0) j += g.K[d];
                    in = j < J && cc < (d == 0 ? ter : tec);
                    const float x = 2.f * a.rec_f[e * 2 + d] - 1.f;
                    const int jc = in ? j : 0;
                    float cf[CP];
#pragma unroll
                    for (int q = 0; q < CP / 4; ++q) {
                        const float4 c4 = s_coef[jc * (CP / 4) + q];
                        cf[4 * q] = c4.x, cf[4 * q + 1] = c4.y, cf[4 * q + 2] = c4.z, cf[4 * q + 3] = c4.w;
                    }
                    float acc_w = cf[KBN_NCOEF - 1];
#pragma unroll
                    for (int k = KBN_NCOEF - 2; k >= 0; --k) acc_w = fmaf(acc_w, x, cf[k]);
                    wv = in ? acc_w : 0.f;
                }
                reinterpret_cast<float *>(s_w)[idx] = wv;
                const unsigned long long bal = __ballot(in);
                if ((lane & (2 * T - 1)) == 0) s_m[t] = (int)((bal >> (lane & ~(2 * T - 1))) & 0xFF);
            }
            __syncthreads();
            // values: 64 channels x EB entries, entries fastest (consecutive
            // list entries are mostly consecutive samples); a lane keeps one
            // entry and steps over channels.  Loads past the batch or the
            // channel count re-read a valid value, so that all are issued
            // without branches and are in flight together; their addresses
            // are 32-bit byte offsets from the group's first channel (the
            // host takes this kernel only when 64 channels of k-space span
            // less than 2 GiB).
            {
                constexpr int KS = NC / EB;  // channels per load round
                const int t = lane % EB, kb = lane / EB;
                const int q = t < n ? s_p[t] : 0;
                const char *base = reinterpret_cast<const char *>(a.y + (int64_t)ch0 * a.M);
                const unsigned cs = (unsigned)a.M * 8u;  // bytes per channel
                float2 v[EB];
#pragma unroll
                for (int r = 0; r < EB; ++r) {
                    const unsigned k = (unsigned)min(kb + KS * r, nchg - 1);
                    v[r] = *reinterpret_cast<const float2 *>(base + ((unsigned)q * 8u + k * cs));
                }
#pragma unroll
                for (int r = 0; r < EB; ++r) s_y[t * YP + kb + KS * r] = v[r];
            }
            __syncthreads();
            for (int i = 0; i < n; ++i) {
                const float2 v = s_y[i * YP + lane];
                const int m = __builtin_amdgcn_readfirstlane(s_m[i]);
                float wr[T], wc[T];
#pragma unroll
                for (int q = 0; q < T / 4; ++q) {
                    const float4 r4 = s_w[i][0][q], c4 = s_w[i][1][q];
                    wr[4 * q] = r4.x, wr[4 * q + 1] = r4.y, wr[4 * q + 2] = r4.z, wr[4 * q + 3] = r4.w;
                    wc[4 * q] = c4.x, wc[4 * q + 1] = c4.y, wc[4 * q + 2] = c4.z, wc[4 * q + 3] = c4.w;
                }
#pragma unroll
                for (int r = 0; r < T; ++r) {
                    if (m & (1 << r)) {
#pragma unroll
                        for (int c = 0; c < T; ++c) {
                            const float w = wr[r] * wc[c];
                            acc[r][c].x = fmaf(w, v.x, acc[r][c].x);
                            acc[r][c].y = fmaf(w, v.y, acc[r][c].y);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int r0 = 0; r0 < T; r0 += 2) {
            __syncthreads();
#pragma unroll
            for (int dr = 0; dr < 2; ++dr)
#pragma unroll
                for (int c = 0; c < T; ++c) s_y[lane * TP + dr * T + c] = acc[r0 + dr][c];
            __syncthreads();
            // lane -> one cell of the two rows, stepping over channels
            const int cell = lane % (2 * T), kb = lane / (2 * T);
            constexpr int KS = NC / (2 * T);
            const int r = r0 + cell / T, c = cell % T;
            if (r < ter && c < tec) {
                float2 *dst;
                int64_t step;
                if (slot >= 0) {
                    dst = a.partial + ((int64_t)slot * a.nch + ch0 + kb) * (T * T) + r * tec + c;
                    step = (int64_t)KS * T * T;
                } else {
                    dst = a.grid + (int64_t)(ch0 + kb) * a.gsize + (int64_t)(a0r + r) * g.K[1] + a0c + c;
                    step = (int64_t)KS * a.gsize;
                }
#pragma unroll
                for (int it = 0; it < 2 * T; ++it) {
                    const int k = kb + KS * it;
                    if (k < nchg) dst[it * step] = s_y[k * TP + cell];
                }
            }
        }
    }
}

// Tiles split into several work items: sum their partial tiles in slot
// order (deterministic) and write the grid tile.  Block = (channel, tile).
template <int D>
__global__ void __launch_bounds__(KBN_BLOCK) k_spread_combine(KbnGeom g, KbnSpreadArgs a) {
    const int ncomb = a.scounts[1];
    const int ch = blockIdx.x;
    float2 *G = a.grid + (int64_t)ch * a.gsize;
    for (int k = blockIdx.y; k < ncomb; k += gridDim.y) {
        const int tile = a.scomb[3 * k], slot0 = a.scomb[3 * k + 1], ns = a.scomb[3 * k + 2];
        int a0[KBN_MAX_D], te[KBN_MAX_D];
        int rem = tile;
        for (int d = D - 1; d >= 0; --d) {
            const int tc = rem % g.nto[d];
            rem /= g.nto[d];
            a0[d] = tc * g.To[d];
            te[d] = min(g.To[d], g.K[d] - a0[d]);
        }
        int tsize = 1, pstride = 1;
        for (int d = 0; d < D; ++d) {
            tsize *= te[d];
            pstride *= g.To[d];
        }
        for (int i = threadIdx.x; i < tsize; i += blockDim.x) {
            float2 sum = make_float2(0.f, 0.f);
            for (int s = 0; s < ns; ++s) {
                const float2 v = a.partial[((int64_t)(slot0 + s) * a.nch + ch) * pstride + i];
                sum.x += v.x;
                sum.y += v.y;
            }
            int r = i;
            int64_t off = 0, stride = 1;
            for (int d = D - 1; d >= 0; --d) {
                const int l = r % te[d];
                r /= te[d];
                off += (int64_t)(a0[d] + l) * stride;
                stride *= g.K[d];
            }
            G[off] = sum;
        }
    }
}

// ys[ch][p] = y[ch][order[p]]: k-space values in tile order, so that the
// spread reads them with coalesced loads.
__global__ void __launch_bounds__(KBN_BLOCK)
k_permute(const float2 *__restrict__ y, float2 *__restrict__ ys, const int *__restrict__ order,
          int64_t M) {
    const int64_t p = (int64_t)blockIdx.x * KBN_BLOCK + threadIdx.x;
    if (p >= M) return;
    const int64_t ch = blockIdx.y;
    ys[ch * M + p] = y[ch * M + order[p]];
}

// dst[i] = (accumulate ? dst[i] : 0) + sum_g part[g][i], summed in group order.
__global__ void __launch_bounds__(KBN_BLOCK)
k_reduce_parts(float *__restrict__ dst, const float *__restrict__ part, int64_t n, int groups,
               int accumulate) {
    const int64_t i = (int64_t)blockIdx.x * KBN_BLOCK + threadIdx.x;
    if (i >= n) return;
    float s = accumulate ? dst[i] : 0.f;
    for (int g = 0; g < groups; ++g) s += part[(int64_t)g * n + i];
    dst[i] = s;
}

}  // namespace

// About KBN_GATHER_WG_TARGET workgroups over point blocks x groups (1024
// and fixed groups of 16, 24 or 32 channel sets measured slower on the
// 256-image step; 16 sets gained 4% on the 8-coil training step).
int64_t kbn_gather_groups(int64_t blocks, int64_t nbc) {
    return std::max<int64_t>(1, std::min<int64_t>(nbc, (KBN_GATHER_WG_TARGET + blocks - 1) / blocks));
}

// Launch shape of the gather: staged (LDS region fits 48 KiB) or direct, and
// the channel grouping (whole weight-channel sets per group).
KbnGatherShape kbn_gather_shape(const KbnGeom &g, int64_t M, int nch, int nw) {
    KbnGatherShape sh;
    const int lo = (g.J & 1) ? g.J / 2 : g.J / 2 - 1;
    const int hi = (g.J & 1) ? g.J / 2 + 1 : g.J / 2;
    int64_t region = 1;
    for (int d = 0; d < g.D; ++d) region *= (int64_t)std::min(g.T[d], g.K[d]) + lo + hi;
    // channels interpolated per pass: pairs (4 at a time measured slower: the
    // larger region allows fewer workgroups per CU)
    sh.cp = 2;
    sh.lds = sh.cp * sizeof(float2) * (size_t)region;
    sh.staged = sh.lds <= 48 * 1024;
    const int64_t nbc = std::max(1, nch / nw);
    int64_t blocks;
    if (sh.staged)
        blocks = (M + KBN_SUB - 1) / KBN_SUB + g.ntiles + 1;
    else
        blocks = (M + KBN_BLOCK - 1) / KBN_BLOCK;
    sh.blocks = blocks;
    const int64_t groups = kbn_gather_groups(blocks, nbc);
    sh.cg = (int)(((nbc + groups - 1) / groups) * nw);
    sh.groups = (nch + sh.cg - 1) / sh.cg;
    return sh;
}

namespace {

// the epilogue of the omega-Jacobian gather: the channel groups' partial
// gradients summed in group order
hipError_t reduce_parts(const KbnGeom &g, const KbnGatherArgs &a, int groups, hipStream_t s) {
    const int64_t n = a.M * g.D;
    k_reduce_parts<<<dim3((unsigned)((n + KBN_BLOCK - 1) / KBN_BLOCK)), dim3(KBN_BLOCK), 0, s>>>(
        a.domega, a.part, n, groups, a.accumulate);
    return hipGetLastError();
}

template <int D, int J>
hipError_t gather_dj(const KbnGeom &g, const KbnGatherArgs &a, int mode, hipStream_t s) {
    if (a.M == 0 || a.nch == 0) return hipSuccess;
    const KbnGatherShape sh = kbn_gather_shape(g, a.M, a.nch, a.nw);
    dim3 grid((unsigned)sh.blocks, (unsigned)sh.groups);
    if (sh.staged) {
        // loading ahead pays in 3D (96^3 x 8 coils: 11-14%); in 2D it cost
        // occupancy for no gain in the full step
        constexpr bool LA = D == 3;
        if (mode == 0)
            k_gather_staged<D, J, 0, 2, LA><<<grid, dim3(KBN_BLOCK), sh.lds, s>>>(g, a, sh.cg);
        else
            k_gather_staged<D, J, 1, 2, LA><<<grid, dim3(KBN_BLOCK), sh.lds, s>>>(g, a, sh.cg);
    } else {
        if (mode == 0)
            k_gather<D, J, 0><<<grid, dim3(KBN_BLOCK), 0, s>>>(g, a, sh.cg);
        else
            k_gather<D, J, 1><<<grid, dim3(KBN_BLOCK), 0, s>>>(g, a, sh.cg);
    }
    if (mode == 1) {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return reduce_parts(g, a, sh.groups, s);
    }
    return hipGetLastError();
}

template <int D, int J>
hipError_t gather_multi_dj(int mode, const KbnGatherJob *jobs, const int64_t *start, int njobs, int64_t total,
                           size_t lds, hipStream_t s) {
    constexpr bool LA = D == 3;
    const dim3 grid((unsigned)total);
    if (mode == 0)
        k_gather_multi<D, J, 0, 2, LA><<<grid, dim3(KBN_BLOCK), lds, s>>>(jobs, start, njobs);
    else
        k_gather_multi<D, J, 1, 2, LA><<<grid, dim3(KBN_BLOCK), lds, s>>>(jobs, start, njobs);
    return hipGetLastError();
}

// Launch shape of the spread: lanes per tap group (A), channels per wave,
// waves per workgroup, and the LDS bytes.
struct SpreadShape {
    int A, cw, nwave;
    size_t lds;
};

SpreadShape spread_shape(const KbnGeom &g, int nch) {
    SpreadShape sh;
    const int J = g.J, D = g.D;
    sh.A = (D >= 2 && nch < 64 / J) ? 2 : 1;
    sh.cw = sh.A == 1 ? 64 / J : std::max(1, 64 / (J * J));
    int psize = 1;
    for (int d = 0; d < D; ++d) psize *= acc_pitch(d, std::min(g.To[d], g.K[d]));
    const int plane = spread_plane(psize);
    const int EB = KBN_SPREAD_EB;
    auto bytes = [&](int nw) {
        const int ng = nw * sh.cw;
        return sizeof(float2) * (size_t)ng * plane + sizeof(int) * EB * (1 + D * J) +
               sizeof(float) * EB * D * J + sizeof(float2) * (size_t)ng * (EB + 1);
    };
    sh.nwave = 1;
    const int want = (nch + sh.cw - 1) / sh.cw;  // waves that have channels
    while (sh.nwave < 2 && sh.nwave < want && bytes(sh.nwave + 1) <= KBN_SPREAD_LDS) ++sh.nwave;
    sh.lds = bytes(sh.nwave);
    return sh;
}

template <int D, int J>
hipError_t launch_os(const KbnSpreadSel &sel, dim3 grid, const KbnGeom &g, const KbnSpreadArgs &a, hipStream_t s) {
    const dim3 blk((unsigned)sel.tcells);
    if constexpr (D == 3) {
        switch (sel.cpt) {
            case 1: k_spread_os<D, J, 1, 64><<<grid, blk, sel.lds, s>>>(g, a); break;
            case 2: k_spread_os<D, J, 2, 64><<<grid, blk, sel.lds, s>>>(g, a); break;
            case 4: k_spread_os<D, J, 4, 64><<<grid, blk, sel.lds, s>>>(g, a); break;
            case 8: k_spread_os<D, J, 8, 64><<<grid, blk, sel.lds, s>>>(g, a); break;
            case 16: k_spread_os<D, J, 16, 64><<<grid, blk, sel.lds, s>>>(g, a); break;
            default: k_spread_os<D, J, 32, 32><<<grid, blk, sel.lds, s>>>(g, a); break;
        }
    } else {
        switch (sel.cpt) {
            case 1: k_spread_os<D, J, 1, 32><<<grid, blk, sel.lds, s>>>(g, a); break;
            case 2: k_spread_os<D, J, 2, 32><<<grid, blk, sel.lds, s>>>(g, a); break;
            case 4: k_spread_os<D, J, 4, 32><<<grid, blk, sel.lds, s>>>(g, a); break;
            case 8: k_spread_os<D, J, 8, 32><<<grid, blk, sel.lds, s>>>(g, a); break;
            case 16: k_spread_os<D, J, 16, 32><<<grid, blk, sel.lds, s>>>(g, a); break;
            default: k_spread_os<D, J, 32, 32><<<grid, blk, sel.lds, s>>>(g, a); break;
        }
    }
    return hipGetLastError();
}

template <int D, int J>
hipError_t launch_os_multi(const KbnSpreadSel &sel, dim3 grid, const KbnSpreadJob *jobs, const int *ystart,
                           int njobs, hipStream_t s) {
    const dim3 blk((unsigned)sel.tcells);
    if constexpr (D == 3) {
        switch (sel.cpt) {
            case 1: k_spread_os_multi<D, J, 1, 64><<<grid, blk, sel.lds, s>>>(jobs, ystart, njobs); break;
            case 2: k_spread_os_multi<D, J, 2, 64><<<grid, blk, sel.lds, s>>>(jobs, ystart, njobs); break;
            case 4: k_spread_os_multi<D, J, 4, 64><<<grid, blk, sel.lds, s>>>(jobs, ystart, njobs); break;
            case 8: k_spread_os_multi<D, J, 8, 64><<<grid, blk, sel.lds, s>>>(jobs, ystart, njobs); break;
            case 16: k_spread_os_multi<D, J, 16, 64><<<grid, blk, sel.lds, s>>>(jobs, ystart, njobs); break;
            default: k_spread_os_multi<D, J, 32, 32><<<grid, blk, sel.lds, s>>>(jobs, ystart, njobs); break;
        }
    } else {
        switch (sel.cpt) {
            case 1: k_spread_os_multi<D, J, 1, 32><<<grid, blk, sel.lds, s>>>(jobs, ystart, njobs); break;
            case 2: k_spread_os_multi<D, J, 2, 32><<<grid, blk, sel.lds, s>>>(jobs, ystart, njobs); break;
            case 4: k_spread_os_multi<D, J, 4, 32><<<grid, blk, sel.lds, s>>>(jobs, ystart, njobs); break;
            case 8: k_spread_os_multi<D, J, 8, 32><<<grid, blk, sel.lds, s>>>(jobs, ystart, njobs); break;
            case 16: k_spread_os_multi<D, J, 16, 32><<<grid, blk, sel.lds, s>>>(jobs, ystart, njobs); break;
            default: k_spread_os_multi<D, J, 32, 32><<<grid, blk, sel.lds, s>>>(jobs, ystart, njobs); break;
        }
    }
    return hipGetLastError();
}

// the partial tiles of owner tiles split over several work items, summed
// in item order
template <int D>
hipError_t spread_combine(const KbnSpreadSel &sel, const KbnGeom &g, const KbnSpreadArgs &a, hipStream_t s) {
    if (a.ncomb_max <= 0) return hipSuccess;
    if (sel.path == KBN_SPREAD_PATH_CL) {
        const int ny = std::max(1, std::min(a.ncomb_max, 8 * 256 * 4 / a.nch + 1));
        k_spread_combine<D><<<dim3((unsigned)a.nch, (unsigned)ny), dim3(64), 0, s>>>(g, a);
    } else if (sel.path == KBN_SPREAD_PATH_OS) {
        const int cb = std::min(KBN_BLOCK, (sel.tcells + 63) / 64 * 64);
        const int ny = std::max(1, std::min(a.ncomb_max, 8 * 256 * 4 / a.nch + 1));
        k_spread_combine<D><<<dim3((unsigned)a.nch, (unsigned)ny), dim3(cb), 0, s>>>(g, a);
    } else {
        k_spread_combine<D><<<dim3((unsigned)a.nch, (unsigned)a.ncomb_max), dim3(KBN_BLOCK), 0, s>>>(g, a);
    }
    return hipGetLastError();
}

template <int D, int J>
hipError_t spread_dj(const KbnGeom &g, const KbnSpreadArgs &a, hipStream_t s) {
    if (a.nch == 0) return hipSuccess;
    const KbnSpreadSel sel = kbn_spread_select(g, a);
    hipError_t e = hipSuccess;
    if (sel.path == KBN_SPREAD_PATH_CL) {
        dim3 grid_cl((unsigned)((a.nch + 63) / 64), (unsigned)std::min(a.nwork_max, KBN_GRID_Y_MAX));
        k_spread_cl<J, KBN_SPREAD_CL_EB><<<grid_cl, dim3(64), 0, s>>>(g, a);
        e = hipGetLastError();
    } else if (sel.path == KBN_SPREAD_PATH_OS) {
        e = launch_os<D, J>(sel, dim3((unsigned)sel.ngr, (unsigned)sel.ny), g, a, s);
    } else {
        const SpreadShape sh = spread_shape(g, a.nch);
        const int ngroup = sh.nwave * sh.cw;
        const int ng = (a.nch + ngroup - 1) / ngroup;
        if (a.M > 0) {  // the scatter kernel reads k-space values in tile order
            dim3 pgrid((unsigned)((a.M + KBN_BLOCK - 1) / KBN_BLOCK), (unsigned)a.nch);
            k_permute<<<pgrid, dim3(KBN_BLOCK), 0, s>>>(a.y, a.ys, a.order, a.M);
        }
        dim3 grid((unsigned)ng, (unsigned)a.nwork_max);  // one workgroup row per work item
        if (sh.A == 1 || D == 1)
            k_spread<D, J, 1><<<grid, dim3(64 * sh.nwave), sh.lds, s>>>(g, a, sh.cw, sh.nwave);
        else
            k_spread<D, J, (D >= 2 ? 2 : 1)><<<grid, dim3(64 * sh.nwave), sh.lds, s>>>(g, a, sh.cw, sh.nwave);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    return spread_combine<D>(sel, g, a, s);
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
hipError_t gather_multi_d(int J, int mode, const KbnGatherJob *jobs, const int64_t *start, int njobs, int64_t total,
                          size_t lds, hipStream_t s) {
    switch (J) {
        case 2: return gather_multi_dj<D, 2>(mode, jobs, start, njobs, total, lds, s);
        case 3: return gather_multi_dj<D, 3>(mode, jobs, start, njobs, total, lds, s);
        case 4: return gather_multi_dj<D, 4>(mode, jobs, start, njobs, total, lds, s);
        case 5: return gather_multi_dj<D, 5>(mode, jobs, start, njobs, total, lds, s);
        case 6: return gather_multi_dj<D, 6>(mode, jobs, start, njobs, total, lds, s);
        case 7: return gather_multi_dj<D, 7>(mode, jobs, start, njobs, total, lds, s);
        default: return gather_multi_dj<D, 8>(mode, jobs, start, njobs, total, lds, s);
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

template <int D>
hipError_t spread_os_multi_d(const KbnSpreadSel &sel, int J, dim3 grid, const KbnSpreadJob *jobs, const int *ystart,
                             int njobs, hipStream_t s) {
    switch (J) {
        case 2: return launch_os_multi<D, 2>(sel, grid, jobs, ystart, njobs, s);
        case 3: return launch_os_multi<D, 3>(sel, grid, jobs, ystart, njobs, s);
        case 4: return launch_os_multi<D, 4>(sel, grid, jobs, ystart, njobs, s);
        case 5: return launch_os_multi<D, 5>(sel, grid, jobs, ystart, njobs, s);
        case 6: return launch_os_multi<D, 6>(sel, grid, jobs, ystart, njobs, s);
        case 7: return launch_os_multi<D, 7>(sel, grid, jobs, ystart, njobs, s);
        default: return launch_os_multi<D, 8>(sel, grid, jobs, ystart, njobs, s);
    }
}

}  // namespace

// Which spread kernel a call takes, with its launch shape: the
// channel-per-lane kernel (2D 8 x 8 owner tiles, at least 64 channels and
// enough tiles x channel groups to fill the chip's wave slots twice), the
// output-stationary one (2D/3D owner tiles of at most 512 cells), else the
// scatter kernel.  All give the same sums for finite data.
KbnSpreadSel kbn_spread_select(const KbnGeom &g, const KbnSpreadArgs &a) {
    static const bool os_on = [] {
        const char *e = std::getenv("KBN_SPREAD_OS");
        return !(e && e[0] == '0');
    }();
    static const bool cl_on = [] {
        const char *e = std::getenv("KBN_SPREAD_CL");
        return !(e && e[0] == '0');
    }();
    KbnSpreadSel sel;
    const int D = g.D;
    int tcells = 1, tmax = 1;
    for (int d = 0; d < D; ++d) {
        tcells *= g.To[d];
        tmax = std::max(tmax, g.To[d]);
    }
    sel.tcells = tcells;
    const int64_t cl_waves = (int64_t)g.ntiles_own * ((a.nch + 63) / 64);
    if (D == 2 && os_on && cl_on && g.To[0] == 8 && g.To[1] == 8 && a.nch >= 64 && cl_waves >= 4096 &&
        64 * a.M * (int64_t)sizeof(float2) < ((int64_t)1 << 31)) {
        sel.path = KBN_SPREAD_PATH_CL;
        return sel;
    }
    if (D >= 2 && tcells <= 512 && os_on) {
        sel.path = KBN_SPREAD_PATH_OS;
        const int want = std::min(a.nch, 32);
        int cpt = 1;
        while (cpt < want) cpt *= 2;
        sel.cpt = cpt;
        sel.ngr = (a.nch + cpt - 1) / cpt;
        sel.ny = std::min(a.nwork_max, KBN_GRID_Y_MAX);
        // entries per batch of the chosen kernel, and the 3D weight tables
        sel.ebv = D == 3 ? (cpt <= 16 ? 64 : 32) : 32;
        sel.lds = D == 3 ? sizeof(float) * (size_t)sel.ebv * D * tmax : 0;
        return sel;
    }
    sel.path = KBN_SPREAD_PATH_GENERIC;
    return sel;
}

hipError_t kbn_launch_gather(const KbnGeom &g, const KbnGatherArgs &a, int mode, hipStream_t s) {
    switch (g.D) {
        case 1: return gather_d<1>(g, a, mode, s);
        case 2: return gather_d<2>(g, a, mode, s);
        default: return gather_d<3>(g, a, mode, s);
    }
}

hipError_t kbn_launch_gather_reduce(const KbnGeom &g, const KbnGatherArgs &a, hipStream_t s) {
    if (a.M == 0 || a.nch == 0) return hipSuccess;
    return reduce_parts(g, a, kbn_gather_shape(g, a.M, a.nch, a.nw).groups, s);
}

hipError_t kbn_launch_gather_multi(int D, int J, int mode, const KbnGatherJob *jobs, const int64_t *start, int njobs,
                                   int64_t total, size_t lds, hipStream_t s) {
    if (njobs == 0 || total == 0) return hipSuccess;
    switch (D) {
        case 1: return gather_multi_d<1>(J, mode, jobs, start, njobs, total, lds, s);
        case 2: return gather_multi_d<2>(J, mode, jobs, start, njobs, total, lds, s);
        default: return gather_multi_d<3>(J, mode, jobs, start, njobs, total, lds, s);
    }
}

hipError_t kbn_launch_spread(const KbnGeom &g, const KbnSpreadArgs &a, hipStream_t s) {
    switch (g.D) {
        case 1: return spread_d<1>(g, a, s);
        case 2: return spread_d<2>(g, a, s);
        default: return spread_d<3>(g, a, s);
    }
}

hipError_t kbn_launch_spread_os_multi(const KbnSpreadSel &sel, int D, int J, int maxngr, const KbnSpreadJob *jobs,
                                      const int *ystart, int njobs, int total_y, hipStream_t s) {
    if (njobs == 0 || total_y == 0) return hipSuccess;
    const dim3 grid((unsigned)maxngr, (unsigned)total_y);
    if (D == 2) return spread_os_multi_d<2>(sel, J, grid, jobs, ystart, njobs, s);
    return spread_os_multi_d<3>(sel, J, grid, jobs, ystart, njobs, s);
}

hipError_t kbn_launch_spread_combine(const KbnSpreadSel &sel, const KbnGeom &g, const KbnSpreadArgs &a,
                                     hipStream_t s) {
    switch (g.D) {
        case 1: return spread_combine<1>(sel, g, a, s);
        case 2: return spread_combine<2>(sel, g, a, s);
        default: return spread_combine<3>(sel, g, a, s);
    }
}
