// Index pass: grid cell, in-cell fraction and tile of every sample location,
// a stable counting sort of the samples by tile, and the spread's owner-tile
// lists.
//
// The appendix interpolates each sample from J uniform frequencies at
// offsets k_m + j.  Those taps follow from the cell that contains
// u = omega K / (2 pi) and the fraction of u inside it; the tile order puts
// samples that touch the same region of the oversampled grid next to each
// other, which the gather (cache locality) and the spread (tile ownership)
// rely on.
//
// Arithmetic (bit-exact by construction):
//   u = (double)omega * scale_d   (one FP64 multiply, never contracted)
//   fl = floor(u); frac = (float)(u - fl); cell = fl mod K (integer)
// Non-finite omega or |u| >= 2^40 marks the sample as flagged: cell 0,
// frac 0, tile id ntiles (sorted after every finite sample).
#include "kbn_internal.h"
#include "kbn_window.h"

namespace {

constexpr double kULimit = 1099511627776.0;  // 2^40

// One workgroup per chunk of `chunk` samples: cell, fraction and tile of
// every sample, and the chunk's tile histogram (LDS), stored bin-major
// (counts[bin * nchunks + chunk]) for the scan.
__global__ void __launch_bounds__(256)
k_points_hist(int D, int64_t M, int chunk, int nchunks, int nbins, const float *__restrict__ omega,
              double s0, double s1, double s2, int K0, int K1, int K2, int T0, int T1, int T2, int nt1,
              int nt2, int ntiles, int *__restrict__ cell_tmp, float *__restrict__ frac_tmp,
              int *__restrict__ tile, int *__restrict__ flag, int *__restrict__ counts) {
#pragma clang fp contract(off)
    extern __shared__ int hist[];
    const int ch = blockIdx.x;
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const double sc[3] = {s0, s1, s2};
    const int Kd[3] = {K0, K1, K2};
    const int64_t beg = (int64_t)ch * chunk;
    const int64_t end = beg + chunk < M ? beg + chunk : M;
    for (int64_t m = beg + threadIdx.x; m < end; m += blockDim.x) {
        int c[3] = {0, 0, 0};
        float f[3] = {0.f, 0.f, 0.f};
        bool bad = false;
        for (int d = 0; d < D; ++d) {
            const double u = (double)omega[m * D + d] * sc[d];
            if (!(fabs(u) < kULimit)) {
                bad = true;
                continue;
            }
            const double fl = floor(u);
            f[d] = (float)(u - fl);
            const long long l = (long long)fl;
            long long r = l % (long long)Kd[d];
            if (r < 0) r += Kd[d];
            c[d] = (int)r;
        }
        int t;
        if (bad) {
            for (int d = 0; d < 3; ++d) {
                c[d] = 0;
                f[d] = 0.f;
            }
            t = ntiles;
            atomicOr(flag, 1);
        } else {
            t = c[0] / T0;
            if (D > 1) t = t * nt1 + c[1] / T1;
            if (D > 2) t = t * nt2 + c[2] / T2;
        }
        for (int d = 0; d < D; ++d) {
            cell_tmp[d * M + m] = c[d];
            frac_tmp[d * M + m] = f[d];
        }
        tile[m] = t;
        atomicAdd(&hist[t], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) counts[(int64_t)i * nchunks + ch] = hist[i];
}

// Workgroup barrier that orders LDS only: unlike __syncthreads it does not
// wait for the caller's outstanding global stores.  Where threads exchange
// data through global memory, __syncthreads is used.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ int block_scan_1024(int x, int *wsum, int &total) {
    // inclusive scan over a 1024-thread block; returns the exclusive prefix
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int inc = x;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wid] = inc;
    lds_barrier();
    int wpre = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
        const int ws = wsum[w];
        if (w < wid) wpre += ws;
        tot += ws;
    }
    lds_barrier();
    total = tot;
    return wpre + inc - x;
}

// Gather subproblems from the tile offsets: bin t with n points contributes
// ceil(n / sub) entries (bin, first sorted position); the last bin holds the
// flagged points.  Run by one 1024-thread workgroup after toff is complete.
__device__ void subproblems_block(int nbins, int sub, const int *__restrict__ toff, int *__restrict__ subs,
                                  int *__restrict__ nsub, int *wsum) {
    const int tid = threadIdx.x;
    const int seg = (nbins + 1023) / 1024;
    const int beg = min(tid * seg, nbins);
    const int end = min(beg + seg, nbins);
    int sum = 0;
    for (int t = beg; t < end; ++t) sum += (toff[t + 1] - toff[t] + sub - 1) / sub;
    int total;
    int run = block_scan_1024(sum, wsum, total);
    for (int t = beg; t < end; ++t) {
        for (int q = toff[t]; q < toff[t + 1]; q += sub) {
            subs[2 * run] = t;
            subs[2 * run + 1] = q;
            ++run;
        }
    }
    if (tid == 0) *nsub = total;
}

// Bins x chunks matrices up to this many counts are scanned by one workgroup
// through LDS (48 KiB); larger ones by the three-phase scan below.
#define KBN_SCAN_SMALL 12288

// One workgroup: exclusive scan of the S bin-major counts in place
// (counts[b * nchunks + c] becomes the first output position of chunk c's
// samples of bin b), the bin offsets toff[0..nbins] and the gather
// subproblem list.  The counts are loaded and stored coalesced; each thread
// scans a contiguous run of them in LDS.
__global__ void __launch_bounds__(1024)
k_scan_small(int S, int nchunks, int nbins, int sub, int *__restrict__ counts, int *__restrict__ toff,
             int *__restrict__ subs, int *__restrict__ nsub) {
    __shared__ int buf[KBN_SCAN_SMALL];
    __shared__ int wsum[16];
    const int tid = threadIdx.x;
#pragma unroll 4
    for (int i = tid; i < S; i += 1024) buf[i] = counts[i];
    __syncthreads();
    const int per = (S + 1023) / 1024;
    const int beg = min(tid * per, S), end = min(beg + per, S);
    int sum = 0;
    for (int i = beg; i < end; ++i) sum += buf[i];
    int total;
    int run = block_scan_1024(sum, wsum, total);
    for (int i = beg; i < end; ++i) {
        const int v = buf[i];
        buf[i] = run;
        if (i % nchunks == 0) toff[i / nchunks] = run;
        run += v;
    }
    if (S == 0)
        for (int b = tid; b < nbins; b += 1024) toff[b] = 0;
    if (tid == 0) toff[nbins] = total;
    __syncthreads();
#pragma unroll 4
    for (int i = tid; i < S; i += 1024) counts[i] = buf[i];
    subproblems_block(nbins, sub, toff, subs, nsub, wsum);
}

// Three-phase scan of larger count matrices over spans of KBN_SCAN_SPAN
// counts: span sums, an exclusive scan of the span sums (one workgroup),
// then each span rescanned with its offset.  Integer sums, so the order of
// additions does not matter.
#define KBN_SCAN_SPAN 8192

__global__ void __launch_bounds__(1024)
k_scan_sums(int64_t S, const int *__restrict__ counts, int *__restrict__ bsum) {
    __shared__ int wsum[16];
    const int64_t base = (int64_t)blockIdx.x * KBN_SCAN_SPAN;
    int acc = 0;
    for (int k = 0; k < KBN_SCAN_SPAN / 1024; ++k) {
        const int64_t i = base + (int64_t)k * 1024 + threadIdx.x;
        acc += i < S ? counts[i] : 0;
    }
    int tot;
    (void)block_scan_1024(acc, wsum, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// exclusive scan of nb span sums in place; bsum[nb] = total
__global__ void __launch_bounds__(1024) k_scan_top(int nb, int *__restrict__ bsum) {
    __shared__ int wsum[16];
    int run = 0;
    for (int base = 0; base < nb; base += 1024) {
        const int i = base + (int)threadIdx.x;
        const int v = i < nb ? bsum[i] : 0;
        int tot;
        const int ex = block_scan_1024(v, wsum, tot);
        if (i < nb) bsum[i] = run + ex;
        run += tot;
    }
    if (threadIdx.x == 0) bsum[nb] = run;
}

__global__ void __launch_bounds__(1024)
k_scan_apply(int64_t S, int *__restrict__ counts, const int *__restrict__ bsum) {
    __shared__ int wsum[16];
    const int64_t base = (int64_t)blockIdx.x * KBN_SCAN_SPAN;
    int run = bsum[blockIdx.x];
    for (int k = 0; k < KBN_SCAN_SPAN / 1024; ++k) {
        const int64_t i = base + (int64_t)k * 1024 + threadIdx.x;
        const int v = i < S ? counts[i] : 0;
        int tot;
        const int ex = block_scan_1024(v, wsum, tot);
        if (i < S) counts[i] = run + ex;
        run += tot;
    }
}

__global__ void __launch_bounds__(256)
k_scan_offsets(int64_t S, int nchunks, int nbins, const int *__restrict__ counts,
               const int *__restrict__ bsum, int nb, int *__restrict__ toff) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b < nbins) toff[b] = S > 0 ? counts[(int64_t)b * nchunks] : 0;
    if (b == 0) toff[nbins] = S > 0 ? bsum[nb] : 0;
}

__global__ void __launch_bounds__(1024)
k_subproblems(int nbins, int sub, const int *__restrict__ toff, int *__restrict__ subs, int *__restrict__ nsub) {
    __shared__ int wsum[16];
    subproblems_block(nbins, sub, toff, subs, nsub, wsum);
}

__global__ void __launch_bounds__(256) k_zero_ints(int *__restrict__ p, int n) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0;
}

// One wavefront per chunk: stable scatter.  Lanes with equal tile ids are
// grouped with ballots; rank = number of equal lanes below, so within a
// chunk the input order is kept, and chunks occupy consecutive ranges.
// The workgroups also clear zero[0..nzero).
template <int D>
__global__ void __launch_bounds__(64)
k_tile_scatter(int64_t M, int chunk, int nchunks, int nbins, int nbits,
               const int *__restrict__ tile, const int *__restrict__ counts,
               const int *__restrict__ cell_tmp, const float *__restrict__ frac_tmp,
               int *__restrict__ order, int *__restrict__ cell, float *__restrict__ frac,
               int *__restrict__ zero, int nzero) {
    extern __shared__ int cursor[];
    const int ch = blockIdx.x;
    const int lane = threadIdx.x;
    // clear the owner-tile counters for the next kernels
    for (int i = ch * 64 + lane; i < nzero; i += nchunks * 64) zero[i] = 0;
#pragma unroll 8
    for (int i = lane; i < nbins; i += 64) cursor[i] = counts[(int64_t)i * nchunks + ch];
    __syncthreads();
    const int64_t beg = (int64_t)ch * chunk;
    const int64_t end = beg + chunk < M ? beg + chunk : M;
    const unsigned long long below = (1ull << lane) - 1ull;
    // steps of 64 samples in batches: every load of a batch is issued before
    // its first ranking step, so only LDS work and stores remain in the steps
    constexpr int NB = 12;
    for (int64_t b0 = beg; b0 < end; b0 += 64 * NB) {
        int tv[NB], cv[NB][D];
        float fv[NB][D];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const int64_t m = b0 + 64 * k + lane;
            const bool in = m < end;
            tv[k] = in ? tile[m] : -1;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                cv[k][d] = in ? cell_tmp[d * M + m] : 0;
                fv[k][d] = in ? frac_tmp[d * M + m] : 0.f;
            }
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            if (b0 + 64 * k >= end) break;
            const int64_t m = b0 + 64 * k + lane;
            const bool valid = m < end;
            const int t = tv[k];
            unsigned long long peers = ~0ull;
            for (int bit = 0; bit <= nbits; ++bit) {
                const bool on = (t >> bit) & 1;
                const unsigned long long bal = __ballot(on);
                peers &= on ? bal : ~bal;
            }
            const int rank = __popcll(peers & below);
            const int cnt = __popcll(peers);
            int pos = 0;
            if (valid) pos = cursor[t] + rank;
            // the workgroup is one wavefront: its LDS accesses complete in
            // program order, so the cursor update needs no workgroup barrier
            // (which would also wait for the global stores)
            __builtin_amdgcn_wave_barrier();
            if (valid && rank == 0) cursor[t] = pos + cnt;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
            __builtin_amdgcn_wave_barrier();
            if (valid) {
                order[pos] = (int)m;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    cell[d * M + pos] = cv[k][d];
                    frac[d * M + pos] = fv[k][d];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Owner-tile lists for the spread.  A finite sample whose J taps along axis
// d start at grid cell s_d (modulo K_d) reaches owner tile t when its tap
// interval meets t's cell range on every axis.  Each owner tile collects its
// samples by looking only at the sort tiles whose cells can reach it (the
// samples are already sorted by tile): the cells [lo - HI, hi + LO] around
// its range, taps of a sample in cell c lying in [c - LO, c + HI].  Entries
// of a tile are ordered by candidate sort tile, then by sorted position, so
// the spread's accumulation order is fixed.  Every entry gets its record:
// sorted position, the sample's caller-order index, the tap origin relative
// to the tile's first cell (mod K) and the window fraction per axis.
struct OwnerGeom {
    int D, J, LO, HI;
    int ntiles_sort, ntiles_own;
    int K[3], To[3], nto[3], T[3], nt[3];
};

#define KBN_OWN_BLOCK 256
#define KBN_OWN_ILP 4    // candidate positions per thread and step
#define KBN_OWN_MAXC 64  // candidate sort tiles staged per round (one wavefront)
#define KBN_OWN_LDS 12288  // owner tiles that k_owner_finish keeps in LDS (3 ints each, 144 KiB)

// Cell range [lo, hi] of owner tile t and, per axis, the first candidate
// sort tile and their count (walked as (first + i) mod nt).
template <int D>
__device__ __forceinline__ void owner_span(const OwnerGeom &o, int t, int lo[3], int hi[3], int first[3],
                                           int num[3]) {
    int rem = t;
#pragma unroll
    for (int d = D - 1; d >= 0; --d) {
        const int a = rem % o.nto[d];
        rem /= o.nto[d];
        lo[d] = a * o.To[d];
        hi[d] = min(lo[d] + o.To[d], o.K[d]) - 1;
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const int K = o.K[d], T = o.T[d], nt = o.nt[d];
        const int L = hi[d] - lo[d] + 1 + o.LO + o.HI;
        int c0 = lo[d] - o.HI;
        if (c0 < 0) c0 += K;
        first[d] = 0;
        num[d] = nt;
        if (L >= K) continue;
        const int f = c0 / T, c1 = c0 + L - 1;
        if (c1 < K) {
            first[d] = f;
            num[d] = c1 / T - f + 1;
        } else {
            const int e = (c1 - K) / T;  // last tile of the part past the wrap
            if (e < f) {
                first[d] = f;
                num[d] = nt - f + e + 1;
            }
        }
    }
}

template <int D>
__device__ __forceinline__ int owner_candidate(const OwnerGeom &o, const int first[3], const int num[3], int k) {
    int sel[3] = {0, 0, 0};
#pragma unroll
    for (int d = D - 1; d >= 0; --d) {
        sel[d] = k % num[d];
        k /= num[d];
    }
    int st = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        int i = first[d] + sel[d];
        if (i >= o.nt[d]) i -= o.nt[d];
        st = st * o.nt[d] + i;
    }
    return st;
}

// Does the sample at sorted position p reach the owner tile with cell
// ranges [lo, hi]?  On success also the tap origin relative to lo (mod K)
// and the window fraction per axis.
template <int D>
__device__ __forceinline__ bool owner_touch(const OwnerGeom &o, int p, int64_t M, const int *__restrict__ cell,
                                            const float *__restrict__ frac, const int lo[3], const int hi[3],
                                            int rel[3], float fr[3]) {
    bool hit = true;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        int s;
        float f;
        tap_origin(o.J, cell[d * M + p], frac[d * M + p], s, f);
        const int K = o.K[d];
        const int sw = s < 0 ? s + K : s;
        int a = lo[d] - sw;  // (lo - s) mod K: lo inside the taps when <= J - 1
        if (a < 0) a += K;
        int b = sw - lo[d];  // (s - lo) mod K: s inside the tile when <= hi - lo
        if (b < 0) b += K;
        hit = hit && (a <= o.J - 1 || b <= hi[d] - lo[d]);
        rel[d] = b;
        fr[d] = f;
    }
    return hit;
}

// Wavefront 0 stages up to KBN_OWN_MAXC candidate sort tiles: their first
// sorted position and the exclusive prefix of their sizes (coff[nk] = total).
template <int D>
__device__ __forceinline__ void owner_stage(const OwnerGeom &o, const int first[3], const int num[3], int k0,
                                            int nk, const int *__restrict__ toff, int *cbeg, int *coff) {
    if (threadIdx.x < 64) {
        const int k = threadIdx.x;
        int b = 0, n = 0;
        if (k < nk) {
            const int st = owner_candidate<D>(o, first, num, k0 + k);
            b = toff[st];
            n = toff[st + 1] - b;
        }
        int inc = n;
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(inc, off, 64);
            if (k >= off) inc += y;
        }
        if (k < nk) {
            cbeg[k] = b;
            coff[k] = inc - n;
        }
        if (k == nk - 1) coff[nk] = inc;
    }
}

__device__ __forceinline__ int owner_find(const int *coff, int nk, int i) {  // last k with coff[k] <= i
    int lo = 0, hi = nk - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (coff[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Exclusive scan over a KBN_OWN_BLOCK-thread workgroup (total to all).
__device__ __forceinline__ int block_scan_own(int x, int *wsum, int &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = x;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wid] = inc;
    lds_barrier();
    int wpre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < KBN_OWN_BLOCK / 64; ++w) {
        const int ws = wsum[w];
        if (w < wid) wpre += ws;
        tot += ws;
    }
    lds_barrier();
    total = tot;
    return wpre + inc - x;
}

// The candidate walk of owner tile t shared by the count and write kernels:
// each step hands a thread KBN_OWN_ILP consecutive walk positions (all loads
// issued before the tests), and the caller folds the hits in walk order.
template <int D, class F>
__device__ __forceinline__ void owner_walk(const OwnerGeom &o, int t, int64_t M, const int *__restrict__ cell,
                                           const float *__restrict__ frac, const int *__restrict__ toff,
                                           int *cbeg, int *coff, F &&fold) {
    int lo[3], hi[3], first[3], num[3];
    owner_span<D>(o, t, lo, hi, first, num);
    int ncand = 1;
#pragma unroll
    for (int d = 0; d < D; ++d) ncand *= num[d];
    for (int k0 = 0; k0 < ncand; k0 += KBN_OWN_MAXC) {
        const int nk = min(KBN_OWN_MAXC, ncand - k0);
        __syncthreads();
        owner_stage<D>(o, first, num, k0, nk, toff, cbeg, coff);
        __syncthreads();
        const int tot = coff[nk];
        for (int i0 = 0; i0 < tot; i0 += KBN_OWN_BLOCK * KBN_OWN_ILP) {
            int p[KBN_OWN_ILP], rel[KBN_OWN_ILP][3];
            float fr[KBN_OWN_ILP][3];
            bool hit[KBN_OWN_ILP];
#pragma unroll
            for (int u = 0; u < KBN_OWN_ILP; ++u) {
                const int i = i0 + (int)threadIdx.x * KBN_OWN_ILP + u;
                const bool in = i < tot;
                const int k = owner_find(coff, nk, in ? i : 0);
                p[u] = in ? cbeg[k] + i - coff[k] : -1;
            }
#pragma unroll
            for (int u = 0; u < KBN_OWN_ILP; ++u)
                hit[u] = p[u] >= 0 && owner_touch<D>(o, p[u] < 0 ? 0 : p[u], M, cell, frac, lo, hi, rel[u], fr[u]);
            fold(p, hit, rel, fr);
        }
    }
}

// Entry count of every owner tile, pushed from the samples: a finite sample
// reaches, per axis, the owner tile holding its first tap and, when its J
// taps cross into the next tile (modulo K), that one too (owner tiles are at
// least J wide, so these are exactly the tiles whose cells its taps meet, the
// relation k_owner_write tests).  Lanes of a wavefront that reach the same
// tile add with one atomic; integer counts do not depend on the order.
template <int D>
__global__ void __launch_bounds__(KBN_BLOCK)
k_owner_count(OwnerGeom o, int64_t M, const int *__restrict__ cell, const float *__restrict__ frac,
              const int *__restrict__ toff, int *__restrict__ ocount) {
    const int64_t p = (int64_t)blockIdx.x * KBN_BLOCK + threadIdx.x;
    const bool act = p < toff[o.ntiles_sort];
    const int lane = threadIdx.x & 63;
    int first[3] = {0, 0, 0}, second[3] = {0, 0, 0}, num[3] = {1, 1, 1};
    if (act) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            int st;
            float f;
            tap_origin(o.J, cell[d * M + p], frac[d * M + p], st, f);
            const int K = o.K[d];
            const int sw = st < 0 ? st + K : st;
            int se = sw + o.J - 1;
            if (se >= K) se -= K;
            first[d] = sw / o.To[d];
            second[d] = se / o.To[d];
            num[d] = first[d] == second[d] ? 1 : 2;
        }
    }
#pragma unroll
    for (int k = 0; k < (1 << D); ++k) {
        bool on = act;
        int id = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int bit = (k >> (D - 1 - d)) & 1;
            on = on && bit < num[d];
            id = id * o.nto[d] + (bit ? second[d] : first[d]);
        }
        unsigned long long todo = __ballot(on);
        while (todo) {
            const int leader = __ffsll((long long)todo) - 1;
            const int key = __shfl(id, leader, 64);
            const unsigned long long same = __ballot(on && id == key) & todo;
            if (lane == leader) atomicAdd(&ocount[key], __popcll(same));
            todo &= ~same;
        }
    }
}

// Entries and their records of every owner tile (one workgroup per tile,
// the tiles with most entries dispatched first): the reaching samples of
// the candidate walk, compacted in walk order.
template <int D>
__global__ void __launch_bounds__(KBN_OWN_BLOCK)
k_owner_write(OwnerGeom o, int64_t M, const int *__restrict__ cell, const float *__restrict__ frac,
              const int *__restrict__ toff, const int *__restrict__ order, const int *__restrict__ ooff,
              const int *__restrict__ otile_order, int *__restrict__ rec_p, int *__restrict__ rec_q,
              int *__restrict__ rec_l, float *__restrict__ rec_f) {
    __shared__ int cbeg[KBN_OWN_MAXC], coff[KBN_OWN_MAXC + 1];
    __shared__ int wsum[KBN_OWN_BLOCK / 64];
    const int t = otile_order[blockIdx.x];  // tiles with the most entries first
    int run = ooff[t];
    owner_walk<D>(o, t, M, cell, frac, toff, cbeg, coff,
                  [&](const int *p, const bool *hit, int (*rel)[3], float (*fr)[3]) {
                      int h = 0;
#pragma unroll
                      for (int u = 0; u < KBN_OWN_ILP; ++u) h += hit[u] ? 1 : 0;
                      int total;
                      int e = run + block_scan_own(h, wsum, total);
#pragma unroll
                      for (int u = 0; u < KBN_OWN_ILP; ++u) {
                          if (!hit[u]) continue;
                          rec_p[e] = p[u];
                          rec_q[e] = order[p[u]];
#pragma unroll
                          for (int d = 0; d < D; ++d) {
                              rec_l[(int64_t)e * D + d] = rel[u][d];
                              rec_f[(int64_t)e * D + d] = fr[u][d];
                          }
                          ++e;
                      }
                      run += total;
                  });
}

__device__ __forceinline__ int owner_key(int c) { return c == 0 ? 32 : __clz(c); }  // larger counts first

// atomicAdd(&ctr[key], 1) for the active lanes of a wavefront, one LDS
// atomic per distinct key (lanes with equal keys get consecutive values in
// lane order); returns the lane's value.
__device__ __forceinline__ int wave_key_add(int *ctr, int key, bool active) {
    const int lane = threadIdx.x & 63;
    unsigned long long todo = __ballot(active);
    int mine = 0;
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int k = __shfl(key, leader, 64);
        const unsigned long long same = __ballot(active && key == k) & todo;
        int base = 0;
        if (lane == leader) base = atomicAdd(&ctr[k], __popcll(same));
        base = __shfl(base, leader, 64);
        if ((same >> lane) & 1ull) mine = base + __popcll(same & ((1ull << lane) - 1ull));
        todo &= ~same;
    }
    return mine;
}

// Exclusive scans of three values over a 1024-thread workgroup at once.
__device__ __forceinline__ void block_scan3_1024(int x[3], int ex[3], int tot[3], int (*wsum)[16]) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc[3] = {x[0], x[1], x[2]};
    for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int y = __shfl_up(inc[j], o, 64);
            if (lane >= o) inc[j] += y;
        }
    }
    if (lane == 63)
        for (int j = 0; j < 3; ++j) wsum[j][wid] = inc[j];
    lds_barrier();
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        int wpre = 0, t = 0;
        for (int w = 0; w < 16; ++w) {
            const int ws = wsum[j][w];
            if (w < wid) wpre += ws;
            t += ws;
        }
        ex[j] = wpre + inc[j] - x[j];
        tot[j] = t;
    }
    lds_barrier();
}

// One workgroup: owner offsets (exclusive scan of the counts, ooff[n] =
// total), the tiles in decreasing order of entry count, and the spread work
// items.
//
// Order: bins of log2 count, so the spread dispatches its longest
// workgroups first.  The order inside a bin is arbitrary; tiles are
// independent and a split tile's partial slots are consecutive and summed in
// item order, so results do not depend on it.
//
// Work items: tile t (hottest first) with n entries becomes ceil(n / seg)
// items of at most seg entries (one item if n == 0, so that every tile is
// written).  Tiles with several items get consecutive partial slots; seg
// doubles until the slots fit in `smax`.  Outputs:
//   work[i] = (tile, first entry, end entry, slot or -1), counts2[0] = items
//   comb[k] = (tile, first slot, number of slots),     counts2[1] = tiles
template <bool STAGED>
__global__ void __launch_bounds__(1024)
k_owner_finish(int ntiles, int seg, int smax, const int *__restrict__ ocount, int *__restrict__ ooff,
               int *__restrict__ order, int *__restrict__ work, int *__restrict__ comb,
               int *__restrict__ counts2) {
    // STAGED: counts, offsets and order live in LDS (dynamic, 3 ntiles ints)
    // and are written out at the end; else they are read and written in
    // global memory
    extern __shared__ int lds[];
    __shared__ int wsum[16];
    __shared__ int wsum3[3][16];
    __shared__ int hist[33], start[33];
    const int tid = threadIdx.x;
    const int nr = (ntiles + 1023) / 1024;
    int *off = STAGED ? lds + ntiles : ooff;
    int *ord = STAGED ? lds + 2 * ntiles : order;
    if (STAGED) {
#pragma unroll 4
        for (int t = tid; t < ntiles; t += 1024) lds[t] = ocount[t];
        lds_barrier();
    }
    const int *cnt = STAGED ? lds : ocount;
    // offsets
    int carry = 0;
    for (int r = 0; r < nr; ++r) {
        const int t = r * 1024 + tid;
        int total;
        const int ex = block_scan_1024(t < ntiles ? cnt[t] : 0, wsum, total);
        if (t < ntiles) off[t] = carry + ex;
        carry += total;
    }
    if (tid == 0) ooff[ntiles] = carry;
    // hottest-first order
    if (tid < 33) hist[tid] = 0;
    lds_barrier();
    for (int t0 = 0; t0 < ntiles; t0 += 1024) {
        const int t = t0 + tid;
        (void)wave_key_add(hist, t < ntiles ? owner_key(cnt[t]) : 0, t < ntiles);
    }
    lds_barrier();
    if (tid == 0) {
        int acc = 0;
        for (int k = 0; k < 33; ++k) {
            start[k] = acc;
            acc += hist[k];
        }
    }
    lds_barrier();
    for (int t0 = 0; t0 < ntiles; t0 += 1024) {
        const int t = t0 + tid;
        const int q = wave_key_add(start, owner_key(t < ntiles ? cnt[t] : 0), t < ntiles);
        if (t < ntiles) ord[q] = t;
    }
    // entries per work item: double seg until the split tiles' slots fit
    int sg = seg;
    for (int it = 0; it < 31; ++it) {
        int sl = 0;
        for (int t = tid; t < ntiles; t += 1024) {
            const int c = cnt[t];
            if (c > sg) sl += (c + sg - 1) / sg;
        }
        int total;
        (void)block_scan_1024(sl, wsum, total);
        if (total <= smax) break;
        sg *= 2;
    }
    if (STAGED)
        lds_barrier();
    else
        __syncthreads();  // order and offsets complete in global memory
    // positions in rounds: prefixes of items, slots and split tiles, and the
    // position's items written at once
    int cw = 0, cs = 0, cc = 0;
    for (int r = 0; r < nr; ++r) {
        const int q = r * 1024 + tid;
        const bool in = q < ntiles;
        const int t = in ? ord[q] : 0;
        const int c = in ? cnt[t] : 0;
        const int ns = in ? (c > sg ? (c + sg - 1) / sg : 1) : 0;
        int x[3] = {ns, ns > 1 ? ns : 0, ns > 1 ? 1 : 0}, ex[3], tot[3];
        block_scan3_1024(x, ex, tot, wsum3);
        if (in) {
            const int e0 = off[t];
            const int wi = cw + ex[0], si = cs + ex[1];
            for (int k = 0; k < ns; ++k) {
                int *w = work + 4 * (wi + k);
                w[0] = t;
                w[1] = e0 + k * sg;
                w[2] = min(e0 + (k + 1) * sg, e0 + c);
                w[3] = ns > 1 ? si + k : -1;
            }
            if (ns > 1) {
                int *cb = comb + 3 * (cc + ex[2]);
                cb[0] = t;
                cb[1] = si;
                cb[2] = ns;
            }
        }
        cw += tot[0];
        cs += tot[1];
        cc += tot[2];
    }
    if (tid == 0) {
        counts2[0] = cw;
        counts2[1] = cc;
    }
    if (STAGED) {
#pragma unroll 4
        for (int t = tid; t < ntiles; t += 1024) {
            ooff[t] = off[t];
            order[t] = ord[t];
        }
    }
}

}  // namespace

// Histograms of more than 16384 bins need more than the default 64 KiB of
// dynamic LDS per workgroup; gfx950 allows up to 160 KiB once a kernel opts in.
hipError_t allow_large_lds(size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    static const hipError_t once = [] {
        const void *ks[] = {(const void *)k_points_hist, (const void *)k_tile_scatter<1>,
                            (const void *)k_tile_scatter<2>, (const void *)k_tile_scatter<3>,
                            (const void *)k_owner_finish<true>};
        hipError_t r = hipSuccess;
        for (const void *k : ks) {
            // the dynamic part may take what the kernel's static LDS leaves
            hipFuncAttributes fa;
            hipError_t e = hipFuncGetAttributes(&fa, k);
            if (e == hipSuccess)
                e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        160 * 1024 - (int)fa.sharedSizeBytes);
            if (e != hipSuccess) r = e;
        }
        return r;
    }();
    return once;
}

int kbn_points_chunks(int64_t M, int ntiles, int *chunk) {
    const int64_t nbins = (int64_t)ntiles + 1;
    if (M <= 0) {
        *chunk = 64;
        return 0;
    }
    // at most 4096 samples per chunk (one wavefront ranks a chunk in steps of
    // 64); otherwise as many chunks as keep the count matrix within one
    // workgroup's scan, and at least 256 samples per chunk
    const int64_t nmin = (M + 4095) / 4096;
    const int64_t nsmall = std::max<int64_t>(1, KBN_SCAN_SMALL / nbins);
    const int64_t n256 = std::max<int64_t>(1, M / 256);
    const int64_t want = std::max(nmin, std::min(nsmall, n256));
    int64_t c = (M + want - 1) / want;
    c = (c + 63) / 64 * 64;
    *chunk = (int)c;
    return (int)((M + c - 1) / c);
}

int64_t kbn_points_owner_base(int64_t M, int ntiles) {
    int chunk;
    const int64_t nch = kbn_points_chunks(M, ntiles, &chunk);
    const int64_t S = nch * ((int64_t)ntiles + 1);
    return S + S / KBN_SCAN_SPAN + 2;  // the count matrix and the three-phase scan's span sums
}

int64_t kbn_points_counts_size(int64_t M, int ntiles, int ntiles_own) {
    // then the owner tiles' entry counts
    return kbn_points_owner_base(M, ntiles) + (int64_t)ntiles_own + 1;
}

hipError_t kbn_launch_points(int D, int64_t M, const float *omega, const double *scale,
                             const int *K, const int *T, const int *nt, int ntiles, int ntiles_own,
                             int sub, const KbnPointsBufs &b, hipStream_t s, hipEvent_t omega_read) {
    const int nbins = ntiles + 1;
    int *ocount = b.counts + kbn_points_owner_base(M, ntiles);
    {
        const hipError_t e = allow_large_lds(sizeof(int) * (size_t)nbins);
        if (e != hipSuccess) return e;
    }
    int chunk;
    const int nchunks = kbn_points_chunks(M, ntiles, &chunk);
    if (M > 0)
        k_points_hist<<<dim3(nchunks), dim3(256), sizeof(int) * nbins, s>>>(
            D, M, chunk, nchunks, nbins, omega, scale[0], D > 1 ? scale[1] : 0.0, D > 2 ? scale[2] : 0.0,
            K[0], D > 1 ? K[1] : 1, D > 2 ? K[2] : 1, T[0], D > 1 ? T[1] : 1, D > 2 ? T[2] : 1,
            D > 1 ? nt[1] : 1, D > 2 ? nt[2] : 1, ntiles, b.cell_tmp, b.frac_tmp, b.tile, b.flag, b.counts);
    if (omega_read) {  // omega is not read after this kernel
        const hipError_t e = hipEventRecord(omega_read, s);
        if (e != hipSuccess) return e;
    }
    const int64_t S = (int64_t)nbins * nchunks;
    if (S <= KBN_SCAN_SMALL) {
        k_scan_small<<<dim3(1), dim3(1024), 0, s>>>((int)S, std::max(nchunks, 1), nbins, sub, b.counts, b.toff,
                                                    b.subs, b.nsub);
    } else {
        int *bsum = b.counts + S;
        const int nb = (int)((S + KBN_SCAN_SPAN - 1) / KBN_SCAN_SPAN);
        k_scan_sums<<<dim3(nb), dim3(1024), 0, s>>>(S, b.counts, bsum);
        k_scan_top<<<dim3(1), dim3(1024), 0, s>>>(nb, bsum);
        k_scan_apply<<<dim3(nb), dim3(1024), 0, s>>>(S, b.counts, bsum);
        k_scan_offsets<<<dim3((nbins + 256) / 256), dim3(256), 0, s>>>(S, nchunks, nbins, b.counts, bsum, nb,
                                                                       b.toff);
        k_subproblems<<<dim3(1), dim3(1024), 0, s>>>(nbins, sub, b.toff, b.subs, b.nsub);
    }
    if (M > 0) {
        int nbits = 0;
        while ((1 << nbits) < nbins) ++nbits;
        auto kern = D == 1 ? k_tile_scatter<1> : (D == 2 ? k_tile_scatter<2> : k_tile_scatter<3>);
        kern<<<dim3(nchunks), dim3(64), sizeof(int) * nbins, s>>>(M, chunk, nchunks, nbins, nbits, b.tile,
                                                                  b.counts, b.cell_tmp, b.frac_tmp, b.order,
                                                                  b.cell, b.frac, ocount, ntiles_own);
    } else {
        k_zero_ints<<<dim3((ntiles_own + 255) / 256), dim3(256), 0, s>>>(ocount, ntiles_own);
    }
    return hipGetLastError();
}

hipError_t kbn_launch_owner_lists(const KbnGeom &g, int64_t M, const int *cell, const float *frac,
                                  const int *toff, const int *order, int *ocount, int *ooff,
                                  int *otile_order, int seg, int smax, int *swork, int *scomb, int *scounts,
                                  int *rec_p, int *rec_q, int *rec_l, float *rec_f, hipStream_t s) {
    OwnerGeom o;
    o.D = g.D;
    o.J = g.J;
    o.LO = (g.J & 1) ? g.J / 2 : g.J / 2 - 1;
    o.HI = (g.J & 1) ? g.J / 2 + 1 : g.J / 2;
    o.ntiles_sort = g.ntiles;
    o.ntiles_own = g.ntiles_own;
    for (int d = 0; d < 3; ++d) {
        o.K[d] = d < g.D ? g.K[d] : 1;
        o.To[d] = d < g.D ? g.To[d] : 1;
        o.nto[d] = d < g.D ? g.nto[d] : 1;
        o.T[d] = d < g.D ? g.T[d] : 1;
        o.nt[d] = d < g.D ? g.nt[d] : 1;
    }
    const int n = g.ntiles_own;
    {
        const hipError_t e = allow_large_lds(3 * sizeof(int) * (size_t)std::min(n, KBN_OWN_LDS));
        if (e != hipSuccess) return e;
    }
    switch (g.D) {
#define KBN_OWN(d)                                                                                     \
    case d:                                                                                            \
        if (M > 0)                                                                                     \
            k_owner_count<d><<<dim3((unsigned)((M + KBN_BLOCK - 1) / KBN_BLOCK)), dim3(KBN_BLOCK), 0,  \
                               s>>>(o, M, cell, frac, toff, ocount);                                   \
        if (n <= KBN_OWN_LDS)                                                                          \
            k_owner_finish<true><<<dim3(1), dim3(1024), 3 * sizeof(int) * n, s>>>(                     \
                n, seg, smax, ocount, ooff, otile_order, swork, scomb, scounts);                       \
        else                                                                                           \
            k_owner_finish<false><<<dim3(1), dim3(1024), 0, s>>>(n, seg, smax, ocount, ooff,           \
                                                                 otile_order, swork, scomb, scounts);  \
        k_owner_write<d><<<dim3(n), dim3(KBN_OWN_BLOCK), 0, s>>>(o, M, cell, frac, toff, order, ooff,  \
                                                                 otile_order, rec_p, rec_q, rec_l,     \
                                                                 rec_f);                               \
        break;
        KBN_OWN(1) KBN_OWN(2) KBN_OWN(3)
#undef KBN_OWN
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
