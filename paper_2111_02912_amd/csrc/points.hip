// Index pass: grid cell, in-cell fraction and tile of every sample location,
// then a stable counting sort of the samples by tile.
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

namespace {

constexpr double kULimit = 1099511627776.0;  // 2^40

__global__ void __launch_bounds__(KBN_BLOCK)
k_points_cells(int D, int64_t M, const float *__restrict__ omega, double s0, double s1,
               double s2, int K0, int K1, int K2, int T0, int T1, int T2, int nt1, int nt2,
               int ntiles, int *__restrict__ cell_tmp, float *__restrict__ frac_tmp,
               int *__restrict__ tile, int *__restrict__ flag) {
#pragma clang fp contract(off)
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const double sc[3] = {s0, s1, s2};
    const int Kd[3] = {K0, K1, K2};
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
}

// One wavefront per chunk: histogram of tile ids in LDS, written bin-major.
__global__ void __launch_bounds__(64)
k_tile_hist(int64_t M, int chunk, int nchunks, int nbins, const int *__restrict__ tile,
            int *__restrict__ counts) {
    extern __shared__ int hist[];
    const int ch = blockIdx.x;
    for (int i = threadIdx.x; i < nbins; i += 64) hist[i] = 0;
    __syncthreads();
    const int64_t beg = (int64_t)ch * chunk;
    const int64_t end = beg + chunk < M ? beg + chunk : M;
    for (int64_t m = beg + threadIdx.x; m < end; m += 64) atomicAdd(&hist[tile[m]], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += 64) counts[(int64_t)i * nchunks + ch] = hist[i];
}

// Exclusive scan of the per-(bin, chunk) counts, in bin-major order, in
// place: counts[b * nchunks + c] becomes the first output position of chunk c's
// points of bin b; toff[b] = start of bin b and toff[nbins] = total count.
// Three phases over spans of KBN_SCAN_SPAN counts: span sums, an exclusive
// scan of the span sums (one workgroup), then each span rescanned with its
// offset.  Integer sums, so the order of additions does not matter.
#define KBN_SCAN_SPAN 8192

__device__ __forceinline__ int block_scan_1024(int x, int *wsum, int &total) {
    // inclusive scan over a 1024-thread block; returns the exclusive prefix
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int inc = x;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int wpre = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
        const int ws = wsum[w];
        if (w < wid) wpre += ws;
        tot += ws;
    }
    __syncthreads();
    total = tot;
    return wpre + inc - x;
}

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

hipError_t scan_counts(int64_t S, int nchunks, int nbins, int *counts, int *bsum, int *toff,
                       hipStream_t s) {
    const int nb = (int)((S + KBN_SCAN_SPAN - 1) / KBN_SCAN_SPAN);
    if (nb > 0) {
        k_scan_sums<<<dim3(nb), dim3(1024), 0, s>>>(S, counts, bsum);
        k_scan_top<<<dim3(1), dim3(1024), 0, s>>>(nb, bsum);
        k_scan_apply<<<dim3(nb), dim3(1024), 0, s>>>(S, counts, bsum);
    }
    k_scan_offsets<<<dim3((nbins + 256) / 256), dim3(256), 0, s>>>(S, nchunks, nbins, counts, bsum, nb,
                                                                   toff);
    return hipGetLastError();
}

// One wavefront per chunk: stable scatter.  Lanes with equal tile ids are
// grouped with ballots; rank = number of equal lanes below, so within a
// chunk the input order is kept, and chunks occupy consecutive ranges.
__global__ void __launch_bounds__(64)
k_tile_scatter(int D, int64_t M, int chunk, int nchunks, int nbins, int nbits,
               const int *__restrict__ tile, const int *__restrict__ counts,
               const int *__restrict__ cell_tmp, const float *__restrict__ frac_tmp,
               int *__restrict__ order, int *__restrict__ cell, float *__restrict__ frac) {
    extern __shared__ int cursor[];
    const int ch = blockIdx.x;
    const int lane = threadIdx.x;
    for (int i = lane; i < nbins; i += 64) cursor[i] = counts[(int64_t)i * nchunks + ch];
    __syncthreads();
    const int64_t beg = (int64_t)ch * chunk;
    const int64_t end = beg + chunk < M ? beg + chunk : M;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int64_t base = beg; base < end; base += 64) {
        const int64_t m = base + lane;
        const bool valid = m < end;
        const int t = valid ? tile[m] : -1;
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
        __syncthreads();
        if (valid && rank == 0) cursor[t] = pos + cnt;
        __syncthreads();
        if (valid) {
            order[pos] = (int)m;
            for (int d = 0; d < D; ++d) {
                cell[d * M + pos] = cell_tmp[d * M + m];
                frac[d * M + pos] = frac_tmp[d * M + m];
            }
        }
    }
}

// Subproblem list: bin t with n points contributes ceil(n / sub) entries
// (bin, first sorted position); the last bin holds the flagged points.
// Single workgroup; subs holds at most ceil(M / sub) + nbins entries.
__global__ void __launch_bounds__(1024)
k_subproblems(int nbins, int sub, const int *__restrict__ toff, int *__restrict__ subs,
              int *__restrict__ nsub) {
    __shared__ int part[1024];
    const int tid = threadIdx.x;
    const int seg = (nbins + 1023) / 1024;
    const int beg = tid * seg;
    const int end = min(beg + seg, nbins);
    int sum = 0;
    for (int t = beg; t < end; ++t) sum += (toff[t + 1] - toff[t] + sub - 1) / sub;
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = part[tid] - sum;
    for (int t = beg; t < end; ++t) {
        for (int q = toff[t]; q < toff[t + 1]; q += sub) {
            subs[2 * run] = t;
            subs[2 * run + 1] = q;
            ++run;
        }
    }
    if (tid == 1023) *nsub = part[1023];
}

// ---------------------------------------------------------------------------
// Owner-tile touch lists for the spread.  A finite sample whose J taps along
// axis d start at grid cell s_d reaches owner tiles floor(wrap(s_d)/To_d) and
// floor(wrap(s_d + J - 1)/To_d) (one or two tiles per axis, since To_d >= J
// and no owner tile is narrower than J).  Every (sample, reached tile) pair
// becomes one entry; entries are grouped by tile with a counting sort whose
// order inside a tile is fixed (chunk order, then combination index, then
// sample order), so the spread's accumulation order is deterministic.
struct OwnerGeom {
    int D, J, ntiles_sort;
    int K[3], To[3], nto[3];
};

__device__ __forceinline__ int touch_tiles(const OwnerGeom &o, int p, int64_t M,
                                           const int *__restrict__ cell,
                                           const float *__restrict__ frac, int first[3],
                                           int num[3]) {
    int total = 1;
    for (int d = 0; d < o.D; ++d) {
        const int c = cell[d * M + p];
        const float f = frac[d * M + p];
        int start;
        if ((o.J & 1) == 0)
            start = c - o.J / 2 + 1;
        else
            start = f >= 0.5f ? c - o.J / 2 + 1 : c - o.J / 2;
        int s0 = start < 0 ? start + o.K[d] : start;
        int s1 = start + o.J - 1;
        if (s1 >= o.K[d]) s1 -= o.K[d];
        if (s1 < 0) s1 += o.K[d];
        const int t0 = s0 / o.To[d], t1 = s1 / o.To[d];
        first[d] = t0;
        num[d] = t0 == t1 ? 1 : 2;
        total *= num[d];
    }
    return total;
}

// k-th reached tile of a sample (k < total), row-major over the axes.
__device__ __forceinline__ int touch_tile_id(const OwnerGeom &o, const int first[3],
                                             const int num[3], int k) {
    int id = 0;
    int rem = k;
    int sel[3];
    for (int d = o.D - 1; d >= 0; --d) {
        sel[d] = rem % num[d];
        rem /= num[d];
    }
    for (int d = 0; d < o.D; ++d) {
        int t = first[d] + sel[d];
        if (t >= o.nto[d]) t -= o.nto[d];
        id = id * o.nto[d] + t;
    }
    return id;
}

__global__ void __launch_bounds__(64)
k_owner_hist(OwnerGeom o, int64_t M, int chunk, int nchunks, int nbins,
             const int *__restrict__ cell, const float *__restrict__ frac,
             const int *__restrict__ toff, int *__restrict__ counts) {
    extern __shared__ int hist[];
    const int ch = blockIdx.x;
    for (int i = threadIdx.x; i < nbins; i += 64) hist[i] = 0;
    __syncthreads();
    const int64_t ngood = toff[o.ntiles_sort];
    const int64_t beg = (int64_t)ch * chunk;
    const int64_t end = beg + chunk < ngood ? beg + chunk : ngood;
    for (int64_t p = beg + threadIdx.x; p < end; p += 64) {
        int first[3], num[3];
        const int tot = touch_tiles(o, (int)p, M, cell, frac, first, num);
        for (int k = 0; k < tot; ++k) atomicAdd(&hist[touch_tile_id(o, first, num, k)], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += 64) counts[(int64_t)i * nchunks + ch] = hist[i];
}

__global__ void __launch_bounds__(64)
k_owner_scatter(OwnerGeom o, int64_t M, int chunk, int nchunks, int nbins, int nbits,
                const int *__restrict__ cell, const float *__restrict__ frac,
                const int *__restrict__ toff, const int *__restrict__ counts,
                int *__restrict__ entries) {
    extern __shared__ int cursor[];
    const int ch = blockIdx.x;
    const int lane = threadIdx.x;
    for (int i = lane; i < nbins; i += 64) cursor[i] = counts[(int64_t)i * nchunks + ch];
    __syncthreads();
    const int64_t ngood = toff[o.ntiles_sort];
    const int64_t beg = (int64_t)ch * chunk;
    const int64_t end = beg + chunk < ngood ? beg + chunk : ngood;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int maxk = 1 << o.D;
    for (int64_t base = beg; base < end; base += 64) {
        const int64_t p = base + lane;
        const bool valid = p < end;
        int first[3] = {0, 0, 0}, num[3] = {1, 1, 1};
        int tot = 0;
        if (valid) tot = touch_tiles(o, (int)p, M, cell, frac, first, num);
        for (int k = 0; k < maxk; ++k) {
            const bool act = k < tot;
            const int t = act ? touch_tile_id(o, first, num, k) : -1;
            unsigned long long peers = ~0ull;
            for (int bit = 0; bit <= nbits; ++bit) {
                const bool on = (t >> bit) & 1;
                const unsigned long long bal = __ballot(on);
                peers &= on ? bal : ~bal;
            }
            const int rank = __popcll(peers & below);
            const int cnt = __popcll(peers);
            int pos = 0;
            if (act) pos = cursor[t] + rank;
            __syncthreads();
            if (act && rank == 0) cursor[t] = pos + cnt;
            __syncthreads();
            if (act) entries[pos] = (int)p;
        }
    }
}

// Owner tiles in decreasing order of entry count (bins of log2 count), so
// that the spread dispatches its longest workgroups first.  The order inside
// a bin is arbitrary; tiles are independent, so results do not depend on it.
__global__ void __launch_bounds__(1024)
k_tile_order(int ntiles, const int *__restrict__ ooff, int *__restrict__ order) {
    __shared__ int hist[33];
    __shared__ int start[33];
    const int tid = threadIdx.x;
    if (tid < 33) hist[tid] = 0;
    __syncthreads();
    for (int t = tid; t < ntiles; t += 1024) {
        const int c = ooff[t + 1] - ooff[t];
        const int key = c == 0 ? 32 : __clz(c);  // larger counts -> smaller key
        atomicAdd(&hist[key], 1);
    }
    __syncthreads();
    if (tid == 0) {
        int r = 0;
        for (int k = 0; k < 33; ++k) {
            start[k] = r;
            r += hist[k];
        }
    }
    __syncthreads();
    for (int t = tid; t < ntiles; t += 1024) {
        const int c = ooff[t + 1] - ooff[t];
        const int key = c == 0 ? 32 : __clz(c);
        order[atomicAdd(&start[key], 1)] = t;
    }
}

// Spread work items.  Tile t (taken in hottest-first order) with n entries
// becomes ceil(n / seg) items of at most seg entries (one item if n == 0, so
// that every tile is written).  Tiles with several items get consecutive
// partial slots; seg doubles until the slots fit in `smax`.  Outputs:
//   work[i] = (tile, first entry, end entry, slot or -1), nwork
//   comb[k] = (tile, first slot, number of slots), ncomb
__global__ void __launch_bounds__(1024)
k_spread_work(int ntiles, int seg, int smax, const int *__restrict__ ooff,
              const int *__restrict__ order, int *__restrict__ work, int *__restrict__ comb,
              int *__restrict__ counts2) {
    __shared__ int part_w[1024], part_s[1024], part_c[1024];
    __shared__ int seg_s;
    const int tid = threadIdx.x;
    const int per = (ntiles + 1023) / 1024;
    const int beg = tid * per;
    const int end = min(beg + per, ntiles);
    if (tid == 0) seg_s = seg;
    __syncthreads();
    for (int it = 0; it < 31; ++it) {  // grow seg until the slots fit
        const int sg = seg_s;
        int sl = 0;
        for (int r = beg; r < end; ++r) {
            const int t = order[r];
            const int c = ooff[t + 1] - ooff[t];
            const int ns = c > sg ? (c + sg - 1) / sg : 1;
            if (ns > 1) sl += ns;
        }
        part_s[tid] = sl;
        __syncthreads();
        for (int off = 512; off > 0; off >>= 1) {
            if (tid < off) part_s[tid] += part_s[tid + off];
            __syncthreads();
        }
        const bool fits = part_s[0] <= smax;
        __syncthreads();
        if (fits) break;
        if (tid == 0) seg_s = 2 * sg;
        __syncthreads();
    }
    const int sg = seg_s;
    int nw = 0, ns_tot = 0, nc = 0;
    for (int r = beg; r < end; ++r) {
        const int t = order[r];
        const int c = ooff[t + 1] - ooff[t];
        const int ns = c > sg ? (c + sg - 1) / sg : 1;
        nw += ns;
        if (ns > 1) {
            ns_tot += ns;
            nc += 1;
        }
    }
    part_w[tid] = nw;
    part_s[tid] = ns_tot;
    part_c[tid] = nc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive scans
        const int a = tid >= off ? part_w[tid - off] : 0;
        const int b = tid >= off ? part_s[tid - off] : 0;
        const int cc = tid >= off ? part_c[tid - off] : 0;
        __syncthreads();
        part_w[tid] += a;
        part_s[tid] += b;
        part_c[tid] += cc;
        __syncthreads();
    }
    int wi = part_w[tid] - nw, si = part_s[tid] - ns_tot, ci = part_c[tid] - nc;
    for (int r = beg; r < end; ++r) {
        const int t = order[r];
        const int e0 = ooff[t], c = ooff[t + 1] - e0;
        const int ns = c > sg ? (c + sg - 1) / sg : 1;
        for (int k = 0; k < ns; ++k) {
            int *w = work + 4 * wi++;
            w[0] = t;
            w[1] = e0 + k * sg;
            w[2] = min(e0 + (k + 1) * sg, e0 + c);
            w[3] = ns > 1 ? si + k : -1;
        }
        if (ns > 1) {
            int *cb = comb + 3 * ci++;
            cb[0] = t;
            cb[1] = si;
            cb[2] = ns;
            si += ns;
        }
    }
    if (tid == 1023) {
        counts2[0] = part_w[1023];
        counts2[1] = part_c[1023];
    }
}

}  // namespace

// Histograms of more than 16384 bins need more than the default 64 KiB of
// dynamic LDS per workgroup; gfx950 allows up to 160 KiB once a kernel opts in.
hipError_t allow_large_lds(size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    static const hipError_t once = [] {
        const void *ks[] = {(const void *)k_tile_hist, (const void *)k_tile_scatter,
                            (const void *)k_owner_hist, (const void *)k_owner_scatter};
        hipError_t r = hipSuccess;
        for (const void *k : ks) {
            const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) r = e;
        }
        return r;
    }();
    return once;
}

hipError_t kbn_launch_owner_lists(int D, int J, int ntiles_sort, const int *K, const int *To,
                                  const int *nto, int ntiles_own, int64_t M, int chunk,
                                  int nchunks, const int *cell, const float *frac,
                                  const int *toff, int *counts, int *ooff, int *entries,
                                  int *otile_order, int seg, int smax, int *swork, int *scomb,
                                  int *scounts, hipStream_t s) {
    OwnerGeom o;
    o.D = D;
    o.J = J;
    o.ntiles_sort = ntiles_sort;
    for (int d = 0; d < 3; ++d) {
        o.K[d] = d < D ? K[d] : 1;
        o.To[d] = d < D ? To[d] : 1;
        o.nto[d] = d < D ? nto[d] : 1;
    }
    const int nbins = ntiles_own;
    {
        const hipError_t e = allow_large_lds(sizeof(int) * (size_t)nbins);
        if (e != hipSuccess) return e;
    }
    if (M > 0)
        k_owner_hist<<<dim3(nchunks), dim3(64), sizeof(int) * nbins, s>>>(
            o, M, chunk, nchunks, nbins, cell, frac, toff, counts);
    const int64_t S = (int64_t)nbins * (M > 0 ? nchunks : 0);
    // ooff[nbins] receives the total entry count
    const hipError_t es = scan_counts(S, M > 0 ? nchunks : 1, nbins, counts, counts + S, ooff, s);
    if (es != hipSuccess) return es;
    if (M > 0) {
        int nbits = 0;
        while ((1 << nbits) < nbins) ++nbits;
        k_owner_scatter<<<dim3(nchunks), dim3(64), sizeof(int) * nbins, s>>>(
            o, M, chunk, nchunks, nbins, nbits, cell, frac, toff, counts, entries);
    }
    k_tile_order<<<dim3(1), dim3(1024), 0, s>>>(nbins, ooff, otile_order);
    k_spread_work<<<dim3(1), dim3(1024), 0, s>>>(nbins, seg, smax, ooff, otile_order, swork, scomb,
                                                 scounts);
    return hipGetLastError();
}

hipError_t kbn_launch_points(int D, int64_t M, const float *omega, const double *scale,
                             const int *K, const int *T, const int *nt, int ntiles,
                             int chunk, int nchunks, int sub, const KbnPointsBufs &b, hipStream_t s) {
    const int nbins = ntiles + 1;
    {
        const hipError_t e = allow_large_lds(sizeof(int) * (size_t)nbins);
        if (e != hipSuccess) return e;
    }
    if (M > 0) {
        const int64_t blocks = (M + KBN_BLOCK - 1) / KBN_BLOCK;
        k_points_cells<<<dim3((unsigned)blocks), dim3(KBN_BLOCK), 0, s>>>(
            D, M, omega, scale[0], D > 1 ? scale[1] : 0.0, D > 2 ? scale[2] : 0.0, K[0],
            D > 1 ? K[1] : 1, D > 2 ? K[2] : 1, T[0], D > 1 ? T[1] : 1, D > 2 ? T[2] : 1,
            D > 1 ? nt[1] : 1, D > 2 ? nt[2] : 1, ntiles, b.cell_tmp, b.frac_tmp, b.tile, b.flag);
        k_tile_hist<<<dim3(nchunks), dim3(64), sizeof(int) * nbins, s>>>(M, chunk, nchunks, nbins,
                                                                          b.tile, b.counts);
    }
    const int64_t S = (int64_t)nbins * (M > 0 ? nchunks : 0);
    const hipError_t es = scan_counts(S, M > 0 ? nchunks : 1, nbins, b.counts, b.counts + S, b.toff, s);
    if (es != hipSuccess) return es;
    if (M > 0) {
        int nbits = 0;
        while ((1 << nbits) < nbins) ++nbits;
        k_tile_scatter<<<dim3(nchunks), dim3(64), sizeof(int) * nbins, s>>>(
            D, M, chunk, nchunks, nbins, nbits, b.tile, b.counts, b.cell_tmp, b.frac_tmp, b.order,
            b.cell, b.frac);
    }
    k_subproblems<<<dim3(1), dim3(1024), 0, s>>>(nbins, sub, b.toff, b.subs, b.nsub);
    return hipGetLastError();
}
