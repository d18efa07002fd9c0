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

// Single-workgroup exclusive scan of the bin-major count matrix; also emits
// the tile offsets toff[b] = first sorted position of bin b, toff[nbins] = M.
__global__ void __launch_bounds__(1024)
k_scan(int64_t S, int nchunks, int nbins, int64_t M, int *__restrict__ counts,
       int *__restrict__ toff) {
    __shared__ int part[1024];
    const int tid = threadIdx.x;
    const int64_t seg = (S + 1023) / 1024;
    const int64_t beg = tid * seg;
    const int64_t end = beg + seg < S ? beg + seg : S;
    int sum = 0;
    for (int64_t i = beg; i < end; ++i) sum += counts[i];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // Hillis-Steele inclusive scan
        int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = part[tid] - sum;  // exclusive prefix of this segment
    for (int64_t i = beg; i < end; ++i) {
        const int c = counts[i];
        counts[i] = run;
        run += c;
    }
    __syncthreads();
    for (int b = tid; b < nbins; b += 1024) toff[b] = S > 0 ? counts[(int64_t)b * nchunks] : 0;
    if (tid == 0) toff[nbins] = (int)M;
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

}  // namespace

hipError_t kbn_launch_points(int D, int64_t M, const float *omega, const double *scale,
                             const int *K, const int *T, const int *nt, int ntiles,
                             int chunk, int nchunks, const KbnPointsBufs &b, hipStream_t s) {
    const int nbins = ntiles + 1;
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
    k_scan<<<dim3(1), dim3(1024), 0, s>>>(S, M > 0 ? nchunks : 1, nbins, M, b.counts, b.toff);
    if (M > 0) {
        int nbits = 0;
        while ((1 << nbits) < nbins) ++nbits;
        k_tile_scatter<<<dim3(nchunks), dim3(64), sizeof(int) * nbins, s>>>(
            D, M, chunk, nchunks, nbins, nbits, b.tile, b.counts, b.cell_tmp, b.frac_tmp, b.order,
            b.cell, b.frac);
    }
    return hipGetLastError();
}
