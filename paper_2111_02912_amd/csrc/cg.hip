// Conjugate-gradient vector kernels for the quadratic reconstruction
// (E^H E + lambda T^H T) x = b of Sec. IV-B: T = I (CG-SENSE) or T = the
// first differences along each image axis (QPLS), zero beyond the image
// edge; residual norm ||r|| / ||b|| of Sec. IV-A.  A launch serves a batch
// of independent images: one grid row per image, each with its own partial
// sums and scalars.
//
// Inner products are reduced deterministically: a fixed grid for a given
// length, one FP64 partial per block in a fixed tree order, then one block
// sums the partials in a fixed order and updates the CG scalars on the
// device, so no host round trip is needed between iterations and a solve
// gives the same bits whatever else runs on the GPU.
#include <algorithm>

#include "kbn_internal.h"

namespace {

constexpr int TPB = 256;

__device__ inline double block_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = TPB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    return sh[0];
}

// x = 0, p = r, partial |r|^2
__global__ __launch_bounds__(TPB) void k_cg_init(float2 *__restrict__ x, const float2 *__restrict__ r,
                                                 float2 *__restrict__ p, int64_t n,
                                                 double *__restrict__ part) {
    __shared__ double sh[TPB];
    const int64_t im = blockIdx.y;  // image of this block
    x += im * n;
    r += im * n;
    p += im * n;
    part += im * KBN_CG_MAXPARTS;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
        const float2 v = r[i];
        x[i] = make_float2(0.f, 0.f);
        p[i] = v;
        acc += (double)v.x * v.x + (double)v.y * v.y;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// q += lambda p, partial Re <p, q>
__global__ __launch_bounds__(TPB) void k_cg_q(float2 *__restrict__ q, const float2 *__restrict__ p,
                                              float lam, int64_t n, double *__restrict__ part) {
    __shared__ double sh[TPB];
    const int64_t im = blockIdx.y;  // image of this block
    q += im * n;
    p += im * n;
    part += im * KBN_CG_MAXPARTS;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
        const float2 pv = p[i];
        float2 qv = q[i];
        qv.x += lam * pv.x;
        qv.y += lam * pv.y;
        q[i] = qv;
        acc += (double)pv.x * qv.x + (double)pv.y * qv.y;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// q += lambda T^H T p for T = first differences along each axis (the
// path-graph Laplacian per axis: sum over in-image neighbours of p_i - p_nb),
// partial Re <p, q>.  Image [n0][n1][n2] row-major.
__global__ __launch_bounds__(TPB) void k_cg_q_fd(float2 *__restrict__ q, const float2 *__restrict__ p,
                                                 float lam, int n0, int n1, int n2, int64_t n,
                                                 double *__restrict__ part) {
    __shared__ double sh[TPB];
    const int64_t im = blockIdx.y;  // image of this block
    q += im * n;
    p += im * n;
    part += im * KBN_CG_MAXPARTS;
    const int64_t s0 = (int64_t)n1 * n2;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
        const int i2 = (int)(i % n2);
        const int64_t t = i / n2;
        const int i1 = (int)(t % n1);
        const int i0 = (int)(t / n1);
        const float2 c = p[i];
        float lx = 0.f, ly = 0.f;
        if (i0 > 0) { const float2 v = p[i - s0]; lx += c.x - v.x; ly += c.y - v.y; }
        if (i0 < n0 - 1) { const float2 v = p[i + s0]; lx += c.x - v.x; ly += c.y - v.y; }
        if (i1 > 0) { const float2 v = p[i - n2]; lx += c.x - v.x; ly += c.y - v.y; }
        if (i1 < n1 - 1) { const float2 v = p[i + n2]; lx += c.x - v.x; ly += c.y - v.y; }
        if (i2 > 0) { const float2 v = p[i - 1]; lx += c.x - v.x; ly += c.y - v.y; }
        if (i2 < n2 - 1) { const float2 v = p[i + 1]; lx += c.x - v.x; ly += c.y - v.y; }
        float2 qv = q[i];
        qv.x += lam * lx;
        qv.y += lam * ly;
        q[i] = qv;
        acc += (double)c.x * qv.x + (double)c.y * qv.y;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// x += alpha p, r -= alpha q, partial |r|^2
__global__ __launch_bounds__(TPB) void k_cg_xr(float2 *__restrict__ x, float2 *__restrict__ r,
                                               const float2 *__restrict__ p,
                                               const float2 *__restrict__ q,
                                               const double *__restrict__ scal, int64_t n,
                                               double *__restrict__ part) {
    __shared__ double sh[TPB];
    const int64_t im = blockIdx.y;  // image of this block
    x += im * n;
    r += im * n;
    p += im * n;
    q += im * n;
    scal += im * KBN_CG_NSCAL;
    part += im * KBN_CG_MAXPARTS;
    const float a = (float)scal[KBN_CG_ALPHA];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
        const float2 pv = p[i], qv = q[i];
        float2 xv = x[i], rv = r[i];
        xv.x += a * pv.x;
        xv.y += a * pv.y;
        rv.x -= a * qv.x;
        rv.y -= a * qv.y;
        x[i] = xv;
        r[i] = rv;
        acc += (double)rv.x * rv.x + (double)rv.y * rv.y;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// p = r + beta p
__global__ __launch_bounds__(TPB) void k_cg_p(float2 *__restrict__ p, const float2 *__restrict__ r,
                                              const double *__restrict__ scal, int64_t n) {
    const int64_t im = blockIdx.y;  // image of this block
    p += im * n;
    r += im * n;
    scal += im * KBN_CG_NSCAL;
    const float b = (float)scal[KBN_CG_BETA];
    for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
        const float2 rv = r[i];
        float2 pv = p[i];
        pv.x = rv.x + b * pv.x;
        pv.y = rv.y + b * pv.y;
        p[i] = pv;
    }
}

// Sum the block partials and update the scalars.
//   stage 0 (start):  rr = bb = sum, rel = 1 (0 when b = 0), iters = 0
//   stage 1 (p'q):    pq = sum, alpha = rr / pq (0 unless both are > 0)
//   stage 2 (new rr): beta = sum / rr (0 unless rr > 0), rr = sum,
//                     rel = sqrt(rr / bb), iters += 1
__global__ __launch_bounds__(TPB) void k_cg_scalars(const double *__restrict__ part, int nparts,
                                                    double *__restrict__ scal, int stage) {
    __shared__ double sh[TPB];
    const int64_t im = blockIdx.x;  // one block per image
    part += im * KBN_CG_MAXPARTS;
    scal += im * KBN_CG_NSCAL;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += TPB) acc += part[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x != 0) return;
    if (stage == 0) {
        scal[KBN_CG_RR] = s;
        scal[KBN_CG_BB] = s;
        scal[KBN_CG_REL] = s > 0.0 ? 1.0 : 0.0;
        scal[KBN_CG_ITERS] = 0.0;
        scal[KBN_CG_ALPHA] = 0.0;
        scal[KBN_CG_BETA] = 0.0;
        scal[KBN_CG_PQ] = 0.0;
    } else if (stage == 1) {
        const double rr = scal[KBN_CG_RR];
        scal[KBN_CG_PQ] = s;
        scal[KBN_CG_ALPHA] = (s > 0.0 && rr > 0.0) ? rr / s : 0.0;
    } else {
        const double rr = scal[KBN_CG_RR];
        const double bb = scal[KBN_CG_BB];
        scal[KBN_CG_BETA] = rr > 0.0 ? s / rr : 0.0;
        scal[KBN_CG_RR] = s;
        scal[KBN_CG_REL] = bb > 0.0 ? sqrt(s / bb) : 0.0;
        scal[KBN_CG_ITERS] += 1.0;
    }
}

}  // namespace

int kbn_cg_nparts(int64_t n) {
    const int64_t b = (n + TPB - 1) / TPB;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, KBN_CG_MAXPARTS));
}

hipError_t kbn_launch_cg(int kind, int nimg, int64_t n, float2 *x, float2 *r, float2 *p, float2 *q,
                         float lam, KbnCgImage img, double *scal, double *part, hipStream_t s) {
    // one grid row per image; partials [nimg][KBN_CG_MAXPARTS], scalars [nimg][KBN_CG_NSCAL]
    if (nimg < 1 || nimg > 65535) return hipErrorInvalidValue;
    const int g = kbn_cg_nparts(n);
    const dim3 grid(g, nimg), gs(nimg);
    switch (kind) {
    case KBN_CGK_INIT:
        k_cg_init<<<grid, dim3(TPB), 0, s>>>(x, r, p, n, part);
        k_cg_scalars<<<gs, dim3(TPB), 0, s>>>(part, g, scal, 0);
        break;
    case KBN_CGK_Q:
        if (img.reg == KBN_REG_FINITE_DIFF) {
            if ((int64_t)img.n0 * img.n1 * img.n2 != n) return hipErrorInvalidValue;
            k_cg_q_fd<<<grid, dim3(TPB), 0, s>>>(q, p, lam, img.n0, img.n1, img.n2, n, part);
        } else {
            k_cg_q<<<grid, dim3(TPB), 0, s>>>(q, p, lam, n, part);
        }
        k_cg_scalars<<<gs, dim3(TPB), 0, s>>>(part, g, scal, 1);
        break;
    case KBN_CGK_XR:
        k_cg_xr<<<grid, dim3(TPB), 0, s>>>(x, r, p, q, scal, n, part);
        k_cg_scalars<<<gs, dim3(TPB), 0, s>>>(part, g, scal, 2);
        break;
    case KBN_CGK_P:
        k_cg_p<<<grid, dim3(TPB), 0, s>>>(p, r, scal, n);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
