// Elementwise kernels of the off-resonance model (Sec. II-H):
//   E = sum_l diag(b_l) (I_C kron A) diag(c_l) S,  b: [L][M], c: [L][N..].
// The L time segments are run through the NUFFT like coils: the image-
// domain factors c_l s_k form L*C virtual coil maps (virtual coil v = l*C + k),
// the k-space weights b_l are applied before the spread (conjugated: the
// adjoint and the Jacobians) or after the gather (forward, summed over l).
#include <algorithm>
#include <cmath>

#include "kbn_internal.h"

namespace {

constexpr int TPB = 256;

__device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ inline float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

unsigned grid_for(int64_t n) {
    const int64_t g = (n + TPB - 1) / TPB;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

// vm[l*C + k][j] = c[l][j] * s[k][j]  (s = 1 without coil maps)
__global__ __launch_bounds__(TPB) void k_field_maps(int L, int C, int64_t npix,
                                                    const float2 *__restrict__ c,
                                                    const float2 *__restrict__ s,
                                                    float2 *__restrict__ vm) {
    const int64_t n = (int64_t)L * C * npix;
    for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
        const int64_t j = i % npix;
        const int64_t t = i / npix;
        const int k = (int)(t % C);
        const int l = (int)(t / C);
        const float2 cv = c[(int64_t)l * npix + j];
        vm[i] = s ? cmul(cv, s[(int64_t)k * npix + j]) : cv;
    }
}

// ye[b][l*C + k][m] = conj(bw[l][m]) * y[b][k][m]
__global__ __launch_bounds__(TPB) void k_field_expand(int64_t nb, int L, int C, int64_t M,
                                                      const float2 *__restrict__ bw,
                                                      const float2 *__restrict__ y,
                                                      float2 *__restrict__ ye) {
    const int64_t n = nb * L * C * M;
    for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
        const int64_t m = i % M;
        int64_t t = i / M;
        const int k = (int)(t % C);
        t /= C;
        const int l = (int)(t % L);
        const int64_t b = t / L;
        ye[i] = cmulc(bw[(int64_t)l * M + m], y[(b * C + k) * M + m]);
    }
}

// y[b][k][m] = sum_l bw[l][m] * ye[b][l*C + k][m]   (l in order)
__global__ __launch_bounds__(TPB) void k_field_combine(int64_t nb, int L, int C, int64_t M,
                                                       const float2 *__restrict__ bw,
                                                       const float2 *__restrict__ ye,
                                                       float2 *__restrict__ y) {
    const int64_t n = nb * C * M;
    for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
        const int64_t m = i % M;
        const int64_t t = i / M;
        const int k = (int)(t % C);
        const int64_t b = t / C;
        float2 acc = make_float2(0.f, 0.f);
        for (int l = 0; l < L; ++l) {
            const float2 v = cmul(bw[(int64_t)l * M + m], ye[((b * L + l) * C + k) * M + m]);
            acc.x += v.x;
            acc.y += v.y;
        }
        y[i] = acc;
    }
}

// segment time l: t0 + (t1 - t0) l / (L - 1), or the midpoint when L = 1
__device__ inline double seg_time(int l, int L, double t0, double t1) {
    return L == 1 ? 0.5 * (t0 + t1) : t0 + (t1 - t0) * (double)l / (double)(L - 1);
}

// linear interpolation weights of t_i between its neighbouring segment times
__global__ __launch_bounds__(TPB) void k_field_seg_b(int64_t M, const float *__restrict__ t, double t0,
                                                     double t1, int L, float2 *__restrict__ bw) {
    for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < M; i += (int64_t)gridDim.x * TPB) {
        for (int l = 0; l < L; ++l) bw[(int64_t)l * M + i] = make_float2(0.f, 0.f);
        if (L == 1 || !(t1 > t0)) {
            bw[i] = make_float2(1.f, 0.f);
            continue;
        }
        double pos = ((double)t[i] - t0) / (t1 - t0) * (double)(L - 1);
        pos = fmin(fmax(pos, 0.0), (double)(L - 1));
        int lo = (int)floor(pos);
        if (lo > L - 2) lo = L - 2;
        const double f = pos - (double)lo;
        bw[(int64_t)lo * M + i] = make_float2((float)(1.0 - f), 0.f);
        bw[(int64_t)(lo + 1) * M + i] = make_float2((float)f, 0.f);
    }
}

// c[l][j] = exp(-i w_j tau_l)
__global__ __launch_bounds__(TPB) void k_field_seg_c(int64_t npix, const float *__restrict__ w, double t0,
                                                     double t1, int L, float2 *__restrict__ c) {
    const int64_t n = (int64_t)L * npix;
    for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
        const int l = (int)(i / npix);
        const int64_t j = i - (int64_t)l * npix;
        const double ph = (double)w[j] * seg_time(l, L, t0, t1);
        double s, co;
        sincos(ph, &s, &co);
        c[i] = make_float2((float)co, (float)-s);
    }
}

}  // namespace

hipError_t kbn_launch_field_maps(int L, int C, int64_t npix, const float2 *c, const float2 *smaps,
                                 float2 *vm, hipStream_t s) {
    const int64_t n = (int64_t)L * C * npix;
    if (n == 0) return hipSuccess;
    k_field_maps<<<dim3(grid_for(n)), dim3(TPB), 0, s>>>(L, C, npix, c, smaps, vm);
    return hipGetLastError();
}

hipError_t kbn_launch_field_expand(int64_t nb, int L, int C, int64_t M, const float2 *bw,
                                   const float2 *y, float2 *ye, hipStream_t s) {
    const int64_t n = nb * L * C * M;
    if (n == 0) return hipSuccess;
    k_field_expand<<<dim3(grid_for(n)), dim3(TPB), 0, s>>>(nb, L, C, M, bw, y, ye);
    return hipGetLastError();
}

hipError_t kbn_launch_field_combine(int64_t nb, int L, int C, int64_t M, const float2 *bw,
                                    const float2 *ye, float2 *y, hipStream_t s) {
    const int64_t n = nb * C * M;
    if (n == 0) return hipSuccess;
    k_field_combine<<<dim3(grid_for(n)), dim3(TPB), 0, s>>>(nb, L, C, M, bw, ye, y);
    return hipGetLastError();
}

hipError_t kbn_launch_field_segments(int64_t M, const float *t, double t0, double t1, int64_t npix,
                                     const float *w, int L, float2 *bw, float2 *c, hipStream_t s) {
    if (M > 0) k_field_seg_b<<<dim3(grid_for(M)), dim3(TPB), 0, s>>>(M, t, t0, t1, L, bw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (npix > 0)
        k_field_seg_c<<<dim3(grid_for((int64_t)L * npix)), dim3(TPB), 0, s>>>(npix, w, t0, t1, L, c);
    return hipGetLastError();
}
