// Host side of the KB-NUFFT library: plan constants (FP64), buffer
// management, pipeline dispatch and the C ABI declared in kbnufft.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "kbn_internal.h"
#include "kbnufft.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define KBN_HIP(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(KBN_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

bool debug_sync() {
    static const int v = [] {
        const char *e = std::getenv("KBN_DEBUG_SYNC");
        return e ? std::atoi(e) : 0;
    }();
    return v != 0;
}

int launched(hipError_t e, const char *what, hipStream_t s) {
    if (e != hipSuccess) return fail(KBN_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    if (debug_sync()) {
        hipError_t e2 = hipStreamSynchronize(s);
        if (e2 != hipSuccess)
            return fail(KBN_ERR_HIP, std::string(what) + " (sync): " + hipGetErrorString(e2));
    }
    return KBN_OK;
}

const char *const kClassNames[KBN_NCLASS] = {"index",       "fft_first",    "fft_mid_fwd",
                                               "fft_mid_inv", "fft_last_adj", "gather",
                                               "gather_jac",  "spread"};

// Launch `expr` (a kernel launcher returning hipError_t) of kernel class
// `cls`; with timing enabled the launch is bracketed by events on `stream`.
#define KBN_LAUNCH(cls, expr, name)                                     \
    do {                                                                \
        hipEvent_t e0_ = nullptr;                                       \
        if (p->timing && ((p->timing_mask >> (cls)) & 1u))              \
            e0_ = timing_mark(p, stream);                               \
        int rc_ = launched((expr), name, stream);                       \
        if (p->timing && e0_) {                                         \
            hipEvent_t e1_ = timing_mark(p, stream);                    \
            if (e1_) p->pending.push_back({(cls), e0_, e1_});           \
        }                                                               \
        if (rc_ != KBN_OK) return rc_;                                  \
    } while (0)

// ---- window mathematics (FP64) -------------------------------------------

// Modified Bessel function I0 by its power series sum_k (x^2/4)^k / (k!)^2
// (all terms positive, so the partial sums are accurate to rounding).
double bessel_i0(double x) {
    const double q = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

struct Window {
    int J;
    double beta;
    double i0beta;
    double psi(double t) const {  // normalised KB window, zero outside |t| <= J/2
        const double a = 1.0 - (2.0 * t / J) * (2.0 * t / J);
        if (a < 0.0) return 0.0;
        return bessel_i0(beta * std::sqrt(a)) / i0beta;
    }
    double psi_hat(double f) const {  // continuous Fourier transform of psi
        const double z2 = beta * beta - (M_PI * J * f) * (M_PI * J * f);
        double r;
        if (z2 > 0) {
            const double z = std::sqrt(z2);
            r = std::sinh(z) / z;
        } else if (z2 < 0) {
            const double z = std::sqrt(-z2);
            r = std::sin(z) / z;
        } else {
            r = 1.0;
        }
        return J * r / i0beta;
    }
};

// Degree-(KBN_NCOEF-1) polynomial in x = 2f - 1, f in [0, 1], for each tap
// piece psi(f + J/2 - 1 - j): Chebyshev interpolation, then monomial form.
std::vector<float> window_polys(const Window &w) {
    const int P = KBN_NCOEF - 1;
    const int n = P + 1;
    std::vector<float> out((size_t)w.J * KBN_NCOEF);
    for (int j = 0; j < w.J; ++j) {
        std::vector<double> fx(n), cheb(n, 0.0);
        for (int k = 0; k < n; ++k) {
            const double xk = std::cos(M_PI * (k + 0.5) / n);
            const double f = 0.5 * (xk + 1.0);
            fx[k] = w.psi(f + 0.5 * w.J - 1.0 - j);
        }
        for (int m = 0; m < n; ++m) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += fx[k] * std::cos(M_PI * m * (k + 0.5) / n);
            cheb[m] = (m == 0 ? 1.0 : 2.0) * s / n;
        }
        // T_m in monomial form by the three-term recurrence
        std::vector<double> mono(n, 0.0), tprev(n, 0.0), tcur(n, 0.0), tnext(n, 0.0);
        tprev[0] = 1.0;               // T0
        tcur[1] = 1.0;                // T1
        mono[0] += cheb[0];
        if (n > 1) mono[1] += cheb[1];
        for (int m = 2; m < n; ++m) {
            std::fill(tnext.begin(), tnext.end(), 0.0);
            for (int i = 0; i + 1 < n; ++i) tnext[i + 1] += 2.0 * tcur[i];
            for (int i = 0; i < n; ++i) tnext[i] -= tprev[i];
            for (int i = 0; i < n; ++i) mono[i] += cheb[m] * tnext[i];
            tprev.swap(tcur);
            tcur.swap(tnext);
        }
        for (int i = 0; i < n; ++i) out[(size_t)j * KBN_NCOEF + i] = (float)mono[i];
    }
    return out;
}

int smooth_size(double target) {  // smallest 7-smooth integer >= target
    int k = (int)std::ceil(target - 1e-9);
    if (k < 1) k = 1;
    for (;; ++k) {
        int r = k;
        for (int p : {2, 3, 5, 7})
            while (r % p == 0) r /= p;
        if (r == 1) return k;
    }
}

bool factor(int L, KbnRadix &rp) {
    rp.L = L;
    rp.nst = 0;
    int r = L;
    for (int f : {8, 4, 2, 3, 5, 7}) {
        while (r % f == 0) {
            if (rp.nst >= KBN_MAX_STAGES) return false;
            rp.r[rp.nst++] = f;
            r /= f;
        }
    }
    return r == 1;
}

}  // namespace

struct kbn_plan_s {
    // device memory comes from the caller's allocator (stream-ordered), or
    // from the HIP stream-ordered allocator when none was given
    kbn_allocator alloc{};
    bool custom_alloc = false;
    struct Block {
        void *ptr;
        int64_t bytes;
    };
    std::vector<Block> blocks;  // live device blocks and their sizes
    int64_t dev_bytes = 0;      // sum of the live blocks
    // host copies of the uploaded constants: they stay alive until the
    // asynchronous uploads have read them (upload_done)
    std::vector<float> h_deap[KBN_MAX_D];
    std::vector<float2> h_tw[KBN_MAX_D];
    std::vector<float> h_coef;
    hipEvent_t upload_done = nullptr;
    // The index pass runs on a stream of the plan's own, beside the caller's
    // stream, so that a forward call's FFT passes (which do not read the
    // points) overlap it; every read of the point buffers first makes its
    // stream wait for points_ready.
    hipStream_t istream = nullptr;
    hipEvent_t points_in = nullptr, points_ready = nullptr, omega_read = nullptr;
    bool points_pending = false;
    uint64_t points_gen = 0;               // index passes issued
    hipStream_t waited_stream = nullptr;   // the last stream ordered after pass waited_gen
    uint64_t waited_gen = 0;
    int D = 0;
    int N[KBN_MAX_D] = {1, 1, 1};
    int K[KBN_MAX_D] = {1, 1, 1};
    int J = 6;
    double sigma = 2.0, beta = 0.0;
    int T[KBN_MAX_D] = {1, 1, 1};
    int nt[KBN_MAX_D] = {1, 1, 1};
    int ntiles = 1;
    int To[KBN_MAX_D] = {1, 1, 1};   // spread owner tiles
    int nto[KBN_MAX_D] = {1, 1, 1};
    int ntiles_own = 1;
    double scale[KBN_MAX_D] = {0, 0, 0};
    KbnRadix rad[KBN_MAX_D];
    float *deap[KBN_MAX_D] = {nullptr, nullptr, nullptr};
    float2 *tw[KBN_MAX_D] = {nullptr, nullptr, nullptr};
    float *coef = nullptr;
    int *flag = nullptr;
    int maxe = 16;
    bool fast_fft = true;  // use the specialised FFT passes where available
    // points
    int64_t M = -1, Mcap = 0;
    int *cell_tmp = nullptr, *tile = nullptr, *order = nullptr, *cell = nullptr, *toff = nullptr;
    float *frac_tmp = nullptr, *frac = nullptr;
    int *counts = nullptr;
    int64_t counts_cap = 0;
    int *subs = nullptr, *nsub = nullptr;
    int *ooff = nullptr, *otile_order = nullptr;
    int *swork = nullptr, *scomb = nullptr, *scounts = nullptr;
    int *rec_p = nullptr, *rec_q = nullptr, *rec_l = nullptr;
    float *rec_f = nullptr;
    int64_t swork_cap = 0;
    // grid workspace
    float2 *ws = nullptr;
    int64_t ws_bytes = 0, max_ws = 0;
    // off-resonance workspace: virtual coil maps and expanded k-space
    char *fws = nullptr;
    int64_t fws_bytes = 0;
    // captured batch graphs that hold this plan's buffer addresses; while
    // non-zero the plan refuses anything that would move or resize them
    int graph_refs = 0;
    // bumped by every kbn_set_points: descriptors of phased batch calls that
    // hold this plan's point buffers and M are rebuilt when it changes
    uint64_t epoch = 0;
    // partial-tile slots for owner tiles split into several spread work items
    int smax = KBN_SPREAD_SMAX;
    int sub = KBN_SUB;  // samples per gather subproblem
    // per-kernel-class event timing (kbn_timing)
    struct Timed {
        int cls;
        hipEvent_t e0, e1;
    };
    bool timing = false;
    unsigned int timing_mask = ~0u;  // kernel classes that record events
    std::vector<Timed> pending;
    std::vector<hipEvent_t> pool;
    double t_ms[KBN_NCLASS] = {};
    int64_t t_n[KBN_NCLASS] = {};

    int64_t gsize() const {
        int64_t g = 1;
        for (int d = 0; d < D; ++d) g *= K[d];
        return g;
    }
    KbnGeom geom() const {
        KbnGeom g;
        g.D = D;
        g.J = J;
        for (int d = 0; d < KBN_MAX_D; ++d) {
            g.K[d] = K[d];
            g.T[d] = T[d];
            g.nt[d] = nt[d];
        }
        g.ntiles = ntiles;
        for (int d = 0; d < KBN_MAX_D; ++d) {
            g.To[d] = To[d];
            g.nto[d] = nto[d];
        }
        g.ntiles_own = ntiles_own;
        g.coef = coef;
        return g;
    }
};

namespace {

hipEvent_t timing_mark(kbn_plan p, hipStream_t stream) {
    hipEvent_t e = nullptr;
    if (!p->pool.empty()) {
        e = p->pool.back();
        p->pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        return nullptr;
    }
    if (hipEventRecord(e, stream) != hipSuccess) {
        p->pool.push_back(e);
        return nullptr;
    }
    return e;
}

// Device blocks are rounded up to 256 bytes; every live block is recorded
// with its size so that kbn_plan_info can report the plan's footprint.
int64_t block_bytes(int64_t bytes) { return (std::max<int64_t>(bytes, 1) + 255) / 256 * 256; }

template <typename T>
int dev_alloc(kbn_plan pl, T **p, int64_t count, hipStream_t s) {
    *p = nullptr;
    const int64_t bytes = block_bytes((int64_t)sizeof(T) * std::max<int64_t>(count, 1));
    void *q = nullptr;
    if (pl->custom_alloc) {
        q = pl->alloc.alloc(pl->alloc.ctx, (size_t)bytes, (void *)s);
        if (!q) return fail(KBN_ERR_OOM, "allocator returned NULL for " + std::to_string(bytes) + " bytes");
    } else {
        const hipError_t e = hipMallocAsync(&q, (size_t)bytes, s);
        if (e != hipSuccess || !q) {
            (void)hipGetLastError();
            return fail(KBN_ERR_OOM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
        }
    }
    pl->blocks.push_back({q, bytes});
    pl->dev_bytes += bytes;
    *p = (T *)q;
    return KBN_OK;
}

// Stream-ordered release: work already queued on `s` may still use the block.
template <typename T>
void dev_free(kbn_plan pl, T *&p, hipStream_t s) {
    if (!p) return;
    for (size_t i = 0; i < pl->blocks.size(); ++i) {
        if (pl->blocks[i].ptr == (void *)p) {
            pl->dev_bytes -= pl->blocks[i].bytes;
            pl->blocks[i] = pl->blocks.back();
            pl->blocks.pop_back();
            break;
        }
    }
    if (pl->custom_alloc)
        pl->alloc.free(pl->alloc.ctx, (void *)p, (void *)s);
    else
        (void)hipFreeAsync((void *)p, s);
    p = nullptr;
}

void free_points(kbn_plan p, hipStream_t s) {
    dev_free(p, p->cell_tmp, s);
    dev_free(p, p->tile, s);
    dev_free(p, p->order, s);
    dev_free(p, p->cell, s);
    dev_free(p, p->frac_tmp, s);
    dev_free(p, p->frac, s);
    dev_free(p, p->counts, s);
    dev_free(p, p->subs, s);
    dev_free(p, p->swork, s);
    dev_free(p, p->rec_p, s);
    dev_free(p, p->rec_q, s);
    dev_free(p, p->rec_l, s);
    dev_free(p, p->rec_f, s);
    p->swork_cap = 0;
    p->Mcap = 0;
    p->counts_cap = 0;
}

int points_wait(kbn_plan p, hipStream_t stream);

void free_plan(kbn_plan p, hipStream_t s) {
    (void)points_wait(p, s);  // the frees below come after the last index pass
    for (auto &t : p->pending) {
        (void)hipEventDestroy(t.e0);
        (void)hipEventDestroy(t.e1);
    }
    for (auto e : p->pool) (void)hipEventDestroy(e);
    free_points(p, s);
    for (int d = 0; d < KBN_MAX_D; ++d) {
        dev_free(p, p->deap[d], s);
        dev_free(p, p->tw[d], s);
    }
    dev_free(p, p->coef, s);
    dev_free(p, p->flag, s);
    dev_free(p, p->toff, s);
    dev_free(p, p->nsub, s);
    dev_free(p, p->ooff, s);
    dev_free(p, p->otile_order, s);
    dev_free(p, p->scomb, s);
    dev_free(p, p->scounts, s);
    dev_free(p, p->ws, s);
    dev_free(p, p->fws, s);
    // the host constants may be freed only once their uploads have run
    if (p->points_in) (void)hipEventDestroy(p->points_in);
    if (p->omega_read) (void)hipEventDestroy(p->omega_read);
    if (p->points_ready) (void)hipEventDestroy(p->points_ready);
    if (p->istream) (void)hipStreamDestroy(p->istream);
    if (p->upload_done) {
        if (hipEventQuery(p->upload_done) != hipSuccess) (void)hipEventSynchronize(p->upload_done);
        (void)hipEventDestroy(p->upload_done);
    }
    delete p;
}

// Orders `stream` after the plan's last index pass.  Under graph capture
// the wait would be on an event recorded outside the capture, so a capture
// requires the index pass to be known finished (kbn_check_error, or the
// batch capture's own eager pass); captured plans refuse new points.
int points_wait(kbn_plan p, hipStream_t stream) {
    if (!p->points_pending) return KBN_OK;
    // a stream already ordered after this pass needs no second wait (the
    // launch-bound small problems issue dozens of calls per pass)
    if (p->waited_gen == p->points_gen && p->waited_stream == stream) return KBN_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return fail(KBN_ERR_HIP, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone)  // (no event query either: not allowed in every capture mode)
        return fail(KBN_ERR_UNSUPPORTED,
                    "capture while the index pass of kbn_set_points may still run: call kbn_check_error first");
    if (hipStreamWaitEvent(stream, p->points_ready, 0) != hipSuccess)
        return fail(KBN_ERR_HIP, "hipStreamWaitEvent (points)");
    p->waited_stream = stream;
    p->waited_gen = p->points_gen;
    return KBN_OK;
}

int ensure_ws(kbn_plan p, int64_t bytes, hipStream_t stream) {
    if (bytes <= p->ws_bytes) return KBN_OK;
    if (p->graph_refs > 0)
        return fail(KBN_ERR_UNSUPPORTED, "workspace growth on a plan held by a captured batch");
    dev_free(p, p->ws, stream);  // stream-ordered: queued work may still read it
    p->ws_bytes = 0;
    int rc = dev_alloc(p, (char **)&p->ws, bytes, stream);
    if (rc != KBN_OK) return rc;
    p->ws_bytes = bytes;
    return KBN_OK;
}

// img: an image-space buffer (never empty); ksp: a k-space buffer, which
// holds no element (and may be NULL) when M == 0.
int check_common(kbn_plan p, int B, int C, const void *img, const void *smaps, const void *ksp) {
    if (!p) return fail(KBN_ERR_INVALID_ARG, "null plan");
    if (p->M < 0) return fail(KBN_ERR_NO_POINTS, "kbn_set_points has not been called");
    if (B < 1 || C < 1) return fail(KBN_ERR_INVALID_ARG, "B and C must be >= 1");
    if (!smaps && C != 1) return fail(KBN_ERR_INVALID_ARG, "C > 1 needs coil maps");
    if (!img || (!ksp && p->M > 0)) return fail(KBN_ERR_INVALID_ARG, "null data pointer");
    return KBN_OK;
}

int64_t img_rows(kbn_plan p) {  // product of the leading image axes
    int64_t r = 1;
    for (int d = 0; d + 1 < p->D; ++d) r *= p->N[d];
    return r;
}

// Work split under the workspace cap: whole images (all coils) per chunk
// while one image fits, else one image at a time in runs of coils.
struct Chunks {
    int64_t bc;  // images per chunk
    int cc;      // coils per chunk (C unless one image does not fit)
};

static Chunks split_chunks(int64_t B, int C, int64_t per_coil, int64_t max_ws) {
    if ((int64_t)C * per_coil <= max_ws)
        return {std::max<int64_t>(1, std::min<int64_t>(B, max_ws / ((int64_t)C * per_coil))), C};
    return {1, (int)std::max<int64_t>(1, std::min<int64_t>(C, max_ws / per_coil))};
}

// Bytes of the omega-gradient partials of an omega-Jacobian gather over at
// most `units` image-coil pairs (nw = D weighted channels each).
int64_t jac_part_bytes(const kbn_plan p, int64_t M, int64_t units) {
    const int nw = p->D;
    const int64_t blocks0 = kbn_gather_shape(p->geom(), M, (int)(units * nw), nw).blocks;
    const int64_t groups_max = kbn_gather_groups(blocks0, units);
    return groups_max * M * p->D * (int64_t)sizeof(float);
}

// Grid workspace of one call (bytes), the larger chunk's share under the
// workspace cap.  Type 2 (forward, nw weight channels per coil; mode 1 adds
// the per-group partial omega-gradients: the gather's point blocks do not
// depend on the channel count, and a chunk's channel groups are at most
// kbn_gather_groups of its image-coil pairs, a bound that also holds for
// every smaller chunk).
int64_t ws_type2(const kbn_plan p, int64_t M, int B, int C, int nw, int mode) {
    const int64_t per_coil = (int64_t)nw * p->gsize() * (int64_t)sizeof(float2) * 2;
    const Chunks ck = split_chunks(B, C, per_coil, p->max_ws);
    const int64_t units = ck.bc * ck.cc;
    return units * per_coil + (mode == 1 ? jac_part_bytes(p, M, units) : 0);
}

// Forward plus omega-Jacobian in one pass (run_fwd_jac): D + 1 grids per
// image-coil pair, plus the Jacobian gather's partials.
int64_t fwd_jac_per_coil(const kbn_plan p) { return (int64_t)(p->D + 1) * p->gsize() * (int64_t)sizeof(float2) * 2; }

int64_t ws_fwd_jac(const kbn_plan p, int64_t M, int B, int C) {
    const Chunks ck = split_chunks(B, C, fwd_jac_per_coil(p), p->max_ws);
    const int64_t units = ck.bc * ck.cc;
    return units * fwd_jac_per_coil(p) + jac_part_bytes(p, M, units);
}

// Type 1 (adjoint): per image-coil pair two grids, the k-space in tile order
// and the partial tiles of split owner tiles.
int64_t type1_per_coil(const kbn_plan p, int64_t M) {
    int64_t tcells = 1;
    for (int d = 0; d < p->D; ++d) tcells *= p->To[d];
    return (p->gsize() * 2 + M + (int64_t)p->smax * tcells) * (int64_t)sizeof(float2);
}

int64_t ws_type1(const kbn_plan p, int64_t M, int B, int C) {
    const int64_t per_coil = type1_per_coil(p, M);
    const Chunks ck = split_chunks(B, C, per_coil, p->max_ws);
    return ck.bc * ck.cc * per_coil;
}

// Element counts of the index-pass buffers for M samples: per-sample arrays
// (capacity), the integer scratch, gather subproblems, owner-list entries
// (a sample reaches at most 2^D owner tiles) and spread work items.
struct PointSizes {
    int64_t cap, counts, subs, ent, swork;
};

PointSizes point_sizes(const kbn_plan p, int64_t M) {
    PointSizes z;
    z.cap = std::max<int64_t>(M, 1);
    z.counts = kbn_points_counts_size(M, p->ntiles, p->ntiles_own);
    z.subs = 2 * ((z.cap + KBN_SUB - 1) / KBN_SUB + p->ntiles + 1);
    z.ent = z.cap << p->D;
    z.swork = p->ntiles_own + (z.ent + KBN_SPREAD_SEG - 1) / KBN_SPREAD_SEG + 1;
    return z;
}

int64_t points_bytes(const kbn_plan p, int64_t M) {
    const PointSizes z = point_sizes(p, M);
    const int D = p->D;
    return 4 * block_bytes(4 * z.cap * D) + 2 * block_bytes(4 * z.cap) + block_bytes(4 * z.counts) +
           block_bytes(4 * z.subs) + block_bytes(16 * z.swork) + 2 * block_bytes(4 * z.ent) +
           2 * block_bytes(4 * z.ent * D);
}

// FFT passes of one forward-type chunk (nb images from b0, ncc coils from
// c0, nw weight channels per coil): scaling (+ coil map, + coordinate
// weight) and the last-axis pass into bufA, then the strided passes
// alternating between the buffers; *grid is the buffer that holds the
// oversampled spectra at the end.
int t2_passes(kbn_plan p, int nw, int weighted, const float2 *x, const float2 *smaps, int64_t b0, int c0,
              int64_t nb, int ncc, float2 *bufA, float2 *bufB, float2 **grid, hipStream_t stream) {
    const int D = p->D;
    const int64_t R0 = img_rows(p);
    const int Nl = p->N[D - 1];
    const int64_t nch = nb * ncc * nw;
    KbnFirstPassArgs fa;
    fa.x = x + b0 * R0 * Nl;
    fa.smaps = smaps ? smaps + (int64_t)c0 * R0 * Nl : nullptr;
    fa.out = bufA;
    fa.nlines = nch * R0;
    fa.R0 = (int)R0;
    fa.Nl = Nl;
    fa.C = ncc;
    fa.nw = nw;
    fa.weighted = weighted;
    fa.D = D;
    for (int d = 0; d < KBN_MAX_D; ++d) {
        fa.N[d] = p->N[d];
        fa.deap[d] = p->deap[d];
    }
    if (p->fast_fft && kbn_fast_fft_size(p->K[D - 1]))
        KBN_LAUNCH(KBN_CLASS_FFT_FIRST, kbn_launch_fast_first(fa, p->K[D - 1], p->tw[D - 1], stream),
                   "first pass");
    else
        KBN_LAUNCH(KBN_CLASS_FFT_FIRST,
                   kbn_launch_first_pass(fa, p->rad[D - 1], p->tw[D - 1], p->maxe, stream),
                   "first pass");
    float2 *cur = bufA, *nxt = bufB;
    for (int d = D - 2; d >= 0; --d) {
        int64_t outer = nch, inner = 1;
        for (int e = 0; e < d; ++e) outer *= p->N[e];
        for (int e = d + 1; e < D; ++e) inner *= p->K[e];
        KbnMidPassArgs ma;
        ma.in = cur;
        ma.out = nxt;
        ma.outer = outer;
        ma.nin = p->N[d];
        ma.nout = p->K[d];
        ma.inner = (int)inner;
        ma.pad_in = 1;
        ma.crop_out = 0;
        if (p->fast_fft && kbn_fast_fft_size(p->K[d]))
            KBN_LAUNCH(KBN_CLASS_FFT_MID_FWD, kbn_launch_fast_mid(ma, p->K[d], p->tw[d], 0, stream),
                       "mid pass");
        else
            KBN_LAUNCH(KBN_CLASS_FFT_MID_FWD,
                       kbn_launch_mid_pass(ma, p->rad[d], p->tw[d], 0, p->maxe, stream), "mid pass");
        std::swap(cur, nxt);
    }
    *grid = cur;
    return KBN_OK;
}

// Gather arguments of one forward-type chunk of nch channels (k-space
// offset k0 of its first image-coil pair).
KbnGatherArgs t2_gather_args(kbn_plan p, int64_t nch, int ncc, int nw, int mode, const float2 *grid, int64_t k0,
                             float2 *y, const float2 *v, float *dom, float *part, int accumulate) {
    KbnGatherArgs ga;
    ga.grid = grid;
    ga.gsize = p->gsize();
    ga.nch = (int)nch;
    ga.C = ncc;
    ga.nw = nw;
    ga.M = p->M;
    ga.order = p->order;
    ga.cell = p->cell;
    ga.frac = p->frac;
    ga.toff = p->toff;
    ga.subs = p->subs;
    ga.nsub = p->nsub;
    ga.y = mode == 0 ? y + k0 : nullptr;
    ga.v = mode == 1 ? v + k0 : nullptr;
    ga.domega = dom;
    ga.part = part;
    ga.accumulate = accumulate;
    return ga;
}

// Forward-type pipeline: FFT passes, then gather.  mode 0 writes y; mode 1
// folds the omega-Jacobian.  ext_ws (mode 0 only): a workspace of ext_bytes
// given by the caller instead of the plan's, which is then neither grown
// nor used; the batch is chunked to fit it.
int run_type2(kbn_plan p, int B, int C, int nw, int weighted, const float2 *x,
              const float2 *smaps, int mode, float2 *y, const float2 *v, float *dom,
              int accumulate, hipStream_t stream, void *ext_ws = nullptr, int64_t ext_bytes = 0) {
    const int64_t gsz = p->gsize();
    const int64_t per_coil = (int64_t)nw * gsz * (int64_t)sizeof(float2) * 2;
    const Chunks ck = split_chunks(B, C, per_coil, ext_ws ? ext_bytes : p->max_ws);
    const int64_t units = ck.bc * ck.cc;  // image-coil pairs of the largest chunk
    float2 *ws = (float2 *)ext_ws;
    if (!ws) {
        int rc = ensure_ws(p, ws_type2(p, p->M, B, C, nw, mode), stream);
        if (rc != KBN_OK) return rc;
        ws = p->ws;
    }
    float2 *bufA = ws;
    float2 *bufB = ws + units * nw * gsz;
    float *part = (float *)(ws + 2 * units * nw * gsz);
    const KbnGeom geom = p->geom();
    for (int64_t b0 = 0; b0 < B; b0 += ck.bc)
    for (int c0 = 0; c0 < C; c0 += ck.cc) {
        const int64_t nb = std::min<int64_t>(ck.bc, B - b0);
        const int ncc = std::min(ck.cc, C - c0);
        const int64_t nch = nb * ncc * nw;
        float2 *grid = nullptr;
        int rc = t2_passes(p, nw, weighted, x, smaps, b0, c0, nb, ncc, bufA, bufB, &grid, stream);
        if (rc == KBN_OK) rc = points_wait(p, stream);  // the FFT passes overlap the index pass
        if (rc != KBN_OK) return rc;
        const KbnGatherArgs ga = t2_gather_args(p, nch, ncc, nw, mode, grid, (b0 * C + c0) * p->M, y, v, dom, part,
                                                (accumulate || b0 > 0 || c0 > 0) ? 1 : 0);
        KBN_LAUNCH(mode == 0 ? KBN_CLASS_GATHER : KBN_CLASS_GATHER_JAC, kbn_launch_gather(geom, ga, mode, stream), "gather");
    }
    return KBN_OK;
}

// Spread arguments of one adjoint chunk of nch image-coil pairs (k-space
// from y_chunk) into the grids at bufA, with its k-space copy bufY and
// partial tiles bufP.
KbnSpreadArgs t1_spread_args(kbn_plan p, int64_t nch, const float2 *y_chunk, float2 *bufA, float2 *bufY,
                             float2 *bufP) {
    KbnSpreadArgs sa;
    sa.y = y_chunk;
    sa.ys = bufY;
    sa.grid = bufA;
    sa.gsize = p->gsize();
    sa.nch = (int)nch;
    sa.M = p->M;
    sa.order = p->order;
    sa.cell = p->cell;
    sa.frac = p->frac;
    sa.toff = p->toff;
    sa.otile_order = p->otile_order;
    sa.swork = p->swork;
    sa.scomb = p->scomb;
    sa.scounts = p->scounts;
    sa.partial = bufP;
    sa.rec_p = p->rec_p;
    sa.rec_q = p->rec_q;
    sa.rec_l = p->rec_l;
    sa.rec_f = p->rec_f;
    sa.nwork_max = (int)p->swork_cap;
    sa.ncomb_max = std::min<int>(p->ntiles_own, p->smax / 2);
    return sa;
}

// Inverse FFT passes of one adjoint chunk whose spread grids are in bufA:
// strided passes with cropping, then the last-axis pass with cropping,
// scaling and conj(coil map), summed over the chunk's coils into x.
int t1_passes(kbn_plan p, int64_t b0, int c0, int64_t nb, int ncc, const float2 *smaps, float2 *x, float2 *bufA,
              float2 *bufB, hipStream_t stream) {
    const int D = p->D;
    const int64_t R0 = img_rows(p);
    const int Nl = p->N[D - 1];
    const int64_t nch = nb * ncc;
    float2 *cur = bufA, *nxt = bufB;
    for (int d = 0; d + 1 < D; ++d) {
        int64_t outer = nch, inner = 1;
        for (int e = 0; e < d; ++e) outer *= p->N[e];
        for (int e = d + 1; e < D; ++e) inner *= p->K[e];
        KbnMidPassArgs ma;
        ma.in = cur;
        ma.out = nxt;
        ma.outer = outer;
        ma.nin = p->K[d];
        ma.nout = p->N[d];
        ma.inner = (int)inner;
        ma.pad_in = 0;
        ma.crop_out = 1;
        if (p->fast_fft && kbn_fast_fft_size(p->K[d]))
            KBN_LAUNCH(KBN_CLASS_FFT_MID_INV, kbn_launch_fast_mid(ma, p->K[d], p->tw[d], 1, stream),
                       "mid pass");
        else
            KBN_LAUNCH(KBN_CLASS_FFT_MID_INV,
                       kbn_launch_mid_pass(ma, p->rad[d], p->tw[d], 1, p->maxe, stream), "mid pass");
        std::swap(cur, nxt);
    }
    // With few image rows per coil, the coil loop inside each line would
    // leave the GPU idle: then every (image, coil) line is transformed on
    // its own into the free buffer and the coils are summed afterwards.
    // The choice depends only on the image shape and coil count, so the
    // same problem gives the same bits whatever the batch size.
    const bool split = ncc > 1 && R0 < 2048;
    KbnLastAdjArgs la;
    la.in = cur;
    la.smaps = smaps ? smaps + (int64_t)c0 * R0 * Nl : nullptr;
    la.x = split ? nxt : x + b0 * R0 * Nl;
    la.nlines = split ? nb * ncc * R0 : nb * R0;
    la.R0 = (int)R0;
    la.Nl = Nl;
    la.C = split ? 1 : ncc;
    la.cmod = split ? ncc : 0;
    la.accumulate = (!split && c0 > 0) ? 1 : 0;  // later coil runs add to the image
    la.D = D;
    for (int d = 0; d < KBN_MAX_D; ++d) {
        la.N[d] = p->N[d];
        la.deap[d] = p->deap[d];
    }
    if (p->fast_fft && kbn_fast_last_size(p->K[D - 1]))
        KBN_LAUNCH(KBN_CLASS_FFT_LAST_ADJ, kbn_launch_fast_last(la, p->K[D - 1], p->tw[D - 1], stream),
                   "last adjoint pass");
    else
        KBN_LAUNCH(KBN_CLASS_FFT_LAST_ADJ,
                   kbn_launch_last_adj(la, p->rad[D - 1], p->tw[D - 1], p->maxe, stream),
                   "last adjoint pass");
    if (split)
        KBN_LAUNCH(KBN_CLASS_FFT_LAST_ADJ,
                   kbn_launch_coil_sum(nxt, nb, ncc, R0 * Nl, x + b0 * R0 * Nl, c0 > 0 ? 1 : 0, stream),
                   "coil sum");
    return KBN_OK;
}

// Adjoint pipeline: spread, inverse FFT passes with cropping, scaling and
// conj(coil map) summed over coils.
int run_type1(kbn_plan p, int B, int C, const float2 *y, const float2 *smaps, float2 *x,
              hipStream_t stream) {
    const int64_t gsz = p->gsize();
    const int64_t per_coil = type1_per_coil(p, p->M);
    const Chunks ck = split_chunks(B, C, per_coil, p->max_ws);
    const int64_t units = ck.bc * ck.cc;
    int rc = ensure_ws(p, ws_type1(p, p->M, B, C), stream);
    if (rc == KBN_OK) rc = points_wait(p, stream);
    if (rc != KBN_OK) return rc;
    float2 *bufA = p->ws;
    float2 *bufB = p->ws + units * gsz;
    float2 *bufY = p->ws + 2 * units * gsz;
    float2 *bufP = bufY + units * p->M;
    const KbnGeom geom = p->geom();
    for (int64_t b0 = 0; b0 < B; b0 += ck.bc)
    for (int c0 = 0; c0 < C; c0 += ck.cc) {
        const int64_t nb = std::min<int64_t>(ck.bc, B - b0);
        const int ncc = std::min(ck.cc, C - c0);
        const int64_t nch = nb * ncc;
        const KbnSpreadArgs sa = t1_spread_args(p, nch, y + (b0 * C + c0) * p->M, bufA, bufY, bufP);
        KBN_LAUNCH(KBN_CLASS_SPREAD, kbn_launch_spread(geom, sa, stream), "spread");
        rc = t1_passes(p, b0, c0, nb, ncc, smaps, x, bufA, bufB, stream);
        if (rc != KBN_OK) return rc;
    }
    return KBN_OK;
}

int run_jac(kbn_plan p, int B, int C, const float2 *img, const float2 *smaps, const float2 *v,
            float *dom, int accumulate, hipStream_t stream) {
    if (!dom && p->M > 0) return fail(KBN_ERR_INVALID_ARG, "null domega");
    if (p->M == 0) return KBN_OK;
    return run_type2(p, B, C, p->D, 1, img, smaps, 1, nullptr, v, dom, accumulate, stream);
}

// y = E x and the omega-gradient of run_jac in one pass.  In 2D with the
// specialised FFT lengths, the first pass (along axis 1) transforms the
// unweighted and the r^[1]-weighted images only: r^[0] is constant along
// axis-1 lines, so the axis-0 pass derives the r^[0] channel by scaling the
// unweighted channel's rows (the persistent pass scales the values it holds
// for the source tile).  This saves one grid-row write and one read per image-coil pair
// against kbn_forward followed by kbn_jac_omega_fwd.  The unweighted channel
// goes through the same steps as in kbn_forward (same y bits); the derived
// channel rounds the product r^[0] * window scale in another order than
// the weighted first pass.  Other shapes run the two calls.
int run_fwd_jac(kbn_plan p, int B, int C, const float2 *x, const float2 *smaps, float2 *y, const float2 *g,
                float *dom, int accumulate, hipStream_t stream) {
    const int D = p->D;
    const bool fuse = D == 2 && p->fast_fft && kbn_fast_fft_size(p->K[0]) && kbn_fast_fft_size(p->K[1]);
    if (!fuse) {
        int rc = run_type2(p, B, C, 1, 0, x, smaps, 0, y, nullptr, nullptr, 0, stream);
        return rc == KBN_OK ? run_jac(p, B, C, x, smaps, g, dom, accumulate, stream) : rc;
    }
    const int64_t gsz = p->gsize();
    const int64_t R0 = img_rows(p);
    const int Nl = p->N[D - 1];
    const Chunks ck = split_chunks(B, C, fwd_jac_per_coil(p), p->max_ws);
    const int64_t units = ck.bc * ck.cc;
    int rc = ensure_ws(p, ws_fwd_jac(p, p->M, B, C), stream);
    if (rc != KBN_OK) return rc;
    float2 *bufA = p->ws;
    float2 *bufB = p->ws + units * (D + 1) * gsz;
    float *part = (float *)(p->ws + 2 * units * (D + 1) * gsz);
    const KbnGeom geom = p->geom();
    for (int64_t b0 = 0; b0 < B; b0 += ck.bc)
    for (int c0 = 0; c0 < C; c0 += ck.cc) {
        const int64_t nb = std::min<int64_t>(ck.bc, B - b0);
        const int ncc = std::min(ck.cc, C - c0);
        const int64_t npair = nb * ncc;
        KbnFirstPassArgs fa;
        fa.x = x + b0 * R0 * Nl;
        fa.smaps = smaps ? smaps + (int64_t)c0 * R0 * Nl : nullptr;
        fa.out = bufA;
        fa.nlines = npair * D * R0;
        fa.R0 = (int)R0;
        fa.Nl = Nl;
        fa.C = ncc;
        fa.nw = D;
        fa.weighted = 1;
        fa.D = D;
        for (int d = 0; d < KBN_MAX_D; ++d) {
            fa.N[d] = p->N[d];
            fa.deap[d] = p->deap[d];
        }
        fa.nplain = npair;
        KBN_LAUNCH(KBN_CLASS_FFT_FIRST, kbn_launch_fast_first(fa, p->K[1], p->tw[1], stream), "first pass");
        KbnMidPassArgs ma;
        ma.in = bufA;
        ma.out = bufB;
        ma.outer = npair * (D + 1);
        ma.nin = p->N[0];
        ma.nout = p->K[0];
        ma.inner = p->K[1];
        ma.pad_in = 1;
        ma.crop_out = 0;
        ma.dsplit = npair;
        ma.dnw = D;
        KBN_LAUNCH(KBN_CLASS_FFT_MID_FWD, kbn_launch_fast_mid(ma, p->K[0], p->tw[0], 0, stream), "mid pass");
        // the FFT passes overlap the index pass (waiting before the axis-0
        // pass measured 1.79 against 1.76 ms on the 256-image step)
        rc = points_wait(p, stream);
        if (rc != KBN_OK) return rc;
        const int64_t k0 = (b0 * C + c0) * p->M;
        const KbnGatherArgs gy = t2_gather_args(p, npair, ncc, 1, 0, bufB, k0, y, nullptr, nullptr, nullptr, 0);
        KBN_LAUNCH(KBN_CLASS_GATHER, kbn_launch_gather(geom, gy, 0, stream), "gather");
        const KbnGatherArgs gj = t2_gather_args(p, npair * D, ncc, D, 1, bufB + npair * gsz, k0, nullptr, g, dom,
                                                part, (accumulate || b0 > 0 || c0 > 0) ? 1 : 0);
        KBN_LAUNCH(KBN_CLASS_GATHER_JAC, kbn_launch_gather(geom, gj, 1, stream), "gather");
    }
    return KBN_OK;
}

// Tile edge nearest to `want` (searching down and up, at least J) whose last
// partial tile is empty or at least J cells wide, so that a J-tap footprint
// meets at most two tiles per axis; the whole axis if none exists.
int pick_tile(int K, int want, int J) {
    want = std::max(J, std::min(want, K));
    for (int dlt = 0; dlt <= K; ++dlt) {
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            const int T = want + sgn * dlt;
            if (T < J || T > K) continue;
            if (K % T == 0 || K % T >= J) return T;
            if (dlt == 0) break;
        }
    }
    return K;
}

}  // namespace

// Hooks for the batch executor (batch.cpp).
bool kbn_internal_timing_on(kbn_plan p) { return p->timing; }
void kbn_internal_graph_ref(kbn_plan p, int delta) { p->graph_refs += delta; }
int kbn_internal_fail(int code, const char *msg) { return fail(code, msg); }
double kbn_internal_cost(kbn_plan p, int B, int C, int jac, int type1) {
    // bytes the call moves under the kernel byte model: D + 1 grid sweeps
    // per channel (D channels per coil for an omega-Jacobian) plus the
    // k-space and image traffic
    const double g = (double)p->gsize() * 8.0 * (p->D + 1) * (jac && !type1 ? p->D : 1);
    double n = 1.0;
    for (int d = 0; d < p->D; ++d) n *= p->N[d];
    return (double)B * C * (g + 8.0 * (double)std::max<int64_t>(p->M, 0) + 8.0 * n);
}

uint64_t kbn_internal_epoch(kbn_plan p) { return p->epoch; }
int kbn_internal_points_wait(kbn_plan p, hipStream_t s) { return points_wait(p, s); }
void kbn_internal_points_settle(kbn_plan p) {
    if (p->points_pending && hipEventQuery(p->points_ready) == hipSuccess) p->points_pending = false;
}

int kbn_internal_alloc(kbn_plan p, void **ptr, int64_t bytes, hipStream_t s) {
    return dev_alloc(p, (char **)ptr, bytes, s);
}
void kbn_internal_free(kbn_plan p, void *ptr, hipStream_t s) {
    char *q = (char *)ptr;
    dev_free(p, q, s);
}

// A task in phases: validated as its call, with a workspace of its own so
// that the interpolation of many tasks can run in one launch between the
// tasks' FFT passes.  Tasks that need several chunks, have no points, or
// whose interpolation would take another kernel stay whole (kind -1).
int kbn_internal_phase_prepare(const kbn_task &t, KbnPhased *ph, hipStream_t s) {
    *ph = KbnPhased();
    ph->p = t.plan;
    ph->op = t.op;
    kbn_plan p = t.plan;
    int rc = KBN_OK;
    switch (t.op) {
    case KBN_TASK_FORWARD:
    case KBN_TASK_JAC_X_ADJ:
        rc = check_common(p, t.B, t.C, t.a, t.smaps, t.out);
        ph->kind = 0;
        ph->nw = 1;
        ph->weighted = 0;
        ph->x = (const float2 *)t.a;
        ph->y = (float2 *)t.out;
        break;
    case KBN_TASK_JAC_OMEGA_FWD:
    case KBN_TASK_JAC_OMEGA_ADJ: {
        const bool fwd = t.op == KBN_TASK_JAC_OMEGA_FWD;
        // fwd: image a, upstream k-space g; adj: k-space a, upstream image g
        rc = fwd ? check_common(p, t.B, t.C, t.a, t.smaps, t.g) : check_common(p, t.B, t.C, t.g, t.smaps, t.a);
        if (rc == KBN_OK && !t.out && p->M > 0) rc = fail(KBN_ERR_INVALID_ARG, "null domega");
        ph->kind = 1;
        ph->nw = p->D;
        ph->weighted = 1;
        ph->x = (const float2 *)(fwd ? t.a : t.g);
        ph->v = (const float2 *)(fwd ? t.g : t.a);
        ph->dom = (float *)t.out;
        ph->accumulate = t.accumulate;
        break;
    }
    case KBN_TASK_ADJOINT:
    case KBN_TASK_JAC_X_FWD:
        rc = check_common(p, t.B, t.C, t.out, t.smaps, t.a);
        ph->kind = 2;
        ph->ky = (const float2 *)t.a;
        ph->img = (float2 *)t.out;
        break;
    default:
        return fail(KBN_ERR_INVALID_ARG, "unknown task op");
    }
    if (rc != KBN_OK) return rc;
    ph->B = t.B;
    ph->C = t.C;
    ph->smaps = (const float2 *)t.smaps;
    const KbnGeom geom = p->geom();
    const int64_t gsz = p->gsize();
    const int64_t units = (int64_t)t.B * t.C;
    if (p->M == 0) {
        ph->kind = -1;
        return KBN_OK;
    }
    if (ph->kind <= 1) {
        const int64_t per_coil = (int64_t)ph->nw * gsz * (int64_t)sizeof(float2) * 2;
        const Chunks ck = split_chunks(t.B, t.C, per_coil, p->max_ws);
        const int64_t nch = units * ph->nw;
        const KbnGatherShape sh = kbn_gather_shape(geom, p->M, (int)nch, ph->nw);
        if (ck.bc != t.B || ck.cc != t.C || !sh.staged) {
            ph->kind = -1;
            return KBN_OK;
        }
        const int64_t grids = 2 * nch * gsz * (int64_t)sizeof(float2);
        const int64_t part = ph->kind == 1 ? (int64_t)sh.groups * p->M * p->D * (int64_t)sizeof(float) : 0;
        rc = kbn_internal_alloc(p, (void **)&ph->ws, grids + part, s);
        if (rc != KBN_OK) return rc;
        ph->bufA = (float2 *)ph->ws;
        ph->bufB = ph->bufA + nch * gsz;
        float *partp = (float *)(ph->bufA + 2 * nch * gsz);
        // the grid the passes end in: the last axis pass writes bufA and each
        // strided pass swaps the buffers
        float2 *grid = (p->D - 1) % 2 == 0 ? ph->bufA : ph->bufB;
        ph->gj.g = geom;
        ph->gj.a = t2_gather_args(p, nch, t.C, ph->nw, ph->kind, grid, 0, ph->y, ph->v, ph->dom, partp,
                                  ph->accumulate ? 1 : 0);
        ph->gj.cg = sh.cg;
        ph->gj.blocks = (int)sh.blocks;
        ph->groups = sh.groups;
        ph->lds = sh.lds;
        return KBN_OK;
    }
    const int64_t per_coil = type1_per_coil(p, p->M);
    const Chunks ck = split_chunks(t.B, t.C, per_coil, p->max_ws);
    KbnSpreadArgs probe = t1_spread_args(p, units, ph->ky, nullptr, nullptr, nullptr);
    const KbnSpreadSel sel = kbn_spread_select(geom, probe);
    if (ck.bc != t.B || ck.cc != t.C || sel.path != KBN_SPREAD_PATH_OS) {
        ph->kind = -1;
        return KBN_OK;
    }
    rc = kbn_internal_alloc(p, (void **)&ph->ws, units * per_coil, s);
    if (rc != KBN_OK) return rc;
    ph->bufA = (float2 *)ph->ws;
    ph->bufB = ph->bufA + units * gsz;
    float2 *bufY = ph->bufA + 2 * units * gsz;
    float2 *bufP = bufY + units * p->M;
    ph->sj.g = geom;
    ph->sj.a = t1_spread_args(p, units, ph->ky, ph->bufA, bufY, bufP);
    ph->sj.ngr = sel.ngr;
    ph->sj.ny = sel.ny;
    ph->sel = sel;
    return KBN_OK;
}

// Before the interpolation: the FFT passes of a forward-type task.
int kbn_internal_phase_pre(KbnPhased *ph, hipStream_t stream) {
    if (ph->kind < 0 || ph->kind > 1) return KBN_OK;
    kbn_plan p = ph->p;
    float2 *grid = nullptr;
    return t2_passes(p, ph->nw, ph->weighted, ph->x, ph->smaps, 0, 0, ph->B, ph->C, ph->bufA, ph->bufB, &grid,
                     stream);
}

// After the interpolation: the omega-gradient's sum over channel groups, or
// the adjoint's split-tile sums and inverse FFT passes.
int kbn_internal_phase_post(KbnPhased *ph, hipStream_t stream) {
    kbn_plan p = ph->p;
    if (ph->kind == 1)
        KBN_LAUNCH(KBN_CLASS_GATHER_JAC, kbn_launch_gather_reduce(ph->gj.g, ph->gj.a, stream), "gradient sum");
    if (ph->kind == 2) {
        KBN_LAUNCH(KBN_CLASS_SPREAD, kbn_launch_spread_combine(ph->sel, ph->sj.g, ph->sj.a, stream), "spread combine");
        return t1_passes(p, 0, 0, ph->B, ph->C, ph->smaps, ph->img, ph->bufA, ph->bufB, stream);
    }
    return KBN_OK;
}

void kbn_internal_phase_release(KbnPhased *ph, hipStream_t s) {
    if (ph->ws) kbn_internal_free(ph->p, ph->ws, s);
    ph->ws = nullptr;
}

// Grid workspace of kbn_forward_static: one file-scope array per GPU, for
// callers that cannot allocate.  In host code `scratch` only names the
// symbol; its device address on the current GPU comes from
// hipGetSymbolAddress, once per device, and only that address is used.
static __device__ __align__(256) char scratch[KBN_STATIC_WORKSPACE];

namespace {

#define KBN_MAX_DEVICES 64
std::mutex g_scratch_mu;
void *g_scratch[KBN_MAX_DEVICES] = {};

// The static workspace's device address on the current device.
int static_workspace(void **out) {
    int dev = -1;
    KBN_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= KBN_MAX_DEVICES) return fail(KBN_ERR_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(KBN_ERR_HIP, std::string("hipGetSymbolAddress (static workspace): ") + hipGetErrorString(e));
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return KBN_OK;
}

// Host-only part of plan creation: sizes, window shape, tiles (no device
// memory, no HIP call).  Shared by kbn_plan_create and kbn_plan_footprint.
int plan_setup(kbn_plan p, int D, const int64_t *N, const kbn_opts *opts) {
    if (D < 1 || D > KBN_MAX_D || !N) return fail(KBN_ERR_INVALID_ARG, "D must be 1..3");
    kbn_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    const double sigma = o.sigma == 0.0 ? 2.0 : o.sigma;
    const int J = o.J == 0 ? 6 : o.J;
    if (!(sigma >= 1.0) || sigma > 16.0) return fail(KBN_ERR_INVALID_ARG, "sigma must be in [1, 16]");
    if (J < 2 || J > KBN_MAX_J) return fail(KBN_ERR_INVALID_ARG, "J must be in 2..8");
    const double rad = (J / sigma) * (J / sigma) * (sigma - 0.5) * (sigma - 0.5) - 0.8;
    if (!(rad > 0.0)) return fail(KBN_ERR_INVALID_ARG, "window shape undefined for this (J, sigma)");
    p->D = D;
    p->J = J;
    p->sigma = sigma;
    p->beta = M_PI * std::sqrt(rad);
    p->max_ws = o.max_workspace > 0 ? o.max_workspace : (int64_t)4 << 30;
    if (const char *e = std::getenv("KBN_MAXE")) p->maxe = std::atoi(e) == 32 ? 32 : 16;
    if (const char *e = std::getenv("KBN_GENERIC_FFT")) p->fast_fft = std::atoi(e) == 0;
    const int deftile = D == 1 ? 256 : (D == 2 ? 32 : 8);
    int64_t ntiles = 1;
    for (int d = 0; d < D; ++d) {
        if (N[d] < 1 || N[d] > (1 << 20)) return fail(KBN_ERR_INVALID_ARG, "N_d must be >= 1");
        p->N[d] = (int)N[d];
        const int K = smooth_size(sigma * (double)N[d]);
        if (K > KBN_MAX_K || K < 2 * J)
            return fail(KBN_ERR_UNSUPPORTED, "oversampled size K_d = " + std::to_string(K) +
                                                 " outside [2J, " + std::to_string(KBN_MAX_K) + "]");
        p->K[d] = K;
        p->scale[d] = (double)K * (1.0 / (2.0 * M_PI));
        if (!factor(K, p->rad[d])) return fail(KBN_ERR_UNSUPPORTED, "K_d not 7-smooth");
    }
    // sorting / gather tiles; the automatic size grows until the tile count
    // fits the LDS histogram
    const bool explicit_tile = o.tile[0] > 0 || (D > 1 && o.tile[1] > 0) || (D > 2 && o.tile[2] > 0);
    for (int dt = deftile;; dt += 4) {
        ntiles = 1;
        for (int d = 0; d < D; ++d) {
            const int K = p->K[d];
            const int T = pick_tile(K, o.tile[d] > 0 ? o.tile[d] : dt, J);
            p->T[d] = T;
            p->nt[d] = (K + T - 1) / T;
            ntiles *= p->nt[d];
        }
        if (ntiles <= KBN_MAX_TILES || explicit_tile || dt >= KBN_MAX_K) break;
    }
    if (ntiles > KBN_MAX_TILES) return fail(KBN_ERR_UNSUPPORTED, "too many tiles; use larger tiles");
    p->ntiles = (int)ntiles;
    // spread owner tiles: small enough that several channels' accumulators fit
    // in LDS, large enough that the tile count fits the LDS histogram
    int64_t ntiles_own = 1;
    int defown = o.spread_tile > 0 ? std::max(J, o.spread_tile) : (D == 1 ? 128 : 8);
    for (;;) {
        ntiles_own = 1;
        for (int d = 0; d < D; ++d) {
            const int K = p->K[d];
            const int T = pick_tile(K, defown, J);
            p->To[d] = T;
            p->nto[d] = (K + T - 1) / T;
            ntiles_own *= p->nto[d];
        }
        if (ntiles_own <= KBN_MAX_TILES || defown >= KBN_MAX_K) break;
        defown += 4;
    }
    if (ntiles_own > KBN_MAX_TILES) {
        return fail(KBN_ERR_UNSUPPORTED, "too many spread tiles");
    }
    p->ntiles_own = (int)ntiles_own;
    // partial-tile slots: a larger pool splits hot tiles into more work
    // items, but the extra partial writes and sums cost more than the
    // shorter items save (measured on 2D radial and 3D kooshball inputs)
    p->smax = KBN_SPREAD_SMAX;
    return KBN_OK;
}

// Device constants of a plan: element counts of the blocks created with it.
struct ConstSizes {
    int64_t deap[KBN_MAX_D], tw[KBN_MAX_D], coef, toff, ooff, otile_order, scomb;
};

ConstSizes const_sizes(const kbn_plan p) {
    ConstSizes c{};
    for (int d = 0; d < p->D; ++d) {
        c.deap[d] = p->N[d];
        c.tw[d] = p->K[d];
    }
    c.coef = (int64_t)p->J * KBN_NCOEF;
    c.toff = (int64_t)p->ntiles + 2;
    c.ooff = (int64_t)p->ntiles_own + 1;
    c.otile_order = p->ntiles_own;
    c.scomb = 3 * (int64_t)p->ntiles_own;
    return c;
}

int64_t const_bytes(const kbn_plan p) {
    const ConstSizes c = const_sizes(p);
    int64_t b = 0;
    for (int d = 0; d < p->D; ++d)
        b += block_bytes(4 * c.deap[d]) + block_bytes(8 * c.tw[d]);
    b += block_bytes(4 * c.coef) + block_bytes(4) /*flag*/ + block_bytes(4 * c.toff) +
         block_bytes(4) /*nsub*/ + block_bytes(4 * c.ooff) + block_bytes(4 * c.otile_order) +
         block_bytes(4 * c.scomb) + block_bytes(8) /*scounts*/;
    return b;
}

// The index pass's launches on the plan's stream (omega_read is recorded
// after the kernel that reads omega, or at once if the pass stops before).
int index_pass(kbn_plan p, int64_t M, const float *omega, const KbnPointsBufs &b, hipStream_t stream) {
    if (stream == p->istream) {
        const hipError_t e0 = hipEventRecord(p->omega_read, stream);  // replaced below once omega is read
        if (e0 != hipSuccess) return fail(KBN_ERR_HIP, "index stream order");
    }
    KBN_LAUNCH(KBN_CLASS_INDEX,
               kbn_launch_points(p->D, M, omega, p->scale, p->K, p->T, p->nt, p->ntiles, p->ntiles_own, p->sub, b,
                                 stream, stream == p->istream ? p->omega_read : nullptr),
               "index pass");
    KBN_LAUNCH(KBN_CLASS_INDEX,
               kbn_launch_owner_lists(p->geom(), M, p->cell, p->frac, p->toff, p->order,
                                      p->counts + kbn_points_owner_base(M, p->ntiles), p->ooff, p->otile_order,
                                      KBN_SPREAD_SEG, p->smax, p->swork, p->scomb, p->scounts, p->rec_p, p->rec_q,
                                      p->rec_l, p->rec_f, stream),
               "spread lists");
    return KBN_OK;
}

}  // namespace

extern "C" {

int kbn_plan_create(kbn_plan *out, int D, const int64_t *N, const kbn_opts *opts,
                    const kbn_allocator *alloc, void *stream_) {
    if (!out) return fail(KBN_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    if (alloc && (!alloc->alloc || !alloc->free))
        return fail(KBN_ERR_INVALID_ARG, "allocator needs both alloc and free");
    hipStream_t stream = (hipStream_t)stream_;
    kbn_plan p = new (std::nothrow) kbn_plan_s();
    if (!p) return fail(KBN_ERR_OOM, "host allocation failed");
    if (alloc) {
        p->alloc = *alloc;
        p->custom_alloc = true;
    }
    int rc = plan_setup(p, D, N, opts);
    if (rc != KBN_OK) {
        delete p;
        return rc;
    }
    // constants in FP64 on the host, kept by the plan until uploaded
    Window w{p->J, p->beta, bessel_i0(p->beta)};
    for (int d = 0; d < D; ++d) {
        p->h_deap[d].resize(p->N[d]);
        for (int j = 0; j < p->N[d]; ++j) {
            const double r = (double)(j - p->N[d] / 2);
            p->h_deap[d][j] = (float)(1.0 / w.psi_hat(r / p->K[d]));
        }
        p->h_tw[d].resize(p->K[d]);
        for (int k = 0; k < p->K[d]; ++k) {
            const double a = 2.0 * M_PI * (double)k / (double)p->K[d];
            p->h_tw[d][k] = make_float2((float)std::cos(a), (float)-std::sin(a));
        }
    }
    p->h_coef = window_polys(w);
    const ConstSizes cs = const_sizes(p);
    for (int d = 0; d < D && rc == KBN_OK; ++d) {
        rc = dev_alloc(p, &p->deap[d], cs.deap[d], stream);
        if (rc == KBN_OK) rc = dev_alloc(p, &p->tw[d], cs.tw[d], stream);
        if (rc == KBN_OK && hipMemcpyAsync(p->deap[d], p->h_deap[d].data(), sizeof(float) * cs.deap[d],
                                           hipMemcpyHostToDevice, stream) != hipSuccess)
            rc = fail(KBN_ERR_HIP, "hipMemcpyAsync (scaling factors)");
        if (rc == KBN_OK && hipMemcpyAsync(p->tw[d], p->h_tw[d].data(), sizeof(float2) * cs.tw[d],
                                           hipMemcpyHostToDevice, stream) != hipSuccess)
            rc = fail(KBN_ERR_HIP, "hipMemcpyAsync (twiddles)");
    }
    if (rc == KBN_OK) rc = dev_alloc(p, &p->coef, cs.coef, stream);
    if (rc == KBN_OK && hipMemcpyAsync(p->coef, p->h_coef.data(), sizeof(float) * cs.coef,
                                       hipMemcpyHostToDevice, stream) != hipSuccess)
        rc = fail(KBN_ERR_HIP, "hipMemcpyAsync (window)");
    if (rc == KBN_OK) rc = dev_alloc(p, &p->flag, 1, stream);
    if (rc == KBN_OK && hipMemsetAsync(p->flag, 0, sizeof(int), stream) != hipSuccess)
        rc = fail(KBN_ERR_HIP, "hipMemsetAsync (flag)");
    if (rc == KBN_OK) rc = dev_alloc(p, &p->toff, cs.toff, stream);
    if (rc == KBN_OK) rc = dev_alloc(p, &p->nsub, 1, stream);
    if (rc == KBN_OK) rc = dev_alloc(p, &p->ooff, cs.ooff, stream);
    if (rc == KBN_OK) rc = dev_alloc(p, &p->otile_order, cs.otile_order, stream);
    if (rc == KBN_OK) rc = dev_alloc(p, &p->scomb, cs.scomb, stream);
    if (rc == KBN_OK) rc = dev_alloc(p, &p->scounts, 2, stream);
    if (rc == KBN_OK && (hipEventCreateWithFlags(&p->upload_done, hipEventDisableTiming) != hipSuccess ||
                         hipEventRecord(p->upload_done, stream) != hipSuccess))
        rc = fail(KBN_ERR_HIP, "upload event");
    if (rc == KBN_OK && (hipStreamCreateWithFlags(&p->istream, hipStreamNonBlocking) != hipSuccess ||
                         hipEventCreateWithFlags(&p->points_in, hipEventDisableTiming) != hipSuccess ||
                         hipEventCreateWithFlags(&p->points_ready, hipEventDisableTiming) != hipSuccess ||
                         hipEventCreateWithFlags(&p->omega_read, hipEventDisableTiming) != hipSuccess))
        rc = fail(KBN_ERR_HIP, "index stream");
    if (rc != KBN_OK) {
        const std::string msg = g_err;
        free_plan(p, stream);
        g_err = msg;
        return rc;
    }
    *out = p;
    return KBN_OK;
}

int kbn_set_points(kbn_plan p, int64_t M, const float *omega, void *stream_) {
    hipStream_t stream = (hipStream_t)stream_;
    if (!p) return fail(KBN_ERR_INVALID_ARG, "null plan");
    if (p->graph_refs > 0)
        return fail(KBN_ERR_UNSUPPORTED, "kbn_set_points on a plan held by a captured batch");
    // the owner lists hold up to M 2^D entries with int32 positions
    if (M < 0 || M > (2147483647LL >> p->D))
        return fail(KBN_ERR_INVALID_ARG, "M out of range (0 .. (2^31 - 1) / 2^D)");
    if (M > 0 && !omega) return fail(KBN_ERR_INVALID_ARG, "null omega");
    {
        // the previous index pass may still run: the frees, the new buffers
        // and the new pass come after it
        const int rc = points_wait(p, stream);
        if (rc != KBN_OK) return rc;
    }
    ++p->epoch;
    const PointSizes z = point_sizes(p, M);
    if (M > p->Mcap || z.counts > p->counts_cap) {
        // stream-ordered: work already queued may still read the old buffers
        free_points(p, stream);
        const int D = p->D;
        int rc = dev_alloc(p, &p->cell_tmp, z.cap * D, stream);
        if (rc == KBN_OK) rc = dev_alloc(p, &p->frac_tmp, z.cap * D, stream);
        if (rc == KBN_OK) rc = dev_alloc(p, &p->tile, z.cap, stream);
        if (rc == KBN_OK) rc = dev_alloc(p, &p->order, z.cap, stream);
        if (rc == KBN_OK) rc = dev_alloc(p, &p->cell, z.cap * D, stream);
        if (rc == KBN_OK) rc = dev_alloc(p, &p->frac, z.cap * D, stream);
        if (rc == KBN_OK) rc = dev_alloc(p, &p->counts, z.counts, stream);
        if (rc == KBN_OK) rc = dev_alloc(p, &p->subs, z.subs, stream);
        if (rc == KBN_OK) rc = dev_alloc(p, &p->swork, 4 * z.swork, stream);
        if (rc == KBN_OK) rc = dev_alloc(p, &p->rec_p, z.ent, stream);
        if (rc == KBN_OK) rc = dev_alloc(p, &p->rec_q, z.ent, stream);
        if (rc == KBN_OK) rc = dev_alloc(p, &p->rec_l, z.ent * D, stream);
        if (rc == KBN_OK) rc = dev_alloc(p, &p->rec_f, z.ent * D, stream);
        if (rc != KBN_OK) {
            const std::string msg = g_err;
            free_points(p, stream);
            p->M = -1;
            g_err = msg;
            return rc;
        }
        p->Mcap = z.cap;
        p->counts_cap = z.counts;
        p->swork_cap = z.swork;
    }
    KbnPointsBufs b;
    b.cell_tmp = p->cell_tmp;
    b.frac_tmp = p->frac_tmp;
    b.tile = p->tile;
    b.counts = p->counts;
    b.order = p->order;
    b.cell = p->cell;
    b.frac = p->frac;
    b.toff = p->toff;
    b.flag = p->flag;
    b.subs = p->subs;
    b.nsub = p->nsub;
    int rc;
    if (M < KBN_INDEX_STREAM_MIN) {
        // few points: the pass is a handful of short launches, cheaper on the
        // caller's stream than behind a cross-stream wait (which the
        // points_wait above already made any earlier pass's work precede)
        rc = index_pass(p, M, omega, b, stream);
        p->points_pending = false;
    } else {
        // the index pass on the plan's stream, after everything queued on the
        // caller's stream (omega, the buffers)
        if (hipEventRecord(p->points_in, stream) != hipSuccess ||
            hipStreamWaitEvent(p->istream, p->points_in, 0) != hipSuccess)
            return fail(KBN_ERR_HIP, "index stream order");
        p->points_pending = true;
        ++p->points_gen;
        rc = index_pass(p, M, omega, b, p->istream);
        // whatever was issued is waited for by later reads of the points, and
        // the caller's later work may overwrite omega once the first index
        // kernel has read it; the rest of the pass runs beside that work
        if (hipEventRecord(p->points_ready, p->istream) != hipSuccess ||
            hipStreamWaitEvent(stream, p->omega_read, 0) != hipSuccess)
            return fail(KBN_ERR_HIP, "index stream order");
    }
    if (rc != KBN_OK) {
        p->M = -1;
        return rc;
    }
    p->M = M;
    return KBN_OK;
}

int kbn_forward(kbn_plan p, int B, int C, const void *x, const void *smaps, void *y,
                void *stream) {
    int rc = check_common(p, B, C, x, smaps, y);
    if (rc != KBN_OK) return rc;
    if (p->M == 0) return KBN_OK;
    return run_type2(p, B, C, 1, 0, (const float2 *)x, (const float2 *)smaps, 0, (float2 *)y,
                     nullptr, nullptr, 0, (hipStream_t)stream);
}

int kbn_forward_static(kbn_plan p, int B, int C, const void *x, const void *smaps, void *y, void *stream) {
    int rc = check_common(p, B, C, x, smaps, y);
    if (rc != KBN_OK) return rc;
    if (p->timing) return fail(KBN_ERR_UNSUPPORTED, "kbn_forward_static does not record timing events");
    const int64_t per_coil = p->gsize() * (int64_t)sizeof(float2) * 2;
    if (per_coil > KBN_STATIC_WORKSPACE)
        return fail(KBN_ERR_UNSUPPORTED, "one image-coil pair needs " + std::to_string(per_coil) +
                                             " bytes of grid workspace; the static workspace holds " +
                                             std::to_string((int64_t)KBN_STATIC_WORKSPACE));
    void *ws = nullptr;
    rc = static_workspace(&ws);
    if (rc != KBN_OK) return rc;
    if (p->M == 0) return KBN_OK;
    return run_type2(p, B, C, 1, 0, (const float2 *)x, (const float2 *)smaps, 0, (float2 *)y, nullptr, nullptr,
                     0, (hipStream_t)stream, ws, KBN_STATIC_WORKSPACE);
}

int kbn_adjoint(kbn_plan p, int B, int C, const void *y, const void *smaps, void *x,
                void *stream) {
    int rc = check_common(p, B, C, x, smaps, y);
    if (rc != KBN_OK) return rc;
    return run_type1(p, B, C, (const float2 *)y, (const float2 *)smaps, (float2 *)x,
                     (hipStream_t)stream);
}

int kbn_jac_omega_fwd(kbn_plan p, int B, int C, const void *x, const void *smaps, const void *g,
                      float *domega, int accumulate, void *stream) {
    int rc = check_common(p, B, C, x, smaps, g);
    if (rc != KBN_OK) return rc;
    return run_jac(p, B, C, (const float2 *)x, (const float2 *)smaps, (const float2 *)g, domega,
                   accumulate, (hipStream_t)stream);
}

int kbn_forward_jac_omega(kbn_plan p, int B, int C, const void *x, const void *smaps, void *y, const void *g,
                          float *domega, int accumulate, void *stream) {
    int rc = check_common(p, B, C, x, smaps, y);
    if (rc == KBN_OK) rc = check_common(p, B, C, x, smaps, g);
    if (rc != KBN_OK) return rc;
    if (!domega && p->M > 0) return fail(KBN_ERR_INVALID_ARG, "null domega");
    if (p->M == 0) return KBN_OK;
    return run_fwd_jac(p, B, C, (const float2 *)x, (const float2 *)smaps, (float2 *)y, (const float2 *)g, domega,
                       accumulate, (hipStream_t)stream);
}

int kbn_jac_omega_adj(kbn_plan p, int B, int C, const void *y, const void *smaps, const void *g,
                      float *domega, int accumulate, void *stream) {
    int rc = check_common(p, B, C, g, smaps, y);
    if (rc != KBN_OK) return rc;
    return run_jac(p, B, C, (const float2 *)g, (const float2 *)smaps, (const float2 *)y, domega,
                   accumulate, (hipStream_t)stream);
}

int kbn_jac_x(kbn_plan p, int op, int B, int C, const void *g, const void *smaps, void *out,
              void *stream) {
    if (op == KBN_OP_FORWARD) return kbn_adjoint(p, B, C, g, smaps, out, stream);
    if (op == KBN_OP_ADJOINT) return kbn_forward(p, B, C, g, smaps, out, stream);
    return fail(KBN_ERR_INVALID_ARG, "unknown op");
}

// CG work buffer for B images: scalars [B][KBN_CG_NSCAL], block partials
// [B][KBN_CG_MAXPARTS], r, p, q (images [B][N..]), E p (k-space [B][C][M])
struct CgBufs {
    double *scal, *part;
    float2 *r, *p, *q, *ytmp;
};

static int64_t cg_align(int64_t b) { return (b + 255) / 256 * 256; }

static int64_t cg_bytes(kbn_plan p, int B, int C, CgBufs *b, void *work) {
    int64_t npix = 1;
    for (int d = 0; d < p->D; ++d) npix *= p->N[d];
    const int64_t o_part = cg_align((int64_t)B * KBN_CG_NSCAL * 8);
    const int64_t o_r = o_part + cg_align((int64_t)B * KBN_CG_MAXPARTS * 8);
    const int64_t img = cg_align((int64_t)B * npix * 8);
    const int64_t o_y = o_r + 3 * img;
    const int64_t total = o_y + cg_align(std::max<int64_t>(p->M, 0) * C * B * 8);
    if (b) {
        char *w = (char *)work;
        b->scal = (double *)w;
        b->part = (double *)(w + o_part);
        b->r = (float2 *)(w + o_r);
        b->p = (float2 *)(w + o_r + img);
        b->q = (float2 *)(w + o_r + 2 * img);
        b->ytmp = (float2 *)(w + o_y);
    }
    return total;
}

static int cg_launch(kbn_plan p, int kind, int B, int64_t n, float2 *x, const CgBufs &b, float lam, int reg,
                     hipStream_t s) {
    KbnCgImage img{reg, 1, 1, 1};
    int *ext[3] = {&img.n0, &img.n1, &img.n2};
    for (int d = 0; d < p->D; ++d) *ext[d] = (int)p->N[d];
    return launched(kbn_launch_cg(kind, B, n, x, b.r, b.p, b.q, lam, img, b.scal, b.part, s),
                    "cg vector kernel", s);
}

static int cg_check_batch(int B) {
    if (B < 1 || B > KBN_CG_MAXB) return fail(KBN_ERR_INVALID_ARG, "B must be in 1..65535");
    return KBN_OK;
}

int kbn_cg_work_bytes(kbn_plan p, int B, int C, int64_t *bytes) {
    if (!p || !bytes) return fail(KBN_ERR_INVALID_ARG, "null argument");
    if (p->M < 0) return fail(KBN_ERR_NO_POINTS, "kbn_set_points has not been called");
    if (C < 1) return fail(KBN_ERR_INVALID_ARG, "C must be >= 1");
    int rc = cg_check_batch(B);
    if (rc != KBN_OK) return rc;
    *bytes = cg_bytes(p, B, C, nullptr, nullptr);
    return KBN_OK;
}

int kbn_cg_begin(kbn_plan p, int B, int C, const void *smaps, const void *y, void *x, void *work,
                 void *stream_) {
    int rc = cg_check_batch(B);
    if (rc != KBN_OK) return rc;
    rc = check_common(p, B, C, x, smaps, y);
    if (rc != KBN_OK) return rc;
    if (!work) return fail(KBN_ERR_INVALID_ARG, "null work buffer");
    hipStream_t stream = (hipStream_t)stream_;
    CgBufs b;
    cg_bytes(p, B, C, &b, work);
    int64_t npix = 1;
    for (int d = 0; d < p->D; ++d) npix *= p->N[d];
    // r = b = E^H y (x0 = 0), p = r
    rc = run_type1(p, B, C, (const float2 *)y, (const float2 *)smaps, b.r, stream);
    if (rc != KBN_OK) return rc;
    return cg_launch(p, KBN_CGK_INIT, B, npix, (float2 *)x, b, 0.f, KBN_REG_IDENTITY, stream);
}

int kbn_cg_begin_image(kbn_plan p, int B, int C, const void *b, void *x, void *work, void *stream_) {
    if (!p) return fail(KBN_ERR_INVALID_ARG, "null plan");
    if (p->M < 0) return fail(KBN_ERR_NO_POINTS, "kbn_set_points has not been called");
    if (C < 1) return fail(KBN_ERR_INVALID_ARG, "C must be >= 1");
    int rc = cg_check_batch(B);
    if (rc != KBN_OK) return rc;
    if (!b || !x || !work) return fail(KBN_ERR_INVALID_ARG, "null pointer");
    hipStream_t stream = (hipStream_t)stream_;
    CgBufs cb;
    cg_bytes(p, B, C, &cb, work);
    int64_t npix = 1;
    for (int d = 0; d < p->D; ++d) npix *= p->N[d];
    // r = b (x0 = 0), p = r
    KBN_HIP(hipMemcpyAsync(cb.r, b, sizeof(float2) * npix * B, hipMemcpyDeviceToDevice, stream));
    return cg_launch(p, KBN_CGK_INIT, B, npix, (float2 *)x, cb, 0.f, KBN_REG_IDENTITY, stream);
}

int kbn_cg_step(kbn_plan p, int B, int C, const void *smaps, double lambda, int reg, int iters, void *x,
                void *work, void *stream_) {
    int rc = cg_check_batch(B);
    if (rc != KBN_OK) return rc;
    rc = check_common(p, B, C, x, smaps, work);
    if (rc != KBN_OK) return rc;
    if (!work) return fail(KBN_ERR_INVALID_ARG, "null work buffer");
    if (iters < 0) return fail(KBN_ERR_INVALID_ARG, "iters must be >= 0");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(KBN_ERR_INVALID_ARG, "lambda must be finite and >= 0");
    if (reg != KBN_REG_IDENTITY && reg != KBN_REG_FINITE_DIFF)
        return fail(KBN_ERR_INVALID_ARG, "reg must be KBN_REG_IDENTITY or KBN_REG_FINITE_DIFF");
    hipStream_t stream = (hipStream_t)stream_;
    CgBufs b;
    cg_bytes(p, B, C, &b, work);
    int64_t npix = 1;
    for (int d = 0; d < p->D; ++d) npix *= p->N[d];
    for (int it = 0; it < iters; ++it) {
        // q = E^H E p for every image (+ lambda T^H T p in the vector kernel)
        if (p->M > 0) {
            rc = run_type2(p, B, C, 1, 0, b.p, (const float2 *)smaps, 0, b.ytmp, nullptr, nullptr, 0,
                           stream);
            if (rc != KBN_OK) return rc;
        }
        rc = run_type1(p, B, C, b.ytmp, (const float2 *)smaps, b.q, stream);
        if (rc != KBN_OK) return rc;
        rc = cg_launch(p, KBN_CGK_Q, B, npix, (float2 *)x, b, (float)lambda, reg, stream);
        if (rc == KBN_OK) rc = cg_launch(p, KBN_CGK_XR, B, npix, (float2 *)x, b, 0.f, reg, stream);
        if (rc == KBN_OK) rc = cg_launch(p, KBN_CGK_P, B, npix, (float2 *)x, b, 0.f, reg, stream);
        if (rc != KBN_OK) return rc;
    }
    return KBN_OK;
}

// ---------------------------------------------------------------------------
// Off-resonance model (Sec. II-H): E = sum_l diag(b_l) (I_C kron A) diag(c_l) S.
// The L segments are L*C virtual coils with maps c_l s_k; k-space is expanded
// by conj(b_l) before the spread / Jacobian gather and combined by b_l after
// the forward gather.  Images are processed in chunks so that the expanded
// k-space of a chunk stays under the workspace cap.
// ---------------------------------------------------------------------------
struct FieldBufs {
    float2 *vm, *ye;
    int64_t bc;  // images per chunk
};

static int field_prep(kbn_plan p, int B, int C, int L, const void *smaps, const void *bw, const void *c,
                      FieldBufs *fb, hipStream_t stream) {
    if (L < 1) return fail(KBN_ERR_INVALID_ARG, "L must be >= 1");
    if (!c || (!bw && p->M > 0)) return fail(KBN_ERR_INVALID_ARG, "null segment coefficients");
    int64_t npix = 1;
    for (int d = 0; d < p->D; ++d) npix *= p->N[d];
    const int64_t LC = (int64_t)L * C;
    if (LC > (1 << 20)) return fail(KBN_ERR_INVALID_ARG, "L * C too large");
    const int64_t per_img = LC * std::max<int64_t>(p->M, 0) * (int64_t)sizeof(float2);
    fb->bc = per_img > 0 ? std::max<int64_t>(1, std::min<int64_t>(B, p->max_ws / per_img)) : B;
    const int64_t o_ye = (LC * npix * (int64_t)sizeof(float2) + 255) / 256 * 256;
    const int64_t bytes = o_ye + fb->bc * per_img;
    if (bytes > p->fws_bytes) {
        if (p->graph_refs > 0)
            return fail(KBN_ERR_UNSUPPORTED, "workspace growth on a plan held by a captured batch");
        dev_free(p, p->fws, stream);  // stream-ordered: queued work may still read it
        p->fws_bytes = 0;
        int rc = dev_alloc(p, &p->fws, bytes, stream);
        if (rc != KBN_OK) return rc;
        p->fws_bytes = bytes;
    }
    fb->vm = (float2 *)p->fws;
    fb->ye = (float2 *)(p->fws + o_ye);
    return launched(kbn_launch_field_maps(L, C, npix, (const float2 *)c, (const float2 *)smaps, fb->vm, stream),
                    "field maps", stream);
}

int kbn_field_forward(kbn_plan p, int B, int C, int L, const void *x, const void *smaps, const void *bw,
                      const void *c, void *y, void *stream_) {
    int rc = check_common(p, B, C, x, smaps, y);
    if (rc != KBN_OK) return rc;
    if (p->M == 0) return L < 1 ? fail(KBN_ERR_INVALID_ARG, "L must be >= 1") : KBN_OK;
    hipStream_t stream = (hipStream_t)stream_;
    FieldBufs fb;
    rc = field_prep(p, B, C, L, smaps, bw, c, &fb, stream);
    if (rc != KBN_OK) return rc;
    const int64_t npix = (int64_t)img_rows(p) * p->N[p->D - 1];
    const int LC = L * C;
    for (int64_t b0 = 0; b0 < B; b0 += fb.bc) {
        const int64_t nb = std::min<int64_t>(fb.bc, B - b0);
        rc = run_type2(p, (int)nb, LC, 1, 0, (const float2 *)x + b0 * npix, fb.vm, 0, fb.ye, nullptr,
                       nullptr, 0, stream);
        if (rc != KBN_OK) return rc;
        rc = launched(kbn_launch_field_combine(nb, L, C, p->M, (const float2 *)bw, fb.ye,
                                               (float2 *)y + b0 * C * p->M, stream),
                      "field combine", stream);
        if (rc != KBN_OK) return rc;
    }
    return KBN_OK;
}

int kbn_field_adjoint(kbn_plan p, int B, int C, int L, const void *y, const void *smaps, const void *bw,
                      const void *c, void *x, void *stream_) {
    int rc = check_common(p, B, C, x, smaps, y);
    if (rc != KBN_OK) return rc;
    hipStream_t stream = (hipStream_t)stream_;
    FieldBufs fb;
    rc = field_prep(p, B, C, L, smaps, bw, c, &fb, stream);
    if (rc != KBN_OK) return rc;
    const int64_t npix = (int64_t)img_rows(p) * p->N[p->D - 1];
    for (int64_t b0 = 0; b0 < B; b0 += fb.bc) {
        const int64_t nb = std::min<int64_t>(fb.bc, B - b0);
        rc = launched(kbn_launch_field_expand(nb, L, C, p->M, (const float2 *)bw,
                                              (const float2 *)y + b0 * C * std::max<int64_t>(p->M, 0), fb.ye,
                                              stream),
                      "field expand", stream);
        if (rc != KBN_OK) return rc;
        rc = run_type1(p, (int)nb, L * C, fb.ye, fb.vm, (float2 *)x + b0 * npix, stream);
        if (rc != KBN_OK) return rc;
    }
    return KBN_OK;
}

// shared by the two omega-Jacobians: expand the k-space operand kv by
// conj(b_l) and gather the Jacobian channels of the image operand im
static int field_jac(kbn_plan p, int B, int C, int L, const void *im, const void *smaps, const void *bw,
                     const void *c, const void *kv, float *dom, int accumulate, hipStream_t stream) {
    if (!dom) return fail(KBN_ERR_INVALID_ARG, "null domega");
    FieldBufs fb;
    int rc = field_prep(p, B, C, L, smaps, bw, c, &fb, stream);
    if (rc != KBN_OK) return rc;
    const int64_t npix = (int64_t)img_rows(p) * p->N[p->D - 1];
    for (int64_t b0 = 0; b0 < B; b0 += fb.bc) {
        const int64_t nb = std::min<int64_t>(fb.bc, B - b0);
        rc = launched(kbn_launch_field_expand(nb, L, C, p->M, (const float2 *)bw,
                                              (const float2 *)kv + b0 * C * p->M, fb.ye, stream),
                      "field expand", stream);
        if (rc != KBN_OK) return rc;
        rc = run_jac(p, (int)nb, L * C, (const float2 *)im + b0 * npix, fb.vm, fb.ye, dom,
                     (accumulate || b0 > 0) ? 1 : 0, stream);
        if (rc != KBN_OK) return rc;
    }
    return KBN_OK;
}

int kbn_field_jac_omega_fwd(kbn_plan p, int B, int C, int L, const void *x, const void *smaps,
                            const void *bw, const void *c, const void *g, float *domega, int accumulate,
                            void *stream) {
    int rc = check_common(p, B, C, x, smaps, g);
    if (rc != KBN_OK) return rc;
    if (L < 1) return fail(KBN_ERR_INVALID_ARG, "L must be >= 1");
    if (p->M == 0) return KBN_OK;
    return field_jac(p, B, C, L, x, smaps, bw, c, g, domega, accumulate, (hipStream_t)stream);
}

int kbn_field_jac_omega_adj(kbn_plan p, int B, int C, int L, const void *y, const void *smaps,
                            const void *bw, const void *c, const void *g, float *domega, int accumulate,
                            void *stream) {
    int rc = check_common(p, B, C, g, smaps, y);
    if (rc != KBN_OK) return rc;
    if (L < 1) return fail(KBN_ERR_INVALID_ARG, "L must be >= 1");
    if (p->M == 0) return KBN_OK;
    return field_jac(p, B, C, L, g, smaps, bw, c, y, domega, accumulate, (hipStream_t)stream);
}

int kbn_field_segments(int64_t M, const float *t, double t0, double t1, int64_t npix, const float *w,
                       int L, void *bw, void *c, void *stream) {
    if (M < 0 || npix < 1 || L < 1) return fail(KBN_ERR_INVALID_ARG, "bad sizes");
    if (!std::isfinite(t0) || !std::isfinite(t1) || t1 < t0)
        return fail(KBN_ERR_INVALID_ARG, "segment window must be finite with t1 >= t0");
    if ((M > 0 && (!t || !bw)) || !w || !c) return fail(KBN_ERR_INVALID_ARG, "null pointer");
    return launched(kbn_launch_field_segments(M, t, t0, t1, npix, w, L, (float2 *)bw, (float2 *)c,
                                              (hipStream_t)stream),
                    "field segments", (hipStream_t)stream);
}

int kbn_plan_info(kbn_plan p, int64_t *K, int *tile, int *ntiles, double *beta, int64_t *M,
                  int64_t *workspace_bytes, int64_t *device_bytes) {
    if (!p) return fail(KBN_ERR_INVALID_ARG, "null plan");
    for (int d = 0; d < p->D; ++d) {
        if (K) K[d] = p->K[d];
        if (tile) tile[d] = p->T[d];
    }
    if (ntiles) *ntiles = p->ntiles;
    if (beta) *beta = p->beta;
    if (M) *M = p->M < 0 ? 0 : p->M;
    if (workspace_bytes) *workspace_bytes = p->ws_bytes;
    if (device_bytes) *device_bytes = p->dev_bytes;
    return KBN_OK;
}

int kbn_plan_footprint(int D, const int64_t *N, const kbn_opts *opts, int64_t M, int B, int C, int jac,
                       int64_t *bytes) {
    if (!bytes) return fail(KBN_ERR_INVALID_ARG, "null output pointer");
    if (M < 0 || B < 1 || C < 1) return fail(KBN_ERR_INVALID_ARG, "M >= 0, B >= 1 and C >= 1 required");
    kbn_plan_s q;
    const int rc = plan_setup(&q, D, N, opts);
    if (rc != KBN_OK) return rc;
    if (M > (2147483647LL >> q.D)) return fail(KBN_ERR_INVALID_ARG, "M out of range (0 .. (2^31 - 1) / 2^D)");
    int64_t ws = std::max(M > 0 ? ws_type2(&q, M, B, C, 1, 0) : 0, ws_type1(&q, M, B, C));
    if (jac && M > 0) ws = std::max(ws, ws_type2(&q, M, B, C, q.D, 1));
    *bytes = const_bytes(&q) + points_bytes(&q, M) + block_bytes(ws);
    return KBN_OK;
}

int kbn_get_points(kbn_plan p, int *order, int *cell, float *frac, int *offsets, void *stream_) {
    hipStream_t stream = (hipStream_t)stream_;
    if (!p) return fail(KBN_ERR_INVALID_ARG, "null plan");
    if (p->M < 0) return fail(KBN_ERR_NO_POINTS, "kbn_set_points has not been called");
    const int64_t M = p->M;
    const int rcw = points_wait(p, stream);
    if (rcw != KBN_OK) return rcw;
    if (M > 0) {
        if (order) KBN_HIP(hipMemcpyAsync(order, p->order, sizeof(int) * M, hipMemcpyDeviceToDevice, stream));
        if (cell)
            KBN_HIP(hipMemcpyAsync(cell, p->cell, sizeof(int) * M * p->D, hipMemcpyDeviceToDevice, stream));
        if (frac)
            KBN_HIP(hipMemcpyAsync(frac, p->frac, sizeof(float) * M * p->D, hipMemcpyDeviceToDevice, stream));
    }
    if (offsets)
        KBN_HIP(hipMemcpyAsync(offsets, p->toff, sizeof(int) * (p->ntiles + 2),
                               hipMemcpyDeviceToDevice, stream));
    return KBN_OK;
}

int kbn_check_error(kbn_plan p, void *stream) {
    if (!p) return fail(KBN_ERR_INVALID_ARG, "null plan");
    KBN_HIP(hipStreamSynchronize((hipStream_t)stream));
    if (p->points_pending) {
        KBN_HIP(hipEventSynchronize(p->points_ready));
        p->points_pending = false;
    }
    int h = 0;
    KBN_HIP(hipMemcpy(&h, p->flag, sizeof(int), hipMemcpyDeviceToHost));
    if (h) {
        KBN_HIP(hipMemset(p->flag, 0, sizeof(int)));
        return fail(KBN_ERR_NONFINITE, "non-finite or out-of-range omega");
    }
    return KBN_OK;
}

int kbn_plan_destroy(kbn_plan p, void *stream) {
    if (!p) return fail(KBN_ERR_INVALID_ARG, "null plan");
    if (p->graph_refs > 0)
        return fail(KBN_ERR_INVALID_ARG, "plan is held by a captured batch; destroy the batch first");
    free_plan(p, (hipStream_t)stream);
    return KBN_OK;
}

int kbn_timing_select(kbn_plan p, unsigned int mask) {
    if (!p) return fail(KBN_ERR_INVALID_ARG, "null plan");
    p->timing_mask = mask;
    return KBN_OK;
}

int kbn_timing(kbn_plan p, int enable) {
    if (!p) return fail(KBN_ERR_INVALID_ARG, "null plan");
    if (enable && p->graph_refs > 0)
        return fail(KBN_ERR_UNSUPPORTED, "timing on a plan held by a captured batch");
    if (enable) {
        for (auto &t : p->pending) {
            p->pool.push_back(t.e0);
            p->pool.push_back(t.e1);
        }
        p->pending.clear();
        for (int c = 0; c < KBN_NCLASS; ++c) {
            p->t_ms[c] = 0.0;
            p->t_n[c] = 0;
        }
    }
    p->timing = enable != 0;
    return KBN_OK;
}

int kbn_timing_read(kbn_plan p, int cls, int64_t *launches, double *total_ms) {
    if (!p || cls < 0 || cls >= KBN_NCLASS) return fail(KBN_ERR_INVALID_ARG, "bad plan or class");
    for (auto &t : p->pending) {
        KBN_HIP(hipEventSynchronize(t.e1));
        float ms = 0.f;
        KBN_HIP(hipEventElapsedTime(&ms, t.e0, t.e1));
        p->t_ms[t.cls] += ms;
        p->t_n[t.cls] += 1;
        p->pool.push_back(t.e0);
        p->pool.push_back(t.e1);
    }
    p->pending.clear();
    if (launches) *launches = p->t_n[cls];
    if (total_ms) *total_ms = p->t_ms[cls];
    return KBN_OK;
}

const char *kbn_timing_name(int cls) {
    return (cls >= 0 && cls < KBN_NCLASS) ? kClassNames[cls] : nullptr;
}

const char *kbn_strerror(int code) {
    switch (code) {
        case KBN_OK: return "success";
        case KBN_ERR_INVALID_ARG: return "invalid argument";
        case KBN_ERR_UNSUPPORTED: return "unsupported size";
        case KBN_ERR_OOM: return "out of device memory";
        case KBN_ERR_HIP: return "HIP runtime error";
        case KBN_ERR_NONFINITE: return "non-finite sample location";
        case KBN_ERR_NO_POINTS: return "no sample locations set";
        default: return "unknown error";
    }
}

const char *kbn_last_error(void) { return g_err.c_str(); }

}  // extern "C"
