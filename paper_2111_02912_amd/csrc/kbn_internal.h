// Internal declarations of the KB-NUFFT library (device kernels + host plan).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "kbnufft.h"

#define KBN_MAX_D 3
#define KBN_MAX_J 8
#define KBN_NCOEF 11        // polynomial coefficients per window piece (degree 10)
#define KBN_MAX_STAGES 24
#define KBN_MAX_K 1024      // largest oversampled grid edge handled by the LDS FFT
#define KBN_MAX_TILES 40959 // tile histograms live in LDS (ntiles + 1 counters, at most 160 KiB)
#define KBN_BLOCK 256
#define KBN_INDEX_STREAM_MIN 8192  // points from which the index pass runs beside the caller's stream
#define KBN_SUB 256        // sorted points per gather subproblem (one per thread)
#define KBN_GATHER_WG_TARGET 2048  // workgroups a gather aims for (point blocks x channel groups)
#define KBN_SPREAD_EB 64   // list entries staged per spread batch
#define KBN_SPREAD_SEG 128  // list entries per spread work item (doubled if slots run out)
#define KBN_SPREAD_SMAX 256 // partial-tile slots for tiles split into several work items
#define KBN_GRID_Y_MAX 65535 // output-stationary spreads stride over work items beyond this many workgroup rows
#ifndef KBN_SPREAD_CL_WAVES
#define KBN_SPREAD_CL_WAVES 2 // waves per SIMD the channel-per-lane spread is compiled for
#endif
#ifndef KBN_SPREAD_CL_EB
#define KBN_SPREAD_CL_EB 16 // list entries staged per batch of the channel-per-lane spread
#endif
#define KBN_SPREAD_LDS (64 * 1024)  // LDS budget of one spread workgroup
#ifndef KBN_SPREAD_OS_U
#define KBN_SPREAD_OS_U 3   // entries per step of the 3D cell-per-lane spread's walk
#endif

// kernel classes reported by kbn_timing_read (order of kClassNames)
#define KBN_CLASS_INDEX 0
#define KBN_CLASS_FFT_FIRST 1
#define KBN_CLASS_FFT_MID_FWD 2
#define KBN_CLASS_FFT_MID_INV 3
#define KBN_CLASS_FFT_LAST_ADJ 4
#define KBN_CLASS_GATHER 5
#define KBN_CLASS_GATHER_JAC 6
#define KBN_CLASS_SPREAD 7
#define KBN_NCLASS 8

// Mixed-radix factorisation of one FFT length (radices 2, 3, 4, 5, 7, 8).
struct KbnRadix {
    int L;
    int nst;
    int r[KBN_MAX_STAGES];
};

// Geometry shared by the interpolation kernels (passed by value).
struct KbnGeom {
    int D;
    int J;
    int K[KBN_MAX_D];
    int T[KBN_MAX_D];
    int nt[KBN_MAX_D];
    int ntiles;
    int To[KBN_MAX_D];  // spread owner tile edge per axis
    int nto[KBN_MAX_D];
    int ntiles_own;
    const float *coef;  // [J][KBN_NCOEF] monomial coefficients in x = 2 f - 1
};

// ---------------------------------------------------------------------------
// Index pass (points.hip)
// ---------------------------------------------------------------------------
struct KbnPointsBufs {
    int *cell_tmp;   // [D][M] original order
    float *frac_tmp; // [D][M]
    int *tile;       // [M]
    int *counts;     // [nbins][nchunks], then the scan's span sums
    int *order;      // [M] sorted position -> original index
    int *cell;       // [D][M] sorted
    float *frac;     // [D][M] sorted
    int *toff;       // [nbins + 1]
    int *flag;       // sticky non-finite flag
    int *subs;       // [ceil(M / KBN_SUB) + nbins][2] (bin, first sorted position)
    int *nsub;       // number of subproblems
};

// Histogram chunks of the tile sort for M samples (returns their number and
// sets *chunk, the samples per chunk), and the element count of the plan's
// integer scratch buffer (count matrix and span sums, later the owner
// tiles' entry counts).
int kbn_points_chunks(int64_t M, int ntiles, int *chunk);
int64_t kbn_points_counts_size(int64_t M, int ntiles, int ntiles_own);
// offset in that buffer of the owner tiles' entry counts (cleared by the
// index pass)
int64_t kbn_points_owner_base(int64_t M, int ntiles);

// omega_read (may be null): recorded on s once omega has been read
hipError_t kbn_launch_points(int D, int64_t M, const float *omega, const double *scale,
                             const int *K, const int *T, const int *nt, int ntiles, int ntiles_own,
                             int sub, const KbnPointsBufs &b, hipStream_t s, hipEvent_t omega_read);

// Owner-tile lists for the spread, built from the tile-sorted samples:
// entry counts, offsets ooff[t] .. ooff[t+1], the tiles hottest first, the
// work items, and per entry the record (sorted position, caller-order index,
// tap origin relative to the tile, window fraction).  ocount: int scratch of
// ntiles_own elements, zero on entry.
hipError_t kbn_launch_owner_lists(const KbnGeom &g, int64_t M, const int *cell, const float *frac,
                                  const int *toff, const int *order, int *ocount, int *ooff,
                                  int *otile_order, int seg, int smax, int *swork, int *scomb, int *scounts,
                                  int *rec_p, int *rec_q, int *rec_l, float *rec_f, hipStream_t s);

// ---------------------------------------------------------------------------
// FFT passes (fft.hip)
// ---------------------------------------------------------------------------
struct KbnFirstPassArgs {      // forward: prologue + FFT along the last axis
    const float2 *x;           // [B][R0][Nl] images (batch offset applied)
    const float2 *smaps;       // [C][R0][Nl] or null
    float2 *out;               // [nch][R0][L]
    int64_t nlines;            // nch * R0
    int R0;                    // rows per image (product of leading N)
    int Nl;                    // last-axis image length
    int C, nw;                 // coils, weight channels per coil (1 or D)
    int weighted;              // 1: weight channel w multiplies by r^[w]
    int D;
    int N[KBN_MAX_D];
    const float *deap[KBN_MAX_D];
    // > 0: forward plus omega-Jacobian layout of nplain image-coil pairs.
    // Logical channels are the nplain unweighted ones, then for each pair
    // its weights w = 1..D-1 (nlines = nplain * D * R0); they are written
    // at output channels [nplain unweighted][nplain][D weights], leaving
    // every w = 0 slot for the axis-0 pass to derive (r^[0] is constant
    // along the lines of this pass).
    int64_t nplain = 0;
};

struct KbnMidPassArgs {        // FFT along a non-last axis, strided
    const float2 *in;
    float2 *out;
    int64_t outer;             // independent groups (channels x leading axes)
    int nin, nout;             // line length in / out (pruned or cropped)
    int inner;                 // product of the later axes' (grid) sizes
    int pad_in;                // 1: input rows sit at r mod L (zero-padded)
    int crop_out;              // 1: output rows are taken from r mod L
    // > 0 (forward axis-0 pass with pad_in, outer = channels only): output
    // channel dsplit + q with q % dnw == 0 is r^[0] times the unweighted
    // channel q / dnw, read from that channel's input with each image row
    // r scaled by r - nin / 2 (the other channels read their own input)
    int64_t dsplit = 0;
    int dnw = 1;
};

struct KbnLastAdjArgs {        // adjoint: IFFT along the last axis + crop + scale + coil sum
    const float2 *in;          // [nb*C][R0][L]
    const float2 *smaps;       // [C][R0][Nl] or null
    float2 *x;                 // [nb][R0][Nl] (batch offset applied)
    int64_t nlines;            // nb * R0
    int R0, Nl, C;
    int cmod;                  // > 0: C = 1 and line block bl takes coil map bl % cmod (one
                               // output image per image-coil pair, summed afterwards)
    int accumulate;
    int D;
    int N[KBN_MAX_D];
    const float *deap[KBN_MAX_D];
};

hipError_t kbn_launch_first_pass(const KbnFirstPassArgs &a, const KbnRadix &rp,
                                 const float2 *tw, int maxe, hipStream_t s);
hipError_t kbn_launch_mid_pass(const KbnMidPassArgs &a, const KbnRadix &rp, const float2 *tw,
                               int inverse, int maxe, hipStream_t s);
// x[b][j] (+)= sum_c ws[b * C + c][j] in coil order, j < npix
hipError_t kbn_launch_coil_sum(const float2 *ws, int64_t nb, int C, int64_t npix, float2 *x, int accumulate,
                               hipStream_t s);
hipError_t kbn_launch_last_adj(const KbnLastAdjArgs &a, const KbnRadix &rp, const float2 *tw,
                               int maxe, hipStream_t s);
int kbn_lines_per_block(const KbnRadix &rp, int maxe);

// Compile-time specialised passes (fft_fast.hip) for the lengths where
// kbn_fast_fft_size() is true; they return hipErrorInvalidValue otherwise.
bool kbn_fast_fft_size(int L);
// the specialised last adjoint pass exists for a subset of those lengths (it
// holds E accumulators besides the E values: above E = 32 it would spill)
bool kbn_fast_last_size(int L);
hipError_t kbn_launch_fast_first(const KbnFirstPassArgs &a, int L, const float2 *tw, hipStream_t s);
hipError_t kbn_launch_fast_mid(const KbnMidPassArgs &a, int L, const float2 *tw, int inverse,
                               hipStream_t s);
hipError_t kbn_launch_fast_last(const KbnLastAdjArgs &a, int L, const float2 *tw, hipStream_t s);

// ---------------------------------------------------------------------------
// Interpolation (interp.hip)
// ---------------------------------------------------------------------------
struct KbnGatherArgs {
    const float2 *grid;        // [nch][prod K]
    int64_t gsize;             // prod K
    int nch;                   // channels in this chunk
    int C, nw;                 // channel = (b_local * C + c) * nw + w
    int64_t M;
    const int *order;
    const int *cell;
    const float *frac;
    const int *toff;           // toff[ntiles] = end of finite points
    const int *subs;           // gather subproblems [n][2] (tile, first sorted position)
    const int *nsub;
    float2 *y;                 // mode 0: [B][C][M] with batch offset applied
    const float2 *v;           // mode 1: [B][C][M] with batch offset applied
    float *domega;             // mode 1: [M][D]
    float *part;               // mode 1: [groups][M][D] per-group partial gradients
    int accumulate;            // mode 1: add the reduced gradient onto domega
};

struct KbnGatherShape {
    bool staged;
    int cp;                    // channels interpolated per pass (staged)
    size_t lds;
    int64_t blocks;
    int cg, groups;
};
// Nominal channel groups of a gather over nbc channel sets in `blocks`
// point blocks: never more than nbc, and never fewer for a larger nbc, so
// that it bounds the groups of every smaller chunk as well.
int64_t kbn_gather_groups(int64_t blocks, int64_t nbc);
KbnGatherShape kbn_gather_shape(const KbnGeom &g, int64_t M, int nch, int nw);

struct KbnSpreadArgs {
    const float2 *y;           // [nb][C][M] batch offset applied
    float2 *ys;                // [nb*C][M] workspace: y in sorted order
    float2 *grid;              // [nch][prod K], nch = nb * C
    int64_t gsize;
    int nch;
    int64_t M;
    const int *order;
    const int *cell;
    const float *frac;
    const int *toff;
    const int *otile_order;    // owner tiles by decreasing entry count (coarse)
    const int *swork;          // work items [n][4]: tile, entry begin, entry end, slot (-1: direct)
    const int *scomb;          // multi-item tiles [n][3]: tile, first slot, slots
    const int *scounts;        // [0] work items, [1] multi-item tiles
    float2 *partial;           // [smax][nch][prod To] partial tiles of multi-item tiles
    const int *rec_p;          // per owner-list entry: sorted sample position
    const int *rec_q;          // per owner-list entry: the sample's index in the caller's order
    const int *rec_l;          // [entries][D] tap origin relative to the owning tile
    const float *rec_f;        // [entries][D] window fraction
    int nwork_max, ncomb_max;
};

hipError_t kbn_launch_gather(const KbnGeom &g, const KbnGatherArgs &a, int mode, hipStream_t s);
hipError_t kbn_launch_spread(const KbnGeom &g, const KbnSpreadArgs &a, hipStream_t s);

// Interpolation of several plans in one launch (the batch's fused phases).
// A job is one plan's call: its geometry and arguments as the single-call
// launch takes them, copied to device memory by the caller.
struct KbnGatherJob {
    KbnGeom g;
    KbnGatherArgs a;
    int cg;      // channels per group (kbn_gather_shape)
    int blocks;  // subproblem workgroups per channel group
};
// staged gathers of jobs that share D and J; start[i] = first workgroup of
// job i (blocks x groups each), start[njobs] = total; lds = the largest
// job's region bytes.  Mode 1 leaves each job's epilogue to
// kbn_launch_gather_reduce.
hipError_t kbn_launch_gather_multi(int D, int J, int mode, const KbnGatherJob *jobs, const int64_t *start, int njobs,
                                   int64_t total, size_t lds, hipStream_t s);
hipError_t kbn_launch_gather_reduce(const KbnGeom &g, const KbnGatherArgs &a, hipStream_t s);

#define KBN_SPREAD_PATH_GENERIC 0
#define KBN_SPREAD_PATH_OS 1
#define KBN_SPREAD_PATH_CL 2
struct KbnSpreadSel {
    int path = KBN_SPREAD_PATH_GENERIC;
    int cpt = 0, ebv = 0, tcells = 0;  // output-stationary: channels per thread, entries per batch, cells
    size_t lds = 0;                    // its dynamic LDS
    int ngr = 0, ny = 0;               // its grid: channel groups x work-item rows
};
KbnSpreadSel kbn_spread_select(const KbnGeom &g, const KbnSpreadArgs &a);
struct KbnSpreadJob {
    KbnGeom g;
    KbnSpreadArgs a;
    int ngr;  // channel groups
    int ny;   // workgroup rows striding over the work items
};
// output-stationary spreads of jobs whose kbn_spread_select agree on D, J,
// cpt, ebv and the owner tile (so one workgroup size); ystart[i] = first
// row of job i, grid maxngr x total_y.  Each job's split tiles are then
// summed by kbn_launch_spread_combine.
hipError_t kbn_launch_spread_os_multi(const KbnSpreadSel &sel, int D, int J, int maxngr, const KbnSpreadJob *jobs,
                                      const int *ystart, int njobs, int total_y, hipStream_t s);
hipError_t kbn_launch_spread_combine(const KbnSpreadSel &sel, const KbnGeom &g, const KbnSpreadArgs &a,
                                     hipStream_t s);

// ---------------------------------------------------------------------------
// Plan hooks used by the batch executor (plan.cpp)
// ---------------------------------------------------------------------------
bool kbn_internal_timing_on(kbn_plan p);
void kbn_internal_graph_ref(kbn_plan p, int delta);  // captured graphs holding p
int kbn_internal_fail(int code, const char *msg);    // sets the thread's last error
// estimated bytes moved by one call (jac: D channels per coil; type1: adjoint type)
double kbn_internal_cost(kbn_plan p, int B, int C, int jac, int type1);
uint64_t kbn_internal_epoch(kbn_plan p);  // changes with every kbn_set_points
// order `s` after the plan's last index pass (which runs on its own stream)
int kbn_internal_points_wait(kbn_plan p, hipStream_t s);
// note a finished index pass (before a capture, whose waits cannot name it)
void kbn_internal_points_settle(kbn_plan p);
// device memory through the plan's allocator, counted in its footprint
int kbn_internal_alloc(kbn_plan p, void **ptr, int64_t bytes, hipStream_t s);
void kbn_internal_free(kbn_plan p, void *ptr, hipStream_t s);

// One batch task split into phases around its interpolation (the batch's
// fused mode): kind 0 = forward-type (gather), 1 = omega-Jacobian (gather
// with the gradient epilogue), 2 = adjoint-type (spread), -1 = issued whole.
struct KbnPhased {
    kbn_plan p = nullptr;
    int op = 0, kind = -1;
    int B = 0, C = 0, nw = 1, weighted = 0, accumulate = 0;
    const float2 *x = nullptr, *smaps = nullptr, *v = nullptr, *ky = nullptr;
    float2 *y = nullptr, *img = nullptr;
    float *dom = nullptr;
    char *ws = nullptr;  // the task's own grids (and gradient parts / k-space copy / partial tiles)
    float2 *bufA = nullptr, *bufB = nullptr;
    KbnGatherJob gj;     // kinds 0, 1
    int groups = 0;
    size_t lds = 0;
    KbnSpreadJob sj;     // kind 2
    KbnSpreadSel sel;
};
int kbn_internal_phase_prepare(const kbn_task &t, KbnPhased *ph, hipStream_t s);
int kbn_internal_phase_pre(KbnPhased *ph, hipStream_t s);
int kbn_internal_phase_post(KbnPhased *ph, hipStream_t s);
void kbn_internal_phase_release(KbnPhased *ph, hipStream_t s);

// ---------------------------------------------------------------------------
// CG-SENSE vector kernels (cg.hip)
// ---------------------------------------------------------------------------
// scalar slots (doubles) at the start of a CG work buffer
#define KBN_CG_RR 0
#define KBN_CG_BB 1
#define KBN_CG_PQ 2
#define KBN_CG_ALPHA 3
#define KBN_CG_BETA 4
#define KBN_CG_REL 5
#define KBN_CG_ITERS 6
#define KBN_CG_NSCAL 32
#define KBN_CG_MAXPARTS 1024
// kernel groups of one CG step
#define KBN_CGK_INIT 0  // x = 0, p = r, rr = bb = |r|^2
#define KBN_CGK_Q 1     // q += lambda T^H T p, alpha = rr / <p, q>
#define KBN_CGK_XR 2    // x += alpha p, r -= alpha q, beta, rr, rel
#define KBN_CGK_P 3     // p = r + beta p
int kbn_cg_nparts(int64_t n);

// ---------------------------------------------------------------------------
// Off-resonance model kernels (field.hip): virtual coil maps c_l s_k
// (v = l*C + k), k-space expansion by conj(b_l) and combination by b_l, and
// linear-interpolation time segmentation
// ---------------------------------------------------------------------------
hipError_t kbn_launch_field_maps(int L, int C, int64_t npix, const float2 *c, const float2 *smaps,
                                 float2 *vm, hipStream_t s);
hipError_t kbn_launch_field_expand(int64_t nb, int L, int C, int64_t M, const float2 *bw,
                                   const float2 *y, float2 *ye, hipStream_t s);
hipError_t kbn_launch_field_combine(int64_t nb, int L, int C, int64_t M, const float2 *bw,
                                    const float2 *ye, float2 *y, hipStream_t s);
hipError_t kbn_launch_field_segments(int64_t M, const float *t, double t0, double t1, int64_t npix,
                                     const float *w, int L, float2 *bw, float2 *c, hipStream_t s);
// image extent for the regulariser stencil, unused axes 1 (row-major, n0 slowest)
struct KbnCgImage {
    int reg;  // KBN_REG_IDENTITY or KBN_REG_FINITE_DIFF
    int n0, n1, n2;
};
#define KBN_CG_MAXB 65535  // images per CG launch (grid rows)
hipError_t kbn_launch_cg(int kind, int nimg, int64_t n, float2 *x, float2 *r, float2 *p, float2 *q,
                         float lam, KbnCgImage img, double *scal, double *part, hipStream_t s);
