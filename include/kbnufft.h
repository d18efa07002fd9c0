/*
 * kbnufft.h -- C ABI of the MI355X Kaiser-Bessel NUFFT library.
 *
 * Operation (Wang & Fessler, "Efficient approximation of Jacobian matrices
 * involving a non-uniform fast Fourier transform", Sec. II-B eq. (e,ndft)):
 *
 *     A(omega) in C^{M x N},  a_ij = exp(-i omega_i . r_j),
 *
 * for M sample locations omega (an M x D real matrix, radians per voxel) and
 * voxel centres r_j on a D-dimensional Cartesian grid.  The library applies
 * a Kaiser-Bessel NUFFT approximation of A and A^H (appendix: scaling
 * factors, zero-padded K-point FFT, J-tap interpolation), and the paper's
 * Jacobians with respect to omega, evaluated as extra NUFFTs of images
 * weighted by the coordinate grids r^[d] (Sec. II-C eq. (e,Ax), Sec. II-D
 * eq. (e,A'y), JVP rule eq. (e,jac,Ax,v) of Sec. III), for the multi-coil
 * SENSE model E = (I_C kron A) S of Sec. II-G.
 *
 * Conventions (all binding):
 *   - D in {1, 2, 3}.  Images are row-major, axis 0 slowest; the coordinate
 *     of index j on an axis of length n is r = j - floor(n/2).
 *   - omega is float32 [M][D], row-major; column d pairs with image axis d.
 *     Any finite value is accepted (the operator is 2 pi-periodic in omega).
 *   - complex data are interleaved float32 pairs (re, im) ("c64"):
 *       images  x      c64 [B][N_0]...[N_{D-1}]
 *       maps    smaps  c64 [C][N_0]...[N_{D-1}]   (NULL: C must be 1, S = I)
 *       k-space y      c64 [B][C][M]
 *   - forward uses exp(-i ...), adjoint exp(+i ...), no normalisation.
 *   - gradients follow PyTorch's convention for complex tensors: the
 *     gradient of a real loss L w.r.t. z is dL/dRe z + i dL/dIm z.
 *   - Every data pointer is a DEVICE pointer (HIP device memory) unless the
 *     argument says "host".  The caller owns all input and output buffers;
 *     the plan owns its internal buffers (allocated through the plan's
 *     allocator).
 *   - Every call is asynchronous on `stream` (a hipStream_t, NULL = the
 *     null stream) and never synchronises it, except kbn_check_error.
 *     Device memory of a plan comes from the caller's kbn_allocator (or
 *     HIP's stream-ordered allocator) and is allocated and released in
 *     stream order.
 *   - A plan is not thread-safe: calls on one plan must be ordered (one
 *     stream, or the caller's synchronisation).  Distinct plans are
 *     independent.
 *   - Calls return 0 on success or a negative KBN_ERR_* code; they never
 *     throw and never abort.  kbn_last_error() gives a message for the last
 *     failing call of the calling thread.
 */
#ifndef KBNUFFT_H
#define KBNUFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KBN_OK 0
#define KBN_ERR_INVALID_ARG (-1)     /* bad pointer, size, dimension or option */
#define KBN_ERR_UNSUPPORTED (-2)     /* valid request outside supported sizes  */
#define KBN_ERR_OOM (-3)             /* device allocation failed                */
#define KBN_ERR_HIP (-4)             /* a HIP runtime call or launch failed      */
#define KBN_ERR_NONFINITE (-5)       /* some omega was non-finite or too large  */
#define KBN_ERR_NO_POINTS (-6)       /* operator call before kbn_set_points     */

#define KBN_OP_FORWARD 0             /* the operator y = E x                    */
#define KBN_OP_ADJOINT 1             /* the operator x = E^H y                  */
#define KBN_REG_IDENTITY 0           /* CG regulariser T = I (CG-SENSE)         */
#define KBN_REG_FINITE_DIFF 1        /* T = first differences per axis (QPLS)   */

typedef struct kbn_plan_s *kbn_plan;

/* Plan options.  Zero-initialised fields take the defaults shown. */
typedef struct {
    double sigma;            /* grid oversampling factor, >= 1 (default 2.0)        */
    int J;                   /* window width in grid cells, 2..8 (default 6)        */
    int tile[3];             /* tile edge per axis for sorting the points and for
                                the interpolation subproblems
                                (0 = automatic: 1D 256, 2D 32, 3D 8, grown until
                                the tile count fits)                                 */
    int64_t max_workspace;   /* byte cap for the plan's grid workspace; batches
                                larger than fits are processed in chunks
                                (0 = 4 GiB)                                          */
    int spread_tile;         /* edge of the grid tiles that one spreading work
                                group owns, >= J (0 = automatic: 1D 128, 2D 8,
                                3D 8; grown until the tile count fits)               */
} kbn_opts;

/*
 * Device memory of a plan.  The plan allocates every internal buffer
 * (constants, sorted points, owner lists, grid workspace) through this
 * interface and frees each through it, stream-ordered: alloc(ctx, bytes,
 * stream) returns a block usable by work issued to `stream` after the call
 * (NULL on failure: the library call then fails with KBN_ERR_OOM and leaves
 * no partial plan); free(ctx, ptr, stream) may run before work queued on
 * `stream` has finished, so the allocator must not hand the block out again
 * until that work is done (PyTorch's caching allocator with record_stream
 * does this).  Blocks are multiples of 256 bytes.  ctx is passed through.
 * Not an operation of the paper: it lets the caller's framework (PyTorch in
 * the Python binding) own all device memory.
 */
typedef struct {
    void *ctx;
    void *(*alloc)(void *ctx, size_t bytes, void *stream);
    void (*free)(void *ctx, void *ptr, void *stream);
} kbn_allocator;

/*
 * Create a plan for images of shape N (host int64[D]).
 *
 * Chooses per axis K_d = smallest integer >= sigma N_d whose prime factors
 * are 2, 3, 5, 7 (appendix: "K-point FFT ... via zero-padding"), the window
 * psi(t) = I0(beta sqrt(1 - (2t/J)^2)) / I0(beta) with the Beatty et al.
 * beta = pi sqrt((J/sigma)^2 (sigma - 1/2)^2 - 0.8) (the paper defers the
 * window to its NUFFT library), scaling factors s_n = 1/psi_hat(r_n/K_d)
 * (appendix "scaling factors s_n"), and FFT twiddles, all in FP64 on the
 * host, and uploads them asynchronously on `stream` (the plan keeps the host
 * copies until the uploads have run).  Does not synchronise.
 *
 * alloc: the allocator for every device buffer of the plan (copied; its
 * functions must stay valid until kbn_plan_destroy returns), or NULL for
 * HIP's stream-ordered allocator (hipMallocAsync / hipFreeAsync).
 * Allocations happen on the stream of the call that needs them (creation,
 * kbn_set_points, a workspace growth in an operator call).
 *
 * The grid workspace is allocated on first use and grown when a larger
 * batch arrives; the old block is released stream-ordered on the call's
 * stream.  Calls on one plan must be ordered: successive calls on
 * different streams need the caller's synchronisation between them.
 *
 * Errors: INVALID_ARG (out == NULL, D not in 1..3, N_d < 1, sigma < 1,
 * J outside 2..8, an allocator without alloc or free), UNSUPPORTED
 * (K_d > 1024 or K_d < 2J), OOM, HIP.
 */
int kbn_plan_create(kbn_plan *out, int D, const int64_t *N, const kbn_opts *opts,
                    const kbn_allocator *alloc, void *stream);

/*
 * Device bytes a plan would hold (host-only computation, no HIP call): its
 * constants, the index-pass buffers for M points, and the grid workspace of
 * forward and adjoint calls with B images of C coils (and of the
 * omega-Jacobian with jac != 0) under opts->max_workspace.  Equal to
 * kbn_plan_info's device_bytes after kbn_set_points(M) and those calls.
 * The off-resonance workspace and that of kbn_forward_jac_omega (D + 1
 * grids per image-coil pair) are not included.  For admission control.
 * Errors: INVALID_ARG (null bytes, M < 0 or too large, B < 1, C < 1, and the
 * option errors of kbn_plan_create), UNSUPPORTED.
 */
int kbn_plan_footprint(int D, const int64_t *N, const kbn_opts *opts, int64_t M, int B, int C,
                       int jac, int64_t *bytes);

/*
 * Set (or replace) the M sample locations.  omega: device float32 [M][D].
 *
 * Computes, per point and axis, u = omega K_d / (2 pi) in FP64, the grid
 * cell floor(u) mod K_d and the in-cell fraction (float32), the tile id, and
 * a stable order of the points by tile (the appendix's offsets k_m and J
 * taps k_m + j are derived from these).  M = 0 is allowed.
 *
 * From 8192 points the pass runs on a stream of the plan's own (smaller
 * passes run on `stream`), after the work already queued on `stream`;
 * `stream` waits only until omega has been read (the
 * caller may then overwrite it), so a following call's FFT passes run beside
 * the rest of the pass.  Every later read of the points (interpolation,
 * kbn_get_points, kbn_check_error, a batch) waits for the pass on its own
 * stream.  A call made under HIP graph capture cannot wait for it: capture
 * calls of the plan only after kbn_check_error (kbn_batch_capture does this
 * itself), else they return UNSUPPORTED while the pass may still run.
 *
 * A non-finite omega (or |u| >= 2^40) sets a sticky device flag reported by
 * kbn_check_error; such points give NaN in forward outputs and omega
 * gradients and contribute nothing to adjoint outputs.
 *
 * Buffers for the points are allocated (or grown) stream-ordered on
 * `stream`; the old ones are released the same way.
 *
 * Errors: INVALID_ARG (M < 0, M > (2^31 - 1) / 2^D -- the spread's owner
 * lists index up to 2^D entries per point with 32-bit positions --, omega ==
 * NULL with M > 0), OOM, HIP.
 */
int kbn_set_points(kbn_plan p, int64_t M, const float *omega, void *stream);

/*
 * y[b][c] = A(omega) (s_c (.) x_b)   (type-2 NUFFT; Sec. II-B, II-G).
 * x: c64 [B][N...]; smaps: c64 [C][N...] or NULL (then C == 1);
 * y: c64 [B][C][M], overwritten.
 * Errors: INVALID_ARG (B < 1, C < 1, NULL pointers, smaps NULL with C > 1),
 * NO_POINTS, OOM, HIP.
 */
int kbn_forward(kbn_plan p, int B, int C, const void *x, const void *smaps, void *y,
                void *stream);

/*
 * kbn_forward for callers that cannot allocate device memory: code under HIP
 * graph capture, serving loops that must not allocate, harnesses that
 * forbid allocation.  Same operation, arguments and results as kbn_forward
 * (bit for bit), but the grid workspace is a library-owned static device
 * array of KBN_STATIC_WORKSPACE bytes on each GPU (held from library load
 * to process end) instead of the plan's workspace, so the call allocates
 * nothing and never grows the plan; batches are processed in chunks that
 * fit it.  All calls on one GPU share that array: calls that overlap on a
 * GPU (other streams, other threads, other plans) race and must be
 * serialised by the caller.  The plan must have been created and its points
 * set beforehand (those calls allocate).
 * Errors: as kbn_forward; UNSUPPORTED when one image-coil pair needs more
 * than KBN_STATIC_WORKSPACE bytes (2 x 8 x prod K bytes) or timing is on;
 * HIP if the array's address cannot be obtained.
 */
#define KBN_STATIC_WORKSPACE 67108864
int kbn_forward_static(kbn_plan p, int B, int C, const void *x, const void *smaps, void *y,
                       void *stream);

/*
 * x_b = sum_c conj(s_c) (.) A(omega)^H y[b][c]   (type-1 NUFFT; Sec. II-D,
 * II-G).  y: c64 [B][C][M]; x: c64 [B][N...], overwritten.
 * Errors as kbn_forward.
 */
int kbn_adjoint(kbn_plan p, int B, int C, const void *y, const void *smaps, void *x,
                void *stream);

/*
 * Gradient of a real loss w.r.t. omega through y = E(omega) x, given the
 * upstream gradient g = dL/dy (c64 [B][C][M]):
 *
 *   domega[m][d] (+)= sum_{b,c} Im{ [A(s_c x_b (.) r^[d])]_m conj(g[b][c][m]) }
 *
 * which is eq. (e,Ax), dA x / d omega^[d] = -i diag{A (x (.) r^[d])}, applied
 * through the JVP rule eq. (e,jac,Ax,v) with the NUFFT standing in for A.
 * domega: device float32 [M][D]; accumulate = 0 overwrites it, 1 adds.
 * Errors as kbn_forward.
 */
int kbn_jac_omega_fwd(kbn_plan p, int B, int C, const void *x, const void *smaps,
                      const void *g, float *domega, int accumulate, void *stream);

/*
 * kbn_forward and kbn_jac_omega_fwd of the same images in one call, for an
 * upstream gradient g that is known before y (Sec. II-C and eq. (e,Ax)):
 *
 *   y[b][c] = A(omega) (s_c (.) x_b)          (overwritten)
 *   domega[m][d] (+)= sum_{b,c} Im{ [A(s_c x_b (.) r^[d])]_m conj(g[b][c][m]) }
 *
 * In 2D the weight r^[0] is constant along the lines of the first FFT pass,
 * so that channel is not transformed on its own there: the axis-0 pass
 * derives it from the unweighted channel, one grid-row write and read less
 * per image-coil pair than the two separate calls.  y equals kbn_forward's
 * bit for bit; domega agrees with kbn_jac_omega_fwd to float32 rounding
 * (the r^[0] scaling is applied after the first pass instead of before).
 * Other dimensions and FFT lengths run the two calls.  x: c64 [B][N...];
 * y, g: c64 [B][C][M] (y and g must not overlap); domega: device float32
 * [M][D]; accumulate = 0 overwrites domega, 1 adds.  The workspace holds
 * D + 1 grids per image-coil pair (kbn_plan_footprint does not count it).
 * Errors as kbn_forward, plus INVALID_ARG for a null domega.
 */
int kbn_forward_jac_omega(kbn_plan p, int B, int C, const void *x, const void *smaps, void *y,
                          const void *g, float *domega, int accumulate, void *stream);

/*
 * Gradient of a real loss w.r.t. omega through x = E(omega)^H y, given the
 * upstream gradient g = dL/dx (c64 [B][N...]):
 *
 *   domega[m][d] (+)= sum_{b,c} Im{ [A(s_c g_b (.) r^[d])]_m conj(y[b][c][m]) }
 *
 * the transpose of eq. (e,A'y), dA^H y / d omega^[d] = i diag{r^[d]} A^H
 * diag{y}, applied to g.  y: c64 [B][C][M].  Errors as kbn_forward.
 */
int kbn_jac_omega_adj(kbn_plan p, int B, int C, const void *y, const void *smaps,
                      const void *g, float *domega, int accumulate, void *stream);

/*
 * Gradient w.r.t. the linear input (Sec. II-C: dAx/dx = A; Sec. II-D:
 * dA^H y/dy = A^H):
 *   op = KBN_OP_FORWARD: out = E^H g, g c64 [B][C][M], out c64 [B][N...];
 *   op = KBN_OP_ADJOINT: out = E g,   g c64 [B][N...], out c64 [B][C][M].
 * Errors as kbn_forward, plus INVALID_ARG for an unknown op.
 */
int kbn_jac_x(kbn_plan p, int op, int B, int C, const void *g, const void *smaps,
              void *out, void *stream);

/*
 * Plan facts (host outputs; any pointer may be NULL):
 *   K       int64[D]  oversampled grid size per axis
 *   tile    int[D]    tile edge per axis; ntiles total tile count
 *   beta    window shape parameter
 *   M       current number of points (0 before kbn_set_points)
 *   workspace_bytes  currently allocated grid workspace
 *   device_bytes     all device memory the plan holds now (constants,
 *                    points, owner lists, workspaces)
 */
int kbn_plan_info(kbn_plan p, int64_t *K, int *tile, int *ntiles, double *beta,
                  int64_t *M, int64_t *workspace_bytes, int64_t *device_bytes);

/*
 * Copy the index pass results into caller device buffers (for testing and
 * inspection; any pointer may be NULL):
 *   order   int32 [M]          original index of the point at sorted position q
 *   cell    int32 [D][M]       grid cell floor(u) mod K_d, in sorted order
 *   frac    float32 [D][M]     u - floor(u) rounded to float32, sorted order
 *   offsets int32 [ntiles + 2] first sorted position of each tile; entry
 *                              ntiles is the end of the finite points, entry
 *                              ntiles + 1 is M (flagged points sort last)
 * Asynchronous on stream.
 */
int kbn_get_points(kbn_plan p, int *order, int *cell, float *frac, int *offsets,
                   void *stream);

/*
 * Synchronise `stream` and report the sticky non-finite-omega flag:
 * returns KBN_ERR_NONFINITE (and clears the flag) if any omega given to
 * kbn_set_points since the last check was non-finite, else 0 (or HIP).
 */
int kbn_check_error(kbn_plan p, void *stream);

/*
 * Per-kernel timing, for measurement (not part of the operator).
 *
 * kbn_timing(p, 1) clears the counters and starts bracketing every kernel
 * launch of the plan with HIP events recorded on the launch's own stream;
 * kbn_timing(p, 0) stops recording.  kbn_timing_read waits for the recorded
 * events and returns, for kernel class `cls`, the number of timed launches
 * and their summed durations in milliseconds.  kbn_timing_name gives the
 * class name ("index", "fft_first", "fft_mid_fwd", "fft_mid_inv",
 * "fft_last_adj", "gather", "gather_jac", "spread"), or NULL for cls past
 * the last class.
 * Errors: INVALID_ARG (null plan, bad class), HIP.
 */
int kbn_timing(kbn_plan p, int enable);

/*
 * Restrict the timing events to the kernel classes whose bit is set in
 * `mask` (bit c for class c; all classes after kbn_plan_create), so that a
 * measurement brackets only the kernels it reports and the events of the
 * others do not add to the time being measured.  Takes effect for later
 * launches.  Errors: INVALID_ARG (null plan).
 */
int kbn_timing_select(kbn_plan p, unsigned int mask);
int kbn_timing_read(kbn_plan p, int cls, int64_t *launches, double *total_ms);
const char *kbn_timing_name(int cls);

/* Free the plan: its device buffers are released stream-ordered on `stream`
 * (which must be ordered after the plan's last work, e.g. the stream of its
 * last call), through the plan's allocator.  Does not synchronise (it waits
 * only if the creation's constant uploads have not run yet).
 * Errors: INVALID_ARG (null plan, or a captured batch still holds it). */
int kbn_plan_destroy(kbn_plan p, void *stream);

/*
 * CG-SENSE / QPLS reconstruction (Sec. IV-B: the quadratic reconstruction
 * x = (E^H E + lambda T^H T)^{-1} E^H y solved by conjugate gradients;
 * residual ||r|| / ||b|| as in Sec. IV-A), for B independent images with
 * C coils each, solved together: every iteration applies E^H E to all B
 * images in one forward and one adjoint call, and each image keeps its own
 * CG scalars.
 * reg selects T: KBN_REG_IDENTITY (T = I, CG-SENSE) or KBN_REG_FINITE_DIFF
 * (QPLS: T stacks the first differences (T_d x)_j = x_{j+e_d} - x_j along
 * every image axis d, for j_d < N_d - 1; no wrap-around at the edges).
 *
 * Plain CG from x0 = 0 (Shewchuk): r = b = E^H y, p = r; per iteration
 * q = E^H E p + lambda T^H T p, alpha = r'r / p'q, x += alpha p, r -= alpha q,
 * beta = r'r(new) / r'r(old), p = r + beta p.  Exactly `iters` iterations
 * (no early stop); if p'q or r'r is not positive the step is zero.  Image
 * vectors and arithmetic are FP32; inner products are summed in FP64 with
 * a fixed reduction order, and the scalars stay on the device, so a solve
 * needs no host synchronisation and its result does not depend on other
 * work running on the GPU.
 *
 * work: a caller-owned device buffer of kbn_cg_work_bytes(p, B, C) bytes
 * holding the solver state between calls; it starts with 32 doubles per
 * image (image b at doubles 32 b ..):
 *   [0] r'r  [1] b'b  [2] p'q  [3] alpha  [4] beta
 *   [5] ||r|| / ||b|| (0 if b = 0)  [6] iterations done
 * kbn_cg_begin sets x = 0 and the state for y; kbn_cg_step runs `iters`
 * more iterations (calls may be split, e.g. one iteration at a time; B and
 * C must stay those of the begin call).
 * x: c64 [B][N..]; y: c64 [B][C][M]; smaps: c64 [C][N..] or NULL (C = 1).
 * The same plan's points must stay set between begin and the last step.
 * Errors: INVALID_ARG (null pointers, B outside 1..65535, C < 1, iters < 0,
 * lambda < 0 or not finite, unknown reg), NO_POINTS, OOM/HIP (workspace
 * growth, launches).
 */
int kbn_cg_work_bytes(kbn_plan p, int B, int C, int64_t *bytes);
int kbn_cg_begin(kbn_plan p, int B, int C, const void *smaps, const void *y, void *x, void *work,
                 void *stream);
int kbn_cg_step(kbn_plan p, int B, int C, const void *smaps, double lambda, int reg, int iters,
                void *x, void *work, void *stream);

/*
 * Start a solve of (E^H E + lambda T^H T) x = b for image right-hand sides b
 * (c64 [B][N..], device) instead of b = E^H y: x = 0, r = p = b.  Used to
 * apply the regularised inverse of Sec. II-F to images (and to their
 * upstream gradients).  Continue with kbn_cg_step.  Errors as kbn_cg_begin.
 */
int kbn_cg_begin_image(kbn_plan p, int B, int C, const void *b, void *x, void *work,
                       void *stream);

/*
 * Off-resonance (field inhomogeneity) model, Sec. II-H.  The exact system
 * matrix a_ij = exp(-i omega_i . r_j) exp(-i w_j t_i) is approximated by
 *   E_f = sum_l diag(b_l) A(omega) diag(c_l),   b_l in C^M, c_l in C^N,
 * and with coil maps E = sum_l diag(b_l) (I_C kron A) diag(c_l) S.  The
 * Jacobians follow by putting E_f in place of A (b and c do not depend on
 * omega).
 *   b: c64 [L][M] k-space weights;  c: c64 [L][N..] image-domain factors
 *   (device, caller-owned); x, y, smaps, g, domega as for the plain calls.
 * kbn_field_forward:        y[b][k] = sum_l b_l (.) A(c_l s_k x_b)
 * kbn_field_adjoint:        x_b = sum_{l,k} conj(c_l s_k) (.) A^H(conj(b_l) (.) y[b][k])
 * kbn_field_jac_omega_fwd:  dL/domega for y = E x, upstream g [B][C][M]
 *                           = sum_{b,k,l} Im{ b_l A(c_l s_k x_b (.) r^[d]) conj(g_{b,k}) }
 * kbn_field_jac_omega_adj:  dL/domega for x = E^H y, upstream g [B][N..]
 *                           = sum_{b,k,l} Im{ A(c_l s_k g_b (.) r^[d]) b_l conj(y_{b,k}) }
 * The x-gradients are the other operator: E^H g (forward) and E g (adjoint).
 * The plan keeps a second workspace for the L*C virtual coil maps c_l s_k
 * and the k-space of L*C virtual coils for a chunk of images (chunked to
 * stay under max_workspace); it grows on demand like the grid workspace.
 * Errors: as the plain calls, and INVALID_ARG for L < 1 or null b / c.
 */
int kbn_field_forward(kbn_plan p, int B, int C, int L, const void *x, const void *smaps,
                      const void *b, const void *c, void *y, void *stream);
int kbn_field_adjoint(kbn_plan p, int B, int C, int L, const void *y, const void *smaps,
                      const void *b, const void *c, void *x, void *stream);
int kbn_field_jac_omega_fwd(kbn_plan p, int B, int C, int L, const void *x, const void *smaps,
                            const void *b, const void *c, const void *g, float *domega,
                            int accumulate, void *stream);
int kbn_field_jac_omega_adj(kbn_plan p, int B, int C, int L, const void *y, const void *smaps,
                            const void *b, const void *c, const void *g, float *domega,
                            int accumulate, void *stream);

/*
 * Linear-interpolation time segmentation for the model above (the paper
 * leaves the choice of b and c to the approximation methods it cites):
 * segment times tau_l = t0 + (t1 - t0) l / (L - 1) (the midpoint when
 * L = 1), c_lj = exp(-i w_j tau_l), and b_il the linear interpolation
 * weights of t_i between its two neighbouring tau_l (t_i clamped to
 * [t0, t1]; sum_l b_il = 1).
 *   t: float [M] readout times (s);  w: float [npix] field map (rad/s);
 *   b: c64 [L][M] out;  c: c64 [L][npix] out   (device pointers)
 * Errors: INVALID_ARG (M < 0, npix < 1, L < 1, t0/t1 not finite or t1 < t0,
 * null pointers), HIP.
 */
int kbn_field_segments(int64_t M, const float *t, double t0, double t1, int64_t npix,
                       const float *w, int L, void *b, void *c, void *stream);

/*
 * Batches: many independent operator calls issued together.
 *
 * Not an operation of the paper; an executor for running many SENSE
 * problems of different shapes (training on several trajectories or
 * image sizes, serving) without per-call host overhead.  A task is one
 * of the single-plan calls above with its arguments:
 *
 *   op                    a            g          out
 *   KBN_TASK_FORWARD      x            -          y        (kbn_forward)
 *   KBN_TASK_ADJOINT      y            -          x        (kbn_adjoint)
 *   KBN_TASK_JAC_OMEGA_FWD x           g [B][C][M] domega  (kbn_jac_omega_fwd)
 *   KBN_TASK_JAC_OMEGA_ADJ y           g [B][N..]  domega  (kbn_jac_omega_adj)
 *   KBN_TASK_JAC_X_FWD    g [B][C][M]  -          E^H g    (kbn_jac_x, FORWARD)
 *   KBN_TASK_JAC_X_ADJ    g [B][N..]   -          E g      (kbn_jac_x, ADJOINT)
 *
 * Tasks of one plan run in list order on one stream (they share the
 * plan's workspace); tasks of different plans must be independent (no
 * task may read another plan's task output) and run concurrently on the
 * batch's own streams: each plan's chain goes to the stream with the
 * least estimated traffic so far, largest chains first.
 */
#define KBN_TASK_FORWARD 0
#define KBN_TASK_ADJOINT 1
#define KBN_TASK_JAC_OMEGA_FWD 2
#define KBN_TASK_JAC_OMEGA_ADJ 3
#define KBN_TASK_JAC_X_FWD 4
#define KBN_TASK_JAC_X_ADJ 5

typedef struct {
    kbn_plan plan;
    int op;                  /* KBN_TASK_*                                          */
    int B, C;                /* images and coils, as for the single call            */
    const void *a;           /* first data argument (table above), device           */
    const void *smaps;       /* c64 [C][N..] or NULL                                */
    const void *g;           /* upstream gradient of the JAC_OMEGA tasks, else NULL */
    void *out;               /* output, device                                      */
    int accumulate;          /* JAC_OMEGA tasks: add onto out                       */
} kbn_task;

typedef struct kbn_batch_s *kbn_batch;

/*
 * Create a batch of `ntasks` tasks (host array, copied) executed on
 * `nstreams` streams of default priority (0 = 8, at most 16).  The plans
 * must have their points set and stay alive while the batch exists.
 * Errors: INVALID_ARG (null/empty arguments, null plan, unknown op), HIP.
 */
int kbn_batch_create(kbn_batch *out, int ntasks, const kbn_task *tasks, int nstreams);

/*
 * Run every task once, asynchronously: the batch's streams wait for the
 * work already queued on `stream`, and `stream` waits for all of them, so
 * the results are ordered after later work on `stream`.
 * Errors: those of the task calls (the first failing task stops the
 * issue; already-issued tasks still run), HIP.
 */
int kbn_batch_run(kbn_batch b, void *stream);

/*
 * Record the batch into a HIP graph for kbn_batch_launch.  Runs the
 * batch once first (on `stream`, as kbn_batch_run, and waits for it) so
 * that every plan workspace has its final size, then captures the same
 * launches.  The graph holds the task buffers' and plans' addresses: until
 * the batch is destroyed its plans refuse kbn_set_points, workspace
 * growth, kbn_timing and kbn_plan_destroy.  Replays read the task inputs
 * as they are at replay time.
 * Errors: INVALID_ARG (a plan has timing on), UNSUPPORTED (fused batch),
 * the task calls' errors, HIP.
 */
int kbn_batch_capture(kbn_batch b, void *stream);

/*
 * Fused mode (on != 0; before kbn_batch_capture): the tasks run in phases
 * around their interpolation, so that the interpolation of the whole batch
 * takes one launch per phase and kernel shape instead of one per task:
 *   1. on the batch's streams, each forward-type task's FFT passes (scaling,
 *      coil maps, coordinate weights, oversampled FFT; Sec. II, the
 *      approximation of A(omega) x as interpolation of an oversampled FFT);
 *   2. one staged gather launch for all FORWARD / JAC_X_ADJ tasks of one
 *      dimension and window width J, one for all JAC_OMEGA tasks (the
 *      Jacobian expressions evaluated as extra NUFFTs of x weighted by the
 *      coordinate grids, folded with the upstream gradient), and one
 *      output-stationary spread launch for all ADJOINT / JAC_X_FWD tasks
 *      with the same owner-tile shape and channels per thread (the
 *      transpose of the interpolation, A(omega)^H y);
 *   3. each task's epilogue on its stream: the omega-gradient's sum over
 *      channel groups, or the adjoint's split-tile sums and inverse FFT
 *      passes.
 * A task that needs several workspace chunks, has no points, or whose
 * interpolation takes another kernel (an unstaged gather, the
 * channel-per-lane or scatter spread) runs whole in phase 1.  Results are
 * bitwise those of the single calls.  Because the phases of different tasks
 * interleave, fused tasks must be independent even within one plan: no task
 * may read another task's output, and only JAC_OMEGA tasks with accumulate
 * set may share an output (their sums run in list order on one stream).
 * Each phased task holds device memory of its own (its grids, through its
 * plan's allocator, counted in kbn_plan_info) while the batch is fused; the
 * first run after kbn_set_points on a plan of the batch rebuilds the phases
 * and waits for `stream`.  on = 0 returns to per-task issue and frees them.
 * A fused batch runs with kbn_batch_run only: kbn_batch_capture refuses it
 * (UNSUPPORTED).
 * Errors: INVALID_ARG (null batch, batch already captured), HIP.
 */
int kbn_batch_fuse(kbn_batch b, int on);

/* Replay the captured graph on `stream` (asynchronous).
 * Errors: INVALID_ARG (not captured), HIP. */
int kbn_batch_launch(kbn_batch b, void *stream);

/* Wait for the batch's streams, free the graph and the streams, and
 * release the plans.  Errors: INVALID_ARG (null). */
int kbn_batch_destroy(kbn_batch b);

/* Static description of an error code. */
const char *kbn_strerror(int code);

/* Message of the calling thread's last failing call ("" if none). */
const char *kbn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KBNUFFT_H */
