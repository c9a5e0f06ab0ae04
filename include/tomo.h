/*
 * tomo.h - C ABI of the MI355X local-ROI tomography library.
 *
 * Method: D. M. Pelt, K. J. Batenburg, "A method for locally approximating
 * regularized iterative tomographic reconstruction methods" (arXiv 1604.02292).
 * Section 2.1 defines the data p (N_d N_theta line integrals), the image x
 * (N x N pixels), the projector W, its transpose, and the local / outer
 * operators W_L = W M_L, W_F = W M_F with W = W_L + W_F (eq. 1, eq. locouter).
 * Section 2.2 defines FBP(p, h) = W^T C_h p; Section 2.3 the regularised
 * problem argmin_{x in D} ||p - W x||^2 + lambda g(x) (eq. priorsys), here with
 * D = {x >= 0} and g = TV.  Section 3.3 pads the local part on each side and
 * crops the result; Section 5.6 reconstructs independent local parts in
 * parallel and places them side by side.
 *
 * Conventions (all sizes in pixels; FP32 data, row-major, contiguous):
 *   pixel (r, c) of the N x N grid has centre x = c - (N-1)/2, y = r - (N-1)/2;
 *   detector bin i has centre s_i = (i - (N_d-1)/2) * det_spacing + det_offset;
 *   a sinogram is float[N_theta][N_d] (detector index fastest);
 *   a ray is {x cos(theta) + y sin(theta) = s}.  W uses Joseph interpolation:
 *   w = max(0, 1 - |s_i - t| / m) / m,  t = x cos + y sin,  m = max(|cos|, |sin|).
 *
 * Memory: every array argument is a DEVICE pointer owned by the caller (e.g. a
 * torch tensor's data_ptr) unless stated otherwise.  The library allocates no
 * device memory of its own: all internal state lives in the caller-supplied
 * workspace given to tomo_create, whose size is also the HBM budget that
 * admission control in roi_submit works against.
 *
 * Streams: calls taking `hip_stream` enqueue on that hipStream_t (NULL = the
 * null stream) and return before the GPU work is done, unless stated.
 *
 * Errors: every call returns a tomo_status; nothing aborts or throws across
 * the ABI.  The text of the last error on a context is tomo_last_error(ctx).
 * A context may be used from one host thread at a time; the serving calls
 * (roi_submit / roi_poll) may be called while the library's own scheduler
 * thread runs.
 */
#ifndef TOMO_H
#define TOMO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TOMO_OK = 0,
    TOMO_EINVAL = -1,   /* invalid argument (size < 1, rect outside grid, null pointer, ...) */
    TOMO_ENOMEM = -2,   /* the request cannot fit in the workspace, even when it is empty */
    TOMO_EHIP = -3,     /* a HIP runtime error; see tomo_last_error */
    TOMO_EBUSY = -4,    /* the resource is in use (e.g. unregistering a sinogram with live requests) */
    TOMO_ENOENT = -5,   /* unknown geometry id, sinogram id or ticket */
    TOMO_EAGAIN = -6,   /* the bounded request queue is full; try again later */
    TOMO_ESTATE = -7    /* call not valid in this state (e.g. GPU call on a host-only context) */
} tomo_status;

typedef struct tomo_ctx tomo_ctx;

/* Half-open rectangle of pixels on the global N x N lattice. */
typedef struct { int32_t row0, col0, rows, cols; } tomo_rect;

/* Create a context on HIP device `device` using the caller's device buffer
 * `workspace` of `workspace_bytes` bytes (kept alive by the caller until
 * tomo_destroy).  device = -1 creates a host-only planning context that
 * accepts tomo_set_geometry / tomo_roi_band / tomo_roi_ext only.
 * Errors: EINVAL (null out, device < -1, workspace NULL or < 1 MiB on a GPU
 * context), EHIP. */
tomo_status tomo_create(int device, void* workspace, size_t workspace_bytes, tomo_ctx** out);

/* Stop the scheduler thread, wait for the GPU work the context issued, free host state.
 * The workspace is not freed (it belongs to the caller). */
tomo_status tomo_destroy(tomo_ctx* ctx);

/* Text of the last error on ctx; valid until the next call on ctx.  Never NULL. */
const char* tomo_last_error(const tomo_ctx* ctx);

/* Define a parallel-beam geometry (Section 2.1): an n x n grid, n_angles angles
 * (angles = host array of n_angles radians, or NULL for theta_k = k pi / n_angles),
 * n_det bins of width det_spacing (>= 1 pixel) shifted by det_offset.  The
 * Joseph branch (|cos| >= |sin|: step along rows) is decided here in FP64.
 * Returns a geometry id in *geom_id.  Errors: EINVAL. */
tomo_status tomo_set_geometry(tomo_ctx* ctx, int32_t n, int32_t n_angles, int32_t n_det,
                              const double* angles, double det_spacing, double det_offset,
                              int32_t* geom_id);

/* Detector band of a region (the nonzero rows of W_L, Section 2.1, widened by
 * one bin on each side and NOT clipped to the detector): per angle k the
 * bins [i0[k], i0[k] + width[k]) may be touched by pixels of `region`.
 * i0 and width are HOST arrays of n_angles entries.  Errors: EINVAL, ENOENT. */
tomo_status tomo_roi_band(tomo_ctx* ctx, int32_t geom, tomo_rect region, int32_t* i0,
                          int32_t* width);

/* Extended local part of Section 3.3: `roi` padded by `margin` on each side and
 * clipped to the grid, written to *ext (host).  Errors: EINVAL. */
tomo_status tomo_roi_ext(tomo_ctx* ctx, int32_t geom, tomo_rect roi, int32_t margin,
                         tomo_rect* ext);

/* Forward projection W_L img = W M_L img (Section 2.1 eq. 1): img is the
 * region's image float[rows][cols]; sino is float[n_angles][n_det].  With
 * accumulate = 0 the whole sinogram is overwritten (zero outside the region's
 * band); with accumulate = 1 the projection is added.  Errors: EINVAL, ENOENT,
 * ENOMEM (region scratch), EHIP. */
tomo_status tomo_fp(tomo_ctx* ctx, int32_t geom, tomo_rect region, const float* img,
                    float* sino, int accumulate, void* hip_stream);

/* Backprojection W_L^T sino = M_L W^T sino onto `region`: img is
 * float[rows][cols], overwritten (accumulate = 0) or added to.  Errors as tomo_fp. */
tomo_status tomo_bp(tomo_ctx* ctx, int32_t geom, tomo_rect region, const float* sino,
                    float* img, int accumulate, void* hip_stream);

/* FBP with the Ram-Lak filter (Section 2.2 eq. fbp): img (float[n][n]) =
 * (pi / n_angles) * det_spacing * W^T (det_spacing * h (*) sino), where h is the
 * spatial Ram-Lak filter for sampling interval det_spacing and (*) is a linear
 * (zero-padded) convolution along the detector.  Errors as tomo_fp. */
tomo_status tomo_fbp_ramlak(tomo_ctx* ctx, int32_t geom, const float* sino, float* img,
                            void* hip_stream);

/* tomo_fbp_ramlak for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation).  Same
 * arguments and the same result bits; the call allocates nothing (no hipMalloc,
 * no workspace block, no pinned staging): its scratch - work list, job
 * descriptor, per-angle tables and the filtered band, about
 * 4 * n_angles * (sqrt(2) * n + 8) + n^2 / 16 bytes - lives in one static
 * 32 MiB device array per GPU, set up when the first context on that GPU is
 * created and held until the process ends.  Every call on a GPU shares that
 * array, so calls that overlap on one GPU (on different streams or from
 * different threads) race; calls in one stream order do not.  Errors: EINVAL
 * when the geometry needs more scratch than the array holds (the 4096-pixel,
 * 512-angle geometry needs 12.4 MiB, an 8192-pixel, 1024-angle one 49 MiB);
 * otherwise as tomo_fbp_ramlak. */
tomo_status tomo_fbp_ramlak_noalloc(tomo_ctx* ctx, int32_t geom, const float* sino, float* img,
                                    void* hip_stream);

/* Exterior subtraction through W = W_L + W_F (eq. locouter): for the extended
 * local part ext_roi, sino_local = sino - W M_F x_ext on every bin of the
 * region's band that lies on the detector, and 0 on all other bins.
 * x_ext is float[n][n]; sino and sino_local are float[n_angles][n_det].
 * Errors as tomo_fp. */
tomo_status tomo_exterior_subtract(tomo_ctx* ctx, int32_t geom, tomo_rect ext_roi,
                                   const float* sino, const float* x_ext, float* sino_local,
                                   void* hip_stream);

typedef enum {
    ROI_TV_NONNEG_CP = 0,   /* Chambolle-Pock on h^2 ||W_L x - b||^2 + lambda TV(x), x >= 0
                               (eq. priorsys), h = 1/n: path lengths and line integrals
                               measured with the image side as the unit of length
                               (h = 1 with ROI_FLAG_PIXEL_UNITS) */
    ROI_NONNEG_SIRT = 1,    /* x <- P(x + alpha W_L^T (b - W_L x)), alpha = 1/(N_theta N_d),
                               P the box of eq. sirtbox: [0, inf), or [box_lo, box_hi] with
                               ROI_FLAG_BOX (eq. sirtit) */
    ROI_LOCAL_SIRT = 2,     /* the paper's local method (Section 3.2, eq. localmethod, Alg. 2)
                               for SIRT with the box prior of eq. sirtbox ([0, inf) unless
                               ROI_FLAG_BOX); only through roi_solve_local */
    ROI_LOCAL_FISTA_TV = 3, /* the paper's local FISTA for lambda TV (Alg. 3) with an FGP
                               inner solver of inner_iters iterations (box: none unless
                               ROI_FLAG_BOX); only through roi_solve_local */
    ROI_LOCAL_FISTA_HAAR = 4 /* the same local FISTA for lambda ||B x||_1, B the orthonormal
                               Haar transform with inner_iters levels (eq. sirtista);
                               no box; only through roi_solve_local */
} roi_method;

enum {
    ROI_FLAG_HALF_DATA = 1, /* use 1/2 ||W_L x - b||^2 as the data term */
    ROI_FLAG_ANISO_TV = 2,  /* anisotropic TV (sum of |d/dr| + |d/dc|) */
    ROI_FLAG_BOX = 4,       /* SIRT-type methods: box [box_lo, box_hi] instead of [0, inf) */
    ROI_FLAG_NO_MOMENTUM = 8, /* local FISTA methods without momentum: the ISTA form
                               (eq. sirtista), z = x^k */
    ROI_FLAG_PIXEL_UNITS = 16 /* CP only: data term in pixel units, ||W_L x - b||^2 (h = 1) */
};

/* One local reconstruction request.  roi: the part the caller wants; margin:
 * padding on each side (Section 3.3), clipped to the grid; lambda: TV weight;
 * iters: fixed iteration count (no early stop); sigma, tau: CP step sizes, or
 * 0 for sigma = tau = 1/sqrt(1.01 h^2 mu + 8), mu = lambda_max(W_L^T W_L - Laplacian)
 * from a cached power iteration (per geometry and extended shape), an upper bound of
 * ||[h W_L; grad]||^2 since ||grad||^2 <= 8; box_lo,
 * box_hi: the box of SIRT-type methods when flags has ROI_FLAG_BOX (box_lo may
 * be -inf, box_hi +inf; box_lo <= box_hi; not accepted for CP and the Haar prior);
 * inner_iters: FGP iterations per outer iteration of ROI_LOCAL_FISTA_TV (0 = 100, the
 * paper's count), Haar levels of ROI_LOCAL_FISTA_HAAR (0 = 4, at most 6); ignored by
 * the other methods. */
typedef struct {
    tomo_rect roi;
    int32_t margin;
    int32_t method;     /* roi_method */
    float lambda;
    int32_t iters;
    float sigma, tau;
    uint32_t flags;     /* ROI_FLAG_* */
    float box_lo, box_hi;
    int32_t inner_iters;
} roi_params;

/* Solve one ROI: extend, subtract the exterior (x_ext = float[n][n], or NULL to
 * use the Ram-Lak FBP of sino computed here), run `iters` iterations on the
 * extended part from x = 0, and write the crop to out (float[roi.rows][roi.cols]).
 * Stream-ordered on hip_stream.  Errors: EINVAL, ENOENT, ENOMEM, EHIP. */
tomo_status roi_solve(tomo_ctx* ctx, int32_t geom, const float* sino, const float* x_ext,
                      const roi_params* params, float* out, void* hip_stream);

/* Solve `count` independent ROIs of one sinogram together (Section 5.6: local
 * parts are independent and can be reconstructed in parallel): every
 * iteration runs as one launch per operator over the work items of all ROIs.
 * params and outs are HOST arrays of count entries; outs[i] is a device
 * pointer to float[roi.rows][roi.cols].  Each result equals the one roi_solve
 * gives for the same ROI.  Errors as roi_solve. */
tomo_status roi_solve_batch(tomo_ctx* ctx, int32_t geom, const float* sino, const float* x_ext,
                            int32_t count, const roi_params* params, float* const* outs,
                            void* hip_stream);

/* roi_solve_batch with the crops stitched into one image (Section 5.6: local parts
 * placed side by side, no blending, as in the tiled reconstruction of a whole slice):
 * ROI i's crop is written to img[roi.row0 + r][roi.col0 + c] (img is a device
 * float[n][ld], ld >= n); pixels no ROI covers are left as they are, and where ROIs
 * overlap the later one in params wins.  Errors as roi_solve_batch, and EINVAL for
 * ld < n. */
tomo_status roi_solve_stitched(tomo_ctx* ctx, int32_t geom, const float* sino,
                               const float* x_ext, int32_t count, const roi_params* params,
                               float* img, int32_t ld, void* hip_stream);

/* Bytes of the iteration state of one CP-TV or SIRT solve (Section 2.2, Algorithm
 * CP: the primal x, the extrapolated primal in two buffers and its transposed copy,
 * the TV dual in two buffers, the data dual on the detector band), for
 * roi_solve_resume.  Host call.  Errors: EINVAL (also for the local methods), ENOENT. */
tomo_status roi_state_bytes(tomo_ctx* ctx, int32_t geom, const roi_params* params,
                            size_t* bytes);

/* roi_solve in pieces: runs params->iters iterations that follow `done` earlier
 * ones.  state (device, roi_state_bytes, caller-owned) holds the iteration state
 * after those `done` iterations (ignored when done = 0: the solve starts from
 * zero) and receives the state after done + iters; out receives the crop as in
 * roi_solve.  Running K1 iterations from done = 0 and then K2 from done = K1 with
 * the same params otherwise gives the bits of one roi_solve of K1 + K2 iterations
 * (the steps of a CP-TV solve are fixed by the region's shape, as in roi_solve).
 * A state of other params, or a wrong `done` parity, gives wrong results.
 * Stream-ordered on hip_stream.  Errors as roi_solve, and EINVAL for done < 0. */
tomo_status roi_solve_resume(tomo_ctx* ctx, int32_t geom, const float* sino, const float* x_ext,
                             const roi_params* params, int32_t done, void* state, float* out,
                             void* hip_stream);

/* SIRT-approximating FBP filters (Section 3.1: eq. filtcalc, eq. sirtapp, Alg. 1).
 * filters: device float[iters][n_angles][n_det], caller-owned; plane k - 1
 * receives u_k = alpha W q_k with q_k = sum_{j<k} A^j e, A = I - alpha W^T W,
 * alpha = 1/(n_angles n_det) and e the unit image at pixel (n/2, n/2) (the grid
 * centre for odd n).  One projection and one backprojection of the whole grid per
 * filter, each from the previous one, in FP32; the filters depend only on the
 * geometry.  Stream-ordered on hip_stream.
 * Errors: EINVAL (iters < 1, null pointer), ENOENT, ENOMEM, EHIP. */
tomo_status tomo_sirt_filters(tomo_ctx* ctx, int32_t geom, int32_t iters, float* filters,
                              void* hip_stream);

/* Filtered data of the local method (Section 3.1 eq. sirtapp; Section 3.3: computed
 * once per sinogram and shared by all local parts): for k < count,
 *   out[k][a][i] = sum_j filters[k][a][i - j + c_a] sino[a][j],
 * terms with an index outside [0, n_det) being zero, where c_a is the bin nearest
 * the projection of pixel (n/2, n/2) at angle a (the filters' zero lag), decided
 * in FP64.  filters, sino (float[n_angles][n_det]) and out (float[count][n_angles]
 * [n_det]) are caller-owned device arrays.  Computed by FFT in FP32; n_det <= 8192.
 * Stream-ordered.  Errors: EINVAL (count < 1, n_det > 8192, null), ENOENT,
 * ENOMEM, EHIP. */
tomo_status tomo_sirt_filter_sino(tomo_ctx* ctx, int32_t geom, const float* filters,
                                  int32_t count, const float* sino, float* out,
                                  void* hip_stream);

/* The paper's local method (Section 3.2: eq. localmethod, Alg. 2, Alg. 3) for `count`
 * independent ROIs together.  On the extended part L of each ROI, from v = 0, for
 * k = 1..iters, with d_k = filtered[k - 1] (tomo_sirt_filter_sino: W_L^T d_k is the
 * local SIRT approximation FBP_L(p, u_k)) and alpha = 1/(n_angles n_det):
 *   ROI_LOCAL_SIRT (Alg. 2, box prior of eq. sirtbox, P the request's box):
 *     x = P(v + W_L^T (d_k - alpha W_L v)),   v <- x - W_L^T d_k;
 *   ROI_LOCAL_FISTA_TV (Alg. 3, FISTA on eq. priorsys with g = TV):
 *     x^k = FGP(v + W_L^T (d_k - alpha W_L v)),   t^k = (1 + sqrt(1 + 4 (t^{k-1})^2)) / 2,
 *     v <- x^k + ((t^{k-1} - 1) / t^k)(x^k - x^{k-1}) - W_L^T d_k,   t^0 = 1, x^0 = 0,
 *     FGP being inner_iters iterations of min_P ||x - w||^2 + 2 gamma TV(x) from a zero
 *     dual, gamma = alpha lambda / 2 (alpha lambda with ROI_FLAG_HALF_DATA),
 *     isotropic TV unless ROI_FLAG_ANISO_TV;
 *   ROI_LOCAL_FISTA_HAAR: the same iteration with x^k = B^T soft(B w, gamma), B the
 *     orthonormal Haar transform with inner_iters levels on the extended part (pairs
 *     (a, b) -> ((a + b)/sqrt 2, (a - b)/sqrt 2) along rows then columns of the block
 *     of sums, an unpaired last entry carried as a sum), every coefficient thresholded.
 * The crop of x is written to outs[i] (float[roi.rows][roi.cols], device).
 * filtered: device float[planes][n_angles][n_det]; params and outs are host arrays of
 * count entries; every params[i].method is ROI_LOCAL_SIRT, ROI_LOCAL_FISTA_TV or
 * ROI_LOCAL_FISTA_HAAR with iters <= planes (sigma, tau are ignored).  Stream-ordered.
 * Errors: EINVAL, ENOENT, ENOMEM, EHIP. */
tomo_status roi_solve_local(tomo_ctx* ctx, int32_t geom, const float* filtered, int32_t planes,
                            int32_t count, const roi_params* params, float* const* outs,
                            void* hip_stream);

/* Disc subtraction (Section 3.3): out = sino - c W disc, where disc is the image that
 * is 1 on the pixels whose centres lie within n/2 of the grid centre (decided exactly)
 * and c = sum_a S_a T_a / sum_a T_a^2 minimises the l2 norm of the projections'
 * zero-frequency components (S_a, T_a: FP64 row sums of sino and of W disc).  c is
 * written to *value (device float, caller-owned); out may be sino.  Undo it on a
 * result with tomo_disc_add.  Stream-ordered; the disc's projection lives in the
 * workspace during the call.  Errors: EINVAL (null), ENOENT, ENOMEM, EHIP. */
tomo_status tomo_disc_subtract(tomo_ctx* ctx, int32_t geom, const float* sino, float* out,
                               float* value, void* hip_stream);

/* Adds *value (device float) to the pixels of img (float[region.rows][region.cols],
 * the given region of the grid, device) that belong to the disc of
 * tomo_disc_subtract.  Stream-ordered.  Errors: EINVAL, ENOENT, EHIP. */
tomo_status tomo_disc_add(tomo_ctx* ctx, int32_t geom, tomo_rect region, const float* value,
                          float* img, void* hip_stream);

/* Constant padding of truncated data (Section 4): trunc holds n_bins measured bins per
 * angle (float[n_angles][n_bins], device), detector bins first_bin .. first_bin +
 * n_bins - 1 of the geometry; out (float[n_angles][n_det], device) receives them with
 * every row extended by its first and last measured values.  Stream-ordered.
 * Errors: EINVAL (null, bins outside the detector), ENOENT, EHIP. */
tomo_status tomo_pad_truncated(tomo_ctx* ctx, int32_t geom, const float* trunc, int32_t first_bin,
                               int32_t n_bins, float* out, void* hip_stream);

/* The CP step size the library would use for extended region `ext` (host float
 * out).  Runs the power iteration if the shape is not cached (blocking).
 * Errors: EINVAL, ENOENT, ENOMEM, EHIP. */
tomo_status roi_step_size(tomo_ctx* ctx, int32_t geom, tomo_rect ext, float* sigma_tau);

/* Make a sinogram resident for serving: the library computes and keeps its
 * Ram-Lak FBP exterior estimate x_ext and the residual r = sino - W x_ext in
 * the workspace (Section 3.3: precompute once, reuse for every local part).
 * `sino` (float[n_angles][n_det]) is borrowed: it must stay alive and unchanged
 * until tomo_unregister_sinogram.  Blocking.  Errors: EINVAL (also for a sinogram
 * that holds NaN or infinite values: nothing is registered), ENOENT, ENOMEM, EHIP. */
tomo_status tomo_register_sinogram(tomo_ctx* ctx, int32_t geom, const float* sino,
                                   int32_t* sino_id);

/* Release a registered sinogram.  Errors: ENOENT, EBUSY (requests still queued or running). */
tomo_status tomo_unregister_sinogram(tomo_ctx* ctx, int32_t sino_id);

/* Submit a request against a registered sinogram.  Never blocks: the request
 * joins a bounded queue; the scheduler thread admits it into the running batch
 * when a slot and workspace memory are free (continuous batching), runs it on
 * its own stream together with the other admitted requests, and writes the
 * crop into out (device float[roi.rows][roi.cols], kept alive by the caller
 * until roi_poll reports done).  Errors: EINVAL, ENOENT, ENOMEM (cannot fit even
 * in an empty workspace), EAGAIN (queue full). */
tomo_status roi_submit(tomo_ctx* ctx, int32_t sino_id, const roi_params* params, float* out,
                       uint64_t* ticket);

/* Poll a ticket: *done = 1 once its result is in `out` (then *latency_ms, if
 * not NULL, is the host-clock time from roi_submit to completion).  A done
 * ticket is forgotten after the poll that reports it.  Never blocks.
 * Errors: ENOENT (unknown or already reported ticket), EHIP (the request failed). */
tomo_status roi_poll(tomo_ctx* ctx, uint64_t ticket, int* done, float* latency_ms);

/* roi_poll with the request's timeline: stages_ms (float[4]) receives, once
 * *done = 1, host-clock times on the scheduler thread: from submission to admission
 * (queued), from admission to the enqueueing of its first iteration (preparation:
 * tables, b = r + W_L x_ext|L, step size; work that only needs enqueueing costs
 * little here and runs on the GPU during the next stage), from there to completion
 * (iterations, crop), and the total (the latency of roi_poll); -1 while not done.
 * Same ticket rules and errors as roi_poll. */
tomo_status roi_poll_stages(tomo_ctx* ctx, uint64_t ticket, int* done, float* stages_ms);

/* Serving knobs: maximum concurrent slots (default 32) and iterations per
 * scheduler tick (default 4); 0 leaves a value unchanged. */
tomo_status tomo_serving_config(tomo_ctx* ctx, int32_t max_slots, int32_t iters_per_tick);

/* Host-side testing of serving without a GPU.  On a host-only context (device -1)
 * the first call (budget_bytes > 0) replaces the GPU work of serving by a test
 * executor: registration, submission, admission against a workspace budget of
 * budget_bytes (bookkeeping only: no memory is allocated or touched),
 * continuous batching, ticket lifecycle and retirement run as on a GPU context,
 * but `sino` and `out` are host memory, nothing is reconstructed, and a retired
 * request's out holds the number of iterations that its slot ran.  Each tick takes
 * tick_us microseconds per iteration; tick_us < 0 stalls the executor (ticks wait)
 * until a later call with budget_bytes = 0 sets tick_us >= 0.  tomo_destroy ends a
 * stall.  Errors: EINVAL (budget under 1 MiB), ESTATE (GPU context; a second
 * set-up; a tick change before the set-up). */
tomo_status tomo_serving_fake(tomo_ctx* ctx, size_t budget_bytes, int32_t tick_us);

/* Iteration graphs: when enabled (the default), the second and later solves
 * with the same work-list layout replay a captured hipGraph of the whole
 * iteration loop instead of launching its kernels one by one (same kernels,
 * same arguments, same results).  enable = 0 always launches eagerly. */
tomo_status tomo_set_graphs(tomo_ctx* ctx, int enable);

/* Kernel launch shape of the two projector kernels.  Every field 0 = choose
 * automatically (from an autotuned entry for the problem's shape class when
 * tomo_autotune has measured one, else from the problem size).
 *   fp_segments           forward projector: waves per ray, 1, 2, 4 or 8 (8: blocks
 *                         of 8 waves, one group of 64 rays each)
 *   fp_rays_per_lane      1, or 2 (with one segment): each lane projects two
 *                         adjacent rays from 4-pixel reads (detector spacing
 *                         below sqrt 2 pixels; otherwise 1 is used), or 4: the
 *                         LDS-staged forward projector (32 lines of the regions
 *                         at a time in LDS, 24 when the padded lines hold more
 *                         than 336 entries, 16 when more than 480, shared by
 *                         groups of up to 64 angles; regions whose padded lines
 *                         hold at most 784 entries, about 776 pixels a side, and
 *                         bands of at most 4096 rays; elsewhere 2 is used)
 *   fp_xcd_order          order in which forward-projector work items are dealt
 *                         to the chip's 8 XCDs: 1 = one contiguous eighth of the
 *                         item list per XCD (L2 locality), 2 = round-robin
 *   bp_variant            backprojector: 1 = direct band reads from memory,
 *                         2 = band windows staged in LDS per block of angles
 *   bp_groups             backprojector angle groups per pixel, 1, 2, 4 or 8
 *                         (8: blocks of 8 waves; variant 2 always uses 1, and the
 *                         two-channel bands of the local method use 4 for 8)
 *   bp_pixels_per_thread  1 or 2
 *   bp_xcd_order          as fp_xcd_order, for the backprojector
 * Results agree to FP32 rounding across shapes; the two variants give
 * identical results for the same groups and pixels per thread. */
typedef struct {
    int32_t fp_segments, fp_rays_per_lane, fp_xcd_order;
    int32_t bp_variant, bp_groups, bp_pixels_per_thread, bp_xcd_order;
} tomo_launch;

/* Force a launch shape for every later call on ctx (NULL = all automatic).
 * Errors: EINVAL (a field outside the values above). */
tomo_status tomo_set_launch(tomo_ctx* ctx, const tomo_launch* cfg);
/* The shape last set with tomo_set_launch.  Errors: EINVAL. */
tomo_status tomo_get_launch(tomo_ctx* ctx, tomo_launch* cfg);

/* The launch shape roi_solve / roi_solve_batch would use now for this batch of
 * ROI parameters (host array of count entries): forced fields, else an
 * autotuned entry for the batch's class, else the size heuristics.  Errors:
 * EINVAL, ENOENT. */
tomo_status tomo_resolve_launch(tomo_ctx* ctx, int32_t geom, int32_t count,
                                const roi_params* params, tomo_launch* out);

/* Autotuner: times every forward-projector shape (segments x XCD order) and
 * every backprojector shape (variant x groups x pixels per thread x XCD
 * order) on this batch of ROI solves, one iteration each with HIP events
 * around back-to-back launches, and records the fastest of each for the
 * batch's shape class (geometry, total extended pixels to within a factor
 * of 2, one ROI or many).  Later roi_solve / roi_solve_batch calls of that
 * class use it unless tomo_set_launch forces a shape.  Arguments as for
 * roi_solve_batch (outs receive the one-iteration results and are then
 * undefined); best (nullable, host) receives the chosen shape and ms
 * (nullable, host, 2 floats) the chosen FP and BP launch times in ms.
 * Synchronizes `hip_stream`.  Errors: as roi_solve_batch. */
tomo_status tomo_autotune(tomo_ctx* ctx, int32_t geom, const float* sino, const float* x_ext,
                          int32_t count, const roi_params* params, float* const* outs,
                          void* hip_stream, tomo_launch* best, float* ms);

/* Algorithmic work: the exact number of nonzeros of W_L for `region` (the
 * pixel-ray pairs with w > 0, counted in FP64 on the host from the entry
 * formula above), i.e. the updates one forward projection (or one
 * backprojection) of the region performs.  Works on host-only contexts.
 * Errors: EINVAL, ENOENT. */
tomo_status tomo_roi_nnz(tomo_ctx* ctx, int32_t geom, tomo_rect region, int64_t* nnz);

/* Measurement hook for the iteration kernels, forward projection (kernel 0),
 * backprojection (kernel 1) and the FGP steps of local FISTA-TV (kernel 2, all
 * FGP launches of one outer iteration together).  mode 1: the solve calls record a
 * HIP event pair on their stream around every iteration launch.  mode 2: each solve
 * first runs 50 back-to-back launches of each kernel on its own data, captured
 * in a hipGraph (no dispatch gaps between them) and bracketed by two HIP events
 * on the solve's stream, then clears its state and solves as usual (results
 * are unchanged; roi_solve and roi_solve_batch only).  mode 0: off.  tomo_kernel_time
 * waits for the recorded
 * events and returns, per kernel, the number of timed launches and their total
 * GPU time in milliseconds (host outputs); reset = 1 clears the totals. */
tomo_status tomo_kernel_timing(tomo_ctx* ctx, int mode);
tomo_status tomo_kernel_time(tomo_ctx* ctx, int32_t kernel, int64_t* launches, double* total_ms,
                             int reset);

/* Calibration of the projectors' ALU roof; not a step of the method.  One launch on
 * hip_stream of `blocks` blocks of 256 threads in which every lane runs iters x 16
 * steps on each of eight independent chains and writes the sum of its chains to
 * out[block * 256 + lane] (device, caller-owned, blocks x 256 floats).  A step is, by
 * mode: 0 one FP32 FMA v = v a + b; 1 an FMA and a fraction, v = fract(v a + b) (two
 * instructions); 2 one FP32 add v = v + b.  The launch issues blocks x 256 x iters x
 * 128 steps' vector lane-instructions besides a few per lane; timed by the caller
 * (events on the same stream), it gives the rate at which the chip retires them.
 * Errors: EINVAL (null out, blocks or iters outside [1, 2^20], unknown mode), EHIP. */
tomo_status tomo_valu_probe(tomo_ctx* ctx, int32_t blocks, int32_t iters, int32_t mode, float a,
                            float b, float* out, void* hip_stream);

/* Workspace bytes in use now and at peak (host outputs). */
tomo_status tomo_workspace_usage(tomo_ctx* ctx, size_t* used, size_t* peak);

/* Wait until all GPU work issued by the context's own streams is done (with the
 * serving test executor on a host-only context: until no request is queued or
 * running). */
tomo_status tomo_synchronize(tomo_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* TOMO_H */
