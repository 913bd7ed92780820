/*
 * sfft.h -- C ABI of the MI355X (gfx950) SFFT image-differencing library.
 *
 * The method (paper Sec. 1 and Sec. 2.3.2, image differencing): between an
 * aligned reference image R and science image S, fit by least squares a
 * matching kernel in a delta-function basis (free pixel values on an L x L
 * grid) whose values vary over the image as a polynomial of total degree DK,
 * plus a differential-background polynomial of degree DB; the fit is
 * assembled in the Fourier domain; then convolve R with the fitted kernel and
 * subtract it from S. The paper gives no equations; the operation computed
 * here is the periodic least-squares problem
 *
 *   theta* = argmin sum_x ( S'(x) - M(x) )^2,
 *   M(x)   = sum_i sum_d a_(i,d) p_i(x-d) R'(x-d) + sum_c b_c q_c(x),
 *   D(x)   = S'(x) - M(x),
 *
 * with R' = R - ref_pedestal, S' = S - sci_pedestal, indices modulo (W, H),
 * p_i / q_c the monomials xt^a yt^b of total degree <= DK / <= DB in
 * xt = 2x/(W-1) - 1, yt = 2y/(H-1) - 1, ordered for d = 0..D, for b = 0..d:
 * (a = d - b, b). Unknowns: kernel coefficient (i, dy, dx), dy, dx in
 * [-r, r], r = (L-1)/2, at index i*L*L + (dy+r)*L + (dx+r); background
 * coefficient c at n(DK)*L*L + c; n(D) = (D+1)(D+2)/2.
 *
 * Memory: every image, matrix and vector pointer is a HIP device pointer
 * owned by the caller; the library never frees caller memory. Workspaces are
 * caller-provided device buffers of at least the queried size. Images are
 * row-major, W columns by H rows, with a row pitch of `ld` elements.
 *
 * Execution: every compute call is asynchronous and ordered on `stream`
 * (a hipStream_t; NULL means the null stream). The returned status covers
 * argument validation, plan set-up and launch errors only; conditions found
 * on the device (non-finite pixels, a matrix that is not positive definite)
 * are written to device memory (sfft_solve_info) and must be read after the
 * stream is synchronised. No call aborts or throws.
 *
 * Threading: a handle is not thread-safe; use one handle per host thread.
 * The first call for a new image shape builds device-side plan tables with
 * blocking copies (do it before any stream capture).
 */
#ifndef SFFT_MI355X_SFFT_H
#define SFFT_MI355X_SFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SFFT_OK = 0,
  SFFT_ERR_INVALID_ARG = 1,   /* null pointer, even or non-positive L, degree out of range, ld < W */
  SFFT_ERR_UNSUPPORTED = 2,   /* valid problem this build does not run (see sfft_validate) */
  SFFT_ERR_WORKSPACE = 3,     /* workspace pointer null or smaller than required */
  SFFT_ERR_NONFINITE = 4,     /* a NaN/Inf input pixel was seen (device-side, via info) */
  SFFT_ERR_NOT_SPD = 5,       /* normal matrix not positive definite (device-side, via info) */
  SFFT_ERR_HIP = 6,           /* a HIP runtime call failed (no device, launch failure, ...) */
  SFFT_ERR_INTERNAL = 7
} sfft_status;

typedef enum { SFFT_F32 = 0, SFFT_F64 = 1 } sfft_dtype;   /* element type of R, S, D */

typedef enum {
  SFFT_COMPUTE_FP64 = 0,      /* FP64 spectra, correlations and normal matrix (plain form) */
  SFFT_COMPUTE_FP32 = 1       /* FP32 spectra and products, FP32 accumulation; FP64 solve */
} sfft_compute;

/* Where the kernel's spatial polynomial is evaluated (paper Sec. 1 leaves it
 * open). INPUT_PIXEL: M(x) = sum_i sum_d a_(i,d) p_i(x-d) R'(x-d) + ... (the
 * default, every call). OUTPUT_PIXEL: M(x) = sum_i p_i(x) sum_d a_(i,d)
 * R'(x-d) + ...; the FFT builds then fit with R' taken as zero on the
 * r-pixel frame of the image (there the periodic wrap would make the
 * output-pixel polynomial differ from a shifted input-pixel one), which
 * makes the output-pixel normal equations exactly T^T G T, T^T h of the
 * input-pixel ones (T: binomial expansion of the shifted monomials, per
 * kernel offset). Dropping the frame leaves the model without the sky of
 * those pixels: take the sky out with the pedestals (e.g. image means). Supported by sfft_build_system, sfft_build_system_masked,
 * sfft_solve, sfft_subtract(_noalloc) and sfft_difference_multi; the stamp,
 * batched and background-refit calls return SFFT_ERR_UNSUPPORTED. */
typedef enum { SFFT_CONV_INPUT_PIXEL = 0, SFFT_CONV_OUTPUT_PIXEL = 1 } sfft_convention;

typedef struct {
  int32_t width;              /* W: columns (x) */
  int32_t height;             /* H: rows (y) */
  int64_t ld;                 /* row pitch of R, S and D in elements, >= width */
  int32_t L;                  /* kernel size, odd, 1 <= L <= min(W, H) */
  int32_t dk;                 /* kernel polynomial degree, 0..4 */
  int32_t db;                 /* background polynomial degree, 0..4 */
  int32_t image_dtype;        /* sfft_dtype of R, S, D */
  int32_t compute;            /* sfft_compute of the build */
  int32_t convention;         /* sfft_convention: where the kernel polynomial is evaluated */
  double ref_pedestal;        /* c_R, subtracted from R before fitting */
  double sci_pedestal;        /* c_S, subtracted from S before fitting */
} sfft_desc;

/* Written by sfft_solve into device memory. */
typedef struct {
  int32_t status;             /* SFFT_OK, SFFT_ERR_NOT_SPD or SFFT_ERR_NONFINITE */
  int32_t failed_pivot;       /* 0-based first non-positive pivot (LAPACK potrf style), -1 if none */
  int32_t refine_iters;       /* iterative-refinement steps applied */
  int32_t nonfinite;          /* nonzero when the build saw a NaN/Inf pixel */
  double backward_err;        /* ||h - G theta||_inf / (||G||_inf ||theta||_inf + ||h||_inf) */
  double min_pivot;           /* smallest / largest diagonal of the Cholesky factor of the */
  double max_pivot;           /* equilibrated matrix (their squared ratio bounds cond below) */
} sfft_solve_info;

typedef struct sfft_handle_s* sfft_handle;

/* Handle lifetime. sfft_create binds the handle to the current HIP device;
 * it owns only plan tables (FFT twiddles). Errors: SFFT_ERR_INVALID_ARG for
 * a null out pointer, SFFT_ERR_HIP when no device is usable. */
sfft_status sfft_create(sfft_handle* out);
sfft_status sfft_destroy(sfft_handle handle);

/* Human-readable name of a status code (static string, never NULL). */
const char* sfft_status_string(sfft_status status);

/* Number of unknowns N = L*L*n(DK) + n(DB), or -1 for an invalid descriptor.
 * Host-only; needs no device. */
int64_t sfft_num_unknowns(const sfft_desc* desc);

/* Host-only validation of a descriptor for sfft_build_system.
 * SFFT_ERR_INVALID_ARG: see sfft_status. SFFT_ERR_UNSUPPORTED: L > 15 or
 * DK > 2 (every call); W odd, not of the form 2^a 3^b 5^c, or outside
 * [16, 4096], H < 2L or W < 2L (FFT build only: sfft_solve, sfft_subtract
 * and sfft_build_system_stamps accept any width and height >= L). */
sfft_status sfft_validate(const sfft_desc* desc);

/* Bytes of device workspace needed by sfft_build_system, sfft_solve and
 * sfft_subtract for this descriptor (one buffer of this size serves all
 * three; the build leaves a non-finite flag in it that sfft_solve reports).
 * Host-only. */
sfft_status sfft_workspace_size(sfft_handle handle, const sfft_desc* desc, size_t* bytes);

/* Normal equations G theta = h of the least-squares problem above.
 * Kernel-kernel and kernel-science blocks come from cross-correlations
 * computed in the Fourier domain (row FFTs along x, blocked FFT correlation
 * along y, pruned inverse along x); kernel-background and background blocks
 * from exact polynomial moments with periodic seam corrections.
 *   ref, sci : device images (image_dtype, pitch ld)
 *   G        : device, N*N doubles, row-major, both triangles written
 *   h        : device, N doubles
 *   ws       : device workspace of ws_bytes >= sfft_workspace_size
 * Non-finite pixels are flagged in ws (reported by sfft_solve). */
sfft_status sfft_build_system(sfft_handle handle, const sfft_desc* desc,
                              const void* ref, const void* sci,
                              double* G, double* h,
                              void* ws, size_t ws_bytes, void* stream);

/* Masked fit (SFFT's way of fitting on star stamps only): as
 * sfft_build_system with R' and S' taken as zero wherever mask == 0, i.e. the
 * periodic least-squares problem above on the masked images (every pixel
 * still enters the sum). The difference image is then formed by
 * sfft_subtract from the unmasked images. With the output-pixel convention R'
 * is also zero on the r-pixel frame.
 *   mask    : device uint8, W x H, row pitch mask_ld >= W bytes; nonzero = use
 * Non-finite pixels outside the mask are ignored (neither used nor flagged). */
sfft_status sfft_build_system_masked(sfft_handle handle, const sfft_desc* desc,
                                     const void* ref, const void* sci,
                                     const uint8_t* mask, int64_t mask_ld,
                                     double* G, double* h,
                                     void* ws, size_t ws_bytes, void* stream);

/* theta = G^-1 h in FP64: equilibrate with D = diag(G)^-1/2, Cholesky-factor
 * the equilibrated matrix, forward/back substitution, then up to max_refine
 * (0..8) steps of iterative refinement on the residual h - G theta.
 *   G, h : device (from sfft_build_system or any SPD system of size N)
 *   coef : device, N doubles (written; NaN when the solve fails)
 *   info : device sfft_solve_info (written)
 *   ws   : the same workspace the build used (reads its non-finite flag) */
sfft_status sfft_solve(sfft_handle handle, const sfft_desc* desc,
                       const double* G, const double* h, double* coef,
                       int32_t max_refine, sfft_solve_info* info,
                       void* ws, size_t ws_bytes, void* stream);

/* Size of the team of workgroups that runs sfft_solve (and the solves of
 * sfft_difference_multi) on this handle. The paper's pipeline differences a
 * queue of CCD pairs one after another on each GPU (Sec. 5.2); the solve of
 * one pair is a persistent kernel whose duration is set by its diagonal
 * Cholesky chain, and at the default (team = 0: up to half the CUs) most of
 * those CUs wait. With several pairs in flight on separate streams (each
 * with its own handle, workspace and buffers), a smaller team leaves CUs to
 * the other pairs' builds and subtracts. Results are deterministic for a
 * given team size; teams of different sizes add the solve's partial sums in
 * different groupings, so their coefficients can differ in the last bits.
 *   team : 0 (default) or 2..128; a team larger than the default is not
 *          used (the default applies). Other values: SFFT_ERR_INVALID_ARG. */
sfft_status sfft_set_solve_team(sfft_handle handle, int32_t team);
sfft_status sfft_get_solve_team(sfft_handle handle, int32_t* team);

/* Stage order of the row pass's FFTs along x (the transforms of the FFT
 * form of the least-squares build, paper Sec. 1) on this handle. Every plan
 * is a mixed-radix Stockham transform of length W = 2^a 3^b 5^c with stages
 * of radix 8 (as many as fit), then one of 4 or 2, then 3s, then 5s:
 *   order 0 (default): that sequence; order 1: the same stages reversed.
 * Both compute the same DFT; the sums are grouped differently, so spectra
 * (and everything fitted from them) can differ in the last bits. The
 * batched form has its own setting (sfft_batch_knobs).
 * Other values: SFFT_ERR_INVALID_ARG. */
sfft_status sfft_set_radix_order(sfft_handle handle, int32_t order);
sfft_status sfft_get_radix_order(sfft_handle handle, int32_t* order);

/* D = S' - M_coef(R') with periodic boundaries, accumulated in FP64, in the
 * descriptor's kernel convention (the whole image; no mask).
 * chi2 (nullable, device double): reduced chi^2 of D over the image minus an
 * r-pixel frame, dof = |frame interior| - N, variance per pixel
 * max(S,1) + kappa2(x) max(R,1), kappa2(x) = sum_d (sum_i a_(i,d) p_i(x))^2
 * (Poisson noise, gain 1, on the raw images).
 *   diff : device, image_dtype, pitch ld (may not alias ref or sci) */
sfft_status sfft_subtract(sfft_handle handle, const sfft_desc* desc,
                          const void* ref, const void* sci, const double* coef,
                          void* diff, double* chi2,
                          void* ws, size_t ws_bytes, void* stream);

/* sfft_subtract without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation). The chi2 partial sums and kappa2 coefficients live in
 * a fixed library-owned device array (one per GPU, about 0.5 MB, held until
 * the process ends); the call allocates nothing. Limit: at most 65536 output
 * tiles of 64 x 32 pixels (ceil(W/64) * ceil(H/32) <= 65536, e.g. 8192 x
 * 16384), else SFFT_ERR_WORKSPACE. Calls that overlap on one GPU share the
 * array and race (order them on one stream). Results are identical to
 * sfft_subtract's. */
sfft_status sfft_subtract_noalloc(sfft_handle handle, const sfft_desc* desc,
                                  const void* ref, const void* sci, const double* coef,
                                  void* diff, double* chi2, void* stream);

/* ---- Batched form ------------------------------------------------------
 * All pairs of an exposure (equal-size CCDs and uneven cutouts, possibly
 * different L) differenced together: every phase of build, solve and
 * subtract is one launch over all items (per-item block ranges in one grid;
 * the solve runs teams of co-resident workgroups over a queue of the items,
 * largest first; the subtract
 * is one launch per distinct L), and the whole sequence can be captured in
 * one HIP graph. The launch configuration (sfft_batch_knobs: row-pass rows
 * per workgroup, row FFT radix order, subtract tile height, solve team
 * size) comes from an autotuner (sfft_batch_tune), remembered per batch
 * composition and device in the handle and, when the environment variable
 * SFFT_TUNE_CACHE names a file, across processes.
 * Restrictions: compute SFFT_COMPUTE_FP32, image_dtype SFFT_F32, width <=
 * 2048, one DK for all items (else SFFT_ERR_UNSUPPORTED); n <= 4096. Each item carries its own buffers, exactly as the
 * single-pair calls take them; chi2 is required. */
typedef struct {
  sfft_desc desc;
  const void* ref;
  const void* sci;
  void* diff;
  double* G;
  double* h;
  double* coef;
  sfft_solve_info* info;
  double* chi2;
  void* ws;                   /* >= sfft_workspace_size(desc) bytes, 256-byte aligned */
  size_t ws_bytes;
} sfft_batch_item;

typedef struct sfft_batch_s* sfft_batch;

/* Validates the items and builds the per-phase tables on the device (blocking
 * copies; not inside a stream capture). The items array is copied. */
sfft_status sfft_batch_create(sfft_handle handle, const sfft_batch_item* items, int32_t n,
                              int32_t max_refine, sfft_batch* out);
/* build + solve + subtract (+ chi2) of every item, stream-ordered. */
sfft_status sfft_batch_run(sfft_batch batch, void* stream);
/* The same, captured into a HIP graph on the first call and replayed
 * (stream must not be the null stream). */
sfft_status sfft_batch_run_graph(sfft_batch batch, void* stream);
/* Launch configuration of a batch (the autotuner's search space):
 *   rows_per_block : row-pass image rows per workgroup, 1..64
 *   radix_order    : stage order of the row FFTs, 0 or 1 (as in
 *                    sfft_set_radix_order)
 *   tile_rows      : subtract output tile height, 16, 32 or 64 (tiles are
 *                    64 pixels wide; one workgroup of 8 * tile_rows threads
 *                    per tile)
 *   team           : solve workgroups per team, 1..128, or 0 for one team
 *                    per item (CUs / n, at most 64)
 * The column pass (4 spectrum columns per 512-thread workgroup, the
 * 128-point y-correlation's thread mapping) and the Cholesky tile (64, the
 * FP64 matrix-core tile) are fixed by their kernels' designs.
 * rows_per_block and tile_rows change no bit of the coefficients or the
 * difference image (chi2 adds one partial sum per subtract tile, so
 * tile_rows can change its last bits); team (as in sfft_set_solve_team)
 * and radix_order group sums differently and can change the last bits of
 * the coefficients. */
typedef struct {
  int32_t rows_per_block;
  int32_t radix_order;
  int32_t tile_rows;
  int32_t team;
} sfft_batch_knobs;

/* Times candidate configurations on the stream and keeps the fastest: the
 * row-pass rows per workgroup with the radix order, then the solve team,
 * then the subtract tile height (the phases run one after another, so each
 * group is timed with the others fixed). Runs the batch several times;
 * results of the last run are valid. Either out pointer may be NULL; the
 * whole choice is read back with sfft_batch_get_knobs. */
sfft_status sfft_batch_tune(sfft_batch batch, void* stream, int32_t* rows_per_block, int32_t* team);
/* Sets (without timing) or reads the whole configuration. Out-of-range
 * values: SFFT_ERR_INVALID_ARG, the batch unchanged. Setting is blocking
 * (re-uploads the tables; not inside a stream capture); a captured graph is
 * discarded and captured again on the next sfft_batch_run_graph. */
sfft_status sfft_batch_set_knobs(sfft_batch batch, const sfft_batch_knobs* knobs);
sfft_status sfft_batch_get_knobs(sfft_batch batch, sfft_batch_knobs* knobs);
/* Sets two knobs without timing (the others keep their values): row-pass
 * rows per workgroup 1..64, solve team size 1..128 workgroups, or 0 for one
 * team per item (CUs / n, at most 64).
 * Out-of-range values: SFFT_ERR_INVALID_ARG, the batch unchanged. Blocking
 * (re-uploads the tables; not inside a stream capture); a captured graph is
 * discarded and captured again on the next sfft_batch_run_graph. */
sfft_status sfft_batch_plan(sfft_batch batch, int32_t rows_per_block, int32_t team);
/* Replaces every item's pedestals (ref_pedestals[k], sci_pedestals[k]: host
 * arrays of the batch's item count, finite). The precision form of the
 * build runs its FP32 spectra on R - c_R and S - c_S with c the FP64 image
 * means (the pedestals leave the difference image unchanged up to the
 * periodic seam rows, and keep the sky level out of the FP32 sums).
 * Blocking (re-uploads the tables; not inside a stream capture); a captured
 * graph is discarded. SFFT_ERR_INVALID_ARG for null or non-finite values. */
sfft_status sfft_batch_set_pedestals(sfft_batch batch, const double* ref_pedestals,
                                     const double* sci_pedestals);
sfft_status sfft_batch_destroy(sfft_batch batch);

/* Precision form of the build: the same least-squares problem restricted to
 * the pixels of n_stamps square stamps of side `size` (odd) centred on
 * star pixels (the star-stamp mode of SFFT, paper Sec. 1 and Sec. 2.3.2),
 * with periodic indexing as above. Writes G_s = A_s^T A_s and h_s = A_s^T S'
 * where A_s holds the design rows of the stamp pixels. The Gram sums run on
 * the matrix cores: each operand is rounded to FP32 and split exactly into
 * three bfloat16 terms, hi = bf16(a), mid = bf16(a - hi),
 * lo = bf16(a - hi - mid) (round to nearest even), each product is taken as
 * the six term products of order <= 2 (hi*hi, hi*mid, mid*hi, hi*lo, lo*hi,
 * mid*mid; the dropped ones are below 2^-23 of |a b|), accumulated in FP32
 * over runs of at most 8 x 32 stamp pixels and in FP64 beyond them (relative
 * error per entry a few 2^-24 of the sum of absolute products).
 *   centers : device int32[n_stamps][2] = (x, y) stamp centre pixels
 *   size    : odd, 1..127, <= min(W, H); n_stamps in [1, 65536]
 *   G, h    : device, as for sfft_build_system
 *   ws      : device workspace of at least sfft_stamps_workspace_size bytes
 *             (partial tiles and the split planes of every stamp); it also
 *             serves sfft_solve and sfft_subtract for this descriptor
 * SFFT_ERR_UNSUPPORTED when the planes a Gram tile reads do not fit in LDS
 * (large stamps with DB = 4). Non-finite pixels near the stamps are flagged
 * in ws for sfft_solve. The compute field of desc is ignored. */
sfft_status sfft_stamps_workspace_size(sfft_handle handle, const sfft_desc* desc,
                                       int32_t n_stamps, int32_t size, size_t* bytes);
sfft_status sfft_build_system_stamps(sfft_handle handle, const sfft_desc* desc,
                                     const void* ref, const void* sci,
                                     const int32_t* centers, int32_t n_stamps, int32_t size,
                                     double* G, double* h,
                                     void* ws, size_t ws_bytes, void* stream);

/* Least-squares background for given kernel coefficients: with the kernel
 * part of coef (indices < n(DK) L^2) held fixed, overwrite the background
 * part with b = G_bb^-1 (h_b - G_kb^T a), the exact minimiser of the problem
 * above over the background alone (the kernel-background block, background
 * block and background right-hand side, from polynomial moments of R' and S'
 * with periodic seam corrections; no transforms). Used by the learned form:
 * stamp pairs carry no information on the two images' sky levels.
 *   coef : device, N doubles (kernel part read, background part written;
 *          NaN if the background block is not positive definite)
 *   G, h : device scratch, N*N and N doubles (only the blocks named are written)
 *   ws   : device workspace of at least sfft_workspace_size bytes */
sfft_status sfft_refit_background(sfft_handle handle, const sfft_desc* desc, const void* ref,
                                  const void* sci, double* coef, double* G, double* h,
                                  void* ws, size_t ws_bytes, void* stream);

/* ---- Multi-template differencing -----------------------------------------
 * Paper Sec. 2.3.2 (image differencing) with the multi-exposure template set
 * of Sec. 2.2.1 (N_TEMP templates, default 5): the science image is
 * differenced against each template separately, every difference image is
 * brought to one common photometric zero point and the stack is
 * median-combined pixel by pixel. A difference image with zero point zp[t]
 * is scaled by 10^(0.4 (zp_common - zp[t])) (magnitudes m = zp - 2.5
 * log10(flux)); the median of an even count is the mean of the two middle
 * values; a NaN in any input gives NaN. At most SFFT_MAX_TEMPLATES images. */
#define SFFT_MAX_TEMPLATES 16

/* out = median_t( scale_t * diffs[t] ). diffs: host array of n device
 * pointers to W x H images (image_dtype, pitch ld of desc; only width,
 * height, ld and image_dtype are used); zp: host array of n zero points;
 * out: device image of the same layout (may alias none of the inputs). */
sfft_status sfft_median_combine(sfft_handle handle, const sfft_desc* desc, const void* const* diffs,
                                int32_t n, const double* zp, double zp_common, void* out,
                                void* stream);

/* The whole multi-template path for one science image: for each template t,
 * sfft_build_system (reference refs[t], pedestal ref_pedestals[t] when that
 * host array is non-NULL, else desc's), sfft_solve (max_refine steps) and
 * sfft_subtract into diffs[t] with its chi2, then sfft_median_combine into
 * `combined`. The science image's row spectrum is computed by the first
 * template's build and reused by the others (when the workspace layout keeps
 * it across the solve; otherwise every build transforms it again). All
 * templates share desc's L, DK, DB, compute, convention and science pedestal.
 *   refs, diffs : host arrays of n device image pointers (diffs written)
 *   G, h        : device scratch, N*N and N doubles (hold the last template's system)
 *   coefs       : device, n*N doubles (template t at t*N)
 *   infos       : device, n sfft_solve_info; chi2s: device, n doubles
 *   combined    : device image (written)
 *   ws          : device workspace of at least sfft_workspace_size(desc) bytes
 * Errors as for the single-pair calls; n outside [1, SFFT_MAX_TEMPLATES]
 * or aliased outputs: SFFT_ERR_INVALID_ARG. */
sfft_status sfft_difference_multi(sfft_handle handle, const sfft_desc* desc, const void* const* refs,
                                  const void* sci, int32_t n, const double* ref_pedestals,
                                  const double* zp, double zp_common, int32_t max_refine,
                                  double* G, double* h, double* coefs, sfft_solve_info* infos,
                                  double* chi2s, void* const* diffs, void* combined,
                                  void* ws, size_t ws_bytes, void* stream);

/* ---- Aperture photometry on difference images ---------------------------
 * Paper Sec. 2.3.3 (differential photometry: aperture fluxes at random
 * background positions give the 5-sigma limiting magnitude) and Sec. 2.4.3
 * (forced aperture photometry at fixed positions). The flux in a circle of
 * `radius` pixels (0 < radius <= 64) centred on (x, y) is the sum over pixels
 * of the pixel value times the exact area of the pixel square
 * [px - 1/2, px + 1/2] x [py - 1/2, py + 1/2] inside the circle (pixel
 * centres at integer coordinates; pixels outside the image contribute
 * nothing), accumulated in FP64. Only width, height, ld and image_dtype of
 * desc are used. xy: device double[n][2] = (x, y); 1 <= n <= 2^24. */
sfft_status sfft_aperture_flux(sfft_handle handle, const sfft_desc* desc, const void* image,
                               const double* xy, int32_t n, double radius, double* flux,
                               void* stream);

/* Aperture fluxes at n >= 2 background positions (written to flux, device
 * double[n]) and result (device double[3]) = {sigma, m_lim, mean flux}:
 * sigma = sample standard deviation of the fluxes (n - 1 in the
 * denominator), m_lim = zp - 2.5 log10(nsigma * sigma) (nsigma = 5 for the
 * paper's 5-sigma limit). */
sfft_status sfft_limiting_magnitude(sfft_handle handle, const sfft_desc* desc, const void* image,
                                    const double* xy, int32_t n, double radius, double zp,
                                    double nsigma, double* flux, double* result, void* stream);

/* Forced photometry: flux (device double[n]); mag (nullable) = zp - 2.5
 * log10(flux), NaN for flux <= 0; mag_err (nullable; needs sigma, a device
 * scalar such as result[0] of sfft_limiting_magnitude) = (2.5 / ln 10)
 * sigma / |flux|, NaN for flux == 0. */
sfft_status sfft_forced_photometry(sfft_handle handle, const sfft_desc* desc, const void* image,
                                   const double* xy, int32_t n, double radius, double zp,
                                   const double* sigma, double* flux, double* mag, double* mag_err,
                                   void* stream);

/* ---- Real-bogus scorer (inference) ---------------------------------------
 * Paper Sec. 2.3.4: every candidate of a difference image is scored by a
 * rotation-invariant convolutional network with residual connections (after
 * ResNet-18) on a three-channel stamp (science, template, difference)
 * centred on it; output: the probability that it is real. The trained
 * weights and layer sizes are not published; this network (the reading used
 * here, weights supplied by the caller):
 *   the 3 x 32 x 32 stamp is rotated by 0, 90, 180, 270 degrees; each copy:
 *     conv 3x3 3->32 + ReLU; residual block (conv 3x3 32->32 + ReLU,
 *     conv 3x3 32->32, + block input, ReLU); block (conv 3x3 stride 2
 *     32->64 + ReLU, conv 3x3 64->64, + conv 1x1 stride 2 32->64 of the
 *     block input, ReLU); block (the same, 64->128); global average pool;
 *   mean of the four copies' 128 features (invariant under quarter turns);
 *   linear 128->64 + ReLU; linear 64->1 = logit; probability = sigmoid.
 * Convolutions: cross-correlation, zero padding 1 for 3x3; output (i, j)
 * reads input (s i + ky - 1, s j + kx - 1). They run on the bf16 matrix
 * cores: stamps, convolution weights and every activation are rounded to
 * bfloat16 (nearest even), sums in FP32; pooling and linear layers in FP32.
 * Parameters: one flat FP32 vector (sfft_rb_num_params() = 315009 values):
 * conv weights [out][in][3][3] (1x1: [out][in]) each followed by its bias,
 * in the order stem, block 1 (a, b), block 2 (a, b, projection), block 3
 * (a, b, projection); then fc1 [64][128], bias [64], fc2 [1][64], bias [1]. */
int64_t sfft_rb_num_params(void);

/* Device workspace bytes for sfft_rb_score on n candidates (1..16384). */
sfft_status sfft_rb_workspace_size(int32_t n, size_t* bytes);

/* stamps (device FP32 [n][3][32][32]): channel c of candidate k is
 * (I_c[cy - 16 + i][cx - 16 + j] - offsets[c]) * scales[c], I = (sci, ref,
 * diff) (periodic indices; only width, height, ld and image_dtype of desc
 * are used); centers: device int32 [n][2] = (cx, cy); offsets, scales: host
 * float[3]. */
sfft_status sfft_rb_extract(sfft_handle handle, const sfft_desc* desc, const void* sci, const void* ref,
                            const void* diff, const int32_t* centers, int32_t n, const float* offsets,
                            const float* scales, float* stamps, void* stream);

/* logits (device FP32 [n]) and, when probs is not NULL, probabilities of n
 * stamps; params: device FP32 [sfft_rb_num_params()]; ws: device workspace
 * of sfft_rb_workspace_size(n) bytes (packed bf16 weights and activations). */
sfft_status sfft_rb_score(sfft_handle handle, const float* params, const float* stamps, int32_t n,
                          float* logits, float* probs, void* ws, size_t ws_bytes, void* stream);

/* ---- Learned form ------------------------------------------------------
 * A small convolutional network predicts the kernel and background
 * coefficients of the fit from star-stamp pairs, so that a pair whose
 * predicted difference image passes the chi2 judge skips the build and the
 * solve (the paper's pipeline couples the differencing with learned models,
 * Sec. 2.3). Architecture, per stamp: conv 3x3 2->16 (stride 1), 16->32,
 * 32->64, 64->64 (stride 2), ReLU after each, linear 1024->128 ReLU; per
 * pair: pooled[i][c] = mean over stamps of p_i(xt, yt) h[c] for the six
 * monomials 1, xt, yt, xt^2, xt yt, yt^2 of the stamp centre; linear
 * 768->512 ReLU; linear 512->n_out. Convolutions: zero padding 1,
 * cross-correlation. Outputs are standardised coefficients
 * (coef = mean + scale * pred, see sfft_surrogate_destandardize).
 * Parameters: one flat FP32 device vector, in order conv1..conv4 (weight
 * [out][in][3][3], bias [out]), fc1, fc2, fc3 (weight [out][in], bias).
 * Stamps: FP32 [n][2][32][32] (reference, science); positions FP32 [n][2]
 * (xt, yt); the n_stamps stamps of a pair are contiguous.
 * Every reduction has a fixed order: results are bit-reproducible. */
typedef enum { SFFT_NET_FP32 = 0, SFFT_NET_BF16 = 1 } sfft_net_precision;

/* Number of parameters for n_out outputs (960812 for n_out = 732), -1 if invalid. */
int64_t sfft_surrogate_num_params(int32_t n_out);

/* Device workspace bytes for sfft_surrogate_forward / _grad at this shape
 * (n_pairs <= 4096, n_stamps <= 1024, n_pairs * n_stamps <= 2^20). */
sfft_status sfft_surrogate_workspace_size(int32_t n_pairs, int32_t n_stamps, int32_t n_out, size_t* bytes);

/* Stamp pairs for the network: the 32 x 32 windows [cx-16, cx+16) x
 * [cy-16, cy+16) of ref and sci (periodic), each minus the mean of its
 * window's border pixels, both divided by the reference window's
 * sky-subtracted sum (1 if not positive) and multiplied by 100; positions
 * xt = 2 cx / (W-1) - 1, yt = 2 cy / (H-1) - 1. centers: device int32 [n][2]. */
sfft_status sfft_extract_stamps(sfft_handle handle, const sfft_desc* desc, const void* ref,
                                const void* sci, const int32_t* centers, int32_t n,
                                float* stamps, float* pos, void* stream);

/* pred (device FP32 [n_pairs][n_out]) = network(params, stamps, pos).
 * precision SFFT_NET_BF16 rounds parameters, stamps and every activation to
 * bfloat16 (round to nearest even) and accumulates in FP32. */
sfft_status sfft_surrogate_forward(sfft_handle handle, const float* params, const float* stamps,
                                   const float* pos, int32_t n_pairs, int32_t n_stamps, int32_t n_out,
                                   int32_t precision, float* pred, void* ws, size_t ws_bytes,
                                   void* stream);

/* FP32 forward pass, loss = mean over pairs and outputs of (pred - target)^2
 * (device double), and the gradient of the loss with respect to every
 * parameter into grads (device FP32, parameter layout). */
sfft_status sfft_surrogate_grad(sfft_handle handle, const float* params, const float* stamps,
                                const float* pos, const float* target, int32_t n_pairs,
                                int32_t n_stamps, int32_t n_out, float* grads, double* loss,
                                void* ws, size_t ws_bytes, void* stream);

/* One Adam step (Kingma and Ba) on n parameters, step counted from 1:
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps). */
sfft_status sfft_surrogate_adam(sfft_handle handle, float* params, const float* grads, float* m,
                                float* v, int64_t n, int32_t step, float lr, float beta1,
                                float beta2, float eps, void* stream);

/* coef[b][j] = mean[j] + scale[j] pred[b][j] (FP64 out; mean, scale FP64 [n_out]). */
sfft_status sfft_surrogate_destandardize(sfft_handle handle, const float* pred, const double* mean,
                                         const double* scale, int32_t n_pairs, int32_t n_out,
                                         double* coef, void* stream);

/* Kernel timing hook (measurement support, not part of the method).
 * Kernels / launch groups that can be bracketed by events: */
typedef enum {
  SFFT_PROF_ROW_PASS = 1,     /* row DFTs + row moments (one kernel) */
  SFFT_PROF_COL_PASS = 2,     /* blocked y-correlation (one kernel) */
  SFFT_PROF_XINV = 3,         /* pruned x-inverse of the correlation strips (one kernel) */
  SFFT_PROF_SUBTRACT = 4,     /* convolve-and-subtract + chi2 partials (one kernel) */
  SFFT_PROF_SOLVE = 5,        /* every launch of sfft_solve */
  SFFT_PROF_BUILD = 6,        /* every launch of sfft_build_system */
  SFFT_PROF_STAMP_GRAM = 7,   /* stamp Gram sums on matrix cores (one kernel) */
  SFFT_PROF_MAX = 8
} sfft_prof_slot;

/* From now on, every call that launches `slot` records start_event
 * (a hipEvent_t created by the caller) on the call's stream immediately
 * before it and stop_event immediately after it. NULL events clear the slot.
 * Events must stay valid while set. SFFT_ERR_INVALID_ARG for a bad slot. */
sfft_status sfft_profile_events(sfft_handle handle, int32_t slot, void* start_event,
                                void* stop_event);

#ifdef __cplusplus
}
#endif

#endif /* SFFT_MI355X_SFFT_H */
