/*
 * mapmaker.h -- C ABI of the MI355X map-making library (libmapmaker.so).
 *
 * Solves the generalised-least-squares map-making system of Puglisi et al.
 * (2018), "Iterative map-making with two-level preconditioning for polarized
 * CMB data sets":
 *
 *     A x = b,   A = P^T N^-1 P,   b = P^T N^-1 d            (Eqs. estimator, linearsystem)
 *
 * with P the polarised pointing matrix (three non-zeros per row, 1, cos 2phi,
 * sin 2phi; Eq. datamodel), N^-1 a banded-Toeplitz inverse-noise matrix per
 * stationary interval (W = N^-1, Sect. 2), by preconditioned conjugate
 * gradients (Eq. pcg) with either the block-diagonal preconditioner M_BD
 * (Eq. mbd) or the two-level preconditioner
 *
 *     M_2l = M_BD (1 - A Z E^-1 Z^T) + Z E^-1 Z^T,   E = Z^T A Z   (Eq. m2l)
 *
 * whose deflation space Z is built from Ritz vectors of an Arnoldi run on
 * M_BD A (Sect. 6, Appendix A).
 *
 * Conventions
 *  - Every call returns mm_status.  MM_OK = 0.  MM_NOT_CONVERGED = 1 is a
 *    non-error outcome (solve info is filled).  Negative values are errors;
 *    the message is in mm_last_error(ctx).  Arguments are validated before
 *    any device work; an invalid argument leaves outputs untouched.
 *  - Array arguments marked [device] are device pointers on the context's
 *    device (e.g. a torch tensor's data_ptr()); [host] marks host pointers.
 *    The caller owns every array it passes; the library never frees them and
 *    keeps no reference to them after the call returns.
 *  - Handles (mm_ctx, mm_pointing, mm_noise, mm_precond) own all memory the
 *    library allocates; mm_*_destroy releases it.  A handle must be destroyed
 *    before the context that created it.
 *  - Work is enqueued on the HIP stream given at context creation.  Calls that
 *    return host-visible results (counts, status, solve info) synchronise that
 *    stream; others are asynchronous with respect to the host.
 *  - Map layout: pixel-major, I,Q,U interleaved, FP64: x[(3 j + a) * nrhs + r]
 *    for compact pixel j, Stokes a, right-hand side r.  n = 3 * n_obs.
 *  - TOD layout: time-major, x[t * nrhs + r]; FP64, or FP32 for an MM_F32
 *    pointing/noise pair.
 *  - nrhs (right-hand sides processed together) must be 1, 2, 4, 8, 16, 32
 *    or 64.  Columns are processed independently and in a fixed order, so a
 *    column's result does not depend on the values in the other columns.
 *  - Not thread safe per context: calls on one context must not overlap.
 *  - Sharing handles: a pointing, noise or preconditioner handle is read-only
 *    once its set-up calls are done (the build that created it, then
 *    mm_pointing_set_grid, mm_noise_set_fft_block, mm_autotune).  After that
 *    several contexts, on one host thread or several, may use it at the same
 *    time: every apply, solve and build reads it only, and each context
 *    works in its own stream and scratch.  A set-up call must not overlap
 *    any other use of the handle.  A PCG session belongs to its context.
 */
#ifndef MAPMAKER_H
#define MAPMAKER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MM_OK = 0,
    MM_NOT_CONVERGED = 1,
    MM_E_INVALID = -1,        /* bad argument (sizes, ranges, layout) */
    MM_E_OOM = -2,            /* device allocation failed */
    MM_E_DEVICE = -3,         /* HIP runtime error */
    MM_E_SINGULAR_BLOCK = -4, /* a 3x3 M_BD block is not invertible */
    MM_E_COARSE_NOT_SPD = -5, /* E = Z^T A Z is not positive definite */
    MM_E_BREAKDOWN = -6,      /* PCG: p^T A p <= 0 */
    MM_E_NONFINITE = -7,      /* NaN/Inf in an input */
    MM_E_BUSY = -8            /* request exceeds the configured memory budget */
} mm_status;

/* Precision of the time-domain work (TOD, pointing weights, N^-1 band and its
 * accumulation).  Map-domain vectors, reductions, the 3x3 M_BD inverses and
 * the coarse matrix E are always FP64. */
typedef enum { MM_F64 = 0, MM_F32 = 1 } mm_precision;

/* How N^-1 is applied: AUTO picks the FFT when the bandwidth allows it and
 * half_bw >= 32 (FP64 streams of 2^22 samples or more), >= 64 (FP32 streams
 * of that length) or >= 128 (shorter streams), the measured crossovers with
 * the direct band; else the direct band.  MM_NOISE_POLY marks a
 * weight built by mm_polyfilter_build (a template filter, not a band). */
typedef enum {
    MM_NOISE_AUTO = 0,
    MM_NOISE_DIRECT = 1,
    MM_NOISE_FFT = 2,
    MM_NOISE_POLY = 3
} mm_noise_method;

/* Map components.  IQU: a sample measures I + Q cos 2psi + U sin 2psi (Eq.
 * datamodel), 3 unknowns per pixel.  The sum and difference streams of a
 * detector pair with orthogonal polarisers separate the two (Sect. 4, Eqs.
 * d+ and d-): I (the sum stream, 1 unknown per pixel, weight 1) and QU (the
 * difference stream, 2 per pixel, weights cos 2psi, sin 2psi).  The map
 * layout keeps the components of a pixel together: x[(nc j + a) * nrhs + r]
 * with nc = 3, 1 or 2, and n = nc * n_obs. */
typedef enum { MM_STOKES_IQU = 0, MM_STOKES_I = 1, MM_STOKES_QU = 2 } mm_stokes;

typedef struct mm_ctx mm_ctx;
typedef struct mm_pointing mm_pointing;
typedef struct mm_noise mm_noise;
typedef struct mm_precond mm_precond;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to
 * enqueue on, or NULL for a stream the context creates (default priority). */
mm_status mm_ctx_create(int device, void *hip_stream, mm_ctx **out);
void mm_ctx_destroy(mm_ctx *ctx);
/* Message of the last failed call on this context ("" if none).  Owned by the
 * context; valid until the next call. */
const char *mm_last_error(const mm_ctx *ctx);
/* Library version string. */
const char *mm_version(void);

/* --------------------------------------------------------------- pointing */

/* Build P from per-sample pixels and angles (Eq. datamodel).  Samples with
 * pix = -1 are flagged.  Pixels with fewer than min_hits unflagged samples
 * are dropped and their samples flagged too (the paper keeps only pixels
 * observed with enough redundancy, Sect. 5).  Observed pixels get compact
 * ids 0..n_obs-1 in ascending global id.
 *   n_samp       number of samples, 0 < n_samp < 2^31
 *   n_pix_total  number of global pixels; pix must lie in [-1, n_pix_total)
 *   pix  [device] int32[n_samp];  psi [device] f64[n_samp], radians
 *   prec         precision of the stored weights (cos 2psi, sin 2psi)
 * Errors: MM_E_INVALID (sizes, pixel out of range), MM_E_NONFINITE (psi). */
mm_status mm_pointing_build(mm_ctx *ctx, int64_t n_samp, int32_t n_pix_total,
                            const int32_t *pix, const double *psi, int32_t min_hits,
                            mm_precision prec, mm_pointing **out);
/* The same for the map components `stokes` (mm_pointing_build is
 * MM_STOKES_IQU).  With MM_STOKES_I, psi may be NULL (it is not used).
 * M_BD on such a pointing has 1x1 (I) or 2x2 (QU) blocks; every operator and
 * solver takes maps of n = nc * n_obs entries.  Errors: as mm_pointing_build,
 * and MM_E_INVALID for an unknown `stokes` or a NULL psi with QU or IQU. */
mm_status mm_pointing_build_stokes(mm_ctx *ctx, int64_t n_samp, int32_t n_pix_total,
                                   const int32_t *pix, const double *psi, int32_t min_hits,
                                   mm_precision prec, mm_stokes stokes, mm_pointing **out);
/* The pointing's map components and their count nc (3, 1 or 2).  [host] outputs. */
mm_status mm_pointing_stokes(const mm_pointing *p, mm_stokes *stokes, int32_t *nc);
/* Sum and difference streams of a detector pair (Eqs. d+ and d-):
 * plus_t = (a_t + b_t) / 2, minus_t = (a_t - b_t) / 2.  a, b are the two
 * detectors' time-aligned streams, [device] f64 or f32 (prec) [n]; plus and
 * minus [device] of the same type (either may be NULL; they may alias a or b
 * element for element).  Errors: MM_E_INVALID (n < 0, null inputs). */
mm_status mm_pair_sum_diff(mm_ctx *ctx, int64_t n, mm_precision prec, const void *a,
                           const void *b, void *plus, void *minus);
/* Optional locality hint: the global pixel ids are row-major on a grid of
 * `width` columns (id = row * width + column).  The one-wave-per-pixel P^T
 * then visits the pixels in 32 x 32 tiles of that grid, so the pixels reduced
 * together are hit by the same stretches of the scan and share cache lines.
 * The
 * single-column IQU P (FP64 and FP32) gathers from up to 4 copies of the
 * map, one per scan direction found in the samples (chunks of 4,096 samples
 * vote by their displacement over 8 samples), each ordered by the first
 * sample of its chunks that hits each pixel, so the lanes of a wave, which
 * take consecutive samples along the scan, read few cache lines.  The
 * sliced single-column P^T is then cut by the same directions: each
 * direction's slices take 64 pixels in that copy's order, a lane sums its
 * pixel's samples of that direction in time order per segment, and the
 * (segment, direction) partial maps are added in a fixed order.  P gathers
 * the same values, so P is bitwise unchanged; with one direction (or
 * without the sliced form) P^T and A are bitwise unchanged too; with
 * several, P^T sums each pixel's samples in another fixed order: bitwise
 * repeatable, equal to the unhinted result to rounding.  width = 0
 * restores ascending order and one map copy.
 * Errors: MM_E_INVALID (negative width). */
mm_status mm_pointing_set_grid(mm_ctx *ctx, mm_pointing *p, int32_t width);
/* Map copies the single-column IQU P gathers from: 0 without a grid (one
 * copy in compact id order), else 1 to 4.  [host] output. */
mm_status mm_pointing_p_layout(const mm_pointing *p, int32_t *copies);
/* n_obs (observed pixels) and n_valid (unflagged samples).  [host] outputs. */
mm_status mm_pointing_counts(const mm_pointing *p, int32_t *n_obs, int64_t *n_valid);
/* Execution layout of the single-column P^T (Eq. mapmaking's P^T as a
 * pixel-sorted reduction): *slices = pixel slices of 64 (over all scan
 * directions when the grid hint cuts them by direction) and *segments = time
 * segments of the sliced form, both 0 when the problem is small enough for
 * the one-wave-per-pixel form.  Each pixel sums its samples in time order
 * within a segment (and scan direction), then those partial sums in order;
 * the layout is a function of the pointing (n_obs, n_valid, the directions
 * found), never of the device.  [host] outputs. */
mm_status mm_pointing_pt_layout(const mm_pointing *p, int32_t *slices, int32_t *segments);
/* Hit counts per global pixel and the observed pixels' global ids.
 *   hits [device] int32[n_pix_total]; obs_pix [device] int32[n_obs] (either may be NULL) */
mm_status mm_pointing_hits(mm_ctx *ctx, const mm_pointing *p, int32_t *hits, int32_t *obs_pix);
/* The sample-to-pixel structure: j [device] int32[n_samp] compact pixel per
 * sample (-1 = flagged); perm [device] int32[n_valid] samples sorted by
 * (pixel, time); off [device] int32[n_obs+1] segment offsets (any may be NULL). */
mm_status mm_pointing_export(mm_ctx *ctx, const mm_pointing *p, int32_t *j, int32_t *perm,
                             int32_t *off);
void mm_pointing_destroy(mm_pointing *p);

/* ------------------------------------------------------------------ noise */

/* Banded-Toeplitz N^-1, block diagonal over stationary intervals: for t in
 * interval i = [s_i, s_{i+1}) with filter f = filter_id[i],
 *     (N^-1 y)_t = sum_{u in [s_i, s_{i+1}), |t-u| <= half_bw} c^f_{|t-u|} y_u.
 *   interval_start [host] int64[n_intervals+1], s_0 = 0, strictly increasing
 *   filter_id [host] int32[n_intervals] in [0, n_filters)
 *   band [host] f64[n_filters][half_bw+1] = c_0..c_lambda of each filter
 * Errors: MM_E_INVALID if intervals do not tile [0, s_n) or
 * 2 * half_bw >= the shortest interval; MM_E_NONFINITE for NaN/Inf bands. */
mm_status mm_noise_build(mm_ctx *ctx, int32_t n_intervals, const int64_t *interval_start,
                         const int32_t *filter_id, int32_t n_filters, int32_t half_bw,
                         const double *band, mm_noise_method method, mm_precision prec,
                         mm_noise **out);
/* Template filter as the time-domain weight, in place of N^-1 (Sect. 2, Eqs.
 * filt and filtnoise; Sect. 4: long modes are removed by low-order
 * polynomials per subscan, the remaining noise taken as white, and ground
 * pickup by azimuth-binned templates).  Polynomial part:
 *     F_B = W - W B (B^T W B)^-1 B^T W,
 * B block diagonal over subscans, each block the Legendre polynomials of
 * degree 0..order of the subscan time mapped onto [-1, 1] (F depends only on
 * their span); W = diag(w), w_t = weight of the sample's interval times the
 * flag mask of pointing p (flagged samples neither weigh in a fit nor receive
 * output).  A subscan with at most order + 1 weighted samples is fitted
 * exactly: its output is 0.  Ground part (optional): G[t, b] = 1 when sample
 * t falls in azimuth bin b; F_G is the same formula with G, i.e. each bin's
 * w-weighted mean is removed (a bin without weight removes nothing).  With
 * both, the filter is the symmetric combination of Sect. 4,
 *     F = F_B W^+ F_G W^+ F_B    (W^+ zero on flagged samples).
 * M_BD built on this handle uses diag(W) (Eq. mbd), and A = P^T F P,
 * b = P^T F d follow (Eqs. unb, linearsystem).
 *   p               the pointing (its n_samp, precision and flags)
 *   interval_start  [host] int64[n_intervals+1], tiles [0, n_samp)
 *   weight          [host] f64[n_intervals] >= 0 (inverse white-noise variance)
 *   subscan_start   [host] int64[n_subscans+1], tiles [0, n_samp); every
 *                   subscan lies inside one interval
 *   order           0..7
 *   ground_bin      [device] int32[n_samp] azimuth bin of each sample in
 *                   [0, n_ground_bins), -1 = in no bin; NULL = no ground part
 *   n_ground_bins   number of bins (0 when ground_bin is NULL)
 * The handle keeps copies (it does not refer to p or ground_bin afterwards).
 * Errors: MM_E_INVALID (tiling, a subscan across intervals, order, weight < 0,
 * a bin outside [-1, n_ground_bins)), MM_E_NONFINITE (weight). */
mm_status mm_polyfilter_build(mm_ctx *ctx, const mm_pointing *p, int32_t n_intervals,
                              const int64_t *interval_start, const double *weight,
                              int64_t n_subscans, const int64_t *subscan_start, int32_t order,
                              const int32_t *ground_bin, int32_t n_ground_bins,
                              mm_noise **out);
/* The method actually used (MM_NOISE_DIRECT, MM_NOISE_FFT or MM_NOISE_POLY). */
mm_status mm_noise_method_used(const mm_noise *nz, mm_noise_method *method);
/* Overlap-save block geometry of the FFT method (a way of applying the
 * banded W = N^-1 of Sect. 2: each interval's Toeplitz block as circulant
 * products of blocks): each block transforms *n_fft samples and keeps
 * *n_valid = *n_fft - 2 lambda outputs.  Both 0 for the direct method.
 * *n_fft is 16,384 (lambda <= 6,144; two blocks share a compute unit) or
 * 32,768 (one block per compute unit), picked at build by a measured time
 * model (blocks run in waves over the compute units; a wave of the large
 * blocks takes 1.1 times as long), so it depends on the interval lengths,
 * lambda and the device's compute-unit count; mm_noise_set_fft_block and
 * mm_autotune can change it. */
mm_status mm_noise_fft_block(const mm_noise *nz, int32_t *n_fft, int32_t *n_valid);
/* Rebuild the FFT method's tables for blocks of n_fft real samples: 16,384
 * (lambda <= 6,144) or 32,768, or 0 for the time model's pick.  Results are
 * the same to rounding (<= 1e-11 relative in FP64), not bitwise.  The handle
 * is modified: no other call may use it meanwhile.  Errors: MM_E_INVALID for
 * a non-FFT handle or an unsupported size. */
mm_status mm_noise_set_fft_block(mm_ctx *ctx, mm_noise *nz, int32_t n_fft);
/* z = N^-1 y (or z = F y for a template filter) on the TOD layout.  y, z
 * [device], TOD precision, distinct. */
mm_status mm_noise_apply(mm_ctx *ctx, const mm_noise *nz, int32_t nrhs, const void *y, void *z);
void mm_noise_destroy(mm_noise *nz);

/* ------------------------------------------------------------- operators */

/* y = P x (map -> TOD).  x [device] f64 map layout; y [device] TOD layout and
 * precision. */
mm_status mm_apply_P(mm_ctx *ctx, const mm_pointing *p, int32_t nrhs, const double *x, void *y);
/* x = P^T z (TOD -> map), a deterministic pixel-sorted segmented reduction.
 * z [device] TOD layout/precision; x [device] f64 map layout. */
mm_status mm_apply_PT(mm_ctx *ctx, const mm_pointing *p, int32_t nrhs, const void *z, double *x);
/* y = A x = P^T N^-1 P x (matrix-free; Eq. linearsystem).  x, y [device] f64
 * map layout, distinct.  The pointing and noise must have the same precision
 * and n_samp. */
mm_status mm_apply_A(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz, int32_t nrhs,
                     const double *x, double *y);
/* y = A x as mm_apply_A, allocating nothing: for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The temporaries (two TOD vectors of
 * nrhs columns and the largest stage scratch) live in one static device
 * array per GPU of mm_apply_A_noalloc_max_bytes() bytes (128 MiB; about 4e6
 * FP64 or 8e6 FP32 samples at nrhs = 1), held until the process ends.
 * Same kernels and bitwise the same result as mm_apply_A.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * contexts or threads) race, and must be serialised by the caller.
 *   scratch_used [host] or NULL: bytes of scratch this call needs.
 * Errors: MM_E_INVALID (as mm_apply_A, or a problem needing more scratch than
 * the maximum; use mm_apply_A there).  Per-stage profiling is not recorded. */
mm_status mm_apply_A_noalloc(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                             int32_t nrhs, const double *x, double *y, size_t *scratch_used);
/* Size in bytes of the static scratch array of mm_apply_A_noalloc. */
size_t mm_apply_A_noalloc_max_bytes(void);
/* b = P^T N^-1 (mask . d): flagged samples are zeroed before weighting.
 * tod [device] TOD precision, layout [nrhs][n_samp] (each realisation
 * contiguous); b [device] f64 map layout.  Errors: MM_E_NONFINITE. */
mm_status mm_rhs(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz, int32_t nrhs,
                 const void *tod, double *b);

/* --------------------------------------------------------- preconditioners */

/* M_BD: the 3x3 blocks B_j = sum_{t in j} c_0^{f(t)} w_t w_t^T (Eq. mbd, with
 * diag(N^-1) = the zero-lag coefficient c_0 of the sample's interval), each
 * inverted in FP64.  Errors: MM_E_SINGULAR_BLOCK if a block is not positive
 * definite or its 1-norm reciprocal condition number is below 1e-12. */
mm_status mm_mbd_build(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz, mm_precond **out);
/* Smallest 1-norm reciprocal condition number over the 3x3 blocks. */
mm_status mm_mbd_rcond(const mm_precond *M, double *rcond_min);

/* Arnoldi diagnostics of mm_defl_build. */
typedef struct {
    int32_t m;            /* Arnoldi steps taken */
    int32_t k;            /* deflation vectors kept */
    double h_last;        /* h_{m+1,m} at exit */
    double setup_seconds; /* wall time of the whole build */
} mm_arnoldi_info;

/* Arnoldi stop rules (Appendix A; the paper stops once the error term of
 * Eq. factoriz, h_{m+1,m} w_{m+1} e_m^T, falls below eps_Arn):
 *   MM_ARN_STOP_H         h_{j+1,j} <= eps_arn, the test of the algorithm box;
 *   MM_ARN_STOP_RESIDUAL  the error term applied to the Arnoldi solution of
 *                         B x = r_0, h_{j+1,j} |(H_j^-1 e_1)_j|, relative to
 *                         ||r_0||, <= eps_arn (the reading under which a lower
 *                         eps_Arn solves the system to that residual, Sect. 6).
 * Both also stop when h_{j+1,j} = 0 (an invariant Krylov space). */
enum { MM_ARN_STOP_H = 0, MM_ARN_STOP_RESIDUAL = 1 };

/* M_2l from Ritz vectors (Sect. 6, Appendix A): Arnoldi on B = M_BD A from
 * r_0 = M_BD b_seed, classical Gram-Schmidt applied twice, until
 * h_{j+1,j} <= eps_arn or m_max steps; eigenpairs of H_m ordered by real
 * part; keep the k smallest (k+1 rather than split a complex pair) or, if
 * eps_lambda > 0, all with Re(theta) < eps_lambda; Z = orthonormalised
 * W_m [Re y | Im y]; E = Z^T A Z (FP64 MFMA), Cholesky-factorised on device.
 * A Z comes from the Arnoldi factorisation B W_m = W_{m+1} Hbar_m (Eq.
 * factoriz), A W_m = M_BD^-1 W_{m+1} Hbar_m, instead of k applies of A: the
 * same matrix up to rounding.
 *   mbd       an M_BD handle built for the same pointing and noise
 *   b_seed    [device] f64[n] start vector seed (typically b)
 *   h_history [host] f64[m_max] or NULL: h_{j+1,j} per step
 *   info      [host] or NULL
 * Errors: MM_E_INVALID (k, m_max), MM_E_COARSE_NOT_SPD. */
mm_status mm_defl_build(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                        const mm_precond *mbd, const double *b_seed, int32_t k,
                        double eps_lambda, double eps_arn, int32_t m_max,
                        double *h_history, mm_arnoldi_info *info, mm_precond **out);
/* mm_defl_build with a chosen Arnoldi stop rule (MM_ARN_STOP_*);
 * mm_defl_build is this call with MM_ARN_STOP_H and res_history NULL.
 *   b_seed      r_0 = M_BD b_seed: b for x_0 = 0, b - A x_0 for a guess x_0
 *   res_history [host] f64[m_max] or NULL: the Arnoldi solution's relative
 *               residual h_{j+1,j} |(H_j^-1 e_1)_j| per step (+inf where H_j is
 *               singular), whichever rule stops the run
 * Errors: as mm_defl_build; MM_E_INVALID for an unknown stop rule. */
mm_status mm_defl_build_stop(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                             const mm_precond *mbd, const double *b_seed, int32_t k,
                             double eps_lambda, double eps_arn, int32_t stop_rule, int32_t m_max,
                             double *h_history, double *res_history, mm_arnoldi_info *info,
                             mm_precond **out);
/* M_2l from the Ritz vectors of a prior M_BD solve: PCG with M_BD on
 * A x = b from x_0 = 0 (Eq. pcg) until ||r||/||b|| <= tol or m_max
 * iterations, whose coefficients give the
 * Lanczos tridiagonal of B = M_BD A, T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
 * T_{j,j+1} = -sqrt(beta_j)/alpha_j, with Lanczos vectors z_j / sqrt(r_j.z_j)
 * (orthonormal in the M_BD^-1 inner product).  The Ritz selection, V = V_m Y
 * and the orthonormal Z follow mm_defl_build, except that numerically
 * dependent Ritz vectors are dropped (finite-precision Lanczos repeats
 * converged Ritz values), so info->k may be below k; AZ and E as there.  Same
 * Krylov space as mm_defl_build's Arnoldi from M_BD b, with the CG inner
 * product and no Gram-Schmidt.
 *   b [device] f64[n]; theta [host] f64[m_max] Ritz values ascending (or NULL)
 *   x_out [device] f64[n] or NULL: the prior solve's solution (its iterate
 *         after the last step), so the first solve and the deflation space
 *         come from one run
 *   info [host]: m = Lanczos steps, k, h_last = |T_{m,m+1}|, setup time
 * Errors: as mm_defl_build; MM_E_BREAKDOWN if p^T A p <= 0. */
mm_status mm_defl_build_pcg(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                            const mm_precond *mbd, const double *b, int32_t k,
                            double eps_lambda, double tol, int32_t m_max, double *theta,
                            double *x_out, mm_arnoldi_info *info, mm_precond **out);
/* M_2l from a caller-supplied deflation matrix (Eq. m2l).
 *   Z [device] f64[k][n] column-major (column c at Z + c*n), 1 <= k <= 64.
 * Errors: MM_E_COARSE_NOT_SPD if Z^T A Z is not (numerically) SPD: a Cholesky
 * pivot^2 below 1e-13 times the largest diagonal entry. */
mm_status mm_defl_from_Z(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                         const mm_precond *mbd, int32_t k, const double *Z, mm_precond **out);
/* The "simplified" two-level preconditioner of the divide-and-conquer runs
 * (Sect. 7.3): the deflation vectors of an M_2l built on one data subset
 * (src, over p_src's observed pixels) reused on another subset's system.
 * Rows are matched by global pixel id; pixels p_src did not observe get 0.
 * A Z and E = Z^T A Z are then rebuilt with this subset's A (p, nz), and
 * M_BD is this subset's (mbd).  Z is not re-orthonormalised (only span(Z)
 * enters M_2l).  Both pointings must hold the same Stokes components.
 * Errors: MM_E_INVALID for mismatched handles; MM_E_COARSE_NOT_SPD as
 * mm_defl_from_Z (e.g. when the subsets share too few pixels). */
mm_status mm_defl_transfer(mm_ctx *ctx, const mm_pointing *p_src, const mm_precond *src,
                           const mm_pointing *p, const mm_noise *nz, const mm_precond *mbd,
                           mm_precond **out);
/* Copy out Z, A Z ([device] f64[k][n] each, either may be NULL) and E
 * ([device] f64[k][k], symmetrised). */
mm_status mm_defl_export(mm_ctx *ctx, const mm_precond *M, int32_t *k, double *Z, double *AZ,
                         double *E);
/* Arnoldi basis and Hessenberg matrix of the last mm_defl_build on this
 * handle: W [device] f64[m+1][n] column-major, H [host] f64[(m+1) * m]
 * column-major (either may be NULL). */
mm_status mm_defl_arnoldi_export(mm_ctx *ctx, const mm_precond *M, int32_t *m, double *W,
                                 double *H);
/* out = M v for an M_BD or M_2l handle.  v, out [device] f64 map layout, distinct. */
mm_status mm_precond_apply(mm_ctx *ctx, const mm_precond *M, int32_t nrhs, const double *v,
                           double *out);
void mm_precond_destroy(mm_precond *M);

/* ------------------------------------------------------------------ solve */

typedef struct {
    int32_t iters;             /* PCG iterations taken */
    int32_t converged;         /* 1 if ||r||/||b|| <= tol */
    int32_t breakdown;         /* 1 if p^T A p <= 0 stopped the column */
    int32_t pad;
    double rel_res_recursive;  /* ||r_k|| / ||b|| from the recursion */
    double rel_res_true;       /* ||b - A x_k|| / ||b|| recomputed at exit */
    double solve_seconds;      /* wall time of the solve (all columns) */
    double rel_res_precond;    /* ||M (b - A x_k)|| / ||M b|| at exit: Eq. residuals
                                  read literally (= rel_res_true when M is NULL) */
} mm_solve_info;

/* PCG flags */
#define MM_SOLVE_CHECK_EVERY(c) ((c) & 0xff)  /* host convergence poll period (0 = 1) */
#define MM_SOLVE_GRAPH (1u << 8) /* replay each poll period's iterations as one captured HIP graph */
#define MM_SOLVE_BLOCK (1u << 9) /* block PCG over the nrhs columns (O'Leary), nrhs >= 2 */
#define MM_SOLVE_FLEXIBLE (1u << 10) /* beta = r'.(z' - z) / rho (Polak-Ribiere), for a
                                        preconditioner that is not symmetric, such as
                                        M_2l; not with MM_SOLVE_BLOCK */

/* Preconditioned conjugate gradients (Eq. pcg), column-independent for
 * nrhs > 1 (with MM_SOLVE_BLOCK: block PCG, O'Leary 1980, whose search space
 * is the block Krylov space of all columns; its Gram and block products run
 * on FP64 MFMA and numerically dependent directions are dropped):  r = b - A x; z = M r; p = z; rho = r.z; repeat q = A p;
 * alpha = rho / p.q; x += alpha p; r -= alpha q; z = M r; rho' = r.z;
 * beta = rho'/rho; p = z + beta p -- until ||r|| / ||b|| <= tol (the
 * unpreconditioned residual, Sect. 7.1) or max_iter.  M may be NULL (no
 * preconditioner), an M_BD or an M_2l handle.
 *   b [device] f64 map layout; x [device] in: x_0, out: solution
 *   history [host] f64[nrhs][max_iter+1] or NULL: ||r_k||/||b|| per column
 *   info [host] mm_solve_info[nrhs] or NULL
 * Returns MM_OK if every column converged, MM_NOT_CONVERGED otherwise,
 * MM_E_BREAKDOWN if a column broke down. */
mm_status mm_solve(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz, const mm_precond *M,
                   int32_t nrhs, const double *b, double *x, double tol, int32_t max_iter,
                   uint32_t flags, double *history, mm_solve_info *info);

/* Mixed-precision iterative refinement: the true residual in the precision
 * of (p_hi, nz_hi) (FP64), corrections solved by PCG with (p_lo, nz_lo)
 * (typically the FP32 form) and M.  From x (in: x0, out: x):
 *   repeat  r = A_hi x - b (one A_hi apply per outer step, stop when every
 *           column has ||r|| / ||b|| <= tol); solve A_lo e = r by mm_solve to
 *           the relative accuracy the remaining gap needs, max(inner_tol,
 *           tol / (2 max_c ||r_c|| / ||b_c||)) capped at 0.5 (at most
 *           max_inner iterations); x -= e.
 * It reaches residuals the FP32 PCG stalls above (its recursion drifts from
 * the FP64 residual near 5e-8).  Both pointings must hold the same observed
 * pixels and Stokes components (built from the same pix), both noise handles
 * the same samples; b, x [device] f64 map layout, nrhs columns.
 *   info [host] mm_refine_info or NULL.
 * Returns MM_OK when every column reaches tol, MM_NOT_CONVERGED after
 * max_outer steps; errors as mm_solve. */
typedef struct {
    int32_t outer;          /* outer steps (A_hi applies after the first) */
    int32_t inner_iters;    /* PCG iterations summed over the outer steps (max over columns) */
    int32_t converged;      /* 1 if every column reached tol */
    int32_t pad;
    double rel_res_true;    /* max over columns of ||b - A_hi x|| / ||b|| at exit */
    double solve_seconds;
} mm_refine_info;
mm_status mm_solve_refined(mm_ctx *ctx, const mm_pointing *p_lo, const mm_noise *nz_lo,
                           const mm_pointing *p_hi, const mm_noise *nz_hi, const mm_precond *M,
                           int32_t nrhs, const double *b, double *x, double tol, double inner_tol,
                           int32_t max_outer, int32_t max_inner, mm_refine_info *info);

/* ------------------------------------------------- step-wise PCG sessions */

/* A PCG session holds nrhs column slots that iterate in lockstep with the
 * same pointing, noise and preconditioner; each slot carries its own
 * right-hand side, tolerance and iteration budget.  A slot can be (re)started
 * while other slots are mid-solve: this is the continuous-batching primitive
 * of the serving layer.  Column results do not depend on what the other
 * slots hold.  Iterations are Eq. pcg exactly as in mm_solve. */
typedef struct mm_pcg mm_pcg;

mm_status mm_pcg_create(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                        const mm_precond *M, int32_t nrhs, mm_pcg **out);
/* Start slot from x_0 = 0: r = b, z = M r, p = z.  b [device] f64[n]
 * (contiguous, one column).  tol: relative residual target; max_iter: budget. */
mm_status mm_pcg_start(mm_ctx *ctx, mm_pcg *s, int32_t slot, const double *b, double tol,
                       int32_t max_iter);
/* Run n_iter lockstep iterations over the live slots (finished and free slots
 * are skipped). */
mm_status mm_pcg_iterate(mm_ctx *ctx, mm_pcg *s, int32_t n_iter);
/* Replay iterations in captured HIP graphs of `chunk` iterations (0 = off).
 * The first iteration after creation runs eagerly; results are bitwise the
 * same as eager iterations. */
mm_status mm_pcg_use_graph(mm_ctx *ctx, mm_pcg *s, int32_t chunk);
/* Per-slot state [host] arrays of nrhs (any may be NULL): state 0 = free,
 * 1 = running, 2 = converged, 3 = iteration budget spent, 4 = breakdown;
 * iterations taken; recursive relative residual. */
mm_status mm_pcg_poll(mm_ctx *ctx, mm_pcg *s, int32_t *state, int32_t *iters, double *rel_res);
/* Copy a slot's current solution to x [device] f64[n] and free the slot. */
mm_status mm_pcg_finish(mm_ctx *ctx, mm_pcg *s, int32_t slot, double *x);
void mm_pcg_destroy(mm_pcg *s);

/* ---------------------------------------------------- small dense products */

/* The FP64 MFMA products of the two-level preconditioner and of block CG
 * (Eq. m2l: E = Z^T (A Z); the Ritz step Z = W_m Y of Sect. 6; the Gram and
 * update products of block PCG), exposed for callers that build their own
 * deflation spaces and for measurement.  All arrays [device] f64, distinct.
 * The sums run in a fixed order (bitwise repeatable).
 * C = X^T Y with X(i, a) = X[i x_rs + a x_cs], Y(i, b) likewise, i < n;
 * C [ka][kb] row-major; 1 <= ka, kb <= 64. */
mm_status mm_dense_gram(mm_ctx *ctx, int64_t n, int32_t ka, int32_t kb, const double *X,
                        int64_t x_rs, int64_t x_cs, const double *Y, int64_t y_rs, int64_t y_cs,
                        double *C);
/* Z = V Y: V n x kin and Z n x kout column-major (column c at + c n), Y
 * kin x kout column-major; kin >= 1, 1 <= kout <= 64. */
mm_status mm_dense_tall(mm_ctx *ctx, int64_t n, int32_t kin, int32_t kout, const double *V,
                        const double *Y, double *Z);
/* Out = beta Out + alpha In S for column-batched In, Out ([n][R], column
 * fastest) and S [R][R] row-major; R a power of two <= 64 (beta = 0 does not
 * read Out). */
mm_status mm_dense_rows(mm_ctx *ctx, int64_t n, int32_t R, const double *In, const double *S,
                        double alpha, double beta, double *Out);

/* ----------------------------------------------------------------- serving */

/* A serving engine for map-making solves of several recurring scan
 * strategies on one GPU, continuously batched.  Each strategy gets its own
 * context (HIP stream), pointing, noise and M_BD at registration, and a
 * two-level M_2l built from its first request's right-hand side and reused for
 * every later request of that strategy (Sect. 7.3: M_2l pays off when the
 * same system is solved many times).  The M_2l build runs on a host thread of
 * its own (own context and stream) and blocks no request: until it is ready,
 * requests of that strategy are solved with M_BD.  mm_server_step admits
 * queued requests into free column slots of the strategy's lockstep PCG
 * session for the current preconditioner -- also while other slots are
 * mid-solve; a lane's session is created (and charged against the budget)
 * when it admits its first request, and idle sessions are evicted when a
 * waiting request needs their memory -- runs `iters_per_step` iterations on
 * every session with running
 * slots (all streams enqueued before any is waited on, so strategies overlap
 * on the device), and retires finished slots into the caller's output
 * buffers.  A request's result does not depend on which other requests share
 * its session.  The server's calls are not thread safe (one caller thread). */
typedef struct mm_server mm_server;

typedef struct {
    int32_t state;          /* 0 queued, 1 running, 2 converged, 3 budget spent, 4 failed */
    int32_t iters;
    int32_t slot;
    int32_t m2l_built;      /* 1 if this request started the M_2l build (cache miss) */
    int32_t precond;        /* preconditioner it runs with: 0 M_BD, 1 M_2l; -1 queued */
    int32_t waited;         /* what it waited for before admission (bits): 1 a free slot
                               of its lane's session, 2 memory for that session */
    double rel_res;         /* recursive ||r|| / ||b|| at exit */
    double queue_seconds;   /* submit -> admitted */
    double latency_seconds; /* submit -> done (or now) */
} mm_request_info;

/* hbm_budget_bytes: cap on the library memory of the server: every
 * registered strategy's resident part plus every live lane session (see
 * mm_server_memory);
 * slots: columns per strategy session (1..64, power of two); defl_k: M_2l
 * deflation vectors (0 = M_BD only); iters_per_step: PCG iterations per step. */
mm_status mm_server_create(int device, int64_t hbm_budget_bytes, int32_t slots, int32_t defl_k,
                           int32_t iters_per_step, mm_server **out);
/* on != 0: strategies registered from now on get their M_2l at registration,
 * built synchronously on the strategy's stream from the Ritz vectors of an
 * M_BD solve (mm_defl_build_pcg, to 1e-12) of A x = A u with u a fixed
 * pseudo-random map, so every request of the strategy runs with M_2l;
 * registration takes that much longer.  Off (the default): M_2l is built in
 * the background from the first request's right-hand side. */
mm_status mm_server_set_prebuild(mm_server *srv, int32_t on);
/* Arnoldi of the background M_2l build (mm_defl_build_stop): stop rule
 * MM_ARN_STOP_*, eps_arn >= 0, m_max in [1, 500].  The default is
 * MM_ARN_STOP_H, 1e-8, 256.  Set before any strategy is registered (the
 * registration charges the Arnoldi basis of m_max + 1 vectors).
 * Errors: MM_E_INVALID (arguments, or strategies already registered). */
mm_status mm_server_set_arnoldi(mm_server *srv, int32_t stop_rule, double eps_arn, int32_t m_max);
/* Register a scan strategy; arguments as mm_pointing_build / mm_noise_build
 * (pix, psi [device] are read during the call only; grid_width as
 * mm_pointing_set_grid, 0 = none).  Errors: MM_E_BUSY if its estimated
 * resident footprint plus one lane session exceeds the budget left by the
 * other strategies' resident parts; the build errors otherwise. */
mm_status mm_server_add_strategy(mm_server *srv, int32_t id, int64_t n_samp, int32_t n_pix_total,
                                 const int32_t *pix, const double *psi, int32_t min_hits,
                                 int32_t grid_width, int32_t n_intervals,
                                 const int64_t *interval_start, const int32_t *filter_id,
                                 int32_t n_filters, int32_t half_bw, const double *band,
                                 mm_precision prec);
/* Queue a solve.  tod [device] (the strategy's TOD precision, n_samp values)
 * must stay valid until the request is admitted; x_out [device] f64[n]
 * receives the map when it is done.  request_id [host] out. */
mm_status mm_server_submit(mm_server *srv, int32_t strategy, const void *tod, double tol,
                           int32_t max_iter, double *x_out, int64_t *request_id);
/* One scheduling step; n_running, n_queued [host] or NULL. */
mm_status mm_server_step(mm_server *srv, int32_t *n_running, int32_t *n_queued);
/* State of a strategy's M_2l cache: 0 not started, 1 building, 2 ready,
 * 3 build failed (its requests keep M_BD).  [host] output. */
mm_status mm_server_strategy_state(mm_server *srv, int32_t strategy, int32_t *m2l_state);
mm_status mm_server_poll(mm_server *srv, int64_t request_id, mm_request_info *info);
/* Memory accounting [host] outputs, any may be NULL: the budget, the bytes in
 * use (resident parts of all strategies plus live sessions), and for
 * `strategy` its resident bytes (pointing, noise, M_BD, M_2l build reserve,
 * charged at registration) and the bytes of one lane session (`slots`
 * columns of PCG vectors and TOD workspaces, charged when the lane admits its
 * first request and released when the idle session is evicted to make room
 * for another). */
mm_status mm_server_memory(mm_server *srv, int32_t strategy, int64_t *budget, int64_t *used,
                           int64_t *resident, int64_t *session);
const char *mm_server_last_error(const mm_server *srv);
void mm_server_destroy(mm_server *srv);

/* -------------------------------------------------------------- autotuning */

/* Per-stage autotuner: for nrhs columns, time candidates with HIP events and
 * keep the fastest, stored in the handles for later calls with that nrhs
 * (the handles are modified: no other call may use them meanwhile).
 *   stage 0, P: the grid size;
 *   stage 1, direct band N^-1: taps per LDS chunk (less LDS per block, more
 *            blocks per compute unit);
 *   stage 2, P^T with several columns: tiled or ascending pixel order;
 *   stage 3, FFT N^-1, only with MM_TUNE_FFT_BLOCK in flags: the overlap-save
 *            block length (16,384 or 32,768; see mm_noise_set_fft_block).
 * Stages 0-2 change speed only: every output sums its terms in an order no
 * candidate changes, so results stay bitwise the same.  Stage 3 changes
 * results at the rounding level (<= 1e-11 relative in FP64).
 *   report [host] f64[3 * max_report] or NULL: (stage, candidate, ms) triples
 *   n_report [host] or NULL: entries written */
enum { MM_TUNE_FFT_BLOCK = 1 };
mm_status mm_autotune(mm_ctx *ctx, mm_pointing *p, mm_noise *nz, int32_t nrhs, int32_t flags,
                      double *report, int32_t max_report, int32_t *n_report);

/* ---------------------------------------------------------- profiling aid */

/* When on, each kernel of mm_apply_A / mm_solve is bracketed by HIP events on
 * the context's stream and its time accumulated per stage (P, N^-1, P^T,
 * precond, vector ops).  Stage names and totals via mm_profile_read. */
mm_status mm_profile_enable(mm_ctx *ctx, int on);
/* names [host] receives up to max entries of "name" (each <= 31 chars + NUL,
 * 32 bytes per entry), ms [host] total milliseconds, calls [host] launches.
 * *n receives the number of stages.  Resets the counters. */
mm_status mm_profile_read(mm_ctx *ctx, int32_t max, char *names, double *ms, int64_t *calls,
                          int32_t *n);

/* ---------------------------------------------------- host-only utilities */

/* Eigenvalues and eigenvectors of a real m x m upper Hessenberg matrix (the
 * Ritz step of Appendix A), host FP64: Francis double-shift QR for the
 * eigenvalues, inverse iteration for the vectors.  H [host] column-major
 * m x m (entries below the subdiagonal ignored); wr, wi [host] f64[m];
 * vr, vi [host] f64[m*m] column-major (eigenvector i in column i, unit
 * 2-norm; a real eigenvalue has vi column 0).  Needs no GPU. */
mm_status mm_hessenberg_eig(int32_t m, const double *H, double *wr, double *wi, double *vr,
                            double *vi);

#ifdef __cplusplus
}
#endif
#endif /* MAPMAKER_H */
