/*
 * xpcs.h -- C ABI of the MI355X (gfx950) library for homomorphically compressed
 * XPCS two-time correlation.
 *
 * Method: Strempfer et al., "Homomorphic data compression for real time photon
 * correlation analysis" (arXiv 2407.20356).  The two-time correlation of the
 * photon counts (Sec. 2.1, Eqs. 1-2) is computed either from the raw frames or
 * directly from a low-rank compression of them (Sec. 2.1, Eqs. 3-10) without
 * decompressing, and g2 is taken from its diagonals (Sec. 3.1, Eq. 12).
 *
 * Notation.  A series of N frames of M pixels is passed frame-contiguous: frame
 * t occupies elements [t*M, (t+1)*M) of `frames` (the paper's X, one flattened
 * image per row).  Read column-major, the same buffer is the pixel-by-frame
 * matrix X (M x N) of the formulas below.  A q-ROI R is a set of pixels given by
 * an int32 label per pixel (label r selects ROI r, -1 selects none; Sec. 2.2
 * compresses and analyses such pixel subsets directly).
 *
 * Conventions for every entry point.
 *  - Array arguments are DEVICE pointers owned by the caller; the library never
 *    frees, reallocates or retains them after the call returns.  Memory owned by
 *    the library is the workspace inside an xpcs_ctx (grown on demand, bounded by
 *    the context's HBM budget, released by xpcs_destroy).
 *  - Work is enqueued on the context's stream (xpcs_set_stream) and the call
 *    returns without waiting for the device, except where noted.  Calls on one
 *    context must be ordered on that stream: they share its workspace.
 *  - The return value is an xpcs_status.  A negative value means the call was
 *    rejected on the host and nothing was enqueued; xpcs_last_error() then
 *    describes the problem.  Conditions only the device can detect (a label
 *    outside [-1, n_roi), a count too large for the exact integer path, a
 *    numerically rank-deficient sketch) raise a device flag that the next
 *    xpcs_sync() reports.
 *  - Frames whose ROI photon sum is zero have no defined correlation: their rows
 *    and columns of C are NaN and they are left out of g2 and of its pair counts.
 */
#ifndef XPCS_H
#define XPCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t xpcs_status;
#define XPCS_OK 0
#define XPCS_EINVAL (-1)        /* bad argument (null pointer, size, label, dtype)      */
#define XPCS_ENOMEM (-2)        /* device allocation failed                             */
#define XPCS_ERANGE (-3)        /* reserved: a value outside what an exact path holds   */
#define XPCS_EBUDGET (-4)       /* the workspace would exceed the context's HBM budget  */
#define XPCS_EDEVICE (-5)       /* HIP runtime error or a failed device-side step      */
#define XPCS_EUNSUPPORTED (-6)  /* valid request outside what this build implements    */
#define XPCS_EQUEUED (-7)       /* the served stream still waits for admission          */

/* element type of the frames */
#define XPCS_U8 1
#define XPCS_U16 2
/* element type of a two-time matrix */
#define XPCS_F32 10
#define XPCS_F64 11
/* arithmetic of the compression products (FP32 accumulation in every case) */
#define XPCS_PREC_BF16 0
#define XPCS_PREC_FP8 1
#define XPCS_BASIS_RANDOMIZED 0
#define XPCS_BASIS_EXACT 1

/* `roi` argument selecting every ROI in one call */
#define XPCS_ALL_ROIS (-1)

typedef struct xpcs_ctx xpcs_ctx;

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * library-owned workspace (0 = no bound).  *out receives the context. */
xpcs_status xpcs_create(int device, size_t hbm_budget_bytes, xpcs_ctx **out);

/* Destroy a context: waits for its stream, frees its workspace.  NULL is a no-op. */
void xpcs_destroy(xpcs_ctx *ctx);

/* Bind the stream (a hipStream_t, NULL = the default stream) subsequent calls
 * enqueue on, e.g. torch.cuda.current_stream().cuda_stream. */
xpcs_status xpcs_set_stream(xpcs_ctx *ctx, void *hip_stream);

/* Wait for the context's stream, then report and clear device-side flags.
 * Returns XPCS_OK, XPCS_EINVAL (a label outside [-1, n_roi)) or XPCS_EDEVICE. */
xpcs_status xpcs_sync(xpcs_ctx *ctx);

/* Message for the last error on this context ("" if none).  Owned by the context. */
const char *xpcs_last_error(const xpcs_ctx *ctx);

/* Bytes of device workspace the context currently holds. */
size_t xpcs_workspace_bytes(const xpcs_ctx *ctx);

/* Diagnostics: device time per kernel phase.  When enabled (which also clears
 * earlier records), every entry point records a pair of HIP events on the
 * context's stream around each of its kernel phases.  xpcs_phase_times waits
 * for the stream and fills, for up to `cap` distinct phase names, the name
 * (NUL-terminated, at most 31 characters, in names[i*32]), the summed device
 * milliseconds and the number of launches since timing was enabled; *n_out
 * receives the number of phases filled.  names, ms and launches are host
 * memory of at least cap entries.  Recording costs a few microseconds of host
 * time per phase; it does not stall the device. */
xpcs_status xpcs_enable_phase_timing(xpcs_ctx *ctx, int32_t enable);
/* Restrict the recording to the phases whose names appear in `names` (host
 * string, comma-separated, e.g. "lowrank_tiles,raw_gram_tiles"); NULL or "" records
 * every phase again.  Applies from the next recorded phase on. */
xpcs_status xpcs_phase_filter(xpcs_ctx *ctx, const char *names);
xpcs_status xpcs_phase_times(xpcs_ctx *ctx, int32_t cap, char *names, double *ms, int64_t *launches,
                             int32_t *n_out);

/* Compressed state of one series: X ~= U diag(sigma) V^T plus the per-ROI data
 * the compressed correlation needs.  All buffers are caller-allocated device
 * memory of the sizes stated; compress_frames fills them.
 *   U        M x k floats, column-major (U[j*M + p]): the pixel basis, orthonormal
 *            columns -- the paper's encoding matrix V_K (Eq. 6).
 *   sigma    k doubles, descending: singular values (the paper calls the diagonal
 *            of Sigma its eigenvalues, Sec. 2.1 below Eq. 3).
 *   V        N x k floats, column-major (V[j*N + t]); W = V diag(sigma) = X^T U is
 *            the compressed data, the paper's Y_K (Eq. 7).
 *   roi_npix n_roi int64: pixel count |R| of each ROI.
 *   roi_sum  n_roi x N int64 (roi_sum[r*N + t]): exact photon sum of frame t over
 *            ROI r, recorded from the raw counts while encoding.
 *   roi_gram n_roi x k x k doubles (roi_gram[(r*k + a)*k + b]): G_R = U_R^T U_R,
 *            the basis restricted to the ROI's pixels. */
typedef struct {
    int64_t M, N;
    int32_t k, n_roi;
    float *U;
    double *sigma;
    float *V;
    int64_t *roi_npix;
    int64_t *roi_sum;
    double *roi_gram;
} xpcs_factors;

/* Options of compress_frames.
 *   k            rank kept (the paper's K, Eq. 6), 1 <= k.
 *   oversample   extra sketch columns p (sketch width l = k + p); 16 by default.
 *   power_iters  subspace iterations q (0 or 1).
 *   precision    XPCS_PREC_BF16, or XPCS_PREC_FP8 (offline mode, XPCS_U8 frames
 *                only): the subspace passes that choose the basis (the sketch
 *                X Omega and, with q = 1, X^T Q and X Z) take e4m3 operands -- the
 *                counts as two exact nibble planes, the +-1 sketch exactly, the
 *                intermediate bases rounded to e4m3 -- on the fp8 MFMA; the
 *                encoding pass keeps the split-bf16 basis either way.  With q = 0
 *                both precisions give the same factors (every rounded operand is
 *                exact).  XPCS_PREC_FP8 with XPCS_U16 frames: EUNSUPPORTED.
 *   seed         seed of the Rademacher sketch Omega[t][j] = +-1, sign = top bit of
 *                SplitMix64(seed XOR (t*2^32 + j)).
 *   basis        NULL: offline mode, the basis is computed from these frames
 *                (Sec. 2.2, "offline").  Non-NULL: online mode, an M x k
 *                column-major device basis generated beforehand (Sec. 2.2,
 *                "online"); it is copied to out->U and the frames are only
 *                encoded; sigma_j = |W e_j| and V = W diag(1/sigma).
 *   method       offline mode: XPCS_BASIS_RANDOMIZED (above), or XPCS_BASIS_EXACT:
 *                the paper's own construction (Sec. 2.1, Eqs. 3 and 6) -- the
 *                exact N x N frame Gram F F^T (FP64 MFMA over the integer counts,
 *                exact while every sum stays below 2^53: always for uint8, for
 *                uint16 when M * amax^2 < 2^53), its full FP64 eigendecomposition
 *                (block Jacobi), the k leading eigenvectors as V (largest-magnitude
 *                entry positive), sigma = sqrt(eigenvalue) and the basis
 *                U = X V diag(1/sigma) in FP64.  k = N (with M >= N) is the
 *                lossless mode of Eq. 11: C~ equals the raw C.  N <= 4096;
 *                oversample, power_iters, precision and seed are not used.
 *   spectrum     NULL, or (XPCS_BASIS_EXACT) device, N doubles: every eigenvalue of
 *                the frame Gram in decreasing order (the input of the rank rule
 *                of Sec. 3.1, xpcs_rank_rule). */
typedef struct {
    int32_t k;
    int32_t oversample;
    int32_t power_iters;
    int32_t precision;
    uint64_t seed;
    const float *basis;
    int32_t method;
    int32_t reserved;
    double *spectrum;
} xpcs_compress_opts;

/* Compress N frames of M pixels (Sec. 2.1, Eqs. 3-7; Sec. 2.2).
 * Offline mode: a rank-k basis of X by randomized subspace iteration (Halko,
 * Martinsson & Tropp 2011, Algs. 4.4 + 5.1): Y = X Omega, orthonormalise,
 * q x (Z = X^T Q, Y = X Z), orthonormalise, W_l = X^T Q, then the FP64
 * eigendecomposition of W_l^T W_l ranks the l directions and the top k are
 * kept.  The products with X run on BF16 MFMA with FP32 accumulation; the final
 * W = X^T U carries a second (residual) BF16 term so that W is accurate to FP32
 * level; Gram, Cholesky and eigen steps are FP64.
 * frames: device, dtype XPCS_U8 or XPCS_U16, N*M elements, frame-contiguous.
 * roi_label: device int32[M], values in [-1, n_roi).
 * out: caller-allocated factors with out->M == M, out->N == N, out->k == opts->k,
 *      out->n_roi == n_roi.
 * Errors: EINVAL (null, sizes, k + oversample > min(M, N) offline, k > min(M, N)
 * exact), EUNSUPPORTED (k + oversample > 1024 offline, k > 1024, N > 4096 exact),
 * EBUDGET, ENOMEM. */
xpcs_status compress_frames(xpcs_ctx *ctx, const void *frames, int32_t dtype, int64_t M,
                            int64_t N, const int32_t *roi_label, int32_t n_roi,
                            const xpcs_compress_opts *opts, xpcs_factors *out);

/* Two-time correlation on the compressed data (Sec. 2.1, Eqs. 8-10 per ROI):
 *   C~_R[t1][t2] = |R| * (W G_R W^T)[t1][t2] / (S_R[t1] S_R[t2]),  W = V diag(sigma),
 * for frames t1, t2 in the window [t0, t1) and ROI `roi` (or every ROI).
 * C: device, (t1-t0) x (t1-t0) elements of c_dtype with row stride ldc; for
 *    XPCS_ALL_ROIS, n_roi such matrices, ROI r at C + r*(t1-t0)*ldc elements.
 *    May be NULL (g2 only, no matrix is written).  C is exactly symmetric.
 * g2, npairs: device, (t1-t0) entries per ROI (ROI-major for XPCS_ALL_ROIS), or
 *    NULL.  g2[tau] = mean of C[t][t+tau] over the valid pairs in the window
 *    (Sec. 3.1, Eq. 12 read as the mean along C's diagonals), fused into the
 *    tile pass; npairs[tau] = number of those pairs.
 * Arithmetic: split-BF16 MFMA products (three terms) with FP32 accumulation.
 * Errors: EINVAL (null factors, window, ldc, roi), EBUDGET, ENOMEM. */
xpcs_status correlate_two_time(xpcs_ctx *ctx, const xpcs_factors *f, int32_t roi, int64_t t0,
                               int64_t t1, void *C, int32_t c_dtype, int64_t ldc, double *g2,
                               int64_t *npairs);

/* correlate_two_time for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, kernels and results, but every temporary buffer lives in a
 * static scratch array of the library (32 MiB, one copy per device, held until
 * the process ends) instead of the context's workspace, and the call makes no
 * hipMalloc, hipFree or other allocation (phase timing is suspended for it).
 * The caller passes the factors and the outputs.  Scratch needed: about
 * n_roi_call * (4 * nw * k32 + 8 * k^2 + nw) bytes (k32 = k rounded up to 32)
 * plus, with g2, 3060 bytes per 128 x 128 tile on and above the diagonal of each
 * ROI's window; a call needing more is refused with EUNSUPPORTED (split the ROIs
 * or the window).  Every call on a device shares that device's scratch: calls
 * that overlap on one device (different streams or host threads) race, so
 * serialise them.
 * Errors: as correlate_two_time, plus EUNSUPPORTED (scratch too small) and
 * EDEVICE (no static scratch on the device). */
xpcs_status correlate_two_time_noalloc(xpcs_ctx *ctx, const xpcs_factors *f, int32_t roi, int64_t t0,
                                       int64_t t1, void *C, int32_t c_dtype, int64_t ldc, double *g2,
                                       int64_t *npairs);

/* Two-time correlation from the raw frames (Sec. 2.1, Eqs. 1-2 per ROI), the path
 * the compressed correlation replaces:
 *   C_R[t1][t2] = |R| * G_R[t1][t2] / (S_R[t1] S_R[t2]),  G_R = X_R^T X_R exact.
 * The counts are split into 7-bit planes, count = P0 + 128 P1 + 16384 P2 (P2 for
 * uint16 only).  Plane 0 of every ROI pixel is gathered once into int8 and its
 * Gram runs on int8 MFMA with int32 accumulation (int64 across pixel chunks); the
 * pixels where some count reaches 128 add the other plane pairs,
 * 2^(7 (a + b)) P_a P_b^T, the same way.  G_R is exact for every count (while it
 * stays below 2^63; C is its FP64 normalisation).
 * Arguments as correlate_two_time; gram_out (device int64, same layout as C with
 * row stride t1-t0, or NULL) receives the exact G_R. */
xpcs_status correlate_two_time_raw(xpcs_ctx *ctx, const void *frames, int32_t dtype, int64_t M,
                                   int64_t N, const int32_t *roi_label, int32_t n_roi,
                                   int32_t roi, int64_t t0, int64_t t1, void *C, int32_t c_dtype,
                                   int64_t ldc, double *g2, int64_t *npairs, int64_t *gram_out);

/* g2 from a two-time matrix already in device memory (Sec. 3.1, Eq. 12):
 * g2[tau] = mean of C[t][t+tau] over the non-NaN entries, tau = 0..n-1, and
 * npairs[tau] their number (g2 is NaN where npairs is 0).  Only the upper
 * triangle of C is read.  C: device, n x n of c_dtype, row stride ldc. */
xpcs_status g2_from_two_time(xpcs_ctx *ctx, const void *C, int32_t c_dtype, int64_t n,
                             int64_t ldc, double *g2, int64_t *npairs);

/* g2 of the compressed two-time correlation without forming C~ (Sec. 3.1, Eq. 12
 * as the mean along the diagonals of C~_R, Sec. 2.1, Eqs. 8-10 per ROI): the same
 * g2 and npairs as correlate_two_time with C = NULL, computed by FFT in
 * O(k n log n) per ROI instead of O(k n^2).  With G_R = L_R L_R^T and
 * Z[t] = sqrt(|R|) (W[t] / S_R[t]) L_R, the diagonal sums of C~_R = Z Z^T are the
 * summed autocorrelations of Z's k columns and the pair counts the autocorrelation
 * of the mask of frames with S_R > 0; both come from power spectra of the columns
 * zero-padded to a power of two L >= 2n (two columns per complex transform).
 * Arithmetic: FP64 throughout (Z, transforms, sums); npairs is the rounded
 * transform of the mask, exact for every window allowed here.
 * f: factors from compress_frames.  roi: ROI index or XPCS_ALL_ROIS.
 * g2: device, (t1-t0) doubles per ROI (ROI-major for XPCS_ALL_ROIS), NaN where a
 *     lag has no valid pair; npairs: device int64, same layout, or NULL.
 * Workspace: about k*n*8 + (k/2+1)*L*16 bytes per ROI, ROIs processed in batches
 * of at most 2 GiB.
 * Errors: EINVAL (null factors or g2, window, roi), EUNSUPPORTED (k > 192 or a
 * window of more than 2^21 frames), EBUDGET, ENOMEM. */
xpcs_status g2_from_factors(xpcs_ctx *ctx, const xpcs_factors *f, int32_t roi, int64_t t0, int64_t t1,
                            double *g2, int64_t *npairs);

/* Background level of the compressed two-time correlation without forming C~
 * (Sec. 3.2: a correlation peak counts as observable when it is stronger than
 * twice the standard deviation of the TTC): mean and population standard
 * deviation of C~_R over the off-diagonal pairs (t1 != t2) of valid frames
 * (S_R > 0) in the window [t0, t1).  With Z[t] = sqrt(|R|) (W[t] / S_R[t]) L_R and
 * C~_R = Z Z^T, the sum of the entries is |sum_t Z[t]|^2 and the sum of their
 * squares |Z^T Z|_F^2; the diagonal's share is subtracted.  FP64 throughout.
 * mean, stdev: device, one double per ROI of the call (NaN without pairs);
 * npairs: device int64 per ROI, the number of entries averaged.
 * Errors: EINVAL (null factors or outputs, window, roi), EUNSUPPORTED (k > 192),
 * EBUDGET, ENOMEM. */
xpcs_status two_time_stats(xpcs_ctx *ctx, const xpcs_factors *f, int32_t roi, int64_t t0, int64_t t1,
                           double *mean, double *stdev, int64_t *npairs);

/* Relaxation fit of g2 (Sec. 3.1, Eq. 13): g2(tau) = B + beta exp(-2 Gamma tau)
 * with baseline B, contrast beta and Gamma = 1 / t0 (t0 the relaxation time in
 * frames), fitted by unweighted least squares to each ROI's g2 over the lags
 * tau_lo <= tau < tau_hi that have pairs (npairs > 0) and a finite value.
 * Levenberg-Marquardt in FP64, one workgroup per ROI, at most max_iter steps.
 * g2: device, n_roi x n doubles (ROI-major, as correlate_two_time writes them).
 * npairs: device, n_roi x n int64, or NULL (then only finite values count).
 * p0: device, n_roi x 3 doubles (B, beta, Gamma) to start from, or NULL: then
 *     B = the last valid g2, beta = max(first - last, 1e-3), Gamma = 1 / mean lag.
 * params: device, n_roi x 3 doubles (B, beta, Gamma); NaN for a ROI with fewer
 *     than three valid lags.
 * status: device, n_roi int32: the number of accepted or rejected steps taken,
 *     -1 for fewer than three valid lags.
 * Errors: EINVAL (null g2/params/status, n or n_roi, lag range outside [0, n),
 * max_iter outside [0, 10000]). */
xpcs_status fit_relaxation(xpcs_ctx *ctx, const double *g2, const int64_t *npairs, int64_t n, int32_t n_roi,
                           int64_t tau_lo, int64_t tau_hi, const double *p0, int32_t max_iter, double *params,
                           int32_t *status);

/* The stretched form of the relaxation law that Sec. 3.1 names after Kohlrausch,
 * Williams and Watts: g2(tau) = B + beta exp(-2 (Gamma tau)^gamma), the exponent
 * gamma fitted with (B, beta, Gamma); gamma = 1 is fit_relaxation's form.  Same
 * arguments with four parameters per ROI: p0 and params are n_roi x 4 doubles
 * (B, beta, Gamma, gamma); the default start is fit_relaxation's with gamma = 1.
 * A ROI needs four valid lags (else NaN parameters and status -1).  A trial step
 * to Gamma <= 0 has no defined model value and is rejected like one that raises
 * the cost.  Errors as fit_relaxation. */
xpcs_status fit_relaxation_stretched(xpcs_ctx *ctx, const double *g2, const int64_t *npairs, int64_t n,
                                     int32_t n_roi, int64_t tau_lo, int64_t tau_hi, const double *p0,
                                     int32_t max_iter, double *params, int32_t *status);

/* Rank rule of Sec. 3.1: the data is described by the eigenvectors whose
 * eigenvalues are at least twice the smallest one.  spectrum: device, n doubles
 * (e.g. compress_frames' spectrum output of the exact basis: the eigenvalues of
 * the frame Gram, which are those of the pixel Gram).  *rank (device int32) =
 * the number of entries that are positive and at least factor * min(spectrum)
 * (factor = 2 in the paper; zero and negative eigenvalues never count).
 * Errors: EINVAL (NULL, n < 1, factor < 1). */
xpcs_status xpcs_rank_rule(xpcs_ctx *ctx, const double *spectrum, int64_t n, double factor, int32_t *rank);

/* Peak visibility of g2 (Sec. 3.1: the peak minus the background level of g2)
 * and its detectability (Sec. 3.2: a correlation peak is observable when it is
 * stronger than twice the background level of the TTC, its standard deviation).
 * Per ROI r of g2 (device, n_roi x n, ROI-major; npairs device or NULL: lags
 * without pairs and non-finite values are skipped):
 *   visibility[r] = max g2 over the lags [peak_lo, peak_hi)
 *                   - mean g2 over the lags [bg_lo, bg_hi)   (NaN if a range is empty),
 *   detectable[r] = visibility[r] > factor * ttc_stdev[r]     (1 / 0).
 * ttc_stdev: device, n_roi doubles (two_time_stats' stdev), or NULL when
 * detectable is NULL.  visibility: device, n_roi doubles; detectable: device
 * int32 or NULL.  Errors: EINVAL (NULL, sizes, empty or out-of-range lag ranges). */
xpcs_status peak_visibility(xpcs_ctx *ctx, const double *g2, const int64_t *npairs, int32_t n_roi, int64_t n,
                            int64_t peak_lo, int64_t peak_hi, int64_t bg_lo, int64_t bg_hi, const double *ttc_stdev,
                            double factor, double *visibility, int32_t *detectable);

/* Frames for an encoding basis that knows nothing of the sample (Sec. 3.2: the
 * basis is generated from randomly shifted copies of one unrelated image): frame
 * t is the texture (height x width, row-major, dtype XPCS_U8 or XPCS_U16) shifted
 * cyclically by (dy_t, dx_t), dy_t = (h mod 2^32) mod height, dx_t = (h >> 32) mod
 * width, h = SplitMix64(seed XOR t); frames[t][y][x] = texture[(y + dy_t) mod
 * height][(x + dx_t) mod width].  compress_frames on these frames (offline mode,
 * randomized or exact) gives the basis, which other series then use in online mode.
 * texture: device; frames: device, n_frames * height * width elements of dtype.
 * Errors: EINVAL (NULL, dtype, sizes), EUNSUPPORTED (more than 65535 frames). */
xpcs_status shifted_texture_frames(xpcs_ctx *ctx, const void *texture, int32_t dtype, int64_t height, int64_t width,
                                   int64_t n_frames, uint64_t seed, void *frames);

/* ------------------------------------------------------------------ persisted state
 * The compressed data are what the paper keeps for later calculations (Sec. 3.1;
 * Sec. 2.2: compressed frames are appended to the compressed series).  The factors
 * of compress_frames -- with the ROI labels and the sketch seed they came from, if
 * given -- and an online stream's whole state go to a file and come back to device
 * memory bit for bit, in this process or another, so that correlations are
 * recomputed, or a stream resumed, without the raw frames.  Files: an 8-byte magic,
 * int64 header fields with their FNV-1a 64 hash, then sections of raw little-endian
 * arrays, each with its length and hash; any mismatch is reported as EINVAL
 * ("corrupt file").  Calls wait for the context's stream and copy synchronously. */
xpcs_status xpcs_factors_save(xpcs_ctx *ctx, const xpcs_factors *f, const int32_t *roi_label, uint64_t seed,
                              const char *path);
/* Sizes of a factors file (host only, no device work): M, N, k, n_roi, whether it
 * holds ROI labels, the seed.  Errors: EINVAL (unreadable, not a factors file,
 * corrupt header). */
xpcs_status xpcs_factors_info(const char *path, int64_t *M, int64_t *N, int32_t *k, int32_t *n_roi,
                              int32_t *has_labels, uint64_t *seed);
/* Loads a factors file into caller-allocated factors of the file's sizes, and the
 * ROI labels into roi_label (device int32[M]) unless it is NULL.
 * Errors: EINVAL (NULL, sizes differ, no labels in the file, corrupt file). */
xpcs_status xpcs_factors_load(xpcs_ctx *ctx, const char *path, xpcs_factors *f, int32_t *roi_label);

/* ------------------------------------------------------------------ online streams
 * The paper's online strategy (Sec. 2.2): the encoding basis is fixed beforehand
 * (e.g. from compress_frames on an earlier measurement or on the first frames of
 * this one), every new frame is compressed as it arrives (one more row of W,
 * Eq. 7) and its two-time correlations with the recent frames are computed at
 * once (Eqs. 9-10 per ROI).  A stream keeps, per ROI, the compressed rows of the
 * last `window` frames and g2 sums over its whole history.
 *
 * For every pushed frame t the stream produces the band row
 *   band[r][t][tau] = C~_R[t][t - tau],  tau = 0..window-1
 * (NaN where t - tau < 0 or either frame has no photons in the ROI) and adds
 * every valid band entry into g2 sums by lag: after frames 0..n-1 have been
 * pushed, g2[r][tau] = mean of C~_R[t][t - tau] over t < n (Eq. 12 read as the
 * mean along the diagonals, restricted to lags below the window), npairs[r][tau]
 * the number of pairs.  With window >= n this equals correlate_two_time's g2 of
 * the n frames. */
typedef struct xpcs_stream xpcs_stream;

typedef struct {
    int64_t M;                  /* pixels per frame */
    int32_t dtype;              /* XPCS_U8 | XPCS_U16 */
    int32_t n_roi;              /* 1..64 */
    int32_t k;                  /* basis columns, 1..192 */
    int32_t reserved;
    const int32_t *roi_label;   /* device int32[M] in [-1, n_roi); read at open only */
    const float *basis;         /* device M x k column-major, orthonormal columns; read at open only */
    int64_t window;             /* lags kept: 1..65536 */
    int64_t max_block;          /* most frames per push: 1..4096 */
} xpcs_stream_desc;

/* Opens a stream on ctx: converts the basis to split bf16, forms G_R = U_R^T U_R
 * and its Cholesky factor, and allocates the stream's state (compressed rows of
 * window + max_block frames per ROI, g2 sums), which counts against the
 * context's HBM budget until xpcs_stream_close.  The stream runs on ctx's
 * stream; streams of one context run one after the other.
 * Errors: EINVAL (sizes, NULL), EUNSUPPORTED (k > 192, n_roi > 64), EBUDGET, ENOMEM. */
xpcs_status xpcs_stream_open(xpcs_ctx *ctx, const xpcs_stream_desc *desc, xpcs_stream **out);

/* Appends `nframes` frames (device, frame-contiguous, the stream's dtype, M
 * counts each): encodes them (W rows and exact ROI sums), writes their band rows
 * into `band` when it is not NULL (device, n_roi x nframes x window elements of
 * c_dtype, ROI-major, row stride `window`), and adds them to the g2 sums.
 * Asynchronous on ctx's stream.  Errors: EINVAL (NULL frames, nframes outside
 * 1..max_block, c_dtype not XPCS_F32), EBUDGET, ENOMEM. */
xpcs_status xpcs_stream_push(xpcs_stream *s, const void *frames, int64_t nframes, void *band,
                             int32_t c_dtype);

/* Snapshot of the g2 sums: g2[r*window + tau] (device double, NaN where npairs is
 * 0) and npairs[r*window + tau] (device int64); either may be NULL. */
xpcs_status xpcs_stream_g2(xpcs_stream *s, double *g2, int64_t *npairs);

/* Frames pushed so far (host value; 0 for a NULL stream). */
int64_t xpcs_stream_frames(const xpcs_stream *s);

/* Writes the stream's whole state (labels, basis, ROI factors, the window of
 * compressed rows, g2 sums, frame count) to `path`; xpcs_stream_load opens a new
 * stream on ctx from such a file, and pushes to it continue the series exactly
 * as the saved stream would have (bit-identical bands and g2 sums).
 * Errors: EINVAL (NULL, unreadable or corrupt file), EBUDGET, ENOMEM. */
xpcs_status xpcs_stream_save(xpcs_stream *s, const char *path);
xpcs_status xpcs_stream_load(xpcs_ctx *ctx, const char *path, xpcs_stream **out);

/* Releases the stream's device memory (after the work in flight). NULL is ignored. */
void xpcs_stream_close(xpcs_stream *s);

/* ------------------------------------------------------------------ serving
 * A server runs many online streams (above) -- detectors of different sizes
 * and ROI maps -- on one GPU at once (the real-time use of the online strategy,
 * Sec. 2.2 and Sec. 3.2).  Each admitted stream is placed on one of `lanes`
 * lanes (the one with the fewest streams); a lane is a HIP stream with its own
 * workspace, so that the blocks of streams on different lanes run concurrently
 * on the device.  Requests are admitted in the order they are made, while a
 * slot (`max_streams`) and HBM under `hbm_budget_bytes` (0 = no budget) are free
 * -- stream state plus lane workspaces; the others wait, and a close admits the
 * waiting requests that then fit, in order.  Every block is timed from the push
 * call to the end of its work on the GPU with device events.
 *
 * A stream's results are those of the same stream run alone with
 * xpcs_stream_* (the same kernels on the same data, in the same order).  The
 * calls on one server must not overlap (one host thread at a time). */
typedef struct xpcs_server xpcs_server;

#define XPCS_STREAM_QUEUED 1
#define XPCS_STREAM_ADMITTED 2
#define XPCS_STREAM_FAILED 3     /* admitted later, but its open failed (see last_error) */

/* lanes in 1..16, max_streams >= 1.  Errors: EINVAL, EDEVICE, ENOMEM. */
xpcs_status xpcs_server_create(int device, size_t hbm_budget_bytes, int32_t lanes, int32_t max_streams,
                               xpcs_server **out);
/* Closes every stream (after its work) and frees the server. NULL is ignored. */
void xpcs_server_destroy(xpcs_server *srv);
const char *xpcs_server_last_error(const xpcs_server *srv);

/* Requests a stream described as for xpcs_stream_open; *id names it from now on
 * and *state (may be NULL) says whether it was admitted at once -- its open then
 * ran to completion in this call, so roi_label and basis may be released -- or
 * queued, in which case roi_label and basis must stay valid until
 * xpcs_server_state reports XPCS_STREAM_ADMITTED or XPCS_STREAM_FAILED.
 * Errors: those of xpcs_stream_open; EBUDGET when the stream alone exceeds the
 * budget. */
xpcs_status xpcs_server_open(xpcs_server *srv, const xpcs_stream_desc *desc, int64_t *id, int32_t *state);
xpcs_status xpcs_server_state(xpcs_server *srv, int64_t id, int32_t *state);

/* Pushes a block of stream `id` as xpcs_stream_push does, on the stream's lane,
 * after the work enqueued so far on `producer` (a hipStream_t, NULL = none), so
 * that frames written there are complete.  frames and band must stay valid until
 * xpcs_server_poll reports the block.  Errors: EQUEUED while the stream waits;
 * those of xpcs_stream_push. */
xpcs_status xpcs_server_push(xpcs_server *srv, int64_t id, const void *frames, int64_t nframes, void *band,
                             int32_t c_dtype, void *producer);

/* Reports, without waiting, the stream's completed blocks in push order: up to
 * `cap` of them, latency_ms[i] (push call to the end of the block's work on the
 * GPU) and frames[i] (either may be NULL); *count = how many were reported. */
xpcs_status xpcs_server_poll(xpcs_server *srv, int64_t id, int32_t cap, double *latency_ms, int64_t *frames,
                             int32_t *count);

/* g2 snapshot of stream `id` (as xpcs_stream_g2), enqueued on its lane. */
xpcs_status xpcs_server_g2(xpcs_server *srv, int64_t id, double *g2, int64_t *npairs);

/* Waits for the work enqueued for stream `id` (its lane), or for every lane
 * when id == 0, and reports device-side errors as xpcs_sync does. */
xpcs_status xpcs_server_wait(xpcs_server *srv, int64_t id);

/* Closes stream `id` (waiting for its lane) or withdraws its request, releases
 * its memory and admits waiting requests that now fit. */
xpcs_status xpcs_server_close(xpcs_server *srv, int64_t id);

/* Device bytes held (stream state plus lane workspaces), admitted streams and
 * waiting requests; any pointer may be NULL. */
xpcs_status xpcs_server_stats(const xpcs_server *srv, size_t *bytes_used, int32_t *admitted, int32_t *queued);

#ifdef __cplusplus
}
#endif

#endif /* XPCS_H */
