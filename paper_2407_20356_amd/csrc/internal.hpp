// Internal declarations of the gfx950 XPCS library: context, workspace, MFMA
// operand types and the host-side launchers of every kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include <stdio.h>

#include <string>
#include <vector>

#include "xpcs.h"

namespace xpcs {

// ---------------------------------------------------------------- MFMA operand types
// v_mfma_f32_16x16x32_bf16: A/B operands are 8 bf16 per lane, C/D 4 floats.
// v_mfma_i32_16x16x64_i8:   A/B operands are 16 int8 per lane, C/D 4 int32.
// Lane l of a 64-wide wave holds operand row/column (l % 16) and the K group
// (l / 16); the accumulator holds rows 4*(l/16) + i, i = 0..3, of column l % 16.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;
// Widest sketch (k + oversampling) and rank the library accepts; ranks above 192
// take the blocked small-matrix kernels.
constexpr int kMaxRank = 1024;

// Round-to-nearest-even float -> bf16 bit pattern (NaN stays a quiet NaN).
__device__ __forceinline__ unsigned short f32_to_bf16_bits(float x) {
    unsigned int u = __builtin_bit_cast(unsigned int, x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (unsigned short)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(unsigned short b) {
    return __builtin_bit_cast(float, ((unsigned int)b) << 16);
}

__device__ __forceinline__ f32x4 mfma_bf16(const u16x8 &a, const u16x8 &b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}
__device__ __forceinline__ i32x4 mfma_i8(const i32x4 &a, const i32x4 &b, i32x4 c) {
    return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- device flags
enum : int {
    kFlagRange = 0,     // reserved (no path raises it: the raw Gram is exact for every count)
    kFlagLabel = 1,     // a label outside [-1, n_roi)
    kFlagNumeric = 2,   // a numerically singular step (all sketch pivots dropped, no convergence)
    kNumFlags = 4,
};

// ---------------------------------------------------------------- context
struct Workspace {
    char *base = nullptr;
    size_t capacity = 0;
    size_t used = 0;
};

struct PhaseRecord {
    const char *name;
    hipEvent_t start, stop;
};

}  // namespace xpcs

struct xpcs_ctx {
    int device = 0;
    size_t budget = 0;
    hipStream_t stream = nullptr;
    xpcs::Workspace ws;          // per-call buffers (bump allocated, reset by every entry point)
    xpcs::Workspace scratch;     // launcher-private temporaries, reused launch after launch
    size_t persistent = 0;       // device bytes held by open streams (counted in the budget)
    int *flags = nullptr;        // device int[kNumFlags]
    std::string last_error;
    bool timing = false;                         // phase timing enabled
    std::vector<std::string> phase_only;         // record only these phases (empty: all)
    std::vector<xpcs::PhaseRecord> phases;       // recorded, not yet read
    std::vector<hipEvent_t> event_pool;          // reusable events
    void *static_scratch = nullptr;              // this device's copy of the library's static scratch array
};

namespace xpcs {

// Records an error message on the context and returns `st`.
xpcs_status fail(xpcs_ctx *ctx, xpcs_status st, const std::string &msg);
// Converts a HIP error into XPCS_EDEVICE with a message; XPCS_OK otherwise.
xpcs_status check_hip(xpcs_ctx *ctx, hipError_t err, const char *what);

// Workspace: `ws_begin` resets the bump pointer; `ws_reserve` makes sure
// `bytes` more can be carved (growing the arena -- after waiting for the stream
// -- when needed, subject to the budget); `ws_take` carves 256-byte aligned
// pieces and never fails after a successful reserve of the total.
void ws_begin(xpcs_ctx *ctx);
xpcs_status ws_reserve(xpcs_ctx *ctx, size_t total_bytes);
void *ws_take(xpcs_ctx *ctx, size_t bytes);
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
// Scratch: one arena shared by consecutive launchers.  Work on the context's
// stream runs in order, so a launcher may reuse what an earlier launcher's
// kernels used.  Returns NULL (with the status set) when it cannot grow.
void *scratch_get(xpcs_ctx *ctx, size_t bytes, xpcs_status *st);
// Size of the file-scope device array behind the entry points that allocate
// nothing (each device holds its own copy for the life of the process).
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
// Zero `bytes` of device memory with a kernel (safe inside captured graphs).
xpcs_status launch_zero(xpcs_ctx *ctx, void *p, size_t bytes);

// Records the device time of the enclosed launches under `name` when phase
// timing is enabled (no-op otherwise).  `name` must be a string literal.
class Phase {
  public:
    Phase(xpcs_ctx *ctx, const char *name);
    ~Phase();

  private:
    xpcs_ctx *ctx_;
    int idx_ = -1;
};

#define XPCS_LAUNCH_CHECK(ctx, what)                                         \
    do {                                                                      \
        hipError_t e_ = hipGetLastError();                                    \
        if (e_ != hipSuccess) return ::xpcs::check_hip((ctx), e_, (what));    \
    } while (0)

// ---------------------------------------------------------------- persisted state (persist.hip)
// FNV-1a 64 hash of n bytes continuing from h.
uint64_t fnv1a64(const void *p, size_t n, uint64_t h);
// A checksummed state file: magic, int64 header fields with their hash, then
// sections of device memory, each with its length and hash.
struct PersistFile {
    FILE *fp = nullptr;
    ~PersistFile();
    xpcs_status open_write(const char *path);
    xpcs_status open_read(const char *path);
    xpcs_status write_header(const char *magic, const int64_t *fields, int nfields);
    xpcs_status read_header(const char *magic, int64_t *fields, int nfields);
    xpcs_status write_device(xpcs_ctx *ctx, const void *dev, size_t bytes);
    xpcs_status read_device(xpcs_ctx *ctx, void *dev, size_t bytes);
};

// ---------------------------------------------------------------- ROI bookkeeping (ingest.hip)
// roi_npix[r] (int64) and label validation.
xpcs_status launch_roi_count(xpcs_ctx *ctx, const int32_t *labels, int64_t M, int n_roi,
                             int64_t *roi_npix);
// Stable ROI-sorted pixel order: off[r] = start of ROI r (ROI lengths padded to
// `pad`), perm[q] = pixel at sorted position q (-1 in padding), qroi[q] = ROI.
// `total_cap` is the capacity of perm/qroi (M + n_roi*pad is always enough).
xpcs_status launch_roi_order(xpcs_ctx *ctx, const int32_t *labels, int64_t M, int n_roi,
                             const int64_t *roi_npix, int pad, int64_t *off, int32_t *perm,
                             int32_t *qroi, int64_t total_cap);
// Gather the ROI pixels of frames [t0, t0+nw) to int8 rows xs[t][q] (row stride
// ldx >= total) as plane 0 of the counts (count & 127), with exact ROI sums
// S[r*nw + t], the largest plane-0 value amax, and the positions whose counts need
// higher planes: hot[q] (total_cap ints, bit 0: a count >= 128, bit 1: >= 16384),
// per ROI their list hq[off[r] + i], i < hcnt[r] (hq: total_cap entries), and the
// OR of their bits hbits[r].
xpcs_status launch_gather_i8(xpcs_ctx *ctx, const void *frames, int dtype, int64_t M,
                             int64_t t0, int64_t nw, const int32_t *perm, const int32_t *qroi,
                             const int64_t *off, int n_roi, int64_t ldx, int8_t *xs, int64_t *S,
                             int *amax, int *hot, int64_t *hq, int *hcnt, int *hbits, int64_t total_cap);

// ---------------------------------------------------------------- tile pass (tiles.hip)
struct TileOut {
    void *C = nullptr;          // output matrix base (NULL: none)
    int c_dtype = XPCS_F32;
    int64_t ldc = 0;
    int64_t c_roi_stride = 0;   // elements between consecutive ROIs' matrices
    int64_t *gram_out = nullptr;      // raw path only
    int64_t gram_roi_stride = 0;
    double *g2_part = nullptr;  // [roi][tile][255] partial diagonal sums (NULL: no g2)
    int *g2_cnt = nullptr;      // [roi][tile][255] partial pair counts
};
constexpr int kTile = 128;
constexpr int kDiag = 2 * kTile - 1;

inline int64_t n_tiles_upper(int64_t nw) {
    int64_t nb = (nw + kTile - 1) / kTile;
    return nb * (nb + 1) / 2;
}

// The hot positions of a raw pass (from launch_gather_i8) and the frames they are
// read back from for their higher count planes.
struct RawHot {
    const void *frames = nullptr;
    int dtype = XPCS_U8;
    int64_t M = 0, t0 = 0;
    const int32_t *perm = nullptr;
    const int64_t *hq = nullptr;
    const int *hcnt = nullptr;
    const int *hbits = nullptr;
};
// Raw ROI Gram on int8 MFMA + normalisation epilogue, for ROIs [r0, r0+nr); exact
// for every count (plane 0 from xs, the higher planes of the hot positions).
xpcs_status launch_raw_gram_tiles(xpcs_ctx *ctx, const int8_t *xs, int64_t ldx,
                                  const int64_t *off, const int64_t *roi_npix, const int64_t *S,
                                  int64_t nw, int r0, int nr, const int *amax, const RawHot &hot,
                                  const TileOut &out);
// Low-rank tiles C = Z Z^T for ROIs [0, nr) from split-bf16 rows laid out
// [r][t][kp] (hi and lo), with the frame validity mask valid[r*nw + t].
xpcs_status launch_lowrank_tiles(xpcs_ctx *ctx, const unsigned short *z_hi, const unsigned short *z_lo, int kp,
                                 const unsigned char *valid, int64_t nw, int nr, const TileOut &out);
// Partial diagonal sums of an existing matrix (upper triangle only).
xpcs_status launch_matrix_diag_tiles(xpcs_ctx *ctx, const void *C, int c_dtype, int64_t n,
                                     int64_t ldc, double *g2_part, int *g2_cnt);
// g2[r][tau] = sum / count over the tiles covering lag tau.
xpcs_status launch_g2_reduce(xpcs_ctx *ctx, const double *g2_part, const int *g2_cnt, int64_t nw,
                             int nr, double *g2, int64_t *npairs);

// ---------------------------------------------------------------- projections (proj_pixels.hip, proj_frames*.hip)
// Rademacher sketch (sketch.hip): om[j][t] = +-1 (int8) for j < ell, t < N, zero
// padded (row stride ldt, a multiple of 64 >= N; L rows, L a multiple of 16), then
// Y[j][p] = sum_t X[t][p] om[j][t] on the int8 MFMA (exact per 7-bit plane of the
// counts); Y fp32 with row stride M.  `need` is scratch of sketch_need_bytes(M).
size_t sketch_need_bytes(int64_t M);
xpcs_status launch_sketch_i8(xpcs_ctx *ctx, const void *frames, int dtype, int64_t M, int64_t N, uint64_t seed,
                             int ell, int L, int64_t ldt, int8_t *om, float *Y, int *need);
// Pixel-space product Y[j][p] = sum_t X[p][t] B[j][t] (B bf16 rows of stride ldb, L
// columns, L multiple of 16); Y fp32 column-major with stride M.
xpcs_status launch_proj_pixels(xpcs_ctx *ctx, const void *frames, int dtype, int64_t M, int64_t N,
                               const unsigned short *B, int64_t ldb, int L, float *Y);
// Frame-space partial products P[c][t][j] = sum_{p in chunk c} X[p][t] Q[j][p] for
// j < L (bf16 hi, optional lo) and, when n_ind > 0, the indicator columns
// j = L + r (label == r).  Q rows have stride ldq (>= M padded to 64, zero padded).
struct FrameProj {
    int64_t nchunks = 0;
    int64_t chunk = 0;      // pixels per chunk (multiple of 64)
    int ncols = 0;          // L + indicator columns rounded to 16
    int frames_per_block = 0;
};
// Plan for a pass with (lo = true) or without the residual term of Q.
FrameProj plan_proj_frames(int64_t M, int64_t N, int L, int n_ind, bool lo);
// FP8 (e4m3) versions of the power pass for u8 counts (proj_f8.hip): the
// pixel-space product with an e4m3 B (rows of stride ldb) and the frame-space
// product with an e4m3 Q (no residual term, no indicator columns; `plan` from
// plan_proj_frames(M, N, L, 0, false)).
xpcs_status launch_proj_pixels_f8(xpcs_ctx *ctx, const uint8_t *frames, int64_t M, int64_t N, const uint8_t *B,
                                  int64_t ldb, int L, float *Y);
xpcs_status launch_proj_frames_f8(xpcs_ctx *ctx, const uint8_t *frames, int64_t M, int64_t N, const uint8_t *q8,
                                  int64_t ldq, int L, const FrameProj &plan, float *part);
xpcs_status launch_proj_frames(xpcs_ctx *ctx, const void *frames, int dtype, int64_t M, int64_t N,
                               const unsigned short *q_hi, const unsigned short *q_lo, int64_t ldq,
                               int L, const int32_t *labels, int n_ind, const FrameProj &plan,
                               float *part);
// Sum the chunk partials: Z[j*ldz + t] (fp64, column-major) for j < L, and the
// indicator columns into S[r*N + t] (int64) when S != NULL.
xpcs_status launch_proj_frames_reduce(xpcs_ctx *ctx, const float *part, const FrameProj &plan,
                                      int64_t N, int L, int n_ind, double *Z, int64_t ldz,
                                      int64_t *S);

// ---------------------------------------------------------------- small dense FP64 steps (smallmat.hip)
// Gram of a tall column-major matrix A (rows x ncols, column stride lda; fp32 or
// fp64): G = A^T A (ncols x ncols, fp64).  With seg_off (segments of a gathered
// row list row_idx; -1 entries skipped) one Gram per segment: G[s].
xpcs_status launch_tsgram(xpcs_ctx *ctx, const void *A, bool a_f64, int64_t rows, int64_t lda,
                          int ncols, const int32_t *row_idx, const int64_t *seg_off, int nseg,
                          double *G);
// Grams of nbatch tall matrices A + b * bstride (rows x ncols, column stride lda):
// G + b * ncols^2; one launch of the FP64 MFMA kernel for up to 80 columns.
xpcs_status launch_tsgram_batched(xpcs_ctx *ctx, const void *A, bool a_f64, int64_t rows, int64_t lda, int ncols,
                                  int nbatch, int64_t bstride, double *G);
// Cholesky of G (n x n) with pivots below rel_tol*max(diag) dropped, and the
// inverse of the factor: A * Rinv has orthonormal (or zero) columns.  Rinv is
// upper triangular, column-major n x n.  Optionally Rinv <- Rprev * Rinv.
xpcs_status launch_cholinv(xpcs_ctx *ctx, const double *G, int n, double rel_tol,
                           const double *Rprev, double *Rinv);
// Cholesky factors of nb symmetric PSD n x n matrices (row-major lower L, dropped
// pivots give zero columns): G[b] ~= L[b] L[b]^T.  Above 192 the factorization is
// blocked and needs chol_batched_work_bytes(n, nb) of temporaries: `work`, or the
// context's scratch when `work` is NULL.
size_t chol_batched_work_bytes(int n, int nb);
xpcs_status launch_chol_batched(xpcs_ctx *ctx, const double *G, int n, int nb, double *L, void *work = nullptr);
// out[:, j] = sum_i A[:, i] T[i][j] (A column-major rows x n, fp32 or fp64; T
// column-major n x m fp64, optionally scaled per output column by colscale[j]).
// Writes any of: fp32 out32 (stride ld32), fp64 out64 (stride ld64), bf16 hi/lo
// rows (stride ldh) padded with zeros up to Lpad columns and rows_pad rows.  With
// t_upper, T is upper triangular (T[i][j] = 0 for i > j) and its zero blocks are
// skipped.
struct TsOut {
    float *out32 = nullptr; int64_t ld32 = 0;
    double *out64 = nullptr; int64_t ld64 = 0;
    unsigned short *hi = nullptr; unsigned short *lo = nullptr; int64_t ldh = 0;
    uint8_t *f8 = nullptr;      // e4m3 rows of 256 x value (stride ldh, padded as hi)
    int Lpad = 0; int64_t rows_pad = 0;
};
xpcs_status launch_tsmul(xpcs_ctx *ctx, const void *A, bool a_f64, int64_t rows, int64_t lda, int n,
                         const double *T, int m, const double *colscale, const TsOut &out, bool t_upper = false);
// out = X T with X the frames read as the column-major M x N count matrix (FP64
// accumulation of exact products), T column-major N x m, optional column scale.
xpcs_status launch_tsmul_counts(xpcs_ctx *ctx, const void *frames, int dtype, int64_t M, int64_t N,
                                const double *T, int m, const double *colscale, const TsOut &out);
// Symmetric eigendecomposition of B (n x n, n even) by cyclic Jacobi (parallel
// order on chip up to 192, block Jacobi above): eigenvalues lam[n] (unsorted),
// eigenvectors P (row-major n x n, column j = vector j).  `rot` holds the rotation
// log, or the block method's matrices (jacobi_rot_bytes(n) bytes).
size_t jacobi_rot_bytes(int n);
xpcs_status launch_jacobi(xpcs_ctx *ctx, const double *B, int n, double *lam, double *P, void *rot);
// Order by decreasing eigenvalue, pick the first k, fix signs and build the
// column transforms: T_u[i][r] = P[i][perm[r]] * sign_r, scale_v[r] = 1 /
// sigma_r (0 when sigma_r == 0), sigma[r] = sqrt(max(lam, 0)).  The sign makes
// the largest-magnitude entry of W_l P[:, perm[r]] positive.
xpcs_status launch_select_basis(xpcs_ctx *ctx, const double *lam, const double *P, int n, int k,
                                const double *Wl, int64_t N, int64_t ldw, double *T_u,
                                double *scale_v, double *sigma);
// The same selection for the exact basis: T_u = the k leading eigenvectors (columns
// of P, sign: largest-magnitude entry positive), sigma = sqrt(max(lam, 0)),
// scale_v = 1 / sigma; spectrum (optional) = all n eigenvalues in decreasing order.
xpcs_status launch_select_exact(xpcs_ctx *ctx, const double *lam, const double *P, int n, int k, double *T_u,
                                double *scale_v, double *sigma, double *spectrum);
// Online mode: sigma[j] = |W[:, j]|, scale[j] = 1 / sigma[j] (0 if sigma is 0).
xpcs_status launch_column_norms(xpcs_ctx *ctx, const double *W, int64_t N, int64_t ldw, int k,
                                double *sigma, double *scale);
// Copy / convert a basis: U fp32 column-major -> bf16 hi/lo rows (stride ldq).
xpcs_status launch_basis_to_bf16(xpcs_ctx *ctx, const float *U, int64_t M, int k, int64_t ldq,
                                 int Lpad, unsigned short *hi, unsigned short *lo);
// Diagonal identity: T[i][j] = (i == j) for an n x n column-major matrix.
xpcs_status launch_identity(xpcs_ctx *ctx, double *T, int n);

// ---------------------------------------------------------------- the same steps above 192 (bigmat.hip)
size_t chol_blocked_work_bytes(int n, int nb);
xpcs_status launch_chol_blocked(xpcs_ctx *ctx, const double *G, int n, int nb, double rel_tol, double *L,
                                void *work);
size_t cholinv_blocked_work_bytes(int n);
xpcs_status launch_cholinv_blocked(xpcs_ctx *ctx, const double *G, int n, double rel_tol, double *Rinv,
                                   void *work);
size_t jacobi_block_work_bytes(int n);
xpcs_status launch_jacobi_block(xpcs_ctx *ctx, const double *B, int n, double *lam, double *P, void *work);
xpcs_status launch_panel_gram(xpcs_ctx *ctx, const void *A, bool a_f64, int64_t rows, int64_t lda, int ncols,
                              const int32_t *row_idx, const int64_t *seg_off, int nseg, double *G);
// The frame Gram F F^T (N x N, FP64) of N frames of M integer counts: exact while
// every sum stays below 2^53 (always for uint8; M amax^2 < 2^53 for uint16).
xpcs_status launch_frame_gram(xpcs_ctx *ctx, const void *frames, int dtype, int64_t M, int64_t N, double *G);

// ---------------------------------------------------------------- compressed TTC prep (lowrank.hip)
// Per ROI r (Lr = Cholesky factor of G_R, row-major lower, nr x k x k) and frame t of
// the window: z = sqrt(|R|) * (V[t, :] * sigma / S_r[t]) Lr, split to bf16 hi/lo rows
// of kp (zero padded); valid[r][t] = S_r[t] > 0.  Then C~_R = Z Z^T.
xpcs_status launch_lowrank_prep(xpcs_ctx *ctx, const xpcs_factors *f, const double *Lr, int r0, int nr,
                                int64_t t0, int64_t nw, int kp, unsigned short *z_hi, unsigned short *z_lo,
                                unsigned char *valid);

// ---------------------------------------------------------------- online streams (stream.hip)
// Device bytes of a stream's state, and the most workspace its open and pushes take.
size_t stream_state_bytes(const xpcs_stream_desc *d);
size_t stream_workspace_bytes(const xpcs_stream_desc *d);

}  // namespace xpcs
