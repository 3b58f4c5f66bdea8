// The N x N tile pass shared by the raw and the compressed two-time correlation.
//
// C is symmetric (Sec. 2.1, Eq. 2: G = X X^T), so only the tiles on and above
// the block diagonal are computed; each is written at (i, j) and mirrored at
// (j, i) from the same value, which makes C exactly symmetric.  The g2 lag
// average (Sec. 3.1, Eq. 12) is fused into the same pass: every tile leaves the
// sums of its 255 diagonals t2 - t1 = const in a partial buffer, and a second,
// fixed-order pass adds them per lag (no float atomics, deterministic).
//
// Block shape: 256 threads = 4 waves in a 2 x 2 arrangement, each wave owning a
// 64 x 64 quarter of the 128 x 128 tile as 4 x 4 MFMA 16 x 16 blocks.  The
// epilogue stages one 64-row half of the tile in LDS at a time so that both the
// direct and the mirrored writes go out as contiguous rows.
#include <math.h>

#include <type_traits>

#include "internal.hpp"

namespace xpcs {
namespace {

constexpr int kPitch = kTile + 1;   // odd LDS pitch: column reads are conflict-free
constexpr int kHalf = kTile / 2;

// Tiles of one ROI in diagonal-major order: id = start(D) + bi with D = bj - bi and
// start(D) = sum_{d<D} (nb - d) = D nb - D (D - 1) / 2.  D is the root of the
// quadratic, corrected by whole steps against rounding.
__device__ __forceinline__ void tile_coords(int64_t id, int nb, int &bi, int &bj) {
    const double b = 2.0 * nb + 1.0;
    int64_t D = (int64_t)((b - sqrt(b * b - 8.0 * (double)id)) * 0.5);
    if (D < 0) D = 0;
    if (D > nb - 1) D = nb - 1;
    while (D > 0 && D * nb - D * (D - 1) / 2 > id) --D;
    while (D + 1 < nb && (D + 1) * nb - (D + 1) * D / 2 <= id) ++D;
    bi = (int)(id - (D * nb - D * (D - 1) / 2));
    bj = bi + (int)D;
}

template <typename OutT>
__device__ __forceinline__ void nt_store(OutT *p, OutT v) {
    __builtin_nontemporal_store(v, p);
}

template <typename OutT>
__device__ __forceinline__ void store4(OutT *dst, const OutT (&v)[4], const bool (&ok)[4], bool vec) {
    if (vec && ok[0] && ok[1] && ok[2] && ok[3]) {
        if constexpr (sizeof(OutT) == 4) {
            f32x4 x = {(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
            __builtin_nontemporal_store(x, reinterpret_cast<f32x4 *>(dst));
            return;
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (ok[e]) nt_store(dst + e, v[e]);
}

// One 64-row half h of a staged tile: direct rows, mirrored columns, diagonal partials.
// All 256 threads call it; st holds rows [64h, 64h + 64) of the tile at pitch kPitch.
template <typename StageT, typename OutT, typename SumT>
__device__ __forceinline__ void epilogue_half(const StageT *st, int h, int64_t i0, int64_t j0, bool diag,
                                              int64_t nw, OutT *C, int64_t ldc, bool vec, bool any_nan,
                                              double &dsum, int &dcnt) {
    const int tid = threadIdx.x;
    if (C) {
        // Direct rows: 32 threads x 4 columns per row, 8 rows per pass.
#pragma unroll 1
        for (int pass = 0; pass < kHalf / 8; ++pass) {
            const int rl = pass * 8 + tid / 32;
            const int c = (tid % 32) * 4;
            const int r = kHalf * h + rl;
            const int64_t i = i0 + r;
            if (i < nw) {
                OutT v[4];
                bool ok[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    ok[e] = (j0 + c + e < nw) && (!diag || c + e >= r);
                    v[e] = (OutT)st[rl * kPitch + c + e];
                }
                store4(C + i * ldc + j0 + c, v, ok, vec);
            }
        }
        // Mirrored columns: 16 threads x 4 rows per column, 16 columns per pass.
#pragma unroll 1
        for (int pass = 0; pass < kTile / 16; ++pass) {
            const int c = pass * 16 + tid / 16;
            const int rq = tid % 16;
            const int64_t j = j0 + c;
            if (j < nw) {
                OutT v[4];
                bool ok[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int rl = 4 * rq + e;
                    const int r = kHalf * h + rl;
                    ok[e] = (i0 + r < nw) && (!diag || c > r);
                    v[e] = (OutT)st[rl * kPitch + c];
                }
                store4(C + j * ldc + i0 + kHalf * h + 4 * rq, v, ok, vec);
            }
        }
    }
    // Diagonal partials: thread d handles the in-tile offset c - r = d - 127 over the
    // rows of this half where the diagonal exists (exact bounds, no idle iterations).
    // Partial sums within the half (at most 64 terms) are kept in SumT.
    if (tid < kDiag) {
        const int d = tid - (kTile - 1);
        if (!diag || d >= 0) {
            int r_lo = kHalf * h, r_hi = kHalf * h + kHalf;          // rows [r_lo, r_hi)
            if (d < 0 && r_lo < -d) r_lo = -d;                       // c = r + d >= 0
            if (d > 0 && r_hi > kTile - d) r_hi = kTile - d;         // c = r + d < kTile
            if (i0 + r_hi > nw) r_hi = (int)(nw - i0);               // rows inside the window
            const int64_t c_lim = nw - j0 - d;                       // and columns: r < nw - j0 - d
            if (r_hi > c_lim) r_hi = (int)c_lim;
            SumT sum = 0;
            int cnt = 0;
            if (any_nan) {
                for (int r = r_lo; r < r_hi; ++r) {
                    const StageT v = st[(r - kHalf * h) * kPitch + r + d];
                    if (v == v) {
                        sum += (SumT)v;
                        cnt += 1;
                    }
                }
            } else {
#pragma unroll 8
                for (int r = r_lo; r < r_hi; ++r) sum += (SumT)st[(r - kHalf * h) * kPitch + r + d];
                cnt = r_hi > r_lo ? r_hi - r_lo : 0;
            }
            dsum += (double)sum;
            dcnt += cnt;
        }
    }
}

__device__ __forceinline__ void write_diag_partials(double *g2_part, int *g2_cnt, int64_t slot, double dsum,
                                                    int dcnt) {
    if (g2_part && threadIdx.x < kDiag) {
        g2_part[slot * kDiag + threadIdx.x] = dsum;
        g2_cnt[slot * kDiag + threadIdx.x] = dcnt;
    }
}

// ---------------------------------------------------------------- raw Gram (int8 MFMA)
// WIDE = false handles the ROIs whose pixel count fits one int32 accumulation
// chunk (every realistic case: with counts <= 40 a chunk holds 1.3 M pixels);
// WIDE = true the others, folding int32 chunk sums into int64.  Both are
// launched; each block leaves at once when its ROI belongs to the other.
// Raw-Gram operand stages: kRawKs pixels (bytes) of 256 rows per stage, LDS row
// pitch kRawRp (16 bytes of padding against bank conflicts), two buffers.
constexpr int kRawKs = 128;
constexpr int kRawRp = kRawKs + 16;
constexpr int kRawParts = kRawKs / 16;                   // 16-byte pieces per row
constexpr int kRawPer = 2 * kTile * kRawParts / 256;     // pieces per thread
constexpr int kRawBufBytes = 2 * kTile * kRawRp;
constexpr int kRawLdsBytes = 2 * kRawBufBytes > kHalf * kPitch * 8 ? 2 * kRawBufBytes : kHalf * kPitch * 8;
constexpr int kRawLdsDoubles = kRawLdsBytes / 8;

__device__ __forceinline__ int64_t raw_chunk_pixels(const int *__restrict__ amax, int64_t qlen) {
    const int am = *amax;
    // int32 accumulation is exact while (pixels per chunk) * amax^2 < 2^31.
    int64_t kc = am > 0 ? (int64_t)2147483647 / ((int64_t)am * am) : qlen;
    kc = kc / 64 * 64;
    return kc < 64 ? 64 : kc;
}

template <typename OutT, bool WIDE>
__device__ __forceinline__ void raw_gram_tile(
    int bi, int bj, int64_t tile_id, const int8_t *__restrict__ xs, int64_t ldx, const int64_t *__restrict__ off,
    const int64_t *__restrict__ roi_npix, const int64_t *__restrict__ S, int64_t nw, int r0, int slot,
    int64_t ntiles, int64_t kc, bool over, OutT *C, int64_t ldc, int64_t c_roi_stride, bool vec, int64_t *gram_out,
    int64_t gram_roi_stride, double *g2_part, int *g2_cnt) {
    // the operand stages (two buffers of 256 rows x kRawKs bytes) share the LDS of
    // the epilogue's staging buffer
    __shared__ __attribute__((aligned(16))) double stage[kRawLdsDoubles];
    const int roi = r0 + slot;
    const int64_t i0 = (int64_t)bi * kTile, j0 = (int64_t)bj * kTile;
    const bool diag = bi == bj;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
    const int lr = lane & 15, lg = lane >> 4;
    const bool skip = diag && wr > wc;     // strictly below the diagonal: never used

    const int64_t q0 = off[roi], qlen = off[roi + 1] - off[roi];

    // int32 MFMA accumulators; the wide variant folds them into int64 per chunk.
    i32x4 acc[4][4];
    int64_t wide[WIDE ? 4 : 1][WIDE ? 4 : 1][WIDE ? 4 : 1];
    if constexpr (WIDE) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e) wide[a][b][e] = 0;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (i32x4){0, 0, 0, 0};

    // Stages of kRawKs pixels: the tile's rows (128 of the row block, 128 of the
    // column block; 128 in all on the diagonal) are loaded once per block into
    // registers one stage ahead, written to the other LDS buffer after the current
    // stage's MFMAs, one barrier per stage.  Chunks of kc pixels (int32
    // exactness) are whole stages; pixels past a chunk's end load as zero.
    int8_t *ops = reinterpret_cast<int8_t *>(stage);
    const int64_t kcs = WIDE ? kc : (qlen + kRawKs - 1) / kRawKs * kRawKs;   // pixels per chunk, in stages
    const int spc = (int)((kcs + kRawKs - 1) / kRawKs);
    const int nchunk = (int)((qlen + kcs - 1) / kcs);
    const int nstage = nchunk * spc;
    const int jrow0 = diag ? 0 : kTile;
    i32x4 nxt[kRawPer];
    auto fetch = [&](int st) {
        const int64_t c = st / spc;
        const int64_t k = c * kcs + (int64_t)(st % spc) * kRawKs;
        const int64_t c1 = (c + 1) * kcs < qlen ? (c + 1) * kcs : qlen;
#pragma unroll
        for (int q = 0; q < kRawPer; ++q) {
            const int u = threadIdx.x + 256 * q;
            const int row = u / kRawParts, part = u % kRawParts;
            const int64_t t = row < kTile ? i0 + row : j0 + (row - kTile);
            const int64_t kk = k + 16 * part;
            i32x4 v = {0, 0, 0, 0};
            if (t < nw && kk < c1 && !(diag && row >= kTile))
                v = *reinterpret_cast<const i32x4 *>(xs + t * ldx + q0 + kk);
            nxt[q] = v;
        }
    };
    auto put = [&](int buf) {
        int8_t *dst = ops + buf * kRawBufBytes;
#pragma unroll
        for (int q = 0; q < kRawPer; ++q) {
            const int u = threadIdx.x + 256 * q;
            const int row = u / kRawParts, part = u % kRawParts;
            *reinterpret_cast<i32x4 *>(dst + row * kRawRp + 16 * part) = nxt[q];
        }
    };
    if (nstage > 0) {
        fetch(0);
        put(0);
        __syncthreads();
    }
    for (int st = 0; st < nstage; ++st) {
        const int buf = st & 1;
        if (st + 1 < nstage) fetch(st + 1);
        if (!skip) {
            const int8_t *src = ops + buf * kRawBufBytes;
#pragma unroll
            for (int h = 0; h < kRawKs / 64; ++h) {
                i32x4 av[4], bv[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int rb = jrow0 + 64 * wc + 16 * b + lr;
                    bv[b] = *reinterpret_cast<const i32x4 *>(src + rb * kRawRp + 64 * h + 16 * lg);
                }
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int ra = 64 * wr + 16 * a + lr;
                    av[a] = *reinterpret_cast<const i32x4 *>(src + ra * kRawRp + 64 * h + 16 * lg);
                }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[a][b] = mfma_i8(av[a], bv[b], acc[a][b]);
            }
        }
        if constexpr (WIDE) {
            if (st % spc == spc - 1) {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) wide[a][b][e] += acc[a][b][e];
                        acc[a][b] = (i32x4){0, 0, 0, 0};
                    }
            }
        }
        if (st + 1 < nstage) put(buf ^ 1);
        __syncthreads();
    }
    auto gval = [&](int a, int b, int e) -> int64_t {
        if constexpr (WIDE)
            return wide[a][b][e];
        else
            return (int64_t)acc[a][b][e];
    };

    const double npix = (double)roi_npix[roi];
    const int64_t *Sr = S + (int64_t)roi * nw;
    OutT *Cr = C ? C + (int64_t)slot * c_roi_stride : nullptr;
    int64_t *Gr = gram_out ? gram_out + (int64_t)slot * gram_roi_stride : nullptr;

    // Exact Gram straight from the registers (a debugging/verification output).
    if (Gr && !skip) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t i = i0 + 64 * wr + 16 * a + 4 * lg + e;
                    const int64_t j = j0 + 64 * wc + 16 * b + lr;
                    if (i < nw && j < nw && j >= i) {
                        Gr[i * nw + j] = gval(a, b, e);
                        Gr[j * nw + i] = gval(a, b, e);
                    }
                }
    }

    double dsum = 0.0;
    int dcnt = 0;
    // ROI sums of this lane's 16 rows and 4 columns, read once
    double srow[16], scol[4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t i = i0 + 64 * wr + 16 * a + 4 * lg + e;
            srow[4 * a + e] = i < nw ? (double)Sr[i] : 0.0;
        }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t j = j0 + 64 * wc + 16 * b + lr;
        scol[b] = j < nw ? (double)Sr[j] : 0.0;
    }
    for (int h = 0; h < 2; ++h) {
        if (wr == h) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int c = 64 * wc + 16 * b + lr;
                const double sj = scol[b];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int rl = 16 * a + 4 * lg + e;
                        const double si = srow[4 * a + e];
                        double v;
                        // a count above 127 was clamped on its way to int8: no value of this
                        // Gram is exact, so C is NaN throughout and g2 has no pairs
                        if (si > 0.0 && sj > 0.0 && !over)
                            v = (npix * (double)gval(a, b, e)) / (si * sj);
                        else
                            v = __builtin_nan("");
                        stage[rl * kPitch + c] = v;
                    }
            }
        }
        __syncthreads();
        epilogue_half<double, OutT, double>(stage, h, i0, j0, diag, nw, Cr, ldc, vec, true, dsum, dcnt);
        __syncthreads();
    }
    write_diag_partials(g2_part, g2_cnt, (int64_t)slot * ntiles + tile_id, dsum, dcnt);
}

// One block per tile; ROIs that need more than one int32 chunk are left to the wide kernel.
template <typename OutT>
__global__ __launch_bounds__(256, 2) void raw_gram_tile_kernel(
    const int8_t *__restrict__ xs, int64_t ldx, const int64_t *__restrict__ off,
    const int64_t *__restrict__ roi_npix, const int64_t *__restrict__ S, int64_t nw, int r0, int nb,
    const int *__restrict__ amax, OutT *C, int64_t ldc, int64_t c_roi_stride, bool vec,
    int64_t *gram_out, int64_t gram_roi_stride, double *g2_part, int *g2_cnt) {
    const int slot = blockIdx.y, roi = r0 + slot;
    const int64_t qlen = off[roi + 1] - off[roi];
    const int64_t kc = raw_chunk_pixels(amax, qlen);
    if (qlen > kc) return;
    int bi, bj;
    tile_coords(blockIdx.x, nb, bi, bj);
    raw_gram_tile<OutT, false>(bi, bj, blockIdx.x, xs, ldx, off, roi_npix, S, nw, r0, slot, gridDim.x, kc, *amax > 127, C, ldc,
                               c_roi_stride, vec, gram_out, gram_roi_stride, g2_part, g2_cnt);
}

// One block per (tile row, ROI), looping over the row's tiles, for the ROIs whose
// pixel count needs several int32 chunks (int64 between chunks).  Blocks of other
// ROIs leave at once; the grid is small, so the launch costs little when unused.
template <typename OutT>
__global__ __launch_bounds__(256, 2) void raw_gram_wide_kernel(
    const int8_t *__restrict__ xs, int64_t ldx, const int64_t *__restrict__ off,
    const int64_t *__restrict__ roi_npix, const int64_t *__restrict__ S, int64_t nw, int r0, int nb,
    const int *__restrict__ amax, OutT *C, int64_t ldc, int64_t c_roi_stride, bool vec,
    int64_t *gram_out, int64_t gram_roi_stride, double *g2_part, int *g2_cnt) {
    const int slot = blockIdx.y, roi = r0 + slot;
    const int64_t qlen = off[roi + 1] - off[roi];
    const int64_t kc = raw_chunk_pixels(amax, qlen);
    if (qlen <= kc) return;
    const int bi = blockIdx.x;
    const int64_t ntiles = (int64_t)nb * (nb + 1) / 2;
    for (int bj = bi; bj < nb; ++bj) {
        const int64_t D = bj - bi;
        const int64_t tile_id = D * nb - D * (D - 1) / 2 + bi;
        raw_gram_tile<OutT, true>(bi, bj, tile_id, xs, ldx, off, roi_npix, S, nw, r0, slot, ntiles, kc, *amax > 127, C, ldc,
                                  c_roi_stride, vec, gram_out, gram_roi_stride, g2_part, g2_cnt);
    }
}

// ---------------------------------------------------------------- low-rank tiles (split-bf16 MFMA)
// C~[i][j] = Z[i] . Z[j] with Z = sqrt(|R|) (W / S) L_R carried as bf16 hi + lo; the
// three products hi.hi + hi.lo + lo.hi are accumulated in FP32.  The tile's Z rows
// (128 of the row block, 128 of the column block; 128 in all on the diagonal) are
// staged in LDS one 32-wide K chunk at a time, the next chunk being fetched into
// registers while the current one runs on the MFMAs; the epilogue's staging
// buffer then reuses the same LDS.
constexpr int kZp = 40;                                  // LDS row pitch in u16 (32 + 8)
constexpr int kZUnits = 2 * 2 * kTile * 4;               // 16-byte units per chunk: arrays x rows x 4
constexpr int kZPer = kZUnits / 256;
constexpr int kZBytes = 2 * 2 * kTile * kZp * 2;         // 40 KB
constexpr int kStageBytes = kHalf * kPitch * 4;
constexpr int kLowrankLds = kZBytes > kStageBytes ? kZBytes : kStageBytes;

template <typename OutT>
__global__ __launch_bounds__(256, 3) void lowrank_tile_kernel(
    const unsigned short *__restrict__ z_hi, const unsigned short *__restrict__ z_lo, int kp,
    const unsigned char *__restrict__ valid, int64_t nw, int nb, OutT *C, int64_t ldc, int64_t c_roi_stride,
    bool vec, double *g2_part, int *g2_cnt) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[kLowrankLds];
    unsigned short *zs = reinterpret_cast<unsigned short *>(smem);   // [array][row 0..255][kZp]
    float *stage = reinterpret_cast<float *>(smem);
    const int slot = blockIdx.y;
    int bi, bj;
    tile_coords(blockIdx.x, nb, bi, bj);
    const int64_t i0 = (int64_t)bi * kTile, j0 = (int64_t)bj * kTile;
    const bool diag = bi == bj;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
    const int lr = lane & 15, lg = lane >> 4;
    const bool skip = diag && wr > wc;
    const int64_t base = (int64_t)slot * nw * kp;
    const int jrow0 = diag ? 0 : kTile;                  // LDS rows of the column block

    // chunk loader: unit u -> array (u >> 10), LDS row ((u >> 2) & 255), 16-byte part (u & 3)
    i32x4 nxt[kZPer];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < kZPer; ++q) {
            const int u = threadIdx.x + 256 * q;
            const int arr = u >> 10, row = (u >> 2) & 255, part = u & 3;
            const int64_t t = row < kTile ? i0 + row : j0 + (row - kTile);
            i32x4 v = {0, 0, 0, 0};
            if (t < nw && !(diag && row >= kTile)) {
                const unsigned short *src = (arr ? z_lo : z_hi) + base + t * kp + k0 + 8 * part;
                v = *reinterpret_cast<const i32x4 *>(src);
            }
            nxt[q] = v;
        }
    };
    auto put = [&]() {
#pragma unroll
        for (int q = 0; q < kZPer; ++q) {
            const int u = threadIdx.x + 256 * q;
            const int arr = u >> 10, row = (u >> 2) & 255, part = u & 3;
            *reinterpret_cast<i32x4 *>(zs + (arr * 2 * kTile + row) * kZp + 8 * part) = nxt[q];
        }
    };

    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};

    fetch(0);
    for (int k0 = 0; k0 < kp; k0 += 32) {
        put();
        __syncthreads();
        if (k0 + 32 < kp) fetch(k0 + 32);
        if (!skip) {
            u16x8 bh[4], bl[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int rb = jrow0 + 64 * wc + 16 * b + lr;
                bh[b] = *reinterpret_cast<const u16x8 *>(zs + rb * kZp + 8 * lg);
                bl[b] = *reinterpret_cast<const u16x8 *>(zs + (2 * kTile + rb) * kZp + 8 * lg);
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int ra = 64 * wr + 16 * a + lr;
                const u16x8 ah = *reinterpret_cast<const u16x8 *>(zs + ra * kZp + 8 * lg);
                const u16x8 al = *reinterpret_cast<const u16x8 *>(zs + (2 * kTile + ra) * kZp + 8 * lg);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    acc[a][b] = mfma_bf16(al, bh[b], acc[a][b]);
                    acc[a][b] = mfma_bf16(ah, bl[b], acc[a][b]);
                    acc[a][b] = mfma_bf16(ah, bh[b], acc[a][b]);
                }
            }
        }
        __syncthreads();
    }

    const unsigned char *vr = valid + (int64_t)slot * nw;
    OutT *Cr = C ? C + (int64_t)slot * c_roi_stride : nullptr;
    double dsum = 0.0;
    int dcnt = 0;
    // does the tile touch a frame without photons (NaN entries)?
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    {
        const int e = threadIdx.x;                 // 256 threads: 128 rows + 128 columns
        const int64_t t = e < kTile ? i0 + e : j0 + (e - kTile);
        if (t < nw && !vr[t]) s_bad = 1;
    }
    __syncthreads();
    const bool any_nan = s_bad != 0;
    // validity of this lane's 16 rows and 4 columns, read once (all valid in the usual case)
    unsigned rowok = 0xffffu, colok = 0xfu;
    if (any_nan) {
        rowok = colok = 0;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t i = i0 + 64 * wr + 16 * a + 4 * lg + e;
                if (i < nw && vr[i]) rowok |= 1u << (4 * a + e);
            }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t j = j0 + 64 * wc + 16 * b + lr;
            if (j < nw && vr[j]) colok |= 1u << b;
        }
    }
    for (int h = 0; h < 2; ++h) {
        if (wr == h) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int c = 64 * wc + 16 * b + lr;
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int rl = 16 * a + 4 * lg + e;
                        const bool ok = ((rowok >> (4 * a + e)) & (colok >> b) & 1u) != 0;
                        stage[rl * kPitch + c] = ok ? acc[a][b][e] : __builtin_nanf("");
                    }
            }
        }
        __syncthreads();
        epilogue_half<float, OutT, float>(stage, h, i0, j0, diag, nw, Cr, ldc, vec, any_nan, dsum, dcnt);
        __syncthreads();
    }
    write_diag_partials(g2_part, g2_cnt, (int64_t)slot * gridDim.x + blockIdx.x, dsum, dcnt);
}

// ---------------------------------------------------------------- diagonals of a given matrix
template <typename InT>
__global__ __launch_bounds__(256) void matrix_diag_tile_kernel(const InT *__restrict__ C, int64_t n,
                                                               int64_t ldc, int nb, double *g2_part,
                                                               int *g2_cnt) {
    __shared__ InT stage[kHalf * kPitch];
    int bi, bj;
    tile_coords(blockIdx.x, nb, bi, bj);
    const int64_t i0 = (int64_t)bi * kTile, j0 = (int64_t)bj * kTile;
    const bool diag = bi == bj;
    double dsum = 0.0;
    int dcnt = 0;
    for (int h = 0; h < 2; ++h) {
        for (int idx = threadIdx.x; idx < kHalf * kTile; idx += blockDim.x) {
            const int rl = idx / kTile, c = idx % kTile;
            const int64_t i = i0 + kHalf * h + rl, j = j0 + c;
            stage[rl * kPitch + c] = (i < n && j < n) ? C[i * ldc + j] : (InT)0;
        }
        __syncthreads();
        epilogue_half<InT, InT, double>(stage, h, i0, j0, diag, n, (InT *)nullptr, 0, false, true, dsum, dcnt);
        __syncthreads();
    }
    write_diag_partials(g2_part, g2_cnt, blockIdx.x, dsum, dcnt);
}

// ---------------------------------------------------------------- lag reduction
__global__ __launch_bounds__(256) void g2_reduce_kernel(const double *__restrict__ part,
                                                        const int *__restrict__ cnt, int64_t nw, int nb,
                                                        int64_t ntiles, double *g2, int64_t *npairs) {
    const int slot = blockIdx.y;
    const int64_t tau = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (tau >= nw) return;
    const double *P = part + (int64_t)slot * ntiles * kDiag;
    const int *K = cnt + (int64_t)slot * ntiles * kDiag;
    double s = 0.0;
    int64_t c = 0;
    const int64_t D0 = tau / kTile;
    for (int64_t D = D0; D <= D0 + 1 && D < nb; ++D) {
        const int64_t d = tau - D * kTile;          // offset inside the tile
        if (d < -(kTile - 1)) continue;
        if (D == 0 && d < 0) continue;
        const int64_t first = D * nb - D * (D - 1) / 2;
        for (int64_t bi = 0; bi < nb - D; ++bi) {
            const int64_t id = first + bi;
            s += P[id * kDiag + d + kTile - 1];
            c += K[id * kDiag + d + kTile - 1];
        }
    }
    g2[(int64_t)slot * nw + tau] = c ? s / (double)c : __builtin_nan("");
    if (npairs) npairs[(int64_t)slot * nw + tau] = c;
}

}  // namespace

xpcs_status launch_raw_gram_tiles(xpcs_ctx *ctx, const int8_t *xs, int64_t ldx, const int64_t *off,
                                  const int64_t *roi_npix, const int64_t *S, int64_t nw, int r0, int nr,
                                  const int *amax, int64_t max_roi_pixels, const TileOut &o) {
    Phase phase_(ctx, "raw_gram_tiles");
    const int nb = (int)((nw + kTile - 1) / kTile);
    const int64_t nt = n_tiles_upper(nw);
    if (nt > 2147483647LL) return fail(ctx, XPCS_EUNSUPPORTED, "window too large");
    dim3 grid((unsigned)nt, (unsigned)nr);
    const bool vec = o.C && o.c_dtype == XPCS_F32 && (o.ldc % 4 == 0) &&
                     ((uintptr_t)o.C % 16 == 0) && (o.c_roi_stride % 4 == 0);
    // The wide variant is only needed when some ROI can exceed the smallest int32 chunk
    // (counts <= 127: 133,120 pixels); M bounds every ROI.
    const bool maybe_wide = max_roi_pixels > 133120;
    dim3 wgrid((unsigned)nb, (unsigned)nr);
    if (o.C == nullptr || o.c_dtype == XPCS_F32) {
        hipLaunchKernelGGL(raw_gram_tile_kernel<float>, grid, dim3(256), 0, ctx->stream, xs, ldx, off,
                           roi_npix, S, nw, r0, nb, amax, static_cast<float *>(o.C), o.ldc,
                           o.c_roi_stride, vec, o.gram_out, o.gram_roi_stride, o.g2_part, o.g2_cnt);
        if (maybe_wide)
            hipLaunchKernelGGL(raw_gram_wide_kernel<float>, wgrid, dim3(256), 0, ctx->stream, xs, ldx, off,
                               roi_npix, S, nw, r0, nb, amax, static_cast<float *>(o.C), o.ldc,
                               o.c_roi_stride, vec, o.gram_out, o.gram_roi_stride, o.g2_part, o.g2_cnt);
    } else {
        hipLaunchKernelGGL(raw_gram_tile_kernel<double>, grid, dim3(256), 0, ctx->stream, xs, ldx, off,
                           roi_npix, S, nw, r0, nb, amax, static_cast<double *>(o.C), o.ldc,
                           o.c_roi_stride, false, o.gram_out, o.gram_roi_stride, o.g2_part, o.g2_cnt);
        if (maybe_wide)
            hipLaunchKernelGGL(raw_gram_wide_kernel<double>, wgrid, dim3(256), 0, ctx->stream, xs, ldx, off,
                               roi_npix, S, nw, r0, nb, amax, static_cast<double *>(o.C), o.ldc,
                               o.c_roi_stride, false, o.gram_out, o.gram_roi_stride, o.g2_part, o.g2_cnt);
    }
    XPCS_LAUNCH_CHECK(ctx, "raw_gram_tiles");
    return XPCS_OK;
}

xpcs_status launch_lowrank_tiles(xpcs_ctx *ctx, const unsigned short *z_hi, const unsigned short *z_lo, int kp,
                                 const unsigned char *valid, int64_t nw, int nr, const TileOut &o) {
    Phase phase_(ctx, "lowrank_tiles");
    const int nb = (int)((nw + kTile - 1) / kTile);
    const int64_t nt = n_tiles_upper(nw);
    if (nt > 2147483647LL) return fail(ctx, XPCS_EUNSUPPORTED, "window too large");
    if (kp % 32) return fail(ctx, XPCS_EINVAL, "internal: kp must be a multiple of 32");
    dim3 grid((unsigned)nt, (unsigned)nr);
    const bool vec = o.C && o.c_dtype == XPCS_F32 && (o.ldc % 4 == 0) &&
                     ((uintptr_t)o.C % 16 == 0) && (o.c_roi_stride % 4 == 0);
    if (o.C == nullptr || o.c_dtype == XPCS_F32)
        hipLaunchKernelGGL(lowrank_tile_kernel<float>, grid, dim3(256), 0, ctx->stream, z_hi, z_lo, kp, valid, nw,
                           nb, static_cast<float *>(o.C), o.ldc, o.c_roi_stride, vec, o.g2_part, o.g2_cnt);
    else
        hipLaunchKernelGGL(lowrank_tile_kernel<double>, grid, dim3(256), 0, ctx->stream, z_hi, z_lo, kp, valid, nw,
                           nb, static_cast<double *>(o.C), o.ldc, o.c_roi_stride, false, o.g2_part, o.g2_cnt);
    XPCS_LAUNCH_CHECK(ctx, "lowrank_tiles");
    return XPCS_OK;
}

xpcs_status launch_matrix_diag_tiles(xpcs_ctx *ctx, const void *C, int c_dtype, int64_t n, int64_t ldc,
                                     double *g2_part, int *g2_cnt) {
    Phase phase_(ctx, "matrix_diag_tiles");
    const int nb = (int)((n + kTile - 1) / kTile);
    const int64_t nt = n_tiles_upper(n);
    if (c_dtype == XPCS_F32)
        hipLaunchKernelGGL(matrix_diag_tile_kernel<float>, dim3((unsigned)nt), dim3(256), 0, ctx->stream,
                           static_cast<const float *>(C), n, ldc, nb, g2_part, g2_cnt);
    else
        hipLaunchKernelGGL(matrix_diag_tile_kernel<double>, dim3((unsigned)nt), dim3(256), 0, ctx->stream,
                           static_cast<const double *>(C), n, ldc, nb, g2_part, g2_cnt);
    XPCS_LAUNCH_CHECK(ctx, "matrix_diag_tiles");
    return XPCS_OK;
}

xpcs_status launch_g2_reduce(xpcs_ctx *ctx, const double *g2_part, const int *g2_cnt, int64_t nw, int nr,
                             double *g2, int64_t *npairs) {
    Phase phase_(ctx, "g2_reduce");
    const int nb = (int)((nw + kTile - 1) / kTile);
    dim3 grid((unsigned)((nw + 255) / 256), (unsigned)nr);
    hipLaunchKernelGGL(g2_reduce_kernel, grid, dim3(256), 0, ctx->stream, g2_part, g2_cnt, nw, nb,
                       n_tiles_upper(nw), g2, npairs);
    XPCS_LAUNCH_CHECK(ctx, "g2_reduce");
    return XPCS_OK;
}

}  // namespace xpcs
