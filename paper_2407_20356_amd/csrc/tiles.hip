// The N x N tile pass shared by the raw and the compressed two-time correlation.
//
// C is symmetric (Sec. 2.1, Eq. 2: G = X X^T), so only the tiles on and above
// the block diagonal are computed; each is written at (i, j) and mirrored at
// (j, i) from the same value, which makes C exactly symmetric.  The g2 lag
// average (Sec. 3.1, Eq. 12) is fused into the same pass: every tile leaves the
// sums of its 255 diagonals t2 - t1 = const in a partial buffer, and a second,
// fixed-order pass adds them per lag (no float atomics, deterministic).
//
// Block shapes: the low-rank tiles and the wide raw variant use 256 threads = 4
// waves in a 2 x 2 arrangement, each wave owning a 64 x 64 quarter of the
// 128 x 128 tile as 4 x 4 MFMA 16 x 16 blocks, and an epilogue that stages one
// 64-row half of the tile in LDS at a time so that both the direct and the
// mirrored writes go out as contiguous rows; the common raw case uses 256 x 256
// super-tiles (one 128-tile per wave, below).
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

// The tile a block of the low-rank tile pass takes.  The hardware deals the linear
// block ids round-robin over the 8 XCDs; here XCD v's blocks take consecutive
// positions of one range of the (ROI, tile) sequence, and each ROI's tiles go in
// bands of kOrderRows tile rows, column by column, so that the blocks an XCD runs
// at once read the Z rows of a few tile rows and columns through its own L2.  tid is
// the tile's diagonal-major index (as tile_coords), which places its partial sums.
constexpr int kOrderRows = 8;
__device__ __forceinline__ void xcd_tile_order(int64_t bx, int64_t by, int64_t nt, int64_t nr, int nb, int &slot,
                                               int &bi, int &bj, int64_t &tid) {
    const int64_t T = nt * nr, L = bx + nt * by;
    const int64_t q = T / 8, r = T % 8, v = L % 8, s = L / 8;
    const int64_t g = v * q + (v < r ? v : r) + s;       // a bijection of [0, T)
    slot = (int)(g / nt);
    int64_t rem = g % nt;
    int i0 = 0, h = 0;
    for (;;) {
        h = nb - i0 < kOrderRows ? nb - i0 : kOrderRows;
        const int64_t band = (int64_t)h * (h + 1) / 2 + (int64_t)h * (nb - i0 - h);
        if (rem < band || i0 + h >= nb) break;
        rem -= band;
        i0 += h;
    }
    const int64_t tri = (int64_t)h * (h + 1) / 2;        // the band's diagonal block, column c holds c + 1 tiles
    if (rem < tri) {
        int c = (int)((sqrt(8.0 * (double)rem + 1.0) - 1.0) * 0.5);
        while (c > 0 && (int64_t)c * (c + 1) / 2 > rem) --c;
        while ((int64_t)(c + 1) * (c + 2) / 2 <= rem) ++c;
        bi = i0 + (int)(rem - (int64_t)c * (c + 1) / 2);
        bj = i0 + c;
    } else {                                             // then h tiles per column
        const int64_t r2 = rem - tri;
        bi = i0 + (int)(r2 % h);
        bj = i0 + h + (int)(r2 / h);
    }
    const int64_t D = bj - bi;
    tid = D * nb - D * (D - 1) / 2 + bi;
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

// The counts of the hot positions (a count of 128 or more somewhere) of a ROI, for
// the higher planes that the int8 gather leaves out (WIDE path only).
template <typename T>
struct HotIn {
    const T *frames = nullptr;          // the frames of the window start at frames + t0 * M
    int64_t M = 0, t0 = 0;
    const int32_t *perm = nullptr;      // pixel of each ROI-sorted position
    const int64_t *hq = nullptr;        // hot positions of ROI r: hq[off[r] + i], i < hcnt[r]
    const int *hcnt = nullptr;
    const int *hbits = nullptr;         // bit 1: some count of the ROI needs plane 2
};
constexpr int kHotPitch = 64 + 8;       // LDS row pitch (u16) of 64 staged hot counts

// 16 counts (u16, K order) -> one int8 operand of their 7-bit plane p.
__device__ __forceinline__ i32x4 hot_plane_frag(const unsigned short *src, int p) {
    const i32x4 lo = *reinterpret_cast<const i32x4 *>(src), hi = *reinterpret_cast<const i32x4 *>(src + 8);
    const unsigned m = p == 2 ? 3u : 127u;
    const int sh = 7 * p;
    i32x4 out;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const unsigned w0 = (unsigned)(d < 2 ? lo[2 * d] : hi[2 * d - 4]);
        const unsigned w1 = (unsigned)(d < 2 ? lo[2 * d + 1] : hi[2 * d - 3]);
        const unsigned b0 = ((w0 & 0xffffu) >> sh) & m, b1 = ((w0 >> 16) >> sh) & m;
        const unsigned b2 = ((w1 & 0xffffu) >> sh) & m, b3 = ((w1 >> 16) >> sh) & m;
        out[d] = (int)(b0 | (b1 << 8) | (b2 << 16) | (b3 << 24));
    }
    return out;
}

template <typename OutT, bool WIDE, typename T = uint8_t>
__device__ __forceinline__ void raw_gram_tile(
    int bi, int bj, int64_t tile_id, const int8_t *__restrict__ xs, int64_t ldx, const int64_t *__restrict__ off,
    const int64_t *__restrict__ roi_npix, const int64_t *__restrict__ S, int64_t nw, int r0, int slot,
    int64_t ntiles, int64_t kc, OutT *C, int64_t ldc, int64_t c_roi_stride, bool vec, int64_t *gram_out,
    int64_t gram_roi_stride, double *g2_part, int *g2_cnt, const HotIn<T> &hot = HotIn<T>()) {
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
    // Higher planes of the hot positions: the Gram of the counts is the sum over
    // plane pairs (pa, pb) of 2^(7 (pa + pb)) P_pa P_pb^T; plane 0 of every position
    // is done above, the other pairs only involve the hot positions.  Their counts
    // are staged in LDS 64 positions at a time (rows as in the main loop), each
    // pair's products formed in int32 over the 64 positions and added shifted.
    if constexpr (WIDE) {
        const int nh = hot.hcnt[roi];
        if (nh > 0) {
            const int np = (hot.hbits[roi] & 2) ? 3 : 2;
            const int64_t *hl = hot.hq + q0;
            unsigned short *hs = reinterpret_cast<unsigned short *>(stage);
            for (int h0 = 0; h0 < nh; h0 += 64) {
                {
                    const int c = threadIdx.x & 63;
                    const int px = h0 + c < nh ? hot.perm[hl[h0 + c]] : -1;
                    for (int i = 0; i < 64; ++i) {
                        const int row = (threadIdx.x >> 6) + 4 * i;
                        const int64_t t = row < kTile ? i0 + row : j0 + (row - kTile);
                        unsigned v = 0;
                        if (px >= 0 && t < nw && !(diag && row >= kTile)) v = hot.frames[(hot.t0 + t) * hot.M + px];
                        hs[row * kHotPitch + c] = (unsigned short)v;
                    }
                }
                __syncthreads();
                if (!skip) {
                    for (int pa = 0; pa < np; ++pa)
                        for (int pb = 0; pb < np; ++pb) {
                            if (pa == 0 && pb == 0) continue;
                            i32x4 av[4], bv[4];
#pragma unroll
                            for (int a = 0; a < 4; ++a)
                                av[a] = hot_plane_frag(hs + (64 * wr + 16 * a + lr) * kHotPitch + 16 * lg, pa);
#pragma unroll
                            for (int b = 0; b < 4; ++b)
                                bv[b] = hot_plane_frag(hs + (jrow0 + 64 * wc + 16 * b + lr) * kHotPitch + 16 * lg, pb);
#pragma unroll
                            for (int a = 0; a < 4; ++a)
#pragma unroll
                                for (int b = 0; b < 4; ++b) {
                                    const i32x4 tp = mfma_i8(av[a], bv[b], (i32x4){0, 0, 0, 0});
#pragma unroll
                                    for (int e = 0; e < 4; ++e) wide[a][b][e] += (int64_t)tp[e] << (7 * (pa + pb));
                                }
                        }
                }
                __syncthreads();
            }
        }
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
                        const double v = (si > 0.0 && sj > 0.0) ? (npix * (double)gval(a, b, e)) / (si * sj)
                                                                : __builtin_nan("");
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

// Whether a ROI takes the int32 fast path: its plane-0 sums are exact in one chunk
// and none of its positions needs a higher plane.
__device__ __forceinline__ bool raw_fast_roi(const int *__restrict__ amax, int64_t qlen, const int *__restrict__ hcnt,
                                             int roi) {
    return qlen <= raw_chunk_pixels(amax, qlen) && hcnt[roi] == 0;
}

// One block per 128-tile (windows too short to fill the GPU with super-tiles), for
// the fast-path ROIs.
template <typename OutT>
__global__ __launch_bounds__(256, 2) void raw_gram_tile_kernel(
    const int8_t *__restrict__ xs, int64_t ldx, const int64_t *__restrict__ off,
    const int64_t *__restrict__ roi_npix, const int64_t *__restrict__ S, int64_t nw, int r0, int nb,
    const int *__restrict__ amax, const int *__restrict__ hcnt, OutT *C, int64_t ldc, int64_t c_roi_stride, bool vec,
    int64_t *gram_out, int64_t gram_roi_stride, double *g2_part, int *g2_cnt) {
    const int slot = blockIdx.y, roi = r0 + slot;
    const int64_t qlen = off[roi + 1] - off[roi];
    if (!raw_fast_roi(amax, qlen, hcnt, roi)) return;
    int bi, bj;
    tile_coords(blockIdx.x, nb, bi, bj);
    raw_gram_tile<OutT, false>(bi, bj, blockIdx.x, xs, ldx, off, roi_npix, S, nw, r0, slot, gridDim.x,
                               raw_chunk_pixels(amax, qlen), C, ldc, c_roi_stride, vec, gram_out, gram_roi_stride,
                               g2_part, g2_cnt);
}

// One block per 128-tile for the other ROIs: int32 chunks of plane 0 folded into
// int64, then the higher planes of the hot positions.  Blocks of fast-path ROIs
// leave at once.
template <typename OutT, typename T>
__global__ __launch_bounds__(256, 2) void raw_gram_slow_kernel(
    const int8_t *__restrict__ xs, int64_t ldx, const int64_t *__restrict__ off,
    const int64_t *__restrict__ roi_npix, const int64_t *__restrict__ S, int64_t nw, int r0, int nb,
    const int *__restrict__ amax, OutT *C, int64_t ldc, int64_t c_roi_stride, bool vec, int64_t *gram_out,
    int64_t gram_roi_stride, double *g2_part, int *g2_cnt, HotIn<T> hot) {
    const int slot = blockIdx.y, roi = r0 + slot;
    const int64_t qlen = off[roi + 1] - off[roi];
    if (raw_fast_roi(amax, qlen, hot.hcnt, roi)) return;
    int bi, bj;
    tile_coords(blockIdx.x, nb, bi, bj);
    raw_gram_tile<OutT, true, T>(bi, bj, blockIdx.x, xs, ldx, off, roi_npix, S, nw, r0, slot, gridDim.x,
                                 raw_chunk_pixels(amax, qlen), C, ldc, c_roi_stride, vec, gram_out, gram_roi_stride,
                                 g2_part, g2_cnt, hot);
}

// ---------------------------------------------------------------- raw Gram, 256 x 256 super-tiles
// The common case of the raw path -- a ROI whose int32 sums are exact in one chunk
// (every count fits int8, pixels * amax^2 < 2^31) -- runs on super-tiles of 256 x 256
// frames: 4 waves, each owning one 128 x 128 tile of it as 8 x 8 int8 MFMA blocks
// (256 accumulator registers per lane), so that every 16-byte operand fragment read
// from LDS feeds 8 MFMAs and every staged row serves two tiles; a super-tile reads
// half the operand bytes per output of a 128-tile block.  Each wave then writes its
// own tile (waves whose tile lies below the diagonal or past the window skip it).
constexpr int kSup = 2 * kTile;
constexpr int kSupKs = 64;                                  // pixels (bytes) per K step
constexpr int kSupRows = 2 * kSup;                          // staged rows: row block, column block
constexpr int kSupStage = kSupRows * kSupKs;                // bytes per staged K step (rows of 64 bytes)
constexpr int kSupUnits = kSupStage / 1024 / 4;             // 1 KB direct-to-LDS loads per wave and K step
constexpr int kEpiRows = 32;                                // rows of a tile staged at a time
constexpr int kEpiWave = kEpiRows * kPitch;                 // doubles of one wave's staging area
static_assert(kSupStage <= kEpiWave * 8, "a K stage fits one wave's epilogue area");

// s_waitcnt vmcnt(n) with no wait on the other counters (gfx9 encoding).
template <int N>
__device__ __forceinline__ void sup_wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// Wave-level epilogue of one 128 x 128 tile held in acc[8][8] (rows 16a + 4lg + e,
// columns 16b + lr of the tile): four passes of 32 rows, each staged as normalised
// doubles in the wave's own LDS area, then written as direct rows and mirrored
// columns (contiguous in both), and summed along the tile's 255 diagonals (lane l
// owns diagonals l - 127 + 64k, k = 0..3).
template <typename OutT, bool GRAM>
__device__ __forceinline__ void raw_tile_epilogue_wave(const i32x4 (&acc)[8][8], double *st, int64_t i0,
                                                       int64_t j0, bool diag, int64_t nw,
                                                       const int64_t *__restrict__ Sr, double npix,
                                                       OutT *C, int64_t ldc, bool vec, int64_t *Gr,
                                                       double *g2p, int *g2c) {
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    // C = npix G / (S_i S_j) as npix G (1 / S_i) (1 / S_j): one division per row and
    // per column instead of one per element (a few ulp from the quotient)
    double rcol[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int64_t j = j0 + 16 * b + lr;
        const double sj = j < nw ? (double)Sr[j] : 0.0;
        rcol[b] = sj > 0.0 ? 1.0 / sj : __builtin_nan("");
    }
    double dsum[4] = {0.0, 0.0, 0.0, 0.0};
    int dcnt[4] = {0, 0, 0, 0};
    // no NaN in the tile when every frame of its rows and columns has photons: then the
    // diagonal sums need no per-entry check (same terms, same order)
    bool has_ph = true;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t i = i0 + 64 * h + lane, j = j0 + 64 * h + lane;
        if (i < nw && !(Sr[i] > 0)) has_ph = false;
        if (j < nw && !(Sr[j] > 0)) has_ph = false;
    }
    const bool nan_free = __all(has_ph);
#pragma unroll
    for (int qr = 0; qr < 4; ++qr) {
        // stage rows [32 qr, 32 qr + 32) of the tile
#pragma unroll
        for (int ah = 0; ah < 2; ++ah)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int rl = 16 * ah + 4 * lg + e;
                const int64_t i = i0 + kEpiRows * qr + rl;
                const double si = i < nw ? (double)Sr[i] : 0.0;
                const double ri = si > 0.0 ? npix / si : __builtin_nan("");
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const int g = acc[2 * qr + ah][b][e];
                    st[rl * kPitch + 16 * b + lr] = ((double)g * ri) * rcol[b];
                    if constexpr (GRAM) {
                        // the exact Gram (a verification output), mirrored
                        const int64_t j = j0 + 16 * b + lr;
                        if (i < nw && j < nw && j >= i) {
                            Gr[i * nw + j] = (int64_t)g;
                            Gr[j * nw + i] = (int64_t)g;
                        }
                    }
                }
            }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int r0 = kEpiRows * qr;
        if (C) {
            // direct rows: 32 lanes x 4 columns per row, 2 rows per pass
#pragma unroll 1
            for (int pass = 0; pass < kEpiRows / 2; ++pass) {
                const int rl = 2 * pass + (lane >> 5);
                const int c = (lane & 31) * 4;
                const int64_t i = i0 + r0 + rl;
                if (i < nw) {
                    OutT v[4];
                    bool ok[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        ok[e] = (j0 + c + e < nw) && (!diag || c + e >= r0 + rl);
                        v[e] = (OutT)st[rl * kPitch + c + e];
                    }
                    store4(C + i * ldc + j0 + c, v, ok, vec);
                }
            }
            // mirrored columns: 8 lanes x 4 rows per column, 8 columns per pass
#pragma unroll 1
            for (int pass = 0; pass < kTile / 8; ++pass) {
                const int c = 8 * pass + (lane >> 3);
                const int rq = (lane & 7) * 4;
                const int64_t j = j0 + c;
                if (j < nw) {
                    OutT v[4];
                    bool ok[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int r = r0 + rq + e;
                        ok[e] = (i0 + r < nw) && (!diag || c > r);
                        v[e] = (OutT)st[(rq + e) * kPitch + c];
                    }
                    store4(C + j * ldc + i0 + r0 + rq, v, ok, vec);
                }
            }
        }
        if (g2p) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int d = lane - (kTile - 1) + 64 * k;        // c - r
                if (d > kTile - 1 || (diag && d < 0)) continue;
                int r_lo = r0, r_hi = r0 + kEpiRows;
                if (d < 0 && r_lo < -d) r_lo = -d;                     // c = r + d >= 0
                if (d > 0 && r_hi > kTile - d) r_hi = kTile - d;       // c = r + d < kTile
                if (i0 + r_hi > nw) r_hi = (int)(nw - i0);             // rows inside the window
                const int64_t c_lim = nw - j0 - d;                     // and columns
                if (r_hi > c_lim) r_hi = (int)c_lim;
                if (nan_free) {
#pragma unroll 8
                    for (int r = r_lo; r < r_hi; ++r) dsum[k] += st[(r - r0) * kPitch + r + d];
                    dcnt[k] += r_hi > r_lo ? r_hi - r_lo : 0;
                } else {
                    for (int r = r_lo; r < r_hi; ++r) {
                        const double v = st[(r - r0) * kPitch + r + d];
                        if (v == v) {
                            dsum[k] += v;
                            dcnt[k] += 1;
                        }
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (g2p) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int slot = lane + 64 * k;
            if (slot < kDiag) {
                g2p[slot] = dsum[k];
                g2c[slot] = dcnt[k];
            }
        }
    }
}

template <typename OutT, bool GRAM>
__global__ __launch_bounds__(256, 1) void raw_gram_super_kernel(
    const int8_t *__restrict__ xs, int64_t ldx, const int64_t *__restrict__ off,
    const int64_t *__restrict__ roi_npix, const int64_t *__restrict__ S, int64_t nw, int r0, int nb, int nb2,
    const int *__restrict__ amax, const int *__restrict__ hcnt, OutT *C, int64_t ldc, int64_t c_roi_stride, bool vec,
    int64_t *gram_out, int64_t gram_roi_stride, double *g2_part, int *g2_cnt) {
    // four LDS areas, one per wave for the epilogue; the first three are the stage
    // buffers of the K loop (distinct arrays, so that the compiler sees which buffer a
    // load fills)
    __shared__ __attribute__((aligned(1024))) double e0[kEpiWave], e1[kEpiWave], e2[kEpiWave], e3[kEpiWave];
    const int slot = blockIdx.y, roi = r0 + slot;
    const int64_t q0 = off[roi], qlen = off[roi + 1] - off[roi];
    if (!raw_fast_roi(amax, qlen, hcnt, roi)) return;            // the slow kernel's ROI
    int bi2, bj2;
    tile_coords(blockIdx.x, nb2, bi2, bj2);
    const bool dsup = bi2 == bj2;
    const int64_t I0 = (int64_t)bi2 * kSup, J0 = (int64_t)bj2 * kSup;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
    const int lr = lane & 15, lg = lane >> 4;

    i32x4 acc[8][8];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = (i32x4){0, 0, 0, 0};

    // K steps of 64 pixels: the super-tile's 512 rows (256 of the row block, 256 of the
    // column block; on the diagonal the row block twice) reach LDS by direct-to-LDS
    // loads (each lane's 16 bytes land at the wave's LDS address + 16 * lane), rows of
    // 64 bytes whose four 16-byte pieces are XOR-swizzled (piece p of row r in slot
    // p ^ ((r >> 1) & 3): the fragment reads of eight consecutive rows fall on distinct
    // banks).  Two buffers alternate: after the barrier that publishes step st, a wave
    // reads all its fragments of step st, then starts the loads of step st + 1 into the
    // other buffer (which every wave finished reading before the barrier) and
    // multiplies while they fly; no load is pending while LDS is read.  Rows past the
    // window read the block's first row (their products land in tiles nobody reads).
    const int nsteps = (int)((qlen + kSupKs - 1) / kSupKs);
    const int jrow0 = dsup ? 0 : kSup;
    const int8_t *lsrc[kSupUnits];
#pragma unroll
    for (int j = 0; j < kSupUnits; ++j) {
        const int u = w + 4 * j;
        const int row = 16 * u + (lane >> 2);
        const int piece = (lane & 3) ^ ((row >> 1) & 3);
        const int64_t base = row < kSup || dsup ? I0 : J0;
        int64_t t = base + (row & (kSup - 1));
        if (t >= nw) t = base;
        lsrc[j] = xs + t * ldx + q0 + 16 * piece;
    }
    auto issue = [&](int st, double *dst) {
#pragma unroll
        for (int j = 0; j < kSupUnits; ++j) {
            const int u = w + 4 * j;
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const void *>(lsrc[j] + (int64_t)st * kSupKs),
                                             (__attribute__((address_space(3))) void *)(
                                                 reinterpret_cast<char *>(dst) + 1024 * u),
                                             16, 0, 0);
        }
    };
    // the lane's fragment rows: 16 a + lr of its row block, 16 b + lr of its column block
    const int arow = 128 * wr + lr, brow = jrow0 + 128 * wc + lr;
    const int aoff = arow * kSupKs + 16 * (lg ^ ((arow >> 1) & 3));
    const int boff = brow * kSupKs + 16 * (lg ^ ((brow >> 1) & 3));
    if (nsteps > 0) issue(0, e0);
    for (int st = 0; st < nsteps; ++st) {
        double *cur = st & 1 ? e1 : e0, *nxt = st & 1 ? e0 : e1;
        asm volatile("" ::: "memory");
        sup_wait_vmcnt<0>();
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        // every wave multiplies (a wave whose tile is below the diagonal or past the
        // window computes values nobody reads): a branch here would move the
        // accumulators out of their registers every step
        const int8_t *src = reinterpret_cast<const int8_t *>(cur);
        i32x4 av[8], bv[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) bv[b] = *reinterpret_cast<const i32x4 *>(src + boff + 1024 * b);
#pragma unroll
        for (int a = 0; a < 8; ++a) av[a] = *reinterpret_cast<const i32x4 *>(src + aoff + 1024 * a);
        asm volatile("" ::: "memory");
        if (st + 1 < nsteps) issue(st + 1, nxt);
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int b = 0; b < 8; ++b) acc[a][b] = mfma_i8(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();

    // each wave writes its own tile through its own LDS area
    const int tbi = 2 * bi2 + wr, tbj = 2 * bj2 + wc;
    if (tbi >= nb || tbj >= nb || tbi > tbj) return;
    const int64_t i0 = (int64_t)tbi * kTile, j0 = (int64_t)tbj * kTile;
    const int64_t *Sr = S + (int64_t)roi * nw;
    const int64_t D = tbj - tbi;
    const int64_t tile = (int64_t)slot * ((int64_t)nb * (nb + 1) / 2) + D * nb - D * (D - 1) / 2 + tbi;
    double *const area = w == 0 ? e0 : (w == 1 ? e1 : (w == 2 ? e2 : e3));
    raw_tile_epilogue_wave<OutT, GRAM>(acc, area, i0, j0, tbi == tbj, nw, Sr, (double)roi_npix[roi],
                                 C ? C + (int64_t)slot * c_roi_stride : nullptr, ldc, vec,
                                 gram_out ? gram_out + (int64_t)slot * gram_roi_stride : nullptr,
                                 g2_part ? g2_part + tile * kDiag : nullptr, g2_part ? g2_cnt + tile * kDiag : nullptr);
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
    int slot, bi, bj;
    int64_t tile;
    xcd_tile_order(blockIdx.x, blockIdx.y, gridDim.x, gridDim.y, nb, slot, bi, bj, tile);
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
    write_diag_partials(g2_part, g2_cnt, (int64_t)slot * gridDim.x + tile, dsum, dcnt);
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
                                  const int *amax, const RawHot &h, const TileOut &o) {
    Phase phase_(ctx, "raw_gram_tiles");
    const int nb = (int)((nw + kTile - 1) / kTile);
    const int64_t nt = n_tiles_upper(nw);
    if (nt > 2147483647LL) return fail(ctx, XPCS_EUNSUPPORTED, "window too large");
    const bool vec = o.C && o.c_dtype == XPCS_F32 && (o.ldc % 4 == 0) &&
                     ((uintptr_t)o.C % 16 == 0) && (o.c_roi_stride % 4 == 0);
    const bool f32 = o.C == nullptr || o.c_dtype == XPCS_F32;
    float *Cf = static_cast<float *>(o.C);
    double *Cd = static_cast<double *>(o.C);
    const int nb2 = (int)((nw + kSup - 1) / kSup);
    const int64_t nsup = (int64_t)nb2 * (nb2 + 1) / 2;
    const dim3 sgrid((unsigned)nsup, (unsigned)nr), grid((unsigned)nt, (unsigned)nr);
    // Fast-path ROIs on super-tiles once there are enough of them to give every CU a
    // block, else on 128-tiles; the slow kernel takes the other ROIs (which ROI is
    // which is only known on the device, so both launch).
    const bool sup = nsup * nr >= 256;
    if (!sup && f32)
        hipLaunchKernelGGL(raw_gram_tile_kernel<float>, grid, dim3(256), 0, ctx->stream, xs, ldx, off, roi_npix, S, nw,
                           r0, nb, amax, h.hcnt, Cf, o.ldc, o.c_roi_stride, vec, o.gram_out, o.gram_roi_stride,
                           o.g2_part, o.g2_cnt);
    else if (!sup)
        hipLaunchKernelGGL(raw_gram_tile_kernel<double>, grid, dim3(256), 0, ctx->stream, xs, ldx, off, roi_npix, S,
                           nw, r0, nb, amax, h.hcnt, Cd, o.ldc, o.c_roi_stride, false, o.gram_out,
                           o.gram_roi_stride, o.g2_part, o.g2_cnt);
    else if (f32 && o.gram_out)
        hipLaunchKernelGGL((raw_gram_super_kernel<float, true>), sgrid, dim3(256), 0, ctx->stream, xs, ldx, off,
                           roi_npix, S, nw, r0, nb, nb2, amax, h.hcnt, Cf, o.ldc, o.c_roi_stride, vec, o.gram_out,
                           o.gram_roi_stride, o.g2_part, o.g2_cnt);
    else if (f32)
        hipLaunchKernelGGL((raw_gram_super_kernel<float, false>), sgrid, dim3(256), 0, ctx->stream, xs, ldx, off,
                           roi_npix, S, nw, r0, nb, nb2, amax, h.hcnt, Cf, o.ldc, o.c_roi_stride, vec, o.gram_out,
                           o.gram_roi_stride, o.g2_part, o.g2_cnt);
    else if (o.gram_out)
        hipLaunchKernelGGL((raw_gram_super_kernel<double, true>), sgrid, dim3(256), 0, ctx->stream, xs, ldx, off,
                           roi_npix, S, nw, r0, nb, nb2, amax, h.hcnt, Cd, o.ldc, o.c_roi_stride, false, o.gram_out,
                           o.gram_roi_stride, o.g2_part, o.g2_cnt);
    else
        hipLaunchKernelGGL((raw_gram_super_kernel<double, false>), sgrid, dim3(256), 0, ctx->stream, xs, ldx, off,
                           roi_npix, S, nw, r0, nb, nb2, amax, h.hcnt, Cd, o.ldc, o.c_roi_stride, false, o.gram_out,
                           o.gram_roi_stride, o.g2_part, o.g2_cnt);
    XPCS_LAUNCH_CHECK(ctx, "raw_gram_tiles");
    auto slow = [&](auto tag) {
        typedef decltype(tag) T;
        HotIn<T> hi;
        hi.frames = static_cast<const T *>(h.frames);
        hi.M = h.M;
        hi.t0 = h.t0;
        hi.perm = h.perm;
        hi.hq = h.hq;
        hi.hcnt = h.hcnt;
        hi.hbits = h.hbits;
        if (f32)
            hipLaunchKernelGGL((raw_gram_slow_kernel<float, T>), grid, dim3(256), 0, ctx->stream, xs, ldx, off,
                               roi_npix, S, nw, r0, nb, amax, Cf, o.ldc, o.c_roi_stride, vec, o.gram_out,
                               o.gram_roi_stride, o.g2_part, o.g2_cnt, hi);
        else
            hipLaunchKernelGGL((raw_gram_slow_kernel<double, T>), grid, dim3(256), 0, ctx->stream, xs, ldx, off,
                               roi_npix, S, nw, r0, nb, amax, Cd, o.ldc, o.c_roi_stride, false, o.gram_out,
                               o.gram_roi_stride, o.g2_part, o.g2_cnt, hi);
    };
    if (h.dtype == XPCS_U8)
        slow(uint8_t{});
    else
        slow(uint16_t{});
    XPCS_LAUNCH_CHECK(ctx, "raw_gram_slow");
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
