// Small dense FP64 steps of the compression: orthonormalisation of the
// tall-skinny sketches (Cholesky QR), the l x l symmetric eigendecomposition that
// ranks the sketched directions by their eigenvalue (Sec. 2.1, Eq. 3: the
// encoding vectors are Gram eigenvectors; Eq. 6: keep the K largest), and the
// tall x small products that assemble the basis.
#include <math.h>

#include <type_traits>

#include "internal.hpp"

namespace xpcs {
namespace {

constexpr int kMaxSmall = 192;                    // largest l handled on chip
constexpr int kPacked = kMaxSmall * (kMaxSmall + 1) / 2;

// ---------------------------------------------------------------- tall-skinny Gram
// Partial Grams over row ranges: part[(seg*gridDim.x + blk)][a][b] (upper 4x4 blocks
// written in full), FP64 throughout (products of fp32 inputs are exact in FP64).
// A block of 1, 2 or 4 groups of 256 threads walks its rows in chunks, each chunk
// staged in LDS as doubles (coalesced column reads, the next chunk fetched into
// registers while the current one is multiplied).  Each group takes an equal
// share of every chunk; thread j of a group owns 4x4 blocks j, j + 256, ... of the
// upper block triangle, and the groups' sums are added in a fixed order at the end.
// Groups per block and rows per chunk by blocks per thread (register budget):
// BPT 1: 4 groups x 32 rows; BPT 2: 2 x 32; BPT >= 3: 1 x 16.
template <int BPT>
struct GramShape {
    static constexpr int kGroups = BPT == 1 ? 4 : (BPT == 2 ? 2 : 1);
    static constexpr int kRows = BPT <= 2 ? 32 : 16;
};

template <typename T, int BPT>
__global__ __launch_bounds__(256 * GramShape<BPT>::kGroups) void tsgram_kernel(const T *__restrict__ A, int64_t rows, int64_t lda,
                                                              int ncols, const int32_t *__restrict__ row_idx,
                                                              const int64_t *__restrict__ seg_off, double *part) {
    constexpr int kGramGroups = GramShape<BPT>::kGroups, kGramRows = GramShape<BPT>::kRows;
    constexpr int kGramThreads = 256 * kGramGroups;
    extern __shared__ double tile[];                 // [kGramRows][pitch], later the groups' sums
    const int seg = blockIdx.y;
    const int nc4 = (ncols + 3) / 4;
    const int pitch = nc4 * 4 + 2;                   // even (16-byte reads), not a multiple of 32 banks
    const int nblk = nc4 * (nc4 + 1) / 2;
    int64_t r_begin = 0, r_end = rows;
    if (seg_off) {
        r_begin = seg_off[seg];
        r_end = seg_off[seg + 1];
    }
    const int64_t span = r_end - r_begin;
    const int64_t per = (span + gridDim.x - 1) / gridDim.x;
    const int64_t my0 = r_begin + per * blockIdx.x;
    const int64_t my1 = my0 + per < r_end ? my0 + per : r_end;
    const int grp = threadIdx.x >> 8, tj = threadIdx.x & 255;

    int ab[BPT], bb[BPT];
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int b = tj + 256 * k;
        ab[k] = bb[k] = -1;
        if (b < nblk) {
            // linear b -> (x <= y) in the row-major upper block triangle
            int x = 0, rem = b;
            while (rem >= nc4 - x) {
                rem -= nc4 - x;
                ++x;
            }
            ab[k] = x;
            bb[k] = x + rem;
        }
    }
    double acc[BPT][4][4];
#pragma unroll
    for (int k = 0; k < BPT; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[k][i][j] = 0.0;

    // chunk element e = c * kGramRows + rr (consecutive threads: consecutive rows of a column)
    const int per_thr = (kGramRows * nc4 * 4 + kGramThreads - 1) / kGramThreads;
    constexpr int kMaxPer = (kGramRows * kMaxSmall + kGramThreads - 1) / kGramThreads;
    double nxt[kMaxPer];
    auto fetch = [&](int64_t r0) {
#pragma unroll
        for (int q = 0; q < kMaxPer; ++q) {
            if (q >= per_thr) break;
            const int e = threadIdx.x + kGramThreads * q;
            const int c = e / kGramRows, rr = e % kGramRows;
            const int64_t r = r0 + rr;
            double v = 0.0;
            if (c < ncols && r < my1) {
                const int64_t src = row_idx ? (int64_t)row_idx[r] : r;
                if (src >= 0) v = (double)A[(int64_t)c * lda + src];
            }
            nxt[q] = v;
        }
    };
    auto put = [&]() {
#pragma unroll
        for (int q = 0; q < kMaxPer; ++q) {
            if (q >= per_thr) break;
            const int e = threadIdx.x + kGramThreads * q;
            const int c = e / kGramRows, rr = e % kGramRows;
            if (c < nc4 * 4) tile[rr * pitch + c] = nxt[q];
        }
    };
    if (my0 < my1) fetch(my0);
    for (int64_t r0 = my0; r0 < my1; r0 += kGramRows) {
        __syncthreads();
        put();
        __syncthreads();
        if (r0 + kGramRows < my1) fetch(r0 + kGramRows);
        constexpr int kRowsPerGroup = kGramRows / kGramGroups;
        const int rbeg = grp * kRowsPerGroup;
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            if (ab[k] >= 0) {
                const double *xa = tile + 4 * ab[k], *ya = tile + 4 * bb[k];
                // the next row's operands are read while the current row is multiplied
                double2 x01 = *reinterpret_cast<const double2 *>(xa + rbeg * pitch);
                double2 x23 = *reinterpret_cast<const double2 *>(xa + rbeg * pitch + 2);
                double2 y01 = *reinterpret_cast<const double2 *>(ya + rbeg * pitch);
                double2 y23 = *reinterpret_cast<const double2 *>(ya + rbeg * pitch + 2);
#pragma unroll
                for (int q = 0; q < kRowsPerGroup; ++q) {
                    const double x[4] = {x01.x, x01.y, x23.x, x23.y}, y[4] = {y01.x, y01.y, y23.x, y23.y};
                    if (q + 1 < kRowsPerGroup) {
                        const int o = (rbeg + q + 1) * pitch;
                        x01 = *reinterpret_cast<const double2 *>(xa + o);
                        x23 = *reinterpret_cast<const double2 *>(xa + o + 2);
                        y01 = *reinterpret_cast<const double2 *>(ya + o);
                        y23 = *reinterpret_cast<const double2 *>(ya + o + 2);
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) acc[k][i][j] = fma(x[i], y[j], acc[k][i][j]);
                }
            }
        }
    }
    // groups 1..3 hand their sums to group 0 through LDS, one at a time; group 0
    // adds them in group order and writes the partial
    for (int g = 1; g < kGramGroups; ++g) {
        __syncthreads();
        if (grp == g) {
#pragma unroll
            for (int k = 0; k < BPT; ++k)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (ab[k] >= 0) tile[((k * 256 + tj) * 4 + i) * 4 + j] = acc[k][i][j];
        }
        __syncthreads();
        if (grp == 0) {
#pragma unroll
            for (int k = 0; k < BPT; ++k)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (ab[k] >= 0) acc[k][i][j] += tile[((k * 256 + tj) * 4 + i) * 4 + j];
        }
    }
    if (grp == 0) {
        const int pw = nc4 * 4;
        double *out = part + ((int64_t)seg * gridDim.x + blockIdx.x) * pw * pw;
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            if (ab[k] >= 0) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) out[(4 * ab[k] + i) * pw + 4 * bb[k] + j] = acc[k][i][j];
            }
        }
    }
}

// Unsegmented Gram on FP64 MFMA (v_mfma_f64_16x16x4f64), up to 16 * NCB <= 80 columns:
// every 16 x 16 tile (I <= J) of a wave's Gram stays in registers.  In step j of a
// 16-row group, lane l supplies column 16 cb + l % 16 at row r0 + 4 (l / 16) + j,
// which serves as the A operand (tile rows) and as the B operand (tile columns)
// alike.  Entry (i, j) of a tile is lane l's value v with i = l / 16 + 4 v,
// j = l % 16.  Waves take every eighth 16-row group of the block's range, load
// the next group while multiplying the current one, and add their tiles in LDS in
// wave order; the block writes its partial (upper tiles) for the fixed-order reduce.
// Eight waves per block, two per SIMD, so that one's loads overlap the other's MFMAs.
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int kGramMfmaThreads = 512;     // 8 waves: two per SIMD
constexpr int kGramMfmaWaves = kGramMfmaThreads / 64;
// Four consecutive rows of one column in 16-byte loads (p 16-byte aligned).
__device__ __forceinline__ void load_rows4(const float *p, float (&x)[4]) {
    const float4 v = *reinterpret_cast<const float4 *>(p);
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
}
__device__ __forceinline__ void load_rows4(const double *p, double (&x)[4]) {
    const double2 a = reinterpret_cast<const double2 *>(p)[0], b = reinterpret_cast<const double2 *>(p)[1];
    x[0] = a.x; x[1] = a.y; x[2] = b.x; x[3] = b.y;
}

template <typename TA, int NCB>
__global__ __launch_bounds__(kGramMfmaThreads) void tsgram_mfma_kernel(const TA *__restrict__ A, int64_t rows, int64_t lda,
                                                          int ncols, int pw, double *__restrict__ part,
                                                          int64_t bstride, const int32_t *__restrict__ row_idx,
                                                          const int64_t *__restrict__ seg_off, bool vec) {
    // blockIdx.y selects one matrix of a batch (A + y * bstride) or, with seg_off,
    // one segment of the gathered row list row_idx (-1 entries count as zero
    // rows); partials follow the previous matrices' / segments' gridDim.x parts.
    // vec: no row list or segments, A, lda and bstride allow 16-byte loads of four
    // rows starting at a multiple of 4
    A += (int64_t)blockIdx.y * bstride;
    part += (int64_t)blockIdx.y * gridDim.x * pw * pw;
    const int64_t r_begin = seg_off ? seg_off[blockIdx.y] : 0;
    const int64_t r_end = seg_off ? seg_off[blockIdx.y + 1] : rows;
    constexpr int NT = NCB * (NCB + 1) / 2;
    constexpr int W = NCB * 16;
    __shared__ double red[W * W];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int cl = lane & 15, kq = lane >> 4;
    const int64_t ngroups = (r_end - r_begin + 15) / 16;
    const int64_t per_blk = (ngroups + gridDim.x - 1) / gridDim.x;
    const int64_t g0 = (int64_t)blockIdx.x * per_blk;
    const int64_t g1 = g0 + per_blk < ngroups ? g0 + per_blk : ngroups;
    f64x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = (f64x4){0.0, 0.0, 0.0, 0.0};
    auto load = [&](int64_t g, TA (&x)[NCB][4]) {
        const int64_t r = r_begin + g * 16 + 4 * kq;
        if (vec && r + 4 <= r_end) {
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const int c = 16 * cb + cl;
                if (c < ncols) {
                    load_rows4(A + (int64_t)c * lda + r, x[cb]);
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) x[cb][j] = (TA)0;
                }
            }
            return;
        }
        int64_t rowj[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t pos = r + j;
            rowj[j] = pos < r_end ? (row_idx ? (int64_t)row_idx[pos] : pos) : -1;
        }
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int c = 16 * cb + cl;
            const TA *src = A + (int64_t)(c < ncols ? c : 0) * lda;
#pragma unroll
            for (int j = 0; j < 4; ++j) x[cb][j] = (c < ncols && rowj[j] >= 0) ? src[rowj[j]] : (TA)0;
        }
    };
    TA cur[NCB][4], nxt[NCB][4];
    int64_t g = g0 + wv;
    if (g < g1) load(g, nxt);
    for (; g < g1; g += kGramMfmaWaves) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int j = 0; j < 4; ++j) cur[cb][j] = nxt[cb][j];
        if (g + kGramMfmaWaves < g1) load(g + kGramMfmaWaves, nxt);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double f[NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) f[cb] = (double)cur[cb][j];
            int t = 0;
#pragma unroll
            for (int I = 0; I < NCB; ++I)
#pragma unroll
                for (int J = I; J < NCB; ++J) {
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[I], f[J], acc[t], 0, 0, 0);
                    ++t;
                }
        }
    }
    for (int w = 0; w < kGramMfmaWaves; ++w) {
        if (wv == w) {
            int t = 0;
#pragma unroll
            for (int I = 0; I < NCB; ++I)
#pragma unroll
                for (int J = I; J < NCB; ++J) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int idx = (16 * I + kq + 4 * v) * W + 16 * J + cl;
                        red[idx] = (w == 0 ? 0.0 : red[idx]) + acc[t][v];
                    }
                    ++t;
                }
        }
        __syncthreads();
    }
    double *out = part + (int64_t)blockIdx.x * pw * pw;
    for (int idx = threadIdx.x; idx < pw * pw; idx += kGramMfmaThreads) {
        const int a = idx / pw, b = idx % pw;
        if (a / 16 <= b / 16) out[idx] = red[a * W + b];
    }
}

// Wider Grams (80 < columns <= 192) on the same FP64 MFMA.  The column blocks are
// split into ng groups of G blocks (blocks past the last column read as zeros and
// their tiles are not multiplied) and a launch takes the pairs of groups (P, Q):
// DIAG, P = Q = blockIdx.z, the upper G(G+1)/2 tiles of the group; otherwise the
// z-th pair P < Q and all G x G tiles.  Four waves per block (one per SIMD: a pair
// holds up to 25 tiles, 200 accumulator registers); each wave walks every fourth
// 16-row group of the block's rows, loading the next group while multiplying the
// current one, and the waves' tiles are added in LDS in wave order.  Tile layout
// and the partial's upper-tile format are those of the narrow kernel above.
constexpr int kGramPairThreads = 256;
constexpr int kGramPairWaves = kGramPairThreads / 64;

template <typename TA, int NB>
__device__ __forceinline__ void gram_rows_load(const TA *__restrict__ A, int64_t lda, int ncols, int c0, int64_t r,
                                               int64_t r_end, bool vec, const int32_t *__restrict__ row_idx,
                                               int cl, TA (&x)[NB][4]) {
    if (vec && r + 4 <= r_end) {
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
            const int c = c0 + 16 * cb + cl;
            if (c < ncols) {
                load_rows4(A + (int64_t)c * lda + r, x[cb]);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) x[cb][j] = (TA)0;
            }
        }
        return;
    }
    int64_t rowj[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t pos = r + j;
        rowj[j] = pos < r_end ? (row_idx ? (int64_t)row_idx[pos] : pos) : -1;
    }
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
        const int c = c0 + 16 * cb + cl;
        const TA *src = A + (int64_t)(c < ncols ? c : 0) * lda;
#pragma unroll
        for (int j = 0; j < 4; ++j) x[cb][j] = (c < ncols && rowj[j] >= 0) ? src[rowj[j]] : (TA)0;
    }
}

template <typename TA, int G, bool DIAG>
__global__ __launch_bounds__(kGramPairThreads) void tsgram_pair_kernel(const TA *__restrict__ A, int64_t rows,
                                                                       int64_t lda, int ncols, int pw, int ng,
                                                                       double *__restrict__ part,
                                                                       const int32_t *__restrict__ row_idx,
                                                                       const int64_t *__restrict__ seg_off, bool vec) {
    part += (int64_t)blockIdx.y * gridDim.x * pw * pw;
    const int64_t r_begin = seg_off ? seg_off[blockIdx.y] : 0;
    const int64_t r_end = seg_off ? seg_off[blockIdx.y + 1] : rows;
    int P = blockIdx.z, Q = blockIdx.z;
    if (!DIAG) {
        int rem = blockIdx.z;
        P = 0;
        while (rem >= ng - 1 - P) {
            rem -= ng - 1 - P;
            ++P;
        }
        Q = P + 1 + rem;
    }
    const int p0 = 16 * G * P, q0 = 16 * G * Q;          // first column of each group
    constexpr int W = 16 * G;
    __shared__ double red[W * W];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int cl = lane & 15, kq = lane >> 4;
    // blocks of the groups that hold columns (uniform across the block)
    const int nbp = (ncols - p0 + 15) / 16 < G ? (ncols - p0 + 15) / 16 : G;
    const int nbq = (ncols - q0 + 15) / 16 < G ? (ncols - q0 + 15) / 16 : G;
    const int64_t ngroups = (r_end - r_begin + 15) / 16;
    const int64_t per_blk = (ngroups + gridDim.x - 1) / gridDim.x;
    const int64_t g0 = (int64_t)blockIdx.x * per_blk;
    const int64_t g1 = g0 + per_blk < ngroups ? g0 + per_blk : ngroups;
    f64x4 acc[G][G];
#pragma unroll
    for (int I = 0; I < G; ++I)
#pragma unroll
        for (int J = 0; J < G; ++J) acc[I][J] = (f64x4){0.0, 0.0, 0.0, 0.0};
    constexpr int GJ = DIAG ? 1 : G;                     // the second group's rows (unused when DIAG)
    TA ci[G][4], ni[G][4], cj[GJ][4], nj[GJ][4];
    int64_t g = g0 + wv;
    if (g < g1) {
        const int64_t r = r_begin + g * 16 + 4 * kq;
        gram_rows_load<TA, G>(A, lda, ncols, p0, r, r_end, vec, row_idx, cl, ni);
        if constexpr (!DIAG) gram_rows_load<TA, GJ>(A, lda, ncols, q0, r, r_end, vec, row_idx, cl, nj);
    }
    for (; g < g1; g += kGramPairWaves) {
#pragma unroll
        for (int b = 0; b < G; ++b)
#pragma unroll
            for (int j = 0; j < 4; ++j) ci[b][j] = ni[b][j];
        if constexpr (!DIAG) {
#pragma unroll
            for (int b = 0; b < GJ; ++b)
#pragma unroll
                for (int j = 0; j < 4; ++j) cj[b][j] = nj[b][j];
        }
        if (g + kGramPairWaves < g1) {
            const int64_t r = r_begin + (g + kGramPairWaves) * 16 + 4 * kq;
            gram_rows_load<TA, G>(A, lda, ncols, p0, r, r_end, vec, row_idx, cl, ni);
            if constexpr (!DIAG) gram_rows_load<TA, GJ>(A, lda, ncols, q0, r, r_end, vec, row_idx, cl, nj);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double fi[G], fj[G];
#pragma unroll
            for (int b = 0; b < G; ++b) {
                fi[b] = (double)ci[b][j];
                fj[b] = DIAG ? fi[b] : (double)cj[DIAG ? 0 : b][j];
            }
#pragma unroll
            for (int I = 0; I < G; ++I)
#pragma unroll
                for (int J = DIAG ? I : 0; J < G; ++J)
                    if (I < nbp && J < nbq) acc[I][J] = __builtin_amdgcn_mfma_f64_16x16x4f64(fi[I], fj[J], acc[I][J], 0, 0, 0);
        }
    }
    for (int w = 0; w < kGramPairWaves; ++w) {
        if (wv == w) {
#pragma unroll
            for (int I = 0; I < G; ++I)
#pragma unroll
                for (int J = DIAG ? I : 0; J < G; ++J)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int idx = (16 * I + kq + 4 * v) * W + 16 * J + cl;
                        red[idx] = (w == 0 ? 0.0 : red[idx]) + acc[I][J][v];
                    }
        }
        __syncthreads();
    }
    double *out = part + (int64_t)blockIdx.x * pw * pw;
    for (int idx = threadIdx.x; idx < W * W; idx += kGramPairThreads) {
        const int la = idx / W, lb = idx % W;
        const int a = p0 + la, b = q0 + lb;
        if (a < pw && b < pw && (!DIAG || la / 16 <= lb / 16)) out[(int64_t)a * pw + b] = red[idx];
    }
}

// G[seg][a][b] = sum over parts of part[.][ra][rb], (ra, rb) the copy in an upper block.
// 8 threads per entry sum interleaved parts; the 8 sums are added in a fixed order.
__global__ __launch_bounds__(256) void tsgram_reduce_kernel(const double *__restrict__ part, int nparts, int ncols,
                                                            int pitch, double *__restrict__ G) {
    __shared__ double red[256];
    const int seg = blockIdx.y;
    const int64_t n2 = (int64_t)ncols * ncols;
    const int sub = threadIdx.x & 7;
    const int64_t idx = (int64_t)blockIdx.x * 32 + (threadIdx.x >> 3);
    double s = 0.0;
    if (idx < n2) {
        const int a = (int)(idx / ncols), b = (int)(idx % ncols);
        int ra = a, rb = b;
        if (a / 4 > b / 4) {
            ra = b;
            rb = a;
        }
        const double *p = part + (int64_t)seg * nparts * pitch * pitch + (int64_t)ra * pitch + rb;
        for (int k = sub; k < nparts; k += 8) s += p[(int64_t)k * pitch * pitch];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (sub == 0 && idx < n2) {
        double t = 0.0;
        for (int q = 0; q < 8; ++q) t += red[threadIdx.x + q];
        G[(int64_t)seg * n2 + idx] = t;
    }
}

// Reciprocal and inverse square root refined from the hardware estimates by two
// Newton steps (quadratic convergence from the estimate's ~2^-22 to full FP64).
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rsq_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

// ---------------------------------------------------------------- Cholesky + inverse
// L (packed lower, LDS) with pivots below rel_tol * max(diag) dropped (column
// zeroed); Rinv = L^{-T} written column-major.  For n <= kInvLds the inverse is
// built row by row in LDS (row i of L^{-1} from rows < i, all columns in
// parallel); larger n solve one column per thread against global memory.
__device__ __forceinline__ int pidx_lower(int i, int j) { return i * (i + 1) / 2 + j; }
constexpr int kInvLds = 128;
constexpr int kPackedInv = kInvLds * (kInvLds + 1) / 2;

// One barrier per column: every thread reads the pivot d_j itself, and the trailing
// update uses the column before scaling, L[r][c] -= L[r][j] L[c][j] / d_j; the
// columns are scaled by 1 / sqrt(d_j) once the factorization is done.  A pivot
// at or below the threshold leaves its column out (zero).
__device__ __forceinline__ void chol_packed_lds(double *L, double *piv, int n, double thresh) {
    const int tid = threadIdx.x, ty = tid >> 5, tx = tid & 31;
    for (int j = 0; j < n; ++j) {
        const double d = L[pidx_lower(j, j)];
        const bool keep = d > thresh && d > 0.0;
        if (keep) {
            const double rd = 1.0 / d;
            for (int r = j + 1 + ty; r < n; r += 32) {
                const double lrj = L[pidx_lower(r, j)] * rd;
                if (lrj == 0.0) continue;
                for (int c = j + 1 + tx; c <= r; c += 32) L[pidx_lower(r, c)] -= lrj * L[pidx_lower(c, j)];
            }
        }
        if (tid == 0) piv[j] = keep ? sqrt(d) : 0.0;
        __syncthreads();
    }
    // scale: L[r][j] /= piv_j below the diagonal, L[j][j] = piv_j
    for (int r = ty; r < n; r += 32)
        for (int c = tx; c <= r; c += 32) {
            const double pj = piv[c];
            L[pidx_lower(r, c)] = r == c ? pj : (pj > 0.0 ? L[pidx_lower(r, c)] / pj : 0.0);
        }
    __syncthreads();
}

// Cholesky factor and inverse, with the matrix in registers: thread t owns the
// lower elements t, t + 1024, ... in column-major order (n <= NMAX).  Right-looking Cholesky, one
// barrier per column:
// in step j every thread updates its trailing elements from column j (unscaled,
// L[r][c] -= L[r][j] L[c][j] / d_j), read from a column buffer that the owners of
// column j wrote at the end of step j - 1, and the owners of column j + 1 write
// theirs into the other buffer.  The inverse of L runs the same way on [L | I] by
// rows: in step j the rows below take row j (final after step j - 1) times
// L[i][j] / L[j][j] off, and the owners of row j + 1 publish it.
template <int NMAX, int NT>
__global__ __launch_bounds__(NT) void cholinv_reg_kernel(const double *__restrict__ G, int n, double rel_tol,
                                                         double *__restrict__ Rinv, int *flags) {
    constexpr int kRegEl = (NMAX * (NMAX + 1) / 2 + NT - 1) / NT;
    __shared__ double Lu[NMAX * (NMAX + 1) / 2];       // final L, then its columns divided by the diagonal
    __shared__ double buf[2][NMAX];
    __shared__ double piv[NMAX];
    __shared__ double s_max;
    const int tid = threadIdx.x, npk = n * (n + 1) / 2;
    int rc[kRegEl];                                   // row | column << 16, -1: none
    double v[kRegEl];
#pragma unroll
    for (int u = 0; u < kRegEl; ++u) {
        const int e = tid + NT * u;
        rc[u] = -1;
        v[u] = 0.0;
        if (e < npk) {
            // column-major over the lower triangle (column c holds rows c..n-1), so that the
            // elements still active in a step sit in whole waves
            int c = 0, off = 0;
            while (off + (n - c) <= e) {
                off += n - c;
                ++c;
            }
            const int r = c + (e - off);
            rc[u] = r | (c << 16);
            v[u] = G[(int64_t)r * n + c];
            if (c == 0) buf[0][r] = v[u];
        }
    }
    if (tid < 64) {
        double m = 0.0;
        for (int i = tid; i < n; i += 64) m = fmax(m, G[(int64_t)i * n + i]);
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
        if (tid == 0) s_max = m;
    }
    __syncthreads();
    const double thresh = rel_tol * s_max;
    for (int j = 0; j < n; ++j) {
        const double *col = buf[j & 1];
        double *nxt = buf[(j + 1) & 1];
        const double d = col[j];
        const bool keep = d > thresh && d > 0.0;
        const double rd = keep ? rcp_nr(d) : 0.0;
#pragma unroll
        for (int u = 0; u < kRegEl; ++u) {
            const int r = rc[u] < 0 ? -1 : (rc[u] & 0xffff), c = rc[u] < 0 ? 0 : (rc[u] >> 16);
            if (c > j) {
                if (keep) v[u] -= col[r] * col[c] * rd;
                if (c == j + 1) nxt[r] = v[u];
            }
        }
        if (tid == 0) piv[j] = keep ? sqrt(d) : 0.0;
        __syncthreads();
    }
    // scaled factor into LDS: L[r][c] = v / piv_c below the diagonal, piv_c on it
#pragma unroll
    for (int u = 0; u < kRegEl; ++u) {
        const int r = rc[u] < 0 ? -1 : (rc[u] & 0xffff), c = rc[u] < 0 ? 0 : (rc[u] >> 16);
        if (r < 0) continue;
        const double pc = piv[c];
        Lu[r * (r + 1) / 2 + c] = r == c ? pc : (pc > 0.0 ? v[u] / pc : 0.0);
    }
    if (tid == 0) {
        bool any = false;
        for (int j = 0; j < n; ++j) any |= piv[j] > 0.0;
        if (!any) atomicOr(&flags[kFlagNumeric], 1);
    }
    __syncthreads();
    // L[i][j] / L[j][j] below the diagonal (0 for a dropped column)
#pragma unroll
    for (int u = 0; u < kRegEl; ++u) {
        const int r = rc[u] < 0 ? -1 : (rc[u] & 0xffff), c = rc[u] < 0 ? 0 : (rc[u] >> 16);
        if (r < 0 || r == c) continue;
        const double pc = piv[c];
        Lu[r * (r + 1) / 2 + c] = pc > 0.0 ? Lu[r * (r + 1) / 2 + c] / pc : 0.0;
    }
    // [L | I] by rows: v now holds L^{-1} (rows unscaled), starting from I
#pragma unroll
    for (int u = 0; u < kRegEl; ++u) {
        const int r = rc[u] < 0 ? -1 : (rc[u] & 0xffff), c = rc[u] < 0 ? 0 : (rc[u] >> 16);
        v[u] = r >= 0 && r == c ? 1.0 : 0.0;
        if (r == 0) buf[0][0] = 1.0;
    }
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        const double *row = buf[j & 1];
        double *nxt = buf[(j + 1) & 1];
#pragma unroll
        for (int u = 0; u < kRegEl; ++u) {
            const int i = rc[u] < 0 ? -1 : (rc[u] & 0xffff), c = rc[u] < 0 ? 0 : (rc[u] >> 16);
            if (i > j) {
                if (c <= j) v[u] -= Lu[i * (i + 1) / 2 + j] * row[c];
                if (i == j + 1) nxt[c] = v[u];
            }
        }
        __syncthreads();
    }
    // Rinv (column-major) = Linv^T, rows of Linv scaled by 1 / L[i][i]
#pragma unroll
    for (int u = 0; u < kRegEl; ++u) {
        const int i = rc[u] < 0 ? -1 : (rc[u] & 0xffff), c = rc[u] < 0 ? 0 : (rc[u] >> 16);
        if (i < 0) continue;
        const double lii = piv[i];
        Rinv[(int64_t)i * n + c] = lii != 0.0 ? v[u] / lii : 0.0;
    }
    for (int e = tid; e < n * n; e += NT) {
        const int i = e / n, c = e % n;
        if (c > i) Rinv[e] = 0.0;
    }
}

// Batched Cholesky factor: one block per matrix G[bch] (n x n, symmetric PSD),
// L[bch] row-major lower triangular (upper part zero), pivots below
// rel_tol * max(diag) dropped (their column of L is zero).
__global__ __launch_bounds__(1024) void chol_batched_kernel(const double *__restrict__ Gb, int n, double rel_tol,
                                                            double *__restrict__ Lb) {
    __shared__ double L[kPacked];
    __shared__ double piv[kMaxSmall];
    __shared__ double s_max;
    const double *G = Gb + (int64_t)blockIdx.x * n * n;
    double *Lo = Lb + (int64_t)blockIdx.x * n * n;
    const int tid = threadIdx.x, ty = tid >> 5, tx = tid & 31;
    for (int i = ty; i < n; i += 32)
        for (int j = tx; j <= i; j += 32) L[pidx_lower(i, j)] = 0.5 * (G[(int64_t)i * n + j] + G[(int64_t)j * n + i]);
    if (tid == 0) {
        double m = 0.0;
        for (int i = 0; i < n; ++i) m = fmax(m, G[(int64_t)i * n + i]);
        s_max = m;
    }
    __syncthreads();
    chol_packed_lds(L, piv, n, rel_tol * s_max);
    for (int i = ty; i < n; i += 32)
        for (int j = tx; j < n; j += 32) Lo[(int64_t)i * n + j] = j <= i ? L[pidx_lower(i, j)] : 0.0;
}

// C = A B for small column-major n x n matrices (one block).
__global__ __launch_bounds__(256) void small_matmul_kernel(const double *__restrict__ A, const double *__restrict__ B,
                                                           int n, double *__restrict__ C) {
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int col = idx / n, row = idx % n;
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += A[(int64_t)k * n + row] * B[(int64_t)col * n + k];
        C[idx] = s;
    }
}

// ---------------------------------------------------------------- tall x small product
// out = A T (rows x m) with A column-major (rows x n, fp32 or fp64) and T column-major
// n x m, in FP64.  Grid: (row blocks of 256 * kTsRows, column groups of kTsCols).
// A thread owns kTsRows rows (strided by 256, so every load and store of a column
// is contiguous across the wave) and the group's kTsCols columns; the block stages
// those columns of T in LDS (row-major, read as broadcasts).  The next inner term's
// operands are loaded while the current one is multiplied.
constexpr int kTsRows = 2;
constexpr int kTsCols = 16;
constexpr int kTsAhead = 8;

template <typename TA>
__global__ __launch_bounds__(256) void tsmul_kernel(const TA *__restrict__ A, int64_t rows, int64_t lda, int n,
                                                    const double *__restrict__ T, int m,
                                                    const double *__restrict__ colscale, float *out32,
                                                    int64_t ld32, double *out64, int64_t ld64, unsigned short *hi,
                                                    unsigned short *lo, uint8_t *f8, int64_t ldh, int Lpad,
                                                    int64_t rows_pad) {
    __shared__ double Ts[kMaxSmall * kTsCols];        // T[k0 + i][j0 + jj] at i * kTsCols + jj
    const int j0 = blockIdx.y * kTsCols;
    const int64_t base = (int64_t)blockIdx.x * (256 * kTsRows) + threadIdx.x;
    int64_t rr[kTsRows];
    bool live[kTsRows];
#pragma unroll
    for (int q = 0; q < kTsRows; ++q) {
        const int64_t row = base + 256 * q;
        live[q] = row < rows;
        rr[q] = live[q] ? row : 0;
    }
    double acc[kTsRows][kTsCols];
#pragma unroll
    for (int q = 0; q < kTsRows; ++q)
#pragma unroll
        for (int jj = 0; jj < kTsCols; ++jj) acc[q][jj] = 0.0;
    // the inner dimension in chunks of at most kMaxSmall rows of T (one LDS fill each)
    for (int k0 = 0; j0 < m && k0 < n; k0 += kMaxSmall) {
        const int kc = n - k0 < kMaxSmall ? n - k0 : kMaxSmall;
        __syncthreads();
        for (int idx = threadIdx.x; idx < kc * kTsCols; idx += 256) {
            const int i = idx / kTsCols, jj = idx % kTsCols;
            Ts[idx] = j0 + jj < m ? T[(int64_t)(j0 + jj) * n + k0 + i] : 0.0;
        }
        __syncthreads();
        const TA *Ak = A + (int64_t)k0 * lda;
        // A is read kTsAhead columns ahead of its use (the loads of the next group are
        // in flight while the current one is multiplied)
        TA an[kTsAhead][kTsRows];
#pragma unroll
        for (int u = 0; u < kTsAhead; ++u)
#pragma unroll
            for (int q = 0; q < kTsRows; ++q) an[u][q] = u < kc ? Ak[(int64_t)u * lda + rr[q]] : (TA)0;
        for (int i0 = 0; i0 < kc; i0 += kTsAhead) {
            TA a[kTsAhead][kTsRows];
#pragma unroll
            for (int u = 0; u < kTsAhead; ++u)
#pragma unroll
                for (int q = 0; q < kTsRows; ++q) a[u][q] = an[u][q];
#pragma unroll
            for (int u = 0; u < kTsAhead; ++u) {
                const int i = i0 + kTsAhead + u;
#pragma unroll
                for (int q = 0; q < kTsRows; ++q) an[u][q] = i < kc ? Ak[(int64_t)i * lda + rr[q]] : (TA)0;
            }
#pragma unroll
            for (int u = 0; u < kTsAhead; ++u) {
                const int i = i0 + u;
                if (i >= kc) break;
#pragma unroll
                for (int jj = 0; jj < kTsCols; jj += 2) {
                    const double2 t = *reinterpret_cast<const double2 *>(&Ts[i * kTsCols + jj]);
#pragma unroll
                    for (int q = 0; q < kTsRows; ++q) {
                        acc[q][jj] = fma((double)a[u][q], t.x, acc[q][jj]);
                        acc[q][jj + 1] = fma((double)a[u][q], t.y, acc[q][jj + 1]);
                    }
                }
            }
        }
    }
    if (j0 < m) {
#pragma unroll
        for (int q = 0; q < kTsRows; ++q) {
            if (!live[q]) continue;
            const int64_t row = rr[q];
#pragma unroll
            for (int jj = 0; jj < kTsCols; ++jj) {
                const int j = j0 + jj;
                if (j < m) {
                    double v = acc[q][jj];
                    if (colscale) v *= colscale[j];
                    if (out32) out32[(int64_t)j * ld32 + row] = (float)v;
                    if (out64) out64[(int64_t)j * ld64 + row] = v;
                    if (hi) {
                        const unsigned short h = f32_to_bf16_bits((float)v);
                        hi[(int64_t)j * ldh + row] = h;
                        if (lo) lo[(int64_t)j * ldh + row] = f32_to_bf16_bits((float)(v - (double)bf16_bits_to_f32(h)));
                    }
                    if (f8)
                        f8[(int64_t)j * ldh + row] =
                            (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32((float)v * 256.f, 0.f, 0, false) & 0xff);
                }
            }
        }
    }
    // zero padding of the bf16 rows (column group 0 only): columns [m, Lpad) of live
    // rows, all columns of pad rows
    if ((hi || f8) && blockIdx.y == 0) {
#pragma unroll
        for (int q = 0; q < kTsRows; ++q) {
            const int64_t row = base + 256 * q;
            if (row >= rows_pad) continue;
            for (int j = row < rows ? m : 0; j < Lpad; ++j) {
                if (hi) hi[(int64_t)j * ldh + row] = 0;
                if (lo) lo[(int64_t)j * ldh + row] = 0;
                if (f8) f8[(int64_t)j * ldh + row] = 0;
            }
        }
    }
}

// ---------------------------------------------------------------- tall x small product on the FP64 MFMA
// out = A T computed as out^T = T^T A^T with v_mfma_f64_16x16x4: the MFMA's rows are
// 16 output columns (T^T, from LDS), its columns 16 rows of A.  A wave owns strips
// of 16 SUB rows: lane l reads rows SUB (l % 16) .. SUB (l % 16) + SUB - 1 of inner
// index k + l / 16 in one load, so the SUB components feed SUB MFMA column sets (rows
// SUB i + s) that share every T fragment, and the results leave as stores of SUB
// consecutive rows of one output column.  The loads of the next AH 4-deep inner
// groups are in flight while a group is multiplied.  A block stages up to kTsmK
// rows of T for one group of kTsmCols output columns (blockIdx.y), in MFMA fragment
// order, and its waves walk the strips.  For an upper triangular T (the inverse
// Cholesky factors) the 4 x 16 blocks below the diagonal are zero: their products
// and the rows of A that only meet them are skipped.  The products are FP64
// throughout (A entries are exact in FP64).
constexpr int kTsmCols = 80;
constexpr int kTsmTiles = kTsmCols / 16;
constexpr int kTsmK = 96;
enum : int { kTsmVecA = 1, kTsmVec32 = 2, kTsmVec64 = 4, kTsmVecH = 8, kTsmVecF8 = 16 };

// SUB consecutive elements at p (vector access when vec; the caller guarantees the
// alignment of SUB elements)
template <typename U, int SUB>
__device__ __forceinline__ void tsm_ld(const U *p, U (&x)[SUB]) {
    if constexpr (sizeof(U) * SUB <= 16) {
        using V = U __attribute__((ext_vector_type(SUB)));
        const V q = *reinterpret_cast<const V *>(p);
#pragma unroll
        for (int s = 0; s < SUB; ++s) x[s] = q[s];
    } else {
        using V = U __attribute__((ext_vector_type(SUB / 2)));
        const V q0 = reinterpret_cast<const V *>(p)[0], q1 = reinterpret_cast<const V *>(p)[1];
#pragma unroll
        for (int s = 0; s < SUB / 2; ++s) {
            x[s] = q0[s];
            x[s + SUB / 2] = q1[s];
        }
    }
}
template <typename U, int SUB>
__device__ __forceinline__ void tsm_st(U *p, const U (&x)[SUB], bool vec, int nvalid) {
    if (vec && nvalid >= SUB) {
        if constexpr (sizeof(U) * SUB <= 16) {
            using V = U __attribute__((ext_vector_type(SUB)));
            V q;
#pragma unroll
            for (int s = 0; s < SUB; ++s) q[s] = x[s];
            *reinterpret_cast<V *>(p) = q;
        } else {
            using V = U __attribute__((ext_vector_type(SUB / 2)));
            V q0, q1;
#pragma unroll
            for (int s = 0; s < SUB / 2; ++s) {
                q0[s] = x[s];
                q1[s] = x[s + SUB / 2];
            }
            reinterpret_cast<V *>(p)[0] = q0;
            reinterpret_cast<V *>(p)[1] = q1;
        }
        return;
    }
#pragma unroll
    for (int s = 0; s < SUB; ++s)
        if (s < nvalid) p[s] = x[s];
}

template <typename TA, bool NARROW, int SUB, int W, int WPE, int AH>
__global__ __launch_bounds__(64 * W, WPE) void tsmul_mfma_kernel(
    const TA *__restrict__ A, int64_t rows, int64_t lda, int n, const double *__restrict__ T, int m, int upper,
    const double *__restrict__ colscale, float *out32, int64_t ld32, double *out64, int64_t ld64,
    unsigned short *hi, unsigned short *lo, uint8_t *f8, int64_t ldh, int Lpad, int64_t rows_pad, int64_t span,
    int vflags) {
    constexpr int RS = 16 * SUB;                      // rows per strip
    // T in MFMA fragment order: the operand of inner group g and column tile c for
    // lane l, T[k0 + 4 g + l / 16][j0 + 16 c + l % 16], at (g * kTsmTiles + c) * 64 + l
    __shared__ double Ts[kTsmK * kTsmCols];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int j0 = blockIdx.y * kTsmCols;
    const int ncg = m - j0 < kTsmCols ? m - j0 : kTsmCols;
    const int nct = (ncg + 15) / 16;
    // inner indices that meet this group: all of them, or (upper) those up to its last column
    const int kend = upper && j0 + ncg < n ? j0 + ncg : n;
    const int nchunks = (kend + kTsmK - 1) / kTsmK;
    const int64_t nstrips = (span + RS - 1) / RS;
    const bool vec_a = vflags & kTsmVecA;
    for (int64_t sb = (int64_t)blockIdx.x * W; sb < nstrips; sb += (int64_t)gridDim.x * W) {
        const int64_t r0 = (sb + wv) * RS;
        const bool live = sb + wv < nstrips;
        const int64_t row = r0 + SUB * li;           // this lane's first row
        const bool full = vec_a && r0 + RS <= rows;
        f64x4 acc[kTsmTiles][SUB];
#pragma unroll
        for (int c = 0; c < kTsmTiles; ++c)
#pragma unroll
            for (int s = 0; s < SUB; ++s) acc[c][s] = (f64x4){0.0, 0.0, 0.0, 0.0};
        for (int ch = 0; ch < nchunks; ++ch) {
            const int k0 = ch * kTsmK;
            const int kc = kend - k0 < kTsmK ? kend - k0 : kTsmK;
            if (nchunks > 1 || sb == (int64_t)blockIdx.x * W) {
                __syncthreads();
                for (int idx = threadIdx.x; idx < kTsmK * kTsmCols; idx += 64 * W) {
                    const int l = idx & 63, gc = idx >> 6;
                    const int i = 4 * (gc / kTsmTiles) + (l >> 4), jj = 16 * (gc % kTsmTiles) + (l & 15);
                    Ts[idx] = i < kc && jj < ncg ? T[(int64_t)(j0 + jj) * n + k0 + i] : 0.0;
                }
                __syncthreads();
            }
            if (!live || rows <= 0) continue;         // (rows <= 0: only padding rows, nothing to read)
            const int ng = (kc + 3) / 4;
            // the loads are unconditional (indices clamped into the matrix) and the
            // values outside it are replaced by zeros when used, so no branch splits
            // the loads in flight
            int64_t rc[SUB];
            bool ok[SUB];
#pragma unroll
            for (int s = 0; s < SUB; ++s) {
                ok[s] = row + s < rows;
                rc[s] = ok[s] ? row + s : rows - 1;
            }
            const TA *Ak = A + (int64_t)k0 * lda;
            auto kloop = [&](auto full_c) {
                constexpr bool F = decltype(full_c)::value;
                auto fetch = [&](int g, TA (&x)[SUB]) {
                    const int kk = 4 * g + lk < kc ? 4 * g + lk : kc - 1;
                    const TA *p = Ak + (int64_t)kk * lda;
                    if constexpr (F) {
                        tsm_ld<TA, SUB>(p + row, x);
                    } else {
#pragma unroll
                        for (int s = 0; s < SUB; ++s) x[s] = p[rc[s]];
                    }
                };
                // the chunk's inner groups fully unrolled (static ring slots, so each
                // group waits for its own loads only)
                constexpr int kG = kTsmK / 4;
                TA ring[AH][SUB];
#pragma unroll
                for (int u = 0; u < AH; ++u) fetch(u, ring[u]);
#pragma unroll
                for (int g = 0; g < kG; ++g) {
                    if (g >= ng) break;
                    const int u = g % AH;
                    const bool kv = 4 * g + lk < kc;
                    double a[SUB];
#pragma unroll
                    for (int s = 0; s < SUB; ++s) a[s] = kv && (F || ok[s]) ? (double)ring[u][s] : 0.0;
                    if (g + AH < kG) fetch(g + AH, ring[u]);
                    const int kg = k0 + 4 * g;
                    const int cmin = upper && kg > j0 ? (kg - j0) / 16 : 0;
                    const double *tf = Ts + g * (kTsmTiles * 64) + lane;
                    double t[kTsmTiles];
#pragma unroll
                    for (int c = 0; c < kTsmTiles; ++c) t[c] = tf[64 * c];
#pragma unroll
                    for (int c = 0; c < kTsmTiles; ++c) {
                        if (c < cmin || c >= nct) continue;
#pragma unroll
                        for (int s = 0; s < SUB; ++s)
                            acc[c][s] = __builtin_amdgcn_mfma_f64_16x16x4f64(t[c], a[s], acc[c][s], 0, 0, 0);
                    }
                }
            };
            if (full) kloop(std::true_type{});
            else kloop(std::false_type{});
        }
        if (!live) continue;
        // acc[c][s][v]: column j0 + 16 c + lk + 4 v, row r0 + SUB li + s.  The column
        // offsets are recomputed per strip (kept out of registers across the loop).
        int64_t l32 = ld32, l64 = ld64, lh = ldh;
        const double *cs = colscale;
        int lkx = lk;
        asm volatile("" : "+s"(l32), "+s"(l64), "+s"(lh), "+s"(cs), "+v"(lkx));
        const int nv = rows - row < SUB ? (int)(rows - row) : SUB;          // valid rows of this lane
        const int nvp = rows_pad - row < SUB ? (int)(rows_pad - row) : SUB; // valid padded rows
#pragma unroll
        for (int c = 0; c < kTsmTiles; ++c) {
            if (c >= nct) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int jl = 16 * c + lkx + 4 * v;
                if (jl >= ncg) continue;
                const int j = j0 + jl;
                const double sc = cs ? cs[j] : 1.0;
                double x[SUB];
#pragma unroll
                for (int s = 0; s < SUB; ++s) x[s] = acc[c][s][v] * sc;
                if (out32 && nv > 0) {
                    float y[SUB];
#pragma unroll
                    for (int s = 0; s < SUB; ++s) y[s] = (float)x[s];
                    tsm_st<float, SUB>(out32 + (int64_t)j * l32 + row, y, vflags & kTsmVec32, nv);
                }
                if (out64 && nv > 0) tsm_st<double, SUB>(out64 + (int64_t)j * l64 + row, x, vflags & kTsmVec64, nv);
                if (NARROW && nvp > 0) {
                    const int64_t off = (int64_t)j * lh + row;
                    if (hi) {
                        unsigned short h[SUB], l[SUB];
#pragma unroll
                        for (int s = 0; s < SUB; ++s) {
                            h[s] = f32_to_bf16_bits((float)x[s]);
                            l[s] = f32_to_bf16_bits((float)(x[s] - (double)bf16_bits_to_f32(h[s])));
                        }
                        tsm_st<unsigned short, SUB>(hi + off, h, vflags & kTsmVecH, nvp);
                        if (lo) tsm_st<unsigned short, SUB>(lo + off, l, vflags & kTsmVecH, nvp);
                    }
                    if (f8) {
                        uint8_t e[SUB];
#pragma unroll
                        for (int s = 0; s < SUB; s += 2) {
                            const uint32_t q =
                                __builtin_amdgcn_cvt_pk_fp8_f32((float)x[s] * 256.f, (float)x[s + 1] * 256.f, 0, false);
                            e[s] = (uint8_t)(q & 0xff);
                            e[s + 1] = (uint8_t)((q >> 8) & 0xff);
                        }
                        tsm_st<uint8_t, SUB>(f8 + off, e, vflags & kTsmVecF8, nvp);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // zero columns [m, Lpad) of the padded bf16 / e4m3 rows (last column group)
        if (NARROW && blockIdx.y == gridDim.y - 1 && nvp > 0) {
            for (int j = m + lkx; j < Lpad; j += 4) {
                const int64_t off = (int64_t)j * lh + row;
#pragma unroll
                for (int s = 0; s < SUB; ++s)
                    if (s < nvp) {
                        if (hi) hi[off + s] = 0;
                        if (lo) lo[off + s] = 0;
                        if (f8) f8[off + s] = 0;
                    }
            }
        }
    }
}

// launch shapes (measured at 262,144 x 80 fp32 rows): rows per strip 16 SUB, waves
// per block W, waves per SIMD WPE, inner groups loaded ahead AH, blocks per CU BPC
template <typename TA>
struct TsmShape {
    static constexpr int SUB = 4, W = 8, WPE = 2, AH = 2, BPC = 1;
};
template <>
struct TsmShape<double> {       // the FP64 rows (the frame side): fewer rows, more strips
    static constexpr int SUB = 2, W = 4, WPE = 2, AH = 4, BPC = 2;
};

// ---------------------------------------------------------------- Jacobi eigensolver
// Parallel-order (round-robin) cyclic Jacobi on a symmetric n x n matrix, n even.
// In step s the n/2 disjoint pairs are (0, x(0)) and (x(a), x(m-a)), a = 1..n/2-1,
// with m = n-1 and x(i) = 1 + (i + s) mod m; every pair occurs once per sweep.
// The eigensolvers below keep B in slot order; for n > 128 they log each step's
// rotations in the roles (p, q) = (smaller, larger index) of the pair, and the
// eigenvectors P = J_1 J_2 ... are formed afterwards from that log, one row per wave.
__device__ __forceinline__ void rr_pair(int s, int a, int n, int &p, int &q) {
    const int m = n - 1;
    int u, v;
    if (a == 0) {
        u = 0;
        v = 1 + (s % m);
    } else {
        u = 1 + ((a + s) % m);
        v = 1 + ((m - a + s) % m);
    }
    p = u < v ? u : v;
    q = u < v ? v : u;
}

constexpr int kMaxSweeps = 30;

// Eigenvectors from the rotation log: row i of P = e_i^T J_1 J_2 ... J_S.  Rows are
// independent, so each wave forms one row in its own piece of LDS, lane a applying
// pair a's rotation of every step in order (a wave's LDS accesses complete in
// program order, so no barrier is needed between steps); the next step's
// rotations are loaded while the current one is applied.
constexpr int kReplayWaves = 4;
__global__ __launch_bounds__(64 * kReplayWaves) void jacobi_replay_kernel(const double2 *__restrict__ rot_log,
                                                                          const int *__restrict__ nsteps_ptr, int n,
                                                                          double *__restrict__ P) {
    __shared__ double rowv[kReplayWaves][kMaxSmall];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * kReplayWaves + w;
    const int h = n / 2, m = n - 1;
    if (row >= n) return;
    double *rv = rowv[w];
    for (int j = lane; j < n; j += 64) rv[j] = (j == row) ? 1.0 : 0.0;
    const int nsteps = *nsteps_ptr;
    // lane a handles pairs a and a + 64 (h <= 96)
    double2 c0 = make_double2(1.0, 0.0), c1 = make_double2(1.0, 0.0);
    if (nsteps > 0) {
        if (lane < h) c0 = rot_log[lane];
        if (lane + 64 < h) c1 = rot_log[lane + 64];
    }
    for (int st = 0; st < nsteps; ++st) {
        const double2 r0 = c0, r1 = c1;
        if (st + 1 < nsteps) {
            if (lane < h) c0 = rot_log[(int64_t)(st + 1) * h + lane];
            if (lane + 64 < h) c1 = rot_log[(int64_t)(st + 1) * h + lane + 64];
        }
        const int s = st % m;
        int p, q;
        double x0 = 0.0, y0 = 0.0, x1 = 0.0, y1 = 0.0;
        int p1 = 0, q1 = 0;
        if (lane < h) {
            rr_pair(s, lane, n, p, q);
            x0 = rv[p];
            y0 = rv[q];
        }
        if (lane + 64 < h) {
            rr_pair(s, lane + 64, n, p1, q1);
            x1 = rv[p1];
            y1 = rv[q1];
        }
        if (lane < h) {
            rv[p] = r0.x * x0 - r0.y * y0;
            rv[q] = r0.y * x0 + r0.x * y0;
        }
        if (lane + 64 < h) {
            rv[p1] = r1.x * x1 - r1.y * y1;
            rv[q1] = r1.y * x1 + r1.x * y1;
        }
    }
    for (int j = lane; j < n; j += 64) P[(int64_t)row * n + j] = rv[j];
}

// ---------------------------------------------------------------- Jacobi on slots (n <= 128)
// The same round-robin order, with B physically permuted after every step so
// that the pairs are always slots (2a, 2a+1).  Circle position c (0 <= c < m)
// holds index 1 + (c + s) mod m at step s; slot 0 holds index 0, slot 1 circle
// 0, slot 2a circle a and slot 2a+1 circle m-a (a >= 1).  Between steps every
// circle position moves down by one, a fixed slot permutation pi, so each
// thread reads and writes the same LDS words in every step.
//
// B is kept as 2x2 blocks of slot pairs (a <= b) in four planes (plane 2r+t
// holds element (2a+r, 2b+t) of block b(b+1)/2 + a), double-buffered: a step
// reads one buffer and writes the rotated, permuted blocks into the other.
// Wave 0 computes the next step's rotations while the other waves update B: the
// next diagonal block of pair a comes from three blocks of the current step
// (those of the two slots that move into 2a and 2a+1), so the only barrier of a
// step is the one that ends it.  Rotations are logged in slot roles.
constexpr int kSlotMaxH = 64;
constexpr int kSlotMaxBlk = kSlotMaxH * (kSlotMaxH + 1) / 2;
constexpr int kSlotThreads = 1024;

__device__ __forceinline__ int slot_circ(int j, int m) { return j == 1 ? 0 : ((j & 1) ? m - (j >> 1) : (j >> 1)); }
__device__ __forceinline__ int circ_slot(int c, int h, int m) { return c == 0 ? 1 : (c < h ? 2 * c : 2 * (m - c) + 1); }
__device__ __forceinline__ int next_slot(int j, int h, int m) {
    if (j == 0) return 0;
    const int c = slot_circ(j, m);
    return circ_slot(c == 0 ? m - 1 : c - 1, h, m);
}
__device__ __forceinline__ int prev_slot(int j, int h, int m) {
    if (j == 0) return 0;
    const int c = slot_circ(j, m) + 1;
    return circ_slot(c == m ? 0 : c, h, m);
}
__device__ __forceinline__ int slot_index_at0(int j, int m) { return j == 0 ? 0 : 1 + slot_circ(j, m); }
// LDS word of element (i, j) of the slot matrix, either order
__device__ __forceinline__ int slot_elem(int i, int j) {
    int pa = i >> 1, pb = j >> 1, r = i & 1, t = j & 1;
    if (pa > pb) {
        int x = pa;
        pa = pb;
        pb = x;
        x = r;
        r = t;
        t = x;
    }
    if (pa == pb && r > t) {
        r = 0;
        t = 1;
    }
    return (r * 2 + t) * kSlotMaxBlk + pb * (pb + 1) / 2 + pa;
}
__device__ __forceinline__ void slot_blk_ab(int idx, int &a, int &b) {
    int j = (int)((sqrtf(8.0f * (float)idx + 1.0f) - 1.0f) * 0.5f);
    while (j * (j + 1) / 2 > idx) --j;
    while ((j + 1) * (j + 2) / 2 <= idx) ++j;
    b = j;
    a = idx - j * (j + 1) / 2;
}
__device__ __forceinline__ int slot_blk(int a, int b) { return a <= b ? b * (b + 1) / 2 + a : a * (a + 1) / 2 + b; }

// Rotation of the pair (x, y) with entries (app, apq, aqq): t = tan of the smaller
// angle, t = sign(d) 2 apq / (|d| + sqrt(d^2 + 4 apq^2)), d = aqq - app, from the
// hardware estimates (the angle need not be exact: the rotated off-diagonal
// entry is computed, not assumed zero); c = 1 / sqrt(1 + t^2) to full precision,
// so the rotation is orthogonal to rounding.
__device__ __forceinline__ double2 slot_rotation(double app, double apq, double aqq) {
    double c = 1.0, sn = 0.0;
    if (fabs(apq) > 1e-300 && apq * apq > 1e-30 * fabs(app) * fabs(aqq)) {
        const double d = aqq - app, a2 = 2.0 * apq;
        const double r2 = fma(d, d, a2 * a2);
        const double hyp = r2 * __builtin_amdgcn_rsq(r2);
        const double t = (d >= 0.0 ? a2 : -a2) * __builtin_amdgcn_rcp(fabs(d) + hyp);
        c = rsq_nr(fma(t, t, 1.0));
        sn = t * c;
    }
    return make_double2(c, sn);
}
// column r of the rotation [[c, s], [-s, c]]
__device__ __forceinline__ void rot_col(double2 q, int r, double &u0, double &u1) {
    u0 = r == 0 ? q.x : q.y;
    u1 = r == 0 ? -q.y : q.x;
}

__global__ __launch_bounds__(kSlotThreads) void jacobi_slots_kernel(const double *__restrict__ Bg, int n,
                                                                    double *__restrict__ lam,
                                                                    double2 *__restrict__ rot_log,
                                                                    int *__restrict__ nsteps_out, int *flags) {
    constexpr int kWork = kSlotThreads - 64;       // waves 1.. own the blocks
    constexpr int kIPT = (kSlotMaxBlk + kWork - 1) / kWork;
    constexpr int kW = kSlotThreads / 64;
    __shared__ __align__(16) double buf[2][4 * kSlotMaxBlk];
    __shared__ __align__(16) double2 rot[2][kSlotMaxH];
    __shared__ double red_off[kW], red_dg[kW];
    __shared__ int s_done;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int h = n / 2, m = n - 1, nblk = h * (h + 1) / 2;
    // blocks owned by this thread: pairs (a, b), destinations of their four elements
    int ia[kIPT], ib[kIPT], dst[kIPT][4];
#pragma unroll
    for (int u = 0; u < kIPT; ++u) {
        const int idx = tid - 64 + kWork * u;
        ia[u] = -1;
        ib[u] = 0;
        dst[u][0] = dst[u][1] = dst[u][2] = dst[u][3] = 0;
        if (wv > 0 && idx < nblk) {
            int a, b;
            slot_blk_ab(idx, a, b);
            ia[u] = a;
            ib[u] = b;
            const int p0 = next_slot(2 * a, h, m), p1 = next_slot(2 * a + 1, h, m);
            const int q0 = next_slot(2 * b, h, m), q1 = next_slot(2 * b + 1, h, m);
            dst[u][0] = slot_elem(p0, q0);
            dst[u][1] = slot_elem(p0, q1);
            dst[u][2] = slot_elem(p1, q0);
            dst[u][3] = slot_elem(p1, q1);
        }
    }
    // wave 0, lane a: the slots that move into 2a and 2a+1, their pairs and blocks
    const int la = lane < h ? lane : 0;
    const int s0 = prev_slot(2 * la, h, m), s1 = prev_slot(2 * la + 1, h, m);
    const int P0 = s0 >> 1, P1 = s1 >> 1, r0 = s0 & 1, r1 = s1 & 1;
    const int d0 = P0 * (P0 + 3) / 2, d1 = P1 * (P1 + 3) / 2, xb = slot_blk(P0, P1);
    for (int e = tid; e < nblk * 4; e += kSlotThreads) {
        const int blk = e >> 2, pos = e & 3;
        int a, b;
        slot_blk_ab(blk, a, b);
        const int gi = slot_index_at0(2 * a + (pos >> 1), m), gj = slot_index_at0(2 * b + (pos & 1), m);
        buf[0][pos * kSlotMaxBlk + blk] = 0.5 * (Bg[(int64_t)gi * n + gj] + Bg[(int64_t)gj * n + gi]);
    }
    __syncthreads();
    if (wv == 0 && lane < h) {
        const int dblk = lane * (lane + 3) / 2;
        const double2 r = slot_rotation(buf[0][dblk], buf[0][kSlotMaxBlk + dblk], buf[0][3 * kSlotMaxBlk + dblk]);
        rot[0][lane] = r;
        rot_log[lane] = r;
    }
    // circle offsets of the indices in slots 2a (a >= 1) and 2a+1 of pair `lane`
    int xa = lane % m, ya = (m - lane) % m;
    int cur = 0, nsteps = 0;
    bool converged = false;
    for (int sweep = 0; sweep <= kMaxSweeps; ++sweep) {
        double off = 0.0, dg = 0.0;
        for (int e = tid; e < nblk; e += kSlotThreads) {
            int a, b;
            slot_blk_ab(e, a, b);
            const double *q = buf[cur] + e;
            const double x = q[0], y = q[kSlotMaxBlk], z = q[2 * kSlotMaxBlk], w = q[3 * kSlotMaxBlk];
            if (a == b) {
                off += y * y;
                dg += x * x + w * w;
            } else {
                off += x * x + y * y + z * z + w * w;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_xor(off, o);
            dg += __shfl_xor(dg, o);
        }
        if (lane == 0) {
            red_off[wv] = off;
            red_dg[wv] = dg;
        }
        __syncthreads();
        if (tid == 0) {
            double so = 0.0, sd = 0.0;
            for (int w = 0; w < kW; ++w) {
                so += red_off[w];
                sd += red_dg[w];
            }
            s_done = (so <= 1e-26 * sd) || so == 0.0;
        }
        __syncthreads();
        if (s_done) {
            converged = true;
            break;
        }
        if (sweep == kMaxSweeps) break;
        for (int s = 0; s < m; ++s) {
            const double *B = buf[cur];
            double *Bn = buf[cur ^ 1];
            const double2 *R = rot[nsteps & 1];
            if (wv == 0) {
                if (lane < h) {
                    // next step's diagonal block of pair `lane`, rotated out of this step's blocks
                    double u00, u01, u10, u11;
                    rot_col(R[P0], r0, u00, u01);
                    rot_col(R[P1], r1, u10, u11);
                    const double a0 = B[d0], b0 = B[kSlotMaxBlk + d0], c0 = B[3 * kSlotMaxBlk + d0];
                    const double a1 = B[d1], b1 = B[kSlotMaxBlk + d1], c1 = B[3 * kSlotMaxBlk + d1];
                    const double x = B[xb], y = B[kSlotMaxBlk + xb], z = B[2 * kSlotMaxBlk + xb],
                                 w = B[3 * kSlotMaxBlk + xb];
                    const double app = u00 * (u00 * a0 + u01 * b0) + u01 * (u00 * b0 + u01 * c0);
                    const double aqq = u10 * (u10 * a1 + u11 * b1) + u11 * (u10 * b1 + u11 * c1);
                    double apq;
                    if (P0 < P1)
                        apq = u00 * (x * u10 + y * u11) + u01 * (z * u10 + w * u11);
                    else if (P0 > P1)
                        apq = u10 * (x * u00 + y * u01) + u11 * (z * u00 + w * u01);
                    else   // n = 2: the same pair again
                        apq = u00 * (u10 * a0 + u11 * b0) + u01 * (u10 * b0 + u11 * c0);
                    const double2 r = slot_rotation(app, apq, aqq);
                    rot[(nsteps + 1) & 1][lane] = r;
                    rot_log[(int64_t)(nsteps + 1) * h + lane] = r;
                }
            } else {
#pragma unroll
                for (int u = 0; u < kIPT; ++u) {
                    if (ia[u] < 0) continue;
                    const int a = ia[u], b = ib[u];
                    const double *q = B + (b * (b + 1) / 2 + a);
                    const double x = q[0], y = q[kSlotMaxBlk], z = q[2 * kSlotMaxBlk], w = q[3 * kSlotMaxBlk];
                    const double2 ra = R[a], rb = R[b];
                    if (a != b) {
                        const double x1 = rb.x * x - rb.y * y, y1 = rb.y * x + rb.x * y;
                        const double z1 = rb.x * z - rb.y * w, w1 = rb.y * z + rb.x * w;
                        Bn[dst[u][0]] = ra.x * x1 - ra.y * z1;
                        Bn[dst[u][1]] = ra.x * y1 - ra.y * w1;
                        Bn[dst[u][2]] = ra.y * x1 + ra.x * z1;
                        Bn[dst[u][3]] = ra.y * y1 + ra.x * w1;
                    } else {
                        const double c = ra.x, sn = ra.y;
                        Bn[dst[u][0]] = c * c * x - 2.0 * c * sn * y + sn * sn * w;
                        Bn[dst[u][3]] = sn * sn * x + 2.0 * c * sn * y + c * c * w;
                        Bn[dst[u][1]] = (c * c - sn * sn) * y + c * sn * (x - w);
                    }
                }
            }
            __syncthreads();
            cur ^= 1;
            ++nsteps;
            xa = xa + 1 == m ? 0 : xa + 1;
            ya = ya + 1 == m ? 0 : ya + 1;
        }
    }
    if (wv == 0 && lane < h) {
        const int dblk = lane * (lane + 3) / 2;
        lam[lane == 0 ? 0 : 1 + xa] = buf[cur][dblk];
        lam[1 + ya] = buf[cur][3 * kSlotMaxBlk + dblk];
    }
    if (tid == 0) {
        *nsteps_out = nsteps;
        if (!converged) atomicOr(&flags[kFlagNumeric], 1);
    }
}

// The same order and slot layout for 64 < h <= 96 pairs (n <= 192), where two copies
// of B do not fit in LDS: one copy, two barriers per step (every owner reads its
// blocks and rotates them in registers, then all write the permuted blocks), wave 0
// computing the next rotations for two pairs per lane.  Rotations are logged in the
// roles of the packed-triangle kernel (p < q by index) for its eigenvector replay.
constexpr int kWideMaxH = kMaxSmall / 2;
constexpr int kWideMaxBlk = kWideMaxH * (kWideMaxH + 1) / 2;
__device__ __forceinline__ int slot_elem_wide(int i, int j) {
    int pa = i >> 1, pb = j >> 1, r = i & 1, t = j & 1;
    if (pa > pb) {
        int x = pa;
        pa = pb;
        pb = x;
        x = r;
        r = t;
        t = x;
    }
    if (pa == pb && r > t) {
        r = 0;
        t = 1;
    }
    return (r * 2 + t) * kWideMaxBlk + pb * (pb + 1) / 2 + pa;
}

__global__ __launch_bounds__(kSlotThreads) void jacobi_slots_wide_kernel(const double *__restrict__ Bg, int n,
                                                                         double *__restrict__ lam,
                                                                         double2 *__restrict__ rot_log,
                                                                         int *__restrict__ nsteps_out, int *flags) {
    constexpr int kWork = kSlotThreads - 64;
    constexpr int kIPT = (kWideMaxBlk + kWork - 1) / kWork;
    constexpr int kW = kSlotThreads / 64;
    constexpr int S = kWideMaxBlk;
    __shared__ __align__(16) double buf[4 * kWideMaxBlk];
    __shared__ __align__(16) double2 rot[2][kWideMaxH];
    __shared__ double red_off[kW], red_dg[kW];
    __shared__ int s_done;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int h = n / 2, m = n - 1, nblk = h * (h + 1) / 2;
    int ia[kIPT], ib[kIPT], dst[kIPT][4];
#pragma unroll
    for (int u = 0; u < kIPT; ++u) {
        const int idx = tid - 64 + kWork * u;
        ia[u] = -1;
        ib[u] = 0;
        dst[u][0] = dst[u][1] = dst[u][2] = dst[u][3] = 0;
        if (wv > 0 && idx < nblk) {
            int a, b;
            slot_blk_ab(idx, a, b);
            ia[u] = a;
            ib[u] = b;
            const int p0 = next_slot(2 * a, h, m), p1 = next_slot(2 * a + 1, h, m);
            const int q0 = next_slot(2 * b, h, m), q1 = next_slot(2 * b + 1, h, m);
            dst[u][0] = slot_elem_wide(p0, q0);
            dst[u][1] = slot_elem_wide(p0, q1);
            dst[u][2] = slot_elem_wide(p1, q0);
            dst[u][3] = slot_elem_wide(p1, q1);
        }
    }
    // wave 0: pairs lane and lane + 64, their look-ahead sources and index offsets
    int P0[2], P1[2], r0[2], r1[2], d0[2], d1[2], xb[2], xa[2], ya[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int a = lane + 64 * k < h ? lane + 64 * k : 0;
        const int s0 = prev_slot(2 * a, h, m), s1 = prev_slot(2 * a + 1, h, m);
        P0[k] = s0 >> 1;
        P1[k] = s1 >> 1;
        r0[k] = s0 & 1;
        r1[k] = s1 & 1;
        d0[k] = P0[k] * (P0[k] + 3) / 2;
        d1[k] = P1[k] * (P1[k] + 3) / 2;
        xb[k] = slot_blk(P0[k], P1[k]);
        xa[k] = a % m;
        ya[k] = (m - a) % m;
    }
    for (int e = tid; e < nblk * 4; e += kSlotThreads) {
        const int blk = e >> 2, pos = e & 3;
        int a, b;
        slot_blk_ab(blk, a, b);
        const int gi = slot_index_at0(2 * a + (pos >> 1), m), gj = slot_index_at0(2 * b + (pos & 1), m);
        buf[pos * S + blk] = 0.5 * (Bg[(int64_t)gi * n + gj] + Bg[(int64_t)gj * n + gi]);
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int a = lane + 64 * k;
            if (a >= h) continue;
            const int dblk = a * (a + 3) / 2;
            const double2 r = slot_rotation(buf[dblk], buf[S + dblk], buf[3 * S + dblk]);
            rot[0][a] = r;
            // logged with p < q by index: slot 2a holds 0 (a = 0) or 1 + xa, slot 2a+1 holds 1 + ya
            rot_log[a] = make_double2(r.x, (a == 0 || xa[k] < ya[k]) ? r.y : -r.y);
        }
    }
    int nsteps = 0;
    bool converged = false;
    for (int sweep = 0; sweep <= kMaxSweeps; ++sweep) {
        double off = 0.0, dg = 0.0;
        for (int e = tid; e < nblk; e += kSlotThreads) {
            int a, b;
            slot_blk_ab(e, a, b);
            const double x = buf[e], y = buf[S + e], z = buf[2 * S + e], w = buf[3 * S + e];
            if (a == b) {
                off += y * y;
                dg += x * x + w * w;
            } else {
                off += x * x + y * y + z * z + w * w;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_xor(off, o);
            dg += __shfl_xor(dg, o);
        }
        if (lane == 0) {
            red_off[wv] = off;
            red_dg[wv] = dg;
        }
        __syncthreads();
        if (tid == 0) {
            double so = 0.0, sd = 0.0;
            for (int w = 0; w < kW; ++w) {
                so += red_off[w];
                sd += red_dg[w];
            }
            s_done = (so <= 1e-26 * sd) || so == 0.0;
        }
        __syncthreads();
        if (s_done) {
            converged = true;
            break;
        }
        if (sweep == kMaxSweeps) break;
        for (int st = 0; st < m; ++st) {
            const double2 *R = rot[nsteps & 1];
            double out[kIPT][4];
            if (wv == 0) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int a = lane + 64 * k;
                    if (a >= h) continue;
                    double u00, u01, u10, u11;
                    rot_col(R[P0[k]], r0[k], u00, u01);
                    rot_col(R[P1[k]], r1[k], u10, u11);
                    const double a0 = buf[d0[k]], b0 = buf[S + d0[k]], c0 = buf[3 * S + d0[k]];
                    const double a1 = buf[d1[k]], b1 = buf[S + d1[k]], c1 = buf[3 * S + d1[k]];
                    const double x = buf[xb[k]], y = buf[S + xb[k]], z = buf[2 * S + xb[k]], w = buf[3 * S + xb[k]];
                    const double app = u00 * (u00 * a0 + u01 * b0) + u01 * (u00 * b0 + u01 * c0);
                    const double aqq = u10 * (u10 * a1 + u11 * b1) + u11 * (u10 * b1 + u11 * c1);
                    const double apq = P0[k] < P1[k] ? u00 * (x * u10 + y * u11) + u01 * (z * u10 + w * u11)
                                                     : u10 * (x * u00 + y * u01) + u11 * (z * u00 + w * u01);
                    const double2 r = slot_rotation(app, apq, aqq);
                    rot[(nsteps + 1) & 1][a] = r;
                    const int x1 = xa[k] + 1 == m ? 0 : xa[k] + 1, y1 = ya[k] + 1 == m ? 0 : ya[k] + 1;
                    rot_log[(int64_t)(nsteps + 1) * h + a] = make_double2(r.x, (a == 0 || x1 < y1) ? r.y : -r.y);
                }
            } else {
#pragma unroll
                for (int u = 0; u < kIPT; ++u) {
                    if (ia[u] < 0) continue;
                    const int a = ia[u], b = ib[u];
                    const int e = b * (b + 1) / 2 + a;
                    const double x = buf[e], y = buf[S + e], z = buf[2 * S + e], w = buf[3 * S + e];
                    const double2 ra = R[a], rb = R[b];
                    if (a != b) {
                        const double x1 = rb.x * x - rb.y * y, y1 = rb.y * x + rb.x * y;
                        const double z1 = rb.x * z - rb.y * w, w1 = rb.y * z + rb.x * w;
                        out[u][0] = ra.x * x1 - ra.y * z1;
                        out[u][1] = ra.x * y1 - ra.y * w1;
                        out[u][2] = ra.y * x1 + ra.x * z1;
                        out[u][3] = ra.y * y1 + ra.x * w1;
                    } else {
                        const double c = ra.x, sn = ra.y;
                        out[u][0] = c * c * x - 2.0 * c * sn * y + sn * sn * w;
                        out[u][3] = sn * sn * x + 2.0 * c * sn * y + c * c * w;
                        out[u][1] = (c * c - sn * sn) * y + c * sn * (x - w);
                        out[u][2] = 0.0;
                    }
                }
            }
            __syncthreads();
            if (wv != 0) {
#pragma unroll
                for (int u = 0; u < kIPT; ++u) {
                    if (ia[u] < 0) continue;
                    buf[dst[u][0]] = out[u][0];
                    buf[dst[u][1]] = out[u][1];
                    buf[dst[u][3]] = out[u][3];
                    if (ia[u] != ib[u]) buf[dst[u][2]] = out[u][2];
                }
            }
            __syncthreads();
            ++nsteps;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                xa[k] = xa[k] + 1 == m ? 0 : xa[k] + 1;
                ya[k] = ya[k] + 1 == m ? 0 : ya[k] + 1;
            }
        }
    }
    if (wv == 0) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int a = lane + 64 * k;
            if (a >= h) continue;
            const int dblk = a * (a + 3) / 2;
            lam[a == 0 ? 0 : 1 + xa[k]] = buf[dblk];
            lam[1 + ya[k]] = buf[3 * S + dblk];
        }
    }
    if (tid == 0) {
        *nsteps_out = nsteps;
        if (!converged) atomicOr(&flags[kFlagNumeric], 1);
    }
}

// Lane shifts across the wave (DPP wave_shl:1 / wave_shr:1), on the two halves of a double.
__device__ __forceinline__ double wave_from_next(double v) {   // lane i receives lane i + 1
    const int2 x = __builtin_bit_cast(int2, v);
    int2 y;
    y.x = __builtin_amdgcn_update_dpp(0, x.x, 0x130, 0xf, 0xf, false);
    y.y = __builtin_amdgcn_update_dpp(0, x.y, 0x130, 0xf, 0xf, false);
    return __builtin_bit_cast(double, y);
}
__device__ __forceinline__ double wave_from_prev(double v) {   // lane i receives lane i - 1
    const int2 x = __builtin_bit_cast(int2, v);
    int2 y;
    y.x = __builtin_amdgcn_update_dpp(0, x.x, 0x138, 0xf, 0xf, false);
    y.y = __builtin_amdgcn_update_dpp(0, x.y, 0x138, 0xf, 0xf, false);
    return __builtin_bit_cast(double, y);
}

// Eigenvectors from the slot log: one wave per row of P, lane a holding the row's
// entries in slots 2a and 2a+1.  A step rotates them in registers and applies pi
// with lane shifts (pi moves slot 2a to 2a-2 and slot 2a+1 to 2a+3, except at
// pairs 0, 1 and h-1); rotations are prefetched kSlotRing steps ahead.
constexpr int kSlotRing = 8;
__global__ __launch_bounds__(256) void jacobi_slots_replay_kernel(const double2 *__restrict__ rot_log,
                                                                  const int *__restrict__ nsteps_ptr, int n,
                                                                  double *__restrict__ P) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const int h = n / 2, m = n - 1;
    const int srow = row == 0 ? 0 : circ_slot(row - 1, h, m);
    double v0 = (lane < h && 2 * lane == srow) ? 1.0 : 0.0;
    double v1 = (lane < h && 2 * lane + 1 == srow) ? 1.0 : 0.0;
    const int nsteps = *nsteps_ptr;
    const int la = lane < h ? lane : h - 1;
    const int last = nsteps > 0 ? nsteps - 1 : 0;
    double2 ring[kSlotRing];
#pragma unroll
    for (int d = 0; d < kSlotRing; ++d) ring[d] = rot_log[(int64_t)(d < last ? d : last) * h + la];
    for (int st = 0; st < nsteps; st += kSlotRing) {
#pragma unroll
        for (int d = 0; d < kSlotRing; ++d) {
            const double2 r = ring[d];
            const int nx = st + d + kSlotRing < last ? st + d + kSlotRing : last;
            ring[d] = rot_log[(int64_t)nx * h + la];
            if (st + d < nsteps) {
                const double a0 = r.x * v0 - r.y * v1, a1 = r.y * v0 + r.x * v1;
                const double from_next = wave_from_next(a0), from_prev = wave_from_prev(a1);
                v0 = lane == 0 ? a0 : (lane == h - 1 ? a1 : from_next);
                v1 = lane == 0 ? (h == 1 ? a1 : from_next) : from_prev;
            }
        }
    }
    if (lane < h) {
        P[(int64_t)row * n + (lane == 0 ? 0 : 1 + (lane + nsteps) % m)] = v0;
        P[(int64_t)row * n + 1 + (m - lane + nsteps) % m] = v1;
    }
}

// ---------------------------------------------------------------- basis selection
// perm by decreasing eigenvalue (ties by index), T_u[i][r] = P[i][perm[r]], sigma.
__global__ __launch_bounds__(256) void select_kernel(const double *__restrict__ lam, const double *__restrict__ P,
                                                     int n, int k, double *__restrict__ T_u,
                                                     double *__restrict__ sigma, int *__restrict__ perm) {
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        int rank = 0;
        const double lj = lam[j];
        for (int i = 0; i < n; ++i) {
            const double li = lam[i];
            rank += (li > lj) || (li == lj && i < j);
        }
        if (rank < k) {
            perm[rank] = j;
            sigma[rank] = sqrt(fmax(lj, 0.0));
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < n * k; idx += blockDim.x) {
        const int r = idx / n, i = idx % n;
        T_u[(int64_t)r * n + i] = P[(int64_t)i * n + perm[r]];
    }
}

// Sign of each column: the entry of largest magnitude (first such index) of
// Wk[:, r] becomes positive.  Flips T_u column r and sets scale_v[r] = 1 / sigma.
__global__ __launch_bounds__(256) void sign_fix_kernel(const double *__restrict__ Wk, int64_t N, int64_t ldw,
                                                       int n, double *__restrict__ T_u,
                                                       const double *__restrict__ sigma, double *__restrict__ scale_v) {
    const int r = blockIdx.x;
    __shared__ double s_val[256];
    __shared__ int64_t s_idx[256];
    double best = -1.0;
    int64_t bidx = 0;
    double bval = 0.0;
    for (int64_t t = threadIdx.x; t < N; t += blockDim.x) {
        const double v = Wk[(int64_t)r * ldw + t];
        if (fabs(v) > best) {
            best = fabs(v);
            bidx = t;
            bval = v;
        }
    }
    s_val[threadIdx.x] = best;
    s_idx[threadIdx.x] = bidx;
    __shared__ double s_sgn[256];
    s_sgn[threadIdx.x] = bval;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double a = s_val[threadIdx.x], b = s_val[threadIdx.x + o];
            const int64_t ia = s_idx[threadIdx.x], ib = s_idx[threadIdx.x + o];
            if (b > a || (b == a && ib < ia)) {
                s_val[threadIdx.x] = b;
                s_idx[threadIdx.x] = ib;
                s_sgn[threadIdx.x] = s_sgn[threadIdx.x + o];
            }
        }
        __syncthreads();
    }
    const double sg = s_sgn[0] < 0.0 ? -1.0 : 1.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) T_u[(int64_t)r * n + i] *= sg;
    if (threadIdx.x == 0) {
        const double sv = sigma[r];
        scale_v[r] = sv > 0.0 ? 1.0 / sv : 0.0;   // the sign is already in T_u
    }
}

// spectrum[rank(j)] = lam[j]: every eigenvalue in decreasing order (ties by index).
__global__ __launch_bounds__(256) void spectrum_kernel(const double *__restrict__ lam, int n,
                                                       double *__restrict__ spectrum) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double lj = lam[j];
    int rank = 0;
    for (int i = 0; i < n; ++i) {
        const double li = lam[i];
        rank += (li > lj) || (li == lj && i < j);
    }
    spectrum[rank] = lj;
}

__global__ __launch_bounds__(256) void column_norm_kernel(const double *__restrict__ W, int64_t N, int64_t ldw,
                                                          double *__restrict__ sigma, double *__restrict__ scale) {
    const int j = blockIdx.x;
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < N; t += blockDim.x) {
        const double v = W[(int64_t)j * ldw + t];
        s += v * v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double nrm = sqrt(red[0]);
        sigma[j] = nrm;
        scale[j] = nrm > 0.0 ? 1.0 / nrm : 0.0;
    }
}

__global__ void basis_to_bf16_kernel(const float *__restrict__ U, int64_t M, int k, int64_t ldq, int Lpad,
                                     unsigned short *__restrict__ hi, unsigned short *__restrict__ lo) {
    const int64_t total = (int64_t)Lpad * ldq;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = idx / ldq, p = idx % ldq;
        unsigned short h = 0, l = 0;
        if (j < k && p < M) {
            const float v = U[j * M + p];
            h = f32_to_bf16_bits(v);
            l = f32_to_bf16_bits(v - bf16_bits_to_f32(h));
        }
        hi[idx] = h;
        if (lo) lo[idx] = l;
    }
}

__global__ void identity_kernel(double *T, int n) {
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * n; idx += gridDim.x * blockDim.x)
        T[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
}

}  // namespace

size_t jacobi_rot_bytes(int n) {
    if (n > kMaxSmall) return jacobi_block_work_bytes(n);
    return (size_t)(kMaxSweeps + 1) * (size_t)(n - 1) * (size_t)(n / 2) * sizeof(double2) + 256;
}

xpcs_status launch_tsgram(xpcs_ctx *ctx, const void *A, bool a_f64, int64_t rows, int64_t lda, int ncols,
                          const int32_t *row_idx, const int64_t *seg_off, int nseg, double *G) {
    Phase phase_(ctx, "tsgram");
    if (ncols > kMaxSmall) return launch_panel_gram(ctx, A, a_f64, rows, lda, ncols, row_idx, seg_off, nseg, G);
    const int nc4 = (ncols + 3) / 4;
    const int pw = nc4 * 4;
    const int nblk = nc4 * (nc4 + 1) / 2;
    const int bpt = (nblk + 255) / 256;
    // up to 256 blocks (one per CU) of at least 64 rows; segmented Grams split the blocks
    int nparts = (int)(rows / 64);
    if (nparts > 256) nparts = 256;
    if (seg_off) nparts = (int)(256 / (nseg > 0 ? nseg : 1)) + 1;
    if (nparts < 1) nparts = 1;
    const size_t pbytes = (size_t)nseg * nparts * pw * pw * sizeof(double);
    xpcs_status st;
    double *part = static_cast<double *>(scratch_get(ctx, pbytes, &st));
    if (!part) return st;
    const int grows = bpt <= 2 ? GramShape<1>::kRows : GramShape<3>::kRows;
    const int gthreads = 256 * (bpt == 1 ? GramShape<1>::kGroups : (bpt == 2 ? GramShape<2>::kGroups : 1));
    const size_t lds_tile = (size_t)grows * (pw + 2) * sizeof(double);
    const size_t lds_sums = (size_t)nblk * 16 * sizeof(double);     // one 4x4 block per owned block id
    const size_t lds = lds_tile > lds_sums ? lds_tile : lds_sums;
    dim3 grid(nparts, nseg);
    // 81..192 columns: the FP64 MFMA kernel over pairs of column groups
    if (ncols > 80 && (seg_off || (!row_idx && nseg == 1))) {
        const int nbatch = seg_off ? nseg : 1;
        const int ncb = (ncols + 15) / 16;
        const int ng = (ncb + 4) / 5;                  // groups of at most 5 blocks
        const int gsz = (ncb + ng - 1) / ng;      // blocks per group
        const bool vec = !row_idx && !seg_off && lda % 4 == 0 && (uintptr_t)A % 16 == 0;
        const int npairs = ng * (ng - 1) / 2;
#define XPCS_TSGP(T, GG)                                                                                            \
    do {                                                                                                          \
        hipLaunchKernelGGL((tsgram_pair_kernel<T, GG, true>), dim3(nparts, nbatch, ng), dim3(kGramPairThreads), 0,   \
                           ctx->stream, static_cast<const T *>(A), rows, lda, ncols, pw, ng, part, row_idx, seg_off, \
                           vec);                                                                                  \
        if (npairs > 0)                                                                                           \
            hipLaunchKernelGGL((tsgram_pair_kernel<T, GG, false>), dim3(nparts, nbatch, npairs),                   \
                               dim3(kGramPairThreads), 0, ctx->stream, static_cast<const T *>(A), rows, lda, ncols, \
                               pw, ng, part, row_idx, seg_off, vec);                                              \
    } while (0)
#define XPCS_TSGP_T(T)                      \
    switch (gsz) {                          \
        case 3: XPCS_TSGP(T, 3); break;     \
        case 4: XPCS_TSGP(T, 4); break;     \
        default: XPCS_TSGP(T, 5); break;    \
    }
        if (a_f64) {
            XPCS_TSGP_T(double)
        } else {
            XPCS_TSGP_T(float)
        }
#undef XPCS_TSGP_T
#undef XPCS_TSGP
        XPCS_LAUNCH_CHECK(ctx, "tsgram_pair");
        hipLaunchKernelGGL(tsgram_reduce_kernel, dim3((ncols * ncols + 31) / 32, nseg), dim3(256), 0, ctx->stream,
                           part, nparts, ncols, pw, G);
        XPCS_LAUNCH_CHECK(ctx, "tsgram_reduce");
        return XPCS_OK;
    }
    // up to 80 columns: the FP64 MFMA kernel (one matrix, or one segment per blockIdx.y)
    if (ncols <= 80 && (seg_off || (!row_idx && nseg == 1))) {
        const int nbatch = seg_off ? nseg : 1;
        const int64_t bstride = 0;
        const int ncb = (ncols + 15) / 16;
        const bool vec = !row_idx && !seg_off && lda % 4 == 0 && (uintptr_t)A % 16 == 0;
#define XPCS_TSGM(T, C)                                                                                       \
    hipLaunchKernelGGL((tsgram_mfma_kernel<T, C>), dim3(nparts, nbatch), dim3(kGramMfmaThreads), 0, ctx->stream, \
                       static_cast<const T *>(A), rows, lda, ncols, pw, part, bstride, row_idx, seg_off, vec)
#define XPCS_TSGM_T(T)                \
    switch (ncb) {                    \
        case 1: XPCS_TSGM(T, 1); break; \
        case 2: XPCS_TSGM(T, 2); break; \
        case 3: XPCS_TSGM(T, 3); break; \
        case 4: XPCS_TSGM(T, 4); break; \
        default: XPCS_TSGM(T, 5); break; \
    }
        if (a_f64) {
            XPCS_TSGM_T(double)
        } else {
            XPCS_TSGM_T(float)
        }
#undef XPCS_TSGM_T
#undef XPCS_TSGM
        XPCS_LAUNCH_CHECK(ctx, "tsgram_mfma");
        hipLaunchKernelGGL(tsgram_reduce_kernel, dim3((ncols * ncols + 31) / 32, nseg), dim3(256), 0, ctx->stream,
                           part, nparts, ncols, pw, G);
        XPCS_LAUNCH_CHECK(ctx, "tsgram_reduce");
        return XPCS_OK;
    }
#define XPCS_TSG(T, B)                                                                                          \
    hipLaunchKernelGGL((tsgram_kernel<T, B>), grid, dim3(gthreads), lds, ctx->stream,                            \
                       static_cast<const T *>(A), rows, lda, ncols, row_idx, seg_off, part)
#define XPCS_TSG_T(T)                   \
    switch (bpt) {                      \
        case 1: XPCS_TSG(T, 1); break;  \
        case 2: XPCS_TSG(T, 2); break;  \
        case 3: XPCS_TSG(T, 3); break;  \
        case 4: XPCS_TSG(T, 4); break;  \
        default: XPCS_TSG(T, 5); break; \
    }
    if (a_f64) {
        XPCS_TSG_T(double)
    } else {
        XPCS_TSG_T(float)
    }
#undef XPCS_TSG_T
#undef XPCS_TSG
    XPCS_LAUNCH_CHECK(ctx, "tsgram");
    hipLaunchKernelGGL(tsgram_reduce_kernel, dim3((ncols * ncols + 31) / 32, nseg), dim3(256), 0, ctx->stream,
                       part, nparts, ncols, pw, G);
    XPCS_LAUNCH_CHECK(ctx, "tsgram_reduce");
    return XPCS_OK;
}

// Grams of nbatch tall matrices A + b * bstride (rows x ncols, column stride lda):
// G + b * ncols^2.  One launch of the FP64 MFMA kernel for up to 80 columns,
// otherwise one Gram after the other.
xpcs_status launch_tsgram_batched(xpcs_ctx *ctx, const void *A, bool a_f64, int64_t rows, int64_t lda, int ncols,
                                  int nbatch, int64_t bstride, double *G) {
    if (ncols > 80 || nbatch == 1) {
        xpcs_status st;
        const size_t esz = a_f64 ? 8 : 4;
        for (int b = 0; b < nbatch; ++b)
            if ((st = launch_tsgram(ctx, static_cast<const char *>(A) + (size_t)b * bstride * esz, a_f64, rows, lda,
                                    ncols, nullptr, nullptr, 1, G + (int64_t)b * ncols * ncols)))
                return st;
        return XPCS_OK;
    }
    Phase phase_(ctx, "tsgram");
    const int pw = (ncols + 3) / 4 * 4;
    int nparts = (int)(rows / 64);
    if (nparts > 256 / nbatch + 1) nparts = 256 / nbatch + 1;
    if (nparts < 1) nparts = 1;
    xpcs_status st;
    double *part = static_cast<double *>(scratch_get(ctx, (size_t)nbatch * nparts * pw * pw * sizeof(double), &st));
    if (!part) return st;
    const int ncb = (ncols + 15) / 16;
    const bool vec = lda % 4 == 0 && bstride % 4 == 0 && (uintptr_t)A % 16 == 0;
#define XPCS_TSGB(T, C)                                                                                          \
    hipLaunchKernelGGL((tsgram_mfma_kernel<T, C>), dim3(nparts, nbatch), dim3(kGramMfmaThreads), 0, ctx->stream, \
                       static_cast<const T *>(A), rows, lda, ncols, pw, part, bstride, nullptr, nullptr, vec)
#define XPCS_TSGB_T(T)                 \
    switch (ncb) {                     \
        case 1: XPCS_TSGB(T, 1); break; \
        case 2: XPCS_TSGB(T, 2); break; \
        case 3: XPCS_TSGB(T, 3); break; \
        case 4: XPCS_TSGB(T, 4); break; \
        default: XPCS_TSGB(T, 5); break; \
    }
    if (a_f64) {
        XPCS_TSGB_T(double)
    } else {
        XPCS_TSGB_T(float)
    }
#undef XPCS_TSGB_T
#undef XPCS_TSGB
    XPCS_LAUNCH_CHECK(ctx, "tsgram_mfma");
    hipLaunchKernelGGL(tsgram_reduce_kernel, dim3((ncols * ncols + 31) / 32, nbatch), dim3(256), 0, ctx->stream, part,
                       nparts, ncols, pw, G);
    XPCS_LAUNCH_CHECK(ctx, "tsgram_reduce");
    return XPCS_OK;
}

xpcs_status launch_cholinv(xpcs_ctx *ctx, const double *G, int n, double rel_tol, const double *Rprev,
                           double *Rinv) {
    Phase phase_(ctx, "cholinv");
    if (n > kMaxSmall) {
        if (Rprev) return fail(ctx, XPCS_EUNSUPPORTED, "internal: product with a previous factor above 192");
        xpcs_status st;
        void *work = scratch_get(ctx, cholinv_blocked_work_bytes(n), &st);
        if (!work) return st;
        return launch_cholinv_blocked(ctx, G, n, rel_tol, Rinv, work);
    }
    double *dst = Rinv;
    if (Rprev) {
        xpcs_status st;
        dst = static_cast<double *>(scratch_get(ctx, (size_t)n * n * sizeof(double), &st));
        if (!dst) return st;
    }
    if (n <= 96)        // fewer owned elements per thread: each step's loop is shorter
        hipLaunchKernelGGL((cholinv_reg_kernel<96, 1024>), dim3(1), dim3(1024), 0, ctx->stream, G, n, rel_tol, dst,
                           ctx->flags);
    else if (n <= 128)
        hipLaunchKernelGGL((cholinv_reg_kernel<128, 1024>), dim3(1), dim3(1024), 0, ctx->stream, G, n, rel_tol, dst,
                           ctx->flags);
    else if (n <= 160)
        hipLaunchKernelGGL((cholinv_reg_kernel<160, 1024>), dim3(1), dim3(1024), 0, ctx->stream, G, n, rel_tol, dst,
                           ctx->flags);
    else        // 512 threads: the 37 elements a thread holds need more than 128 registers
        hipLaunchKernelGGL((cholinv_reg_kernel<kMaxSmall, 512>), dim3(1), dim3(512), 0, ctx->stream, G, n, rel_tol,
                           dst, ctx->flags);
    XPCS_LAUNCH_CHECK(ctx, "cholinv");
    if (Rprev) {
        hipLaunchKernelGGL(small_matmul_kernel, dim3(1), dim3(256), 0, ctx->stream, Rprev, dst, n, Rinv);
        XPCS_LAUNCH_CHECK(ctx, "small_matmul");
    }
    return XPCS_OK;
}

size_t chol_batched_work_bytes(int n, int nb) { return n > kMaxSmall ? chol_blocked_work_bytes(n, nb) : 0; }

xpcs_status launch_chol_batched(xpcs_ctx *ctx, const double *G, int n, int nb, double *L, void *work) {
    Phase phase_(ctx, "chol_batched");
    if (n > kMaxSmall) {
        xpcs_status st;
        if (!work && !(work = scratch_get(ctx, chol_blocked_work_bytes(n, nb), &st))) return st;
        return launch_chol_blocked(ctx, G, n, nb, 1e-13, L, work);
    }
    hipLaunchKernelGGL(chol_batched_kernel, dim3(nb), dim3(1024), 0, ctx->stream, G, n, 1e-13, L);
    XPCS_LAUNCH_CHECK(ctx, "chol_batched");
    return XPCS_OK;
}

xpcs_status launch_tsmul(xpcs_ctx *ctx, const void *A, bool a_f64, int64_t rows, int64_t lda, int n,
                         const double *T, int m, const double *colscale, const TsOut &out, bool t_upper) {
    Phase phase_(ctx, "tsmul");
    const int64_t span = (out.hi || out.f8) && out.rows_pad > rows ? out.rows_pad : rows;
    if (span <= 0 || m <= 0) return XPCS_OK;
    auto al = [](const void *p, size_t b) { return (reinterpret_cast<uintptr_t>(p) & (b - 1)) == 0; };
    auto go = [&](auto ta, auto narrow_c) {
        using TA = decltype(ta);
        using S = TsmShape<TA>;
        constexpr int SUB = S::SUB;
        int vf = 0;
        if (al(A, SUB * sizeof(TA) < 16 ? SUB * sizeof(TA) : 16) && lda % SUB == 0) vf |= kTsmVecA;
        if (out.out32 && al(out.out32, SUB * 4 < 16 ? SUB * 4 : 16) && out.ld32 % SUB == 0) vf |= kTsmVec32;
        if (out.out64 && al(out.out64, 16) && out.ld64 % SUB == 0) vf |= kTsmVec64;
        if ((!out.hi || al(out.hi, SUB * 2)) && (!out.lo || al(out.lo, SUB * 2)) && out.ldh % SUB == 0) vf |= kTsmVecH;
        if (out.f8 && al(out.f8, SUB) && out.ldh % SUB == 0) vf |= kTsmVecF8;
        const int gy = (m + kTsmCols - 1) / kTsmCols;
        const int64_t nstrips = (span + 16 * SUB - 1) / (16 * SUB);
        const int64_t want = (nstrips + S::W - 1) / S::W;
        const int64_t cap = (S::BPC * 256 + gy - 1) / gy;
        dim3 grid((unsigned)(want < cap ? want : cap), (unsigned)gy);
        hipLaunchKernelGGL((tsmul_mfma_kernel<TA, decltype(narrow_c)::value, SUB, S::W, S::WPE, S::AH>), grid,
                           dim3(64 * S::W), 0, ctx->stream, static_cast<const TA *>(A), rows, lda, n, T, m,
                           (int)t_upper, colscale, out.out32, out.ld32, out.out64, out.ld64, out.hi, out.lo, out.f8,
                           out.ldh, out.Lpad, out.rows_pad, span, vf);
    };
    const bool narrow = out.hi || out.f8;
    if (a_f64)
        narrow ? go(double(), std::true_type{}) : go(double(), std::false_type{});
    else
        narrow ? go(float(), std::true_type{}) : go(float(), std::false_type{});
    XPCS_LAUNCH_CHECK(ctx, "tsmul");
    return XPCS_OK;
}

xpcs_status launch_tsmul_counts(xpcs_ctx *ctx, const void *frames, int dtype, int64_t M, int64_t N,
                                const double *T, int m, const double *colscale, const TsOut &out) {
    Phase phase_(ctx, "tsmul");
    dim3 grid((unsigned)((M + 256 * kTsRows - 1) / (256 * kTsRows)), (unsigned)((m + kTsCols - 1) / kTsCols));
    if (dtype == XPCS_U8)
        hipLaunchKernelGGL(tsmul_kernel<uint8_t>, grid, dim3(256), 0, ctx->stream, static_cast<const uint8_t *>(frames),
                           M, M, (int)N, T, m, colscale, out.out32, out.ld32, out.out64, out.ld64, out.hi, out.lo,
                           out.f8, out.ldh, out.Lpad, out.rows_pad);
    else
        hipLaunchKernelGGL(tsmul_kernel<uint16_t>, grid, dim3(256), 0, ctx->stream,
                           static_cast<const uint16_t *>(frames), M, M, (int)N, T, m, colscale, out.out32, out.ld32,
                           out.out64, out.ld64, out.hi, out.lo, out.f8, out.ldh, out.Lpad, out.rows_pad);
    XPCS_LAUNCH_CHECK(ctx, "tsmul");
    return XPCS_OK;
}

xpcs_status launch_jacobi(xpcs_ctx *ctx, const double *B, int n, double *lam, double *P, void *rot) {
    Phase phase_(ctx, "jacobi");
    if (n % 2) return fail(ctx, XPCS_EUNSUPPORTED, "internal: eigen size must be even");
    if (n > kMaxSmall) return launch_jacobi_block(ctx, B, n, lam, P, rot);
    int *nsteps = static_cast<int *>(rot);
    double2 *log = reinterpret_cast<double2 *>(static_cast<char *>(rot) + 256);
    if (n <= 2 * kSlotMaxH) {
        hipLaunchKernelGGL(jacobi_slots_kernel, dim3(1), dim3(kSlotThreads), 0, ctx->stream, B, n, lam, log, nsteps,
                           ctx->flags);
        XPCS_LAUNCH_CHECK(ctx, "jacobi_slots");
        hipLaunchKernelGGL(jacobi_slots_replay_kernel, dim3((n + 3) / 4), dim3(256), 0, ctx->stream, log, nsteps, n, P);
        XPCS_LAUNCH_CHECK(ctx, "jacobi_slots_replay");
        return XPCS_OK;
    }
    hipLaunchKernelGGL(jacobi_slots_wide_kernel, dim3(1), dim3(kSlotThreads), 0, ctx->stream, B, n, lam, log,
                       nsteps, ctx->flags);
    XPCS_LAUNCH_CHECK(ctx, "jacobi_slots_wide");
    hipLaunchKernelGGL(jacobi_replay_kernel, dim3((n + kReplayWaves - 1) / kReplayWaves), dim3(64 * kReplayWaves), 0,
                       ctx->stream, log, nsteps, n, P);
    XPCS_LAUNCH_CHECK(ctx, "jacobi_replay");
    return XPCS_OK;
}

xpcs_status launch_select_basis(xpcs_ctx *ctx, const double *lam, const double *P, int n, int k, const double *Wl,
                                int64_t N, int64_t ldw, double *T_u, double *scale_v, double *sigma) {
    Phase phase_(ctx, "select_basis");
    xpcs_status st;
    const size_t pb = align_up((size_t)k * sizeof(int), 256);
    char *sc = static_cast<char *>(scratch_get(ctx, pb + (size_t)N * k * sizeof(double), &st));
    if (!sc) return st;
    int *perm = reinterpret_cast<int *>(sc);
    double *Wk = reinterpret_cast<double *>(sc + pb);
    hipLaunchKernelGGL(select_kernel, dim3(1), dim3(256), 0, ctx->stream, lam, P, n, k, T_u, sigma, perm);
    XPCS_LAUNCH_CHECK(ctx, "select");
    TsOut o;
    o.out64 = Wk;
    o.ld64 = N;
    st = launch_tsmul(ctx, Wl, true, N, ldw, n, T_u, k, nullptr, o);
    if (st != XPCS_OK) return st;
    hipLaunchKernelGGL(sign_fix_kernel, dim3(k), dim3(256), 0, ctx->stream, Wk, N, N, n, T_u, sigma, scale_v);
    XPCS_LAUNCH_CHECK(ctx, "sign_fix");
    return XPCS_OK;
}

xpcs_status launch_select_exact(xpcs_ctx *ctx, const double *lam, const double *P, int n, int k, double *T_u,
                                double *scale_v, double *sigma, double *spectrum) {
    Phase phase_(ctx, "select_basis");
    xpcs_status st;
    int *perm = static_cast<int *>(scratch_get(ctx, (size_t)k * sizeof(int), &st));
    if (!perm) return st;
    hipLaunchKernelGGL(select_kernel, dim3(1), dim3(256), 0, ctx->stream, lam, P, n, k, T_u, sigma, perm);
    XPCS_LAUNCH_CHECK(ctx, "select");
    // the sign of each selected eigenvector from its own largest-magnitude entry
    hipLaunchKernelGGL(sign_fix_kernel, dim3(k), dim3(256), 0, ctx->stream, T_u, (int64_t)n, (int64_t)n, n, T_u,
                       sigma, scale_v);
    XPCS_LAUNCH_CHECK(ctx, "sign_fix");
    if (spectrum) {
        hipLaunchKernelGGL(spectrum_kernel, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, lam, n, spectrum);
        XPCS_LAUNCH_CHECK(ctx, "spectrum");
    }
    return XPCS_OK;
}

xpcs_status launch_column_norms(xpcs_ctx *ctx, const double *W, int64_t N, int64_t ldw, int k, double *sigma,
                                double *scale) {
    Phase phase_(ctx, "column_norms");
    hipLaunchKernelGGL(column_norm_kernel, dim3(k), dim3(256), 0, ctx->stream, W, N, ldw, sigma, scale);
    XPCS_LAUNCH_CHECK(ctx, "column_norms");
    return XPCS_OK;
}

xpcs_status launch_basis_to_bf16(xpcs_ctx *ctx, const float *U, int64_t M, int k, int64_t ldq, int Lpad,
                                 unsigned short *hi, unsigned short *lo) {
    Phase phase_(ctx, "basis_to_bf16");
    const int64_t total = (int64_t)Lpad * ldq;
    int grid = (int)((total + 255) / 256);
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(basis_to_bf16_kernel, dim3(grid), dim3(256), 0, ctx->stream, U, M, k, ldq, Lpad, hi, lo);
    XPCS_LAUNCH_CHECK(ctx, "basis_to_bf16");
    return XPCS_OK;
}

xpcs_status launch_identity(xpcs_ctx *ctx, double *T, int n) {
    Phase phase_(ctx, "identity");
    hipLaunchKernelGGL(identity_kernel, dim3((n * n + 255) / 256), dim3(256), 0, ctx->stream, T, n);
    XPCS_LAUNCH_CHECK(ctx, "identity");
    return XPCS_OK;
}

}  // namespace xpcs
