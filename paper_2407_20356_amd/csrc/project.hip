// Products of the count matrix X with thin dense matrices on BF16 MFMA.
//
// These are the passes over the raw frames that build and apply the encoding
// basis (Sec. 2.1, Eqs. 3-7): Y = X Omega, Z = X^T Q, Y = X Z, W = X^T Q.  They
// read X once each and are bound by HBM bandwidth: a pass over a 2-byte count
// does 2*l flops per element, well under the BF16 MFMA ridge.
//
// Counts are integers, so bf16 holds them exactly up to 256; larger counts are
// carried as bf16 hi + lo (both exact), decided per wave and K step.
//
// X is stored frame-contiguous, X[t][p] = frames[t*M + p].
//  * proj_pixels contracts over frames (output per pixel).  A wave owns 16*RB
//    pixels, RB interleaved 16-row MFMA blocks (pixel = base + RB*row + s), so a
//    lane loads RB adjacent pixels of each of its 8 frames and every load of a
//    frame row is contiguous across the wave.
//  * proj_frames contracts over pixels (output per frame).  A lane loads 8
//    adjacent pixels of one frame, which is directly an MFMA K-group.  The pixel
//    range is split into chunks (partial sums reduced afterwards in a fixed
//    order); blocks sharing a chunk are placed on the same XCD so that the
//    chunk's slice of Q stays in that XCD's L2.
#include "internal.hpp"

namespace xpcs {
namespace {

constexpr unsigned short kBfOne = 0x3F80, kBfMinusOne = 0xBF80;

// ---------------------------------------------------------------- sketch
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void sketch_omega_kernel(uint64_t seed, int64_t N, int L, int ell, int64_t ldt,
                                    unsigned short *om) {
    const int64_t total = (int64_t)L * ldt;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = idx / ldt, t = idx % ldt;
        unsigned short v = 0;
        if (j < ell && t < N) {
            const uint64_t h = splitmix64(seed ^ (((uint64_t)t << 32) | (uint64_t)j));
            v = (h >> 63) ? kBfMinusOne : kBfOne;
        }
        om[idx] = v;
    }
}

// Integer count -> bf16 bits by truncation (exact for counts <= 256) and the
// exact remainder for larger counts.
__device__ __forceinline__ unsigned short count_hi_bits(unsigned v) {
    return (unsigned short)(__builtin_bit_cast(unsigned, (float)v) >> 16);
}
__device__ __forceinline__ unsigned short count_lo_bits(unsigned v) {
    const float hi = bf16_bits_to_f32(count_hi_bits(v));
    return (unsigned short)(__builtin_bit_cast(unsigned, (float)v - hi) >> 16);
}

template <typename T, int RB>
struct PixVec;
template <>
struct PixVec<uint16_t, 4> { typedef unsigned long long type; };
template <>
struct PixVec<uint16_t, 2> { typedef unsigned type; };
template <>
struct PixVec<uint8_t, 4> { typedef unsigned type; };
template <>
struct PixVec<uint8_t, 2> { typedef unsigned short type; };

template <typename T, int RB>
__device__ __forceinline__ void load_pixels(const T *__restrict__ src, bool vec, int nvalid,
                                            unsigned (&v)[RB]) {
    if (vec && nvalid >= RB) {
        typedef typename PixVec<T, RB>::type V;
        const V x = *reinterpret_cast<const V *>(src);
#pragma unroll
        for (int s = 0; s < RB; ++s) v[s] = (unsigned)((x >> (8 * sizeof(T) * s)) & ((1u << (8 * sizeof(T))) - 1u));
    } else {
#pragma unroll
        for (int s = 0; s < RB; ++s) v[s] = s < nvalid ? (unsigned)src[s] : 0u;
    }
}

// ---------------------------------------------------------------- pixel-space product
// Y[j][p] = sum_t X[t][p] * B[j][t], j < 16*NCB (+ column-group offset).
template <typename T, int RB, int NCB>
__global__ __launch_bounds__(256) void proj_pixels_kernel(const T *__restrict__ X, int64_t M, int64_t N,
                                                          const unsigned short *__restrict__ B, int64_t ldb,
                                                          float *__restrict__ Y, bool vec) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int jg = blockIdx.y * 16 * NCB;                  // column-group offset
    const int64_t pb = ((int64_t)blockIdx.x * 4 + wv) * (16 * RB);
    const int64_t pl = pb + RB * lr;                       // this lane's first pixel
    const int nvalid = pl >= M ? 0 : (M - pl >= RB ? RB : (int)(M - pl));

    f32x4 acc[RB][NCB];
#pragma unroll
    for (int s = 0; s < RB; ++s)
#pragma unroll
        for (int c = 0; c < NCB; ++c) acc[s][c] = (f32x4){0.f, 0.f, 0.f, 0.f};

    const unsigned short *brow[NCB];
#pragma unroll
    for (int c = 0; c < NCB; ++c) brow[c] = B + (int64_t)(jg + 16 * c + lr) * ldb + 8 * lg;

    for (int64_t tk = 0; tk < N; tk += 32) {
        unsigned v[8][RB];
        bool big = false;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t t = tk + 8 * lg + e;
            if (t < N && nvalid > 0) {
                load_pixels<T, RB>(X + t * M + pl, vec, nvalid, v[e]);
            } else {
#pragma unroll
                for (int s = 0; s < RB; ++s) v[e][s] = 0u;
            }
#pragma unroll
            for (int s = 0; s < RB; ++s) big |= v[e][s] > 256u;
        }
        u16x8 bf[NCB];
#pragma unroll
        for (int c = 0; c < NCB; ++c) bf[c] = *reinterpret_cast<const u16x8 *>(brow[c] + tk);
#pragma unroll
        for (int s = 0; s < RB; ++s) {
            u16x8 a;
#pragma unroll
            for (int e = 0; e < 8; ++e) a[e] = count_hi_bits(v[e][s]);
#pragma unroll
            for (int c = 0; c < NCB; ++c) acc[s][c] = mfma_bf16(a, bf[c], acc[s][c]);
        }
        if (sizeof(T) > 1 && __ballot(big)) {
#pragma unroll
            for (int s = 0; s < RB; ++s) {
                u16x8 a;
#pragma unroll
                for (int e = 0; e < 8; ++e) a[e] = count_lo_bits(v[e][s]);
#pragma unroll
                for (int c = 0; c < NCB; ++c) acc[s][c] = mfma_bf16(a, bf[c], acc[s][c]);
            }
        }
    }
    // acc[s][c][i] = Y[j = jg + 16c + lr][p = pb + RB*(4*lg + i) + s]
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
        float *yrow = Y + (int64_t)(jg + 16 * c + lr) * M;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int s = 0; s < RB; ++s) {
                const int64_t p = pb + RB * (4 * lg + i) + s;
                if (p < M) yrow[p] = acc[s][c][i];
            }
        }
    }
}

// ---------------------------------------------------------------- frame-space product
// part[chunk][t][j] = sum_{p in chunk} X[t][p] * Q[j][p] for j < 16*NCB (hi [+ lo]),
// and for j = 16*NCB + i < 16*(NCB + NIB) the indicator (label[p] == i).
template <typename T, int RB, int NCB, int NIB, bool LO>
__global__ __launch_bounds__(256) void proj_frames_kernel(const T *__restrict__ X, int64_t M, int64_t N,
                                                          const unsigned short *__restrict__ qh,
                                                          const unsigned short *__restrict__ ql,
                                                          int64_t ldq, const int32_t *__restrict__ labels,
                                                          int64_t chunk, int nfb, int ncols,
                                                          float *__restrict__ part, bool vec) {
    constexpr int FB = RB * 16 * 4;       // frames per block
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    // XCD-aware placement: consecutive blocks on one XCD walk the frame blocks of one chunk.
    const int bid = blockIdx.x, xcd = bid & 7, sl = bid >> 3;
    const int ch = xcd + 8 * (sl / nfb), fb = sl % nfb;
    const int64_t p_begin = (int64_t)ch * chunk;
    const int64_t p_end = p_begin + chunk < M ? p_begin + chunk : M;
    const int64_t tb = (int64_t)fb * FB + (int64_t)wv * RB * 16;

    f32x4 acc[RB][NCB + NIB];
#pragma unroll
    for (int s = 0; s < RB; ++s)
#pragma unroll
        for (int c = 0; c < NCB + NIB; ++c) acc[s][c] = (f32x4){0.f, 0.f, 0.f, 0.f};

    const T *xrow[RB];
    bool rok[RB];
#pragma unroll
    for (int s = 0; s < RB; ++s) {
        const int64_t t = tb + 16 * s + lr;
        rok[s] = t < N;
        xrow[s] = X + (rok[s] ? t : 0) * M + 8 * lg;
    }
    const unsigned short *qhr[NCB], *qlr[NCB];
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
        qhr[c] = qh + (int64_t)(16 * c + lr) * ldq + 8 * lg;
        qlr[c] = LO ? ql + (int64_t)(16 * c + lr) * ldq + 8 * lg : nullptr;
    }

    for (int64_t p0 = p_begin; p0 < p_end; p0 += 32) {
        const int64_t pl = p0 + 8 * lg;
        const int nv = pl >= p_end ? 0 : (p_end - pl >= 8 ? 8 : (int)(p_end - pl));
        unsigned v[RB][8];
        bool big = false;
#pragma unroll
        for (int s = 0; s < RB; ++s) {
            if (rok[s] && nv == 8 && vec) {
                if constexpr (sizeof(T) == 2) {
                    const u16x8 x = *reinterpret_cast<const u16x8 *>(xrow[s] + p0);
#pragma unroll
                    for (int e = 0; e < 8; ++e) v[s][e] = x[e];
                } else {
                    const unsigned long long x = *reinterpret_cast<const unsigned long long *>(xrow[s] + p0);
#pragma unroll
                    for (int e = 0; e < 8; ++e) v[s][e] = (unsigned)((x >> (8 * e)) & 0xffull);
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) v[s][e] = (rok[s] && e < nv) ? (unsigned)xrow[s][p0 + e] : 0u;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) big |= v[s][e] > 256u;
        }
        u16x8 a[RB];
#pragma unroll
        for (int s = 0; s < RB; ++s)
#pragma unroll
            for (int e = 0; e < 8; ++e) a[s][e] = count_hi_bits(v[s][e]);
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
            const u16x8 bh = *reinterpret_cast<const u16x8 *>(qhr[c] + p0);
#pragma unroll
            for (int s = 0; s < RB; ++s) acc[s][c] = mfma_bf16(a[s], bh, acc[s][c]);
            if constexpr (LO) {
                const u16x8 bl = *reinterpret_cast<const u16x8 *>(qlr[c] + p0);
#pragma unroll
                for (int s = 0; s < RB; ++s) acc[s][c] = mfma_bf16(a[s], bl, acc[s][c]);
            }
        }
        if constexpr (NIB > 0) {
            int lab[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) lab[e] = e < nv ? labels[pl + e] : -1;
#pragma unroll
            for (int ib = 0; ib < NIB; ++ib) {
                u16x8 ind;
                const int want = 16 * ib + lr;
#pragma unroll
                for (int e = 0; e < 8; ++e) ind[e] = lab[e] == want ? kBfOne : (unsigned short)0;
#pragma unroll
                for (int s = 0; s < RB; ++s) acc[s][NCB + ib] = mfma_bf16(a[s], ind, acc[s][NCB + ib]);
            }
        }
        if (sizeof(T) > 1 && __ballot(big)) {
            u16x8 al[RB];
#pragma unroll
            for (int s = 0; s < RB; ++s)
#pragma unroll
                for (int e = 0; e < 8; ++e) al[s][e] = count_lo_bits(v[s][e]);
#pragma unroll
            for (int c = 0; c < NCB; ++c) {
                const u16x8 bh = *reinterpret_cast<const u16x8 *>(qhr[c] + p0);
#pragma unroll
                for (int s = 0; s < RB; ++s) acc[s][c] = mfma_bf16(al[s], bh, acc[s][c]);
                if constexpr (LO) {
                    const u16x8 bl = *reinterpret_cast<const u16x8 *>(qlr[c] + p0);
#pragma unroll
                    for (int s = 0; s < RB; ++s) acc[s][c] = mfma_bf16(al[s], bl, acc[s][c]);
                }
            }
            if constexpr (NIB > 0) {
                int lab[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) lab[e] = e < nv ? labels[pl + e] : -1;
#pragma unroll
                for (int ib = 0; ib < NIB; ++ib) {
                    u16x8 ind;
                    const int want = 16 * ib + lr;
#pragma unroll
                    for (int e = 0; e < 8; ++e) ind[e] = lab[e] == want ? kBfOne : (unsigned short)0;
#pragma unroll
                    for (int s = 0; s < RB; ++s) acc[s][NCB + ib] = mfma_bf16(al[s], ind, acc[s][NCB + ib]);
                }
            }
        }
    }
    // acc[s][c][i] = part[ch][t = tb + 16s + 4lg + i][j = 16c + lr]
    float *pc = part + (int64_t)ch * N * ncols;
#pragma unroll
    for (int s = 0; s < RB; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t t = tb + 16 * s + 4 * lg + i;
            if (t < N) {
#pragma unroll
                for (int c = 0; c < NCB + NIB; ++c) pc[t * ncols + 16 * c + lr] = acc[s][c][i];
            }
        }
}

__global__ void proj_frames_reduce_kernel(const float *__restrict__ part, int64_t nch, int64_t N, int ncols,
                                          int L, int n_ind, double *__restrict__ Z, int64_t ldz,
                                          int64_t *__restrict__ S) {
    const int64_t total = N * ncols;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = idx / ncols;
        const int j = (int)(idx % ncols);
        const bool isq = j < L;
        const bool isind = S && j >= L && j - L < n_ind;
        if (!isq && !isind) continue;
        double s = 0.0;
        for (int64_t c = 0; c < nch; ++c) s += (double)part[(c * N + t) * ncols + j];
        if (isq)
            Z[(int64_t)j * ldz + t] = s;
        else
            S[(int64_t)(j - L) * N + t] = (int64_t)__builtin_rint(s);
    }
}

// ---------------------------------------------------------------- dispatch helpers
template <typename T, int RB, int NCB>
void launch_pp(dim3 grid, hipStream_t st, const void *X, int64_t M, int64_t N, const unsigned short *B,
               int64_t ldb, float *Y, bool vec) {
    hipLaunchKernelGGL((proj_pixels_kernel<T, RB, NCB>), grid, dim3(256), 0, st,
                       static_cast<const T *>(X), M, N, B, ldb, Y, vec);
}

template <typename T>
bool dispatch_pp(int ncb, int &rb_out, int ngroups_cb, dim3 gridx, hipStream_t st, const void *X, int64_t M,
                 int64_t N, const unsigned short *B, int64_t ldb, float *Y, bool vec4, bool vec2) {
    (void)ngroups_cb;
    switch (ncb) {
#define XPCS_PP4(n)                                                                             \
    case n: {                                                                                   \
        rb_out = 4;                                                                             \
        dim3 g((unsigned)((M + 255) / 256), gridx.y);                                           \
        launch_pp<T, 4, n>(g, st, X, M, N, B, ldb, Y, vec4);                                    \
        return true;                                                                            \
    }
        XPCS_PP4(1) XPCS_PP4(2) XPCS_PP4(3) XPCS_PP4(4) XPCS_PP4(5) XPCS_PP4(6)
#undef XPCS_PP4
#define XPCS_PP2(n)                                                                             \
    case n: {                                                                                   \
        rb_out = 2;                                                                             \
        dim3 g((unsigned)((M + 127) / 128), gridx.y);                                           \
        launch_pp<T, 2, n>(g, st, X, M, N, B, ldb, Y, vec2);                                    \
        return true;                                                                            \
    }
        XPCS_PP2(7) XPCS_PP2(8) XPCS_PP2(9) XPCS_PP2(10) XPCS_PP2(11) XPCS_PP2(12)
#undef XPCS_PP2
        default:
            return false;
    }
}

template <typename T, int RB, int NCB, int NIB, bool LO>
void launch_pf(int nblocks, hipStream_t st, const void *X, int64_t M, int64_t N, const unsigned short *qh,
               const unsigned short *ql, int64_t ldq, const int32_t *labels, int64_t chunk, int nfb,
               int ncols, float *part, bool vec) {
    hipLaunchKernelGGL((proj_frames_kernel<T, RB, NCB, NIB, LO>), dim3(nblocks), dim3(256), 0, st,
                       static_cast<const T *>(X), M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
}

// Frames per block as a function of the accumulator columns (NCB + NIB).
inline int pf_rb(int ncb, int nib) { return ncb + nib <= 8 ? 4 : 2; }

template <typename T, int NIB, bool LO>
bool dispatch_pf_ncb(int ncb, int nblocks, hipStream_t st, const void *X, int64_t M, int64_t N,
                     const unsigned short *qh, const unsigned short *ql, int64_t ldq, const int32_t *labels,
                     int64_t chunk, int nfb, int ncols, float *part, bool vec) {
    switch (ncb) {
#define XPCS_PF(n)                                                                                     \
    case n:                                                                                            \
        if (n + NIB <= 8)                                                                              \
            launch_pf<T, 4, n, NIB, LO>(nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols,   \
                                        part, vec);                                                    \
        else                                                                                           \
            launch_pf<T, 2, n, NIB, LO>(nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols,   \
                                        part, vec);                                                    \
        return true;
        XPCS_PF(1) XPCS_PF(2) XPCS_PF(3) XPCS_PF(4) XPCS_PF(5) XPCS_PF(6)
        XPCS_PF(7) XPCS_PF(8) XPCS_PF(9) XPCS_PF(10) XPCS_PF(11) XPCS_PF(12)
#undef XPCS_PF
        default:
            return false;
    }
}

template <typename T, bool LO>
bool dispatch_pf(int ncb, int nib, int nblocks, hipStream_t st, const void *X, int64_t M, int64_t N,
                 const unsigned short *qh, const unsigned short *ql, int64_t ldq, const int32_t *labels,
                 int64_t chunk, int nfb, int ncols, float *part, bool vec) {
    switch (nib) {
        case 0: return dispatch_pf_ncb<T, 0, LO>(ncb, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
        case 1: return dispatch_pf_ncb<T, 1, LO>(ncb, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
        case 2: return dispatch_pf_ncb<T, 2, LO>(ncb, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
        case 3: return dispatch_pf_ncb<T, 3, LO>(ncb, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
        case 4: return dispatch_pf_ncb<T, 4, LO>(ncb, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
        default: return false;
    }
}

}  // namespace

xpcs_status launch_sketch_omega(xpcs_ctx *ctx, uint64_t seed, int64_t N, int L, int ell, int64_t ldt,
                                unsigned short *om) {
    Phase phase_(ctx, "sketch_omega");
    int64_t total = (int64_t)L * ldt;
    int grid = (int)((total + 255) / 256);
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(sketch_omega_kernel, dim3(grid), dim3(256), 0, ctx->stream, seed, N, L, ell, ldt, om);
    XPCS_LAUNCH_CHECK(ctx, "sketch_omega");
    return XPCS_OK;
}

xpcs_status launch_proj_pixels(xpcs_ctx *ctx, const void *frames, int dtype, int64_t M, int64_t N,
                               const unsigned short *B, int64_t ldb, int L, float *Y) {
    Phase phase_(ctx, "proj_pixels");
    if (L % 16 || L <= 0) return fail(ctx, XPCS_EINVAL, "internal: L must be a positive multiple of 16");
    if (ldb % 32) return fail(ctx, XPCS_EINVAL, "internal: sketch row stride must be a multiple of 32");
    const int ncb_total = L / 16;
    // Column groups of at most 12 blocks (grid.y); all groups have the same size.
    int ngroups = (ncb_total + 11) / 12;
    while (ncb_total % ngroups) ++ngroups;
    const int ncb = ncb_total / ngroups;
    const size_t esz = dtype == XPCS_U8 ? 1 : 2;
    const bool vec4 = (M % 4 == 0) && ((uintptr_t)frames % (4 * esz) == 0);
    const bool vec2 = (M % 2 == 0) && ((uintptr_t)frames % (2 * esz) == 0);
    int rb = 0;
    dim3 g(1, (unsigned)ngroups);
    bool ok = dtype == XPCS_U8
                  ? dispatch_pp<uint8_t>(ncb, rb, ngroups, g, ctx->stream, frames, M, N, B, ldb, Y, vec4, vec2)
                  : dispatch_pp<uint16_t>(ncb, rb, ngroups, g, ctx->stream, frames, M, N, B, ldb, Y, vec4, vec2);
    if (!ok) return fail(ctx, XPCS_EUNSUPPORTED, "too many sketch columns for proj_pixels");
    XPCS_LAUNCH_CHECK(ctx, "proj_pixels");
    return XPCS_OK;
}

FrameProj plan_proj_frames(int64_t M, int64_t N, int L, int n_ind) {
    FrameProj p;
    const int nib = (n_ind + 15) / 16;
    p.ncols = L + 16 * nib;
    const int rb = pf_rb(L / 16, nib);
    const int64_t fbf = (int64_t)rb * 64;
    const int64_t nfb = (N + fbf - 1) / fbf;
    int64_t want = (2048 + nfb - 1) / nfb;                 // blocks ~ 2048
    if (want < 8) want = 8;
    int64_t chunk = (M + want - 1) / want;
    chunk = (chunk + 31) / 32 * 32;
    if (chunk < 256) chunk = 256;
    int64_t nch = (M + chunk - 1) / chunk;
    nch = (nch + 7) / 8 * 8;
    p.nchunks = nch;
    p.chunk = chunk;
    return p;
}

xpcs_status launch_proj_frames(xpcs_ctx *ctx, const void *frames, int dtype, int64_t M, int64_t N,
                               const unsigned short *q_hi, const unsigned short *q_lo, int64_t ldq, int L,
                               const int32_t *labels, int n_ind, const FrameProj &plan, float *part) {
    Phase phase_(ctx, "proj_frames");
    if (L % 16 || L <= 0) return fail(ctx, XPCS_EINVAL, "internal: L must be a positive multiple of 16");
    const int ncb = L / 16, nib = (n_ind + 15) / 16;
    if (nib > 4) return fail(ctx, XPCS_EUNSUPPORTED, "more than 64 ROIs in the fused ROI sums");
    const int rb = pf_rb(ncb, nib);
    const int64_t fbf = (int64_t)rb * 64;
    const int nfb = (int)((N + fbf - 1) / fbf);
    const int64_t nblocks = (int64_t)nfb * plan.nchunks;
    if (nblocks > 2147483647LL) return fail(ctx, XPCS_EUNSUPPORTED, "projection grid too large");
    const size_t esz = dtype == XPCS_U8 ? 1 : 2;
    const bool vec = (M % 8 == 0) && ((uintptr_t)frames % (8 * esz) == 0);
    bool ok;
    if (q_lo) {
        ok = dtype == XPCS_U8
                 ? dispatch_pf<uint8_t, true>(ncb, nib, (int)nblocks, ctx->stream, frames, M, N, q_hi, q_lo, ldq,
                                              labels, plan.chunk, nfb, plan.ncols, part, vec)
                 : dispatch_pf<uint16_t, true>(ncb, nib, (int)nblocks, ctx->stream, frames, M, N, q_hi, q_lo, ldq,
                                               labels, plan.chunk, nfb, plan.ncols, part, vec);
    } else {
        ok = dtype == XPCS_U8
                 ? dispatch_pf<uint8_t, false>(ncb, nib, (int)nblocks, ctx->stream, frames, M, N, q_hi, q_lo, ldq,
                                               labels, plan.chunk, nfb, plan.ncols, part, vec)
                 : dispatch_pf<uint16_t, false>(ncb, nib, (int)nblocks, ctx->stream, frames, M, N, q_hi, q_lo,
                                                ldq, labels, plan.chunk, nfb, plan.ncols, part, vec);
    }
    if (!ok) return fail(ctx, XPCS_EUNSUPPORTED, "too many basis columns for proj_frames");
    XPCS_LAUNCH_CHECK(ctx, "proj_frames");
    return XPCS_OK;
}

xpcs_status launch_proj_frames_reduce(xpcs_ctx *ctx, const float *part, const FrameProj &plan, int64_t N,
                                      int L, int n_ind, double *Z, int64_t ldz, int64_t *S) {
    Phase phase_(ctx, "proj_frames_reduce");
    int64_t total = N * plan.ncols;
    int grid = (int)((total + 255) / 256);
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(proj_frames_reduce_kernel, dim3(grid), dim3(256), 0, ctx->stream, part, plan.nchunks, N,
                       plan.ncols, L, n_ind, Z, ldz, S);
    XPCS_LAUNCH_CHECK(ctx, "proj_frames_reduce");
    return XPCS_OK;
}

}  // namespace xpcs
