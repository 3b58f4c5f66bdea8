// FP8 (OCP e4m3) versions of the power pass over the counts (X^T Q and X Z of
// Sec. 2.1; the sketch X Omega is exact on the int8 MFMA in every mode): these only
// choose the span of the basis, so their B operands may be rounded to e4m3; the
// encoding pass W = X^T U keeps the split-bf16 basis.  The counts stay exact:
// a count c < 256 (u8 frames) enters as two nibble planes, c & 15 and
// (c >> 4) * 16, integers with at most 4 significant bits, which e4m3 holds
// exactly; plane 1 runs only in the K steps of a wave where a count reaches 16.
// The MFMA is v_mfma_f32_16x16x32_fp8_fp8: the same lane layout as the bf16
// 16x16x32 (lane l: row l % 16, K group l / 16 of 8 values), 8 bytes per operand.
//
// B operands are fp8 rows of an orthonormal basis
// scaled by 256 (entries of a unit column are at most 1, so the scale keeps them
// in e4m3's normal range and below its largest finite value 448).  The scale is
// left in the products: the passes feed orthonormalisations, which remove it.
#include "proj_frames.hpp"

namespace xpcs {
namespace {

using namespace proj;

constexpr int kF8Pitch = 40;          // LDS row pitch (bytes) of a 32-wide K step: conflict-free 8-byte reads
constexpr int kF8PitchF = 72;         // the same for the frame-space pass's 64-wide K step

__device__ __forceinline__ unsigned f8_pack4(float a, float b, float c, float d) {
    const int p = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    return (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(c, d, p, true);
}
// Eight counts, one per byte of (lo, hi), as e4m3: plane 0 (c & 15) or plane 1 ((c >> 4) * 16).
__device__ __forceinline__ long f8_plane0(unsigned lo, unsigned hi) {
    lo &= 0x0f0f0f0fu;
    hi &= 0x0f0f0f0fu;
    const unsigned a = f8_pack4((float)(lo & 0xffu), (float)((lo >> 8) & 0xffu), (float)((lo >> 16) & 0xffu),
                                (float)(lo >> 24));
    const unsigned b = f8_pack4((float)(hi & 0xffu), (float)((hi >> 8) & 0xffu), (float)((hi >> 16) & 0xffu),
                                (float)(hi >> 24));
    return (long)(((unsigned long long)b << 32) | a);
}
__device__ __forceinline__ long f8_plane1(unsigned lo, unsigned hi) {
    opaque(lo);
    opaque(hi);
    lo = (lo >> 4) & 0x0f0f0f0fu;
    hi = (hi >> 4) & 0x0f0f0f0fu;
    const unsigned a = f8_pack4((float)(lo & 0xffu) * 16.f, (float)((lo >> 8) & 0xffu) * 16.f,
                                (float)((lo >> 16) & 0xffu) * 16.f, (float)(lo >> 24) * 16.f);
    const unsigned b = f8_pack4((float)(hi & 0xffu) * 16.f, (float)((hi >> 8) & 0xffu) * 16.f,
                                (float)((hi >> 16) & 0xffu) * 16.f, (float)(hi >> 24) * 16.f);
    return (long)(((unsigned long long)b << 32) | a);
}
__device__ __forceinline__ f32x4 mfma_f8(long a, long b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
}

// One K step (rows j < 16 * NCB of an fp8 row-major operand, KB bytes of K) held in
// registers between its global load and its LDS store; every thread issues the
// same loads (surplus threads repeat the last unit).
template <int NCB, int KB, int PITCH>
struct StageF8 {
    static constexpr int kParts = KB / 16;
    static constexpr int kUnits = NCB * 16 * kParts;
    static constexpr int kPer = (kUnits + 255) / 256;
    i32x4 r[kPer];
    __device__ __forceinline__ void load(const uint8_t *__restrict__ src, int64_t ld, int64_t k0) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            int u = threadIdx.x + 256 * i;
            if (kUnits % 256) u = u < kUnits ? u : kUnits - 1;
            r[i] = *reinterpret_cast<const i32x4 *>(src + (int64_t)(u / kParts) * ld + k0 + 16 * (u % kParts));
        }
    }
    __device__ __forceinline__ void store(uint8_t *dst) const {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int u = threadIdx.x + 256 * i;
            if (u < kUnits) {
                // 8-byte halves: PITCH keeps rows 8-byte aligned, not always 16
                int2 *d = reinterpret_cast<int2 *>(dst + (u / kParts) * PITCH + 16 * (u % kParts));
                d[0] = int2{r[i][0], r[i][1]};
                d[1] = int2{r[i][2], r[i][3]};
            }
        }
    }
};

// ---------------------------------------------------------------- pixel-space pass
// Y[j][p] = sum_t X[t][p] B[j][t]: as proj_pixels_kernel (a wave owns 16 RB pixels,
// pixel = base + RB row + s; a lane loads RB adjacent pixels of each of its 8 frames),
// with K steps of 32 frames and fp8 operands.
template <int RB, int NCB, bool VEC>
__global__ __launch_bounds__(256) void proj_pixels_f8_kernel(const uint8_t *__restrict__ X, int64_t M, int64_t N,
                                                             const uint8_t *__restrict__ B, int64_t ldb,
                                                             float *__restrict__ Y) {
    static_assert(RB == 4, "four pixels per lane and frame");
    __shared__ __align__(16) uint8_t sb[2][NCB * 16 * kF8Pitch];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int jg = blockIdx.y * 16 * NCB;
    const int64_t pb = ((int64_t)blockIdx.x * 4 + wv) * (16 * RB);
    const int64_t pl = pb + RB * lr;
    const int nvalid = pl >= M ? 0 : (M - pl >= RB ? RB : (int)(M - pl));
    const int64_t plc = pl < M ? pl : 0;
    const uint8_t *Bg = B + (int64_t)jg * ldb;
    f32x4 acc[RB][NCB];
#pragma unroll
    for (int s = 0; s < RB; ++s)
#pragma unroll
        for (int c = 0; c < NCB; ++c) acc[s][c] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const int nsteps = (int)((N + 31) / 32);
    // x[e]: pixels pl .. pl + 3 of frame tk + 8 lg + e
    auto load_step = [&](int64_t tk, unsigned (&x)[8]) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t t = tk + 8 * lg + e;
            if constexpr (VEC) {
                const int64_t tc = t < N ? t : N - 1;
                x[e] = *reinterpret_cast<const unsigned *>(X + tc * M + plc);
            } else {
                unsigned v = 0;
                if (t < N)
                    for (int s = 0; s < nvalid; ++s) v |= (unsigned)X[t * M + pl + s] << (8 * s);
                x[e] = v;
            }
        }
    };
    // the 8 frames' counts of pixel s as two words (frames 0-3, 4-7), one count per byte
    auto gather = [&](const unsigned (&x)[8], int s, unsigned &lo, unsigned &hi) {
        lo = ((x[0] >> (8 * s)) & 0xffu) | (((x[1] >> (8 * s)) & 0xffu) << 8) | (((x[2] >> (8 * s)) & 0xffu) << 16) |
             (((x[3] >> (8 * s)) & 0xffu) << 24);
        hi = ((x[4] >> (8 * s)) & 0xffu) | (((x[5] >> (8 * s)) & 0xffu) << 8) | (((x[6] >> (8 * s)) & 0xffu) << 16) |
             (((x[7] >> (8 * s)) & 0xffu) << 24);
    };
    auto mma = [&](const long (&a)[RB], const uint8_t *cur) {
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
            const long b = *reinterpret_cast<const long *>(cur + (16 * c + lr) * kF8Pitch + 8 * lg);
#pragma unroll
            for (int s = 0; s < RB; ++s) acc[s][c] = mfma_f8(a[s], b, acc[s][c]);
        }
    };
    auto multiply = [&](const unsigned (&xc)[8], const uint8_t *cur) {
        long a[RB];
        bool big = false;
#pragma unroll
        for (int s = 0; s < RB; ++s) {
            unsigned lo, hi;
            gather(xc, s, lo, hi);
            a[s] = f8_plane0(lo, hi);
            big |= ((lo | hi) & 0xf0f0f0f0u) != 0;
        }
        mma(a, cur);
        if (__ballot(big)) {
#pragma unroll
            for (int s = 0; s < RB; ++s) {
                unsigned lo, hi;
                gather(xc, s, lo, hi);
                a[s] = f8_plane1(lo, hi);
            }
            mma(a, cur);
        }
    };
    StageF8<NCB, 32, kF8Pitch> st[2];
    unsigned xr[2][8];
    st[0].load(Bg, ldb, 0);
    load_step(0, xr[0]);
    st[0].store(sb[0]);
    __syncthreads();
    for (int step0 = 0; step0 < nsteps; step0 += 2) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int step = step0 + j;
            if (step >= nsteps) break;
            const int sn = step + 1 < nsteps ? step + 1 : step;
            st[j ^ 1].load(Bg, ldb, (int64_t)sn * 32);
            load_step((int64_t)sn * 32, xr[j ^ 1]);
            multiply(xr[j], sb[step & 1]);
            if (step + 1 < nsteps) st[j ^ 1].store(sb[(step + 1) & 1]);
            __syncthreads();
        }
    }
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
        float *yrow = Y + (int64_t)(jg + 16 * c + lr) * M;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int s = 0; s < RB; ++s) {
                const int64_t p = pb + RB * (4 * lg + i) + s;
                if (p < M) yrow[p] = acc[s][c][i];
            }
    }
}

// ---------------------------------------------------------------- frame-space pass
// part[c][t][j] = sum_{p in chunk c} X[t][p] Q[j][p] (the power pass, no residual
// term and no indicator columns): as proj_frames_kernel with K steps of 64 pixels
// (lane: pixels 16 lg + 8 kk .. + 8 of its frame row) and fp8 operands.
template <int RB, int NCB, bool VEC>
__global__ __launch_bounds__(256) void proj_frames_f8_kernel(const uint8_t *__restrict__ X, int64_t M, int64_t N,
                                                             const uint8_t *__restrict__ q8, int64_t ldq,
                                                             int64_t chunk, int nfb, int ncols,
                                                             float *__restrict__ part) {
    constexpr int KS = 64, kKK = 2;
    constexpr int FB = RB * 16 * 4;
    __shared__ __align__(16) uint8_t sq[2][NCB * 16 * kF8PitchF];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int bid = blockIdx.x, xcd = bid & 7, sl = bid >> 3;
    const int ch = xcd + 8 * (sl / nfb), fb = sl % nfb;
    const int64_t p_begin = (int64_t)ch * chunk;
    const int64_t p_end = p_begin + chunk < M ? p_begin + chunk : M;
    const int64_t tb = (int64_t)fb * FB + (int64_t)wv * RB * 16;
    f32x4 acc[RB][NCB];
#pragma unroll
    for (int s = 0; s < RB; ++s)
#pragma unroll
        for (int c = 0; c < NCB; ++c) acc[s][c] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const uint8_t *xrow[RB];
    bool rok[RB];
#pragma unroll
    for (int s = 0; s < RB; ++s) {
        const int64_t t = tb + 16 * s + lr;
        rok[s] = t < N;
        xrow[s] = X + (t < N ? t : N - 1) * M;
    }
    const int nsteps = p_end > p_begin ? (int)((p_end - p_begin + KS - 1) / KS) : 0;
    auto load_x = [&](int64_t p0, int2 (&x)[RB][kKK]) {
#pragma unroll
        for (int kk = 0; kk < kKK; ++kk) {
            const int64_t pl = p0 + 16 * lg + 8 * kk;
            if constexpr (VEC) {
                const int64_t pc = pl < p_end ? pl : p_begin;
#pragma unroll
                for (int s = 0; s < RB; ++s) x[s][kk] = *reinterpret_cast<const int2 *>(xrow[s] + pc);
            } else {
                const int nv = pl >= p_end ? 0 : (p_end - pl >= 8 ? 8 : (int)(p_end - pl));
#pragma unroll
                for (int s = 0; s < RB; ++s) {
                    unsigned v[2] = {0u, 0u};
                    if (rok[s])
                        for (int e = 0; e < nv; ++e) v[e >> 2] |= (unsigned)xrow[s][pl + e] << (8 * (e & 3));
                    x[s][kk] = int2{(int)v[0], (int)v[1]};
                }
            }
        }
    };
    auto mma = [&](const long (&a)[RB], const uint8_t *cur, int kk) {
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
            const long b = *reinterpret_cast<const long *>(cur + (16 * c + lr) * kF8PitchF + 16 * lg + 8 * kk);
#pragma unroll
            for (int s = 0; s < RB; ++s) acc[s][c] = mfma_f8(a[s], b, acc[s][c]);
        }
    };
    auto multiply = [&](const int2 (&xc)[RB][kKK], const uint8_t *cur) {
        bool big = false;
#pragma unroll
        for (int kk = 0; kk < kKK; ++kk) {
            long a[RB];
#pragma unroll
            for (int s = 0; s < RB; ++s) {
                a[s] = f8_plane0((unsigned)xc[s][kk].x, (unsigned)xc[s][kk].y);
                big |= (((unsigned)xc[s][kk].x | (unsigned)xc[s][kk].y) & 0xf0f0f0f0u) != 0;
            }
            mma(a, cur, kk);
        }
        if (__ballot(big)) {
#pragma unroll
            for (int kk = 0; kk < kKK; ++kk) {
                long a[RB];
#pragma unroll
                for (int s = 0; s < RB; ++s) a[s] = f8_plane1((unsigned)xc[s][kk].x, (unsigned)xc[s][kk].y);
                mma(a, cur, kk);
            }
        }
    };
    if (nsteps > 0) {
        StageF8<NCB, KS, kF8PitchF> sr;
        int2 xr[2][RB][kKK];
        sr.load(q8, ldq, p_begin);
        load_x(p_begin, xr[0]);
        sr.store(sq[0]);
        __syncthreads();
        for (int step0 = 0; step0 < nsteps; step0 += 2) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int step = step0 + j;
                if (step >= nsteps) break;
                const int64_t pn = p_begin + KS * (int64_t)(step + 1 < nsteps ? step + 1 : step);
                sr.load(q8, ldq, pn);
                load_x(pn, xr[j ^ 1]);
                multiply(xr[j], sq[step & 1]);
                if (step + 1 < nsteps) sr.store(sq[(step + 1) & 1]);
                __syncthreads();
            }
        }
    }
    float *pdst = part + (int64_t)ch * N * ncols;
#pragma unroll
    for (int s = 0; s < RB; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t t = tb + 16 * s + 4 * lg + i;
            if (t < N) {
#pragma unroll
                for (int c = 0; c < NCB; ++c) pdst[t * ncols + 16 * c + lr] = acc[s][c][i];
            }
        }
}

template <int NCB>
void launch_pp_f8(dim3 grid, hipStream_t st, const uint8_t *X, int64_t M, int64_t N, const uint8_t *B,
                  int64_t ldb, float *Y, bool vec) {
    if (vec)
        hipLaunchKernelGGL((proj_pixels_f8_kernel<4, NCB, true>), grid, dim3(256), 0, st, X, M, N, B, ldb, Y);
    else
        hipLaunchKernelGGL((proj_pixels_f8_kernel<4, NCB, false>), grid, dim3(256), 0, st, X, M, N, B, ldb, Y);
}

template <int RB, int NCB>
void launch_pf_f8(int nblocks, hipStream_t st, const uint8_t *X, int64_t M, int64_t N, const uint8_t *q8,
                  int64_t ldq, int64_t chunk, int nfb, int ncols, float *part, bool vec) {
    if (vec)
        hipLaunchKernelGGL((proj_frames_f8_kernel<RB, NCB, true>), dim3(nblocks), dim3(256), 0, st, X, M, N, q8, ldq,
                           chunk, nfb, ncols, part);
    else
        hipLaunchKernelGGL((proj_frames_f8_kernel<RB, NCB, false>), dim3(nblocks), dim3(256), 0, st, X, M, N, q8,
                           ldq, chunk, nfb, ncols, part);
}

}  // namespace

xpcs_status launch_proj_pixels_f8(xpcs_ctx *ctx, const uint8_t *frames, int64_t M, int64_t N, const uint8_t *B,
                                  int64_t ldb, int L, float *Y) {
    Phase phase_(ctx, "proj_pixels");
    if (L % 16 || L <= 0) return fail(ctx, XPCS_EINVAL, "internal: L must be a positive multiple of 16");
    if (ldb % 32 || ldb < N) return fail(ctx, XPCS_EINVAL, "internal: sketch row stride must cover N in steps of 32");
    const int ncb_total = L / 16;
    // column groups of at most 6 blocks (grid.y of one launch per group size): the
    // sizes differ by at most one, the larger groups first
    const int ngroups = (ncb_total + 5) / 6;
    const int sz = ncb_total / ngroups, nbig = ncb_total % ngroups;
    const bool vec = (M % 4 == 0) && ((uintptr_t)frames % 4 == 0);
    for (int part = 0; part < 2; ++part) {
        const int ncb = part == 0 ? sz + 1 : sz, gy = part == 0 ? nbig : ngroups - nbig;
        if (gy == 0) continue;
        const int c0 = part == 0 ? 0 : nbig * (sz + 1);
        const uint8_t *Bp = B + (int64_t)16 * c0 * ldb;
        float *Yp = Y + (int64_t)16 * c0 * M;
        dim3 grid((unsigned)((M + 255) / 256), (unsigned)gy);
        switch (ncb) {
            case 1: launch_pp_f8<1>(grid, ctx->stream, frames, M, N, Bp, ldb, Yp, vec); break;
            case 2: launch_pp_f8<2>(grid, ctx->stream, frames, M, N, Bp, ldb, Yp, vec); break;
            case 3: launch_pp_f8<3>(grid, ctx->stream, frames, M, N, Bp, ldb, Yp, vec); break;
            case 4: launch_pp_f8<4>(grid, ctx->stream, frames, M, N, Bp, ldb, Yp, vec); break;
            case 5: launch_pp_f8<5>(grid, ctx->stream, frames, M, N, Bp, ldb, Yp, vec); break;
            case 6: launch_pp_f8<6>(grid, ctx->stream, frames, M, N, Bp, ldb, Yp, vec); break;
            default: return fail(ctx, XPCS_EUNSUPPORTED, "too many sketch columns for the fp8 pass");
        }
        XPCS_LAUNCH_CHECK(ctx, "proj_pixels_f8");
    }
    return XPCS_OK;
}

xpcs_status launch_proj_frames_f8(xpcs_ctx *ctx, const uint8_t *frames, int64_t M, int64_t N, const uint8_t *q8,
                                  int64_t ldq, int L, const FrameProj &plan, float *part) {
    Phase phase_(ctx, "proj_frames");
    if (L % 16 || L <= 0) return fail(ctx, XPCS_EINVAL, "internal: L must be a positive multiple of 16");
    if (ldq % 64 || ldq < M) return fail(ctx, XPCS_EINVAL, "internal: basis row stride must cover M in steps of 64");
    const int ncb_total = L / 16;
    if (plan.ncols != L) return fail(ctx, XPCS_EINVAL, "internal: projection plan made for another variant");
    if (ncb_total <= 12 && pf_rb(ncb_total, 0, false) * 64 != plan.frames_per_block)
        return fail(ctx, XPCS_EINVAL, "internal: projection plan made for another variant");
    const bool vec = (M % 8 == 0) && ((uintptr_t)frames % 8 == 0);
    // more than 12 column blocks: one launch per group of at most 12 (sizes differing by at
    // most one), each writing its own columns of the partial sums
    const int ngroups = (ncb_total + 11) / 12;
    int c0 = 0;
    for (int g = 0; g < ngroups; ++g) {
        const int ncb = ncb_total / ngroups + (g < ncb_total % ngroups ? 1 : 0);
        const int64_t fbf = (int64_t)pf_rb(ncb, 0, false) * 64;
        const int nfb = (int)((N + fbf - 1) / fbf);
        const int64_t nblocks = (int64_t)nfb * plan.nchunks;
        if (nblocks > 2147483647LL) return fail(ctx, XPCS_EUNSUPPORTED, "projection grid too large");
        const int nb = (int)nblocks;
        const uint8_t *qg = q8 + (int64_t)16 * c0 * ldq;
        float *pg = part + 16 * c0;
#define XPCS_PF8(R, C) launch_pf_f8<R, C>(nb, ctx->stream, frames, M, N, qg, ldq, plan.chunk, nfb, L, pg, vec)
        switch (ncb) {
            case 1: XPCS_PF8(4, 1); break;
            case 2: XPCS_PF8(4, 2); break;
            case 3: XPCS_PF8(4, 3); break;
            case 4: XPCS_PF8(4, 4); break;
            case 5: XPCS_PF8(4, 5); break;
            case 6: XPCS_PF8(4, 6); break;
            case 7: XPCS_PF8(4, 7); break;
            case 8: XPCS_PF8(4, 8); break;
            case 9: XPCS_PF8(2, 9); break;
            case 10: XPCS_PF8(2, 10); break;
            case 11: XPCS_PF8(2, 11); break;
            case 12: XPCS_PF8(2, 12); break;
            default: return fail(ctx, XPCS_EUNSUPPORTED, "too many basis columns for the fp8 pass");
        }
#undef XPCS_PF8
        XPCS_LAUNCH_CHECK(ctx, "proj_frames_f8");
        c0 += ncb;
    }
    return XPCS_OK;
}

}  // namespace xpcs
