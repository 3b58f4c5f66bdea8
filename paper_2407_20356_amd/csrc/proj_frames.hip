// Frame-space products X^T Q (Sec. 2.1): planning, launch and the fixed-order
// reduction of the per-chunk partial sums.
#include "proj_frames_dma.hpp"

namespace xpcs {
namespace {

// Z[j][t] (or the exact ROI sum of an indicator column) = sum over pixel chunks c
// of part[c][t][j]: a wave takes 64 consecutive outputs and the chunks c = wave
// (mod 4); the four wave sums are added in a fixed order.
__global__ __launch_bounds__(256) void proj_frames_reduce_kernel(const float *__restrict__ part, int64_t nch,
                                                                 int64_t N, int ncols, int L, int n_ind,
                                                                 double *__restrict__ Z, int64_t ldz,
                                                                 int64_t *__restrict__ S) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t total = N * ncols;
    const int64_t idx = (int64_t)blockIdx.x * 64 + lane;
    double s = 0.0;
    if (idx < total)
        for (int64_t c = wv; c < nch; c += 4) s += (double)part[c * total + idx];
    red[wv][lane] = s;
    __syncthreads();
    if (wv != 0 || idx >= total) return;
    s = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
    const int64_t t = idx / ncols;
    const int j = (int)(idx % ncols);
    if (j < L)
        Z[(int64_t)j * ldz + t] = s;
    else if (S && j - L < n_ind)
        S[(int64_t)(j - L) * N + t] = (int64_t)__builtin_rint(s);
}

// ind[r][p] = bf16(1) where labels[p] == r, else 0, for r < nrows and p < ldq
// (zero past M): the indicator rows of the direct-to-LDS frame pass.
__global__ __launch_bounds__(256) void indicator_rows_kernel(const int32_t *__restrict__ labels, int64_t M,
                                                             int64_t ldq, int nrows, unsigned short *__restrict__ ind) {
    const int64_t p8 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 8;
    if (p8 >= ldq) return;
    int lab[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) lab[e] = p8 + e < M ? labels[p8 + e] : -1;
    for (int r = 0; r < nrows; ++r) {
        i32x4 w;
#pragma unroll
        for (int d = 0; d < 4; ++d)
            w[d] = (int)((lab[2 * d] == r ? (unsigned)proj::kBfOne : 0u) |
                         ((lab[2 * d + 1] == r ? (unsigned)proj::kBfOne : 0u) << 16));
        *reinterpret_cast<i32x4 *>(ind + (int64_t)r * ldq + p8) = w;
    }
}

}  // namespace

using proj::pf_rb;

namespace proj {
bool dispatch_pf_u8_lo_plain(int ncb, int nblocks, hipStream_t st, const void *X, int64_t M, int64_t N,
                             const unsigned short *qh, const unsigned short *ql, int64_t ldq, int64_t chunk, int nfb,
                             int ncols, float *part, bool vec);
bool dispatch_pf_u16_lo_plain(int ncb, int nblocks, hipStream_t st, const void *X, int64_t M, int64_t N,
                              const unsigned short *qh, const unsigned short *ql, int64_t ldq, int64_t chunk, int nfb,
                              int ncols, float *part, bool vec);
}  // namespace proj

namespace {
// A residual-term pass over uint8 counts with more operand fragments per K step
// than this runs as several launches over groups of column blocks (the counts are
// read once per launch, and a uint8 pass is bound by the MFMA and LDS work per
// count, not by its bytes): measured at 1024 x 1024 px x 20,000 frames, k = 128,
// the two launches take 28.9 ms where the single wide one took 31.7 ms.  uint16
// passes stay single (their count bytes dominate).
constexpr int kMaxFragsPerLaunch = 13;
static_assert(kMaxFragsPerLaunch == proj::kDmaMaxBlocks, "column groups of both frame-pass kernels");
// Fewest frames for the direct-to-LDS frame pass.
constexpr int64_t kDmaMinFrames = 1024;
}  // namespace

FrameProj plan_proj_frames(int64_t M, int64_t N, int L, int n_ind, bool lo) {
    FrameProj p;
    const int nib = (n_ind + 15) / 16;
    p.ncols = L + 16 * nib;
    const int rb = pf_rb(L / 16, nib, lo);
    const int64_t fbf = (int64_t)rb * 64;
    const int64_t nfb = (N + fbf - 1) / fbf;
    int64_t want = (2048 + nfb - 1) / nfb;                 // blocks ~ 2048
    if (want < 8) want = 8;
    // few frames (an online push): at most 256 pixel chunks, so that the partial
    // sums stay small next to the counts and their reduction stays short
    if (want > 256) want = 256;
    int64_t chunk = (M + want - 1) / want;
    chunk = (chunk + 63) / 64 * 64;                        // a multiple of either K step
    if (chunk < 256) chunk = 256;
    int64_t nch = (M + chunk - 1) / chunk;
    nch = (nch + 7) / 8 * 8;
    p.nchunks = nch;
    p.chunk = chunk;
    p.frames_per_block = (int)fbf;
    return p;
}

xpcs_status launch_proj_frames(xpcs_ctx *ctx, const void *frames, int dtype, int64_t M, int64_t N,
                               const unsigned short *q_hi, const unsigned short *q_lo, int64_t ldq, int L,
                               const int32_t *labels, int n_ind, const FrameProj &plan, float *part) {
    Phase phase_(ctx, "proj_frames");
    if (L % 16 || L <= 0) return fail(ctx, XPCS_EINVAL, "internal: L must be a positive multiple of 16");
    if (ldq % 64 || ldq < M)
        return fail(ctx, XPCS_EINVAL, "internal: basis row stride must cover M in steps of 64");
    const int ncb = L / 16, nib = (n_ind + 15) / 16;
    if (nib > 4) return fail(ctx, XPCS_EUNSUPPORTED, "more than 64 ROIs in the fused ROI sums");
    const bool lo = q_lo != nullptr;
    const size_t esz = dtype == XPCS_U8 ? 1 : 2;
    const bool vec = (M % 8 == 0) && ((uintptr_t)frames % (8 * esz) == 0) &&
                     (nib == 0 || (uintptr_t)labels % 16 == 0);
    const int frags = ncb * (lo ? 2 : 1) + nib;
    // Direct-to-LDS loads need 16-byte aligned rows of counts and basis; passes over
    // few frames (an online push) keep the register-staged kernel, which needs no
    // indicator matrix.
    const bool dma = N >= kDmaMinFrames && (uintptr_t)frames % 16 == 0 && ((size_t)M * esz) % 16 == 0 &&
                     (uintptr_t)q_hi % 16 == 0 && (!lo || (uintptr_t)q_lo % 16 == 0);
    const unsigned short *ind = nullptr;
    if (dma && nib > 0) {
        xpcs_status st;
        auto *buf = static_cast<unsigned short *>(scratch_get(ctx, (size_t)16 * nib * ldq * 2, &st));
        if (!buf) return st;
        hipLaunchKernelGGL(indicator_rows_kernel, dim3((unsigned)((ldq / 8 + 255) / 256)), dim3(256), 0, ctx->stream,
                           labels, M, ldq, 16 * nib, buf);
        XPCS_LAUNCH_CHECK(ctx, "indicator_rows");
        ind = buf;
    }
    // the direct-to-LDS kernel picks its own frames per block; the chunks are the plan's
    auto run = [&](int ncb_g, int nib_g, const unsigned short *qh, const unsigned short *ql,
                   const unsigned short *ind_g, float *pg) {
        if (dtype == XPCS_U8)
            return proj::dispatch_pf_dma_u8(ncb_g, nib_g, lo, plan.nchunks, ctx->stream, frames, M, N, qh, ql, ind_g,
                                            ldq, plan.chunk, plan.ncols, pg);
        return proj::dispatch_pf_dma_u16(ncb_g, nib_g, lo, plan.nchunks, ctx->stream, frames, M, N, qh, ql, ind_g,
                                         ldq, plan.chunk, plan.ncols, pg);
    };
    if (ncb <= 12 && (!lo || frags <= kMaxFragsPerLaunch || (dtype != XPCS_U8 && !dma))) {
        const int rb = pf_rb(ncb, nib, lo);
        if (rb * 64 != plan.frames_per_block)
            return fail(ctx, XPCS_EINVAL, "internal: projection plan made for another variant");
        const int64_t fbf = (int64_t)rb * 64;
        const int nfb = (int)((N + fbf - 1) / fbf);
        const int64_t nblocks = (int64_t)nfb * plan.nchunks;
        if (nblocks > 2147483647LL) return fail(ctx, XPCS_EUNSUPPORTED, "projection grid too large");
        const bool ok =
            dma ? run(ncb, nib, q_hi, q_lo, ind, part)
            : dtype == XPCS_U8
                ? proj::dispatch_pf_u8(ncb, nib, lo, (int)nblocks, ctx->stream, frames, M, N, q_hi, q_lo, ldq, labels,
                                       plan.chunk, nfb, plan.ncols, part, vec)
                : proj::dispatch_pf_u16(ncb, nib, lo, (int)nblocks, ctx->stream, frames, M, N, q_hi, q_lo, ldq,
                                        labels, plan.chunk, nfb, plan.ncols, part, vec);
        if (!ok) return fail(ctx, XPCS_EUNSUPPORTED, "unsupported basis width or ROI count for proj_frames");
        XPCS_LAUNCH_CHECK(ctx, "proj_frames");
        return XPCS_OK;
    }
    // Several launches over groups of column blocks, each writing its own columns of
    // the partial sums; the indicator columns ride with the last group.  Up to 12
    // blocks the residual-term uint8 pass keeps its measured split (frags / 13 groups
    // of balanced size); otherwise the last group takes at most 6 blocks and as many
    // as fit 13 operand fragments with the indicators, the rest groups of at most 6
    // (12 without the residual term).
    int sizes[64], groups = 0;
    if (lo && ncb <= 12) {
        groups = (frags + kMaxFragsPerLaunch - 1) / kMaxFragsPerLaunch;
        int c = 0;
        for (int g = 0; g < groups; ++g) {
            const int last = g == groups - 1;
            sizes[g] = last ? ncb - c : (ncb - c + (groups - g) - 1) / (groups - g);
            c += sizes[g];
        }
        if (sizes[groups - 1] * 2 + nib > kMaxFragsPerLaunch) groups = 0;     // use the general split
    }
    if (groups == 0) {
        const int per = lo ? 6 : 12;
        int last = lo ? (kMaxFragsPerLaunch - nib) / 2 : per;
        if (last > per) last = per;
        if (last > ncb) last = ncb;
        if (last < 1) return fail(ctx, XPCS_EUNSUPPORTED, "unsupported basis width or ROI count for proj_frames");
        const int rest = ncb - last, nplain = (rest + per - 1) / per;
        if (nplain + 1 > 64) return fail(ctx, XPCS_EUNSUPPORTED, "basis too wide for proj_frames");
        for (int g = 0; g < nplain; ++g) sizes[g] = rest / nplain + (g < rest % nplain ? 1 : 0);
        sizes[nplain] = last;
        groups = nplain + 1;
    }
    int c0 = 0;
    for (int g = 0; g < groups; ++g) {
        const int last = g == groups - 1;
        const int ncb_g = sizes[g];
        const int nib_g = last ? nib : 0;
        const int rb = pf_rb(ncb_g, nib_g, lo);
        const int64_t fbf = (int64_t)rb * 64;
        const int nfb = (int)((N + fbf - 1) / fbf);
        const int64_t nblocks = (int64_t)nfb * plan.nchunks;
        if (nblocks > 2147483647LL) return fail(ctx, XPCS_EUNSUPPORTED, "projection grid too large");
        const unsigned short *qh = q_hi + (int64_t)16 * c0 * ldq;
        const unsigned short *ql = lo ? q_lo + (int64_t)16 * c0 * ldq : nullptr;
        float *pg = part + 16 * c0;
        bool ok;
        if (dma)
            ok = run(ncb_g, nib_g, qh, ql, last ? ind : nullptr, pg);
        else if (nib_g || !lo)
            ok = dtype == XPCS_U8
                     ? proj::dispatch_pf_u8(ncb_g, nib_g, lo, (int)nblocks, ctx->stream, frames, M, N, qh, ql, ldq,
                                            labels, plan.chunk, nfb, plan.ncols, pg, vec)
                     : proj::dispatch_pf_u16(ncb_g, nib_g, lo, (int)nblocks, ctx->stream, frames, M, N, qh, ql, ldq,
                                             labels, plan.chunk, nfb, plan.ncols, pg, vec);
        else
            ok = dtype == XPCS_U8
                     ? proj::dispatch_pf_u8_lo_plain(ncb_g, (int)nblocks, ctx->stream, frames, M, N, qh, ql, ldq,
                                                     plan.chunk, nfb, plan.ncols, pg, vec)
                     : proj::dispatch_pf_u16_lo_plain(ncb_g, (int)nblocks, ctx->stream, frames, M, N, qh, ql, ldq,
                                                      plan.chunk, nfb, plan.ncols, pg, vec);
        if (!ok) return fail(ctx, XPCS_EUNSUPPORTED, "unsupported basis width or ROI count for proj_frames");
        XPCS_LAUNCH_CHECK(ctx, "proj_frames");
        c0 += ncb_g;
    }
    return XPCS_OK;
}

xpcs_status launch_proj_frames_reduce(xpcs_ctx *ctx, const float *part, const FrameProj &plan, int64_t N,
                                      int L, int n_ind, double *Z, int64_t ldz, int64_t *S) {
    Phase phase_(ctx, "proj_frames_reduce");
    const int64_t total = N * plan.ncols;
    const int64_t grid = (total + 63) / 64;
    if (grid > 2147483647LL) return fail(ctx, XPCS_EUNSUPPORTED, "projection reduction too large");
    hipLaunchKernelGGL(proj_frames_reduce_kernel, dim3((unsigned)grid), dim3(256), 0, ctx->stream, part,
                       plan.nchunks, N, plan.ncols, L, n_ind, Z, ldz, S);
    XPCS_LAUNCH_CHECK(ctx, "proj_frames_reduce");
    return XPCS_OK;
}

}  // namespace xpcs
