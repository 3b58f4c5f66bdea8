// Operands of the compressed two-time correlation (Sec. 2.1, Eqs. 8-10 per ROI).
//
// With W = V diag(sigma) (the compressed data, Eq. 7), G_R = U_R^T U_R = L_R L_R^T
// (Cholesky, FP64),
//   C~_R[i][j] = |R| (W G_R W^T)[i][j] / (S_R[i] S_R[j]) = Z[i] . Z[j],
//   Z[t] = sqrt(|R|) (W[t] / S_R[t]) L_R.
// Z is formed in FP64 and split into bf16 hi + lo so that the tile pass can run
// three BF16 MFMA products (hi.hi + hi.lo + lo.hi) with FP32 accumulation,
// accurate to ~2^-16 relative per term; the symmetric form needs one operand.
#include "internal.hpp"

namespace xpcs {
namespace {

constexpr int kPrepFrames = 64;     // frames per block
constexpr int kPrepMaxK = 192;
constexpr int kPrepChunk = 32;      // rows of L staged at a time

// Thread (fr, cb) = (tid / 16, tid % 16) forms z for frames 4 fr .. 4 fr + 3 and
// columns cb + 16 j, j < CPT: a 4 x CPT register block, so that each pair of LDS
// reads feeds 4 * CPT / (1 + CPT / 2) FMAs.  w / S (transposed, [a][frame]) and a
// chunk of L's rows live in LDS.
template <int CPT>
__global__ __launch_bounds__(256) void lowrank_prep_kernel(
    const float *__restrict__ V, const double *__restrict__ sigma, const int64_t *__restrict__ roi_sum,
    const int64_t *__restrict__ roi_npix, const double *__restrict__ Lr, int64_t N, int k, int r0, int64_t t0,
    int64_t nw, int kp, unsigned short *__restrict__ z_hi, unsigned short *__restrict__ z_lo,
    unsigned char *__restrict__ valid) {
    extern __shared__ double sm[];
    const int kc = 16 * CPT;                          // columns covered (>= k)
    double *wT = sm;                                  // [kc][kPrepFrames]
    double *Lc = sm + (size_t)kc * kPrepFrames;       // [kPrepChunk][kc]
    const int slot = blockIdx.y, roi = r0 + slot;
    const int64_t f0 = (int64_t)blockIdx.x * kPrepFrames;
    const double sq = sqrt((double)roi_npix[roi]);
    const int64_t *Sr = roi_sum + (int64_t)roi * N;
    const double *L = Lr + (int64_t)slot * k * k;     // row-major lower factor of this ROI
    for (int idx = threadIdx.x; idx < kc * kPrepFrames; idx += 256) {
        const int a = idx / kPrepFrames, f = idx % kPrepFrames;
        const int64_t tl = f0 + f;
        double w = 0.0;
        if (tl < nw && a < k) {
            const int64_t sv = Sr[t0 + tl];
            if (sv > 0) w = (double)V[(int64_t)a * N + t0 + tl] * sigma[a] / (double)sv;
        }
        wT[idx] = w;
    }
    const int fr = threadIdx.x >> 4, cb = threadIdx.x & 15;
    double acc[4][CPT];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < CPT; ++j) acc[i][j] = 0.0;
    for (int a0 = 0; a0 < k; a0 += kPrepChunk) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < kPrepChunk * kc; idx += 256) {
            const int aa = idx / kc, b = idx % kc;
            Lc[idx] = (a0 + aa < k && b < k) ? L[(int64_t)(a0 + aa) * k + b] : 0.0;
        }
        __syncthreads();
        const int na = k - a0 < kPrepChunk ? k - a0 : kPrepChunk;
        for (int aa = 0; aa < na; ++aa) {
            const double2 x01 = *reinterpret_cast<const double2 *>(&wT[(a0 + aa) * kPrepFrames + 4 * fr]);
            const double2 x23 = *reinterpret_cast<const double2 *>(&wT[(a0 + aa) * kPrepFrames + 4 * fr + 2]);
            const double x[4] = {x01.x, x01.y, x23.x, x23.y};
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const double l = Lc[aa * kc + cb + 16 * j];
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[i][j] = fma(x[i], l, acc[i][j]);
            }
        }
    }
    const int64_t base = (int64_t)slot * nw * kp;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t tl = f0 + 4 * fr + i;
        if (tl >= nw) continue;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int b = cb + 16 * j;
            if (b < kp) {
                unsigned short zh = 0, zl = 0;
                if (b < k) {
                    const double zv = sq * acc[i][j];
                    zh = f32_to_bf16_bits((float)zv);
                    zl = f32_to_bf16_bits((float)(zv - (double)bf16_bits_to_f32(zh)));
                }
                z_hi[base + tl * kp + b] = zh;
                z_lo[base + tl * kp + b] = zl;
            }
        }
        // K padding beyond the covered columns (kp may exceed 16 * CPT)
        for (int b = kc + cb; b < kp; b += 16) {
            z_hi[base + tl * kp + b] = 0;
            z_lo[base + tl * kp + b] = 0;
        }
    }
    for (int f = threadIdx.x; f < kPrepFrames; f += 256) {
        const int64_t tl = f0 + f;
        if (tl < nw) valid[(int64_t)slot * nw + tl] = Sr[t0 + tl] > 0 ? 1 : 0;
    }
}

}  // namespace

xpcs_status launch_lowrank_prep(xpcs_ctx *ctx, const xpcs_factors *f, const double *Lr, int r0, int nr, int64_t t0,
                                int64_t nw, int kp, unsigned short *z_hi, unsigned short *z_lo,
                                unsigned char *valid) {
    Phase phase_(ctx, "lowrank_prep");
    if (f->k > kPrepMaxK) return fail(ctx, XPCS_EUNSUPPORTED, "rank above 192 in the compressed correlation");
    const int cpt = (f->k + 15) / 16;
    const size_t lds = ((size_t)16 * cpt * kPrepFrames + (size_t)kPrepChunk * 16 * cpt) * sizeof(double);
    dim3 grid((unsigned)((nw + kPrepFrames - 1) / kPrepFrames), (unsigned)nr);
#define XPCS_PREP(c)                                                                                            \
    case c:                                                                                                     \
        hipLaunchKernelGGL(lowrank_prep_kernel<c>, grid, dim3(256), lds, ctx->stream, f->V, f->sigma, f->roi_sum, \
                           f->roi_npix, Lr, f->N, f->k, r0, t0, nw, kp, z_hi, z_lo, valid);                      \
        break;
    switch (cpt) {
        XPCS_PREP(1) XPCS_PREP(2) XPCS_PREP(3) XPCS_PREP(4) XPCS_PREP(5) XPCS_PREP(6)
        XPCS_PREP(7) XPCS_PREP(8) XPCS_PREP(9) XPCS_PREP(10) XPCS_PREP(11) XPCS_PREP(12)
        default:
            return fail(ctx, XPCS_EUNSUPPORTED, "rank above 192 in the compressed correlation");
    }
#undef XPCS_PREP
    XPCS_LAUNCH_CHECK(ctx, "lowrank_prep");
    return XPCS_OK;
}

}  // namespace xpcs
