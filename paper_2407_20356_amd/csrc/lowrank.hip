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

constexpr int kPrepFrames = 32;
constexpr int kPrepMaxK = 192;
constexpr int kPrepChunk = 16;

__global__ __launch_bounds__(256) void lowrank_prep_kernel(
    const float *__restrict__ V, const double *__restrict__ sigma, const int64_t *__restrict__ roi_sum,
    const int64_t *__restrict__ roi_npix, const double *__restrict__ Lr, int64_t N, int k, int r0, int64_t t0,
    int64_t nw, int kp, unsigned short *__restrict__ z_hi, unsigned short *__restrict__ z_lo,
    unsigned char *__restrict__ valid) {
    __shared__ double wl[kPrepFrames][kPrepMaxK + kPrepChunk];
    __shared__ double gc[kPrepChunk][kPrepMaxK];
    const int slot = blockIdx.y, roi = r0 + slot;
    const int64_t f0 = (int64_t)blockIdx.x * kPrepFrames;
    const double sq = sqrt((double)roi_npix[roi]);
    const int64_t *Sr = roi_sum + (int64_t)roi * N;
    const double *L = Lr + (int64_t)slot * k * k;          // row-major lower factor of this ROI

    const int k16 = (k + kPrepChunk - 1) / kPrepChunk * kPrepChunk;
    for (int idx = threadIdx.x; idx < kPrepFrames * k16; idx += blockDim.x) {
        const int a = idx / kPrepFrames, f = idx % kPrepFrames;
        const int64_t tl = f0 + f;
        double w = 0.0;
        if (tl < nw && a < k) {
            const int64_t s = Sr[t0 + tl];
            if (s > 0) w = (double)V[(int64_t)a * N + t0 + tl] * sigma[a] / (double)s;
        }
        wl[f][a] = w;
    }
    // outputs owned by this thread: o = tid + 256*j, frame o / k, column o % k
    constexpr int kMaxOwn = kPrepFrames * kPrepMaxK / 256;
    double acc[kMaxOwn];
#pragma unroll
    for (int j = 0; j < kMaxOwn; ++j) acc[j] = 0.0;
    const int nout = kPrepFrames * k;
    for (int a0 = 0; a0 < k; a0 += kPrepChunk) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < kPrepChunk * k; idx += blockDim.x) {
            const int aa = idx / k, b = idx % k;
            gc[aa][b] = a0 + aa < k ? L[(int64_t)(a0 + aa) * k + b] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kMaxOwn; ++j) {
            const int o = threadIdx.x + 256 * j;
            if (o < nout) {
                const int f = o / k, b = o % k;
                double s = acc[j];
#pragma unroll 4
                for (int aa = 0; aa < kPrepChunk; ++aa) s = fma(wl[f][a0 + aa], gc[aa][b], s);
                acc[j] = s;
            }
        }
    }
    const int64_t base = (int64_t)slot * nw * kp;
#pragma unroll
    for (int j = 0; j < kMaxOwn; ++j) {
        const int o = threadIdx.x + 256 * j;
        if (o < nout) {
            const int f = o / k, b = o % k;
            const int64_t tl = f0 + f;
            if (tl < nw) {
                const double zv = sq * acc[j];
                const unsigned short zh = f32_to_bf16_bits((float)zv);
                z_hi[base + tl * kp + b] = zh;
                z_lo[base + tl * kp + b] = f32_to_bf16_bits((float)(zv - (double)bf16_bits_to_f32(zh)));
            }
        }
    }
    // zero the K padding and record validity
    for (int idx = threadIdx.x; idx < kPrepFrames * (kp - k); idx += blockDim.x) {
        const int f = idx / (kp - k), b = k + idx % (kp - k);
        const int64_t tl = f0 + f;
        if (tl < nw) {
            z_hi[base + tl * kp + b] = 0;
            z_lo[base + tl * kp + b] = 0;
        }
    }
    for (int f = threadIdx.x; f < kPrepFrames; f += blockDim.x) {
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
    dim3 grid((unsigned)((nw + kPrepFrames - 1) / kPrepFrames), (unsigned)nr);
    hipLaunchKernelGGL(lowrank_prep_kernel, grid, dim3(256), 0, ctx->stream, f->V, f->sigma, f->roi_sum,
                       f->roi_npix, Lr, f->N, f->k, r0, t0, nw, kp, z_hi, z_lo, valid);
    XPCS_LAUNCH_CHECK(ctx, "lowrank_prep");
    return XPCS_OK;
}

}  // namespace xpcs
