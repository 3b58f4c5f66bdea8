// Quantities the paper derives from the compression and the correlation to judge
// them (Sec. 3.1, Sec. 3.2), and the stand-in for an encoding basis made from
// unrelated images (Sec. 3.2):
//   * the rank rule: how many eigenvalues of the data Gram are at least twice the
//     smallest one (the number of directions that describe the data);
//   * peak visibility: a g2 peak above the background level of g2, and whether it
//     is detectable: stronger than twice the standard deviation of the TTC;
//   * frames that are randomly shifted copies of one texture image, from which an
//     encoding basis that knows nothing of the sample is built.
#include <math.h>

#include "internal.hpp"

namespace xpcs {
namespace {

// rank = #{i : spectrum[i] > 0 and spectrum[i] >= factor * min(spectrum)}: one block,
// fixed-order reductions.
__global__ __launch_bounds__(256) void rank_rule_kernel(const double *__restrict__ spec, int64_t n, double factor,
                                                        int32_t *__restrict__ rank) {
    __shared__ double s_min[4];
    __shared__ long long s_cnt[4];
    __shared__ double s_lo;
    double m = INFINITY;
    for (int64_t i = threadIdx.x; i < n; i += 256) m = fmin(m, spec[i]);
    for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) s_lo = factor * fmin(fmin(s_min[0], s_min[1]), fmin(s_min[2], s_min[3]));
    __syncthreads();
    const double lo = s_lo;
    long long c = 0;
    for (int64_t i = threadIdx.x; i < n; i += 256) c += (spec[i] > 0.0 && spec[i] >= lo) ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) *rank = (int32_t)(s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3]);
}

// Per ROI (one block): peak = max g2 over the valid lags of [plo, phi), background =
// mean g2 over the valid lags of [blo, bhi), visibility = peak - background (NaN when
// either range has no valid lag); detectable = visibility > factor * stdev.
__global__ __launch_bounds__(256) void peak_visibility_kernel(const double *__restrict__ g2,
                                                              const int64_t *__restrict__ npairs, int64_t n,
                                                              int64_t plo, int64_t phi, int64_t blo, int64_t bhi,
                                                              const double *__restrict__ stdev, double factor,
                                                              double *__restrict__ vis, int32_t *__restrict__ det) {
    __shared__ double s_pk[4], s_bs[4];
    __shared__ long long s_pn[4], s_bn[4];
    const int r = blockIdx.x;
    const double *g = g2 + (int64_t)r * n;
    const int64_t *np = npairs ? npairs + (int64_t)r * n : nullptr;
    double pk = -INFINITY, bs = 0.0;
    long long pn = 0, bn = 0;
    for (int64_t t = plo + threadIdx.x; t < phi; t += 256) {
        const double v = g[t];
        if ((!np || np[t] > 0) && isfinite(v)) {
            pk = fmax(pk, v);
            ++pn;
        }
    }
    for (int64_t t = blo + threadIdx.x; t < bhi; t += 256) {
        const double v = g[t];
        if ((!np || np[t] > 0) && isfinite(v)) {
            bs += v;
            ++bn;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        pk = fmax(pk, __shfl_xor(pk, o));
        bs += __shfl_xor(bs, o);
        pn += __shfl_xor(pn, o);
        bn += __shfl_xor(bn, o);
    }
    if ((threadIdx.x & 63) == 0) {
        const int w = threadIdx.x >> 6;
        s_pk[w] = pk;
        s_bs[w] = bs;
        s_pn[w] = pn;
        s_bn[w] = bn;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double peak = -INFINITY, bsum = 0.0;
    long long npk = 0, nbg = 0;
    for (int w = 0; w < 4; ++w) {
        peak = fmax(peak, s_pk[w]);
        bsum += s_bs[w];
        npk += s_pn[w];
        nbg += s_bn[w];
    }
    const double v = (npk > 0 && nbg > 0) ? peak - bsum / (double)nbg : __builtin_nan("");
    vis[r] = v;
    if (det) det[r] = (stdev && v > factor * stdev[r]) ? 1 : 0;
}

__device__ __forceinline__ uint64_t splitmix64_dev(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// frames[t][y][x] = texture[(y + dy_t) mod H][(x + dx_t) mod W] with h = SplitMix64(seed XOR t),
// dy_t = (h & 0xffffffff) mod H, dx_t = (h >> 32) mod W.  Grid: (row chunks, frames).
template <typename T>
__global__ __launch_bounds__(256) void shifted_texture_kernel(const T *__restrict__ tex, int64_t H, int64_t W,
                                                              uint64_t seed, T *__restrict__ frames) {
    const int64_t t = blockIdx.y;
    const uint64_t h = splitmix64_dev(seed ^ (uint64_t)t);
    const int64_t dy = (int64_t)((h & 0xffffffffull) % (uint64_t)H), dx = (int64_t)((h >> 32) % (uint64_t)W);
    T *out = frames + t * H * W;
    for (int64_t y = blockIdx.x; y < H; y += gridDim.x) {
        const T *src = tex + ((y + dy) % H) * W;
        for (int64_t x = threadIdx.x; x < W; x += 256) out[y * W + x] = src[(x + dx) % W];
    }
}

}  // namespace
}  // namespace xpcs

using namespace xpcs;

extern "C" {

xpcs_status xpcs_rank_rule(xpcs_ctx *ctx, const double *spectrum, int64_t n, double factor, int32_t *rank) {
    if (!ctx) return XPCS_EINVAL;
    if (!spectrum || !rank) return fail(ctx, XPCS_EINVAL, "spectrum and rank must not be NULL");
    if (n < 1) return fail(ctx, XPCS_EINVAL, "n must be positive");
    if (!(factor >= 1.0)) return fail(ctx, XPCS_EINVAL, "factor must be at least 1");
    (void)hipSetDevice(ctx->device);
    Phase phase_(ctx, "rank_rule");
    hipLaunchKernelGGL(rank_rule_kernel, dim3(1), dim3(256), 0, ctx->stream, spectrum, n, factor, rank);
    XPCS_LAUNCH_CHECK(ctx, "rank_rule");
    return XPCS_OK;
}

xpcs_status peak_visibility(xpcs_ctx *ctx, const double *g2, const int64_t *npairs, int32_t n_roi, int64_t n,
                            int64_t peak_lo, int64_t peak_hi, int64_t bg_lo, int64_t bg_hi, const double *ttc_stdev,
                            double factor, double *visibility, int32_t *detectable) {
    if (!ctx) return XPCS_EINVAL;
    if (!g2 || !visibility) return fail(ctx, XPCS_EINVAL, "g2 and visibility must not be NULL");
    if (detectable && !ttc_stdev) return fail(ctx, XPCS_EINVAL, "detectable needs ttc_stdev");
    if (n_roi < 1 || n < 1) return fail(ctx, XPCS_EINVAL, "need n_roi >= 1 and n >= 1");
    if (peak_lo < 0 || peak_hi <= peak_lo || peak_hi > n || bg_lo < 0 || bg_hi <= bg_lo || bg_hi > n)
        return fail(ctx, XPCS_EINVAL, "lag ranges must lie in [0, n) and be non-empty");
    (void)hipSetDevice(ctx->device);
    Phase phase_(ctx, "peak_visibility");
    hipLaunchKernelGGL(peak_visibility_kernel, dim3((unsigned)n_roi), dim3(256), 0, ctx->stream, g2, npairs, n,
                       peak_lo, peak_hi, bg_lo, bg_hi, ttc_stdev, factor, visibility, detectable);
    XPCS_LAUNCH_CHECK(ctx, "peak_visibility");
    return XPCS_OK;
}

xpcs_status shifted_texture_frames(xpcs_ctx *ctx, const void *texture, int32_t dtype, int64_t height, int64_t width,
                                   int64_t n_frames, uint64_t seed, void *frames) {
    if (!ctx) return XPCS_EINVAL;
    if (!texture || !frames) return fail(ctx, XPCS_EINVAL, "texture and frames must not be NULL");
    if (dtype != XPCS_U8 && dtype != XPCS_U16) return fail(ctx, XPCS_EINVAL, "dtype must be XPCS_U8 or XPCS_U16");
    if (height < 1 || width < 1 || n_frames < 1) return fail(ctx, XPCS_EINVAL, "sizes must be positive");
    if (n_frames > 65535) return fail(ctx, XPCS_EUNSUPPORTED, "at most 65535 frames");
    (void)hipSetDevice(ctx->device);
    Phase phase_(ctx, "shifted_texture");
    dim3 grid((unsigned)(height < 64 ? height : 64), (unsigned)n_frames);
    if (dtype == XPCS_U8)
        hipLaunchKernelGGL(shifted_texture_kernel<uint8_t>, grid, dim3(256), 0, ctx->stream,
                           static_cast<const uint8_t *>(texture), height, width, seed, static_cast<uint8_t *>(frames));
    else
        hipLaunchKernelGGL(shifted_texture_kernel<uint16_t>, grid, dim3(256), 0, ctx->stream,
                           static_cast<const uint16_t *>(texture), height, width, seed,
                           static_cast<uint16_t *>(frames));
    XPCS_LAUNCH_CHECK(ctx, "shifted_texture");
    return XPCS_OK;
}

}  // extern "C"
