// ROI bookkeeping and the int8 gather of the raw path.
//
// A q-ROI is an arbitrary pixel subset (Sec. 2.2: the analysis runs on the
// flattened pixels of a q range).  The raw path gathers each ROI's pixels once
// into a dense int8 matrix xs[t][q] (frames x ROI-sorted pixels) so that the
// Gram X_R^T X_R (Sec. 2.1, Eq. 2) reads contiguous K ranges on the int8 MFMA,
// and records the exact per-frame ROI photon sums S_R[t] used to normalise it
// (Eq. 1).
#include "internal.hpp"

namespace xpcs {
namespace {

constexpr int kMaxRoiLds = 4096;

__global__ void fill_i64_kernel(int64_t *p, int64_t n, int64_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Histogram of labels into roi_npix; flags labels outside [-1, n_roi).
__global__ __launch_bounds__(256) void roi_count_kernel(const int32_t *__restrict__ labels, int64_t M,
                                                        int n_roi, unsigned long long *roi_npix,
                                                        int *flags) {
    __shared__ int hist[kMaxRoiLds];
    for (int r = threadIdx.x; r < n_roi; r += blockDim.x) hist[r] = 0;
    __syncthreads();
    bool bad = false;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < M;
         p += (int64_t)gridDim.x * blockDim.x) {
        int l = labels[p];
        if (l >= 0 && l < n_roi)
            atomicAdd(&hist[l], 1);
        else if (l != -1)
            bad = true;
    }
    if (bad) atomicOr(&flags[kFlagLabel], 1);
    __syncthreads();
    for (int r = threadIdx.x; r < n_roi; r += blockDim.x)
        if (hist[r]) atomicAdd(&roi_npix[r], (unsigned long long)hist[r]);
}

// One block per ROI: stable compaction of the ROI's pixel indices.
__global__ __launch_bounds__(1024) void roi_order_kernel(const int32_t *__restrict__ labels, int64_t M,
                                                         int n_roi, const int64_t *__restrict__ roi_npix,
                                                         int pad, int64_t *off, int32_t *perm,
                                                         int32_t *qroi) {
    const int r = blockIdx.x;
    __shared__ int wave_tot[16];
    __shared__ int64_t s_start;
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int i = 0; i < r; ++i) s += (roi_npix[i] + pad - 1) / pad * pad;
        s_start = s;
        off[r] = s;
        if (r == n_roi - 1) off[n_roi] = s + (roi_npix[r] + pad - 1) / pad * pad;
    }
    __syncthreads();
    const int64_t start = s_start;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int64_t base = 0;
    for (int64_t c0 = 0; c0 < M; c0 += blockDim.x) {
        int64_t p = c0 + threadIdx.x;
        bool hit = p < M && labels[p] == r;
        unsigned long long m = __ballot(hit);
        int pre = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wave_tot[wid] = __popcll(m);
        __syncthreads();
        int wbase = 0, tot = 0;
        for (int w = 0; w < nw; ++w) {
            if (w < wid) wbase += wave_tot[w];
            tot += wave_tot[w];
        }
        if (hit) {
            int64_t q = start + base + wbase + pre;
            perm[q] = (int32_t)p;
            qroi[q] = r;
        }
        base += tot;
        __syncthreads();
    }
    const int64_t padded = (roi_npix[r] + pad - 1) / pad * pad;
    for (int64_t q = roi_npix[r] + threadIdx.x; q < padded; q += blockDim.x) {
        perm[start + q] = -1;
        qroi[start + q] = r;
    }
}

// Stable ROI order in three short passes over chunks of kOrderChunk pixels:
// per-chunk ROI counts, their scan into per-chunk starting positions, and the
// scatter.  One wave walks a chunk in pixel order, each lane holding the labels
// of its pixels (loaded at once, so the walk waits for memory only once); the
// pixels of a 64-pixel step are grouped by label (ballot of the lanes that share
// the first unplaced label, until none is left), so every ROI's pixels land in
// increasing pixel order.  Running positions live in LDS and are only touched by
// the one wave.
constexpr int kOrderSteps = 16;                      // 64-pixel steps per chunk
constexpr int kOrderChunk = 64 * kOrderSteps;
constexpr int kOrderMaxRoi = 8192;

__device__ __forceinline__ void chunk_labels(const int32_t *__restrict__ labels, int64_t c0, int64_t end, int n_roi,
                                             int (&lab)[kOrderSteps]) {
    const int lane = threadIdx.x;
#pragma unroll
    for (int i = 0; i < kOrderSteps; ++i) {
        const int64_t p = c0 + 64 * i + lane;
        const int r = p < end ? labels[p] : -1;
        lab[i] = (r >= 0 && r < n_roi) ? r : -1;
    }
}

__global__ __launch_bounds__(64) void roi_chunk_count_kernel(const int32_t *__restrict__ labels, int64_t M, int n_roi,
                                                             int64_t *__restrict__ counts) {
    extern __shared__ int64_t cnt[];
    const int lane = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * kOrderChunk;
    const int64_t end = c0 + kOrderChunk < M ? c0 + kOrderChunk : M;
    int lab[kOrderSteps];
    chunk_labels(labels, c0, end, n_roi, lab);
    for (int r = lane; r < n_roi; r += 64) cnt[r] = 0;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kOrderSteps; ++i) {
        unsigned long long left = __ballot(lab[i] >= 0);
        while (left) {
            const int leader = __ffsll((long long)left) - 1;
            const int lr = __shfl(lab[i], leader);
            const unsigned long long mk = __ballot(lab[i] == lr);
            if (lane == leader) cnt[lr] += __popcll(mk);
            left &= ~mk;
        }
    }
    __syncthreads();
    for (int r = lane; r < n_roi; r += 64) counts[(int64_t)blockIdx.x * n_roi + r] = cnt[r];
}

// One block per ROI r: its start (the padded lengths of ROIs below it, summed),
// then the exclusive scan of its per-chunk counts over the chunks, 256 at a
// time, in place; the padding slots after its pixels get perm -1.
__global__ __launch_bounds__(256) void roi_chunk_scan_kernel(int n_roi, int64_t nchunks,
                                                             const int64_t *__restrict__ roi_npix, int pad,
                                                             int64_t *__restrict__ counts, int64_t *off,
                                                             int32_t *perm, int32_t *qroi) {
    __shared__ int64_t wsum[4];
    __shared__ int64_t carry;
    const int r = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    auto padded = [&](int i) { return (roi_npix[i] + pad - 1) / pad * pad; };
    auto block_sum = [&](int64_t v) {        // sum over the block, in a fixed order
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) wsum[wv] = v;
        __syncthreads();
        const int64_t t = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
        return t;
    };
    int64_t below = 0;
    for (int i = tid; i < r; i += 256) below += padded(i);
    const int64_t start = block_sum(below);
    if (tid == 0) {
        off[r] = start;
        if (r == n_roi - 1) off[n_roi] = start + padded(r);
        carry = start;
    }
    __syncthreads();
    for (int64_t c0 = 0; c0 < nchunks; c0 += 256) {
        const int64_t c = c0 + tid;
        const int64_t n = c < nchunks ? counts[c * n_roi + r] : 0;
        // inclusive scan of n over the block: within waves, then the wave totals
        int64_t x = n;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        int64_t before = carry;
        for (int w = 0; w < wv; ++w) before += wsum[w];
        const int64_t total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        if (c < nchunks) counts[c * n_roi + r] = before + x - n;
        __syncthreads();
        if (tid == 0) carry += total;
        __syncthreads();
    }
    for (int64_t q = start + roi_npix[r] + tid; q < start + padded(r); q += 256) {
        perm[q] = -1;
        qroi[q] = r;
    }
}

__global__ __launch_bounds__(64) void roi_chunk_scatter_kernel(const int32_t *__restrict__ labels, int64_t M,
                                                               int n_roi, const int64_t *__restrict__ starts,
                                                               int32_t *perm, int32_t *qroi) {
    extern __shared__ int64_t pos[];
    const int lane = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * kOrderChunk;
    const int64_t end = c0 + kOrderChunk < M ? c0 + kOrderChunk : M;
    int lab[kOrderSteps];
    chunk_labels(labels, c0, end, n_roi, lab);
    for (int r = lane; r < n_roi; r += 64) pos[r] = starts[(int64_t)blockIdx.x * n_roi + r];
    __syncthreads();
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int i = 0; i < kOrderSteps; ++i) {
        const int64_t p = c0 + 64 * i + lane;
        unsigned long long left = __ballot(lab[i] >= 0);
        while (left) {
            const int leader = __ffsll((long long)left) - 1;
            const int lr = __shfl(lab[i], leader);
            const unsigned long long mk = __ballot(lab[i] == lr);
            const int64_t b = pos[lr];
            if (lab[i] == lr) {
                const int64_t q = b + __popcll(mk & below);
                perm[q] = (int32_t)p;
                qroi[q] = lr;
            }
            if (lane == leader) pos[lr] = b + __popcll(mk);
            left &= ~mk;
        }
    }
}

// Block = (4096 ROI-sorted positions) x (32 frames).  A thread owns 4 consecutive
// positions (never split between ROIs: ROI starts are multiples of 64), keeps
// their pixel indices in registers for all 32 frames, and writes one packed
// 4-byte word per frame, so both the gathered loads and the stores are
// contiguous across the wave.  ROI sums go through LDS (int, exact) and then one
// exact 64-bit atomic per (frame, ROI) and block.
//
// xs holds plane 0 of the counts (count & 127), exact in int8; a position with a
// count of 128 or more is marked hot[q] (bit 0: plane 1 is needed; bit 1: plane 2,
// a count of 16384 or more), and the raw Gram adds those pixels' higher planes
// separately.  amax is the largest plane-0 value, which sets the int32 chunk.
constexpr int kGatherQ = 4096;
constexpr int kGatherT = 32;
constexpr int kGatherSlots = 64;

template <typename T>
__global__ __launch_bounds__(256) void gather_i8_kernel(const T *__restrict__ frames, int64_t M, int64_t t0,
                                                        int64_t nw, const int32_t *__restrict__ perm,
                                                        const int32_t *__restrict__ qroi,
                                                        const int64_t *__restrict__ off, int n_roi,
                                                        int64_t ldx, int8_t *__restrict__ xs,
                                                        unsigned long long *__restrict__ S, int *amax,
                                                        int *__restrict__ hot) {
    __shared__ int s_sum[kGatherT][kGatherSlots];
    const int64_t total = off[n_roi];
    const int64_t qb = (int64_t)blockIdx.x * kGatherQ;
    if (qb >= total) return;
    const int64_t tb = (int64_t)blockIdx.y * kGatherT;
    const int r_first = qroi[qb];
    for (int idx = threadIdx.x; idx < kGatherT * kGatherSlots; idx += blockDim.x) (&s_sum[0][0])[idx] = 0;
    __syncthreads();
    int vmax = 0;
    constexpr int kPasses = kGatherQ / (4 * 256);
    int px[kPasses][4];
    int roi[kPasses];
    bool live[kPasses];
    unsigned hb[kPasses][4];
#pragma unroll
    for (int ps = 0; ps < kPasses; ++ps) {
        const int64_t q = qb + 4 * (threadIdx.x + 256 * ps);
        live[ps] = q < total;
        roi[ps] = live[ps] ? qroi[q] : -1;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            px[ps][e] = live[ps] ? perm[q + e] : -1;
            hb[ps][e] = 0;
        }
    }
    const int64_t tend = tb + kGatherT < nw ? tb + kGatherT : nw;
#pragma unroll 4
    for (int64_t tl = tb; tl < tend; ++tl) {
        const T *fr = frames + (t0 + tl) * M;
#pragma unroll
        for (int ps = 0; ps < kPasses; ++ps) {
            if (!live[ps]) continue;
            int v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = px[ps][e] >= 0 ? (int)fr[px[ps][e]] : 0;
            int sum = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                sum += v[e];
                hb[ps][e] |= (v[e] >= 128 ? 1u : 0u) | (v[e] >= 16384 ? 2u : 0u);
                v[e] &= 127;
                vmax = v[e] > vmax ? v[e] : vmax;
            }
            const int word = (v[0] & 0xff) | ((v[1] & 0xff) << 8) | ((v[2] & 0xff) << 16) | ((v[3] & 0xff) << 24);
            const int64_t q = qb + 4 * (threadIdx.x + 256 * ps);
            *reinterpret_cast<int *>(xs + tl * ldx + q) = word;
            if (sum) {
                const int slot = roi[ps] - r_first;
                if (slot < kGatherSlots)
                    atomicAdd(&s_sum[tl - tb][slot], sum);
                else
                    atomicAdd(&S[(int64_t)roi[ps] * nw + tl], (unsigned long long)sum);
            }
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kGatherT * kGatherSlots; idx += blockDim.x) {
        const int tt = idx / kGatherSlots, slot = idx % kGatherSlots;
        const int v = s_sum[tt][slot];
        if (v && r_first + slot < n_roi && tb + tt < nw)
            atomicAdd(&S[(int64_t)(r_first + slot) * nw + tb + tt], (unsigned long long)v);
    }
#pragma unroll
    for (int ps = 0; ps < kPasses; ++ps)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (hb[ps][e]) atomicOr(&hot[qb + 4 * (threadIdx.x + 256 * ps) + e], (int)hb[ps][e]);
    for (int o = 32; o > 0; o >>= 1) {
        int v = __shfl_xor(vmax, o);
        vmax = v > vmax ? v : vmax;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(amax, vmax);
}

// Per ROI (one block): the hot positions of its range in order, hq[off[r] + i]
// (i < hcnt[r]), and the OR of their plane bits in hbits[r].
__global__ __launch_bounds__(256) void hot_list_kernel(const int *__restrict__ hot, const int64_t *__restrict__ off,
                                                       int64_t *__restrict__ hq, int *__restrict__ hcnt,
                                                       int *__restrict__ hbits) {
    __shared__ int s_cnt[4];
    __shared__ int s_base;
    __shared__ int s_bits;
    const int r = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t q0 = off[r], q1 = off[r + 1];
    if (threadIdx.x == 0) {
        s_base = 0;
        s_bits = 0;
    }
    __syncthreads();
    int bits = 0;
    for (int64_t c = q0; c < q1; c += 256) {
        const int64_t q = c + threadIdx.x;
        const int h = q < q1 ? hot[q] : 0;
        bits |= h;
        const unsigned long long m = __ballot(h != 0);
        if (lane == 0) s_cnt[w] = __popcll(m);
        __syncthreads();
        int before = s_base;
        for (int v = 0; v < w; ++v) before += s_cnt[v];
        if (h) hq[q0 + before + __popcll(m & ((1ull << lane) - 1ull))] = q;
        __syncthreads();
        if (threadIdx.x == 0) s_base += s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
        __syncthreads();
    }
    if (bits) atomicOr(&s_bits, bits);
    __syncthreads();
    if (threadIdx.x == 0) {
        hcnt[r] = s_base;
        hbits[r] = s_bits;
    }
}

}  // namespace

xpcs_status launch_roi_count(xpcs_ctx *ctx, const int32_t *labels, int64_t M, int n_roi,
                             int64_t *roi_npix) {
    Phase phase_(ctx, "roi_count");
    if (n_roi > kMaxRoiLds) return fail(ctx, XPCS_EUNSUPPORTED, "more than 4096 ROIs");
    hipLaunchKernelGGL(fill_i64_kernel, dim3(1), dim3(256), 0, ctx->stream, roi_npix, (int64_t)n_roi,
                       (int64_t)0);
    int grid = (int)((M + 255) / 256);
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(roi_count_kernel, dim3(grid), dim3(256), 0, ctx->stream, labels, M, n_roi,
                       reinterpret_cast<unsigned long long *>(roi_npix), ctx->flags);
    XPCS_LAUNCH_CHECK(ctx, "roi_count");
    return XPCS_OK;
}

xpcs_status launch_roi_order(xpcs_ctx *ctx, const int32_t *labels, int64_t M, int n_roi,
                             const int64_t *roi_npix, int pad, int64_t *off, int32_t *perm,
                             int32_t *qroi, int64_t total_cap) {
    Phase phase_(ctx, "roi_order");
    (void)total_cap;
    if (n_roi > kOrderMaxRoi) {
        hipLaunchKernelGGL(roi_order_kernel, dim3(n_roi), dim3(1024), 0, ctx->stream, labels, M, n_roi,
                           roi_npix, pad, off, perm, qroi);
        XPCS_LAUNCH_CHECK(ctx, "roi_order");
        return XPCS_OK;
    }
    const int64_t nchunks = (M + kOrderChunk - 1) / kOrderChunk;
    xpcs_status st;
    auto *counts = static_cast<int64_t *>(scratch_get(ctx, (size_t)nchunks * n_roi * sizeof(int64_t), &st));
    if (!counts) return st;
    const size_t lds = (size_t)n_roi * sizeof(int64_t);
    hipLaunchKernelGGL(roi_chunk_count_kernel, dim3((unsigned)nchunks), dim3(64), lds, ctx->stream, labels, M, n_roi,
                       counts);
    XPCS_LAUNCH_CHECK(ctx, "roi_chunk_count");
    hipLaunchKernelGGL(roi_chunk_scan_kernel, dim3((unsigned)n_roi), dim3(256), 0, ctx->stream, n_roi, nchunks,
                       roi_npix, pad, counts, off, perm, qroi);
    XPCS_LAUNCH_CHECK(ctx, "roi_chunk_scan");
    hipLaunchKernelGGL(roi_chunk_scatter_kernel, dim3((unsigned)nchunks), dim3(64), lds, ctx->stream, labels, M,
                       n_roi, counts, perm, qroi);
    XPCS_LAUNCH_CHECK(ctx, "roi_chunk_scatter");
    return XPCS_OK;
}

xpcs_status launch_gather_i8(xpcs_ctx *ctx, const void *frames, int dtype, int64_t M, int64_t t0, int64_t nw,
                             const int32_t *perm, const int32_t *qroi, const int64_t *off, int n_roi, int64_t ldx,
                             int8_t *xs, int64_t *S, int *amax, int *hot, int64_t *hq, int *hcnt, int *hbits,
                             int64_t total_cap) {
    Phase phase_(ctx, "gather_i8");
    if (ldx % 16) return fail(ctx, XPCS_EINVAL, "internal: gather row stride not a multiple of 16");
    // the sums are accumulated with atomics, the hot marks ORed: start from zero
    hipLaunchKernelGGL(fill_i64_kernel, dim3(256), dim3(256), 0, ctx->stream, S, (int64_t)n_roi * nw, (int64_t)0);
    xpcs_status st = launch_zero(ctx, hot, (size_t)total_cap * sizeof(int));
    if (st) return st;
    dim3 grid((unsigned)((total_cap + kGatherQ - 1) / kGatherQ), (unsigned)((nw + kGatherT - 1) / kGatherT));
    auto *Su = reinterpret_cast<unsigned long long *>(S);
    if (dtype == XPCS_U8)
        hipLaunchKernelGGL(gather_i8_kernel<uint8_t>, grid, dim3(256), 0, ctx->stream,
                           static_cast<const uint8_t *>(frames), M, t0, nw, perm, qroi, off, n_roi, ldx, xs, Su,
                           amax, hot);
    else
        hipLaunchKernelGGL(gather_i8_kernel<uint16_t>, grid, dim3(256), 0, ctx->stream,
                           static_cast<const uint16_t *>(frames), M, t0, nw, perm, qroi, off, n_roi, ldx, xs, Su,
                           amax, hot);
    XPCS_LAUNCH_CHECK(ctx, "gather_i8");
    hipLaunchKernelGGL(hot_list_kernel, dim3((unsigned)n_roi), dim3(256), 0, ctx->stream, hot, off, hq, hcnt, hbits);
    XPCS_LAUNCH_CHECK(ctx, "hot_list");
    return XPCS_OK;
}

}  // namespace xpcs
