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

// Band form of the same gather.  The pixels are cut into bands of kBandPx; since
// every ROI's pixels are in increasing pixel order, the positions of ROI r whose
// pixels lie in band b are one contiguous range [bs[b][r], bs[b + 1][r]) of the ROI
// order (bs[nbands][r] is the padded end of ROI r, so the padding positions fall
// in the last band).  A block takes one band and kBandFrames frames.  Waves 0 and 1
// stream the band's counts, FG frames per stage, into four LDS stage buffers with
// direct-to-LDS loads (contiguous 1 KB per instruction, three stages in flight while
// the fourth is read); the other waves take
// 256-position units of the band's ranges (four 4-aligned positions per lane), look
// each frame's counts up in the stage and write them as one 4-byte word (bytes at a
// range's ends, which neighbouring bands share).  The consumers issue no vector
// loads after their first store (the band pixel of every position is staged in LDS
// once) and no LDS writes (which would wait for the loads in flight), so they never
// wait for their own stores, and the loader waits only for its loads.  A consumer
// takes a contiguous share of the units and adds a ROI's sums per frame in
// registers, then once (exact 64-bit atomic) when the ROI changes; hot marks and
// amax as in the position-order gather.
constexpr int kBandPx = 8192;
constexpr int kBandFrames = 256;
constexpr int kBandMaxRoi = 64;
constexpr int kBandMaxPos = kBandPx + (64 - 1) * kBandMaxRoi;    // pixels plus the last band's padding
constexpr int kBandMaxUnits = kBandPx / 256 + 2 * kBandMaxRoi + 8;
constexpr int kBandWaves = 16;
typedef __attribute__((address_space(3))) void band_lds_t;

// bs[b * n_roi + r] for b in [0, nbands]: the first position of ROI r whose pixel is
// at or past pixel b * kBandPx (the padding, perm -1, counts as past every pixel);
// bs[nbands * n_roi + r] = off[r + 1].
__global__ __launch_bounds__(256) void band_starts_kernel(const int32_t *__restrict__ perm,
                                                          const int64_t *__restrict__ off, int n_roi, int64_t nbands,
                                                          int64_t *__restrict__ bs) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (nbands + 1) * n_roi) return;
    const int64_t b = idx / n_roi;
    const int r = (int)(idx % n_roi);
    int64_t lo = off[r], hi = off[r + 1];
    if (b == nbands) {
        bs[idx] = hi;
        return;
    }
    const int64_t key = b * kBandPx;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        const int32_t p = perm[mid];
        if (p >= 0 && p < key) lo = mid + 1;
        else hi = mid;
    }
    bs[idx] = lo;
}

// Sum over the wave, in every lane: row sums by DPP shifts (lane 15 of each row of
// 16 holds its row's sum), then the four row sums read as scalars.
__device__ __forceinline__ int band_wave_sum(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);    // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);    // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);    // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);    // row_shr:8
    return __builtin_amdgcn_readlane(x, 15) + __builtin_amdgcn_readlane(x, 31) + __builtin_amdgcn_readlane(x, 47) +
           __builtin_amdgcn_readlane(x, 63);
}

template <typename T, int FG>
__global__ __launch_bounds__(64 * kBandWaves, 1) void gather_band_kernel(
    const T *__restrict__ frames, int64_t M, int64_t t0, int64_t nw, const int32_t *__restrict__ perm,
    const int64_t *__restrict__ bs, int n_roi, int64_t ldx, int8_t *__restrict__ xs,
    unsigned long long *__restrict__ S, int *amax, int *__restrict__ hot, int vec) {
    constexpr int kCons = kBandWaves - 2;
    // four stage buffers as distinct arrays, each picked statically, so the compiler
    // sees that the loads in flight never fill the buffer being read
    __shared__ __align__(16) T stage0[FG * kBandPx];
    __shared__ __align__(16) T stage1[FG * kBandPx];
    __shared__ __align__(16) T stage2[FG * kBandPx];
    __shared__ __align__(16) T stage3[FG * kBandPx];
    __shared__ short lpl[kBandMaxPos];               // band pixel of each of the band's positions, -1: padding
    __shared__ int4 units[kBandMaxUnits];            // (first position, range start, range end, ROI | lpl base << 8)
    __shared__ int s_nunits;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t b = blockIdx.x, P0 = b * kBandPx;
    const int npx = M - P0 < kBandPx ? (int)(M - P0) : kBandPx;
    const int64_t tb = (int64_t)blockIdx.y * kBandFrames;
    const int nf_blk = nw - tb < kBandFrames ? (int)(nw - tb) : kBandFrames;
    const int ngroups = (nf_blk + FG - 1) / FG;
    // the band's ranges as units of 256 positions from a 4-aligned first position
    if (wv == 0) {
        int qs = 0, qe = 0, nu = 0;
        if (lane < n_roi) {
            qs = (int)bs[b * n_roi + lane];
            qe = (int)bs[(b + 1) * n_roi + lane];
            if (qe > qs) nu = (qe - (qs & ~3) + 255) / 256;
        }
        int x = nu, y = qe - qs;                     // inclusive scans: units, positions
        for (int o = 1; o < 64; o <<= 1) {
            const int xu = __shfl_up(x, o), yu = __shfl_up(y, o);
            if (lane >= o) {
                x += xu;
                y += yu;
            }
        }
        const int base = y - (qe - qs);
        for (int k = 0; k < nu; ++k) units[x - nu + k] = make_int4((qs & ~3) + 256 * k, qs, qe, lane | (base << 8));
        if (lane == 63) s_nunits = x;
    }
    __syncthreads();
    const int nunits = s_nunits;
    // band pixel of every position (the only reads of perm, before any store): one
    // 16-byte load per lane and unit (positions q..q+3, q 4-aligned, all below the
    // padded end of the ROI order when q is below the range end), all issued first
    for (int u0 = wv; u0 < nunits; u0 += 4 * kBandWaves) {
        int4 pv[4];
        int4 Us[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int u = u0 + k * kBandWaves;
            Us[k] = u < nunits ? units[u] : make_int4(0, 0, 0, 0);
            const int q = Us[k].x + 4 * lane;
            pv[k] = q < Us[k].z ? *reinterpret_cast<const int4 *>(perm + q) : make_int4(-1, -1, -1, -1);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int q = Us[k].x + 4 * lane;
            const int pe[4] = {pv[k].x, pv[k].y, pv[k].z, pv[k].w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (q + e >= Us[k].y && q + e < Us[k].z)
                    lpl[(Us[k].w >> 8) + q + e - Us[k].y] = (short)(pe[e] >= 0 ? pe[e] - (int)P0 : -1);
        }
    }
    // the loaders (waves 0 and 1, half of every frame each): frames [tb + FG g,
    // tb + FG g + FG) of the band into a stage buffer; returns whether the group was
    // a full one (kFullLoads loads by each loader)
    const int bytes = npx * (int)sizeof(T);
    constexpr int kFullLoads = FG * kBandPx * (int)sizeof(T) / 2048;
    static_assert(3 * kFullLoads < 64, "vmcnt range");
    auto load_group = [&](int g, T *dst0) {
        const int half = (bytes / 2 + 1023) / 1024 * 1024;        // the first loader's share, whole KB
        const int c0 = wv == 0 ? 0 : half, c1 = wv == 0 ? (half < bytes ? half : bytes) : bytes;
#pragma unroll
        for (int f = 0; f < FG; ++f) {
            const int tl = FG * g + f;
            if (tl >= nf_blk) break;
            const T *src = frames + (t0 + tb + tl) * M + P0;
            T *dst = dst0 + f * kBandPx;
            if (vec) {
                for (int c = c0; c < c1; c += 1024) {
                    if (c + 16 * lane < c1)
                        __builtin_amdgcn_global_load_lds(
                            reinterpret_cast<const void *>(reinterpret_cast<const char *>(src) + c + 16 * lane),
                            (band_lds_t *)(reinterpret_cast<char *>(dst) + c), 16, 0, 0);
                }
            } else {
                const int e0 = wv == 0 ? 0 : npx / 2, e1 = wv == 0 ? npx / 2 : npx;
                for (int i = e0 + lane; i < e1; i += 64) dst[i] = src[i];
            }
        }
        return vec && npx == kBandPx && FG * g + FG <= nf_blk;
    };
    // wait until no more than the loads of the n newest groups are in flight (all full),
    // else until none is
    auto wait_newest = [&](int n, bool full) {
        if (full && n == 2)
            __builtin_amdgcn_s_waitcnt(((2 * kFullLoads) & 15) | (((2 * kFullLoads) >> 4) << 14) | (0x7 << 4) |
                                       (0xF << 8));
        else if (full && n == 1)
            __builtin_amdgcn_s_waitcnt((kFullLoads & 15) | ((kFullLoads >> 4) << 14) | (0x7 << 4) | (0xF << 8));
        else
            __builtin_amdgcn_s_waitcnt((0 & 15) | ((0 >> 4) << 14) | (0x7 << 4) | (0xF << 8));
    };
    const bool loader = wv < 2;
    if (loader) {
        load_group(0, stage0);
        bool full = true;
        int n = 0;
        if (ngroups > 1) full = load_group(1, stage1) && full, ++n;
        if (ngroups > 2) full = load_group(2, stage2) && full, ++n;
        wait_newest(n, full);                       // group 0 has landed
    }
    __syncthreads();
    // a consumer's contiguous share of the units (consecutive units mostly share a ROI)
    const int cw = wv - 2;
    const int u_begin = loader ? 0 : (int)((int64_t)cw * nunits / kCons);
    const int u_end = loader ? 0 : (int)((int64_t)(cw + 1) * nunits / kCons);
    int vmax = 0;
    // group g: the consumers read stg, the loader fills nxt with group g + 2
    auto step = [&](int g, const T *stg, T *nxt) {
        if (loader) {
            // group g + 3 into the buffer read at g - 1, then group g + 1 must have landed
            const int n = (g + 2 < ngroups) + (g + 3 < ngroups);
            bool full = g + 2 < ngroups ? (vec && npx == kBandPx && FG * (g + 2) + FG <= nf_blk) : true;
            if (g + 3 < ngroups) full = load_group(g + 3, nxt) && full;
            wait_newest(n, full);
        } else {
            const int nf = nf_blk - FG * g < FG ? nf_blk - FG * g : FG;
            int cur = -1;                            // ROI of the sums held in acc
            int acc[FG];
#pragma unroll
            for (int f = 0; f < FG; ++f) acc[f] = 0;
            auto flush = [&]() {
#pragma unroll
                for (int f = 0; f < FG; ++f) {
                    const int t = band_wave_sum(acc[f]);
                    if (lane == 0 && t && f < nf)
                        atomicAdd(&S[(int64_t)cur * nw + tb + FG * g + f], (unsigned long long)t);
                    acc[f] = 0;
                }
            };
            for (int u = u_begin; u < u_end; ++u) {
                const int4 U = units[u];
                const int r = U.w & 255;
                if (r != cur) {
                    if (cur >= 0) flush();
                    cur = r;
                }
                const int q = U.x + 4 * lane;           // lanes past the range take part with zeros
                int lp[4];
                bool in[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    in[e] = q + e >= U.y && q + e < U.z;
                    int li = (U.w >> 8) + q + e - U.y;
                    li = li < 0 ? 0 : (li >= kBandMaxPos ? kBandMaxPos - 1 : li);
                    const int l = lpl[li];
                    lp[e] = in[e] ? l : -1;
                }
                const bool all = in[0] && in[1] && in[2] && in[3];
#pragma unroll
                for (int f = 0; f < FG; ++f) {
                    if (f >= nf) break;
                    int v[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int x = (int)stg[f * kBandPx + (lp[e] < 0 ? 0 : lp[e])];
                        v[e] = lp[e] < 0 ? 0 : x;
                    }
                    acc[f] += v[0] + v[1] + v[2] + v[3];
                    const int vm = max(max(v[0], v[1]), max(v[2], v[3]));
                    if (vm >= 128) {                     // hot pixels (rare): mark their planes
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int hb = (v[e] >= 128 ? 1 : 0) | (v[e] >= 16384 ? 2 : 0);
                            if (hb) atomicOr(&hot[q + e], hb);
                        }
                    }
                    const int p0 = v[0] & 127, p1 = v[1] & 127, p2 = v[2] & 127, p3 = v[3] & 127;
                    vmax = max(vmax, max(max(p0, p1), max(p2, p3)));
                    int8_t *dst = xs + (tb + FG * g + f) * ldx + q;
                    if (all) {
                        *reinterpret_cast<int *>(dst) = p0 | (p1 << 8) | (p2 << 16) | (p3 << 24);
                    } else {
                        if (in[0]) dst[0] = (int8_t)p0;
                        if (in[1]) dst[1] = (int8_t)p1;
                        if (in[2]) dst[2] = (int8_t)p2;
                        if (in[3]) dst[3] = (int8_t)p3;
                    }
                }
            }
            if (cur >= 0) flush();
        }
        // a bare barrier: no wave waits for its stores, the loader's newest group stays
        // in flight (what crosses it in LDS is ordered by the loader's own wait)
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    };
    for (int g = 0; g < ngroups; g += 4) {
        step(g, stage0, stage3);
        if (g + 1 < ngroups) step(g + 1, stage1, stage0);
        if (g + 2 < ngroups) step(g + 2, stage2, stage1);
        if (g + 3 < ngroups) step(g + 3, stage3, stage2);
    }
    for (int o = 32; o > 0; o >>= 1) vmax = max(vmax, __shfl_xor(vmax, o));
    if (lane == 0 && vmax) atomicMax(amax, vmax);
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
    auto *Su = reinterpret_cast<unsigned long long *>(S);
    const int64_t nbands = (M + kBandPx - 1) / kBandPx;
    if (n_roi <= kBandMaxRoi && total_cap < ((int64_t)1 << 31) && nbands < 65536 && nw > 0) {
        auto *bs = static_cast<int64_t *>(scratch_get(ctx, (size_t)(nbands + 1) * n_roi * sizeof(int64_t), &st));
        if (!bs) return st;
        const int64_t nbs = (nbands + 1) * n_roi;
        hipLaunchKernelGGL(band_starts_kernel, dim3((unsigned)((nbs + 255) / 256)), dim3(256), 0, ctx->stream, perm,
                           off, n_roi, nbands, bs);
        XPCS_LAUNCH_CHECK(ctx, "band_starts");
        const size_t esz = dtype == XPCS_U8 ? 1 : 2;
        const int vec = (reinterpret_cast<uintptr_t>(frames) % 16 == 0 && (M * esz) % 16 == 0) ? 1 : 0;
        dim3 bgrid((unsigned)nbands, (unsigned)((nw + kBandFrames - 1) / kBandFrames));
        if (dtype == XPCS_U8)
            hipLaunchKernelGGL((gather_band_kernel<uint8_t, 4>), bgrid, dim3(64 * kBandWaves), 0, ctx->stream,
                               static_cast<const uint8_t *>(frames), M, t0, nw, perm, bs, n_roi, ldx, xs, Su, amax,
                               hot, vec);
        else
            hipLaunchKernelGGL((gather_band_kernel<uint16_t, 2>), bgrid, dim3(64 * kBandWaves), 0, ctx->stream,
                               static_cast<const uint16_t *>(frames), M, t0, nw, perm, bs, n_roi, ldx, xs, Su, amax,
                               hot, vec);
        XPCS_LAUNCH_CHECK(ctx, "gather_band");
        hipLaunchKernelGGL(hot_list_kernel, dim3((unsigned)n_roi), dim3(256), 0, ctx->stream, hot, off, hq, hcnt,
                           hbits);
        XPCS_LAUNCH_CHECK(ctx, "hot_list");
        return XPCS_OK;
    }
    dim3 grid((unsigned)((total_cap + kGatherQ - 1) / kGatherQ), (unsigned)((nw + kGatherT - 1) / kGatherT));
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
