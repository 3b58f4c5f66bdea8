// Frame-space product part[c][t][j] = sum_{p in chunk c} X[t][p] B[j][p] (the
// basis passes X^T Q of Sec. 2.1 and the encoding W = X^T U of Eq. 7).
//
// The staged operand B holds, per 16-row block, the bf16 rows of Q (hi), of its
// residual term (lo, added into the same accumulators) and of the ROI indicator
// matrix (bf16 0/1 rows, label[p] == r, zero past M), whose columns give the exact
// ROI sums S_R[t].  Each K step of KS pixels of B reaches LDS through gfx950's
// direct-to-LDS loads (global_load_lds_dwordx4: each lane's 16 bytes land at the
// wave's LDS address + 16 * lane), XOR-swizzled in 16-byte pieces so that the
// fragment reads of eight consecutive rows fall on distinct banks; three stage
// buffers rotate.  The counts go straight into registers (a lane's 8 or 16 pixels
// of one frame are its MFMA A fragment), two steps ahead.
//
// Vector-memory loads complete in order, so each step issues the counts of step
// s + 2 before the rows of step s + 2: waiting for the rows of step s then also
// covers its counts, while the counts and rows of step s + 1 stay in flight through
// the barrier that publishes every wave's rows.
//
// Chunks and the XCD-aware placement are those of the register-staged kernel (a
// chunk is a multiple of 64 pixels, so only the last chunk ends inside a K step:
// its counts at or past M are read from the chunk's first pixels and meet zero
// columns of B; frames past N read frame N - 1 and their outputs are dropped).
#pragma once

#include <type_traits>

#include "proj_frames.hpp"

namespace xpcs {
namespace proj {

typedef __attribute__((address_space(3))) void lds_void_t;

// s_waitcnt vmcnt(n) with no wait on the other counters (gfx9 encoding: vmcnt in
// bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// Slot of 16-byte piece `piece` of row `row` in rows of P pieces (P = 2, 4, 8): the
// eight rows that share a 128-byte bank window hold each piece in a different slot.
template <int P>
__device__ __forceinline__ int dma_slot(int row, int piece) {
    return piece ^ ((row / (8 / P)) & (P - 1));
}

// Loads per row block and K step of the lane's counts (NL loads of 16 bytes, or
// one of 8 bytes for uint8 counts at KS = 32).
template <typename T, int KS> struct XStep;
template <> struct XStep<uint8_t, 64> { static constexpr int NL = 1; };     // 16 px: both K groups
template <> struct XStep<uint8_t, 32> { static constexpr int NL = 1; };     // 8 px
template <> struct XStep<uint16_t, 32> { static constexpr int NL = 1; };    // 8 px
template <> struct XStep<uint16_t, 64> { static constexpr int NL = 2; };    // 2 x 8 px

template <typename T, int RB, int NCB, int NIB, bool LO, int KS>
struct DmaShape {
    static constexpr int FB = RB * 64;                         // frames per block (4 waves x RB x 16)
    static constexpr int NBR = NCB * (LO ? 2 : 1) + NIB;       // 16-row blocks of B
    static constexpr int BP = KS * 2 / 16;                     // 16-byte pieces per B row
    static constexpr int BBYTES = NBR * 16 * KS * 2;           // one stage of B
    static constexpr int UB = BBYTES / 1024;                   // 1 KB load units per stage
    static constexpr int UPW = (UB + 3) / 4;                   // row load units per wave and step
    static constexpr int NXL = RB * XStep<T, KS>::NL;          // count loads per lane and step
    static_assert(BBYTES % 1024 == 0, "whole load units");
};

template <typename T, int RB, int NCB, int NIB, bool LO, int KS>
__global__ __launch_bounds__(256, 2) void proj_frames_dma_kernel(const T *__restrict__ X, int64_t M, int64_t N,
                                                                 const unsigned short *__restrict__ qh,
                                                                 const unsigned short *__restrict__ ql,
                                                                 const unsigned short *__restrict__ ind, int64_t ldq,
                                                                 int64_t chunk, int nfb, int ncols,
                                                                 float *__restrict__ part) {
    typedef DmaShape<T, RB, NCB, NIB, LO, KS> S;
    constexpr int BP = S::BP, UPW = S::UPW, UB = S::UB, NL = XStep<T, KS>::NL;
    constexpr int kKK = KS / 32;
    __shared__ __attribute__((aligned(1024))) unsigned char st0[S::BBYTES], st1[S::BBYTES], st2[S::BBYTES];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lr = lane & 15, lg = lane >> 4;
    const int bid = blockIdx.x, xcd = bid & 7, sl = bid >> 3;
    const int ch = xcd + 8 * (sl / nfb), fb = sl % nfb;
    const int64_t p_begin = (int64_t)ch * chunk;
    const int64_t p_end = p_begin + chunk < M ? p_begin + chunk : M;
    const int nsteps = p_end > p_begin ? (int)((p_end - p_begin + KS - 1) / KS) : 0;
    const int64_t f0 = (int64_t)fb * S::FB;
    const int xrow0 = wv * RB * 16;

    // B load units u = wv + 4 j
    const unsigned short *bsrc[UPW];
    int bpoff[UPW];
#pragma unroll
    for (int j = 0; j < UPW; ++j) {
        int u = wv + 4 * j;
        u = u < UB ? u : UB - 1;
        const int row = u * (64 / BP) + lane / BP;
        const int piece = dma_slot<BP>(row, lane % BP);
        const unsigned short *r;
        if (row < 16 * NCB)
            r = qh + (int64_t)row * ldq;
        else if (LO && row < 32 * NCB)
            r = ql + (int64_t)(row - 16 * NCB) * ldq;
        else
            r = ind + (int64_t)(row - 16 * NCB * (LO ? 2 : 1)) * ldq;
        bsrc[j] = r;
        bpoff[j] = piece * 8;
    }
    auto issue_b = [&](int step, unsigned char *dst) {
        const int64_t p0 = p_begin + (int64_t)KS * step;
#pragma unroll
        for (int j = 0; j < UPW; ++j) {
            int u = wv + 4 * j;
            u = u < UB ? u : UB - 1;
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const void *>(bsrc[j] + p0 + bpoff[j]),
                                             (lds_void_t *)(dst + 1024 * u), 16, 0, 0);
        }
    };
    // the lane's counts: row xrow0 + 16 s + lr, pixels (KS / 4) lg (+ 8 per load)
    const T *xrow[RB];
#pragma unroll
    for (int s = 0; s < RB; ++s) {
        const int64_t t = f0 + xrow0 + 16 * s + lr;
        xrow[s] = X + (t < N ? t : N - 1) * M;
    }
    typedef typename std::conditional<(sizeof(T) == 1 && KS == 32), int2, i32x4>::type XV;
    auto load_x = [&](int step, XV (&x)[RB][NL]) {
        const int64_t p0 = p_begin + (int64_t)KS * step;
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            int64_t px = p0 + (KS / 4) * lg + i * (16 / (int)sizeof(T));
            if (px >= M) px = p_begin;
#pragma unroll
            for (int s = 0; s < RB; ++s) x[s][i] = *reinterpret_cast<const XV *>(xrow[s] + px);
        }
    };

    f32x4 acc[RB][NCB + NIB];
#pragma unroll
    for (int s = 0; s < RB; ++s)
#pragma unroll
        for (int c = 0; c < NCB + NIB; ++c) acc[s][c] = (f32x4){0.f, 0.f, 0.f, 0.f};

    auto compute = [&](const unsigned char *cur, const XV (&x)[RB][NL]) {
        const unsigned short *bs = reinterpret_cast<const unsigned short *>(cur);
#pragma unroll
        for (int kk = 0; kk < kKK; ++kk) {
            const int q = (KS / 4) * lg + 8 * kk;
            typename Counts8<T>::type xr[RB];
#pragma unroll
            for (int s = 0; s < RB; ++s) {
                if constexpr (sizeof(T) == 1 && KS == 64) {
                    const i32x4 v = x[s][0];
                    xr[s] = kk ? int2{v[2], v[3]} : int2{v[0], v[1]};
                } else if constexpr (sizeof(T) == 1) {
                    xr[s] = x[s][0];
                } else {
                    xr[s] = x[s][kk];
                }
            }
            auto mma = [&](const u16x8 (&a)[RB]) {
#pragma unroll
                for (int c = 0; c < NCB; ++c) {
                    const int rh = 16 * c + lr;
                    const u16x8 bh = *reinterpret_cast<const u16x8 *>(bs + rh * KS + 8 * dma_slot<BP>(rh, q / 8));
#pragma unroll
                    for (int s = 0; s < RB; ++s) acc[s][c] = mfma_bf16(a[s], bh, acc[s][c]);
                    if constexpr (LO) {
                        const int rl = 16 * (NCB + c) + lr;
                        const u16x8 bl = *reinterpret_cast<const u16x8 *>(bs + rl * KS + 8 * dma_slot<BP>(rl, q / 8));
#pragma unroll
                        for (int s = 0; s < RB; ++s) acc[s][c] = mfma_bf16(a[s], bl, acc[s][c]);
                    }
                }
#pragma unroll
                for (int ib = 0; ib < NIB; ++ib) {
                    const int ri = 16 * (NCB * (LO ? 2 : 1) + ib) + lr;
                    const u16x8 bi = *reinterpret_cast<const u16x8 *>(bs + ri * KS + 8 * dma_slot<BP>(ri, q / 8));
#pragma unroll
                    for (int s = 0; s < RB; ++s) acc[s][NCB + ib] = mfma_bf16(a[s], bi, acc[s][NCB + ib]);
                }
            };
            u16x8 a[RB];
#pragma unroll
            for (int s = 0; s < RB; ++s) a[s] = Counts8<T>::plane0(xr[s]);
            mma(a);
            if constexpr (sizeof(T) == 2) {
                bool big = false;
#pragma unroll
                for (int s = 0; s < RB; ++s) big |= Counts8<T>::any_high(xr[s]);
                if (__ballot(big)) {
#pragma unroll
                    for (int s = 0; s < RB; ++s) a[s] = Counts8<T>::plane1(xr[s]);
                    mma(a);
                }
            }
        }
    };
    // Step s: wait until this wave's rows of step s have landed (with them its counts,
    // issued before them; the counts and rows of step s + 1 stay in flight), barrier,
    // start the counts and then the rows of step s + 2 (the last step's repeated past
    // the end, so that the count in flight is fixed), multiply step s.
    XV x0[RB][NL], x1[RB][NL], x2[RB][NL];
    auto sub = [&](int step, const unsigned char *cur, unsigned char *nxt, const XV (&xc)[RB][NL], XV (&xn)[RB][NL]) {
        asm volatile("" ::: "memory");
        wait_vmcnt<S::NXL + UPW>();
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        const int ahead = step + 2 < nsteps ? step + 2 : nsteps - 1;
        load_x(ahead, xn);
        asm volatile("" ::: "memory");
        issue_b(ahead, nxt);
        if (step < nsteps) compute(cur, xc);
    };
    if (nsteps > 0) {
        load_x(0, x0);
        asm volatile("" ::: "memory");
        issue_b(0, st0);
        asm volatile("" ::: "memory");
        load_x(nsteps > 1 ? 1 : 0, x1);
        asm volatile("" ::: "memory");
        issue_b(nsteps > 1 ? 1 : 0, st1);
        for (int step = 0; step < nsteps; step += 3) {
            sub(step, st0, st2, x0, x2);
            sub(step + 1, st1, st0, x1, x0);
            sub(step + 2, st2, st1, x2, x1);
        }
        wait_vmcnt<0>();
    }
    float *pdst = part + (int64_t)ch * N * ncols;
#pragma unroll
    for (int s = 0; s < RB; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t t = f0 + xrow0 + 16 * s + 4 * lg + i;
            if (t < N) {
#pragma unroll
                for (int c = 0; c < NCB + NIB; ++c) pdst[t * ncols + 16 * c + lr] = acc[s][c][i];
            }
        }
}

// Largest B row blocks of one launch (hi + lo + indicator blocks); wider passes are
// split over column groups by the launcher.
constexpr int kDmaMaxBlocks = 13;

// Shape of an instance, by its register budget (two waves per SIMD): four row
// blocks per wave (64 frames: each staged B fragment feeds four MFMAs) where the
// accumulators leave room, and a K step of 64 pixels where the counts in flight
// (three steps, 16 bytes per load) fit beside them, else 32.
template <typename T, int NCB, int NIB, bool LO>
struct DmaPick {
    static constexpr int NB = NCB + NIB;                       // accumulator blocks
    static constexpr int RB = 16 * NB + 48 <= 200 ? 4 : 2;
    static constexpr int NL64 = sizeof(T) == 2 ? 2 : 1;        // count loads per row block at KS = 64
    static constexpr int KS = 4 * RB * NB + 12 * RB * NL64 <= 200 ? 64 : 32;
};

// One launch over nchunks pixel chunks x the frame blocks of this instance.
template <typename T, int NCB, int NIB, bool LO>
void launch_pf_dma(int64_t nchunks, hipStream_t st, const void *X, int64_t M, int64_t N, const unsigned short *qh,
                   const unsigned short *ql, const unsigned short *ind, int64_t ldq, int64_t chunk, int ncols,
                   float *part) {
    constexpr int RB = DmaPick<T, NCB, NIB, LO>::RB, KS = DmaPick<T, NCB, NIB, LO>::KS;
    const int nfb = (int)((N + RB * 64 - 1) / (RB * 64));
    hipLaunchKernelGGL((proj_frames_dma_kernel<T, RB, NCB, NIB, LO, KS>), dim3((unsigned)(nfb * nchunks)), dim3(256),
                       0, st, static_cast<const T *>(X), M, N, qh, ql, ind, ldq, chunk, nfb, ncols, part);
}

template <typename T, int NIB, bool LO>
bool dispatch_pf_dma_ncb(int ncb, int64_t nchunks, hipStream_t st, const void *X, int64_t M, int64_t N,
                         const unsigned short *qh, const unsigned short *ql, const unsigned short *ind, int64_t ldq,
                         int64_t chunk, int ncols, float *part) {
    switch (ncb) {
#define XPCS_PFD(n)                                                                                         \
    case n:                                                                                                 \
        if constexpr (n * (LO ? 2 : 1) + NIB <= (LO ? kDmaMaxBlocks : 12)) {                                \
            launch_pf_dma<T, n, NIB, LO>(nchunks, st, X, M, N, qh, ql, ind, ldq, chunk, ncols, part);       \
            return true;                                                                                    \
        }                                                                                                   \
        return false;
        XPCS_PFD(1) XPCS_PFD(2) XPCS_PFD(3) XPCS_PFD(4) XPCS_PFD(5) XPCS_PFD(6)
        XPCS_PFD(7) XPCS_PFD(8) XPCS_PFD(9) XPCS_PFD(10) XPCS_PFD(11) XPCS_PFD(12)
#undef XPCS_PFD
        default:
            return false;
    }
}

// Passes without the residual term carry no indicator blocks; with it, 0..4.
template <typename T>
bool dispatch_pf_dma(int ncb, int nib, bool lo, int64_t nchunks, hipStream_t st, const void *X, int64_t M, int64_t N,
                     const unsigned short *qh, const unsigned short *ql, const unsigned short *ind, int64_t ldq,
                     int64_t chunk, int ncols, float *part) {
    if (!lo)
        return nib == 0 &&
               dispatch_pf_dma_ncb<T, 0, false>(ncb, nchunks, st, X, M, N, qh, ql, ind, ldq, chunk, ncols, part);
    switch (nib) {
        case 0: return dispatch_pf_dma_ncb<T, 0, true>(ncb, nchunks, st, X, M, N, qh, ql, ind, ldq, chunk, ncols, part);
        case 1: return dispatch_pf_dma_ncb<T, 1, true>(ncb, nchunks, st, X, M, N, qh, ql, ind, ldq, chunk, ncols, part);
        case 2: return dispatch_pf_dma_ncb<T, 2, true>(ncb, nchunks, st, X, M, N, qh, ql, ind, ldq, chunk, ncols, part);
        case 3: return dispatch_pf_dma_ncb<T, 3, true>(ncb, nchunks, st, X, M, N, qh, ql, ind, ldq, chunk, ncols, part);
        case 4: return dispatch_pf_dma_ncb<T, 4, true>(ncb, nchunks, st, X, M, N, qh, ql, ind, ldq, chunk, ncols, part);
        default: return false;
    }
}

// Instantiated once per count type in its own translation unit.
bool dispatch_pf_dma_u8(int ncb, int nib, bool lo, int64_t nchunks, hipStream_t st, const void *X, int64_t M, int64_t N,
                        const unsigned short *qh, const unsigned short *ql, const unsigned short *ind, int64_t ldq,
                        int64_t chunk, int ncols, float *part);
bool dispatch_pf_dma_u16(int ncb, int nib, bool lo, int64_t nchunks, hipStream_t st, const void *X, int64_t M, int64_t N,
                         const unsigned short *qh, const unsigned short *ql, const unsigned short *ind, int64_t ldq,
                         int64_t chunk, int ncols, float *part);

}  // namespace proj
}  // namespace xpcs
