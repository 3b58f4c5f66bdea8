// Frame-space product part[c][t][j] = sum_{p in chunk c} X[t][p] Q[j][p] (the
// basis passes X^T Q of Sec. 2.1 and the encoding W = X^T U of Eq. 7), with the
// ROI indicator columns j = L + r (label[p] == r) riding along so that the exact
// ROI sums S_R[t] come out of the same pass.
//
// A lane loads 8 adjacent pixels of one frame, which is directly an MFMA K group.
// The pixel range is split into chunks (partial sums reduced afterwards in a
// fixed order); blocks sharing a chunk are placed on the same XCD so that the
// chunk's slice of Q stays in that XCD's L2.  Each 32-pixel K step of Q (hi and
// lo) and of the indicator rows (built from the labels) is staged in LDS.
#pragma once

#include "proj_common.hpp"

namespace xpcs {
namespace proj {

// Row blocks per wave (frames per wave / 16): four when the accumulators stay
// small, else two (register budget).
inline int pf_rb(int ncb, int nib, bool lo) { return (lo ? 2 * ncb : ncb) + nib <= 8 ? 4 : 2; }

// VEC: M is a multiple of 8 and X and the labels are aligned, so a lane's 8 pixels are all
// inside or all outside the chunk; every lane then issues the same vector loads
// (pixels past the chunk end read the chunk's first pixels and meet zero rows of
// Q and label -1; frames past N read frame N-1 and their outputs are dropped),
// which keeps the count of loads in flight fixed.
template <typename T, int RB, int NCB, int NIB, bool LO, bool VEC>
__global__ __launch_bounds__(256) void proj_frames_kernel(const T *__restrict__ X, int64_t M, int64_t N,
                                                          const unsigned short *__restrict__ qh,
                                                          const unsigned short *__restrict__ ql,
                                                          int64_t ldq, const int32_t *__restrict__ labels,
                                                          int64_t chunk, int nfb, int ncols,
                                                          float *__restrict__ part) {
    typedef typename Counts8<T>::type PK;
    constexpr int FB = RB * 16 * 4;       // frames per block
    __shared__ unsigned short sqh[2][NCB * 16 * kQp];
    __shared__ unsigned short sql[LO ? 2 : 1][LO ? NCB * 16 * kQp : 1];
    __shared__ unsigned short sind[NIB ? 2 : 1][NIB ? NIB * 16 * kQp : 1];
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

    // frame row of each of the lane's RB row blocks
    const T *xrow[RB];
    bool rok[RB];
#pragma unroll
    for (int s = 0; s < RB; ++s) {
        const int64_t t = tb + 16 * s + lr;
        rok[s] = t < N;
        xrow[s] = X + (t < N ? t : N - 1) * M;
    }
    const int nsteps = p_end > p_begin ? (int)((p_end - p_begin + 31) / 32) : 0;

    // indicator rows of a K step: thread u < 64*NIB builds row u/4 (ROI 16*ib + u/4 % 16)
    // over pixels 8*(u%4) .. +8 from the labels it loaded
    const int iu = threadIdx.x < 64 * NIB ? threadIdx.x : 0;
    const int irow = iu >> 2, ipart = iu & 3;
    auto load_x = [&](int64_t p0, PK (&x)[RB]) {
        const int64_t pl = p0 + 8 * lg;
        if constexpr (VEC) {
            const int64_t pc = pl < p_end ? pl : p_begin;
#pragma unroll
            for (int s = 0; s < RB; ++s) x[s] = *reinterpret_cast<const PK *>(xrow[s] + pc);
        } else {
            const int nv = pl >= p_end ? 0 : (p_end - pl >= 8 ? 8 : (int)(p_end - pl));
#pragma unroll
            for (int s = 0; s < RB; ++s) x[s] = (rok[s] && nv > 0) ? load8_partial<T>(xrow[s] + pl, nv) : PK{};
        }
    };
    struct StageRegs {
        Stage16<NCB> h;
        Stage16<LO ? NCB : 1> l;
        i32x4 lab[2];
    };
    auto stage_load = [&](int64_t p0, StageRegs &r) {
        r.h.load(qh, ldq, p0);
        if constexpr (LO) r.l.load(ql, ldq, p0);
        if constexpr (NIB > 0) {
            const int64_t pl = p0 + 8 * ipart;     // this thread's 8 labels; -1 past the chunk
            if constexpr (VEC) {
                const bool in = pl < p_end;
                const i32x4 *src = reinterpret_cast<const i32x4 *>(labels + (in ? pl : p_begin));
                const i32x4 a = src[0], b = src[1], none = {-1, -1, -1, -1};
                r.lab[0] = in ? a : none;
                r.lab[1] = in ? b : none;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int v = pl + e < p_end ? labels[pl + e] : -1;
                    if (e < 4) r.lab[0][e] = v; else r.lab[1][e - 4] = v;
                }
            }
        }
    };
    auto stage_store = [&](const StageRegs &r, int b) {
        r.h.store(sqh[b]);
        if constexpr (LO) r.l.store(sql[b]);
        if constexpr (NIB > 0) {
            if (threadIdx.x < 64 * NIB) {
                const int want = irow;   // ROI of this indicator row
                i32x4 w;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int l0 = q < 2 ? r.lab[0][2 * q] : r.lab[1][2 * q - 4];
                    const int l1 = q < 2 ? r.lab[0][2 * q + 1] : r.lab[1][2 * q - 3];
                    w[q] = (int)((l0 == want ? (unsigned)kBfOne : 0u) | ((l1 == want ? (unsigned)kBfOne : 0u) << 16));
                }
                *reinterpret_cast<i32x4 *>(&sind[b][irow * kQp + 8 * ipart]) = w;
            }
        }
    };
    auto mma = [&](const u16x8 (&a)[RB], int b) {
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
            const u16x8 bh = lds_frag(sqh[b], 16 * c + lr, lg);
#pragma unroll
            for (int s = 0; s < RB; ++s) acc[s][c] = mfma_bf16(a[s], bh, acc[s][c]);
            if constexpr (LO) {
                const u16x8 bl = lds_frag(sql[b], 16 * c + lr, lg);
#pragma unroll
                for (int s = 0; s < RB; ++s) acc[s][c] = mfma_bf16(a[s], bl, acc[s][c]);
            }
        }
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib) {
            const u16x8 bi = lds_frag(sind[b], 16 * ib + lr, lg);
#pragma unroll
            for (int s = 0; s < RB; ++s) acc[s][NCB + ib] = mfma_bf16(a[s], bi, acc[s][NCB + ib]);
        }
    };
    auto multiply = [&](const PK (&xc)[RB], int b) {
        u16x8 a[RB];
#pragma unroll
        for (int s = 0; s < RB; ++s) a[s] = Counts8<T>::plane0(xc[s]);
        mma(a, b);
        if constexpr (sizeof(T) == 2) {
            bool big = false;
#pragma unroll
            for (int s = 0; s < RB; ++s) big |= Counts8<T>::any_high(xc[s]);
            if (__ballot(big)) {
#pragma unroll
                for (int s = 0; s < RB; ++s) a[s] = Counts8<T>::plane1(xc[s]);
                mma(a, b);
            }
        }
    };

    // One K step in flight beyond the one being multiplied (counts and the staged
    // operands in registers, the operands written to LDS one step before use).
    // Loads are issued every step (the last one repeated at the end) so that their
    // number never varies.
    if (nsteps > 0) {
        StageRegs sr[2];
        PK xr[2][RB];
        stage_load(p_begin, sr[0]);
        load_x(p_begin, xr[0]);
        stage_store(sr[0], 0);
        __syncthreads();
        for (int step0 = 0; step0 < nsteps; step0 += 2) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int step = step0 + j;
                if (step >= nsteps) break;
                const int64_t pn = p_begin + 32 * (int64_t)(step + 1 < nsteps ? step + 1 : step);
                stage_load(pn, sr[j ^ 1]);
                load_x(pn, xr[j ^ 1]);
                multiply(xr[j], step & 1);
                if (step + 1 < nsteps) stage_store(sr[j ^ 1], (step + 1) & 1);
                __syncthreads();
            }
        }
    }
    // acc[s][c][i] = part[ch][t = tb + 16s + 4lg + i][j = 16c + lr]
    float *pdst = part + (int64_t)ch * N * ncols;
#pragma unroll
    for (int s = 0; s < RB; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t t = tb + 16 * s + 4 * lg + i;
            if (t < N) {
#pragma unroll
                for (int c = 0; c < NCB + NIB; ++c) pdst[t * ncols + 16 * c + lr] = acc[s][c][i];
            }
        }
}

template <typename T, int RB, int NCB, int NIB, bool LO>
void launch_pf(int nblocks, hipStream_t st, const void *X, int64_t M, int64_t N, const unsigned short *qh,
               const unsigned short *ql, int64_t ldq, const int32_t *labels, int64_t chunk, int nfb,
               int ncols, float *part, bool vec) {
    if (vec)
        hipLaunchKernelGGL((proj_frames_kernel<T, RB, NCB, NIB, LO, true>), dim3(nblocks), dim3(256), 0, st,
                           static_cast<const T *>(X), M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part);
    else
        hipLaunchKernelGGL((proj_frames_kernel<T, RB, NCB, NIB, LO, false>), dim3(nblocks), dim3(256), 0, st,
                           static_cast<const T *>(X), M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part);
}

template <typename T, int NIB, bool LO>
bool dispatch_pf_ncb(int ncb, int nblocks, hipStream_t st, const void *X, int64_t M, int64_t N,
                     const unsigned short *qh, const unsigned short *ql, int64_t ldq, const int32_t *labels,
                     int64_t chunk, int nfb, int ncols, float *part, bool vec) {
    switch (ncb) {
#define XPCS_PF(n)                                                                                     \
    case n:                                                                                            \
        if (pf_rb(n, NIB, LO) == 4)                                                                    \
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

// The passes without the residual term of Q carry no indicator columns; the
// passes with it carry 1..4 blocks of 16.
template <typename T>
bool dispatch_pf(int ncb, int nib, bool lo, int nblocks, hipStream_t st, const void *X, int64_t M, int64_t N,
                 const unsigned short *qh, const unsigned short *ql, int64_t ldq, const int32_t *labels,
                 int64_t chunk, int nfb, int ncols, float *part, bool vec) {
    if (!lo)
        return nib == 0 &&
               dispatch_pf_ncb<T, 0, false>(ncb, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
    switch (nib) {
        case 1: return dispatch_pf_ncb<T, 1, true>(ncb, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
        case 2: return dispatch_pf_ncb<T, 2, true>(ncb, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
        case 3: return dispatch_pf_ncb<T, 3, true>(ncb, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
        case 4: return dispatch_pf_ncb<T, 4, true>(ncb, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
        default: return false;
    }
}

// Instantiated once per count type in its own translation unit.
bool dispatch_pf_u8(int ncb, int nib, bool lo, int nblocks, hipStream_t st, const void *X, int64_t M, int64_t N,
                    const unsigned short *qh, const unsigned short *ql, int64_t ldq, const int32_t *labels,
                    int64_t chunk, int nfb, int ncols, float *part, bool vec);
bool dispatch_pf_u16(int ncb, int nib, bool lo, int nblocks, hipStream_t st, const void *X, int64_t M, int64_t N,
                     const unsigned short *qh, const unsigned short *ql, int64_t ldq, const int32_t *labels,
                     int64_t chunk, int nfb, int ncols, float *part, bool vec);

}  // namespace proj
}  // namespace xpcs
