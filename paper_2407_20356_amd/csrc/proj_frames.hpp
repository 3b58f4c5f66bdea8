// Frame-space product part[c][t][j] = sum_{p in chunk c} X[t][p] Q[j][p] (the
// basis passes X^T Q of Sec. 2.1 and the encoding W = X^T U of Eq. 7), with the
// ROI indicator columns j = L + r (label[p] == r) riding along so that the exact
// ROI sums S_R[t] come out of the same pass.
//
// A lane loads 8 adjacent pixels of one frame, which is directly an MFMA K group.
// The pixel range is split into chunks (partial sums reduced afterwards in a
// fixed order); blocks sharing a chunk are placed on the same XCD so that the
// chunk's slice of Q stays in that XCD's L2.  Each K step of Q (hi and lo) and of
// the indicator rows (built from the labels) is staged in LDS.
#pragma once

#include "proj_common.hpp"

namespace xpcs {
namespace proj {

// Row blocks per wave (frames per wave / 16): four when the accumulators stay
// small, else two (register budget).
constexpr int pf_rb(int ncb, int nib, bool lo) { return (lo ? 2 * ncb : ncb) + nib <= 8 ? 4 : 2; }

// The K step is KS = 32 or 64 pixels (KS / 32 MFMA K groups per lane: pixels
// (KS / 4) lg .. + KS / 4), so that the four lanes of a frame row read KS * sizeof(T)
// contiguous bytes per step: 128 bytes of u16 counts at KS = 64, which the memory
// system serves better than 64-byte pieces; KS = 32 where the staged operands of a
// wide basis would cost the occupancy.
template <int KS>
struct KStep {
    static constexpr int kPitch = KS + 8;            // LDS row pitch (u16): conflict-free fragment reads
    static constexpr int kParts = KS / 8;            // 16-byte pieces per staged row
    static constexpr int kGroups = KS / 32;          // MFMA K groups per lane and step
};

template <int KS>
__device__ __forceinline__ u16x8 lds_frag_k(const unsigned short *base, int row, int lg, int kk) {
    return *reinterpret_cast<const u16x8 *>(base + row * KStep<KS>::kPitch + (KS / 4) * lg + 8 * kk);
}

// One K step of a bf16 row-major operand (rows j < 16*NCB), held in registers
// between its global load and its LDS store; every thread issues the same loads.
template <int NCB, int KS>
struct StageK {
    static constexpr int kParts = KStep<KS>::kParts;
    static constexpr int kUnits = NCB * 16 * kParts;      // 16-byte units per K step
    static constexpr int kPer = (kUnits + 255) / 256;
    i32x4 r[kPer];
    __device__ __forceinline__ void load(const unsigned short *__restrict__ src, int64_t ld, int64_t k0) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            int u = threadIdx.x + 256 * i;
            if (kUnits % 256) u = u < kUnits ? u : kUnits - 1;
            r[i] = *reinterpret_cast<const i32x4 *>(src + (int64_t)(u / kParts) * ld + k0 + 8 * (u % kParts));
        }
    }
    __device__ __forceinline__ void store(unsigned short *dst) const {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int u = threadIdx.x + 256 * i;
            if (u < kUnits) *reinterpret_cast<i32x4 *>(dst + (u / kParts) * KStep<KS>::kPitch + 8 * (u % kParts)) = r[i];
        }
    }
};

// K step of an instance: 64 unless the accumulators and staged operands are wide.
constexpr int pf_kstep(int rb, int ncb, int nib, bool lo) {
    return (rb * (ncb + nib) <= 20 && ncb * (lo ? 2 : 1) <= 12) ? 64 : 32;
}

// K steps of counts in flight beyond the one being multiplied.
template <typename T>
constexpr int pf_depth(int rb, int ncb, int nib, bool lo) {
    return 1;
}

// VEC: M is a multiple of 8 and X and the labels are aligned, so each 8-pixel group
// of a lane is all inside or all outside the chunk; every lane then issues the same
// vector loads (groups past the chunk end read the chunk's first pixels and meet
// zero rows of Q and label -1; frames past N read frame N-1 and their outputs are
// dropped), which keeps the count of loads in flight fixed.
template <typename T, int RB, int NCB, int NIB, bool LO, bool VEC, int KS, int D>
__global__ __launch_bounds__(256) void proj_frames_kernel(const T *__restrict__ X, int64_t M, int64_t N,
                                                          const unsigned short *__restrict__ qh,
                                                          const unsigned short *__restrict__ ql,
                                                          int64_t ldq, const int32_t *__restrict__ labels,
                                                          int64_t chunk, int nfb, int ncols,
                                                          float *__restrict__ part) {
    typedef typename Counts8<T>::type PK;
    constexpr int FB = RB * 16 * 4;       // frames per block
    constexpr int kP = KStep<KS>::kPitch, kParts = KStep<KS>::kParts, kKK = KStep<KS>::kGroups;
    constexpr int kIndRows = NIB * 16;                     // indicator rows (one per ROI slot)
    constexpr int kRowsPerPass = 256 / kParts;
    constexpr int kIndPer = (kIndRows + kRowsPerPass - 1) / kRowsPerPass;   // rows built per thread
    __shared__ unsigned short sqh[2][NCB * 16 * kP];
    __shared__ unsigned short sql[LO ? 2 : 1][LO ? NCB * 16 * kP : 1];
    __shared__ unsigned short sind[NIB ? 2 : 1][NIB ? NIB * 16 * kP : 1];
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
    const int nsteps = p_end > p_begin ? (int)((p_end - p_begin + KS - 1) / KS) : 0;

    // x[s][kk]: the lane's pixels p0 + (KS / 4) lg + 8 kk .. + 8 of row block s
    auto load_x = [&](int64_t p0, PK (&x)[RB][kKK]) {
#pragma unroll
        for (int kk = 0; kk < kKK; ++kk) {
            const int64_t pl = p0 + (KS / 4) * lg + 8 * kk;
            if constexpr (VEC) {
                const int64_t pc = pl < p_end ? pl : p_begin;
#pragma unroll
                for (int s = 0; s < RB; ++s) x[s][kk] = *reinterpret_cast<const PK *>(xrow[s] + pc);
            } else {
                const int nv = pl >= p_end ? 0 : (p_end - pl >= 8 ? 8 : (int)(p_end - pl));
#pragma unroll
                for (int s = 0; s < RB; ++s)
                    x[s][kk] = (rok[s] && nv > 0) ? load8_partial<T>(xrow[s] + pl, nv) : PK{};
            }
        }
    };
    // Indicator rows: thread (row group tid / parts, part tid % parts) builds rows
    // tid / parts + (256 / parts) q over pixels 8 part .. + 8 of the K step, from the
    // 8 labels it loaded.
    const int ipart = threadIdx.x % kParts, irow0 = threadIdx.x / kParts;
    struct StageRegs {
        StageK<NCB, KS> h;
        StageK<LO ? NCB : 1, KS> l;
        i32x4 lab[2];
    };
    auto stage_load = [&](int64_t p0, StageRegs &r) {
        r.h.load(qh, ldq, p0);
        if constexpr (LO) r.l.load(ql, ldq, p0);
        if constexpr (NIB > 0) {
            const int64_t pl = p0 + 8 * ipart;
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
#pragma unroll
        for (int q = 0; q < kIndPer; ++q) {
            const int want = irow0 + kRowsPerPass * q;   // ROI of this indicator row
            if (want < kIndRows) {
                i32x4 w;
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const int l0 = d < 2 ? r.lab[0][2 * d] : r.lab[1][2 * d - 4];
                    const int l1 = d < 2 ? r.lab[0][2 * d + 1] : r.lab[1][2 * d - 3];
                    w[d] = (int)((l0 == want ? (unsigned)kBfOne : 0u) | ((l1 == want ? (unsigned)kBfOne : 0u) << 16));
                }
                *reinterpret_cast<i32x4 *>(&sind[b][want * kP + 8 * ipart]) = w;
            }
        }
    };
    auto mma = [&](const u16x8 (&a)[RB], int b, int kk) {
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
            const u16x8 bh = lds_frag_k<KS>(sqh[b], 16 * c + lr, lg, kk);
#pragma unroll
            for (int s = 0; s < RB; ++s) acc[s][c] = mfma_bf16(a[s], bh, acc[s][c]);
            if constexpr (LO) {
                const u16x8 bl = lds_frag_k<KS>(sql[b], 16 * c + lr, lg, kk);
#pragma unroll
                for (int s = 0; s < RB; ++s) acc[s][c] = mfma_bf16(a[s], bl, acc[s][c]);
            }
        }
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib) {
            const u16x8 bi = lds_frag_k<KS>(sind[b], 16 * ib + lr, lg, kk);
#pragma unroll
            for (int s = 0; s < RB; ++s) acc[s][NCB + ib] = mfma_bf16(a[s], bi, acc[s][NCB + ib]);
        }
    };
    auto multiply = [&](const PK (&xc)[RB][kKK], int b) {
#pragma unroll
        for (int kk = 0; kk < kKK; ++kk) {
            u16x8 a[RB];
#pragma unroll
            for (int s = 0; s < RB; ++s) a[s] = Counts8<T>::plane0(xc[s][kk]);
            mma(a, b, kk);
        }
        if constexpr (sizeof(T) == 2) {
            bool big = false;
#pragma unroll
            for (int s = 0; s < RB; ++s)
#pragma unroll
                for (int kk = 0; kk < kKK; ++kk) big |= Counts8<T>::any_high(xc[s][kk]);
            if (__ballot(big)) {
#pragma unroll
                for (int kk = 0; kk < kKK; ++kk) {
                    u16x8 a[RB];
#pragma unroll
                    for (int s = 0; s < RB; ++s) a[s] = Counts8<T>::plane1(xc[s][kk]);
                    mma(a, b, kk);
                }
            }
        }
    };

    // The counts of D K steps beyond the one being multiplied are in flight in
    // registers; the staged operands are loaded one step ahead and written to the
    // other LDS buffer after the current step's MFMAs.  Loads are issued every step
    // (the last step's repeated at the end) so that their number never varies.
    if (nsteps > 0) {
        StageRegs sr;
        PK xr[D + 1][RB][kKK];
#pragma unroll
        for (int i = 0; i < D; ++i) load_x(p_begin + KS * (int64_t)(i < nsteps ? i : nsteps - 1), xr[i]);
        stage_load(p_begin, sr);
        stage_store(sr, 0);
        __syncthreads();
        for (int step0 = 0; step0 < nsteps; step0 += D + 1) {
#pragma unroll
            for (int j = 0; j <= D; ++j) {
                const int step = step0 + j;
                if (step >= nsteps) break;
                const int ahead = step + D < nsteps ? step + D : nsteps - 1;
                load_x(p_begin + KS * (int64_t)ahead, xr[(j + D) % (D + 1)]);
                stage_load(p_begin + KS * (int64_t)(step + 1 < nsteps ? step + 1 : step), sr);
                multiply(xr[j], step & 1);
                if (step + 1 < nsteps) stage_store(sr, (step + 1) & 1);
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
    constexpr int KS = pf_kstep(RB, NCB, NIB, LO);
    constexpr int D = pf_depth<T>(RB, NCB, NIB, LO);
    if (vec)
        hipLaunchKernelGGL((proj_frames_kernel<T, RB, NCB, NIB, LO, true, KS, D>), dim3(nblocks), dim3(256), 0, st,
                           static_cast<const T *>(X), M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part);
    else
        hipLaunchKernelGGL((proj_frames_kernel<T, RB, NCB, NIB, LO, false, KS, D>), dim3(nblocks), dim3(256), 0, st,
                           static_cast<const T *>(X), M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part);
}

template <typename T, int NIB, bool LO>
bool dispatch_pf_ncb(int ncb, int nblocks, hipStream_t st, const void *X, int64_t M, int64_t N,
                     const unsigned short *qh, const unsigned short *ql, int64_t ldq, const int32_t *labels,
                     int64_t chunk, int nfb, int ncols, float *part, bool vec) {
    switch (ncb) {
#define XPCS_PF(n)                                                                                     \
    case n:                                                                                            \
        launch_pf<T, pf_rb(n, NIB, LO), n, NIB, LO>(nblocks, st, X, M, N, qh, ql, ldq, labels, chunk,   \
                                                    nfb, ncols, part, vec);                            \
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
