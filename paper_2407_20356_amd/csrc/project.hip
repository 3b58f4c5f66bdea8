// Products of the count matrix X with thin dense matrices on BF16 MFMA.
//
// These are the passes over the raw frames that build and apply the encoding
// basis (Sec. 2.1, Eqs. 3-7): Y = X Omega, Z = X^T Q, Y = X Z, W = X^T Q.  They
// read X once each and are bound by HBM bandwidth: a pass over a 2-byte count
// does 2*l flops per element, well under the BF16 MFMA ridge.
//
// Counts are integers, so bf16 holds them exactly up to 256; larger counts are
// carried as bf16 hi + lo (both exact), decided per wave and K step.
//
// X is stored frame-contiguous, X[t][p] = frames[t*M + p].
//  * proj_pixels contracts over frames (output per pixel).  A wave owns 16*RB
//    pixels, RB interleaved 16-row MFMA blocks (pixel = base + RB*row + s), so a
//    lane loads RB adjacent pixels of each of its 8 frames and every load of a
//    frame row is contiguous across the wave.
//  * proj_frames contracts over pixels (output per frame).  A lane loads 8
//    adjacent pixels of one frame, which is directly an MFMA K-group.  The pixel
//    range is split into chunks (partial sums reduced afterwards in a fixed
//    order); blocks sharing a chunk are placed on the same XCD so that the
//    chunk's slice of Q stays in that XCD's L2.
#include "internal.hpp"

namespace xpcs {
namespace {

constexpr unsigned short kBfOne = 0x3F80, kBfMinusOne = 0xBF80;

// ---------------------------------------------------------------- sketch
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void sketch_omega_kernel(uint64_t seed, int64_t N, int L, int ell, int64_t ldt,
                                    unsigned short *om) {
    const int64_t total = (int64_t)L * ldt;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = idx / ldt, t = idx % ldt;
        unsigned short v = 0;
        if (j < ell && t < N) {
            const uint64_t h = splitmix64(seed ^ (((uint64_t)t << 32) | (uint64_t)j));
            v = (h >> 63) ? kBfMinusOne : kBfOne;
        }
        om[idx] = v;
    }
}

// Integer count -> bf16 bits by truncation (exact for counts <= 256) and the
// exact remainder for larger counts.
__device__ __forceinline__ unsigned short count_hi_bits(unsigned v) {
    return (unsigned short)(__builtin_bit_cast(unsigned, (float)v) >> 16);
}
__device__ __forceinline__ unsigned short count_lo_bits(unsigned v) {
    const float hi = bf16_bits_to_f32(count_hi_bits(v));
    return (unsigned short)(__builtin_bit_cast(unsigned, (float)v - hi) >> 16);
}
// Two counts -> two packed bf16 (hi parts).
__device__ __forceinline__ unsigned pack_hi2(unsigned a, unsigned b) {
    const unsigned fa = __builtin_bit_cast(unsigned, (float)a), fb = __builtin_bit_cast(unsigned, (float)b);
    return (fb & 0xffff0000u) | (fa >> 16);
}

// 8 counts (one MFMA K group) held packed: 16 bytes for u16, 8 bytes for u8.
template <typename T>
struct Pack8;
template <>
struct Pack8<uint16_t> {
    typedef i32x4 type;
    static __device__ __forceinline__ unsigned get(const type &x, int e) {
        return (unsigned)(x[e >> 1] >> (16 * (e & 1))) & 0xffffu;
    }
    static __device__ __forceinline__ bool any_ge256(const type &x) {
        return ((x[0] | x[1] | x[2] | x[3]) & 0xff00ff00) != 0;
    }
};
template <>
struct Pack8<uint8_t> {
    typedef int2 type;
    static __device__ __forceinline__ unsigned get(const type &x, int e) {
        return (unsigned)((e < 4 ? x.x : x.y) >> (8 * (e & 3))) & 0xffu;
    }
    static __device__ __forceinline__ bool any_ge256(const type &) { return false; }
};

template <typename T>
__device__ __forceinline__ u16x8 pack8_to_bf16(const typename Pack8<T>::type &x) {
    i32x4 r;
#pragma unroll
    for (int w = 0; w < 4; ++w) r[w] = (int)pack_hi2(Pack8<T>::get(x, 2 * w), Pack8<T>::get(x, 2 * w + 1));
    return __builtin_bit_cast(u16x8, r);
}
template <typename T>
__device__ __forceinline__ u16x8 pack8_to_bf16_lo(const typename Pack8<T>::type &x) {
    u16x8 r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = count_lo_bits(Pack8<T>::get(x, e));
    return r;
}

// Load 8 consecutive counts src[0..8) (nv of them valid) as one packed K group.
template <typename T>
__device__ __forceinline__ typename Pack8<T>::type load8(const T *__restrict__ src, int nv, bool vec) {
    typedef typename Pack8<T>::type V;
    if (vec && nv == 8) return *reinterpret_cast<const V *>(src);
    unsigned v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = e < nv ? (unsigned)src[e] : 0u;
    V x;
    if constexpr (sizeof(T) == 2) {
#pragma unroll
        for (int w = 0; w < 4; ++w) x[w] = (int)(v[2 * w] | (v[2 * w + 1] << 16));
    } else {
        x.x = (int)(v[0] | (v[1] << 8) | (v[2] << 16) | (v[3] << 24));
        x.y = (int)(v[4] | (v[5] << 8) | (v[6] << 16) | (v[7] << 24));
    }
    return x;
}

// ---------------------------------------------------------------- LDS staging of the thin operand
// One 32-wide K step of a bf16 row-major operand (rows j < 16*NCB, K contiguous),
// staged as rows of kQp u16 (32 + 8 padding against bank conflicts).
constexpr int kQp = 40;

template <int NCB>
struct Stage16 {
    static constexpr int kUnits = NCB * 16 * 4;           // 16-byte units per K step
    static constexpr int kPer = (kUnits + 255) / 256;
    i32x4 r[kPer];
    // global rows src[j*ld + k0 + 8*part], j < 16*NCB
    __device__ __forceinline__ void load(const unsigned short *__restrict__ src, int64_t ld, int64_t k0) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int u = threadIdx.x + 256 * i;
            if (u < kUnits) r[i] = *reinterpret_cast<const i32x4 *>(src + (int64_t)(u >> 2) * ld + k0 + 8 * (u & 3));
        }
    }
    __device__ __forceinline__ void store(unsigned short *dst) const {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int u = threadIdx.x + 256 * i;
            if (u < kUnits) *reinterpret_cast<i32x4 *>(dst + (u >> 2) * kQp + 8 * (u & 3)) = r[i];
        }
    }
};

__device__ __forceinline__ u16x8 lds_frag(const unsigned short *base, int row, int lg) {
    return *reinterpret_cast<const u16x8 *>(base + row * kQp + 8 * lg);
}

// ---------------------------------------------------------------- pixel-space product
// Y[j][p] = sum_t X[t][p] * B[j][t], j in this block's column group (16*NCB columns).
// A wave owns 16*RB pixels as RB interleaved MFMA row blocks (pixel = base + RB*row
// + s); a lane loads RB adjacent pixels of 8 frames.  B's K step is staged in LDS.
template <typename T, int RB>
struct PixPack;
template <>
struct PixPack<uint16_t, 4> { typedef int2 type; };
template <>
struct PixPack<uint16_t, 2> { typedef int type; };
template <>
struct PixPack<uint8_t, 4> { typedef int type; };
template <>
struct PixPack<uint8_t, 2> { typedef unsigned short type; };

template <typename T, int RB>
__device__ __forceinline__ unsigned pix_get(const typename PixPack<T, RB>::type &x, int s) {
    if constexpr (sizeof(T) == 2 && RB == 4) return (unsigned)(((s < 2 ? x.x : x.y) >> (16 * (s & 1))) & 0xffff);
    else return (unsigned)((((unsigned long long)(unsigned)x) >> (8 * sizeof(T) * s)) & ((1u << (8 * sizeof(T))) - 1u));
}

template <typename T, int RB>
__device__ __forceinline__ typename PixPack<T, RB>::type load_pix(const T *__restrict__ src, int nvalid, bool vec) {
    typedef typename PixPack<T, RB>::type V;
    if (vec && nvalid == RB) return *reinterpret_cast<const V *>(src);
    unsigned long long acc = 0;
#pragma unroll
    for (int s = 0; s < RB; ++s)
        if (s < nvalid) acc |= (unsigned long long)src[s] << (8 * sizeof(T) * s);
    if constexpr (sizeof(T) == 2 && RB == 4) {
        int2 r;
        r.x = (int)(acc & 0xffffffffull);
        r.y = (int)(acc >> 32);
        return r;
    } else {
        return (V)acc;
    }
}

template <typename T, int RB, int NCB>
__global__ __launch_bounds__(256) void proj_pixels_kernel(const T *__restrict__ X, int64_t M, int64_t N,
                                                          const unsigned short *__restrict__ B, int64_t ldb,
                                                          float *__restrict__ Y, bool vec) {
    typedef typename PixPack<T, RB>::type PV;
    __shared__ unsigned short sb[2][NCB * 16 * kQp];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int jg = blockIdx.y * 16 * NCB;                  // column-group offset
    const int64_t pb = ((int64_t)blockIdx.x * 4 + wv) * (16 * RB);
    const int64_t pl = pb + RB * lr;                       // this lane's first pixel
    const int nvalid = pl >= M ? 0 : (M - pl >= RB ? RB : (int)(M - pl));
    const unsigned short *Bg = B + (int64_t)jg * ldb;

    f32x4 acc[RB][NCB];
#pragma unroll
    for (int s = 0; s < RB; ++s)
#pragma unroll
        for (int c = 0; c < NCB; ++c) acc[s][c] = (f32x4){0.f, 0.f, 0.f, 0.f};

    const int nsteps = (int)((N + 31) / 32);
    Stage16<NCB> st;
    st.load(Bg, ldb, 0);
    st.store(sb[0]);
    PV xn[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t t = 8 * lg + e;
        xn[e] = (t < N && nvalid > 0) ? load_pix<T, RB>(X + t * M + pl, nvalid, vec) : PV{};
    }
    __syncthreads();
    for (int step = 0; step < nsteps; ++step) {
        const int64_t tk = (int64_t)step * 32;
        PV xc[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) xc[e] = xn[e];
        const bool more = step + 1 < nsteps;
        if (more) {
            st.load(Bg, ldb, tk + 32);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int64_t t = tk + 32 + 8 * lg + e;
                xn[e] = (t < N && nvalid > 0) ? load_pix<T, RB>(X + t * M + pl, nvalid, vec) : PV{};
            }
        }
        const unsigned short *cur = sb[step & 1];
        bool big = false;
        if constexpr (sizeof(T) > 1) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
#pragma unroll
                for (int s = 0; s < RB; ++s) big |= pix_get<T, RB>(xc[e], s) > 255u;
        }
        // plane 0: bf16 of every count (exact below 256); plane 1, only when some
        // count of this K step is >= 256: the exact bf16 remainders.
#pragma unroll 1
        for (int plane = 0; plane < 2; ++plane) {
            if (plane == 1 && (sizeof(T) == 1 || !__ballot(big))) break;
#pragma unroll
            for (int s = 0; s < RB; ++s) {
                u16x8 a;
                if (plane == 0) {
                    i32x4 aw;
#pragma unroll
                    for (int w = 0; w < 4; ++w)
                        aw[w] = (int)pack_hi2(pix_get<T, RB>(xc[2 * w], s), pix_get<T, RB>(xc[2 * w + 1], s));
                    a = __builtin_bit_cast(u16x8, aw);
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) a[e] = count_lo_bits(pix_get<T, RB>(xc[e], s));
                }
#pragma unroll
                for (int c = 0; c < NCB; ++c) acc[s][c] = mfma_bf16(a, lds_frag(cur, 16 * c + lr, lg), acc[s][c]);
            }
        }
        if (more) st.store(sb[(step + 1) & 1]);
        __syncthreads();
    }
    // acc[s][c][i] = Y[j = jg + 16c + lr][p = pb + RB*(4*lg + i) + s]
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
        float *yrow = Y + (int64_t)(jg + 16 * c + lr) * M;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int s = 0; s < RB; ++s) {
                const int64_t p = pb + RB * (4 * lg + i) + s;
                if (p < M) yrow[p] = acc[s][c][i];
            }
        }
    }
}

// ---------------------------------------------------------------- frame-space product
// part[chunk][t][j] = sum_{p in chunk} X[t][p] * Q[j][p] for j < 16*NCB (hi [+ lo]),
// and for j = 16*NCB + i < 16*(NCB + NIB) the indicator (label[p] == i).
// Q's K step (and the labels) are staged in LDS; the next step's counts are
// loaded while the current step runs.
template <typename T, int RB, int NCB, int NIB, bool LO>
__global__ __launch_bounds__(256) void proj_frames_kernel(const T *__restrict__ X, int64_t M, int64_t N,
                                                          const unsigned short *__restrict__ qh,
                                                          const unsigned short *__restrict__ ql,
                                                          int64_t ldq, const int32_t *__restrict__ labels,
                                                          int64_t chunk, int nfb, int ncols,
                                                          float *__restrict__ part, bool vec) {
    typedef typename Pack8<T>::type PK;
    constexpr int FB = RB * 16 * 4;       // frames per block
    __shared__ unsigned short sqh[2][NCB * 16 * kQp];
    __shared__ unsigned short sql[LO ? 2 : 1][LO ? NCB * 16 * kQp : 1];
    __shared__ int slab[2][32];
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

    // lane row offsets (frames tb + 16s + lr) relative to the wave's first frame row
    const T *Xw = X + (tb < N ? tb : 0) * M;
    int xo[RB];
    bool rok[RB];
#pragma unroll
    for (int s = 0; s < RB; ++s) {
        rok[s] = tb + 16 * s + lr < N;
        xo[s] = rok[s] ? (16 * s + lr) * (int)M + 8 * lg : 0;
    }
    const int nsteps = p_end > p_begin ? (int)((p_end - p_begin + 31) / 32) : 0;
    Stage16<NCB> sth, stl;
    int labv = -1;
    auto stage_load = [&](int64_t p0) {
        sth.load(qh, ldq, p0);
        if constexpr (LO) stl.load(ql, ldq, p0);
        if constexpr (NIB > 0) {
            if (threadIdx.x < 32) labv = p0 + threadIdx.x < p_end ? labels[p0 + threadIdx.x] : -1;
        }
    };
    auto stage_store = [&](int b) {
        sth.store(sqh[b]);
        if constexpr (LO) stl.store(sql[b]);
        if constexpr (NIB > 0) {
            if (threadIdx.x < 32) slab[b][threadIdx.x] = labv;
        }
    };
    auto load_x = [&](int64_t p0, PK (&x)[RB]) {
        const int64_t pl = p0 + 8 * lg;
        const int nv = pl >= p_end ? 0 : (p_end - pl >= 8 ? 8 : (int)(p_end - pl));
#pragma unroll
        for (int s = 0; s < RB; ++s) x[s] = (rok[s] && nv > 0) ? load8<T>(Xw + xo[s] + p0, nv, vec) : PK{};
    };

    PK xn[RB];
    if (nsteps > 0) {
        stage_load(p_begin);
        stage_store(0);
        load_x(p_begin, xn);
    }
    __syncthreads();
    for (int step = 0; step < nsteps; ++step) {
        const int64_t p0 = p_begin + (int64_t)step * 32;
        PK xc[RB];
#pragma unroll
        for (int s = 0; s < RB; ++s) xc[s] = xn[s];
        const bool more = step + 1 < nsteps;
        if (more) {
            stage_load(p0 + 32);
            load_x(p0 + 32, xn);
        }
        const int b = step & 1;
        bool big = false;
#pragma unroll
        for (int s = 0; s < RB; ++s) big |= Pack8<T>::any_ge256(xc[s]);
        // plane 0: bf16 of every count (exact below 256); plane 1, only when some
        // count of this K step is >= 256: the exact bf16 remainders.
#pragma unroll 1
        for (int plane = 0; plane < 2; ++plane) {
            if (plane == 1 && (sizeof(T) == 1 || !__ballot(big))) break;
            u16x8 a[RB];
#pragma unroll
            for (int s = 0; s < RB; ++s) a[s] = plane == 0 ? pack8_to_bf16<T>(xc[s]) : pack8_to_bf16_lo<T>(xc[s]);
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
            if constexpr (NIB > 0) {
                int lab[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) lab[e] = slab[b][8 * lg + e];
#pragma unroll
                for (int ib = 0; ib < NIB; ++ib) {
                    u16x8 ind;
                    const int want = 16 * ib + lr;
#pragma unroll
                    for (int e = 0; e < 8; ++e) ind[e] = lab[e] == want ? kBfOne : (unsigned short)0;
#pragma unroll
                    for (int s = 0; s < RB; ++s) acc[s][NCB + ib] = mfma_bf16(a[s], ind, acc[s][NCB + ib]);
                }
            }
        }
        if (more) stage_store(b ^ 1);
        __syncthreads();
    }
    // acc[s][c][i] = part[ch][t = tb + 16s + 4lg + i][j = 16c + lr]
    float *pc = part + (int64_t)ch * N * ncols;
#pragma unroll
    for (int s = 0; s < RB; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t t = tb + 16 * s + 4 * lg + i;
            if (t < N) {
#pragma unroll
                for (int c = 0; c < NCB + NIB; ++c) pc[t * ncols + 16 * c + lr] = acc[s][c][i];
            }
        }
}

__global__ void proj_frames_reduce_kernel(const float *__restrict__ part, int64_t nch, int64_t N, int ncols,
                                          int L, int n_ind, double *__restrict__ Z, int64_t ldz,
                                          int64_t *__restrict__ S) {
    const int64_t total = N * ncols;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = idx / ncols;
        const int j = (int)(idx % ncols);
        const bool isq = j < L;
        const bool isind = S && j >= L && j - L < n_ind;
        if (!isq && !isind) continue;
        double s = 0.0;
        for (int64_t c = 0; c < nch; ++c) s += (double)part[(c * N + t) * ncols + j];
        if (isq)
            Z[(int64_t)j * ldz + t] = s;
        else
            S[(int64_t)(j - L) * N + t] = (int64_t)__builtin_rint(s);
    }
}

// ---------------------------------------------------------------- dispatch helpers
template <typename T, int RB, int NCB>
void launch_pp(dim3 grid, hipStream_t st, const void *X, int64_t M, int64_t N, const unsigned short *B,
               int64_t ldb, float *Y, bool vec) {
    hipLaunchKernelGGL((proj_pixels_kernel<T, RB, NCB>), grid, dim3(256), 0, st,
                       static_cast<const T *>(X), M, N, B, ldb, Y, vec);
}

template <typename T>
bool dispatch_pp(int ncb, int &rb_out, int ngroups_cb, dim3 gridx, hipStream_t st, const void *X, int64_t M,
                 int64_t N, const unsigned short *B, int64_t ldb, float *Y, bool vec4, bool vec2) {
    (void)ngroups_cb;
    switch (ncb) {
#define XPCS_PP4(n)                                                                             \
    case n: {                                                                                   \
        rb_out = 4;                                                                             \
        dim3 g((unsigned)((M + 255) / 256), gridx.y);                                           \
        launch_pp<T, 4, n>(g, st, X, M, N, B, ldb, Y, vec4);                                    \
        return true;                                                                            \
    }
        XPCS_PP4(1) XPCS_PP4(2) XPCS_PP4(3) XPCS_PP4(4) XPCS_PP4(5) XPCS_PP4(6)
#undef XPCS_PP4
#define XPCS_PP2(n)                                                                             \
    case n: {                                                                                   \
        rb_out = 2;                                                                             \
        dim3 g((unsigned)((M + 127) / 128), gridx.y);                                           \
        launch_pp<T, 2, n>(g, st, X, M, N, B, ldb, Y, vec2);                                    \
        return true;                                                                            \
    }
        XPCS_PP2(7) XPCS_PP2(8) XPCS_PP2(9) XPCS_PP2(10) XPCS_PP2(11) XPCS_PP2(12)
#undef XPCS_PP2
        default:
            return false;
    }
}

template <typename T, int RB, int NCB, int NIB, bool LO>
void launch_pf(int nblocks, hipStream_t st, const void *X, int64_t M, int64_t N, const unsigned short *qh,
               const unsigned short *ql, int64_t ldq, const int32_t *labels, int64_t chunk, int nfb,
               int ncols, float *part, bool vec) {
    hipLaunchKernelGGL((proj_frames_kernel<T, RB, NCB, NIB, LO>), dim3(nblocks), dim3(256), 0, st,
                       static_cast<const T *>(X), M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
}

// Row blocks per wave (frames per wave / 16) as a function of the accumulator
// columns: four when the accumulators stay small, else two (register budget).
inline int pf_rb(int ncb, int nib, bool lo) { return (lo ? 2 * ncb : ncb) + nib <= 8 ? 4 : 2; }

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

template <typename T, bool LO>
bool dispatch_pf(int ncb, int nib, int nblocks, hipStream_t st, const void *X, int64_t M, int64_t N,
                 const unsigned short *qh, const unsigned short *ql, int64_t ldq, const int32_t *labels,
                 int64_t chunk, int nfb, int ncols, float *part, bool vec) {
    switch (nib) {
        case 0: return dispatch_pf_ncb<T, 0, LO>(ncb, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
        case 1: return dispatch_pf_ncb<T, 1, LO>(ncb, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
        case 2: return dispatch_pf_ncb<T, 2, LO>(ncb, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
        case 3: return dispatch_pf_ncb<T, 3, LO>(ncb, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
        case 4: return dispatch_pf_ncb<T, 4, LO>(ncb, nblocks, st, X, M, N, qh, ql, ldq, labels, chunk, nfb, ncols, part, vec);
        default: return false;
    }
}

}  // namespace

xpcs_status launch_sketch_omega(xpcs_ctx *ctx, uint64_t seed, int64_t N, int L, int ell, int64_t ldt,
                                unsigned short *om) {
    Phase phase_(ctx, "sketch_omega");
    int64_t total = (int64_t)L * ldt;
    int grid = (int)((total + 255) / 256);
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(sketch_omega_kernel, dim3(grid), dim3(256), 0, ctx->stream, seed, N, L, ell, ldt, om);
    XPCS_LAUNCH_CHECK(ctx, "sketch_omega");
    return XPCS_OK;
}

xpcs_status launch_proj_pixels(xpcs_ctx *ctx, const void *frames, int dtype, int64_t M, int64_t N,
                               const unsigned short *B, int64_t ldb, int L, float *Y) {
    Phase phase_(ctx, "proj_pixels");
    if (L % 16 || L <= 0) return fail(ctx, XPCS_EINVAL, "internal: L must be a positive multiple of 16");
    if (ldb % 32) return fail(ctx, XPCS_EINVAL, "internal: sketch row stride must be a multiple of 32");
    const int ncb_total = L / 16;
    // Column groups of at most 12 blocks (grid.y); all groups have the same size.
    int ngroups = (ncb_total + 11) / 12;
    while (ncb_total % ngroups) ++ngroups;
    const int ncb = ncb_total / ngroups;
    const size_t esz = dtype == XPCS_U8 ? 1 : 2;
    const bool vec4 = (M % 4 == 0) && ((uintptr_t)frames % (4 * esz) == 0);
    const bool vec2 = (M % 2 == 0) && ((uintptr_t)frames % (2 * esz) == 0);
    int rb = 0;
    dim3 g(1, (unsigned)ngroups);
    bool ok = dtype == XPCS_U8
                  ? dispatch_pp<uint8_t>(ncb, rb, ngroups, g, ctx->stream, frames, M, N, B, ldb, Y, vec4, vec2)
                  : dispatch_pp<uint16_t>(ncb, rb, ngroups, g, ctx->stream, frames, M, N, B, ldb, Y, vec4, vec2);
    if (!ok) return fail(ctx, XPCS_EUNSUPPORTED, "too many sketch columns for proj_pixels");
    XPCS_LAUNCH_CHECK(ctx, "proj_pixels");
    return XPCS_OK;
}

FrameProj plan_proj_frames(int64_t M, int64_t N, int L, int n_ind, bool lo) {
    FrameProj p;
    const int nib = (n_ind + 15) / 16;
    p.ncols = L + 16 * nib;
    const int rb = pf_rb(L / 16, nib, lo);
    const int64_t fbf = (int64_t)rb * 64;
    const int64_t nfb = (N + fbf - 1) / fbf;
    int64_t want = (2048 + nfb - 1) / nfb;                 // blocks ~ 2048
    if (want < 8) want = 8;
    int64_t chunk = (M + want - 1) / want;
    chunk = (chunk + 31) / 32 * 32;
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
    const int ncb = L / 16, nib = (n_ind + 15) / 16;
    if (nib > 4) return fail(ctx, XPCS_EUNSUPPORTED, "more than 64 ROIs in the fused ROI sums");
    const int rb = pf_rb(ncb, nib, q_lo != nullptr);
    if (rb * 64 != plan.frames_per_block)
        return fail(ctx, XPCS_EINVAL, "internal: projection plan made for another variant");
    const int64_t fbf = (int64_t)rb * 64;
    const int nfb = (int)((N + fbf - 1) / fbf);
    const int64_t nblocks = (int64_t)nfb * plan.nchunks;
    if (nblocks > 2147483647LL) return fail(ctx, XPCS_EUNSUPPORTED, "projection grid too large");
    const size_t esz = dtype == XPCS_U8 ? 1 : 2;
    const bool vec = (M % 8 == 0) && ((uintptr_t)frames % (8 * esz) == 0);
    bool ok;
    if (q_lo) {
        ok = dtype == XPCS_U8
                 ? dispatch_pf<uint8_t, true>(ncb, nib, (int)nblocks, ctx->stream, frames, M, N, q_hi, q_lo, ldq,
                                              labels, plan.chunk, nfb, plan.ncols, part, vec)
                 : dispatch_pf<uint16_t, true>(ncb, nib, (int)nblocks, ctx->stream, frames, M, N, q_hi, q_lo, ldq,
                                               labels, plan.chunk, nfb, plan.ncols, part, vec);
    } else {
        ok = dtype == XPCS_U8
                 ? dispatch_pf<uint8_t, false>(ncb, nib, (int)nblocks, ctx->stream, frames, M, N, q_hi, q_lo, ldq,
                                               labels, plan.chunk, nfb, plan.ncols, part, vec)
                 : dispatch_pf<uint16_t, false>(ncb, nib, (int)nblocks, ctx->stream, frames, M, N, q_hi, q_lo,
                                                ldq, labels, plan.chunk, nfb, plan.ncols, part, vec);
    }
    if (!ok) return fail(ctx, XPCS_EUNSUPPORTED, "too many basis columns for proj_frames");
    XPCS_LAUNCH_CHECK(ctx, "proj_frames");
    return XPCS_OK;
}

xpcs_status launch_proj_frames_reduce(xpcs_ctx *ctx, const float *part, const FrameProj &plan, int64_t N,
                                      int L, int n_ind, double *Z, int64_t ldz, int64_t *S) {
    Phase phase_(ctx, "proj_frames_reduce");
    int64_t total = N * plan.ncols;
    int grid = (int)((total + 255) / 256);
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(proj_frames_reduce_kernel, dim3(grid), dim3(256), 0, ctx->stream, part, plan.nchunks, N,
                       plan.ncols, L, n_ind, Z, ldz, S);
    XPCS_LAUNCH_CHECK(ctx, "proj_frames_reduce");
    return XPCS_OK;
}

}  // namespace xpcs
