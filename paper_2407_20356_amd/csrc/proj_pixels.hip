// The pixel-space product Y = X B of the power pass (Sec. 2.1: X Z, Z the
// orthonormalised frame-space product).  X is stored frame-contiguous,
// X[t][p] = frames[t*M + p]; the product contracts over frames and is bound by
// HBM bandwidth (2*l flops per 1- or 2-byte count, well under the BF16 ridge).
//
// A wave owns 16*RB pixels as RB interleaved MFMA row blocks (pixel = base +
// RB*row + s), so a lane loads RB adjacent pixels of each of its 8 frames and
// every load of a frame row is contiguous across the wave.  B's K step (32
// frames) is staged in LDS.
#include "proj_common.hpp"

namespace xpcs {
namespace {

using namespace proj;

// ---------------------------------------------------------------- pixel-space product
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

__device__ __forceinline__ bool pv_any_high(const int2 &x) { return ((x.x | x.y) & 0xff00ff00) != 0; }
__device__ __forceinline__ bool pv_any_high(const int &x) { return (x & 0xff00ff00) != 0; }
__device__ __forceinline__ int2 pv_opaque(int2 x) {
    unsigned a = (unsigned)x.x, b = (unsigned)x.y;
    opaque(a);
    opaque(b);
    return int2{(int)a, (int)b};
}
__device__ __forceinline__ int pv_opaque(int x) {
    unsigned a = (unsigned)x;
    opaque(a);
    return (int)a;
}

template <typename T, int RB>
__device__ __forceinline__ typename PixPack<T, RB>::type load_pix_partial(const T *__restrict__ src, int nvalid) {
    typedef typename PixPack<T, RB>::type V;
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

// Y[j][p] = sum_t X[t][p] * B[j][t], j in this block's column group (16*NCB columns).
// VEC: M is a multiple of RB and X is aligned, so a lane's RB pixels are all inside
// or all outside the detector; every lane then issues the same vector loads (lanes
// past M read pixel 0 and their outputs are dropped; frames past N read frame N-1
// and meet the zero rows of B), which keeps the count of loads in flight fixed.
template <typename T, int RB, int NCB, bool VEC, int KG, int D>
__global__ __launch_bounds__(256, sizeof(T) == 1 ? 2 : 1) void proj_pixels_kernel(const T *__restrict__ X, int64_t M, int64_t N,
                                                          const unsigned short *__restrict__ B, int64_t ldb,
                                                          float *__restrict__ Y) {
    typedef typename PixPack<T, RB>::type PV;
    __shared__ unsigned short sb[2][KG][NCB * 16 * kQp];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int jg = blockIdx.y * 16 * NCB;                  // column-group offset
    const int64_t pb = ((int64_t)blockIdx.x * 4 + wv) * (16 * RB);
    const int64_t pl = pb + RB * lr;                       // this lane's first pixel
    const int nvalid = pl >= M ? 0 : (M - pl >= RB ? RB : (int)(M - pl));
    const int64_t plc = pl < M ? pl : 0;
    const unsigned short *Bg = B + (int64_t)jg * ldb;

    f32x4 acc[RB][NCB];
#pragma unroll
    for (int s = 0; s < RB; ++s)
#pragma unroll
        for (int c = 0; c < NCB; ++c) acc[s][c] = (f32x4){0.f, 0.f, 0.f, 0.f};

    const int nsteps = (int)((N + 32 * KG - 1) / (32 * KG));
    auto load_group = [&](int64_t tk, PV (&x)[8]) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t t = tk + 8 * lg + e;
            if constexpr (VEC) {
                const int64_t tc = t < N ? t : N - 1;
                x[e] = *reinterpret_cast<const PV *>(X + tc * M + plc);
            } else {
                x[e] = (t < N && nvalid > 0) ? load_pix_partial<T, RB>(X + t * M + pl, nvalid) : PV{};
            }
        }
    };
    auto mma = [&](const u16x8 (&a)[RB], const unsigned short *cur) {
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
            const u16x8 b = lds_frag(cur, 16 * c + lr, lg);
#pragma unroll
            for (int s = 0; s < RB; ++s) acc[s][c] = mfma_bf16(a[s], b, acc[s][c]);
        }
    };
    auto multiply = [&](const PV (&xc)[8], const unsigned short *cur) {
        u16x8 a[RB];
#pragma unroll
        for (int s = 0; s < RB; ++s) {
            i32x4 aw;
#pragma unroll
            for (int w = 0; w < 4; ++w)
                aw[w] = (int)pack_bf16_pair((float)(pix_get<T, RB>(xc[2 * w], s) & 0xffu),
                                            (float)(pix_get<T, RB>(xc[2 * w + 1], s) & 0xffu));
            a[s] = __builtin_bit_cast(u16x8, aw);
        }
        mma(a, cur);
        if constexpr (sizeof(T) == 2) {
            bool big = false;
#pragma unroll
            for (int e = 0; e < 8; ++e) big |= pv_any_high(xc[e]);
            if (__ballot(big)) {
                PV xh[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) xh[e] = pv_opaque(xc[e]);
#pragma unroll
                for (int s = 0; s < RB; ++s) {
                    i32x4 aw;
#pragma unroll
                    for (int w = 0; w < 4; ++w)
                        aw[w] = (int)pack_bf16_pair((float)(pix_get<T, RB>(xh[2 * w], s) >> 8) * 256.f,
                                                    (float)(pix_get<T, RB>(xh[2 * w + 1], s) >> 8) * 256.f);
                    a[s] = __builtin_bit_cast(u16x8, aw);
                }
                mma(a, cur);
            }
        }
    };

    // The counts of D K steps (KG groups of 32 frames each) beyond the one being
    // multiplied are in flight in registers; B's next K step is loaded into
    // registers and written to the other LDS buffer after the current step's
    // MFMAs.  Loads are issued every step (the last step's repeated at the end) so
    // that their number never varies; frames past N meet B's zero columns.
    Stage16<NCB> st[KG];
    PV xr[D + 1][KG][8];
    auto load_x_step = [&](int step, PV (&x)[KG][8]) {
#pragma unroll
        for (int g = 0; g < KG; ++g) load_group(((int64_t)step * KG + g) * 32, x[g]);
    };
    auto load_b_step = [&](int step) {
#pragma unroll
        for (int g = 0; g < KG; ++g) st[g].load(Bg, ldb, ((int64_t)step * KG + g) * 32);   // < ldb: a multiple of 32 KG
    };
#pragma unroll
    for (int i = 0; i < D; ++i) load_x_step(i < nsteps ? i : nsteps - 1, xr[i]);
    load_b_step(0);
#pragma unroll
    for (int g = 0; g < KG; ++g) st[g].store(sb[0][g]);
    __syncthreads();
    for (int step0 = 0; step0 < nsteps; step0 += D + 1) {
#pragma unroll
        for (int j = 0; j <= D; ++j) {
            const int step = step0 + j;
            if (step >= nsteps) break;
            load_x_step(step + D < nsteps ? step + D : nsteps - 1, xr[(j + D) % (D + 1)]);
            load_b_step(step + 1 < nsteps ? step + 1 : step);
#pragma unroll
            for (int g = 0; g < KG; ++g) multiply(xr[j][g], sb[step & 1][g]);
            if (step + 1 < nsteps) {
#pragma unroll
                for (int g = 0; g < KG; ++g) st[g].store(sb[(step + 1) & 1][g]);
            }
            __syncthreads();
        }
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

// Groups of 32 frames per K step: one (two groups of one-byte counts, with their
// staged operands, cost the occupancy more than the wider loads gain).
template <typename T>
constexpr int pp_groups(int rb, int ncb) { return 1; }
// K steps of counts in flight beyond the one being multiplied.
template <typename T>
constexpr int pp_depth(int rb, int ncb) { return 1; }

template <typename T, int RB, int NCB>
void launch_pp(dim3 grid, hipStream_t st, const void *X, int64_t M, int64_t N, const unsigned short *B,
               int64_t ldb, float *Y, bool vec) {
    constexpr int KG = pp_groups<T>(RB, NCB), D = pp_depth<T>(RB, NCB);
    if (vec)
        hipLaunchKernelGGL((proj_pixels_kernel<T, RB, NCB, true, KG, D>), grid, dim3(256), 0, st,
                           static_cast<const T *>(X), M, N, B, ldb, Y);
    else
        hipLaunchKernelGGL((proj_pixels_kernel<T, RB, NCB, false, KG, D>), grid, dim3(256), 0, st,
                           static_cast<const T *>(X), M, N, B, ldb, Y);
}

// Four row blocks per wave up to 6 column blocks (9 for one-byte counts, whose
// loads take half the registers), else two (register budget).
template <typename T>
bool dispatch_pp(int ncb, unsigned gy, hipStream_t st, const void *X, int64_t M, int64_t N,
                 const unsigned short *B, int64_t ldb, float *Y, bool vec4, bool vec2) {
    constexpr int kMax4 = sizeof(T) == 1 ? 9 : 6;
#define XPCS_PP4(n)                                                                             \
    case n:                                                                                     \
        if (n <= kMax4) {                                                                       \
            dim3 g((unsigned)((M + 255) / 256), gy);                                            \
            launch_pp<T, 4, (n <= kMax4 ? n : 1)>(g, st, X, M, N, B, ldb, Y, vec4);             \
        } else {                                                                                \
            dim3 g((unsigned)((M + 127) / 128), gy);                                            \
            launch_pp<T, 2, n>(g, st, X, M, N, B, ldb, Y, vec2);                                \
        }                                                                                       \
        return true;
    switch (ncb) {
        XPCS_PP4(1) XPCS_PP4(2) XPCS_PP4(3) XPCS_PP4(4) XPCS_PP4(5) XPCS_PP4(6)
        XPCS_PP4(7) XPCS_PP4(8) XPCS_PP4(9) XPCS_PP4(10) XPCS_PP4(11) XPCS_PP4(12)
        default:
            return false;
    }
#undef XPCS_PP4
}

}  // namespace

xpcs_status launch_proj_pixels(xpcs_ctx *ctx, const void *frames, int dtype, int64_t M, int64_t N,
                               const unsigned short *B, int64_t ldb, int L, float *Y) {
    Phase phase_(ctx, "proj_pixels");
    if (L % 16 || L <= 0) return fail(ctx, XPCS_EINVAL, "internal: L must be a positive multiple of 16");
    const int64_t kstep = 32;                              // frames per K step
    if (ldb % kstep || ldb < N)
        return fail(ctx, XPCS_EINVAL, "internal: sketch row stride must cover N in whole K steps");
    const int ncb_total = L / 16;
    // Column groups of at most 12 blocks (grid.y of one launch per group size): the
    // sizes differ by at most one, the larger groups first.
    const int ngroups = (ncb_total + 11) / 12;
    const int sz = ncb_total / ngroups, nbig = ncb_total % ngroups;
    const size_t esz = dtype == XPCS_U8 ? 1 : 2;
    const bool vec4 = (M % 4 == 0) && ((uintptr_t)frames % (4 * esz) == 0);
    const bool vec2 = (M % 2 == 0) && ((uintptr_t)frames % (2 * esz) == 0);
    for (int part = 0; part < 2; ++part) {
        const int ncb = part == 0 ? sz + 1 : sz, gy = part == 0 ? nbig : ngroups - nbig;
        if (gy == 0) continue;
        const int c0 = part == 0 ? 0 : nbig * (sz + 1);
        const unsigned short *Bp = B + (int64_t)16 * c0 * ldb;
        float *Yp = Y + (int64_t)16 * c0 * M;
        bool ok = dtype == XPCS_U8
                      ? dispatch_pp<uint8_t>(ncb, (unsigned)gy, ctx->stream, frames, M, N, Bp, ldb, Yp, vec4, vec2)
                      : dispatch_pp<uint16_t>(ncb, (unsigned)gy, ctx->stream, frames, M, N, Bp, ldb, Yp, vec4, vec2);
        if (!ok) return fail(ctx, XPCS_EUNSUPPORTED, "too many sketch columns for proj_pixels");
        XPCS_LAUNCH_CHECK(ctx, "proj_pixels");
    }
    return XPCS_OK;
}

}  // namespace xpcs
