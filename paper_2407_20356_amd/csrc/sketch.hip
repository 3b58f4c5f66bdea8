// The range finder's sketch Y0 = X Omega (Sec. 2.1), Omega an N x l matrix of
// independent +-1 signs, on the int8 MFMA.
//
// X is stored frame-contiguous (X[t][p] = frames[t*M + p]) and the product
// contracts over frames, so a lane's MFMA operand (16 frames of one pixel) is a
// byte transpose of what it loads: 4 adjacent pixels of each of 16 frames, turned
// into 4 operands of 16 bytes by byte permutes.  Counts enter as 7-bit planes,
// count = plane0 + 128 plane1 + 16384 plane2 (plane2 only for uint16 counts).  The
// first launch multiplies plane 0 and records, per block of 256 pixels, whether
// any count there needs plane 1 or 2; a launch per higher plane then revisits only
// the recorded blocks (the others leave at once).  A plane's products accumulate
// exactly in int32 (|sum| <= 127 N); the planes combine in FP32, so Y0 is exact
// while its entries stay below 2^24 and is otherwise rounded as few times as planes
// were needed.
#include "internal.hpp"

namespace xpcs {
namespace {

constexpr int kSkPitch = 80;                 // LDS row pitch (bytes) of a staged 64-frame K step

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// om[j][t] = -1 when the top bit of SplitMix64(seed ^ (t << 32 | j)) is set, else +1,
// for j < ell and t < N; zero in the padding rows and columns.
__global__ void sketch_signs_kernel(uint64_t seed, int64_t N, int L, int ell, int64_t ldt, int8_t *om) {
    const int64_t total = (int64_t)L * ldt;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = idx / ldt, t = idx % ldt;
        int8_t v = 0;
        if (j < ell && t < N) {
            const uint64_t h = splitmix64(seed ^ (((uint64_t)t << 32) | (uint64_t)j));
            v = (h >> 63) ? (int8_t)-1 : (int8_t)1;
        }
        om[idx] = v;
    }
}

__device__ __forceinline__ unsigned perm(unsigned hi, unsigned lo, unsigned sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}

// 4 x 4 byte transpose: byte e of o_s = byte s of d_e.
__device__ __forceinline__ void transpose4(unsigned d0, unsigned d1, unsigned d2, unsigned d3, unsigned &o0,
                                           unsigned &o1, unsigned &o2, unsigned &o3) {
    const unsigned t0 = perm(d1, d0, 0x05010400u), t1 = perm(d1, d0, 0x07030602u);
    const unsigned t2 = perm(d3, d2, 0x05010400u), t3 = perm(d3, d2, 0x07030602u);
    o0 = perm(t2, t0, 0x05040100u);
    o1 = perm(t2, t0, 0x07060302u);
    o2 = perm(t3, t1, 0x05040100u);
    o3 = perm(t3, t1, 0x07060302u);
}

// Operands a[s] (pixel s of the lane, K = the lane's 16 frames) from p[e] (frame e,
// byte s = pixel s).
__device__ __forceinline__ void operands(const unsigned (&p)[16], i32x4 (&a)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        unsigned o0, o1, o2, o3;
        transpose4(p[4 * q], p[4 * q + 1], p[4 * q + 2], p[4 * q + 3], o0, o1, o2, o3);
        a[0][q] = (int)o0;
        a[1][q] = (int)o1;
        a[2][q] = (int)o2;
        a[3][q] = (int)o3;
    }
}

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// Four adjacent counts of one frame and their 7-bit planes, one byte per pixel.
template <typename T>
struct SkCounts;

template <>
struct SkCounts<uint8_t> {
    typedef unsigned type;
    static constexpr int kPlanes = 2;
    // bit 0: some count needs plane 1 (>= 128)
    static __device__ __forceinline__ unsigned high(const type &x) { return x & 0x80808080u; }
    static __device__ __forceinline__ int need(unsigned h) { return h ? 1 : 0; }
    static __device__ __forceinline__ unsigned plane(const type &x, int p) {
        return p == 0 ? (x & 0x7f7f7f7fu) : ((x >> 7) & 0x01010101u);
    }
    static __device__ __forceinline__ type load_partial(const uint8_t *src, int nv) {
        unsigned v = 0;
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (s < nv) v |= (unsigned)src[s] << (8 * s);
        return v;
    }
};

template <>
struct SkCounts<uint16_t> {
    typedef u32x2 type;
    static constexpr int kPlanes = 3;
    // bytes 0 and 2 of each dword: the low bytes of the four counts
    static __device__ __forceinline__ unsigned pack(unsigned a, unsigned b) { return perm(b, a, 0x06040200u); }
    // bit 0: some count needs plane 1 (>= 128); bit 1: plane 2 (>= 16384)
    static __device__ __forceinline__ unsigned high(const type &x) { return (x.x | x.y) & 0xff80ff80u; }
    static __device__ __forceinline__ int need(unsigned h) {
        return (h ? 1 : 0) | ((h & 0xc000c000u) ? 2 : 0);
    }
    static __device__ __forceinline__ unsigned plane(const type &x, int p) {
        const int sh = 7 * p;
        const unsigned m = p == 2 ? 0x00030003u : 0x007f007fu;
        return pack((x.x >> sh) & m, (x.y >> sh) & m);
    }
    static __device__ __forceinline__ type load_partial(const uint16_t *src, int nv) {
        unsigned v[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = s < nv ? (unsigned)src[s] : 0u;
        return type{v[0] | (v[1] << 16), v[2] | (v[3] << 16)};
    }
};

// Y[j][p] (+)= 128^PLANE sum_t plane_PLANE(X[t][p]) om[j][t] over the N frames, j in
// this block's column group (16*NCB columns).  A wave owns 64 pixels (lane l:
// pixels 4(l % 16) .. + 4 of the wave's range, frames 16(l / 16) .. + 16 of each K
// step); Omega's K step (64 frames of the group's rows) is staged in LDS, and the
// counts of D K steps ahead are in flight.  PLANE 0 writes Y and need[blockIdx.x]
// (from column group 0); PLANE 1 and 2 add to Y in the blocks whose need has bit
// PLANE - 1.
// VEC: M is a multiple of 4 and X aligned: every lane issues the same vector loads
// (lanes past M read pixel 0, their outputs dropped; frames past N read frame N - 1
// and meet Omega's zero padding).
template <typename T, int NCB, bool VEC, int D, int PLANE>
__global__ __launch_bounds__(256, 2) void sketch_i8_kernel(const T *__restrict__ X, int64_t M, int64_t nf,
                                                           const int8_t *__restrict__ om, int64_t ldo,
                                                           float *__restrict__ Y, int *__restrict__ need) {
    typedef SkCounts<T> C;
    typedef typename C::type PV;
    __shared__ __attribute__((aligned(16))) int8_t sb[2][NCB * 16 * kSkPitch];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int jg = blockIdx.y * 16 * NCB;
    const int64_t pb = ((int64_t)blockIdx.x * 4 + wv) * 64;
    const int64_t pl = pb + 4 * lr;
    const int nvalid = pl >= M ? 0 : (M - pl >= 4 ? 4 : (int)(M - pl));
    const int64_t plc = pl < M ? pl : 0;
    const int8_t *Bg = om + (int64_t)jg * ldo;
    if (PLANE > 0 && !((need[blockIdx.x] >> (PLANE - 1)) & 1)) return;     // uniform over the block

    i32x4 acc[4][NCB];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < NCB; ++c) acc[s][c] = (i32x4){0, 0, 0, 0};

    const int nsteps = (int)((nf + 63) / 64);
    auto load_x = [&](int step, PV (&x)[16]) {
        const int64_t tk = (int64_t)step * 64 + 16 * lg;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int64_t t = tk + e < nf ? tk + e : nf - 1;
            if constexpr (VEC)
                x[e] = *reinterpret_cast<const PV *>(X + t * M + plc);
            else
                x[e] = nvalid > 0 ? C::load_partial(X + t * M + pl, nvalid) : PV{};
        }
    };
    constexpr int kUnits = NCB * 16 * 4;                 // 16-byte units of a staged K step
    constexpr int kPer = (kUnits + 255) / 256;
    i32x4 sr[kPer];
    auto stage_load = [&](int step) {
        const int64_t k0 = (int64_t)step * 64;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            int u = threadIdx.x + 256 * i;
            if (kUnits % 256) u = u < kUnits ? u : kUnits - 1;
            sr[i] = *reinterpret_cast<const i32x4 *>(Bg + (int64_t)(u >> 2) * ldo + k0 + 16 * (u & 3));
        }
    };
    auto stage_store = [&](int b) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int u = threadIdx.x + 256 * i;
            if (u < kUnits) *reinterpret_cast<i32x4 *>(&sb[b][(u >> 2) * kSkPitch + 16 * (u & 3)]) = sr[i];
        }
    };
    auto bfrag = [&](int b, int c) {
        return *reinterpret_cast<const i32x4 *>(&sb[b][(16 * c + lr) * kSkPitch + 16 * lg]);
    };
    auto mma = [&](const i32x4 (&a)[4], int b) {
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
            const i32x4 bv = bfrag(b, c);
#pragma unroll
            for (int s = 0; s < 4; ++s) acc[s][c] = mfma_i8(a[s], bv, acc[s][c]);
        }
    };
    unsigned hor = 0;                                    // high bits seen by this lane
    auto compute = [&](const PV (&x)[16], int b) {
        unsigned p[16];
        i32x4 a[4];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            if (PLANE == 0) hor |= C::high(x[e]);
            p[e] = C::plane(x[e], PLANE);
        }
        operands(p, a);
        mma(a, b);
    };

    // Counts of D steps ahead in registers; Omega's next step loaded into registers
    // and written to the other LDS buffer after the current step's MFMAs.  Loads are
    // issued every step (the last step's repeated at the end) so that their number
    // never varies.
    PV xr[D + 1][16];
#pragma unroll
    for (int i = 0; i < D; ++i) load_x(i < nsteps ? i : nsteps - 1, xr[i]);
    stage_load(0);
    stage_store(0);
    __syncthreads();
    for (int step0 = 0; step0 < nsteps; step0 += D + 1) {
#pragma unroll
        for (int j = 0; j <= D; ++j) {
            const int step = step0 + j;
            if (step >= nsteps) break;
            const int ahead = step + D < nsteps ? step + D : nsteps - 1;
            load_x(ahead, xr[(j + D) % (D + 1)]);
            const bool more = step + 1 < nsteps;
            if (more) stage_load(step + 1);
            compute(xr[j], step & 1);
            if (more) stage_store((step + 1) & 1);
            __syncthreads();
        }
    }
    if (PLANE == 0 && blockIdx.y == 0) {
        __shared__ int s_need[4];
        const unsigned long long any1 = __ballot(C::need(hor) & 1), any2 = __ballot(C::need(hor) & 2);
        if (lane == 0) s_need[wv] = (any1 ? 1 : 0) | (any2 ? 2 : 0);
        __syncthreads();
        if (threadIdx.x == 0) need[blockIdx.x] = s_need[0] | s_need[1] | s_need[2] | s_need[3];
    }
    constexpr float kScale = PLANE == 0 ? 1.0f : (PLANE == 1 ? 128.0f : 16384.0f);
    // acc[s][c][i] = Y[j = jg + 16c + lr][p = pb + 16 lg + 4 i + s]
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
        float *yrow = Y + (int64_t)(jg + 16 * c + lr) * M;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t p = pb + 16 * lg + 4 * i;
            f32x4 v = {(float)acc[0][c][i], (float)acc[1][c][i], (float)acc[2][c][i], (float)acc[3][c][i]};
            if (PLANE > 0) v *= kScale;
            if (VEC && p + 3 < M) {
                f32x4 *dst = reinterpret_cast<f32x4 *>(yrow + p);
                if (PLANE > 0) v += *dst;
                *dst = v;
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    if (p + s < M) yrow[p + s] = PLANE > 0 ? yrow[p + s] + v[s] : v[s];
            }
        }
    }
}

template <typename T, int NCB, int PLANE>
void launch_sk(dim3 grid, hipStream_t st, const void *X, int64_t M, int64_t N, const int8_t *om, int64_t ldo,
               float *Y, int *need, bool vec) {
    constexpr int D = 1;
    if (vec)
        hipLaunchKernelGGL((sketch_i8_kernel<T, NCB, true, D, PLANE>), grid, dim3(256), 0, st,
                           static_cast<const T *>(X), M, N, om, ldo, Y, need);
    else
        hipLaunchKernelGGL((sketch_i8_kernel<T, NCB, false, D, PLANE>), grid, dim3(256), 0, st,
                           static_cast<const T *>(X), M, N, om, ldo, Y, need);
}

// Widest column group of one launch: its accumulators and the staged counts fit
// the register budget of two waves per SIMD.
template <typename T>
constexpr int sk_max_ncb() { return sizeof(T) == 1 ? 10 : 8; }

template <typename T, int PLANE>
bool dispatch_sk(int ncb, dim3 grid, hipStream_t st, const void *X, int64_t M, int64_t N, const int8_t *om,
                 int64_t ldo, float *Y, int *need, bool vec) {
    if (ncb > sk_max_ncb<T>()) return false;
    switch (ncb) {
#define XPCS_SK(n)                                                                                  \
    case n:                                                                                         \
        launch_sk<T, (n <= sk_max_ncb<T>() ? n : 1), PLANE>(grid, st, X, M, N, om, ldo, Y, need, vec); \
        return true;
        XPCS_SK(1) XPCS_SK(2) XPCS_SK(3) XPCS_SK(4) XPCS_SK(5)
        XPCS_SK(6) XPCS_SK(7) XPCS_SK(8) XPCS_SK(9) XPCS_SK(10)
#undef XPCS_SK
        default:
            return false;
    }
}

template <typename T>
bool dispatch_plane(int plane, int ncb, dim3 grid, hipStream_t st, const void *X, int64_t M, int64_t N,
                    const int8_t *om, int64_t ldo, float *Y, int *need, bool vec) {
    switch (plane) {
        case 0: return dispatch_sk<T, 0>(ncb, grid, st, X, M, N, om, ldo, Y, need, vec);
        case 1: return dispatch_sk<T, 1>(ncb, grid, st, X, M, N, om, ldo, Y, need, vec);
        default:
            if constexpr (SkCounts<T>::kPlanes > 2) return dispatch_sk<T, 2>(ncb, grid, st, X, M, N, om, ldo, Y, need, vec);
            return false;
    }
}

}  // namespace

size_t sketch_need_bytes(int64_t M) { return (size_t)((M + 255) / 256) * sizeof(int); }

xpcs_status launch_sketch_i8(xpcs_ctx *ctx, const void *frames, int dtype, int64_t M, int64_t N, uint64_t seed,
                             int ell, int L, int64_t ldt, int8_t *om, float *Y, int *need) {
    if (L % 16 || L <= 0 || ell > L) return fail(ctx, XPCS_EINVAL, "internal: L must be a multiple of 16 >= l");
    if (ldt % 64 || ldt < N) return fail(ctx, XPCS_EINVAL, "internal: sign row stride must cover N in steps of 64");
    if (N > (int64_t)1 << 24) return fail(ctx, XPCS_EUNSUPPORTED, "more than 2^24 frames in one sketch");
    {
        Phase phase_(ctx, "sketch_omega");
        const int64_t total = (int64_t)L * ldt;
        int grid = (int)((total + 255) / 256);
        if (grid > 4096) grid = 4096;
        hipLaunchKernelGGL(sketch_signs_kernel, dim3(grid), dim3(256), 0, ctx->stream, seed, N, L, ell, ldt, om);
        XPCS_LAUNCH_CHECK(ctx, "sketch_omega");
    }
    Phase phase_(ctx, "sketch");
    const size_t esz = dtype == XPCS_U8 ? 1 : 2;
    const bool vec = (M % 4 == 0) && ((uintptr_t)frames % (4 * esz) == 0);
    // Column groups of at most sk_max_ncb blocks whose sizes differ by at most one,
    // the larger groups first (one launch per group size).
    const int ncb_total = L / 16;
    const int max_ncb = dtype == XPCS_U8 ? sk_max_ncb<uint8_t>() : sk_max_ncb<uint16_t>();
    const int ngroups = (ncb_total + max_ncb - 1) / max_ncb;
    const int sz = ncb_total / ngroups, nbig = ncb_total % ngroups;
    const unsigned gx = (unsigned)((M + 255) / 256);
    const int nplanes = dtype == XPCS_U8 ? 2 : 3;
    for (int plane = 0; plane < nplanes; ++plane) {
        for (int part = 0; part < 2; ++part) {
            const int ncb = part == 0 ? sz + 1 : sz, gy = part == 0 ? nbig : ngroups - nbig;
            if (gy == 0) continue;
            const int c0 = part == 0 ? 0 : nbig * (sz + 1);
            const int8_t *Bp = om + (int64_t)16 * c0 * ldt;
            float *Yp = Y + (int64_t)16 * c0 * M;
            const dim3 grid(gx, (unsigned)gy);
            // plane 0 of the first launch records need[] (its blockIdx.y 0 is column group 0)
            const bool ok =
                dtype == XPCS_U8
                    ? dispatch_plane<uint8_t>(plane, ncb, grid, ctx->stream, frames, M, N, Bp, ldt, Yp, need, vec)
                    : dispatch_plane<uint16_t>(plane, ncb, grid, ctx->stream, frames, M, N, Bp, ldt, Yp, need, vec);
            if (!ok) return fail(ctx, XPCS_EUNSUPPORTED, "too many sketch columns for the int8 sketch");
            XPCS_LAUNCH_CHECK(ctx, "sketch");
        }
    }
    return XPCS_OK;
}

}  // namespace xpcs
