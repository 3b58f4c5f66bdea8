// Shared pieces of the products of the count matrix X with thin bf16 matrices
// (the passes over the raw frames that build and apply the encoding basis,
// Sec. 2.1, Eqs. 3-7).
//
// Counts enter the BF16 MFMA as two exact planes: the low byte of every count
// (plane 0, always) and the high byte times 256 (plane 1, only in the K steps of
// a wave where some count reaches 256).  Both are integers with at most 8
// significant bits, so their bf16 values are exact and plane 0 + plane 1 is the
// count.  A byte becomes a float in one conversion, and two floats become two
// packed bf16 by keeping their upper halves (exact for these values).
#pragma once

#include "internal.hpp"

namespace xpcs {
namespace proj {

constexpr unsigned short kBfOne = 0x3F80;
constexpr int kQp = 40;   // LDS row pitch (u16) of a staged 32-wide K step: 32 + 8 padding

__device__ __forceinline__ unsigned pack_bf16_pair(float a, float b) {
    return (__builtin_bit_cast(unsigned, b) & 0xffff0000u) | (__builtin_bit_cast(unsigned, a) >> 16);
}

// Keeps the compiler from computing plane 1 ahead of the test that needs it.
__device__ __forceinline__ void opaque(unsigned &v) { asm volatile("" : "+v"(v)); }

// 8 consecutive counts of one frame (one MFMA K group).
template <typename T>
struct Counts8;

template <>
struct Counts8<uint16_t> {
    typedef i32x4 type;
    static __device__ __forceinline__ bool any_high(const type &x) {
        return ((x[0] | x[1] | x[2] | x[3]) & 0xff00ff00) != 0;
    }
    static __device__ __forceinline__ u16x8 plane0(const type &x) {
        i32x4 r;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const unsigned v = (unsigned)x[w];
            r[w] = (int)pack_bf16_pair((float)(v & 0xffu), (float)((v >> 16) & 0xffu));
        }
        return __builtin_bit_cast(u16x8, r);
    }
    static __device__ __forceinline__ u16x8 plane1(const type &x) {
        i32x4 r;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            unsigned v = (unsigned)x[w];
            opaque(v);
            r[w] = (int)pack_bf16_pair((float)((v >> 8) & 0xffu) * 256.f, (float)(v >> 24) * 256.f);
        }
        return __builtin_bit_cast(u16x8, r);
    }
};

template <>
struct Counts8<uint8_t> {
    typedef int2 type;
    static __device__ __forceinline__ bool any_high(const type &) { return false; }
    static __device__ __forceinline__ u16x8 plane0(const type &x) {
        const unsigned a = (unsigned)x.x, b = (unsigned)x.y;
        i32x4 r;
        r[0] = (int)pack_bf16_pair((float)(a & 0xffu), (float)((a >> 8) & 0xffu));
        r[1] = (int)pack_bf16_pair((float)((a >> 16) & 0xffu), (float)(a >> 24));
        r[2] = (int)pack_bf16_pair((float)(b & 0xffu), (float)((b >> 8) & 0xffu));
        r[3] = (int)pack_bf16_pair((float)((b >> 16) & 0xffu), (float)(b >> 24));
        return __builtin_bit_cast(u16x8, r);
    }
    static __device__ __forceinline__ u16x8 plane1(const type &) { return u16x8{}; }
};

// Element-wise load of counts src[0..8) where only the first nv exist.
template <typename T>
__device__ __forceinline__ typename Counts8<T>::type load8_partial(const T *__restrict__ src, int nv) {
    typedef typename Counts8<T>::type V;
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

// One 32-wide K step of a bf16 row-major operand (rows j < 16*NCB, K contiguous),
// held in registers between its global load and its LDS store.  Every thread
// issues the same loads (surplus threads repeat the last unit) so that the
// number of loads in flight is the same on every path.
template <int NCB>
struct Stage16 {
    static constexpr int kUnits = NCB * 16 * 4;           // 16-byte units per K step
    static constexpr int kPer = (kUnits + 255) / 256;
    i32x4 r[kPer];
    __device__ __forceinline__ void load(const unsigned short *__restrict__ src, int64_t ld, int64_t k0) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            int u = threadIdx.x + 256 * i;
            if (kUnits % 256) u = u < kUnits ? u : kUnits - 1;
            r[i] = *reinterpret_cast<const i32x4 *>(src + (int64_t)(u >> 2) * ld + k0 + 8 * (u & 3));
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

}  // namespace proj
}  // namespace xpcs
