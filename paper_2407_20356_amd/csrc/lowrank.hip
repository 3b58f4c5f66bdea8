// Operands of the compressed two-time correlation (Sec. 2.1, Eqs. 8-10 per ROI).
//
// With W = V diag(sigma) (the compressed data, Eq. 7), G_R = U_R^T U_R = L_R L_R^T
// (Cholesky, FP64),
//   C~_R[i][j] = |R| (W G_R W^T)[i][j] / (S_R[i] S_R[j]) = Z[i] . Z[j],
//   Z[t] = sqrt(|R|) (W[t] / S_R[t]) L_R.
// Z is formed in FP64 and split into bf16 hi + lo so that the tile pass can run
// three BF16 MFMA products (hi.hi + hi.lo + lo.hi) with FP32 accumulation,
// accurate to ~2^-16 relative per term; the symmetric form needs one operand.
#include <type_traits>

#include "internal.hpp"
#include "zrows.hpp"

namespace xpcs {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kZFrames = 64;                // frames per block of the wide kernel
constexpr int kZMaxK = 192;                 // widest rank of the on-chip (MFMA) Z-row kernel

// Z rows on the FP64 MFMA (ranks up to kZMaxK): Z_R = diag(sqrt|R| / S_R)
// V (diag(sigma) L_R) computed as its transpose, (diag(sigma) L_R)^T V^T, with
// v_mfma_f64_16x16x4: the MFMA's rows are 16 columns of Z, its columns 16 frames.
// blockIdx.z = ROI slot, blockIdx.y = group of kZmCols columns, the block's waves walk
// 64-frame strips: lane l reads frames 4 (l % 16) .. + 3 of column a + l / 16 of V in
// one 16-byte load, feeding four MFMA column sets that share every fragment of
// diag(sigma) L_R (staged once per block in LDS, in fragment order; the blocks above
// L_R's diagonal are zero and skipped).  Split-bf16 rows leave frame-major through a
// per-wave LDS transpose (one 16-column tile at a time, 32 bytes of hi and of lo per
// frame); FP64 columns leave as four consecutive frames per lane.
constexpr int kZmCols = 80;
constexpr int kZmTiles = kZmCols / 16;
constexpr int kZmK = 96;                      // rows of diag(sigma) L_R per LDS fill
constexpr int kZmWaves = 8;
constexpr int kZmPitch = 17;                  // transpose pitch (32-bit words) against bank conflicts

template <bool BF>
__global__ __launch_bounds__(64 * kZmWaves, 2) void z_rows_mfma_kernel(
    const float *__restrict__ V, const double *__restrict__ sigma, const int64_t *__restrict__ roi_sum,
    const int64_t *__restrict__ roi_npix, const double *__restrict__ Lr, int64_t N, int k, int r0, int64_t t0,
    int64_t n, double *__restrict__ z, unsigned short *__restrict__ z_hi, unsigned short *__restrict__ z_lo, int kp,
    unsigned char *__restrict__ valid, int vec_v, int vec_z) {
    __shared__ double Ts[kZmK * kZmCols];
    __shared__ unsigned Zs[BF ? kZmWaves * 64 * kZmPitch : 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int slot = blockIdx.z, roi = r0 + slot;
    const double *L = Lr + (int64_t)slot * k * k;
    const int j0 = blockIdx.y * kZmCols;
    const int ncg = k - j0 < kZmCols ? k - j0 : kZmCols;
    const int nct = (ncg + 15) / 16;
    const int nchunks = (k + kZmK - 1) / kZmK;
    const int64_t nstrips = (n + 63) / 64;
    const double rn = sqrt((double)roi_npix[roi]);
    const int64_t *Srow = roi_sum + (int64_t)roi * N + t0;
    const float *Vb = V + t0;
    for (int64_t sb = (int64_t)blockIdx.x * kZmWaves; sb < nstrips; sb += (int64_t)gridDim.x * kZmWaves) {
        const int64_t r0s = (sb + wv) * 64;
        const bool live = sb + wv < nstrips;
        const int64_t row = r0s + 4 * li;            // this lane's first frame
        const bool full = vec_v && r0s + 64 <= n;
        f64x4 acc[kZmTiles][4];
#pragma unroll
        for (int c = 0; c < kZmTiles; ++c)
#pragma unroll
            for (int s = 0; s < 4; ++s) acc[c][s] = (f64x4){0.0, 0.0, 0.0, 0.0};
        for (int ch = 0; ch < nchunks; ++ch) {
            const int k0 = ch * kZmK;
            const int kc = k - k0 < kZmK ? k - k0 : kZmK;
            if (nchunks > 1 || sb == (int64_t)blockIdx.x * kZmWaves) {
                __syncthreads();
                for (int idx = threadIdx.x; idx < kZmK * kZmCols; idx += 64 * kZmWaves) {
                    const int l = idx & 63, gc = idx >> 6;
                    const int i = 4 * (gc / kZmTiles) + (l >> 4), jj = 16 * (gc % kZmTiles) + (l & 15);
                    Ts[idx] = i < kc && jj < ncg ? sigma[k0 + i] * L[(int64_t)(k0 + i) * k + j0 + jj] : 0.0;
                }
                __syncthreads();
            }
            if (!live) continue;
            const int ng = (kc + 3) / 4;
            int64_t rc[4];
            bool ok[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                ok[s] = row + s < n;
                rc[s] = ok[s] ? row + s : n - 1;
            }
            const float *Ak = Vb + (int64_t)k0 * N;
            auto kloop = [&](auto full_c) {
                constexpr bool F = decltype(full_c)::value;
                auto fetch = [&](int g, float (&x)[4]) {
                    const int kk = 4 * g + lk < kc ? 4 * g + lk : kc - 1;
                    const float *p = Ak + (int64_t)kk * N;
                    if constexpr (F) {
                        const float4 q = *reinterpret_cast<const float4 *>(p + row);
                        x[0] = q.x;
                        x[1] = q.y;
                        x[2] = q.z;
                        x[3] = q.w;
                    } else {
#pragma unroll
                        for (int s = 0; s < 4; ++s) x[s] = p[rc[s]];
                    }
                };
                constexpr int kG = kZmK / 4, AH = 2;
                float ring[AH][4];
#pragma unroll
                for (int u = 0; u < AH; ++u) fetch(u, ring[u]);
#pragma unroll
                for (int g = 0; g < kG; ++g) {
                    if (g >= ng) break;
                    const int u = g % AH;
                    const bool kv = 4 * g + lk < kc;
                    double a[4];
#pragma unroll
                    for (int s = 0; s < 4; ++s) a[s] = kv && (F || ok[s]) ? (double)ring[u][s] : 0.0;
                    if (g + AH < kG) fetch(g + AH, ring[u]);
                    const int kg = k0 + 4 * g;
                    const double *tf = Ts + g * (kZmTiles * 64) + lane;
                    double t[kZmTiles];
#pragma unroll
                    for (int c = 0; c < kZmTiles; ++c) t[c] = tf[64 * c];
#pragma unroll
                    for (int c = 0; c < kZmTiles; ++c) {
                        // L_R is lower triangular: rows kg .. kg + 3 meet columns up to kg + 3
                        if (c >= nct || j0 + 16 * c > kg + 3) continue;
#pragma unroll
                        for (int s = 0; s < 4; ++s)
                            acc[c][s] = __builtin_amdgcn_mfma_f64_16x16x4f64(t[c], a[s], acc[c][s], 0, 0, 0);
                    }
                }
            };
            if (full) kloop(std::true_type{});
            else kloop(std::false_type{});
        }
        if (!live) continue;
        // acc[c][s][v]: column j0 + 16 c + lk + 4 v of Z, frame r0s + 4 li + s.  The
        // lane's offsets are recomputed per strip (kept out of registers across the loop).
        int lio = li, lko = lk;
        asm volatile("" : "+v"(lio), "+v"(lko));
        double fs[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int64_t sv = row + s < n ? Srow[row + s] : 0;
            fs[s] = sv > 0 ? rn / (double)sv : 0.0;
        }
        if constexpr (BF) {
            unsigned *zw = Zs + wv * 64 * kZmPitch;
            const int64_t t = r0s + lane;             // the frame this lane writes
            const int ntile = (kp - j0 < kZmCols ? kp - j0 : kZmCols) / 16;   // whole 16-column pieces of kp
#pragma unroll
            for (int c = 0; c < kZmTiles; ++c) {
                if (c >= ntile) break;
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const double zv = c < nct ? fs[s] * acc[c][s][v] : 0.0;
                        const unsigned short h = f32_to_bf16_bits((float)zv);
                        const unsigned short lo = f32_to_bf16_bits((float)(zv - (double)bf16_bits_to_f32(h)));
                        zw[(4 * lio + s) * kZmPitch + lko + 4 * v] = (unsigned)h | ((unsigned)lo << 16);
                    }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (t < n) {
                    u16x8 h0, h1, l0, l1;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const unsigned a0 = zw[lane * kZmPitch + e], a1 = zw[lane * kZmPitch + 8 + e];
                        h0[e] = (unsigned short)(a0 & 0xffff);
                        l0[e] = (unsigned short)(a0 >> 16);
                        h1[e] = (unsigned short)(a1 & 0xffff);
                        l1[e] = (unsigned short)(a1 >> 16);
                    }
                    const int64_t off = ((int64_t)slot * n + t) * kp + j0 + 16 * c;
                    *reinterpret_cast<u16x8 *>(z_hi + off) = h0;
                    *reinterpret_cast<u16x8 *>(z_hi + off + 8) = h1;
                    *reinterpret_cast<u16x8 *>(z_lo + off) = l0;
                    *reinterpret_cast<u16x8 *>(z_lo + off + 8) = l1;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            if (blockIdx.y == 0 && t < n) {
                const int64_t sv = Srow[t];
                valid[(int64_t)slot * n + t] = sv > 0 ? 1 : 0;
            }
        } else {
#pragma unroll
            for (int c = 0; c < kZmTiles; ++c) {
                if (c >= nct) continue;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int jl = 16 * c + lko + 4 * v;
                    if (jl >= ncg) continue;
                    double *o = z + ((int64_t)slot * k + j0 + jl) * n + row;
                    double x[4];
#pragma unroll
                    for (int s = 0; s < 4; ++s) x[s] = fs[s] * acc[c][s][v];
                    if (vec_z && row + 4 <= n) {
                        reinterpret_cast<double2 *>(o)[0] = make_double2(x[0], x[1]);
                        reinterpret_cast<double2 *>(o)[1] = make_double2(x[2], x[3]);
                    } else {
#pragma unroll
                        for (int s = 0; s < 4; ++s)
                            if (row + s < n) o[s] = x[s];
                    }
                }
            }
        }
    }
}


// Z rows for ranks above kZMaxK, where W's slice no longer fits LDS: one ROI per
// blockIdx.y, 64 frames per block (lane = frame), and per blockIdx.z a group of 256
// output columns (wave w: columns 64 w .. 64 w + 63 of the group).  The inner
// dimension runs in chunks of 16 rows of L_R, each chunk staging its 16 rows of W
// (source column a at W[a ldw + w_t0 + t], times wscale[a] when given) and of L_R.
// Rows go to z64 (FP64, column-major per slot) or to split-bf16 rows at
// ((slot rows_cap + (ring0 + t) mod ring_cap) kp) with valid[] beside them.
constexpr int kZwCols = 256;
constexpr int kZwChunk = 16;
template <typename TS>
__global__ __launch_bounds__(256) void z_rows_wide_kernel(
    const TS *__restrict__ W, const double *__restrict__ wscale, int64_t ldw, int64_t w_t0,
    const int64_t *__restrict__ S, int64_t s_stride, int64_t s_t0, const int64_t *__restrict__ npix, int r0,
    const double *__restrict__ Lr, int k, int64_t n, double *__restrict__ z64, unsigned short *__restrict__ z_hi,
    unsigned short *__restrict__ z_lo, int kp, unsigned char *__restrict__ valid, int64_t rows_cap, int64_t ring0,
    int64_t ring_cap) {
    __shared__ double wT[kZwChunk][kZFrames];
    __shared__ double Lc[kZwChunk][kZwCols];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int slot = blockIdx.y, roi = r0 + slot;
    const int j0 = blockIdx.z * kZwCols;
    const int64_t f0 = (int64_t)blockIdx.x * kZFrames;
    const double *L = Lr + (int64_t)slot * k * k;
    double acc[64];
#pragma unroll
    for (int m = 0; m < 64; ++m) acc[m] = 0.0;
    for (int a0 = 0; a0 < k; a0 += kZwChunk) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < kZwChunk * kZFrames; idx += 256) {
            const int aa = idx / kZFrames, f = idx % kZFrames;
            const int a = a0 + aa;
            const int64_t t = f0 + f;
            double v = 0.0;
            if (a < k && t < n) {
                v = (double)W[(int64_t)a * ldw + w_t0 + t];
                if (wscale) v *= wscale[a];
            }
            wT[aa][f] = v;
        }
        for (int idx = threadIdx.x; idx < kZwChunk * kZwCols; idx += 256) {
            const int aa = idx / kZwCols, b = idx % kZwCols;
            Lc[aa][b] = (a0 + aa < k && j0 + b < k) ? L[(int64_t)(a0 + aa) * k + j0 + b] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int aa = 0; aa < kZwChunk; ++aa) {
            const double x = wT[aa][lane];
            const double *lw = &Lc[aa][64 * wave];
#pragma unroll
            for (int m = 0; m < 64; m += 2) {
                const double2 l = *reinterpret_cast<const double2 *>(lw + m);
                acc[m] = fma(x, l.x, acc[m]);
                acc[m + 1] = fma(x, l.y, acc[m + 1]);
            }
        }
    }
    const int64_t t = f0 + lane;
    if (t >= n) return;
    const int64_t sv = S[(int64_t)roi * s_stride + s_t0 + t];
    const double sc = sv > 0 ? sqrt((double)npix[roi]) / (double)sv : 0.0;
    const int jw = j0 + 64 * wave;
    if (z64) {
#pragma unroll
        for (int m = 0; m < 64; ++m)
            if (jw + m < k) z64[((int64_t)slot * k + jw + m) * n + t] = sc * acc[m];
        return;
    }
    const int64_t row = (int64_t)slot * rows_cap + (ring0 + t) % ring_cap;
#pragma unroll
    for (int m = 0; m < 64; ++m) {
        const int j = jw + m;
        if (j < kp) {
            const double zv = j < k ? sc * acc[m] : 0.0;
            const unsigned short hb = f32_to_bf16_bits((float)zv);
            z_hi[row * kp + j] = hb;
            z_lo[row * kp + j] = f32_to_bf16_bits((float)(zv - (double)bf16_bits_to_f32(hb)));
        }
    }
    if (blockIdx.z == 0 && wave == 0) valid[row] = sv > 0 ? 1 : 0;
}

}  // namespace


xpcs_status launch_z_rows_wide(xpcs_ctx *ctx, const void *W, bool w_f64, const double *wscale, int64_t ldw,
                               int64_t w_t0, const int64_t *S, int64_t s_stride, int64_t s_t0, const int64_t *npix,
                               int r0, const double *Lr, int k, int nb, int64_t n, double *z64,
                               unsigned short *z_hi, unsigned short *z_lo, int kp, unsigned char *valid,
                               int64_t rows_cap, int64_t ring0, int64_t ring_cap) {
    if (n <= 0 || nb <= 0) return XPCS_OK;
    // the split-bf16 form writes the padded columns k .. kp - 1 too
    const int cols = z64 ? k : kp;
    dim3 grid((unsigned)((n + kZFrames - 1) / kZFrames), (unsigned)nb, (unsigned)((cols + kZwCols - 1) / kZwCols));
    if (w_f64)
        hipLaunchKernelGGL(z_rows_wide_kernel<double>, grid, dim3(256), 0, ctx->stream, static_cast<const double *>(W),
                           wscale, ldw, w_t0, S, s_stride, s_t0, npix, r0, Lr, k, n, z64, z_hi, z_lo, kp, valid,
                           rows_cap, ring0, ring_cap);
    else
        hipLaunchKernelGGL(z_rows_wide_kernel<float>, grid, dim3(256), 0, ctx->stream, static_cast<const float *>(W),
                           wscale, ldw, w_t0, S, s_stride, s_t0, npix, r0, Lr, k, n, z64, z_hi, z_lo, kp, valid,
                           rows_cap, ring0, ring_cap);
    XPCS_LAUNCH_CHECK(ctx, "z_rows_wide");
    return XPCS_OK;
}

xpcs_status launch_z_rows(xpcs_ctx *ctx, const xpcs_factors *f, const double *Lr, int r0, int nb, int64_t t0,
                          int64_t n, double *z64, unsigned short *z_hi, unsigned short *z_lo, int kp,
                          unsigned char *valid) {
    const bool bf = z64 == nullptr;
    if (f->k > kZMaxK) {
        if (bf && (!z_hi || !z_lo || !valid || kp != 32 * ((f->k + 31) / 32)))
            return fail(ctx, XPCS_EINVAL, "internal: split-bf16 Z rows need hi, lo, valid and kp = k rounded to 32");
        return launch_z_rows_wide(ctx, f->V, false, f->sigma, f->N, t0, f->roi_sum, f->N, t0, f->roi_npix, r0, Lr,
                                  f->k, nb, n, z64, z_hi, z_lo, kp, valid, n, 0, n);
    }
    if (bf && (!z_hi || !z_lo || !valid || kp != 32 * ((f->k + 31) / 32)))
        return fail(ctx, XPCS_EINVAL, "internal: split-bf16 Z rows need hi, lo, valid and kp = k rounded to 32");
    {
        if (n <= 0 || nb <= 0) return XPCS_OK;
        const int k = f->k;
        const int gy = ((bf ? kp : k) + kZmCols - 1) / kZmCols;
        const int64_t nstrips = (n + 63) / 64;
        const int vec_v = (reinterpret_cast<uintptr_t>(f->V) % 16 == 0 && f->N % 4 == 0 && t0 % 4 == 0) ? 1 : 0;
        const int vec_z = (z64 && reinterpret_cast<uintptr_t>(z64) % 16 == 0 && n % 2 == 0) ? 1 : 0;
        dim3 grid((unsigned)((nstrips + kZmWaves - 1) / kZmWaves), (unsigned)gy, (unsigned)nb);
        if (bf)
            hipLaunchKernelGGL(z_rows_mfma_kernel<true>, grid, dim3(64 * kZmWaves), 0, ctx->stream, f->V, f->sigma,
                               f->roi_sum, f->roi_npix, Lr, f->N, k, r0, t0, n, z64, z_hi, z_lo, kp, valid, vec_v,
                               vec_z);
        else
            hipLaunchKernelGGL(z_rows_mfma_kernel<false>, grid, dim3(64 * kZmWaves), 0, ctx->stream, f->V, f->sigma,
                               f->roi_sum, f->roi_npix, Lr, f->N, k, r0, t0, n, z64, z_hi, z_lo, kp, valid, vec_v,
                               vec_z);
        XPCS_LAUNCH_CHECK(ctx, "z_rows_mfma");
        return XPCS_OK;
    }
}


xpcs_status launch_lowrank_prep(xpcs_ctx *ctx, const xpcs_factors *f, const double *Lr, int r0, int nr, int64_t t0,
                                int64_t nw, int kp, unsigned short *z_hi, unsigned short *z_lo,
                                unsigned char *valid) {
    Phase phase_(ctx, "lowrank_prep");
    return launch_z_rows(ctx, f, Lr, r0, nr, t0, nw, nullptr, z_hi, z_lo, kp, valid);
}

}  // namespace xpcs
