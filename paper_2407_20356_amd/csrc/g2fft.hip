// g2 of the compressed two-time correlation without forming C~ (Sec. 3.1, Eq. 12
// read as the mean along C~'s diagonals; C~ per ROI from Sec. 2.1, Eqs. 8-10).
//
// With G_R = U_R^T U_R = L_R L_R^T and Z[t] = sqrt(|R|) (W[t] / S_R[t]) L_R (zero
// where S_R[t] = 0), C~_R = Z Z^T, so the sum along diagonal tau is
//   a(tau) = sum_t Z[t] . Z[t + tau] = sum_j (autocorrelation of column j)(tau),
// and the number of valid pairs is the autocorrelation of the 0/1 mask of frames
// with S_R > 0.  Autocorrelations come from power spectra: with the columns
// zero-padded to L >= 2n there is no wrap-around and
//   a(tau) = Re IDFT( sum_j |DFT z_j|^2 )(tau).
// Two real columns share one complex transform, x = z_a + i z_b: |DFT x|^2 is
// |DFT z_a|^2 + |DFT z_b|^2 plus a real odd term, and the inverse transform of a
// real odd spectrum is imaginary, so the real part above is exact.  The work is
// O(k n log n) per ROI instead of the tile pass's O(k n^2), and every step runs in
// FP64, so the result is the same g2 as the tile pass's, without its bf16 terms.
//
// Transforms are radix-2 in FP64, length L = L1 * L2 (L1 <= L2 <= 2048), in two
// passes over HBM (four-step): pass 1 transforms the L1-long columns
// x[a L2 + c] of CC columns at a time in LDS, multiplies by w_L^(b c) and stores
// X1[b][c]; pass 2 transforms RB rows X1[b][.] at a time, giving X[b + L1 d].
// The forward pass 2 accumulates |X|^2 over a ROI's column pairs in registers;
// the inverse transform of the (data, mask) spectra reuses both passes.
#include <algorithm>

#include "internal.hpp"
#include "zrows.hpp"

namespace xpcs {
namespace {

constexpr int kFftThreads = 256;
constexpr int kFftElems = 2048;             // complex elements per LDS tile (32 KB)
constexpr int kFftPerThread = kFftElems / kFftThreads;
constexpr int kFftMaxLog = 22;              // L <= 2^22, i.e. windows up to 2^21 frames

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 expi_2pi(double num, double den, double sgn) {
    // exp(sgn * 2 pi i num / den); den is a power of two, so num / den is exact
    double s, c;
    sincospi(sgn * 2.0 * (num / den), &s, &c);
    return make_double2(c, s);
}
__device__ __forceinline__ int bitrev(int a, int lg) {
    return lg == 0 ? 0 : (int)(__builtin_bitreverse32((unsigned)a) >> (32 - lg));
}

// exp(sgn 2 pi i m / 2^(t+1)) * x for the small constant roots (t <= 2, m < 2^t).
template <int T, int Mi>
__device__ __forceinline__ double2 root_mul(double2 x, double sgn) {
    if (Mi == 0) return x;
    if (T == 1 || Mi == 2) return make_double2(-sgn * x.y, sgn * x.x);        // * (sgn i)
    constexpr double h = 0.70710678118654752440;                            // 2^-1/2
    if (Mi == 1) return cmul(x, make_double2(h, sgn * h));
    return cmul(x, make_double2(-h, sgn * h));                              // Mi == 3
}

// R consecutive radix-2 stages s .. s+R-1 in registers: a work item owns the 2^R
// elements pos + j 2^s (j < 2^R) of one 2^(s+R)-element block of one sequence.
// In stage s+t the pair (j, j + 2^t) takes the twiddle w_(2^(s+t+1))^(pos + m 2^s),
// m = j mod 2^t, i.e. the table entry for pos times a constant root.
template <int R>
__device__ __forceinline__ void fft_stages(double2 *buf, const double2 *tw, int lp, int lg, int s, double sgn) {
    constexpr int E = 1 << R;
    const int G = 1 << lg;
    const int units = (1 << (lp - R)) << lg;
    const int step = (1 << s) * G;
    for (int u = threadIdx.x; u < units; u += kFftThreads) {
        const int g = u & (G - 1), v = u >> lg;
        const int pos = v & ((1 << s) - 1), grp = v >> s;
        const int base = ((grp << (s + R)) + pos) * G + g;
        double2 x[E];
#pragma unroll
        for (int j = 0; j < E; ++j) x[j] = buf[base + j * step];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const double2 w0 = tw[pos << (lp - 1 - s - t)];
#pragma unroll
            for (int j = 0; j < E; ++j) {
                if (j & (1 << t)) continue;
                const int jj = j | (1 << t);
                double2 w;
                switch (j & ((1 << t) - 1)) {
                    case 0: w = w0; break;
                    case 1: w = t == 1 ? root_mul<1, 1>(w0, sgn) : root_mul<2, 1>(w0, sgn); break;
                    case 2: w = root_mul<2, 2>(w0, sgn); break;
                    default: w = root_mul<2, 3>(w0, sgn); break;
                }
                const double2 y = cmul(w, x[jj]);
                x[jj] = make_double2(x[j].x - y.x, x[j].y - y.y);
                x[j] = make_double2(x[j].x + y.x, x[j].y + y.y);
            }
        }
#pragma unroll
        for (int j = 0; j < E; ++j) buf[base + j * step] = x[j];
    }
    __syncthreads();
}

// In-place radix-2 transform of length P = 2^lp over G = 2^lg interleaved
// sequences in LDS (element a of sequence g at buf[a * G + g]), input in
// bit-reversed order, output in natural order; tw[m] = exp(sgn 2 pi i m / P),
// m < P/2.  Stages run three at a time in registers.  Starts and ends with a
// barrier.
__device__ void lds_fft(double2 *buf, const double2 *tw, int lp, int lg, double sgn) {
    __syncthreads();
    int s = 0;
    for (; s + 3 <= lp; s += 3) fft_stages<3>(buf, tw, lp, lg, s, sgn);
    if (lp - s == 2) fft_stages<2>(buf, tw, lp, lg, s, sgn);
    else if (lp - s == 1) fft_stages<1>(buf, tw, lp, lg, s, sgn);
}

__device__ void fill_twiddles(double2 *tw, int lp, double sgn) {
    const int P = 1 << lp;
    for (int m = threadIdx.x; m < P / 2; m += kFftThreads) tw[m] = expi_2pi((double)m, (double)P, sgn);
}

// Pass 1.  INV = false: signal s of the batch is column pair p of ROI slot
// s / (np + 1) (x = z_2p + i z_2p+1, the odd column alone when k is odd) or, for
// p = np, the ROI's 0/1 frame mask; x[t] = 0 for t >= n.  INV = true: signal s
// is the real spectrum spec[s][.] and the transform runs with the opposite sign.
template <bool INV>
__global__ __launch_bounds__(kFftThreads) void g2fft_pass1_kernel(
    const double *__restrict__ z, const int64_t *__restrict__ roi_sum, int64_t N, int r0, int64_t t0, int64_t n,
    int k, int np, const double *__restrict__ spec, int nparts, int lp1, int lp2, int lcc,
    double2 *__restrict__ X1) {
    extern __shared__ double2 fsm[];
    const int L1 = 1 << lp1, L2 = 1 << lp2, CC = 1 << lcc;
    const int64_t L = (int64_t)L1 * L2;
    double2 *buf = fsm, *tw = fsm + (L1 << lcc), *tlo = tw + L1 / 2;
    const double sgn = INV ? 1.0 : -1.0;
    fill_twiddles(tw, lp1, sgn);
    for (int m = threadIdx.x; m < L2; m += kFftThreads) tlo[m] = expi_2pi((double)m, (double)L, sgn);
    const int c0 = blockIdx.x << lcc;
    const int s = blockIdx.y;
    const double *za = nullptr, *zb = nullptr;
    const int64_t *Sr = nullptr;
    if (!INV) {
        const int slot = s / (np + 1), p = s % (np + 1);
        if (p < np) {
            za = z + ((int64_t)slot * k + 2 * p) * n;
            if (2 * p + 1 < k) zb = za + n;
        } else {
            Sr = roi_sum + (int64_t)(r0 + slot) * N + t0;
        }
    }
    for (int e = threadIdx.x; e < (L1 << lcc); e += kFftThreads) {
        const int a = e >> lcc, c = e & (CC - 1);
        const int64_t t = (int64_t)a * L2 + c0 + c;
        double2 v = make_double2(0.0, 0.0);
        if (INV) {
            // signal s = 2 slot + which: the data spectrum is split in nparts partial sums
            const int slot = s >> 1;
            const double *sp = spec + (int64_t)slot * (nparts + 1) * L + t;
            if (s & 1) {
                v.x = sp[(int64_t)nparts * L];
            } else {
                double acc = 0.0;
                for (int q = 0; q < nparts; ++q) acc += sp[(int64_t)q * L];
                v.x = acc;
            }
        } else if (t < n) {
            if (za) {
                v.x = za[t];
                if (zb) v.y = zb[t];
            } else {
                v.x = Sr[t] > 0 ? 1.0 : 0.0;
            }
        }
        buf[(bitrev(a, lp1) << lcc) + c] = v;
    }
    lds_fft(buf, tw, lp1, lcc, sgn);
    // w_L^(b c) = w_L1^(m >> lp2) w_L^(m mod L2), m = b c mod L; w_L1^h = -w_L1^(h - L1/2) for h >= L1/2
    for (int e = threadIdx.x; e < (L1 << lcc); e += kFftThreads) {
        const int b = e >> lcc, c = e & (CC - 1);
        const int64_t m = ((int64_t)b * (c0 + c)) & (L - 1);
        const int mh = (int)(m >> lp2), ml = (int)(m & (L2 - 1));
        double2 wh = tw[mh & (L1 / 2 - 1)];
        if (mh >= L1 / 2) wh = make_double2(-wh.x, -wh.y);
        X1[(int64_t)s * L + (int64_t)b * L2 + c0 + c] = cmul(cmul(buf[e], wh), tlo[ml]);
    }
}

// Pass 2.  INV = false: block (row chunk, slot (nparts + 1) + q) transforms the
// rows of column pairs [q ppb, min(np, (q + 1) ppb)) of the ROI (q < nparts) or of
// its mask signal (q = nparts) and writes their summed power spectrum to
// out[slot (nparts + 1) + q][f].  INV = true: block (row chunk, s) finishes the
// inverse transform of signal s and writes out[s][tau] = Re(x[tau]) / L, tau < n.
template <bool INV>
__global__ __launch_bounds__(kFftThreads) void g2fft_pass2_kernel(const double2 *__restrict__ X1, int np, int nparts,
                                                                  int ppb, int lp1, int lp2, int lrb, int64_t n,
                                                                  double *__restrict__ out) {
    extern __shared__ double2 fsm[];
    const int L1 = 1 << lp1, L2 = 1 << lp2, RB = 1 << lrb;
    const int64_t L = (int64_t)L1 * L2;
    const int tile = L2 << lrb;
    double2 *buf = fsm, *tw = fsm + tile;
    fill_twiddles(tw, lp2, INV ? 1.0 : -1.0);
    const int b0 = blockIdx.x << lrb;
    int s_first, s_count;
    if (INV) {
        s_first = blockIdx.y;
        s_count = 1;
    } else {
        const int slot = blockIdx.y / (nparts + 1), q = blockIdx.y % (nparts + 1);
        s_first = slot * (np + 1) + (q < nparts ? q * ppb : np);
        s_count = q < nparts ? std::min(ppb, np - q * ppb) : 1;
    }
    double acc[kFftPerThread];
#pragma unroll
    for (int i = 0; i < kFftPerThread; ++i) acc[i] = 0.0;
    for (int si = 0; si < s_count; ++si) {
        const double2 *src = X1 + (int64_t)(s_first + si) * L;
        if (si > 0) __syncthreads();                  // the previous signal's tile has been read
        for (int e = threadIdx.x; e < tile; e += kFftThreads) {
            const int g = e >> lp2, c = e & (L2 - 1);
            buf[(bitrev(c, lp2) << lrb) + g] = src[(int64_t)(b0 + g) * L2 + c];
        }
        lds_fft(buf, tw, lp2, lrb, INV ? 1.0 : -1.0);
#pragma unroll
        for (int i = 0; i < kFftPerThread; ++i) {
            const int e = threadIdx.x + i * kFftThreads;
            if (e < tile) {
                const double2 x = buf[e];
                acc[i] = INV ? x.x : fma(x.x, x.x, fma(x.y, x.y, acc[i]));
            }
        }
    }
    const double invL = 1.0 / (double)L;
#pragma unroll
    for (int i = 0; i < kFftPerThread; ++i) {
        const int e = threadIdx.x + i * kFftThreads;
        if (e >= tile) continue;
        const int d = e >> lrb, g = e & (RB - 1);
        const int64_t f = b0 + g + (int64_t)L1 * d;
        if (INV) {
            if (f < n) out[(int64_t)blockIdx.y * n + f] = acc[i] * invL;
        } else {
            out[(int64_t)blockIdx.y * L + f] = acc[i];
        }
    }
}

// g2[(r0 + slot) nw + tau] from the two inverse transforms of the ROI: the
// diagonal sum and the pair count (an integer up to rounding).
__global__ void g2fft_finish_kernel(const double *__restrict__ sums, int64_t n, int slot0, double *__restrict__ g2,
                                    int64_t *__restrict__ npairs) {
    const int slot = blockIdx.y;
    const int64_t tau = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tau >= n) return;
    const double a = sums[(int64_t)(2 * slot) * n + tau];
    const int64_t cnt = llrint(sums[(int64_t)(2 * slot + 1) * n + tau]);
    const int64_t o = (int64_t)(slot0 + slot) * n + tau;
    g2[o] = cnt > 0 ? a / (double)cnt : __builtin_nan("");
    if (npairs) npairs[o] = cnt;
}

// Mean and standard deviation of C~_R over its off-diagonal valid pairs
// (t1 != t2, both frames with S_R > 0), from Z alone: with s = sum_t Z[t] and
// G = Z^T Z, the sum of all entries of C~_R = Z Z^T is |s|^2 and the sum of their
// squares is |G|_F^2; the diagonal contributes sum_t |Z[t]|^2 and sum_t |Z[t]|^4.
// One block per ROI; fixed-order reductions in FP64.
constexpr int kStatFrames = 256;                  // frames per block of the partial-sum kernel

// Per (frame chunk, ROI) partial sums: column sums s_j over the chunk's frames
// (a wave-wide reduction per column, four waves combined in LDS), and the
// chunk's sum of |Z[t]|^2, sum of |Z[t]|^4 and count of valid frames.
__global__ __launch_bounds__(256) void ttc_partial_kernel(const double *__restrict__ z,
                                                          const int64_t *__restrict__ roi_sum, int64_t N, int r0,
                                                          int64_t t0, int64_t n, int k, double *__restrict__ ps,
                                                          double *__restrict__ pd) {
    __shared__ double red[4][kMaxRank + 3];
    const int slot = blockIdx.y, chunk = blockIdx.x, nch = gridDim.x;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    const double *zs = z + (int64_t)slot * k * n;
    const int64_t t = (int64_t)chunk * kStatFrames + threadIdx.x;
    const bool in = t < n;
    double d = 0.0;
    for (int j = 0; j < k; ++j) {
        const double v = in ? zs[(int64_t)j * n + t] : 0.0;
        d = fma(v, v, d);
        double w = v;
        for (int off = kWave / 2; off > 0; off >>= 1) w += __shfl_xor(w, off, kWave);
        if (lane == 0) red[wv][j] = w;
    }
    double x[3] = {d, d * d, (in && roi_sum[(int64_t)(r0 + slot) * N + t0 + t] > 0) ? 1.0 : 0.0};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double w = x[q];
        for (int off = kWave / 2; off > 0; off >>= 1) w += __shfl_xor(w, off, kWave);
        if (lane == 0) red[wv][kMaxRank + q] = w;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += 256)
        ps[((int64_t)slot * nch + chunk) * k + j] = red[0][j] + red[1][j] + red[2][j] + red[3][j];
    if (threadIdx.x < 3)
        pd[((int64_t)slot * nch + chunk) * 3 + threadIdx.x] =
            red[0][kMaxRank + threadIdx.x] + red[1][kMaxRank + threadIdx.x] + red[2][kMaxRank + threadIdx.x] +
            red[3][kMaxRank + threadIdx.x];
}

// Mean and standard deviation of C~_R over its off-diagonal valid pairs
// (t1 != t2, both frames with S_R > 0), from Z alone: with s = sum_t Z[t] and
// G = Z^T Z, the sum of all entries of C~_R = Z Z^T is |s|^2 and the sum of their
// squares is |G|_F^2; the diagonal contributes sum_t |Z[t]|^2 and sum_t |Z[t]|^4.
// One block per ROI over the chunk partials, in a fixed order.
__global__ __launch_bounds__(256) void ttc_stats_kernel(const double *__restrict__ ps, const double *__restrict__ pd,
                                                        const double *__restrict__ G, int nch, int k, int slot0,
                                                        double *__restrict__ mean, double *__restrict__ stdev,
                                                        int64_t *__restrict__ npairs) {
    __shared__ double red[2][4];
    const int slot = blockIdx.x;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    double s2 = 0.0;
    for (int j = threadIdx.x; j < k; j += 256) {
        double sj = 0.0;
        for (int c = 0; c < nch; ++c) sj += ps[((int64_t)slot * nch + c) * k + j];
        s2 = fma(sj, sj, s2);
    }
    double g2s = 0.0;
    const double *Gs = G + (int64_t)slot * k * k;
    for (int e = threadIdx.x; e < k * k; e += 256) g2s = fma(Gs[e], Gs[e], g2s);
    for (int off = kWave / 2; off > 0; off >>= 1) {
        s2 += __shfl_xor(s2, off, kWave);
        g2s += __shfl_xor(g2s, off, kWave);
    }
    if (lane == 0) {
        red[0][wv] = s2;
        red[1][wv] = g2s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s2 = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        g2s = red[1][0] + red[1][1] + red[1][2] + red[1][3];
        double d1 = 0.0, d2 = 0.0, nv = 0.0;
        for (int c = 0; c < nch; ++c) {
            const double *p = pd + ((int64_t)slot * nch + c) * 3;
            d1 += p[0];
            d2 += p[1];
            nv += p[2];
        }
        const double noff = nv * (nv - 1.0);
        const int o = slot0 + slot;
        npairs[o] = (int64_t)noff;
        if (noff > 0.0) {
            const double m = (s2 - d1) / noff;
            const double var = (g2s - d2) / noff - m * m;
            mean[o] = m;
            stdev[o] = sqrt(var > 0.0 ? var : 0.0);
        } else {
            mean[o] = __builtin_nan("");
            stdev[o] = __builtin_nan("");
        }
    }
}

struct FftPlan {
    int lp1, lp2, lcc, lrb;
    int64_t L;
};

FftPlan fft_plan(int64_t n) {
    int p = 2;
    while (((int64_t)1 << p) < 2 * n) ++p;
    FftPlan pl;
    pl.lp1 = p / 2;
    pl.lp2 = p - pl.lp1;
    pl.L = (int64_t)1 << p;
    int lcc = 0;                                      // columns per pass-1 tile
    while (lcc < pl.lp2 && (2 << (pl.lp1 + lcc)) <= kFftElems) ++lcc;
    int lrb = 0;                                      // rows per pass-2 tile
    while (lrb < pl.lp1 && (2 << (pl.lp2 + lrb)) <= kFftElems) ++lrb;
    pl.lcc = lcc;
    pl.lrb = lrb;
    return pl;
}

}  // namespace
}  // namespace xpcs

using namespace xpcs;

extern "C" {

xpcs_status g2_from_factors(xpcs_ctx *ctx, const xpcs_factors *f, int32_t roi, int64_t t0, int64_t t1, double *g2,
                            int64_t *npairs) {
    if (!ctx) return XPCS_EINVAL;
    if (!f || !f->V || !f->sigma || !f->roi_npix || !f->roi_sum || !f->roi_gram)
        return fail(ctx, XPCS_EINVAL, "factors or one of their buffers is NULL");
    if (f->N <= 0 || f->M <= 0 || f->k < 1 || f->n_roi < 1) return fail(ctx, XPCS_EINVAL, "bad factor sizes");
    if (!g2) return fail(ctx, XPCS_EINVAL, "g2 must not be NULL");
    if (roi != XPCS_ALL_ROIS && (roi < 0 || roi >= f->n_roi))
        return fail(ctx, XPCS_EINVAL, "roi outside [0, n_roi) and not XPCS_ALL_ROIS");
    if (t0 < 0 || t1 <= t0 || t1 > f->N) return fail(ctx, XPCS_EINVAL, "window must satisfy 0 <= t0 < t1 <= N");
    if (f->k > kMaxRank) return fail(ctx, XPCS_EUNSUPPORTED, "rank above 1024 in g2_from_factors");
    const int64_t n = t1 - t0;
    if (n > ((int64_t)1 << (kFftMaxLog - 1))) return fail(ctx, XPCS_EUNSUPPORTED, "window above 2^21 frames");
    (void)hipSetDevice(ctx->device);
    ws_begin(ctx);
    const int r0 = roi == XPCS_ALL_ROIS ? 0 : roi;
    const int nr = roi == XPCS_ALL_ROIS ? f->n_roi : 1;
    const int k = f->k, np = (k + 1) / 2;
    const FftPlan pl = fft_plan(n);
    const int64_t L = pl.L;
    // ROIs per batch: z, the pass-1 output of every signal, spectra and sums
    // pass 2 splits a ROI's column pairs over nparts blocks per row chunk (partial
    // spectra summed by the inverse pass 1) so that the grid fills the chip
    const int rows = 1 << (pl.lp1 - pl.lrb);
    int ppb = np;
    while (ppb > 1 && (int64_t)rows * std::min(nr, 64) * ((np + ppb - 1) / ppb) < 4096) ppb = (ppb + 1) / 2;
    const int nparts = (np + ppb - 1) / ppb;
    const size_t per_roi = (size_t)k * n * 8 + (size_t)(np + 1) * L * 16 + (size_t)(nparts + 1) * L * 8 +
                           (size_t)2 * n * 8;
    const size_t cap = (size_t)2 << 30;
    const int nb = (int)std::max<size_t>(1, std::min<size_t>((size_t)nr, cap / per_roi));
    const size_t b_l = (size_t)nr * k * k * 8;
    const size_t b_z = (size_t)nb * k * n * 8, b_x = (size_t)nb * (np + 1) * L * 16;
    const size_t b_s = (size_t)nb * (nparts + 1) * L * 8, b_o = (size_t)nb * 2 * n * 8;
    xpcs_status st = ws_reserve(ctx, align_up(b_l, 256) + align_up(b_z, 256) + align_up(b_x, 256) +
                                         align_up(b_s, 256) + align_up(b_o, 256) + 5 * 256);
    if (st) return st;
    auto *Lr = static_cast<double *>(ws_take(ctx, b_l));
    auto *z = static_cast<double *>(ws_take(ctx, b_z));
    auto *X1 = static_cast<double2 *>(ws_take(ctx, b_x));
    auto *spec = static_cast<double *>(ws_take(ctx, b_s));
    auto *sums = static_cast<double *>(ws_take(ctx, b_o));
    if ((st = launch_chol_batched(ctx, f->roi_gram + (int64_t)r0 * k * k, k, nr, Lr))) return st;
    const size_t lds1 = ((size_t)(1 << (pl.lp1 + pl.lcc)) + (1 << pl.lp1) / 2 + (1 << pl.lp2)) * sizeof(double2);
    const size_t lds2 = ((size_t)(1 << (pl.lp2 + pl.lrb)) + (1 << pl.lp2) / 2) * sizeof(double2);
    const unsigned g1x = (unsigned)(1 << (pl.lp2 - pl.lcc)), g2x = (unsigned)(1 << (pl.lp1 - pl.lrb));
    for (int s0 = 0; s0 < nr; s0 += nb) {
        const int m = std::min(nb, nr - s0);
        {
            Phase phase_(ctx, "g2fft_z");
            if ((st = launch_z_rows(ctx, f, Lr + (int64_t)s0 * k * k, r0 + s0, m, t0, n, z, nullptr, nullptr, 0, nullptr)))
                return st;
        }
        {
            Phase phase_(ctx, "g2fft_pass1");
            hipLaunchKernelGGL(g2fft_pass1_kernel<false>, dim3(g1x, (unsigned)(m * (np + 1))), dim3(kFftThreads),
                               lds1, ctx->stream, z, f->roi_sum, f->N, r0 + s0, t0, n, k, np, nullptr, 0, pl.lp1,
                               pl.lp2, pl.lcc, X1);
            XPCS_LAUNCH_CHECK(ctx, "g2fft_pass1");
        }
        {
            Phase phase_(ctx, "g2fft_pass2");
            hipLaunchKernelGGL(g2fft_pass2_kernel<false>, dim3(g2x, (unsigned)(m * (nparts + 1))),
                               dim3(kFftThreads), lds2, ctx->stream, X1, np, nparts, ppb, pl.lp1, pl.lp2, pl.lrb, n,
                               spec);
            XPCS_LAUNCH_CHECK(ctx, "g2fft_pass2");
        }
        {
            Phase phase_(ctx, "g2fft_inverse");
            hipLaunchKernelGGL(g2fft_pass1_kernel<true>, dim3(g1x, (unsigned)(m * 2)), dim3(kFftThreads), lds1,
                               ctx->stream, nullptr, nullptr, f->N, 0, 0, n, k, np, spec, nparts, pl.lp1, pl.lp2,
                               pl.lcc, X1);
            XPCS_LAUNCH_CHECK(ctx, "g2fft_pass1_inverse");
            hipLaunchKernelGGL(g2fft_pass2_kernel<true>, dim3(g2x, (unsigned)(m * 2)), dim3(kFftThreads), lds2,
                               ctx->stream, X1, np, nparts, ppb, pl.lp1, pl.lp2, pl.lrb, n, sums);
            XPCS_LAUNCH_CHECK(ctx, "g2fft_pass2_inverse");
            hipLaunchKernelGGL(g2fft_finish_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)m), dim3(256), 0,
                               ctx->stream, sums, n, s0, g2, npairs);
            XPCS_LAUNCH_CHECK(ctx, "g2fft_finish");
        }
    }
    return XPCS_OK;
}

xpcs_status two_time_stats(xpcs_ctx *ctx, const xpcs_factors *f, int32_t roi, int64_t t0, int64_t t1, double *mean,
                           double *stdev, int64_t *npairs) {
    if (!ctx) return XPCS_EINVAL;
    if (!f || !f->V || !f->sigma || !f->roi_npix || !f->roi_sum || !f->roi_gram)
        return fail(ctx, XPCS_EINVAL, "factors or one of their buffers is NULL");
    if (f->N <= 0 || f->M <= 0 || f->k < 1 || f->n_roi < 1) return fail(ctx, XPCS_EINVAL, "bad factor sizes");
    if (!mean || !stdev || !npairs) return fail(ctx, XPCS_EINVAL, "mean, stdev and npairs must not be NULL");
    if (roi != XPCS_ALL_ROIS && (roi < 0 || roi >= f->n_roi))
        return fail(ctx, XPCS_EINVAL, "roi outside [0, n_roi) and not XPCS_ALL_ROIS");
    if (t0 < 0 || t1 <= t0 || t1 > f->N) return fail(ctx, XPCS_EINVAL, "window must satisfy 0 <= t0 < t1 <= N");
    if (f->k > kMaxRank) return fail(ctx, XPCS_EUNSUPPORTED, "rank above 1024 in two_time_stats");
    (void)hipSetDevice(ctx->device);
    ws_begin(ctx);
    const int64_t n = t1 - t0;
    const int r0 = roi == XPCS_ALL_ROIS ? 0 : roi;
    const int nr = roi == XPCS_ALL_ROIS ? f->n_roi : 1;
    const int k = f->k;
    const int nch = (int)((n + kStatFrames - 1) / kStatFrames);
    const size_t per_roi = (size_t)k * n * 8 + (size_t)k * k * 8 + (size_t)nch * (k + 3) * 8;
    const size_t cap = (size_t)1 << 30;
    const int nb = (int)std::max<size_t>(1, std::min<size_t>((size_t)nr, cap / per_roi));
    const size_t b_l = (size_t)nr * k * k * 8, b_z = (size_t)nb * k * n * 8, b_g = (size_t)nb * k * k * 8;
    const size_t b_ps = (size_t)nb * nch * k * 8, b_pd = (size_t)nb * nch * 3 * 8;
    xpcs_status st = ws_reserve(ctx, align_up(b_l, 256) + align_up(b_z, 256) + align_up(b_g, 256) +
                                         align_up(b_ps, 256) + align_up(b_pd, 256) + 5 * 256);
    if (st) return st;
    auto *Lr = static_cast<double *>(ws_take(ctx, b_l));
    auto *z = static_cast<double *>(ws_take(ctx, b_z));
    auto *G = static_cast<double *>(ws_take(ctx, b_g));
    auto *ps = static_cast<double *>(ws_take(ctx, b_ps));
    auto *pd = static_cast<double *>(ws_take(ctx, b_pd));
    if ((st = launch_chol_batched(ctx, f->roi_gram + (int64_t)r0 * k * k, k, nr, Lr))) return st;
    for (int s0 = 0; s0 < nr; s0 += nb) {
        const int m = std::min(nb, nr - s0);
        {
            Phase phase_(ctx, "g2fft_z");
            if ((st = launch_z_rows(ctx, f, Lr + (int64_t)s0 * k * k, r0 + s0, m, t0, n, z, nullptr, nullptr, 0, nullptr)))
                return st;
        }
        if ((st = launch_tsgram_batched(ctx, z, true, n, n, k, m, (int64_t)k * n, G))) return st;
        Phase phase_(ctx, "ttc_stats");
        hipLaunchKernelGGL(ttc_partial_kernel, dim3((unsigned)nch, (unsigned)m), dim3(256), 0, ctx->stream, z,
                           f->roi_sum, f->N, r0 + s0, t0, n, k, ps, pd);
        XPCS_LAUNCH_CHECK(ctx, "ttc_partial");
        hipLaunchKernelGGL(ttc_stats_kernel, dim3((unsigned)m), dim3(256), 0, ctx->stream, ps, pd, G, nch, k, s0,
                           mean, stdev, npairs);
        XPCS_LAUNCH_CHECK(ctx, "ttc_stats");
    }
    return XPCS_OK;
}

}  // extern "C"
