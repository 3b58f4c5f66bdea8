// Online streams (Sec. 2.2, online strategy; Sec. 3.2): a fixed encoding basis,
// frames compressed as they arrive (Eq. 7, one row of W per frame) and their
// compressed two-time correlations with the recent frames (Eqs. 9-10 per ROI)
// computed at once, with g2 sums by lag over the whole history (Eq. 12 read as
// the mean along C's diagonals).
//
// Per ROI the stream keeps, for the last window + max_block frames, the rows
//   z[t] = sqrt(|R|) (w_t / S_R[t]) L_R,   G_R = U_R^T U_R = L_R L_R^T,
// as bf16 hi + lo in a ring (slot = t mod cap), so that C~_R[t][s] = z[t] . z[s].
// A push encodes its frames with the frame-space projection (W rows and exact
// ROI sums in one pass over the counts), forms their z rows, and runs one tile
// pass over (new frames) x (frames within `window` lags), writing the band rows
// C~[t][t - tau] and per-tile diagonal partial sums; the partials are added to
// the g2 sums in a fixed order (deterministic).
#include <math.h>

#include <algorithm>

#include "internal.hpp"
#include "zrows.hpp"

struct xpcs_stream {
    xpcs_ctx *ctx = nullptr;
    int64_t M = 0;
    int dtype = 0, n_roi = 0, k = 0, kp = 0, L16 = 0;
    int64_t window = 0, max_block = 0, cap = 0, ldq = 0;
    int64_t n = 0;                      // frames pushed so far
    size_t bytes = 0;                   // device memory held (counted in the context's budget)
    void *mem = nullptr;
    int32_t *labels = nullptr;          // copy of the ROI labels
    unsigned short *u_hi = nullptr, *u_lo = nullptr;   // basis as split bf16 rows [L16][ldq]
    int64_t *roi_npix = nullptr;
    double *Lr = nullptr;               // [n_roi][k][k] row-major lower Cholesky factors of G_R
    unsigned short *z_hi = nullptr, *z_lo = nullptr;   // [n_roi][cap][kp]
    unsigned char *valid = nullptr;     // [n_roi][cap]
    double *g2_sum = nullptr;           // [n_roi][window]
    int64_t *g2_cnt = nullptr;          // [n_roi][window]
};

namespace xpcs {
namespace {

constexpr int kMaxStreamK = 192;

// Offsets of the pieces of a stream's single device allocation.
struct StreamLayout {
    int kp, L16;
    int64_t cap, ldq;
    size_t o_lab, o_uh, o_ul, o_np, o_lr, o_zh, o_zl, o_va, o_gs, o_gc, total;
};
StreamLayout stream_layout(const xpcs_stream_desc *d) {
    StreamLayout l;
    l.kp = (int)((d->k + 31) / 32 * 32);
    l.L16 = (d->k + 15) / 16 * 16;
    l.cap = d->window + d->max_block;
    l.ldq = (d->M + 63) / 64 * 64;                  // basis rows padded to the projection's K step
    size_t off = 0;
    auto carve = [&](size_t b) { size_t o = off; off += align_up(b, 256); return o; };
    l.o_lab = carve((size_t)d->M * 4);
    l.o_uh = carve((size_t)l.L16 * l.ldq * 2);
    l.o_ul = carve((size_t)l.L16 * l.ldq * 2);
    l.o_np = carve((size_t)d->n_roi * 8);
    l.o_lr = carve((size_t)d->n_roi * d->k * d->k * 8);
    l.o_zh = carve((size_t)d->n_roi * l.cap * l.kp * 2);
    l.o_zl = carve((size_t)d->n_roi * l.cap * l.kp * 2);
    l.o_va = carve((size_t)d->n_roi * l.cap);
    l.o_gs = carve((size_t)d->n_roi * d->window * 8);
    l.o_gc = carve((size_t)d->n_roi * d->window * 8);
    l.total = off;
    return l;
}

// Workspace pieces of a push of nb frames after n frames (every piece 256-byte aligned).
struct PushSizes {
    size_t part, zb, sb, tp, tc, total;
};
PushSizes push_sizes(int64_t M, int L16, int n_roi, int64_t window, int64_t nb, int64_t n) {
    const int64_t c0 = n - window + 1 > 0 ? n - window + 1 : 0;
    const int64_t nbi = (nb + kTile - 1) / kTile, nbj = (n + nb - c0 + kTile - 1) / kTile;
    const int64_t ntiles = (int64_t)n_roi * nbi * nbj;
    const FrameProj plan = plan_proj_frames(M, nb, L16, n_roi, true);
    PushSizes p;
    p.part = (size_t)plan.nchunks * plan.ncols * nb * 4;
    p.zb = (size_t)L16 * nb * 8;
    p.sb = (size_t)n_roi * nb * 8;
    p.tp = (size_t)ntiles * kDiag * 8;
    p.tc = (size_t)ntiles * kDiag * 4;
    p.total = align_up(p.part, 256) + align_up(p.zb, 256) + align_up(p.sb, 256) + align_up(p.tp, 256) +
              align_up(p.tc, 256) + 2048;
    return p;
}
// The same for the Gram pieces taken when the stream opens.
size_t open_ws_bytes(const xpcs_stream_desc *d) {
    const int64_t tcap = d->M + d->n_roi;
    return align_up((size_t)(d->n_roi + 1) * 8, 256) + 2 * align_up((size_t)tcap * 4, 256) +
           align_up((size_t)d->n_roi * d->k * d->k * 8, 256) + 1024;
}
constexpr int kPrepF = 32;          // frames per prep block
constexpr int kPrepC = 16;          // rows of L staged per step
constexpr int kPitch = kTile + 1;
constexpr int kHalf = kTile / 2;

// z rows of the pushed frames: z[t] = sqrt(|R|) (W[t] / S_R[t]) L_R, W[t][a] = Zb[a*nb + i].
__global__ __launch_bounds__(256) void stream_prep_kernel(const double *__restrict__ Zb, int64_t nb,
                                                          const int64_t *__restrict__ Sb,
                                                          const int64_t *__restrict__ roi_npix,
                                                          const double *__restrict__ Lr, int k, int kp,
                                                          int64_t n, int64_t cap, unsigned short *__restrict__ z_hi,
                                                          unsigned short *__restrict__ z_lo,
                                                          unsigned char *__restrict__ valid) {
    __shared__ double wl[kPrepF][kMaxStreamK + kPrepC];
    __shared__ double lc[kPrepC][kMaxStreamK];
    const int r = blockIdx.y;
    const int64_t i0 = (int64_t)blockIdx.x * kPrepF;
    const double sq = sqrt((double)roi_npix[r]);
    const int64_t *S = Sb + (int64_t)r * nb;
    const double *L = Lr + (int64_t)r * k * k;
    const int k16 = (k + kPrepC - 1) / kPrepC * kPrepC;
    for (int idx = threadIdx.x; idx < kPrepF * k16; idx += blockDim.x) {
        const int a = idx / kPrepF, f = idx % kPrepF;
        const int64_t i = i0 + f;
        double w = 0.0;
        if (i < nb && a < k) {
            const int64_t s = S[i];
            if (s > 0) w = Zb[(int64_t)a * nb + i] / (double)s;
        }
        wl[f][a] = w;
    }
    constexpr int kOwn = kPrepF * kMaxStreamK / 256;
    double acc[kOwn];
#pragma unroll
    for (int j = 0; j < kOwn; ++j) acc[j] = 0.0;
    const int nout = kPrepF * k;
    for (int a0 = 0; a0 < k; a0 += kPrepC) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < kPrepC * k; idx += blockDim.x) {
            const int aa = idx / k, b = idx % k;
            lc[aa][b] = a0 + aa < k ? L[(int64_t)(a0 + aa) * k + b] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kOwn; ++j) {
            const int o = threadIdx.x + 256 * j;
            if (o < nout) {
                const int f = o / k, b = o % k;
                double s = acc[j];
#pragma unroll 4
                for (int aa = 0; aa < kPrepC; ++aa) s = fma(wl[f][a0 + aa], lc[aa][b], s);
                acc[j] = s;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kOwn; ++j) {
        const int o = threadIdx.x + 256 * j;
        if (o < nout) {
            const int f = o / k, b = o % k;
            const int64_t i = i0 + f;
            if (i < nb) {
                const int64_t row = (int64_t)r * cap + (n + i) % cap;
                const double zv = sq * acc[j];
                const unsigned short zh = f32_to_bf16_bits((float)zv);
                z_hi[row * kp + b] = zh;
                z_lo[row * kp + b] = f32_to_bf16_bits((float)(zv - (double)bf16_bits_to_f32(zh)));
            }
        }
    }
    for (int idx = threadIdx.x; idx < kPrepF * (kp - k); idx += blockDim.x) {
        const int f = idx / (kp - k), b = k + idx % (kp - k);
        const int64_t i = i0 + f;
        if (i < nb) {
            const int64_t row = (int64_t)r * cap + (n + i) % cap;
            z_hi[row * kp + b] = 0;
            z_lo[row * kp + b] = 0;
        }
    }
    for (int f = threadIdx.x; f < kPrepF; f += blockDim.x) {
        const int64_t i = i0 + f;
        if (i < nb) valid[(int64_t)r * cap + (n + i) % cap] = S[i] > 0 ? 1 : 0;
    }
}

// band[r][i][tau] = NaN for tau > n + i (no frame n + i - tau yet).
__global__ void stream_band_head_kernel(float *band, int n_roi, int64_t nb, int64_t W, int64_t n) {
    const int64_t total = (int64_t)n_roi * nb * W;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t tau = idx % W, i = (idx / W) % nb;
        if (tau > n + i) band[idx] = __builtin_nanf("");
    }
}

// One 128 x 128 tile of (pushed frames t) x (frames s within the window), per ROI.
// Operand rows are staged in LDS one 32-wide K chunk at a time (rows 0..127: t,
// rows 128..255: s), the three split-bf16 products accumulate in FP32, and the
// epilogue (through LDS, 64 rows at a time) writes the band entries and the
// tile's partial sums along its 255 diagonals (lag tau = t0 - s0 + r - c).
constexpr int kZp = 40;
constexpr int kZPer = 2 * 2 * kTile * 4 / 256;
constexpr int kZBytes = 2 * 2 * kTile * kZp * 2;
constexpr int kStageBytes = kHalf * kPitch * 4;
constexpr int kLds = kZBytes > kStageBytes ? kZBytes : kStageBytes;

__global__ __launch_bounds__(256, 2) void stream_tile_kernel(
    const unsigned short *__restrict__ z_hi, const unsigned short *__restrict__ z_lo, int kp,
    const unsigned char *__restrict__ valid, int64_t cap, int64_t n, int64_t nb, int64_t c0, int64_t W, int nbj,
    float *band, double *part, int *pcnt) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[kLds];
    __shared__ int s_ok[2 * kTile];
    unsigned short *zs = reinterpret_cast<unsigned short *>(smem);
    float *stage = reinterpret_cast<float *>(smem);
    const int r = blockIdx.y;
    const int bi = blockIdx.x / nbj, bj = blockIdx.x % nbj;
    const int64_t end = n + nb;
    const int64_t t0 = n + (int64_t)kTile * bi, s0 = c0 + (int64_t)kTile * bj;
    const int64_t D = t0 - s0;
    const int64_t tile = (int64_t)r * gridDim.x + blockIdx.x;
    // no entry with s <= t and t - s < W: nothing to do but clear the partials
    const int64_t t_last = std::min(t0 + kTile - 1, end - 1);
    if (s0 > t_last || D - (kTile - 1) >= W) {
        if (threadIdx.x < kDiag) {
            part[tile * kDiag + threadIdx.x] = 0.0;
            pcnt[tile * kDiag + threadIdx.x] = 0;
        }
        return;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
    const int lr = lane & 15, lg = lane >> 4;
    const int64_t zbase = (int64_t)r * cap;
    {
        const int e = threadIdx.x;
        const int64_t f = e < kTile ? t0 + e : s0 + (e - kTile);
        s_ok[e] = (f >= 0 && f < end) ? (int)valid[zbase + f % cap] : -1;   // -1: no such frame
    }
    // every frame of the tile exists and has photons: the diagonal sums need no checks
    const bool all_ok = __syncthreads_and(s_ok[threadIdx.x] == 1);

    i32x4 nxt[kZPer];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < kZPer; ++q) {
            const int u = threadIdx.x + 256 * q;
            const int arr = u >> 10, row = (u >> 2) & 255, prt = u & 3;
            const int64_t f = row < kTile ? t0 + row : s0 + (row - kTile);
            i32x4 v = {0, 0, 0, 0};
            if (f >= 0 && f < end) {
                const unsigned short *src = (arr ? z_lo : z_hi) + (zbase + f % cap) * kp + k0 + 8 * prt;
                v = *reinterpret_cast<const i32x4 *>(src);
            }
            nxt[q] = v;
        }
    };
    auto put = [&]() {
#pragma unroll
        for (int q = 0; q < kZPer; ++q) {
            const int u = threadIdx.x + 256 * q;
            const int arr = u >> 10, row = (u >> 2) & 255, prt = u & 3;
            *reinterpret_cast<i32x4 *>(zs + (arr * 2 * kTile + row) * kZp + 8 * prt) = nxt[q];
        }
    };
    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
    fetch(0);
    for (int k0 = 0; k0 < kp; k0 += 32) {
        put();
        __syncthreads();
        if (k0 + 32 < kp) fetch(k0 + 32);
        u16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int ra = 64 * wr + 16 * b + lr, rb = kTile + 64 * wc + 16 * b + lr;
            ah[b] = *reinterpret_cast<const u16x8 *>(zs + ra * kZp + 8 * lg);
            al[b] = *reinterpret_cast<const u16x8 *>(zs + (2 * kTile + ra) * kZp + 8 * lg);
            bh[b] = *reinterpret_cast<const u16x8 *>(zs + rb * kZp + 8 * lg);
            bl[b] = *reinterpret_cast<const u16x8 *>(zs + (2 * kTile + rb) * kZp + 8 * lg);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                acc[a][b] = mfma_bf16(al[a], bh[b], acc[a][b]);
                acc[a][b] = mfma_bf16(ah[a], bl[b], acc[a][b]);
                acc[a][b] = mfma_bf16(ah[a], bh[b], acc[a][b]);
            }
        __syncthreads();
    }

    double dsum = 0.0;
    int dcnt = 0;
    for (int h = 0; h < 2; ++h) {
        if (wr == h) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int c = 64 * wc + 16 * b + lr;
                const bool cok = s_ok[kTile + c] == 1;
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int rl = 16 * a + 4 * lg + e;
                        const bool ok = cok && s_ok[kHalf * h + rl] == 1;
                        stage[rl * kPitch + c] = ok ? acc[a][b][e] : __builtin_nanf("");
                    }
            }
        }
        __syncthreads();
        // band rows: row t = t0 + 64h + rl, column s = s0 + c at lag t - s
        if (band) {
            for (int pass = 0; pass < kHalf / 2; ++pass) {
                const int rl = 2 * pass + (threadIdx.x >> 7), c = threadIdx.x & 127;
                const int64_t t = t0 + kHalf * h + rl, s = s0 + c, tau = t - s;
                if (t < end && s >= 0 && tau >= 0 && tau < W)
                    band[((int64_t)r * nb + (t - n)) * W + tau] = stage[rl * kPitch + c];
            }
        }
        // diagonal d = r - c of the tile: lag D + d, rows of this half with c in [0, 128)
        if (threadIdx.x < kDiag) {
            const int d = threadIdx.x - (kTile - 1);
            const int64_t tau = D + d;
            if (tau >= 0 && tau < W) {
                int lo = kHalf * h, hi = kHalf * h + kHalf;
                if (lo < d) lo = d;                       // c = r - d >= 0
                if (hi > kTile + d) hi = kTile + d;       // c < 128
                if (all_ok) {
#pragma unroll 8
                    for (int rr = lo; rr < hi; ++rr) dsum += (double)stage[(rr - kHalf * h) * kPitch + rr - d];
                    dcnt += hi > lo ? hi - lo : 0;
                } else {
                    for (int rr = lo; rr < hi; ++rr) {
                        if (s_ok[rr] < 0 || s_ok[kTile + rr - d] < 0) continue;
                        const float v = stage[(rr - kHalf * h) * kPitch + rr - d];
                        if (v == v) {
                            dsum += (double)v;
                            dcnt += 1;
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < kDiag) {
        part[tile * kDiag + threadIdx.x] = dsum;
        pcnt[tile * kDiag + threadIdx.x] = dcnt;
    }
}

// g2 sums += the push's tile partials, lag by lag, tiles in a fixed order.
__global__ void stream_g2_acc_kernel(const double *__restrict__ part, const int *__restrict__ pcnt, int n_roi,
                                     int nbi, int nbj, int64_t n, int64_t c0, int64_t W, double *g2_sum,
                                     int64_t *g2_cnt) {
    const int64_t total = (int64_t)n_roi * W;
    const int ntiles = nbi * nbj;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(idx / W);
        const int64_t tau = idx % W;
        double s = 0.0;
        int64_t c = 0;
        for (int bi = 0; bi < nbi; ++bi)
            for (int bj = 0; bj < nbj; ++bj) {
                const int64_t D = n + (int64_t)kTile * bi - (c0 + (int64_t)kTile * bj);
                const int64_t d = tau - D;
                if (d < -(kTile - 1) || d > kTile - 1) continue;
                const int64_t at = ((int64_t)r * ntiles + bi * nbj + bj) * kDiag + d + kTile - 1;
                s += part[at];
                c += pcnt[at];
            }
        if (c) {
            g2_sum[idx] += s;
            g2_cnt[idx] += c;
        }
    }
}

__global__ void stream_g2_out_kernel(const double *__restrict__ g2_sum, const int64_t *__restrict__ g2_cnt,
                                     int64_t total, double *g2, int64_t *npairs) {
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = g2_cnt[idx];
        if (g2) g2[idx] = c ? g2_sum[idx] / (double)c : __builtin_nan("");
        if (npairs) npairs[idx] = c;
    }
}

inline int grid_for(int64_t total) {
    int64_t g = (total + 255) / 256;
    return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

size_t stream_state_bytes(const xpcs_stream_desc *d) { return stream_layout(d).total; }

size_t stream_workspace_bytes(const xpcs_stream_desc *d) {
    // the Gram pieces of the open, and the largest push: every block size, with
    // the band of the window fully populated (n >= window - 1 frames before it)
    size_t w = open_ws_bytes(d);
    const int L16 = stream_layout(d).L16;
    for (int64_t nb = 1; nb <= d->max_block; ++nb) {
        const size_t p = push_sizes(d->M, L16, d->n_roi, d->window, nb, d->window).total;
        w = p > w ? p : w;
    }
    return w;
}

}  // namespace xpcs

using namespace xpcs;

extern "C" {

xpcs_status xpcs_stream_open(xpcs_ctx *ctx, const xpcs_stream_desc *d, xpcs_stream **out) {
    if (!ctx) return XPCS_EINVAL;
    if (!d || !out) return fail(ctx, XPCS_EINVAL, "desc or out is NULL");
    *out = nullptr;
    if (!d->roi_label || !d->basis) return fail(ctx, XPCS_EINVAL, "roi_label or basis is NULL");
    if (d->M <= 0) return fail(ctx, XPCS_EINVAL, "M must be positive");
    if (d->dtype != XPCS_U8 && d->dtype != XPCS_U16) return fail(ctx, XPCS_EINVAL, "dtype must be XPCS_U8 or XPCS_U16");
    if (d->n_roi < 1) return fail(ctx, XPCS_EINVAL, "n_roi must be >= 1");
    if (d->n_roi > 64) return fail(ctx, XPCS_EUNSUPPORTED, "a stream records at most 64 ROIs");
    if (d->k < 1 || d->k > d->M) return fail(ctx, XPCS_EINVAL, "k must be in 1..M");
    if (d->k > kMaxRank) return fail(ctx, XPCS_EUNSUPPORTED, "basis wider than 1024");
    if (d->window < 1 || d->window > 65536) return fail(ctx, XPCS_EINVAL, "window must be in 1..65536");
    if (d->max_block < 1 || d->max_block > 4096) return fail(ctx, XPCS_EINVAL, "max_block must be in 1..4096");
    (void)hipSetDevice(ctx->device);

    auto *s = new xpcs_stream;
    const StreamLayout lay = stream_layout(d);
    s->ctx = ctx;
    s->M = d->M;
    s->dtype = d->dtype;
    s->n_roi = d->n_roi;
    s->k = d->k;
    s->kp = lay.kp;
    s->L16 = lay.L16;
    s->window = d->window;
    s->max_block = d->max_block;
    s->cap = lay.cap;
    s->ldq = lay.ldq;
    const size_t off = lay.total;
    s->bytes = off;
    if (ctx->budget && ctx->ws.capacity + ctx->scratch.capacity + ctx->persistent + s->bytes > ctx->budget) {
        delete s;
        return fail(ctx, XPCS_EBUDGET, "stream state of " + std::to_string(off) + " bytes exceeds the HBM budget");
    }
    hipError_t e = hipMalloc(&s->mem, off);
    if (e != hipSuccess) {
        delete s;
        return check_hip(ctx, e, "hipMalloc(stream)");
    }
    ctx->persistent += s->bytes;
    char *base = static_cast<char *>(s->mem);
    s->labels = reinterpret_cast<int32_t *>(base + lay.o_lab);
    s->u_hi = reinterpret_cast<unsigned short *>(base + lay.o_uh);
    s->u_lo = reinterpret_cast<unsigned short *>(base + lay.o_ul);
    s->roi_npix = reinterpret_cast<int64_t *>(base + lay.o_np);
    s->Lr = reinterpret_cast<double *>(base + lay.o_lr);
    s->z_hi = reinterpret_cast<unsigned short *>(base + lay.o_zh);
    s->z_lo = reinterpret_cast<unsigned short *>(base + lay.o_zl);
    s->valid = reinterpret_cast<unsigned char *>(base + lay.o_va);
    s->g2_sum = reinterpret_cast<double *>(base + lay.o_gs);
    s->g2_cnt = reinterpret_cast<int64_t *>(base + lay.o_gc);

    auto bail = [&](xpcs_status st) {
        xpcs_stream_close(s);
        return st;
    };
    xpcs_status st;
    if ((e = hipMemcpyAsync(s->labels, d->roi_label, (size_t)d->M * 4, hipMemcpyDeviceToDevice, ctx->stream)))
        return bail(check_hip(ctx, e, "copy of the ROI labels"));
    if ((st = launch_basis_to_bf16(ctx, d->basis, d->M, d->k, s->ldq, s->L16, s->u_hi, s->u_lo))) return bail(st);
    if ((st = launch_roi_count(ctx, s->labels, d->M, d->n_roi, s->roi_npix))) return bail(st);
    // G_R = U_R^T U_R over each ROI's pixels, then its Cholesky factor
    ws_begin(ctx);
    const int64_t tcap = d->M + d->n_roi;
    const size_t b_g = (size_t)d->n_roi * d->k * d->k * 8;
    if ((st = ws_reserve(ctx, open_ws_bytes(d)))) return bail(st);
    auto *roff = static_cast<int64_t *>(ws_take(ctx, (size_t)(d->n_roi + 1) * 8));
    auto *perm = static_cast<int32_t *>(ws_take(ctx, (size_t)tcap * 4));
    auto *qroi = static_cast<int32_t *>(ws_take(ctx, (size_t)tcap * 4));
    auto *gram = static_cast<double *>(ws_take(ctx, b_g));
    if ((st = launch_roi_order(ctx, s->labels, d->M, d->n_roi, s->roi_npix, 1, roff, perm, qroi, tcap))) return bail(st);
    if ((st = launch_tsgram(ctx, d->basis, false, d->M, d->M, d->k, perm, roff, d->n_roi, gram))) return bail(st);
    if ((st = launch_chol_batched(ctx, gram, d->k, d->n_roi, s->Lr))) return bail(st);
    if ((st = launch_zero(ctx, s->g2_sum, (size_t)d->n_roi * d->window * 8))) return bail(st);
    if ((st = launch_zero(ctx, s->g2_cnt, (size_t)d->n_roi * d->window * 8))) return bail(st);
    // (the validity bytes sit in a 256-byte aligned piece: clearing up to a multiple of 4 stays inside it)
    if ((st = launch_zero(ctx, s->valid, align_up((size_t)d->n_roi * s->cap, 4)))) return bail(st);
    *out = s;
    return XPCS_OK;
}

xpcs_status xpcs_stream_push(xpcs_stream *s, const void *frames, int64_t nb, void *band, int32_t c_dtype) {
    if (!s) return XPCS_EINVAL;
    xpcs_ctx *ctx = s->ctx;
    if (!frames) return fail(ctx, XPCS_EINVAL, "frames is NULL");
    if (nb < 1 || nb > s->max_block) return fail(ctx, XPCS_EINVAL, "nframes must be in 1..max_block");
    if (band && c_dtype != XPCS_F32) return fail(ctx, XPCS_EINVAL, "band rows are written as XPCS_F32");
    (void)hipSetDevice(ctx->device);
    ws_begin(ctx);
    const int64_t W = s->window, n = s->n;
    const int64_t c0 = n - W + 1 > 0 ? n - W + 1 : 0;
    const int nbi = (int)((nb + kTile - 1) / kTile);
    const int nbj = (int)((n + nb - c0 + kTile - 1) / kTile);
    const FrameProj plan = plan_proj_frames(s->M, nb, s->L16, s->n_roi, true);
    const PushSizes ps = push_sizes(s->M, s->L16, s->n_roi, W, nb, n);
    xpcs_status st;
    if ((st = ws_reserve(ctx, ps.total))) return st;
    auto *part = static_cast<float *>(ws_take(ctx, ps.part));
    auto *Zb = static_cast<double *>(ws_take(ctx, ps.zb));
    auto *Sb = static_cast<int64_t *>(ws_take(ctx, ps.sb));
    auto *tp = static_cast<double *>(ws_take(ctx, ps.tp));
    auto *tc = static_cast<int *>(ws_take(ctx, ps.tc));
    // 1. W rows and exact ROI sums of the new frames (one pass over their counts)
    if ((st = launch_proj_frames(ctx, frames, s->dtype, s->M, nb, s->u_hi, s->u_lo, s->ldq, s->L16, s->labels,
                                 s->n_roi, plan, part)))
        return st;
    if ((st = launch_proj_frames_reduce(ctx, part, plan, nb, s->L16, s->n_roi, Zb, nb, Sb))) return st;
    // 2. their z rows into the ring
    {
        Phase phase_(ctx, "stream_prep");
        if (s->k > kMaxStreamK) {
            if ((st = launch_z_rows_wide(ctx, Zb, true, nullptr, nb, 0, Sb, nb, 0, s->roi_npix, 0, s->Lr, s->k,
                                         s->n_roi, nb, nullptr, s->z_hi, s->z_lo, s->kp, s->valid, s->cap, n,
                                         s->cap)))
                return st;
        } else {
            dim3 grid((unsigned)((nb + kPrepF - 1) / kPrepF), (unsigned)s->n_roi);
            hipLaunchKernelGGL(stream_prep_kernel, grid, dim3(256), 0, ctx->stream, Zb, nb, Sb, s->roi_npix, s->Lr,
                               s->k, s->kp, n, s->cap, s->z_hi, s->z_lo, s->valid);
            XPCS_LAUNCH_CHECK(ctx, "stream_prep");
        }
    }
    // 3. band rows and per-tile diagonal sums
    {
        Phase phase_(ctx, "stream_tiles");
        float *bf = static_cast<float *>(band);
        if (bf && n < W - 1) {
            hipLaunchKernelGGL(stream_band_head_kernel, dim3(grid_for((int64_t)s->n_roi * nb * W)), dim3(256), 0,
                               ctx->stream, bf, s->n_roi, nb, W, n);
            XPCS_LAUNCH_CHECK(ctx, "stream_band_head");
        }
        if ((int64_t)nbi * nbj > 2147483647LL) return fail(ctx, XPCS_EUNSUPPORTED, "window too large");
        dim3 grid((unsigned)(nbi * nbj), (unsigned)s->n_roi);
        hipLaunchKernelGGL(stream_tile_kernel, grid, dim3(256), 0, ctx->stream, s->z_hi, s->z_lo, s->kp, s->valid,
                           s->cap, n, nb, c0, W, nbj, bf, tp, tc);
        XPCS_LAUNCH_CHECK(ctx, "stream_tiles");
    }
    // 4. g2 sums
    {
        Phase phase_(ctx, "stream_g2");
        hipLaunchKernelGGL(stream_g2_acc_kernel, dim3(grid_for((int64_t)s->n_roi * W)), dim3(256), 0, ctx->stream,
                           tp, tc, s->n_roi, nbi, nbj, n, c0, W, s->g2_sum, s->g2_cnt);
        XPCS_LAUNCH_CHECK(ctx, "stream_g2");
    }
    s->n += nb;
    return XPCS_OK;
}

xpcs_status xpcs_stream_g2(xpcs_stream *s, double *g2, int64_t *npairs) {
    if (!s) return XPCS_EINVAL;
    xpcs_ctx *ctx = s->ctx;
    if (!g2 && !npairs) return XPCS_OK;
    (void)hipSetDevice(ctx->device);
    const int64_t total = (int64_t)s->n_roi * s->window;
    hipLaunchKernelGGL(stream_g2_out_kernel, dim3(grid_for(total)), dim3(256), 0, ctx->stream, s->g2_sum,
                       s->g2_cnt, total, g2, npairs);
    XPCS_LAUNCH_CHECK(ctx, "stream_g2_out");
    return XPCS_OK;
}

int64_t xpcs_stream_frames(const xpcs_stream *s) { return s ? s->n : 0; }

namespace {
const char kStreamMagic[8] = {'X', 'P', 'C', 'S', 'S', 'T', 'R', 1};
enum { kSM, kSDtype, kSRoi, kSK, kSWindow, kSMaxBlock, kSN, kSBytes, kSFields };
}  // namespace

xpcs_status xpcs_stream_save(xpcs_stream *s, const char *path) {
    if (!s) return XPCS_EINVAL;
    xpcs_ctx *ctx = s->ctx;
    if (!path) return fail(ctx, XPCS_EINVAL, "path is NULL");
    (void)hipSetDevice(ctx->device);
    PersistFile pf;
    if (pf.open_write(path)) return fail(ctx, XPCS_EINVAL, std::string("cannot write ") + path);
    const int64_t hdr[kSFields] = {s->M, s->dtype, s->n_roi, s->k, s->window, s->max_block, s->n,
                                   (int64_t)s->bytes};
    if (pf.write_header(kStreamMagic, hdr, kSFields)) return fail(ctx, XPCS_EDEVICE, "write failed");
    return pf.write_device(ctx, s->mem, s->bytes);
}

xpcs_status xpcs_stream_load(xpcs_ctx *ctx, const char *path, xpcs_stream **out) {
    if (!ctx) return XPCS_EINVAL;
    if (!path || !out) return fail(ctx, XPCS_EINVAL, "path and out must not be NULL");
    *out = nullptr;
    (void)hipSetDevice(ctx->device);
    PersistFile pf;
    if (pf.open_read(path)) return fail(ctx, XPCS_EINVAL, std::string("cannot read ") + path);
    int64_t hdr[kSFields];
    if (pf.read_header(kStreamMagic, hdr, kSFields))
        return fail(ctx, XPCS_EINVAL, "not a stream file, or a corrupt header");
    xpcs_stream_desc d{};
    d.M = hdr[kSM];
    d.dtype = (int32_t)hdr[kSDtype];
    d.n_roi = (int32_t)hdr[kSRoi];
    d.k = (int32_t)hdr[kSK];
    d.window = hdr[kSWindow];
    d.max_block = hdr[kSMaxBlock];
    if (d.M <= 0 || d.n_roi < 1 || d.n_roi > 64 || d.k < 1 || d.k > kMaxRank || d.window < 1 ||
        d.window > 65536 || d.max_block < 1 || d.max_block > 4096 || (d.dtype != XPCS_U8 && d.dtype != XPCS_U16) ||
        hdr[kSN] < 0)
        return fail(ctx, XPCS_EINVAL, "corrupt stream header");
    const StreamLayout lay = stream_layout(&d);
    if ((int64_t)lay.total != hdr[kSBytes]) return fail(ctx, XPCS_EINVAL, "the stream file's layout differs");
    auto *s = new xpcs_stream;
    s->ctx = ctx;
    s->M = d.M;
    s->dtype = d.dtype;
    s->n_roi = d.n_roi;
    s->k = d.k;
    s->kp = lay.kp;
    s->L16 = lay.L16;
    s->window = d.window;
    s->max_block = d.max_block;
    s->cap = lay.cap;
    s->ldq = lay.ldq;
    s->n = hdr[kSN];
    s->bytes = lay.total;
    if (ctx->budget && ctx->ws.capacity + ctx->scratch.capacity + ctx->persistent + s->bytes > ctx->budget) {
        delete s;
        return fail(ctx, XPCS_EBUDGET, "stream state of " + std::to_string(lay.total) + " bytes exceeds the HBM budget");
    }
    hipError_t e = hipMalloc(&s->mem, s->bytes);
    if (e != hipSuccess) {
        delete s;
        return check_hip(ctx, e, "hipMalloc(stream)");
    }
    ctx->persistent += s->bytes;
    char *base = static_cast<char *>(s->mem);
    s->labels = reinterpret_cast<int32_t *>(base + lay.o_lab);
    s->u_hi = reinterpret_cast<unsigned short *>(base + lay.o_uh);
    s->u_lo = reinterpret_cast<unsigned short *>(base + lay.o_ul);
    s->roi_npix = reinterpret_cast<int64_t *>(base + lay.o_np);
    s->Lr = reinterpret_cast<double *>(base + lay.o_lr);
    s->z_hi = reinterpret_cast<unsigned short *>(base + lay.o_zh);
    s->z_lo = reinterpret_cast<unsigned short *>(base + lay.o_zl);
    s->valid = reinterpret_cast<unsigned char *>(base + lay.o_va);
    s->g2_sum = reinterpret_cast<double *>(base + lay.o_gs);
    s->g2_cnt = reinterpret_cast<int64_t *>(base + lay.o_gc);
    const xpcs_status st = pf.read_device(ctx, s->mem, s->bytes);
    if (st) {
        xpcs_stream_close(s);
        return st;
    }
    *out = s;
    return XPCS_OK;
}

void xpcs_stream_close(xpcs_stream *s) {
    if (!s) return;
    if (s->mem) {
        (void)hipSetDevice(s->ctx->device);
        (void)hipStreamSynchronize(s->ctx->stream);
        (void)hipFree(s->mem);
        s->ctx->persistent -= s->bytes;
    }
    delete s;
}

}  // extern "C"
