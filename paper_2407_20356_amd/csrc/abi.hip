// extern "C" entry points: argument checks, workspace layout and the launch
// sequence of each call.  Every arithmetic step runs in the kernels of this
// library; the host only validates and enqueues.
#include <string.h>

#include <algorithm>
#include <string>

#include "internal.hpp"

using namespace xpcs;

namespace {

constexpr int kRawPad = 64;          // int8 MFMA K granularity: ROI ranges padded to 64 pixels

inline int64_t up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

xpcs_status check_frames(xpcs_ctx *ctx, const void *frames, int32_t dtype, int64_t M, int64_t N,
                         const int32_t *labels, int32_t n_roi) {
    if (!frames) return fail(ctx, XPCS_EINVAL, "frames is NULL");
    if (!labels) return fail(ctx, XPCS_EINVAL, "roi_label is NULL");
    if (dtype != XPCS_U8 && dtype != XPCS_U16) return fail(ctx, XPCS_EINVAL, "dtype must be XPCS_U8 or XPCS_U16");
    if (M <= 0 || N <= 0) return fail(ctx, XPCS_EINVAL, "M and N must be positive");
    if (M > 2147483647LL) return fail(ctx, XPCS_EUNSUPPORTED, "more than 2^31-1 pixels");
    if (n_roi < 1) return fail(ctx, XPCS_EINVAL, "n_roi must be >= 1");
    if (n_roi > 4096) return fail(ctx, XPCS_EUNSUPPORTED, "more than 4096 ROIs");
    return XPCS_OK;
}

xpcs_status check_window(xpcs_ctx *ctx, int64_t N, int32_t n_roi, int32_t roi, int64_t t0, int64_t t1, void *C,
                         int32_t c_dtype, int64_t ldc) {
    if (roi != XPCS_ALL_ROIS && (roi < 0 || roi >= n_roi))
        return fail(ctx, XPCS_EINVAL, "roi outside [0, n_roi) and not XPCS_ALL_ROIS");
    if (t0 < 0 || t1 <= t0 || t1 > N) return fail(ctx, XPCS_EINVAL, "window must satisfy 0 <= t0 < t1 <= N");
    if (C) {
        if (c_dtype != XPCS_F32 && c_dtype != XPCS_F64) return fail(ctx, XPCS_EINVAL, "c_dtype must be XPCS_F32 or XPCS_F64");
        if (ldc < t1 - t0) return fail(ctx, XPCS_EINVAL, "ldc smaller than the window");
    }
    return XPCS_OK;
}

size_t g2_part_bytes(int64_t nw, int nr) {
    return (size_t)n_tiles_upper(nw) * nr * kDiag * sizeof(double);
}
size_t g2_cnt_bytes(int64_t nw, int nr) { return (size_t)n_tiles_upper(nw) * nr * kDiag * sizeof(int); }

// Buffers of one compressed correlation call, carved in order from one region
// (the context's workspace, or the static scratch of the call that allocates nothing).
struct CorrPlan {
    int64_t nw = 0;
    int r0 = 0, nr = 0, kp = 0;
    size_t b_op = 0, b_l = 0, b_valid = 0, b_part = 0, b_cnt = 0, b_chol = 0;
    size_t bytes = 0;
};

xpcs_status corr_plan(xpcs_ctx *ctx, const xpcs_factors *f, int32_t roi, int64_t t0, int64_t t1, void *C,
                      int32_t c_dtype, int64_t ldc, double *g2, CorrPlan &p) {
    if (!f || !f->V || !f->sigma || !f->roi_npix || !f->roi_sum || !f->roi_gram)
        return fail(ctx, XPCS_EINVAL, "factors or one of their buffers is NULL");
    if (f->N <= 0 || f->M <= 0 || f->k < 1 || f->n_roi < 1) return fail(ctx, XPCS_EINVAL, "bad factor sizes");
    xpcs_status st = check_window(ctx, f->N, f->n_roi, roi, t0, t1, C, c_dtype, ldc);
    if (st) return st;
    if (!C && !g2) return fail(ctx, XPCS_EINVAL, "nothing to compute: C and g2 are both NULL");
    if (f->k > kMaxRank) return fail(ctx, XPCS_EUNSUPPORTED, "rank above 1024");
    p.nw = t1 - t0;
    p.r0 = roi == XPCS_ALL_ROIS ? 0 : roi;
    p.nr = roi == XPCS_ALL_ROIS ? f->n_roi : 1;
    p.kp = (int)up(f->k, 32);
    p.b_op = (size_t)p.nr * p.nw * p.kp * 2;
    p.b_l = (size_t)p.nr * f->k * f->k * sizeof(double);
    p.b_valid = (size_t)p.nr * p.nw;
    p.b_part = g2 ? g2_part_bytes(p.nw, p.nr) : 0;
    p.b_cnt = g2 ? g2_cnt_bytes(p.nw, p.nr) : 0;
    p.b_chol = chol_batched_work_bytes(f->k, p.nr);
    p.bytes = 2 * align_up(p.b_op, 256) + align_up(p.b_l, 256) + align_up(p.b_valid, 256) + align_up(p.b_part, 256) +
              align_up(p.b_cnt, 256) + align_up(p.b_chol, 256);
    return XPCS_OK;
}

// G_R = L_R L_R^T for the ROIs of the call, Z rows, then the tiles and the g2 reduction.
xpcs_status corr_run(xpcs_ctx *ctx, const xpcs_factors *f, const CorrPlan &p, int64_t t0, void *C, int32_t c_dtype,
                     int64_t ldc, double *g2, int64_t *npairs, char *base) {
    size_t used = 0;
    auto take = [&](size_t b) {
        char *q = base + used;
        used += align_up(b, 256);
        return q;
    };
    auto *z_hi = reinterpret_cast<unsigned short *>(take(p.b_op));
    auto *z_lo = reinterpret_cast<unsigned short *>(take(p.b_op));
    auto *Lr = reinterpret_cast<double *>(take(p.b_l));
    auto *valid = reinterpret_cast<unsigned char *>(take(p.b_valid));
    TileOut o;
    o.C = C;
    o.c_dtype = c_dtype;
    o.ldc = ldc;
    o.c_roi_stride = p.nw * ldc;
    if (g2) {
        o.g2_part = reinterpret_cast<double *>(take(p.b_part));
        o.g2_cnt = reinterpret_cast<int *>(take(p.b_cnt));
    }
    void *chol_work = p.b_chol ? take(p.b_chol) : nullptr;
    xpcs_status st;
    if ((st = launch_chol_batched(ctx, f->roi_gram + (int64_t)p.r0 * f->k * f->k, f->k, p.nr, Lr, chol_work)))
        return st;
    if ((st = launch_lowrank_prep(ctx, f, Lr, p.r0, p.nr, t0, p.nw, p.kp, z_hi, z_lo, valid))) return st;
    if ((st = launch_lowrank_tiles(ctx, z_hi, z_lo, p.kp, valid, p.nw, p.nr, o))) return st;
    if (g2 && (st = launch_g2_reduce(ctx, o.g2_part, o.g2_cnt, p.nw, p.nr, g2, npairs))) return st;
    return XPCS_OK;
}

struct Orth {
    // Orthonormalise the first `ell` columns of a tall column-major matrix with
    // Cholesky QR (FP64 Gram and factor): once when the result only feeds a bf16
    // product (the subspace passes), twice when it is the final basis.
    static xpcs_status run(xpcs_ctx *ctx, const void *A, bool a_f64, int64_t rows, int64_t lda, int ell,
                           void *tmp, bool tmp_f64, double *G, double *R1, double *R2, const TsOut &final_out,
                           int passes = 2) {
        xpcs_status st = launch_tsgram(ctx, A, a_f64, rows, lda, ell, nullptr, nullptr, 1, G);
        if (st) return st;
        st = launch_cholinv(ctx, G, ell, 1e-13, nullptr, R1);
        if (st) return st;
        if (passes == 1) return launch_tsmul(ctx, A, a_f64, rows, lda, ell, R1, ell, nullptr, final_out, true);
        TsOut o1;
        if (tmp_f64) {
            o1.out64 = static_cast<double *>(tmp);
            o1.ld64 = rows;
        } else {
            o1.out32 = static_cast<float *>(tmp);
            o1.ld32 = rows;
        }
        st = launch_tsmul(ctx, A, a_f64, rows, lda, ell, R1, ell, nullptr, o1, true);
        if (st) return st;
        st = launch_tsgram(ctx, tmp, tmp_f64, rows, rows, ell, nullptr, nullptr, 1, G);
        if (st) return st;
        st = launch_cholinv(ctx, G, ell, 1e-13, nullptr, R2);
        if (st) return st;
        return launch_tsmul(ctx, tmp, tmp_f64, rows, rows, ell, R2, ell, nullptr, final_out, true);
    }
};

constexpr int kMaxExactFrames = 4096;

// The paper's construction of the basis (Sec. 2.1, Eqs. 3 and 6): the exact frame Gram
// F F^T, its full FP64 eigendecomposition, the k leading eigenvectors V and
// sigma = sqrt(eigenvalue), the pixel basis U = X V diag(1/sigma) in FP64; the exact ROI
// sums come from the encoding pass over the frames with that basis.
xpcs_status compress_exact(xpcs_ctx *ctx, const void *frames, int32_t dtype, int64_t M, int64_t N,
                           const int32_t *roi_label, int32_t n_roi, int k, double *spectrum, xpcs_factors *out) {
    if (N > kMaxExactFrames) return fail(ctx, XPCS_EUNSUPPORTED, "the exact basis takes at most 4096 frames");
    if (k > M || k > N) return fail(ctx, XPCS_EINVAL, "k larger than min(M, N)");
    if (k > kMaxRank) return fail(ctx, XPCS_EUNSUPPORTED, "rank above 1024");
    (void)hipSetDevice(ctx->device);
    ws_begin(ctx);
    const int L = (int)up(k, 16);
    const int64_t ldq = up(M, 64);
    const FrameProj plan = plan_proj_frames(M, N, L, n_roi, true);
    size_t need = 0;
    auto add = [&](size_t b) { need += align_up(b, 256) + 256; };
    const size_t b_nn = (size_t)N * N * 8, b_tu = (size_t)N * k * 8, b_q16 = (size_t)L * ldq * 2;
    const size_t b_part = (size_t)plan.nchunks * plan.ncols * N * 4, b_z = (size_t)L * N * 8;
    add(b_nn); add(b_nn); add((size_t)N * 8); add(jacobi_block_work_bytes((int)N)); add(b_tu); add((size_t)k * 8);
    add((size_t)k * k * 8); add(b_q16); add(b_q16); add(b_part); add(b_z);
    add((size_t)(n_roi + 1) * 8); add((size_t)(M + n_roi) * 4); add((size_t)(M + n_roi) * 4);
    xpcs_status st;
    if ((st = ws_reserve(ctx, need))) return st;
    auto *H = static_cast<double *>(ws_take(ctx, b_nn));
    auto *P = static_cast<double *>(ws_take(ctx, b_nn));
    auto *lam = static_cast<double *>(ws_take(ctx, (size_t)N * 8));
    void *jw = ws_take(ctx, jacobi_block_work_bytes((int)N));
    auto *Tu = static_cast<double *>(ws_take(ctx, b_tu));
    auto *scale = static_cast<double *>(ws_take(ctx, (size_t)k * 8));
    auto *Tid = static_cast<double *>(ws_take(ctx, (size_t)k * k * 8));
    auto *qhi = static_cast<unsigned short *>(ws_take(ctx, b_q16));
    auto *qlo = static_cast<unsigned short *>(ws_take(ctx, b_q16));
    auto *part = static_cast<float *>(ws_take(ctx, b_part));
    auto *Za = static_cast<double *>(ws_take(ctx, b_z));
    auto *off = static_cast<int64_t *>(ws_take(ctx, (size_t)(n_roi + 1) * 8));
    auto *perm = static_cast<int32_t *>(ws_take(ctx, (size_t)(M + n_roi) * 4));
    auto *qroi = static_cast<int32_t *>(ws_take(ctx, (size_t)(M + n_roi) * 4));

    if ((st = launch_roi_count(ctx, roi_label, M, n_roi, out->roi_npix))) return st;
    // Eq. 3: the Gram of the data and its eigenvectors, Eq. 6: the K largest
    if ((st = launch_frame_gram(ctx, frames, dtype, M, N, H))) return st;
    {
        Phase phase_(ctx, "jacobi");
        if ((st = launch_jacobi_block(ctx, H, (int)N, lam, P, jw))) return st;
    }
    if ((st = launch_select_exact(ctx, lam, P, (int)N, k, Tu, scale, out->sigma, spectrum))) return st;
    // U = X V diag(1 / sigma) (the paper's pixel-space encoding vectors), V = the eigenvectors
    TsOut ou;
    ou.out32 = out->U;
    ou.ld32 = M;
    if ((st = launch_tsmul_counts(ctx, frames, dtype, M, N, Tu, k, scale, ou))) return st;
    if ((st = launch_identity(ctx, Tid, k))) return st;
    TsOut ov;
    ov.out32 = out->V;
    ov.ld32 = N;
    if ((st = launch_tsmul(ctx, Tu, true, N, N, k, Tid, k, nullptr, ov, true))) return st;
    // the exact ROI sums ride along the encoding pass W = X^T U (Eq. 7)
    if ((st = launch_basis_to_bf16(ctx, out->U, M, k, ldq, L, qhi, qlo))) return st;
    if ((st = launch_proj_frames(ctx, frames, dtype, M, N, qhi, qlo, ldq, L, roi_label, n_roi, plan, part))) return st;
    if ((st = launch_proj_frames_reduce(ctx, part, plan, N, L, n_roi, Za, N, out->roi_sum))) return st;
    // per-ROI basis Gram G_R = U_R^T U_R
    if ((st = launch_roi_order(ctx, roi_label, M, n_roi, out->roi_npix, 1, off, perm, qroi, M + n_roi))) return st;
    return launch_tsgram(ctx, out->U, false, M, M, k, perm, off, n_roi, out->roi_gram);
}

}  // namespace

extern "C" {

xpcs_status compress_frames(xpcs_ctx *ctx, const void *frames, int32_t dtype, int64_t M, int64_t N,
                            const int32_t *roi_label, int32_t n_roi, const xpcs_compress_opts *opts,
                            xpcs_factors *out) {
    if (!ctx) return XPCS_EINVAL;
    xpcs_status st = check_frames(ctx, frames, dtype, M, N, roi_label, n_roi);
    if (st) return st;
    if (!opts || !out) return fail(ctx, XPCS_EINVAL, "opts and out must not be NULL");
    if (!out->U || !out->sigma || !out->V || !out->roi_npix || !out->roi_sum || !out->roi_gram)
        return fail(ctx, XPCS_EINVAL, "a factor buffer is NULL");
    if (out->M != M || out->N != N || out->n_roi != n_roi || out->k != opts->k)
        return fail(ctx, XPCS_EINVAL, "factor sizes (M, N, k, n_roi) do not match the call");
    const int k = opts->k;
    if (k < 1) return fail(ctx, XPCS_EINVAL, "k must be >= 1");
    if (opts->precision != XPCS_PREC_BF16 && opts->precision != XPCS_PREC_FP8)
        return fail(ctx, XPCS_EINVAL, "precision must be XPCS_PREC_BF16 or XPCS_PREC_FP8");
    // fp8 subspace passes: counts below 256 split into two exact e4m3 nibble planes
    const bool fp8 = opts->precision == XPCS_PREC_FP8 && !opts->basis;
    if (fp8 && dtype != XPCS_U8) return fail(ctx, XPCS_EUNSUPPORTED, "XPCS_PREC_FP8 takes XPCS_U8 frames");
    if (n_roi > 64) return fail(ctx, XPCS_EUNSUPPORTED, "compress_frames records at most 64 ROI sums");
    if (opts->method != XPCS_BASIS_RANDOMIZED && opts->method != XPCS_BASIS_EXACT)
        return fail(ctx, XPCS_EINVAL, "method must be XPCS_BASIS_RANDOMIZED or XPCS_BASIS_EXACT");
    if (!opts->basis && opts->method == XPCS_BASIS_EXACT)
        return compress_exact(ctx, frames, dtype, M, N, roi_label, n_roi, k, opts->spectrum, out);
    const bool online = opts->basis != nullptr;
    int ell = k + (opts->oversample > 0 ? opts->oversample : 0);
    ell += ell & 1;                                 // the eigensolver pairs columns
    if (online) {
        if (k > kMaxRank) return fail(ctx, XPCS_EUNSUPPORTED, "online basis wider than 1024");
        if (k > M) return fail(ctx, XPCS_EINVAL, "k larger than M");
    } else {
        if (opts->power_iters < 0 || opts->power_iters > 1)
            return fail(ctx, XPCS_EUNSUPPORTED, "power_iters must be 0 or 1");
        if (ell > M || ell > N) return fail(ctx, XPCS_EINVAL, "k + oversample exceeds min(M, N)");
        if (ell > kMaxRank) return fail(ctx, XPCS_EUNSUPPORTED, "k + oversample above 1024");
    }
    (void)hipSetDevice(ctx->device);
    ws_begin(ctx);

    const int cols = online ? k : ell;
    const int L = (int)up(cols, 16);
    const int64_t ldt = up(N, 64), ldq = up(M, 64);     // rows padded to the projections' K steps
    const FrameProj plan = plan_proj_frames(M, N, L, n_roi, true);       // final pass: hi + lo + ROI sums
    const FrameProj plan_q = plan_proj_frames(M, N, L, 0, false);        // power pass: hi only
    // workspace layout
    size_t need = 0;
    auto add = [&](size_t b) { need += align_up(b, 256) + 256; };
    const size_t b_om = (size_t)L * ldt * 2, b_y = (size_t)L * M * 4, b_q16 = (size_t)L * ldq * 2;
    const size_t b_z = (size_t)L * N * 8;
    const size_t b_part = (size_t)std::max(plan.nchunks * plan.ncols, plan_q.nchunks * plan_q.ncols) * N * 4;
    const size_t b_small = (size_t)std::max(ell, k) * std::max(ell, k) * 8;
    add(b_om); add(b_y); add(b_y); add(b_q16); add(b_q16); add(b_z); add(b_z); add(b_part);
    for (int i = 0; i < 6; ++i) add(b_small);
    add(jacobi_rot_bytes(ell > 2 ? ell : 2));
    add((size_t)(n_roi + 1) * 8); add((size_t)(M + n_roi) * 4); add((size_t)(M + n_roi) * 4);
    add((size_t)std::max(ell, k) * 8); add((size_t)std::max(ell, k) * 8);
    add(sketch_need_bytes(M));
    if ((st = ws_reserve(ctx, need))) return st;
    unsigned short *om = static_cast<unsigned short *>(ws_take(ctx, b_om));
    float *Ya = static_cast<float *>(ws_take(ctx, b_y));
    float *Yb = static_cast<float *>(ws_take(ctx, b_y));
    unsigned short *qhi = static_cast<unsigned short *>(ws_take(ctx, b_q16));
    unsigned short *qlo = static_cast<unsigned short *>(ws_take(ctx, b_q16));
    double *Za = static_cast<double *>(ws_take(ctx, b_z));
    double *Zb = static_cast<double *>(ws_take(ctx, b_z));
    float *part = static_cast<float *>(ws_take(ctx, b_part));
    double *G = static_cast<double *>(ws_take(ctx, b_small));
    double *R1 = static_cast<double *>(ws_take(ctx, b_small));
    double *R2 = static_cast<double *>(ws_take(ctx, b_small));
    double *P = static_cast<double *>(ws_take(ctx, b_small));
    double *Tu = static_cast<double *>(ws_take(ctx, b_small));
    double *Tid = static_cast<double *>(ws_take(ctx, b_small));
    void *rot = ws_take(ctx, jacobi_rot_bytes(ell > 2 ? ell : 2));
    int64_t *off = static_cast<int64_t *>(ws_take(ctx, (size_t)(n_roi + 1) * 8));
    int32_t *perm = static_cast<int32_t *>(ws_take(ctx, (size_t)(M + n_roi) * 4));
    int32_t *qroi = static_cast<int32_t *>(ws_take(ctx, (size_t)(M + n_roi) * 4));
    double *lam = static_cast<double *>(ws_take(ctx, (size_t)std::max(ell, k) * 8));
    double *scale = static_cast<double *>(ws_take(ctx, (size_t)std::max(ell, k) * 8));
    int *sk_need = static_cast<int *>(ws_take(ctx, sketch_need_bytes(M)));

    if ((st = launch_roi_count(ctx, roi_label, M, n_roi, out->roi_npix))) return st;

    if (online) {
        if (hipMemcpyAsync(out->U, opts->basis, (size_t)M * k * sizeof(float), hipMemcpyDeviceToDevice,
                           ctx->stream) != hipSuccess)
            return fail(ctx, XPCS_EDEVICE, "copy of the supplied basis failed");
        if ((st = launch_basis_to_bf16(ctx, out->U, M, k, ldq, L, qhi, qlo))) return st;
        if ((st = launch_proj_frames(ctx, frames, dtype, M, N, qhi, qlo, ldq, L, roi_label, n_roi, plan, part)))
            return st;
        if ((st = launch_proj_frames_reduce(ctx, part, plan, N, L, n_roi, Za, N, out->roi_sum))) return st;
        if ((st = launch_column_norms(ctx, Za, N, N, k, out->sigma, scale))) return st;
        if ((st = launch_identity(ctx, Tid, k))) return st;
        TsOut ov;
        ov.out32 = out->V;
        ov.ld32 = N;
        if ((st = launch_tsmul(ctx, Za, true, N, N, k, Tid, k, scale, ov, true))) return st;
    } else {
        // 1. sketch Y0 = X Omega, exact on the int8 MFMA (+-1 signs, integer counts)
        uint8_t *om8 = reinterpret_cast<uint8_t *>(om), *q8 = reinterpret_cast<uint8_t *>(qlo);
        const uint8_t *f8frames = static_cast<const uint8_t *>(frames);
        if ((st = launch_sketch_i8(ctx, frames, dtype, M, N, opts->seed, ell, L, ldt, reinterpret_cast<int8_t *>(om),
                                   Ya, sk_need)))
            return st;
        if (opts->power_iters == 1 && fp8) {
            // 2. the same with e4m3 operands: Q0 = orth(Y0), Z = X^T Q0, Qz = orth(Z), Y1 = X Qz
            TsOut o;
            o.f8 = q8;
            o.ldh = ldq;
            o.Lpad = L;
            o.rows_pad = ldq;
            if ((st = Orth::run(ctx, Ya, false, M, M, ell, Yb, false, G, R1, R2, o, 1))) return st;
            if ((st = launch_proj_frames_f8(ctx, f8frames, M, N, q8, ldq, L, plan_q, part))) return st;
            if ((st = launch_proj_frames_reduce(ctx, part, plan_q, N, L, 0, Za, N, nullptr))) return st;
            TsOut oz;
            oz.f8 = om8;                                // reuse the sketch buffer for Qz
            oz.ldh = ldt;
            oz.Lpad = L;
            oz.rows_pad = ldt;
            if ((st = Orth::run(ctx, Za, true, N, N, ell, Zb, true, G, R1, R2, oz, 1))) return st;
            if ((st = launch_proj_pixels_f8(ctx, f8frames, M, N, om8, ldt, L, Ya))) return st;
        } else if (opts->power_iters == 1) {
            // 2. Q0 = orth(Y0) as bf16; Z = X^T Q0; Qz = orth(Z) as bf16; Y1 = X Qz
            TsOut o;
            o.hi = qhi;
            o.ldh = ldq;
            o.Lpad = L;
            o.rows_pad = ldq;
            if ((st = Orth::run(ctx, Ya, false, M, M, ell, Yb, false, G, R1, R2, o, 1))) return st;
            if ((st = launch_proj_frames(ctx, frames, dtype, M, N, qhi, nullptr, ldq, L, roi_label, 0, plan_q, part)))
                return st;
            if ((st = launch_proj_frames_reduce(ctx, part, plan_q, N, L, 0, Za, N, nullptr))) return st;
            TsOut oz;
            oz.hi = om;                                 // reuse the sketch buffer for Qz
            oz.ldh = ldt;
            oz.Lpad = L;
            oz.rows_pad = ldt;
            if ((st = Orth::run(ctx, Za, true, N, N, ell, Zb, true, G, R1, R2, oz, 1))) return st;
            if ((st = launch_proj_pixels(ctx, frames, dtype, M, N, om, ldt, L, Ya))) return st;
        }
        // 3. Q = orth(Y) in fp32 + bf16 hi/lo
        TsOut oq;
        oq.out32 = Yb;
        oq.ld32 = M;
        oq.hi = qhi;
        oq.lo = qlo;
        oq.ldh = ldq;
        oq.Lpad = L;
        oq.rows_pad = ldq;
        // Orth::run writes its intermediate into the tmp buffer and the result into oq;
        // tmp must differ from both the input (Ya) and the fp32 result (Yb).
        if ((st = launch_tsgram(ctx, Ya, false, M, M, ell, nullptr, nullptr, 1, G))) return st;
        if ((st = launch_cholinv(ctx, G, ell, 1e-13, nullptr, R1))) return st;
        {
            TsOut o1;
            o1.out32 = Yb;
            o1.ld32 = M;
            if ((st = launch_tsmul(ctx, Ya, false, M, M, ell, R1, ell, nullptr, o1, true))) return st;
        }
        if ((st = launch_tsgram(ctx, Yb, false, M, M, ell, nullptr, nullptr, 1, G))) return st;
        if ((st = launch_cholinv(ctx, G, ell, 1e-13, nullptr, R2))) return st;
        oq.out32 = Ya;
        if ((st = launch_tsmul(ctx, Yb, false, M, M, ell, R2, ell, nullptr, oq, true))) return st;
        float *Qf = Ya;
        // 4. W_l = X^T Q with the residual term, and the exact ROI sums
        if ((st = launch_proj_frames(ctx, frames, dtype, M, N, qhi, qlo, ldq, L, roi_label, n_roi, plan, part)))
            return st;
        if ((st = launch_proj_frames_reduce(ctx, part, plan, N, L, n_roi, Za, N, out->roi_sum))) return st;
        // 5. eigendecomposition of W_l^T W_l ranks the l directions (Eq. 3, Eq. 6)
        if ((st = launch_tsgram(ctx, Za, true, N, N, ell, nullptr, nullptr, 1, G))) return st;
        if ((st = launch_jacobi(ctx, G, ell, lam, P, rot))) return st;
        if ((st = launch_select_basis(ctx, lam, P, ell, k, Za, N, N, Tu, scale, out->sigma))) return st;
        // 6. U = Q T_u, V = W_l T_u / sigma
        TsOut ou;
        ou.out32 = out->U;
        ou.ld32 = M;
        if ((st = launch_tsmul(ctx, Qf, false, M, M, ell, Tu, k, nullptr, ou))) return st;
        TsOut ov;
        ov.out32 = out->V;
        ov.ld32 = N;
        if ((st = launch_tsmul(ctx, Za, true, N, N, ell, Tu, k, scale, ov))) return st;
    }
    // 7. per-ROI basis Gram G_R = U_R^T U_R
    if ((st = launch_roi_order(ctx, roi_label, M, n_roi, out->roi_npix, 1, off, perm, qroi, M + n_roi))) return st;
    if ((st = launch_tsgram(ctx, out->U, false, M, M, k, perm, off, n_roi, out->roi_gram))) return st;
    return XPCS_OK;
}

xpcs_status correlate_two_time(xpcs_ctx *ctx, const xpcs_factors *f, int32_t roi, int64_t t0, int64_t t1, void *C,
                               int32_t c_dtype, int64_t ldc, double *g2, int64_t *npairs) {
    if (!ctx) return XPCS_EINVAL;
    CorrPlan plan;
    xpcs_status st = corr_plan(ctx, f, roi, t0, t1, C, c_dtype, ldc, g2, plan);
    if (st) return st;
    (void)hipSetDevice(ctx->device);
    ws_begin(ctx);
    if ((st = ws_reserve(ctx, plan.bytes))) return st;
    return corr_run(ctx, f, plan, t0, C, c_dtype, ldc, g2, npairs, static_cast<char *>(ws_take(ctx, plan.bytes)));
}

xpcs_status correlate_two_time_noalloc(xpcs_ctx *ctx, const xpcs_factors *f, int32_t roi, int64_t t0, int64_t t1,
                                       void *C, int32_t c_dtype, int64_t ldc, double *g2, int64_t *npairs) {
    if (!ctx) return XPCS_EINVAL;
    CorrPlan plan;
    xpcs_status st = corr_plan(ctx, f, roi, t0, t1, C, c_dtype, ldc, g2, plan);
    if (st) return st;
    if (plan.bytes > kStaticScratchBytes)
        return fail(ctx, XPCS_EUNSUPPORTED,
                    "correlate_two_time_noalloc needs " + std::to_string(plan.bytes) +
                        " bytes of scratch; the static scratch holds " + std::to_string(kStaticScratchBytes) +
                        " (fewer ROIs per call or a shorter window)");
    if (!ctx->static_scratch) return fail(ctx, XPCS_EDEVICE, "no static scratch on this device");
    (void)hipSetDevice(ctx->device);
    // phase timing would create events; it is suspended for this call
    const bool timing = ctx->timing;
    ctx->timing = false;
    st = corr_run(ctx, f, plan, t0, C, c_dtype, ldc, g2, npairs, static_cast<char *>(ctx->static_scratch));
    ctx->timing = timing;
    return st;
}

xpcs_status correlate_two_time_raw(xpcs_ctx *ctx, const void *frames, int32_t dtype, int64_t M, int64_t N,
                                   const int32_t *roi_label, int32_t n_roi, int32_t roi, int64_t t0, int64_t t1,
                                   void *C, int32_t c_dtype, int64_t ldc, double *g2, int64_t *npairs,
                                   int64_t *gram_out) {
    if (!ctx) return XPCS_EINVAL;
    xpcs_status st = check_frames(ctx, frames, dtype, M, N, roi_label, n_roi);
    if (st) return st;
    if ((st = check_window(ctx, N, n_roi, roi, t0, t1, C, c_dtype, ldc))) return st;
    if (!C && !g2 && !gram_out) return fail(ctx, XPCS_EINVAL, "nothing to compute: C, g2 and gram_out are NULL");
    (void)hipSetDevice(ctx->device);
    ws_begin(ctx);
    const int64_t nw = t1 - t0;
    const int r0 = roi == XPCS_ALL_ROIS ? 0 : roi;
    const int nr = roi == XPCS_ALL_ROIS ? n_roi : 1;
    const int64_t cap = up(M + (int64_t)n_roi * kRawPad, kRawPad);
    const int64_t ldx = cap;
    size_t need = 0;
    auto add = [&](size_t b) { need += align_up(b, 256) + 256; };
    add((size_t)n_roi * 8); add((size_t)(n_roi + 1) * 8); add((size_t)cap * 4); add((size_t)cap * 4);
    add((size_t)nw * ldx); add((size_t)n_roi * nw * 8); add(256);
    add((size_t)cap * 4); add((size_t)cap * 8); add((size_t)n_roi * 4); add((size_t)n_roi * 4);
    if (g2) { add(g2_part_bytes(nw, nr)); add(g2_cnt_bytes(nw, nr)); }
    if ((st = ws_reserve(ctx, need))) return st;
    auto *npix = static_cast<int64_t *>(ws_take(ctx, (size_t)n_roi * 8));
    auto *off = static_cast<int64_t *>(ws_take(ctx, (size_t)(n_roi + 1) * 8));
    auto *perm = static_cast<int32_t *>(ws_take(ctx, (size_t)cap * 4));
    auto *qroi = static_cast<int32_t *>(ws_take(ctx, (size_t)cap * 4));
    auto *xs = static_cast<int8_t *>(ws_take(ctx, (size_t)nw * ldx));
    auto *S = static_cast<int64_t *>(ws_take(ctx, (size_t)n_roi * nw * 8));
    auto *amax = static_cast<int *>(ws_take(ctx, 256));
    auto *hot = static_cast<int *>(ws_take(ctx, (size_t)cap * 4));
    auto *hq = static_cast<int64_t *>(ws_take(ctx, (size_t)cap * 8));
    auto *hcnt = static_cast<int *>(ws_take(ctx, (size_t)n_roi * 4));
    auto *hbits = static_cast<int *>(ws_take(ctx, (size_t)n_roi * 4));
    TileOut o;
    o.C = C;
    o.c_dtype = c_dtype;
    o.ldc = ldc;
    o.c_roi_stride = nw * ldc;
    o.gram_out = gram_out;
    o.gram_roi_stride = nw * nw;
    if (g2) {
        o.g2_part = static_cast<double *>(ws_take(ctx, g2_part_bytes(nw, nr)));
        o.g2_cnt = static_cast<int *>(ws_take(ctx, g2_cnt_bytes(nw, nr)));
    }
    if ((st = launch_roi_count(ctx, roi_label, M, n_roi, npix))) return st;
    if ((st = launch_roi_order(ctx, roi_label, M, n_roi, npix, kRawPad, off, perm, qroi, cap))) return st;
    if ((st = launch_zero(ctx, amax, 256))) return st;
    if ((st = launch_gather_i8(ctx, frames, dtype, M, t0, nw, perm, qroi, off, n_roi, ldx, xs, S, amax, hot, hq, hcnt,
                               hbits, cap)))
        return st;
    RawHot rh;
    rh.frames = frames;
    rh.dtype = dtype;
    rh.M = M;
    rh.t0 = t0;
    rh.perm = perm;
    rh.hq = hq;
    rh.hcnt = hcnt;
    rh.hbits = hbits;
    if ((st = launch_raw_gram_tiles(ctx, xs, ldx, off, npix, S, nw, r0, nr, amax, rh, o))) return st;
    if (g2 && (st = launch_g2_reduce(ctx, o.g2_part, o.g2_cnt, nw, nr, g2, npairs))) return st;
    return XPCS_OK;
}

xpcs_status g2_from_two_time(xpcs_ctx *ctx, const void *C, int32_t c_dtype, int64_t n, int64_t ldc, double *g2,
                             int64_t *npairs) {
    if (!ctx) return XPCS_EINVAL;
    if (!C || !g2) return fail(ctx, XPCS_EINVAL, "C and g2 must not be NULL");
    if (c_dtype != XPCS_F32 && c_dtype != XPCS_F64) return fail(ctx, XPCS_EINVAL, "c_dtype must be XPCS_F32 or XPCS_F64");
    if (n <= 0 || ldc < n) return fail(ctx, XPCS_EINVAL, "need n > 0 and ldc >= n");
    (void)hipSetDevice(ctx->device);
    ws_begin(ctx);
    const size_t bp = g2_part_bytes(n, 1), bc = g2_cnt_bytes(n, 1);
    xpcs_status st = ws_reserve(ctx, align_up(bp, 256) + align_up(bc, 256) + 512);
    if (st) return st;
    auto *part = static_cast<double *>(ws_take(ctx, bp));
    auto *cnt = static_cast<int *>(ws_take(ctx, bc));
    if ((st = launch_matrix_diag_tiles(ctx, C, c_dtype, n, ldc, part, cnt))) return st;
    return launch_g2_reduce(ctx, part, cnt, n, 1, g2, npairs);
}

}  // extern "C"
