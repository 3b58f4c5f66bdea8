// Rows of the symmetric operand of the compressed correlation (Sec. 2.1, Eqs. 8-10
// per ROI): Z[t] = sqrt(|R|) (W[t] / S_R[t]) L_R with W = V diag(sigma) and
// G_R = L_R L_R^T, formed in FP64 for the ROIs r0 .. r0 + nb - 1 and frames
// t0 .. t0 + n - 1 (zero where S_R[t] = 0).  Two output forms:
//  - z64 != NULL: FP64, column-major per ROI, z64[(slot k + j) n + t];
//  - z_hi, z_lo != NULL: split bf16 (hi + lo), frame-major per ROI,
//    z_*[(slot n + t) kp + j], columns k .. kp-1 zero (kp = k rounded up to 32),
//    and valid[slot n + t] = S_R[t] > 0.
#pragma once

#include "internal.hpp"

namespace xpcs {
xpcs_status launch_z_rows(xpcs_ctx *ctx, const xpcs_factors *f, const double *Lr, int r0, int nb, int64_t t0,
                          int64_t n, double *z64, unsigned short *z_hi, unsigned short *z_lo, int kp,
                          unsigned char *valid);
// The same for any rank, from a general source: W[a ldw + w_t0 + t] (fp32 or fp64,
// times wscale[a] when wscale != NULL), S[roi s_stride + s_t0 + t], roi = r0 + slot,
// L_R at Lr + slot k^2; split-bf16 rows at slot rows_cap + (ring0 + t) mod ring_cap.
xpcs_status launch_z_rows_wide(xpcs_ctx *ctx, const void *W, bool w_f64, const double *wscale, int64_t ldw,
                               int64_t w_t0, const int64_t *S, int64_t s_stride, int64_t s_t0, const int64_t *npix,
                               int r0, const double *Lr, int k, int nb, int64_t n, double *z64,
                               unsigned short *z_hi, unsigned short *z_lo, int kp, unsigned char *valid,
                               int64_t rows_cap, int64_t ring0, int64_t ring_cap);
}  // namespace xpcs
