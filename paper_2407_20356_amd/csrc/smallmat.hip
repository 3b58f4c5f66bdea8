// Small dense FP64 steps of the compression: orthonormalisation of the
// tall-skinny sketches (Cholesky QR), the l x l symmetric eigendecomposition that
// ranks the sketched directions by their eigenvalue (Sec. 2.1, Eq. 3: the
// encoding vectors are Gram eigenvectors; Eq. 6: keep the K largest), and the
// tall x small products that assemble the basis.
#include <math.h>

#include "internal.hpp"

namespace xpcs {
namespace {

constexpr int kMaxSmall = 192;                    // largest l handled on chip
constexpr int kPacked = kMaxSmall * (kMaxSmall + 1) / 2;

// ---------------------------------------------------------------- tall-skinny Gram
// Partial Grams over row chunks: part[(seg*gridDim.x + blk)][a][b] (upper 4x4 blocks
// written in full).  A thread owns BPT 4x4 blocks of the upper block triangle.
constexpr int kGramRows = 32;

template <typename T, int BPT>
__global__ __launch_bounds__(256) void tsgram_kernel(const T *__restrict__ A, int64_t rows, int64_t lda, int ncols,
                                                     const int32_t *__restrict__ row_idx,
                                                     const int64_t *__restrict__ seg_off, double *part) {
    __shared__ double tile[kGramRows * (kMaxSmall + 4)];
    const int seg = blockIdx.y;
    const int nc4 = (ncols + 3) / 4;
    const int pitch = nc4 * 4;
    const int nblk = nc4 * (nc4 + 1) / 2;
    int64_t r_begin = 0, r_end = rows;
    if (seg_off) {
        r_begin = seg_off[seg];
        r_end = seg_off[seg + 1];
    }
    const int64_t span = r_end - r_begin;
    const int64_t per = (span + gridDim.x - 1) / gridDim.x;
    const int64_t my0 = r_begin + per * blockIdx.x;
    const int64_t my1 = my0 + per < r_end ? my0 + per : r_end;

    int ab[BPT], bb[BPT];
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        int b = threadIdx.x + 256 * k;
        ab[k] = bb[k] = -1;
        if (b < nblk) {
            // linear b -> (x <= y) in the row-major upper block triangle
            int x = 0, rem = b;
            while (rem >= nc4 - x) {
                rem -= nc4 - x;
                ++x;
            }
            ab[k] = x;
            bb[k] = x + rem;
        }
    }
    double acc[BPT][4][4];
#pragma unroll
    for (int k = 0; k < BPT; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[k][i][j] = 0.0;

    for (int64_t r0 = my0; r0 < my1; r0 += kGramRows) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < kGramRows * pitch; idx += 256) {
            const int rr = idx / pitch, c = idx % pitch;
            const int64_t r = r0 + rr;
            double v = 0.0;
            if (r < my1 && c < ncols) {
                int64_t src = row_idx ? (int64_t)row_idx[r] : r;
                if (src >= 0) v = (double)A[(int64_t)c * lda + src];
            }
            tile[rr * pitch + c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            if (ab[k] >= 0) {
                const int a4 = 4 * ab[k], b4 = 4 * bb[k];
#pragma unroll 4
                for (int rr = 0; rr < kGramRows; ++rr) {
                    double x[4], y[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        x[i] = tile[rr * pitch + a4 + i];
                        y[i] = tile[rr * pitch + b4 + i];
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) acc[k][i][j] = fma(x[i], y[j], acc[k][i][j]);
                }
            }
        }
    }
    double *out = part + ((int64_t)seg * gridDim.x + blockIdx.x) * pitch * pitch;
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        if (ab[k] >= 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) out[(4 * ab[k] + i) * pitch + 4 * bb[k] + j] = acc[k][i][j];
        }
    }
}

// G[seg][a][b] = sum over parts of part[.][ra][rb], (ra, rb) the copy in an upper block.
// 8 threads per entry sum interleaved parts; the 8 sums are added in a fixed order.
__global__ __launch_bounds__(256) void tsgram_reduce_kernel(const double *__restrict__ part, int nparts, int ncols,
                                                            int pitch, double *__restrict__ G) {
    __shared__ double red[256];
    const int seg = blockIdx.y;
    const int64_t n2 = (int64_t)ncols * ncols;
    const int sub = threadIdx.x & 7;
    const int64_t idx = (int64_t)blockIdx.x * 32 + (threadIdx.x >> 3);
    double s = 0.0;
    if (idx < n2) {
        const int a = (int)(idx / ncols), b = (int)(idx % ncols);
        int ra = a, rb = b;
        if (a / 4 > b / 4) {
            ra = b;
            rb = a;
        }
        const double *p = part + (int64_t)seg * nparts * pitch * pitch + (int64_t)ra * pitch + rb;
        for (int k = sub; k < nparts; k += 8) s += p[(int64_t)k * pitch * pitch];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (sub == 0 && idx < n2) {
        double t = 0.0;
        for (int q = 0; q < 8; ++q) t += red[threadIdx.x + q];
        G[(int64_t)seg * n2 + idx] = t;
    }
}

// ---------------------------------------------------------------- Cholesky + inverse
// L (packed lower, LDS) with pivots below rel_tol * max(diag) dropped (column
// zeroed); Rinv = L^{-T} written column-major.  For n <= kInvLds the inverse is
// built row by row in LDS (row i of L^{-1} from rows < i, all columns in
// parallel); larger n solve one column per thread against global memory.
__device__ __forceinline__ int pidx_lower(int i, int j) { return i * (i + 1) / 2 + j; }
constexpr int kInvLds = 128;
constexpr int kPackedInv = kInvLds * (kInvLds + 1) / 2;

template <bool LDS_INV>
__global__ __launch_bounds__(1024) void cholinv_kernel(const double *__restrict__ G, int n, double rel_tol,
                                                       double *__restrict__ Rinv, int *flags) {
    __shared__ double L[LDS_INV ? kPackedInv : kPacked];
    __shared__ double Li[LDS_INV ? kPackedInv : 1];
    __shared__ double s_piv;
    __shared__ double s_max;
    __shared__ int s_kept;
    const int tid = threadIdx.x;
    const int ty = tid >> 5, tx = tid & 31;
    for (int i = ty; i < n; i += 32)
        for (int j = tx; j <= i; j += 32) L[pidx_lower(i, j)] = G[(int64_t)i * n + j];
    if (tid == 0) {
        double m = 0.0;
        for (int i = 0; i < n; ++i) m = fmax(m, G[(int64_t)i * n + i]);
        s_max = m;
        s_kept = 0;
    }
    __syncthreads();
    const double thresh = rel_tol * s_max;
    for (int j = 0; j < n; ++j) {
        if (tid == 0) {
            const double d = L[pidx_lower(j, j)];
            if (d > thresh && d > 0.0) {
                s_piv = sqrt(d);
                ++s_kept;
            } else {
                s_piv = 0.0;
            }
        }
        __syncthreads();
        const double piv = s_piv;
        const double rp = piv > 0.0 ? 1.0 / piv : 0.0;
        for (int i = j + 1 + tid; i < n; i += blockDim.x) L[pidx_lower(i, j)] *= rp;
        if (tid == 0) L[pidx_lower(j, j)] = piv;
        __syncthreads();
        for (int r = j + 1 + ty; r < n; r += 32) {
            const double lrj = L[pidx_lower(r, j)];
            if (lrj == 0.0) continue;
            for (int c = j + 1 + tx; c <= r; c += 32) L[pidx_lower(r, c)] -= lrj * L[pidx_lower(c, j)];
        }
        __syncthreads();
    }
    if (tid == 0 && s_kept == 0) atomicOr(&flags[kFlagNumeric], 1);
    if constexpr (LDS_INV) {
        // L^{-1} by right-looking elimination on [L | I]: row j is final once scaled,
        // then removed from the rows below it.
        for (int i = ty; i < n; i += 32)
            for (int c = tx; c <= i; c += 32) Li[pidx_lower(i, c)] = (i == c) ? 1.0 : 0.0;
        __syncthreads();
        for (int j = 0; j < n; ++j) {
            const double ljj = L[pidx_lower(j, j)];
            const double rj = ljj != 0.0 ? 1.0 / ljj : 0.0;
            for (int c = tid; c <= j; c += blockDim.x) Li[pidx_lower(j, c)] *= rj;
            __syncthreads();
            for (int i = j + 1 + ty; i < n; i += 32) {
                const double lij = L[pidx_lower(i, j)];
                if (lij == 0.0) continue;
                for (int c = tx; c <= j; c += 32) Li[pidx_lower(i, c)] -= lij * Li[pidx_lower(j, c)];
            }
            __syncthreads();
        }
        // Rinv (column-major) = Linv^T: Rinv[c][i] = Linv[i][c] at i*n + c
        for (int i = ty; i < n; i += 32)
            for (int c = tx; c < n; c += 32) Rinv[(int64_t)i * n + c] = c <= i ? Li[pidx_lower(i, c)] : 0.0;
    } else {
        for (int c = tid; c < n; c += blockDim.x) {
            for (int i = 0; i < c; ++i) Rinv[(int64_t)i * n + c] = 0.0;
            for (int i = c; i < n; ++i) {
                const double lii = L[pidx_lower(i, i)];
                double x = 0.0;
                if (lii != 0.0) {
                    double s = (i == c) ? 1.0 : 0.0;
                    for (int m = c; m < i; ++m) s -= L[pidx_lower(i, m)] * Rinv[(int64_t)m * n + c];
                    x = s / lii;
                }
                Rinv[(int64_t)i * n + c] = x;
            }
        }
    }
}

// Batched Cholesky factor: one block per matrix G[bch] (n x n, symmetric PSD),
// L[bch] row-major lower triangular (upper part zero), pivots below
// rel_tol * max(diag) dropped (their column of L is zero).
__global__ __launch_bounds__(1024) void chol_batched_kernel(const double *__restrict__ Gb, int n, double rel_tol,
                                                            double *__restrict__ Lb) {
    __shared__ double L[kPacked];
    __shared__ double s_piv, s_max;
    const double *G = Gb + (int64_t)blockIdx.x * n * n;
    double *Lo = Lb + (int64_t)blockIdx.x * n * n;
    const int tid = threadIdx.x, ty = tid >> 5, tx = tid & 31;
    for (int i = ty; i < n; i += 32)
        for (int j = tx; j <= i; j += 32) L[pidx_lower(i, j)] = 0.5 * (G[(int64_t)i * n + j] + G[(int64_t)j * n + i]);
    if (tid == 0) {
        double m = 0.0;
        for (int i = 0; i < n; ++i) m = fmax(m, G[(int64_t)i * n + i]);
        s_max = m;
    }
    __syncthreads();
    const double thresh = rel_tol * s_max;
    for (int j = 0; j < n; ++j) {
        if (tid == 0) {
            const double d = L[pidx_lower(j, j)];
            s_piv = (d > thresh && d > 0.0) ? sqrt(d) : 0.0;
        }
        __syncthreads();
        const double piv = s_piv;
        const double rp = piv > 0.0 ? 1.0 / piv : 0.0;
        for (int i = j + 1 + tid; i < n; i += blockDim.x) L[pidx_lower(i, j)] *= rp;
        if (tid == 0) L[pidx_lower(j, j)] = piv;
        __syncthreads();
        for (int r = j + 1 + ty; r < n; r += 32) {
            const double lrj = L[pidx_lower(r, j)];
            if (lrj == 0.0) continue;
            for (int c = j + 1 + tx; c <= r; c += 32) L[pidx_lower(r, c)] -= lrj * L[pidx_lower(c, j)];
        }
        __syncthreads();
    }
    for (int i = ty; i < n; i += 32)
        for (int j = tx; j < n; j += 32) Lo[(int64_t)i * n + j] = j <= i ? L[pidx_lower(i, j)] : 0.0;
}

// C = A B for small column-major n x n matrices (one block).
__global__ __launch_bounds__(256) void small_matmul_kernel(const double *__restrict__ A, const double *__restrict__ B,
                                                           int n, double *__restrict__ C) {
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int col = idx / n, row = idx % n;
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += A[(int64_t)k * n + row] * B[(int64_t)col * n + k];
        C[idx] = s;
    }
}

// ---------------------------------------------------------------- tall x small product
// Thread per row, 32 output columns per pass.  T is given row-major (Tr[i*m + j]),
// so the 32 coefficients of row i are one uniform, contiguous read that every
// lane shares; the row of A is streamed once per pass.
constexpr int kTsCols = 32;

template <typename TA>
__global__ __launch_bounds__(256) void tsmul_kernel(const TA *__restrict__ A, int64_t rows, int64_t lda, int n,
                                                    const double *__restrict__ Tr, int m,
                                                    const double *__restrict__ colscale, float *out32,
                                                    int64_t ld32, double *out64, int64_t ld64, unsigned short *hi,
                                                    unsigned short *lo, int64_t ldh, int Lpad, int64_t rows_pad) {
    const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool live = row < rows;
    const int64_t rr = live ? row : 0;
    for (int j0 = 0; j0 < m; j0 += kTsCols) {
        double acc[kTsCols];
#pragma unroll
        for (int jj = 0; jj < kTsCols; ++jj) acc[jj] = 0.0;
        if (j0 + kTsCols <= m) {
            for (int i = 0; i < n; ++i) {
                const double ai = (double)A[(int64_t)i * lda + rr];
                const double *t = Tr + (int64_t)i * m + j0;
#pragma unroll
                for (int jj = 0; jj < kTsCols; ++jj) acc[jj] = fma(ai, t[jj], acc[jj]);
            }
        } else {
            for (int i = 0; i < n; ++i) {
                const double ai = (double)A[(int64_t)i * lda + rr];
                const double *t = Tr + (int64_t)i * m + j0;
#pragma unroll
                for (int jj = 0; jj < kTsCols; ++jj)
                    if (j0 + jj < m) acc[jj] = fma(ai, t[jj], acc[jj]);
            }
        }
        if (live) {
#pragma unroll
            for (int jj = 0; jj < kTsCols; ++jj) {
                const int j = j0 + jj;
                if (j < m) {
                    double v = acc[jj];
                    if (colscale) v *= colscale[j];
                    if (out32) out32[(int64_t)j * ld32 + row] = (float)v;
                    if (out64) out64[(int64_t)j * ld64 + row] = v;
                    if (hi) {
                        const unsigned short h = f32_to_bf16_bits((float)v);
                        hi[(int64_t)j * ldh + row] = h;
                        if (lo) lo[(int64_t)j * ldh + row] = f32_to_bf16_bits((float)(v - (double)bf16_bits_to_f32(h)));
                    }
                }
            }
        }
    }
    // zero padding of the bf16 rows: columns [m, Lpad) for live rows, all columns for pad rows
    if (hi && row < rows_pad) {
        for (int j = live ? m : 0; j < Lpad; ++j) {
            hi[(int64_t)j * ldh + row] = 0;
            if (lo) lo[(int64_t)j * ldh + row] = 0;
        }
    }
}

// Tr[i*m + j] = T[j*n + i] (column-major n x m to row-major).
__global__ void transpose_small_kernel(const double *__restrict__ T, int n, int m, double *__restrict__ Tr) {
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * m; idx += gridDim.x * blockDim.x) {
        const int i = idx / m, j = idx % m;
        Tr[idx] = T[(int64_t)j * n + i];
    }
}

// ---------------------------------------------------------------- Jacobi eigensolver
// Parallel-order (round-robin) cyclic Jacobi on a symmetric n x n matrix, n even.
// In step s the n/2 disjoint pairs are (0, x(0)) and (x(a), x(m-a)), a = 1..n/2-1,
// with m = n-1 and x(i) = 1 + (i + s) mod m; every pair occurs once per sweep.
// B lives in LDS as the packed upper triangle.  The eigenvectors P = J_1 J_2 ...
// are accumulated in LDS when they fit (n <= kJacobiPLds); otherwise every
// step's rotations are logged and replayed row-parallel afterwards.
__device__ __forceinline__ void rr_pair(int s, int a, int n, int &p, int &q) {
    const int m = n - 1;
    int u, v;
    if (a == 0) {
        u = 0;
        v = 1 + (s % m);
    } else {
        u = 1 + ((a + s) % m);
        v = 1 + ((m - a + s) % m);
    }
    p = u < v ? u : v;
    q = u < v ? v : u;
}
__device__ __forceinline__ int pidx_upper(int i, int j) { return j * (j + 1) / 2 + i; }   // i <= j

constexpr int kMaxSweeps = 30;
constexpr int kJacobiPLds = 112;

template <bool P_LDS>
__global__ __launch_bounds__(1024) void jacobi_kernel(const double *__restrict__ Bg, int n, double *__restrict__ lam,
                                                      double *__restrict__ Pout, double2 *__restrict__ rot_log,
                                                      int *__restrict__ nsteps_out, int *flags) {
    constexpr int kPk = P_LDS ? kJacobiPLds * (kJacobiPLds + 1) / 2 : kPacked;
    __shared__ double B[kPk];
    __shared__ double P[P_LDS ? kJacobiPLds * kJacobiPLds : 1];
    __shared__ double2 rot[kMaxSmall / 2];
    __shared__ int pp[kMaxSmall / 2], qq[kMaxSmall / 2];
    __shared__ double red_off[16], red_dg[16];
    __shared__ int s_done;
    const int tid = threadIdx.x, ty = tid >> 5, tx = tid & 31, h = n / 2, m = n - 1;
    for (int j = ty; j < n; j += 32)
        for (int i = tx; i <= j; i += 32) B[pidx_upper(i, j)] = 0.5 * (Bg[(int64_t)i * n + j] + Bg[(int64_t)j * n + i]);
    if constexpr (P_LDS) {
        for (int i = ty; i < n; i += 32)
            for (int j = tx; j < n; j += 32) P[i * n + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    int nsteps = 0;
    bool converged = false;
    for (int sweep = 0; sweep <= kMaxSweeps; ++sweep) {
        double off = 0.0, dg = 0.0;
        for (int j = ty; j < n; j += 32)
            for (int i = tx; i <= j; i += 32) {
                const double v = B[pidx_upper(i, j)];
                if (i == j)
                    dg += v * v;
                else
                    off += v * v;
            }
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_xor(off, o);
            dg += __shfl_xor(dg, o);
        }
        if ((tid & 63) == 0) {
            red_off[tid >> 6] = off;
            red_dg[tid >> 6] = dg;
        }
        __syncthreads();
        if (tid == 0) {
            double so = 0.0, sd = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
                so += red_off[w];
                sd += red_dg[w];
            }
            s_done = (so <= 1e-26 * sd) || so == 0.0;
        }
        __syncthreads();
        if (s_done) {
            converged = true;
            break;
        }
        if (sweep == kMaxSweeps) break;
        for (int s = 0; s < m; ++s) {
            if (tid < h) {
                int p, q;
                rr_pair(s, tid, n, p, q);
                pp[tid] = p;
                qq[tid] = q;
                const double app = B[pidx_upper(p, p)], aqq = B[pidx_upper(q, q)], apq = B[pidx_upper(p, q)];
                double c = 1.0, sn = 0.0;
                if (fabs(apq) > 1e-300 && fabs(apq) > 1e-18 * sqrt(fabs(app) * fabs(aqq))) {
                    const double tau = (aqq - app) / (2.0 * apq);
                    double t;
                    if (fabs(tau) > 1e150)
                        t = 0.5 / tau;
                    else
                        t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    sn = t * c;
                }
                rot[tid] = make_double2(c, sn);
                if constexpr (!P_LDS) rot_log[(int64_t)nsteps * h + tid] = make_double2(c, sn);
            }
            __syncthreads();
            // B <- J^T B J on the 2x2 blocks of pairs (a <= b)
            for (int a = ty; a < h; a += 32) {
                const int pa = pp[a], qa = qq[a];
                const double ca = rot[a].x, sa = rot[a].y;
                for (int b = a + tx; b < h; b += 32) {
                    if (a == b) {
                        const int ipp = pidx_upper(pa, pa), iqq = pidx_upper(qa, qa), ipq = pidx_upper(pa, qa);
                        const double app = B[ipp], aqq = B[iqq], apq = B[ipq];
                        B[ipp] = ca * ca * app - 2.0 * ca * sa * apq + sa * sa * aqq;
                        B[iqq] = sa * sa * app + 2.0 * ca * sa * apq + ca * ca * aqq;
                        B[ipq] = 0.0;
                    } else {
                        const int pb = pp[b], qb = qq[b];
                        const double cb = rot[b].x, sb = rot[b].y;
                        const int i1 = pa < pb ? pidx_upper(pa, pb) : pidx_upper(pb, pa);
                        const int i2 = pa < qb ? pidx_upper(pa, qb) : pidx_upper(qb, pa);
                        const int i3 = qa < pb ? pidx_upper(qa, pb) : pidx_upper(pb, qa);
                        const int i4 = qa < qb ? pidx_upper(qa, qb) : pidx_upper(qb, qa);
                        const double x = B[i1], y = B[i2], z = B[i3], w = B[i4];
                        const double x1 = cb * x - sb * y, y1 = sb * x + cb * y;
                        const double z1 = cb * z - sb * w, w1 = sb * z + cb * w;
                        B[i1] = ca * x1 - sa * z1;
                        B[i3] = sa * x1 + ca * z1;
                        B[i2] = ca * y1 - sa * w1;
                        B[i4] = sa * y1 + ca * w1;
                    }
                }
            }
            if constexpr (P_LDS) {
                // P <- P J: rows i, pairs a
                for (int i = ty; i < n; i += 32)
                    for (int a = tx; a < h; a += 32) {
                        const int p = pp[a], q = qq[a];
                        const double c = rot[a].x, sn = rot[a].y;
                        const double x = P[i * n + p], y = P[i * n + q];
                        P[i * n + p] = c * x - sn * y;
                        P[i * n + q] = sn * x + c * y;
                    }
            }
            __syncthreads();
            ++nsteps;
        }
    }
    for (int i = tid; i < n; i += blockDim.x) lam[i] = B[pidx_upper(i, i)];
    if constexpr (P_LDS) {
        for (int i = ty; i < n; i += 32)
            for (int j = tx; j < n; j += 32) Pout[(int64_t)i * n + j] = P[i * n + j];
    }
    if (tid == 0) {
        *nsteps_out = nsteps;
        if (!converged) atomicOr(&flags[kFlagNumeric], 1);
    }
}

// Eigenvectors from the rotation log: row i of P = e_i^T J_1 J_2 ... J_S, 8 rows per
// block; the rotations of 16 steps are staged in LDS at a time.
constexpr int kReplayRows = 8;
constexpr int kReplayBatch = 16;
__global__ __launch_bounds__(256) void jacobi_replay_kernel(const double2 *__restrict__ rot_log,
                                                            const int *__restrict__ nsteps_ptr, int n,
                                                            double *__restrict__ P) {
    __shared__ double rowv[kReplayRows][kMaxSmall];
    __shared__ double2 cs[kReplayBatch][kMaxSmall / 2];
    const int h = n / 2, m = n - 1;
    const int r0 = blockIdx.x * kReplayRows;
    for (int idx = threadIdx.x; idx < kReplayRows * n; idx += blockDim.x) {
        const int rr = idx / n, j = idx % n;
        rowv[rr][j] = (r0 + rr == j) ? 1.0 : 0.0;
    }
    const int nsteps = *nsteps_ptr;
    for (int st0 = 0; st0 < nsteps; st0 += kReplayBatch) {
        const int nb = nsteps - st0 < kReplayBatch ? nsteps - st0 : kReplayBatch;
        __syncthreads();
        for (int idx = threadIdx.x; idx < nb * h; idx += blockDim.x)
            cs[idx / h][idx % h] = rot_log[(int64_t)(st0 + idx / h) * h + idx % h];
        __syncthreads();
        for (int b = 0; b < nb; ++b) {
            const int s = (st0 + b) % m;
            for (int idx = threadIdx.x; idx < kReplayRows * h; idx += blockDim.x) {
                const int rr = idx / h, a = idx % h;
                int p, q;
                rr_pair(s, a, n, p, q);
                const double2 c = cs[b][a];
                const double x = rowv[rr][p], y = rowv[rr][q];
                rowv[rr][p] = c.x * x - c.y * y;
                rowv[rr][q] = c.y * x + c.x * y;
            }
            __syncthreads();
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kReplayRows * n; idx += blockDim.x) {
        const int rr = idx / n, j = idx % n;
        if (r0 + rr < n) P[(int64_t)(r0 + rr) * n + j] = rowv[rr][j];
    }
}

// ---------------------------------------------------------------- basis selection
// perm by decreasing eigenvalue (ties by index), T_u[i][r] = P[i][perm[r]], sigma.
__global__ __launch_bounds__(256) void select_kernel(const double *__restrict__ lam, const double *__restrict__ P,
                                                     int n, int k, double *__restrict__ T_u,
                                                     double *__restrict__ sigma, int *__restrict__ perm) {
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        int rank = 0;
        const double lj = lam[j];
        for (int i = 0; i < n; ++i) {
            const double li = lam[i];
            rank += (li > lj) || (li == lj && i < j);
        }
        if (rank < k) {
            perm[rank] = j;
            sigma[rank] = sqrt(fmax(lj, 0.0));
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < n * k; idx += blockDim.x) {
        const int r = idx / n, i = idx % n;
        T_u[(int64_t)r * n + i] = P[(int64_t)i * n + perm[r]];
    }
}

// Sign of each column: the entry of largest magnitude (first such index) of
// Wk[:, r] becomes positive.  Flips T_u column r and sets scale_v[r] = 1 / sigma.
__global__ __launch_bounds__(256) void sign_fix_kernel(const double *__restrict__ Wk, int64_t N, int64_t ldw,
                                                       int n, double *__restrict__ T_u,
                                                       const double *__restrict__ sigma, double *__restrict__ scale_v) {
    const int r = blockIdx.x;
    __shared__ double s_val[256];
    __shared__ int64_t s_idx[256];
    double best = -1.0;
    int64_t bidx = 0;
    double bval = 0.0;
    for (int64_t t = threadIdx.x; t < N; t += blockDim.x) {
        const double v = Wk[(int64_t)r * ldw + t];
        if (fabs(v) > best) {
            best = fabs(v);
            bidx = t;
            bval = v;
        }
    }
    s_val[threadIdx.x] = best;
    s_idx[threadIdx.x] = bidx;
    __shared__ double s_sgn[256];
    s_sgn[threadIdx.x] = bval;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double a = s_val[threadIdx.x], b = s_val[threadIdx.x + o];
            const int64_t ia = s_idx[threadIdx.x], ib = s_idx[threadIdx.x + o];
            if (b > a || (b == a && ib < ia)) {
                s_val[threadIdx.x] = b;
                s_idx[threadIdx.x] = ib;
                s_sgn[threadIdx.x] = s_sgn[threadIdx.x + o];
            }
        }
        __syncthreads();
    }
    const double sg = s_sgn[0] < 0.0 ? -1.0 : 1.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) T_u[(int64_t)r * n + i] *= sg;
    if (threadIdx.x == 0) {
        const double sv = sigma[r];
        scale_v[r] = sv > 0.0 ? 1.0 / sv : 0.0;   // the sign is already in T_u
    }
}

__global__ __launch_bounds__(256) void column_norm_kernel(const double *__restrict__ W, int64_t N, int64_t ldw,
                                                          double *__restrict__ sigma, double *__restrict__ scale) {
    const int j = blockIdx.x;
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < N; t += blockDim.x) {
        const double v = W[(int64_t)j * ldw + t];
        s += v * v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double nrm = sqrt(red[0]);
        sigma[j] = nrm;
        scale[j] = nrm > 0.0 ? 1.0 / nrm : 0.0;
    }
}

__global__ void basis_to_bf16_kernel(const float *__restrict__ U, int64_t M, int k, int64_t ldq, int Lpad,
                                     unsigned short *__restrict__ hi, unsigned short *__restrict__ lo) {
    const int64_t total = (int64_t)Lpad * ldq;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = idx / ldq, p = idx % ldq;
        unsigned short h = 0, l = 0;
        if (j < k && p < M) {
            const float v = U[j * M + p];
            h = f32_to_bf16_bits(v);
            l = f32_to_bf16_bits(v - bf16_bits_to_f32(h));
        }
        hi[idx] = h;
        if (lo) lo[idx] = l;
    }
}

__global__ void identity_kernel(double *T, int n) {
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * n; idx += gridDim.x * blockDim.x)
        T[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
}

}  // namespace

size_t jacobi_rot_bytes(int n) {
    return (size_t)(kMaxSweeps + 1) * (size_t)(n - 1) * (size_t)(n / 2) * sizeof(double2) + 256;
}

xpcs_status launch_tsgram(xpcs_ctx *ctx, const void *A, bool a_f64, int64_t rows, int64_t lda, int ncols,
                          const int32_t *row_idx, const int64_t *seg_off, int nseg, double *G) {
    Phase phase_(ctx, "tsgram");
    if (ncols > kMaxSmall) return fail(ctx, XPCS_EUNSUPPORTED, "Gram wider than 192 columns");
    const int nc4 = (ncols + 3) / 4;
    const int pitch = nc4 * 4;
    const int nblk = nc4 * (nc4 + 1) / 2;
    const int bpt = (nblk + 255) / 256;
    int nparts = (int)((rows + 1023) / 1024);
    if (nparts > 256) nparts = 256;
    if (seg_off) nparts = (int)(256 / (nseg > 0 ? nseg : 1)) + 1;
    if (nparts < 1) nparts = 1;
    const size_t pbytes = (size_t)nseg * nparts * pitch * pitch * sizeof(double);
    xpcs_status st;
    double *part = static_cast<double *>(scratch_get(ctx, pbytes, &st));
    if (!part) return st;
    dim3 grid(nparts, nseg);
#define XPCS_TSG(T, B)                                                                                         \
    hipLaunchKernelGGL((tsgram_kernel<T, B>), grid, dim3(256), 0, ctx->stream, static_cast<const T *>(A), rows, \
                       lda, ncols, row_idx, seg_off, part)
#define XPCS_TSG_T(T)                   \
    switch (bpt) {                      \
        case 1: XPCS_TSG(T, 1); break;  \
        case 2: XPCS_TSG(T, 2); break;  \
        case 3: XPCS_TSG(T, 3); break;  \
        case 4: XPCS_TSG(T, 4); break;  \
        default: XPCS_TSG(T, 5); break; \
    }
    if (a_f64) {
        XPCS_TSG_T(double)
    } else {
        XPCS_TSG_T(float)
    }
#undef XPCS_TSG_T
#undef XPCS_TSG
    XPCS_LAUNCH_CHECK(ctx, "tsgram");
    hipLaunchKernelGGL(tsgram_reduce_kernel, dim3((ncols * ncols + 31) / 32, nseg), dim3(256), 0, ctx->stream,
                       part, nparts, ncols, pitch, G);
    XPCS_LAUNCH_CHECK(ctx, "tsgram_reduce");
    return XPCS_OK;
}

xpcs_status launch_cholinv(xpcs_ctx *ctx, const double *G, int n, double rel_tol, const double *Rprev,
                           double *Rinv) {
    Phase phase_(ctx, "cholinv");
    if (n > kMaxSmall) return fail(ctx, XPCS_EUNSUPPORTED, "Cholesky larger than 192");
    double *dst = Rinv;
    if (Rprev) {
        xpcs_status st;
        dst = static_cast<double *>(scratch_get(ctx, (size_t)n * n * sizeof(double), &st));
        if (!dst) return st;
    }
    if (n <= kInvLds)
        hipLaunchKernelGGL(cholinv_kernel<true>, dim3(1), dim3(1024), 0, ctx->stream, G, n, rel_tol, dst, ctx->flags);
    else
        hipLaunchKernelGGL(cholinv_kernel<false>, dim3(1), dim3(1024), 0, ctx->stream, G, n, rel_tol, dst, ctx->flags);
    XPCS_LAUNCH_CHECK(ctx, "cholinv");
    if (Rprev) {
        hipLaunchKernelGGL(small_matmul_kernel, dim3(1), dim3(256), 0, ctx->stream, Rprev, dst, n, Rinv);
        XPCS_LAUNCH_CHECK(ctx, "small_matmul");
    }
    return XPCS_OK;
}

xpcs_status launch_chol_batched(xpcs_ctx *ctx, const double *G, int n, int nb, double *L) {
    Phase phase_(ctx, "chol_batched");
    if (n > kMaxSmall) return fail(ctx, XPCS_EUNSUPPORTED, "Cholesky larger than 192");
    hipLaunchKernelGGL(chol_batched_kernel, dim3(nb), dim3(1024), 0, ctx->stream, G, n, 1e-13, L);
    XPCS_LAUNCH_CHECK(ctx, "chol_batched");
    return XPCS_OK;
}

xpcs_status launch_tsmul(xpcs_ctx *ctx, const void *A, bool a_f64, int64_t rows, int64_t lda, int n,
                         const double *T, int m, const double *colscale, const TsOut &out) {
    Phase phase_(ctx, "tsmul");
    if (n > kMaxSmall || m > kMaxSmall) return fail(ctx, XPCS_EUNSUPPORTED, "tall x small product wider than 192");
    // T (column-major) -> row-major in the context's small-transpose buffer
    double *Tr = static_cast<double *>(ctx->tr_buf);
    hipLaunchKernelGGL(transpose_small_kernel, dim3((n * m + 255) / 256), dim3(256), 0, ctx->stream, T, n, m, Tr);
    const int64_t span = out.hi && out.rows_pad > rows ? out.rows_pad : rows;
    dim3 grid((unsigned)((span + 255) / 256));
    if (a_f64)
        hipLaunchKernelGGL(tsmul_kernel<double>, grid, dim3(256), 0, ctx->stream, static_cast<const double *>(A), rows,
                           lda, n, Tr, m, colscale, out.out32, out.ld32, out.out64, out.ld64, out.hi, out.lo, out.ldh,
                           out.Lpad, out.rows_pad);
    else
        hipLaunchKernelGGL(tsmul_kernel<float>, grid, dim3(256), 0, ctx->stream, static_cast<const float *>(A), rows,
                           lda, n, Tr, m, colscale, out.out32, out.ld32, out.out64, out.ld64, out.hi, out.lo, out.ldh,
                           out.Lpad, out.rows_pad);
    XPCS_LAUNCH_CHECK(ctx, "tsmul");
    return XPCS_OK;
}

xpcs_status launch_jacobi(xpcs_ctx *ctx, const double *B, int n, double *lam, double *P, void *rot) {
    Phase phase_(ctx, "jacobi");
    if (n > kMaxSmall || n % 2) return fail(ctx, XPCS_EUNSUPPORTED, "eigen size must be even and <= 192");
    int *nsteps = static_cast<int *>(rot);
    double2 *log = reinterpret_cast<double2 *>(static_cast<char *>(rot) + 256);
    if (n <= kJacobiPLds) {
        hipLaunchKernelGGL(jacobi_kernel<true>, dim3(1), dim3(1024), 0, ctx->stream, B, n, lam, P, log, nsteps,
                           ctx->flags);
        XPCS_LAUNCH_CHECK(ctx, "jacobi");
        return XPCS_OK;
    }
    hipLaunchKernelGGL(jacobi_kernel<false>, dim3(1), dim3(1024), 0, ctx->stream, B, n, lam, P, log, nsteps,
                       ctx->flags);
    XPCS_LAUNCH_CHECK(ctx, "jacobi");
    hipLaunchKernelGGL(jacobi_replay_kernel, dim3((n + kReplayRows - 1) / kReplayRows), dim3(256), 0, ctx->stream,
                       log, nsteps, n, P);
    XPCS_LAUNCH_CHECK(ctx, "jacobi_replay");
    return XPCS_OK;
}

xpcs_status launch_select_basis(xpcs_ctx *ctx, const double *lam, const double *P, int n, int k, const double *Wl,
                                int64_t N, int64_t ldw, double *T_u, double *scale_v, double *sigma) {
    Phase phase_(ctx, "select_basis");
    xpcs_status st;
    const size_t pb = align_up((size_t)k * sizeof(int), 256);
    char *sc = static_cast<char *>(scratch_get(ctx, pb + (size_t)N * k * sizeof(double), &st));
    if (!sc) return st;
    int *perm = reinterpret_cast<int *>(sc);
    double *Wk = reinterpret_cast<double *>(sc + pb);
    hipLaunchKernelGGL(select_kernel, dim3(1), dim3(256), 0, ctx->stream, lam, P, n, k, T_u, sigma, perm);
    XPCS_LAUNCH_CHECK(ctx, "select");
    TsOut o;
    o.out64 = Wk;
    o.ld64 = N;
    st = launch_tsmul(ctx, Wl, true, N, ldw, n, T_u, k, nullptr, o);
    if (st != XPCS_OK) return st;
    hipLaunchKernelGGL(sign_fix_kernel, dim3(k), dim3(256), 0, ctx->stream, Wk, N, N, n, T_u, sigma, scale_v);
    XPCS_LAUNCH_CHECK(ctx, "sign_fix");
    return XPCS_OK;
}

xpcs_status launch_column_norms(xpcs_ctx *ctx, const double *W, int64_t N, int64_t ldw, int k, double *sigma,
                                double *scale) {
    Phase phase_(ctx, "column_norms");
    hipLaunchKernelGGL(column_norm_kernel, dim3(k), dim3(256), 0, ctx->stream, W, N, ldw, sigma, scale);
    XPCS_LAUNCH_CHECK(ctx, "column_norms");
    return XPCS_OK;
}

xpcs_status launch_basis_to_bf16(xpcs_ctx *ctx, const float *U, int64_t M, int k, int64_t ldq, int Lpad,
                                 unsigned short *hi, unsigned short *lo) {
    Phase phase_(ctx, "basis_to_bf16");
    const int64_t total = (int64_t)Lpad * ldq;
    int grid = (int)((total + 255) / 256);
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(basis_to_bf16_kernel, dim3(grid), dim3(256), 0, ctx->stream, U, M, k, ldq, Lpad, hi, lo);
    XPCS_LAUNCH_CHECK(ctx, "basis_to_bf16");
    return XPCS_OK;
}

xpcs_status launch_identity(xpcs_ctx *ctx, double *T, int n) {
    Phase phase_(ctx, "identity");
    hipLaunchKernelGGL(identity_kernel, dim3((n * n + 255) / 256), dim3(256), 0, ctx->stream, T, n);
    XPCS_LAUNCH_CHECK(ctx, "identity");
    return XPCS_OK;
}

}  // namespace xpcs
