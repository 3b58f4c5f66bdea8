// The FP64 small-matrix steps of the compression for sketch widths beyond what one
// workgroup holds on chip (l > 192, up to the full rank of Eq. 11): the matrix
// lives in global memory (L2 / MALL resident at these sizes) and the work is
// split over many workgroups and launches.
//
//   * blocked Cholesky with the same pivot dropping as the on-chip kernels, and
//     the inverse of the factor by block forward substitution (Cholesky QR of the
//     sketches, Sec. 2.1; per-ROI factors of G_R, Eqs. 8-10 per ROI);
//   * two-sided block Jacobi for the l x l Gram eigendecomposition that ranks the
//     sketched directions (Eq. 3: Gram eigenvectors; Eq. 6: keep the K largest);
//   * the Gram of a tall matrix over pairs of 64-column panels on the FP64 MFMA.
#include <math.h>

#include "internal.hpp"

namespace xpcs {
namespace {

constexpr int kT = 64;            // tile edge
constexpr int kTP = kT + 1;       // LDS pitch of a tile (doubles): odd, so column walks spread over banks
constexpr int kBT = 256;          // threads of the tile kernels

__host__ __device__ __forceinline__ int64_t nblk_of(int n) { return (n + kT - 1) / kT; }

// Ts[i][j] = A[r0 + i][c0 + j] for i < nr, j < nc, zero elsewhere.
__device__ __forceinline__ void tile_load(double *Ts, const double *A, int64_t lda, int64_t r0, int64_t c0, int nr,
                                          int nc) {
    for (int e = threadIdx.x; e < kT * kT; e += kBT) {
        const int i = e / kT, j = e % kT;
        Ts[i * kTP + j] = (i < nr && j < nc) ? A[(r0 + i) * lda + c0 + j] : 0.0;
    }
}
__device__ __forceinline__ void tile_store(const double *Ts, double *A, int64_t lda, int64_t r0, int64_t c0, int nr,
                                           int nc) {
    for (int e = threadIdx.x; e < kT * kT; e += kBT) {
        const int i = e / kT, j = e % kT;
        if (i < nr && j < nc) A[(r0 + i) * lda + c0 + j] = Ts[i * kTP + j];
    }
}

// Thread t owns the 4 x 4 outputs rows 4 (t / 16) + i, columns 4 (t % 16) + j of a 64 x 64 product.
// acc += X Y^T (TRANS_Y) or X Y, X and Y 64 x 64 tiles in LDS.
template <bool TRANS_Y>
__device__ __forceinline__ void tile_mma(const double *X, const double *Y, double (&acc)[4][4]) {
    const int r0 = 4 * (threadIdx.x / 16), c0 = 4 * (threadIdx.x % 16);
    for (int q = 0; q < kT; ++q) {
        double x[4], y[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = X[(r0 + i) * kTP + q];
#pragma unroll
        for (int j = 0; j < 4; ++j) y[j] = TRANS_Y ? Y[(c0 + j) * kTP + q] : Y[q * kTP + c0 + j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = fma(x[i], y[j], acc[i][j]);
    }
}
__device__ __forceinline__ void acc_zero(double (&acc)[4][4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
}
// Ts[row][col] = s * acc (own outputs), after a barrier by the caller where Ts was read.
__device__ __forceinline__ void acc_put(double *Ts, const double (&acc)[4][4], double s) {
    const int r0 = 4 * (threadIdx.x / 16), c0 = 4 * (threadIdx.x % 16);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) Ts[(r0 + i) * kTP + c0 + j] = s * acc[i][j];
}

// ---------------------------------------------------------------- blocked Cholesky
// A (per matrix b: A + b n^2, row-major) holds the lower triangle being factored in
// place; tiles of 64.  Pivot rule of the on-chip kernels: a pivot at or below
// rel_tol * max(diag of the input) is dropped (its column of L is zero), and the
// inverses of the diagonal tiles are pseudo-inverses with the dropped rows zero.

// A[i][j] = (G[i][j] + G[j][i]) / 2 on and below the diagonal, 0 above.
__global__ __launch_bounds__(256) void bc_init_kernel(const double *__restrict__ G, int n, double *__restrict__ A) {
    const int64_t n2 = (int64_t)n * n;
    const double *g = G + blockIdx.y * n2;
    double *a = A + blockIdx.y * n2;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n2; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, j = e % n;
        a[e] = j <= i ? 0.5 * (g[e] + g[j * n + i]) : 0.0;
    }
}

// Diagonal tile j of matrix blockIdx.x: factor in LDS (two barriers a column), write
// L_jj (zero above its diagonal) and its pseudo-inverse Li_jj.  Tile 0 also fixes the
// pivot threshold from the untouched input diagonal.
__global__ __launch_bounds__(kBT) void bc_diag_kernel(double *__restrict__ Ab, int n, int j, double rel_tol,
                                                      double *__restrict__ thr, double *__restrict__ Lib) {
    __shared__ double T[kT * kTP];
    __shared__ double Li[kT * kTP];
    __shared__ double s_red[kBT / 64];
    __shared__ double s_thr;
    const int b = blockIdx.x, tid = threadIdx.x;
    double *A = Ab + (int64_t)b * n * n;
    const int64_t j0 = (int64_t)j * kT;
    const int jb = n - j0 < kT ? (int)(n - j0) : kT;
    if (j == 0) {
        double m = 0.0;
        for (int i = tid; i < n; i += kBT) m = fmax(m, A[(int64_t)i * n + i]);
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
        if ((tid & 63) == 0) s_red[tid >> 6] = m;
        __syncthreads();
        if (tid == 0) {
            double mm = 0.0;
            for (int w = 0; w < kBT / 64; ++w) mm = fmax(mm, s_red[w]);
            s_thr = rel_tol * mm;
            thr[b] = s_thr;
        }
    } else if (tid == 0) {
        s_thr = thr[b];
    }
    tile_load(T, A, n, j0, j0, jb, jb);
    __syncthreads();
    const double thresh = s_thr;
    for (int c = 0; c < jb; ++c) {
        const double d = T[c * kTP + c];
        const bool keep = d > thresh && d > 0.0;
        const double rs = keep ? 1.0 / sqrt(d) : 0.0;
        __syncthreads();                              // every thread has read the pivot
        for (int r = c + 1 + tid; r < jb; r += kBT) T[r * kTP + c] *= rs;
        if (tid == 0) T[c * kTP + c] = keep ? sqrt(d) : 0.0;
        __syncthreads();
        // trailing update of the lower part: T[r][s] -= L[r][c] L[s][c], c < s <= r
        const int m = jb - c - 1;
        for (int e = tid; e < m * m; e += kBT) {
            const int r = c + 1 + e / m, s = c + 1 + e % m;
            if (s <= r) T[r * kTP + s] -= T[r * kTP + c] * T[s * kTP + c];
        }
        __syncthreads();
    }
    // zero above the diagonal
    for (int e = tid; e < kT * kT; e += kBT) {
        const int r = e / kT, s = e % kT;
        if (s > r) T[r * kTP + s] = 0.0;
    }
    __syncthreads();
    // pseudo-inverse by columns: Li[r][c] = (delta_rc - sum_{c<=q<r} L[r][q] Li[q][c]) / L[r][r],
    // 0 where L[r][r] = 0 (a dropped pivot); four threads per column split each sum.
    {
        const int c = tid >> 2, part = tid & 3;
        for (int r = 0; r < kT; ++r) {
            double s = 0.0;
            if (r > c)
                for (int q = c + part; q < r; q += 4) s += T[r * kTP + q] * Li[q * kTP + c];
            s += __shfl_xor(s, 1);
            s += __shfl_xor(s, 2);
            if (part == 0) {
                const double lrr = T[r * kTP + r];
                double v = 0.0;
                if (r >= c && r < jb && lrr > 0.0) v = ((r == c ? 1.0 : 0.0) - s) / lrr;
                Li[r * kTP + c] = v;
            }
            __syncthreads();
        }
    }
    tile_store(T, A, n, j0, j0, jb, jb);
    double *li = Lib + ((int64_t)b * nblk_of(n) + j) * kT * kT;
    for (int e = tid; e < kT * kT; e += kBT) li[e] = Li[(e / kT) * kTP + e % kT];
}

// Panel below diagonal tile j: L_ij = A_ij Li_jj^T for the tile rows i > j.
__global__ __launch_bounds__(kBT) void bc_panel_kernel(double *__restrict__ Ab, int n, int j,
                                                       const double *__restrict__ Lib) {
    __shared__ double X[kT * kTP];
    __shared__ double Y[kT * kTP];
    const int b = blockIdx.y;
    double *A = Ab + (int64_t)b * n * n;
    const int i = j + 1 + blockIdx.x;
    const int64_t i0 = (int64_t)i * kT, j0 = (int64_t)j * kT;
    const int ib = n - i0 < kT ? (int)(n - i0) : kT, jb = n - j0 < kT ? (int)(n - j0) : kT;
    tile_load(X, A, n, i0, j0, ib, jb);
    const double *li = Lib + ((int64_t)b * nblk_of(n) + j) * kT * kT;
    for (int e = threadIdx.x; e < kT * kT; e += kBT) Y[(e / kT) * kTP + e % kT] = li[e];
    __syncthreads();
    double acc[4][4];
    acc_zero(acc);
    tile_mma<true>(X, Y, acc);
    __syncthreads();
    acc_put(X, acc, 1.0);
    __syncthreads();
    tile_store(X, A, n, i0, j0, ib, jb);
}

// Trailing update after panel j: A_il -= L_ij L_lj^T for j < l <= i (lower tiles).
__global__ __launch_bounds__(kBT) void bc_update_kernel(double *__restrict__ Ab, int n, int j) {
    __shared__ double X[kT * kTP];
    __shared__ double Y[kT * kTP];
    __shared__ double Z[kT * kTP];
    const int b = blockIdx.y;
    double *A = Ab + (int64_t)b * n * n;
    const int id = blockIdx.x;
    int ii = (int)((sqrt(8.0 * id + 1.0) - 1.0) * 0.5);
    while (ii * (ii + 1) / 2 > id) --ii;
    while ((ii + 1) * (ii + 2) / 2 <= id) ++ii;
    const int ll = id - ii * (ii + 1) / 2;
    const int i = j + 1 + ii, l = j + 1 + ll;
    const int64_t i0 = (int64_t)i * kT, l0 = (int64_t)l * kT, j0 = (int64_t)j * kT;
    const int ib = n - i0 < kT ? (int)(n - i0) : kT, lb = n - l0 < kT ? (int)(n - l0) : kT;
    const int jb = n - j0 < kT ? (int)(n - j0) : kT;
    tile_load(X, A, n, i0, j0, ib, jb);
    tile_load(Y, A, n, l0, j0, lb, jb);
    tile_load(Z, A, n, i0, l0, ib, lb);
    __syncthreads();
    double acc[4][4];
    acc_zero(acc);
    tile_mma<true>(X, Y, acc);
    const int r0 = 4 * (threadIdx.x / 16), c0 = 4 * (threadIdx.x % 16);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) Z[(r0 + a) * kTP + c0 + c] -= acc[a][c];
    __syncthreads();
    if (i == l) {   // keep the diagonal tile lower (its upper part is never read)
        for (int e = threadIdx.x; e < kT * kT; e += kBT)
            if (e % kT > e / kT) Z[(e / kT) * kTP + e % kT] = 0.0;
        __syncthreads();
    }
    tile_store(Z, A, n, i0, l0, ib, lb);
}

// Block row i of X = L^{-1} (row-major, the memory of Rinv = L^{-T} column-major):
// X_ii = Li_ii, X_ij = -Li_ii sum_{j<=l<i} L_il X_lj for j < i, X_ij = 0 for j > i.
__global__ __launch_bounds__(kBT) void bc_inv_row_kernel(const double *__restrict__ Lb, int n, int i,
                                                         const double *__restrict__ Lib, double *__restrict__ Xb) {
    __shared__ double P[kT * kTP];
    __shared__ double Q[kT * kTP];
    const int b = blockIdx.y, j = blockIdx.x;
    const double *L = Lb + (int64_t)b * n * n;
    double *Xm = Xb + (int64_t)b * n * n;
    const int64_t i0 = (int64_t)i * kT, j0 = (int64_t)j * kT;
    const int ib = n - i0 < kT ? (int)(n - i0) : kT, jb = n - j0 < kT ? (int)(n - j0) : kT;
    const double *li = Lib + ((int64_t)b * nblk_of(n) + i) * kT * kT;
    if (j > i) {
        for (int e = threadIdx.x; e < kT * kT; e += kBT) {
            const int r = e / kT, c = e % kT;
            if (r < ib && c < jb) Xm[(i0 + r) * n + j0 + c] = 0.0;
        }
        return;
    }
    if (j == i) {
        for (int e = threadIdx.x; e < kT * kT; e += kBT) {
            const int r = e / kT, c = e % kT;
            if (r < ib && c < jb) Xm[(i0 + r) * n + j0 + c] = li[e];
        }
        return;
    }
    double acc[4][4];
    acc_zero(acc);
    for (int l = j; l < i; ++l) {
        const int64_t l0 = (int64_t)l * kT;
        const int lb = n - l0 < kT ? (int)(n - l0) : kT;
        __syncthreads();
        tile_load(P, L, n, i0, l0, ib, lb);
        tile_load(Q, Xm, n, l0, j0, lb, jb);
        __syncthreads();
        tile_mma<false>(P, Q, acc);
    }
    __syncthreads();
    acc_put(Q, acc, -1.0);
    for (int e = threadIdx.x; e < kT * kT; e += kBT) P[(e / kT) * kTP + e % kT] = li[e];
    __syncthreads();
    acc_zero(acc);
    tile_mma<false>(P, Q, acc);
    __syncthreads();
    acc_put(P, acc, 1.0);
    __syncthreads();
    tile_store(P, Xm, n, i0, j0, ib, jb);
}

// Flag a factor without any kept pivot (the on-chip kernel's numeric-singularity rule).
__global__ __launch_bounds__(64) void bc_check_kernel(const double *__restrict__ L, int n, int *flags) {
    bool any = false;
    for (int i = threadIdx.x; i < n; i += 64) any |= L[(int64_t)i * n + i] > 0.0;
    if (!__ballot(any) && threadIdx.x == 0) atomicOr(&flags[kFlagNumeric], 1);
}


// ---------------------------------------------------------------- block Jacobi
// Two-sided cyclic block Jacobi on a symmetric n x n matrix, padded to np = a
// multiple of 64 (padded rows and columns are zero with -1 on the diagonal; they
// couple to nothing, so every rotation leaves them exactly in place and the
// leading n x n part of the result is the decomposition of the input).  Blocks of
// 32 indices; in round s of a sweep the nb / 2 block pairs of the circle method
// (every pair once per sweep) each take one cyclic Jacobi sweep of their 64 x 64
// sub-problem in LDS, giving an orthogonal Q_P per pair; then B <- J^T B J and
// V <- V J with J the block-diagonal (after the pair permutation) of the Q_P.
// Sweeps stop once the off-diagonal Frobenius norm is at most 1e-13 of the
// diagonal's (the on-chip kernels' rule), checked at the start of every sweep.
constexpr int kJB = 32;                 // block width
constexpr int kJS = 2 * kJB;            // sub-problem size
constexpr int kJSP = kJS + 1;
constexpr int kBjMaxSweeps = 24;

__device__ __forceinline__ void circle_pair(int s, int a, int n, int &p, int &q) {
    // pairs of the circle method on n (even) players, round s in [0, n - 1)
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
// global index of position x (0..63) of pair (I, J)
__device__ __forceinline__ int64_t pair_index(int I, int J, int x) {
    return x < kJB ? (int64_t)I * kJB + x : (int64_t)J * kJB + (x - kJB);
}

__device__ __forceinline__ double2 jac_rotation(double app, double apq, double aqq) {
    // t = tan of the smaller angle that zeroes apq under J^T A J with J = [[c, s], [-s, c]]
    double c = 1.0, sn = 0.0;
    if (fabs(apq) > 1e-300 && apq * apq > 1e-30 * fabs(app) * fabs(aqq)) {
        const double d = aqq - app, a2 = 2.0 * apq;
        const double hyp = sqrt(fma(d, d, a2 * a2));
        const double t = a2 / (d + (d >= 0.0 ? hyp : -hyp));
        c = 1.0 / sqrt(fma(t, t, 1.0));
        sn = t * c;
    }
    return make_double2(c, sn);
}

__global__ __launch_bounds__(256) void bj_init_kernel(const double *__restrict__ Bs, int n, int np,
                                                      double *__restrict__ B, double *__restrict__ V,
                                                      int *__restrict__ ctrl) {
    const int64_t total = (int64_t)np * np;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / np, j = e % np;
        double v;
        if (i < n && j < n)
            v = 0.5 * (Bs[i * n + j] + Bs[j * n + i]);
        else
            v = i == j ? -1.0 : 0.0;
        B[e] = v;
        V[e] = i == j ? 1.0 : 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ctrl[0] = 0;
}

// ctrl[0] = 1 once off(B) <= 1e-13 diag(B) in Frobenius norm over the leading n x n part.
__global__ __launch_bounds__(1024) void bj_norm_kernel(const double *__restrict__ B, int n, int np,
                                                       int *__restrict__ ctrl) {
    if (ctrl[0]) return;
    __shared__ double s_off[16], s_dg[16];
    double off = 0.0, dg = 0.0;
    const int64_t total = (int64_t)n * n;
    for (int64_t e = threadIdx.x; e < total; e += 1024) {
        const int64_t i = e / n, j = e % n;
        const double v = B[i * np + j];
        if (i == j)
            dg += v * v;
        else
            off += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) {
        off += __shfl_xor(off, o);
        dg += __shfl_xor(dg, o);
    }
    if ((threadIdx.x & 63) == 0) {
        s_off[threadIdx.x >> 6] = off;
        s_dg[threadIdx.x >> 6] = dg;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double so = 0.0, sd = 0.0;
        for (int w = 0; w < 16; ++w) {
            so += s_off[w];
            sd += s_dg[w];
        }
        if (so <= 1e-26 * sd || so == 0.0) ctrl[0] = 1;
    }
}

// One pair of round s: one cyclic Jacobi sweep (63 steps of 32 disjoint rotations) of
// the 64 x 64 sub-problem, Q = the product of the rotations; the rotated sub-problem
// goes back into B, Q into Qb[pair].
__global__ __launch_bounds__(256) void bj_pair_kernel(double *__restrict__ B, int np, int nb, int s,
                                                      double *__restrict__ Qb, const int *__restrict__ ctrl) {
    if (ctrl[0]) return;
    __shared__ double S[kJS * kJSP];
    __shared__ double Q[kJS * kJSP];
    __shared__ double2 rot[kJS / 2];
    const int a = blockIdx.x, tid = threadIdx.x;
    int I, J;
    circle_pair(s, a, nb, I, J);
    for (int e = tid; e < kJS * kJS; e += 256) {
        const int x = e / kJS, y = e % kJS;
        S[x * kJSP + y] = B[pair_index(I, J, x) * np + pair_index(I, J, y)];
        Q[x * kJSP + y] = x == y ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int st = 0; st < kJS - 1; ++st) {
        if (tid < kJS / 2) {
            int p, q;
            circle_pair(st, tid, kJS, p, q);
            rot[tid] = jac_rotation(S[p * kJSP + p], S[p * kJSP + q], S[q * kJSP + q]);
        }
        __syncthreads();
        // rows: row p <- c row p - s row q, row q <- s row p + c row q
        for (int e = tid; e < (kJS / 2) * kJS; e += 256) {
            const int t = e / kJS, y = e % kJS;
            int p, q;
            circle_pair(st, t, kJS, p, q);
            const double2 r = rot[t];
            const double sp = S[p * kJSP + y], sq = S[q * kJSP + y];
            S[p * kJSP + y] = r.x * sp - r.y * sq;
            S[q * kJSP + y] = r.y * sp + r.x * sq;
        }
        __syncthreads();
        // columns of S and of Q
        for (int e = tid; e < (kJS / 2) * kJS; e += 256) {
            const int t = e / kJS, x = e % kJS;
            int p, q;
            circle_pair(st, t, kJS, p, q);
            const double2 r = rot[t];
            const double sp = S[x * kJSP + p], sq = S[x * kJSP + q];
            S[x * kJSP + p] = r.x * sp - r.y * sq;
            S[x * kJSP + q] = r.y * sp + r.x * sq;
            const double qp = Q[x * kJSP + p], qq = Q[x * kJSP + q];
            Q[x * kJSP + p] = r.x * qp - r.y * qq;
            Q[x * kJSP + q] = r.y * qp + r.x * qq;
        }
        __syncthreads();
    }
    double *qo = Qb + (int64_t)a * kJS * kJS;
    for (int e = tid; e < kJS * kJS; e += 256) {
        const int x = e / kJS, y = e % kJS;
        B[pair_index(I, J, x) * np + pair_index(I, J, y)] = S[x * kJSP + y];
        qo[e] = Q[x * kJSP + y];
    }
}

// After round s: blocks [0, nup) take the off-diagonal pair tiles (P < P'):
// B[P][P'] <- Q_P^T B[P][P'] Q_P', mirrored into B[P'][P]; the rest take the
// 64-row slabs of V times each Q_P'.
__global__ __launch_bounds__(256) void bj_update_kernel(double *__restrict__ B, double *__restrict__ V, int np,
                                                        int nb, int s, const double *__restrict__ Qb,
                                                        const int *__restrict__ ctrl) {
    if (ctrl[0]) return;
    __shared__ double X[kT * kTP];
    __shared__ double Y[kT * kTP];
    __shared__ double Z[kT * kTP];
    const int h = nb / 2, nup = h * (h - 1) / 2;
    const int id = blockIdx.x, tid = threadIdx.x;
    auto load_q = [&](double *dst, int pair) {
        const double *q = Qb + (int64_t)pair * kJS * kJS;
        for (int e = tid; e < kJS * kJS; e += 256) dst[(e / kJS) * kTP + e % kJS] = q[e];
    };
    double acc[4][4];
    if (id < nup) {
        // pair tile (P, P2), P < P2: linear id over the strict upper triangle of h x h
        int P = 0, rem = id;
        while (rem >= h - 1 - P) {
            rem -= h - 1 - P;
            ++P;
        }
        const int P2 = P + 1 + rem;
        int I, J, I2, J2;
        circle_pair(s, P, nb, I, J);
        circle_pair(s, P2, nb, I2, J2);
        for (int e = tid; e < kJS * kJS; e += 256) {
            const int x = e / kJS, y = e % kJS;
            Z[x * kTP + y] = B[pair_index(I, J, x) * np + pair_index(I2, J2, y)];
        }
        load_q(X, P);
        __syncthreads();
        // Y = Q_P^T Z: Y[r][c] = sum_q X[q][r] Z[q][c]
        acc_zero(acc);
        {
            const int r0 = 4 * (tid / 16), c0 = 4 * (tid % 16);
            for (int q = 0; q < kT; ++q) {
                double x[4], z[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) x[i] = X[q * kTP + r0 + i];
#pragma unroll
                for (int j = 0; j < 4; ++j) z[j] = Z[q * kTP + c0 + j];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = fma(x[i], z[j], acc[i][j]);
            }
        }
        acc_put(Y, acc, 1.0);
        __syncthreads();
        load_q(X, P2);
        __syncthreads();
        acc_zero(acc);
        tile_mma<false>(Y, X, acc);          // (Q_P^T Z) Q_P2
        __syncthreads();
        acc_put(Z, acc, 1.0);
        __syncthreads();
        for (int e = tid; e < kJS * kJS; e += 256) {
            const int x = e / kJS, y = e % kJS;
            const double v = Z[x * kTP + y];
            B[pair_index(I, J, x) * np + pair_index(I2, J2, y)] = v;
            B[pair_index(I2, J2, y) * np + pair_index(I, J, x)] = v;
        }
        return;
    }
    // V slab: rows [64 rb, 64 rb + 64), the columns of pair P2
    const int vid = id - nup;
    const int rb = vid / h, P2 = vid % h;
    int I2, J2;
    circle_pair(s, P2, nb, I2, J2);
    const int64_t r0g = (int64_t)rb * kT;
    for (int e = tid; e < kT * kJS; e += 256) {
        const int x = e / kJS, y = e % kJS;
        Z[x * kTP + y] = V[(r0g + x) * np + pair_index(I2, J2, y)];
    }
    load_q(X, P2);
    __syncthreads();
    acc_zero(acc);
    tile_mma<false>(Z, X, acc);
    __syncthreads();
    acc_put(Z, acc, 1.0);
    __syncthreads();
    for (int e = tid; e < kT * kJS; e += 256) {
        const int x = e / kJS, y = e % kJS;
        V[(r0g + x) * np + pair_index(I2, J2, y)] = Z[x * kTP + y];
    }
}

__global__ __launch_bounds__(256) void bj_finish_kernel(const double *__restrict__ B, const double *__restrict__ V,
                                                        int n, int np, double *__restrict__ lam,
                                                        double *__restrict__ P, const int *__restrict__ ctrl,
                                                        int *flags) {
    const int64_t total = (int64_t)n * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, j = e % n;
        P[e] = V[i * np + j];
        if (j == 0) lam[i] = B[i * np + i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && !ctrl[0]) atomicOr(&flags[kFlagNumeric], 1);
}

// ---------------------------------------------------------------- Gram over column panels
// G = A^T A for a tall column-major A (fp32 or fp64) with more columns than one
// workgroup's accumulators hold: blockIdx.y picks a pair of 64-column panels
// (I <= J), blockIdx.z a segment (a ROI's rows of a gathered row list, -1 rows
// skipped) or 0, blockIdx.x a share of the rows.  Eight waves walk 16-row groups
// (a wave's 4 x 4 FP64-MFMA tiles of the panel pair, four rows per lane loaded
// one group ahead), add their tiles in LDS in wave order and write the block's
// 64 x 64 partial for the fixed-order reduction.
typedef double f64x4v __attribute__((ext_vector_type(4)));
constexpr int kPgThreads = 256;           // one wave per SIMD: the operands of both panels and the
                                          // 16 accumulator tiles need more than 256 registers in FP64
constexpr int kPgWaves = kPgThreads / 64;

template <typename TA>
__global__ __launch_bounds__(kPgThreads) void panel_gram_kernel(const TA *__restrict__ A, int64_t rows, int64_t lda,
                                                                int ncols, const int32_t *__restrict__ row_idx,
                                                                const int64_t *__restrict__ seg_off,
                                                                double *__restrict__ part, bool vec) {
    __shared__ double red[kT * kT];
    const int np = (ncols + kT - 1) / kT;
    int pid = blockIdx.y, I = 0;
    while (pid >= np - I) {
        pid -= np - I;
        ++I;
    }
    const int J = I + pid;
    const int seg = blockIdx.z;
    const int64_t r_begin = seg_off ? seg_off[seg] : 0;
    const int64_t r_end = seg_off ? seg_off[seg + 1] : rows;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int cl = lane & 15, kq = lane >> 4;
    const int64_t ngroups = (r_end - r_begin + 15) / 16;
    const int64_t per_blk = (ngroups + gridDim.x - 1) / gridDim.x;
    const int64_t g0 = (int64_t)blockIdx.x * per_blk;
    const int64_t g1 = g0 + per_blk < ngroups ? g0 + per_blk : ngroups;
    f64x4v acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (f64x4v){0.0, 0.0, 0.0, 0.0};
    // x[p][cb][j]: panel p (0 = I, 1 = J), column 64 P + 16 cb + cl, row r0 + 4 kq + j
    auto load = [&](int64_t g, TA (&x)[2][4][4]) {
        const int64_t r = r_begin + g * 16 + 4 * kq;
        int64_t rowj[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t pos = r + j;
            rowj[j] = pos < r_end ? (row_idx ? (int64_t)row_idx[pos] : pos) : -1;
        }
        const bool v4 = vec && r + 4 <= r_end;
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const int c = (p == 0 ? I : J) * kT + 16 * cb + cl;
                const TA *src = A + (int64_t)(c < ncols ? c : 0) * lda;
                if (v4 && c < ncols) {
                    if constexpr (sizeof(TA) == 1) {
                        const unsigned v = *reinterpret_cast<const unsigned *>(src + r);
#pragma unroll
                        for (int j = 0; j < 4; ++j) x[p][cb][j] = (TA)((v >> (8 * j)) & 0xffu);
                    } else if constexpr (sizeof(TA) == 2) {
                        const uint2 v = *reinterpret_cast<const uint2 *>(src + r);
                        x[p][cb][0] = (TA)(v.x & 0xffffu); x[p][cb][1] = (TA)(v.x >> 16);
                        x[p][cb][2] = (TA)(v.y & 0xffffu); x[p][cb][3] = (TA)(v.y >> 16);
                    } else if constexpr (sizeof(TA) == 4) {
                        const float4 v = *reinterpret_cast<const float4 *>(src + r);
                        x[p][cb][0] = v.x; x[p][cb][1] = v.y; x[p][cb][2] = v.z; x[p][cb][3] = v.w;
                    } else {
                        const double2 a = reinterpret_cast<const double2 *>(src + r)[0];
                        const double2 b = reinterpret_cast<const double2 *>(src + r)[1];
                        x[p][cb][0] = a.x; x[p][cb][1] = a.y; x[p][cb][2] = b.x; x[p][cb][3] = b.y;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) x[p][cb][j] = (c < ncols && rowj[j] >= 0) ? src[rowj[j]] : (TA)0;
                }
            }
    };
    TA cur[2][4][4], nxt[2][4][4];
    int64_t g = g0 + wv;
    if (g < g1) load(g, nxt);
    for (; g < g1; g += kPgWaves) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int j = 0; j < 4; ++j) cur[p][cb][j] = nxt[p][cb][j];
        if (g + kPgWaves < g1) load(g + kPgWaves, nxt);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)cur[0][a][j], (double)cur[1][b][j],
                                                                     acc[a][b], 0, 0, 0);
    }
    // accumulator layout: acc[a][b][v] = tile row 16 a + kq + 4 v (panel I column),
    // tile column 16 b + cl (panel J column)
    for (int w = 0; w < kPgWaves; ++w) {
        if (wv == w) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int idx = (16 * a + kq + 4 * v) * kT + 16 * b + cl;
                        red[idx] = (w == 0 ? 0.0 : red[idx]) + acc[a][b][v];
                    }
        }
        __syncthreads();
    }
    double *out = part + (((int64_t)seg * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * kT * kT;
    for (int e = threadIdx.x; e < kT * kT; e += kPgThreads) out[e] = red[e];
}

// G[seg][a][b] = sum over the row shares of the partial of the panel pair holding (a, b)
// (transposed when a's panel follows b's); fixed order, one thread per entry.
__global__ __launch_bounds__(256) void panel_gram_reduce_kernel(const double *__restrict__ part, int nparts,
                                                                int npairs, int ncols, double *__restrict__ G) {
    const int seg = blockIdx.y;
    const int64_t n2 = (int64_t)ncols * ncols;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n2) return;
    const int a = (int)(idx / ncols), b = (int)(idx % ncols);
    int pa = a / kT, pb = b / kT, ra = a % kT, rb = b % kT;
    if (pa > pb) {
        int t = pa; pa = pb; pb = t;
        t = ra; ra = rb; rb = t;
    }
    const int np = (ncols + kT - 1) / kT;
    const int pair = pa * np - pa * (pa - 1) / 2 + (pb - pa);
    const double *p = part + ((int64_t)seg * npairs + pair) * nparts * kT * kT + ra * kT + rb;
    double s = 0.0;
    for (int k = 0; k < nparts; ++k) s += p[(int64_t)k * kT * kT];
    G[(int64_t)seg * n2 + idx] = s;
}
}  // namespace

size_t chol_blocked_work_bytes(int n, int nb) {
    return align_up((size_t)nb * nblk_of(n) * kT * kT * sizeof(double), 256) + align_up((size_t)nb * sizeof(double), 256);
}

// Factor nb matrices G (n x n) into L (row-major lower, zero upper) in place in L.
xpcs_status launch_chol_blocked(xpcs_ctx *ctx, const double *G, int n, int nb, double rel_tol, double *L,
                                void *work) {
    const int nbk = (int)nblk_of(n);
    double *Lib = static_cast<double *>(work);
    double *thr = reinterpret_cast<double *>(static_cast<char *>(work) +
                                             align_up((size_t)nb * nbk * kT * kT * sizeof(double), 256));
    const int64_t n2 = (int64_t)n * n;
    int g = (int)((n2 + 255) / 256);
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(bc_init_kernel, dim3(g, nb), dim3(256), 0, ctx->stream, G, n, L);
    XPCS_LAUNCH_CHECK(ctx, "chol_blocked_init");
    for (int j = 0; j < nbk; ++j) {
        hipLaunchKernelGGL(bc_diag_kernel, dim3(nb), dim3(kBT), 0, ctx->stream, L, n, j, rel_tol, thr, Lib);
        XPCS_LAUNCH_CHECK(ctx, "chol_blocked_diag");
        const int rem = nbk - j - 1;
        if (rem == 0) break;
        hipLaunchKernelGGL(bc_panel_kernel, dim3(rem, nb), dim3(kBT), 0, ctx->stream, L, n, j, Lib);
        XPCS_LAUNCH_CHECK(ctx, "chol_blocked_panel");
        hipLaunchKernelGGL(bc_update_kernel, dim3(rem * (rem + 1) / 2, nb), dim3(kBT), 0, ctx->stream, L, n, j);
        XPCS_LAUNCH_CHECK(ctx, "chol_blocked_update");
    }
    return XPCS_OK;
}

size_t cholinv_blocked_work_bytes(int n) {
    return align_up((size_t)n * n * sizeof(double), 256) + chol_blocked_work_bytes(n, 1);
}

// Rinv = L^{-T} (column-major n x n, upper triangular) of one matrix.
xpcs_status launch_cholinv_blocked(xpcs_ctx *ctx, const double *G, int n, double rel_tol, double *Rinv, void *work) {
    double *Lw = static_cast<double *>(work);
    void *cw = static_cast<char *>(work) + align_up((size_t)n * n * sizeof(double), 256);
    xpcs_status st = launch_chol_blocked(ctx, G, n, 1, rel_tol, Lw, cw);
    if (st) return st;
    hipLaunchKernelGGL(bc_check_kernel, dim3(1), dim3(64), 0, ctx->stream, Lw, n, ctx->flags);
    XPCS_LAUNCH_CHECK(ctx, "chol_blocked_check");
    const int nbk = (int)nblk_of(n);
    const double *Lib = static_cast<const double *>(cw);
    for (int i = 0; i < nbk; ++i) {
        hipLaunchKernelGGL(bc_inv_row_kernel, dim3(nbk, 1), dim3(kBT), 0, ctx->stream, Lw, n, i, Lib, Rinv);
        XPCS_LAUNCH_CHECK(ctx, "chol_blocked_inverse");
    }
    return XPCS_OK;
}

size_t jacobi_block_work_bytes(int n) {
    const int64_t np = (n + kJS - 1) / kJS * kJS;
    const int64_t nb = np / kJB;
    return 2 * align_up((size_t)np * np * sizeof(double), 256) +
           align_up((size_t)(nb / 2) * kJS * kJS * sizeof(double), 256) + 256;
}

// Eigenvalues lam[n] (unsorted) and eigenvectors P (row-major n x n, column j =
// vector j) of a symmetric n x n matrix by block Jacobi (n even or odd).
xpcs_status launch_jacobi_block(xpcs_ctx *ctx, const double *Bs, int n, double *lam, double *P, void *work) {
    const int np = (n + kJS - 1) / kJS * kJS;
    const int nb = np / kJB, h = nb / 2;
    char *w = static_cast<char *>(work);
    double *B = reinterpret_cast<double *>(w);
    double *V = reinterpret_cast<double *>(w + align_up((size_t)np * np * sizeof(double), 256));
    double *Qb = reinterpret_cast<double *>(w + 2 * align_up((size_t)np * np * sizeof(double), 256));
    int *ctrl = reinterpret_cast<int *>(w + 2 * align_up((size_t)np * np * sizeof(double), 256) +
                                        align_up((size_t)h * kJS * kJS * sizeof(double), 256));
    int g = (int)(((int64_t)np * np + 255) / 256);
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(bj_init_kernel, dim3(g), dim3(256), 0, ctx->stream, Bs, n, np, B, V, ctrl);
    XPCS_LAUNCH_CHECK(ctx, "jacobi_block_init");
    const int nupd = h * (h - 1) / 2 + (np / kT) * h;
    for (int sweep = 0; sweep < kBjMaxSweeps; ++sweep) {
        hipLaunchKernelGGL(bj_norm_kernel, dim3(1), dim3(1024), 0, ctx->stream, B, n, np, ctrl);
        XPCS_LAUNCH_CHECK(ctx, "jacobi_block_norm");
        for (int s = 0; s < nb - 1; ++s) {
            hipLaunchKernelGGL(bj_pair_kernel, dim3(h), dim3(256), 0, ctx->stream, B, np, nb, s, Qb, ctrl);
            XPCS_LAUNCH_CHECK(ctx, "jacobi_block_pairs");
            hipLaunchKernelGGL(bj_update_kernel, dim3(nupd), dim3(256), 0, ctx->stream, B, V, np, nb, s, Qb, ctrl);
            XPCS_LAUNCH_CHECK(ctx, "jacobi_block_update");
        }
    }
    hipLaunchKernelGGL(bj_norm_kernel, dim3(1), dim3(1024), 0, ctx->stream, B, n, np, ctrl);
    XPCS_LAUNCH_CHECK(ctx, "jacobi_block_norm");
    g = (int)(((int64_t)n * n + 255) / 256);
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(bj_finish_kernel, dim3(g), dim3(256), 0, ctx->stream, B, V, n, np, lam, P, ctrl, ctx->flags);
    XPCS_LAUNCH_CHECK(ctx, "jacobi_block_finish");
    return XPCS_OK;
}

// Gram of a tall matrix (or of each segment of a gathered row list) over 64-column
// panel pairs, for any number of columns.
// a_type: XPCS_F32, XPCS_F64, XPCS_U8 / XPCS_U16 counts (the frame Gram F F^T of integer
// counts is exact in FP64 while every sum stays below 2^53).
static xpcs_status panel_gram_any(xpcs_ctx *ctx, const void *A, int a_type, int64_t rows, int64_t lda, int ncols,
                                  const int32_t *row_idx, const int64_t *seg_off, int nseg, double *G);

xpcs_status launch_panel_gram(xpcs_ctx *ctx, const void *A, bool a_f64, int64_t rows, int64_t lda, int ncols,
                              const int32_t *row_idx, const int64_t *seg_off, int nseg, double *G) {
    return panel_gram_any(ctx, A, a_f64 ? XPCS_F64 : XPCS_F32, rows, lda, ncols, row_idx, seg_off, nseg, G);
}

xpcs_status launch_frame_gram(xpcs_ctx *ctx, const void *frames, int dtype, int64_t M, int64_t N, double *G) {
    Phase phase_(ctx, "frame_gram");
    return panel_gram_any(ctx, frames, dtype, M, M, (int)N, nullptr, nullptr, 1, G);
}

static xpcs_status panel_gram_any(xpcs_ctx *ctx, const void *A, int a_type, int64_t rows, int64_t lda, int ncols,
                                  const int32_t *row_idx, const int64_t *seg_off, int nseg, double *G) {
    const int np = (ncols + kT - 1) / kT, npairs = np * (np + 1) / 2;
    const int64_t seg_rows = seg_off ? rows / (nseg > 0 ? nseg : 1) : rows;
    int nparts = (int)(seg_rows / 256);
    const int target = (512 + npairs * nseg - 1) / (npairs * nseg);   // about two blocks per CU in all
    if (nparts > target) nparts = target;
    if (nparts < 1) nparts = 1;
    xpcs_status st;
    double *part = static_cast<double *>(
        scratch_get(ctx, (size_t)nseg * npairs * nparts * kT * kT * sizeof(double), &st));
    if (!part) return st;
    const size_t esz = a_type == XPCS_F64 ? 8 : (a_type == XPCS_F32 ? 4 : (a_type == XPCS_U8 ? 1 : 2));
    const bool vec = !row_idx && !seg_off && lda % 4 == 0 && (uintptr_t)A % (4 * esz) == 0;
    dim3 grid(nparts, npairs, nseg);
    switch (a_type) {
        case XPCS_F64:
            hipLaunchKernelGGL(panel_gram_kernel<double>, grid, dim3(kPgThreads), 0, ctx->stream,
                               static_cast<const double *>(A), rows, lda, ncols, row_idx, seg_off, part, vec);
            break;
        case XPCS_F32:
            hipLaunchKernelGGL(panel_gram_kernel<float>, grid, dim3(kPgThreads), 0, ctx->stream,
                               static_cast<const float *>(A), rows, lda, ncols, row_idx, seg_off, part, vec);
            break;
        case XPCS_U8:
            hipLaunchKernelGGL(panel_gram_kernel<uint8_t>, grid, dim3(kPgThreads), 0, ctx->stream,
                               static_cast<const uint8_t *>(A), rows, lda, ncols, row_idx, seg_off, part, vec);
            break;
        default:
            hipLaunchKernelGGL(panel_gram_kernel<uint16_t>, grid, dim3(kPgThreads), 0, ctx->stream,
                               static_cast<const uint16_t *>(A), rows, lda, ncols, row_idx, seg_off, part, vec);
            break;
    }
    XPCS_LAUNCH_CHECK(ctx, "panel_gram");
    const int64_t n2 = (int64_t)ncols * ncols;
    hipLaunchKernelGGL(panel_gram_reduce_kernel, dim3((unsigned)((n2 + 255) / 256), nseg), dim3(256), 0, ctx->stream,
                       part, nparts, npairs, ncols, G);
    XPCS_LAUNCH_CHECK(ctx, "panel_gram_reduce");
    return XPCS_OK;
}

}  // namespace xpcs
