// Relaxation fit of g2 (Sec. 3.1, Eq. 13): g2(tau) = B + beta exp(-2 Gamma tau),
// B the baseline, beta the contrast and Gamma = 1 / t0 the inverse relaxation time
// (lags in frames), by unweighted least squares over the valid lags of a range.
//
// Levenberg-Marquardt in FP64 (Marquardt's scaling by the diagonal of J^T J),
// one workgroup per ROI: every iteration evaluates the cost, J^T J and J^T r at
// the trial point in one parallel pass over the lags (block reduction in a fixed
// order), and thread 0 accepts or rejects the step and solves the damped 3 x 3
// system.  Every thread runs the same iterations, at most max_iter.
#include <math.h>

#include "internal.hpp"

namespace xpcs {
namespace {

constexpr int kFitThreads = 256;
constexpr int kFitSums = 10;        // cost, J^T r (3), J^T J upper triangle (6)

struct FitShared {
    double part[kFitThreads / kWave][kFitSums];
    double p[3];                    // trial point evaluated by the next pass
    int done;
};

// Sums over the valid lags of (r^2, J^T r, J^T J) at p, into s[] of thread 0.
__device__ void fit_pass(const double *g, const int64_t *np, int64_t lo, int64_t hi, const double *p,
                         double *s, FitShared &sh) {
    double a[kFitSums];
#pragma unroll
    for (int i = 0; i < kFitSums; ++i) a[i] = 0.0;
    for (int64_t tau = lo + threadIdx.x; tau < hi; tau += kFitThreads) {
        const double y = g[tau];
        if ((np && np[tau] <= 0) || !isfinite(y)) continue;
        const double e = exp(-2.0 * p[2] * (double)tau);
        const double j0 = 1.0, j1 = e, j2 = -2.0 * (double)tau * p[1] * e;
        const double r = p[0] + p[1] * e - y;
        a[0] = fma(r, r, a[0]);
        a[1] = fma(j0, r, a[1]);
        a[2] = fma(j1, r, a[2]);
        a[3] = fma(j2, r, a[3]);
        a[4] = fma(j0, j0, a[4]);
        a[5] = fma(j0, j1, a[5]);
        a[6] = fma(j0, j2, a[6]);
        a[7] = fma(j1, j1, a[7]);
        a[8] = fma(j1, j2, a[8]);
        a[9] = fma(j2, j2, a[9]);
    }
#pragma unroll
    for (int i = 0; i < kFitSums; ++i) {
        double v = a[i];
        for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
        a[i] = v;
    }
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0)
        for (int i = 0; i < kFitSums; ++i) sh.part[w][i] = a[i];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 0; i < kFitSums; ++i) {
            double v = 0.0;
            for (int q = 0; q < kFitThreads / kWave; ++q) v += sh.part[q][i];
            s[i] = v;
        }
}

// Solves (A + lam diag(A)) d = -b for the symmetric 3 x 3 A given by its upper
// triangle (a00 a01 a02 a11 a12 a22) by Cholesky; false if not positive definite.
__device__ bool solve3(const double *A, const double *b, double lam, double *d) {
    double m[3][3] = {{A[0], A[1], A[2]}, {A[1], A[3], A[4]}, {A[2], A[4], A[5]}};
    for (int i = 0; i < 3; ++i) m[i][i] += lam * (m[i][i] > 0.0 ? m[i][i] : 1.0);
    double L[3][3] = {};
    for (int j = 0; j < 3; ++j) {
        double v = m[j][j];
        for (int q = 0; q < j; ++q) v -= L[j][q] * L[j][q];
        if (!(v > 0.0)) return false;
        L[j][j] = sqrt(v);
        for (int i = j + 1; i < 3; ++i) {
            double u = m[i][j];
            for (int q = 0; q < j; ++q) u -= L[i][q] * L[j][q];
            L[i][j] = u / L[j][j];
        }
    }
    double y[3];
    for (int i = 0; i < 3; ++i) {
        double v = -b[i];
        for (int q = 0; q < i; ++q) v -= L[i][q] * y[q];
        y[i] = v / L[i][i];
    }
    for (int i = 2; i >= 0; --i) {
        double v = y[i];
        for (int q = i + 1; q < 3; ++q) v -= L[q][i] * d[q];
        d[i] = v / L[i][i];
    }
    return true;
}

__global__ __launch_bounds__(kFitThreads) void fit_relaxation_kernel(
    const double *__restrict__ g2, const int64_t *__restrict__ npairs, int64_t n, int64_t lo, int64_t hi,
    const double *__restrict__ p0, int max_iter, double *__restrict__ params, int *__restrict__ status) {
    __shared__ FitShared sh;
    const int roi = blockIdx.x;
    const double *g = g2 + (int64_t)roi * n;
    const int64_t *np = npairs ? npairs + (int64_t)roi * n : nullptr;
    // thread 0 state
    double p[3] = {0, 0, 0}, cur[kFitSums], trial[kFitSums];
    double lam = 0.0;
    int iters = 0, nvalid = 0;
    // count the valid lags and find the first / last for the default start
    {
        int c = 0;
        for (int64_t tau = lo + threadIdx.x; tau < hi; tau += kFitThreads)
            if ((!np || np[tau] > 0) && isfinite(g[tau])) ++c;
        for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_down(c, off, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0) sh.part[threadIdx.x / kWave][0] = (double)c;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int q = 0; q < kFitThreads / kWave; ++q) t += sh.part[q][0];
            nvalid = (int)t;
            if (p0) {
                for (int i = 0; i < 3; ++i) p[i] = p0[(int64_t)roi * 3 + i];
            } else {
                int64_t first = -1, last = -1;
                double tsum = 0.0;
                for (int64_t tau = lo; tau < hi; ++tau)
                    if ((!np || np[tau] > 0) && isfinite(g[tau])) {
                        if (first < 0) first = tau;
                        last = tau;
                        tsum += (double)tau;
                    }
                if (nvalid > 0) {
                    p[0] = g[last];
                    p[1] = fmax(g[first] - g[last], 1e-3);
                    p[2] = 1.0 / fmax(tsum / nvalid, 1.0);
                }
            }
            for (int i = 0; i < 3; ++i) sh.p[i] = p[i];
            sh.done = nvalid < 3;
        }
        __syncthreads();
    }
    if (sh.done) {
        if (threadIdx.x == 0) {
            for (int i = 0; i < 3; ++i) params[(int64_t)roi * 3 + i] = __builtin_nan("");
            status[roi] = -1;
        }
        return;
    }
    // cost, gradient and J^T J at the start
    fit_pass(g, np, lo, hi, sh.p, cur, sh);
    if (threadIdx.x == 0) {
        lam = 1e-3;
        sh.done = !(cur[0] > 0.0) || max_iter <= 0;
    }
    __syncthreads();
    // sh.done is written by thread 0 only between two barriers and read by every
    // thread into a register between two barriers, so every thread leaves the
    // loop at the same iteration
    for (int it = 0; it < max_iter; ++it) {
        const int stop0 = sh.done;
        __syncthreads();
        if (stop0) break;
        if (threadIdx.x == 0) {
            // a step from the current point; raise the damping until the system is solvable
            double d[3] = {0, 0, 0};
            bool ok = false;
            for (int tries = 0; tries < 60 && !ok; ++tries) {
                ok = solve3(cur + 4, cur + 1, lam, d);
                if (!ok) lam *= 10.0;
            }
            sh.done = !ok;
            for (int i = 0; i < 3; ++i) sh.p[i] = p[i] + d[i];
        }
        __syncthreads();
        const int stop1 = sh.done;
        __syncthreads();
        if (stop1) break;
        fit_pass(g, np, lo, hi, sh.p, trial, sh);
        if (threadIdx.x == 0) {
            ++iters;
            bool stop = false;
            if (isfinite(trial[0]) && trial[0] < cur[0]) {
                double step = 0.0, size = 0.0;
                for (int i = 0; i < 3; ++i) {
                    step = fmax(step, fabs(sh.p[i] - p[i]));
                    size = fmax(size, fabs(p[i]));
                }
                const double gain = cur[0] - trial[0];
                for (int i = 0; i < 3; ++i) p[i] = sh.p[i];
                for (int i = 0; i < kFitSums; ++i) cur[i] = trial[i];
                lam = fmax(lam * 0.1, 1e-12);
                stop = gain <= 1e-15 * cur[0] || step <= 1e-13 * (size + 1e-13);
            } else {
                lam *= 10.0;
                stop = lam > 1e16;
            }
            sh.done = stop;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int i = 0; i < 3; ++i) params[(int64_t)roi * 3 + i] = p[i];
        status[roi] = iters;
    }
}

}  // namespace
}  // namespace xpcs

using namespace xpcs;

extern "C" {

xpcs_status fit_relaxation(xpcs_ctx *ctx, const double *g2, const int64_t *npairs, int64_t n, int32_t n_roi,
                           int64_t tau_lo, int64_t tau_hi, const double *p0, int32_t max_iter, double *params,
                           int32_t *status) {
    if (!ctx) return XPCS_EINVAL;
    if (!g2 || !params || !status) return fail(ctx, XPCS_EINVAL, "g2, params and status must not be NULL");
    if (n <= 0 || n_roi < 1) return fail(ctx, XPCS_EINVAL, "need n > 0 and n_roi >= 1");
    if (tau_lo < 0 || tau_hi <= tau_lo || tau_hi > n) return fail(ctx, XPCS_EINVAL, "need 0 <= tau_lo < tau_hi <= n");
    if (max_iter < 0 || max_iter > 10000) return fail(ctx, XPCS_EINVAL, "max_iter outside [0, 10000]");
    (void)hipSetDevice(ctx->device);
    Phase phase_(ctx, "fit_relaxation");
    hipLaunchKernelGGL(fit_relaxation_kernel, dim3((unsigned)n_roi), dim3(kFitThreads), 0, ctx->stream, g2, npairs,
                       n, tau_lo, tau_hi, p0, max_iter, params, status);
    XPCS_LAUNCH_CHECK(ctx, "fit_relaxation");
    return XPCS_OK;
}

}  // extern "C"
