// Relaxation fit of g2 (Sec. 3.1, Eq. 13): g2(tau) = B + beta exp(-2 Gamma tau),
// B the baseline, beta the contrast and Gamma = 1 / t0 the inverse relaxation time
// (lags in frames), by unweighted least squares over the valid lags of a range;
// and the stretched (Kohlrausch-Williams-Watts) form the paper names for it,
// g2(tau) = B + beta exp(-2 (Gamma tau)^gamma), with the exponent gamma fitted too
// (gamma = 1 is the form above).
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

// NP = 3: (B, beta, Gamma); NP = 4: (B, beta, Gamma, gamma).  Sums per pass: the
// cost, J^T r (NP) and the upper triangle of J^T J.
template <int NP>
struct FitDims {
    static constexpr int kTri = NP * (NP + 1) / 2;
    static constexpr int kSums = 1 + NP + kTri;
};

template <int NP>
struct FitShared {
    double part[kFitThreads / kWave][FitDims<NP>::kSums];
    double p[NP];                   // trial point evaluated by the next pass
    int done;
};

// Model value and Jacobian at lag tau.  With x = Gamma tau and s = x^gamma:
// e = exp(-2 s), d/dGamma = -2 beta e gamma s / Gamma, d/dgamma = -2 beta e s ln x
// (both 0 at tau = 0, and s = x for gamma = 1).
template <int NP>
__device__ __forceinline__ double fit_model(double tau, const double *p, double *J) {
    if constexpr (NP == 3) {
        const double e = exp(-2.0 * p[2] * tau);
        J[0] = 1.0;
        J[1] = e;
        J[2] = -2.0 * tau * p[1] * e;
        return p[0] + p[1] * e;
    } else {
        const double x = p[2] * tau;
        double sx = 0.0, lx = 0.0;
        if (tau > 0.0) {
            lx = log(x);                            // NaN for Gamma < 0: the trial is rejected
            sx = exp(p[3] * lx);
        }
        const double e = exp(-2.0 * sx);
        J[0] = 1.0;
        J[1] = e;
        J[2] = tau > 0.0 ? -2.0 * p[1] * e * p[3] * sx / p[2] : 0.0;
        J[3] = tau > 0.0 ? -2.0 * p[1] * e * sx * lx : 0.0;
        return p[0] + p[1] * e;
    }
}

// Sums over the valid lags of (r^2, J^T r, J^T J) at p, into s[] of thread 0.
template <int NP>
__device__ void fit_pass(const double *g, const int64_t *np, int64_t lo, int64_t hi, const double *p,
                         double *s, FitShared<NP> &sh) {
    constexpr int kS = FitDims<NP>::kSums;
    double a[kS];
#pragma unroll
    for (int i = 0; i < kS; ++i) a[i] = 0.0;
    for (int64_t tau = lo + threadIdx.x; tau < hi; tau += kFitThreads) {
        const double y = g[tau];
        if ((np && np[tau] <= 0) || !isfinite(y)) continue;
        double J[NP];
        const double r = fit_model<NP>((double)tau, p, J) - y;
        a[0] = fma(r, r, a[0]);
#pragma unroll
        for (int i = 0; i < NP; ++i) a[1 + i] = fma(J[i], r, a[1 + i]);
        int q = 1 + NP;
#pragma unroll
        for (int i = 0; i < NP; ++i)
#pragma unroll
            for (int j = i; j < NP; ++j) {
                a[q] = fma(J[i], J[j], a[q]);
                ++q;
            }
    }
#pragma unroll
    for (int i = 0; i < kS; ++i) {
        double v = a[i];
        for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
        a[i] = v;
    }
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0)
        for (int i = 0; i < kS; ++i) sh.part[w][i] = a[i];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 0; i < kS; ++i) {
            double v = 0.0;
            for (int q = 0; q < kFitThreads / kWave; ++q) v += sh.part[q][i];
            s[i] = v;
        }
}

// Solves (A + lam diag(A)) d = -b for the symmetric NP x NP A given by its upper
// triangle (row by row) by Cholesky; false if not positive definite.
template <int NP>
__device__ bool solve_damped(const double *A, const double *b, double lam, double *d) {
    double m[NP][NP];
    int q = 0;
    for (int i = 0; i < NP; ++i)
        for (int j = i; j < NP; ++j) m[i][j] = m[j][i] = A[q++];
    for (int i = 0; i < NP; ++i) m[i][i] += lam * (m[i][i] > 0.0 ? m[i][i] : 1.0);
    double L[NP][NP] = {};
    for (int j = 0; j < NP; ++j) {
        double v = m[j][j];
        for (int k = 0; k < j; ++k) v -= L[j][k] * L[j][k];
        if (!(v > 0.0)) return false;
        L[j][j] = sqrt(v);
        for (int i = j + 1; i < NP; ++i) {
            double u = m[i][j];
            for (int k = 0; k < j; ++k) u -= L[i][k] * L[j][k];
            L[i][j] = u / L[j][j];
        }
    }
    double y[NP];
    for (int i = 0; i < NP; ++i) {
        double v = -b[i];
        for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
        y[i] = v / L[i][i];
    }
    for (int i = NP - 1; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < NP; ++k) v -= L[k][i] * d[k];
        d[i] = v / L[i][i];
    }
    return true;
}

template <int NP>
__global__ __launch_bounds__(kFitThreads) void fit_relaxation_kernel(
    const double *__restrict__ g2, const int64_t *__restrict__ npairs, int64_t n, int64_t lo, int64_t hi,
    const double *__restrict__ p0, int max_iter, double *__restrict__ params, int *__restrict__ status) {
    constexpr int kS = FitDims<NP>::kSums;
    __shared__ FitShared<NP> sh;
    const int roi = blockIdx.x;
    const double *g = g2 + (int64_t)roi * n;
    const int64_t *np = npairs ? npairs + (int64_t)roi * n : nullptr;
    // thread 0 state
    double p[NP] = {}, cur[kS], trial[kS];
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
                for (int i = 0; i < NP; ++i) p[i] = p0[(int64_t)roi * NP + i];
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
                    if (NP == 4) p[NP - 1] = 1.0;
                }
            }
            for (int i = 0; i < NP; ++i) sh.p[i] = p[i];
            sh.done = nvalid < NP;
        }
        __syncthreads();
    }
    if (sh.done) {
        if (threadIdx.x == 0) {
            for (int i = 0; i < NP; ++i) params[(int64_t)roi * NP + i] = __builtin_nan("");
            status[roi] = -1;
        }
        return;
    }
    // cost, gradient and J^T J at the start
    fit_pass<NP>(g, np, lo, hi, sh.p, cur, sh);
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
            double d[NP] = {};
            bool ok = false;
            for (int tries = 0; tries < 60 && !ok; ++tries) {
                ok = solve_damped<NP>(cur + 1 + NP, cur + 1, lam, d);
                if (!ok) lam *= 10.0;
            }
            sh.done = !ok;
            for (int i = 0; i < NP; ++i) sh.p[i] = p[i] + d[i];
        }
        __syncthreads();
        const int stop1 = sh.done;
        __syncthreads();
        if (stop1) break;
        fit_pass<NP>(g, np, lo, hi, sh.p, trial, sh);
        if (threadIdx.x == 0) {
            ++iters;
            bool stop = false;
            if (isfinite(trial[0]) && trial[0] < cur[0]) {
                double step = 0.0, size = 0.0;
                for (int i = 0; i < NP; ++i) {
                    step = fmax(step, fabs(sh.p[i] - p[i]));
                    size = fmax(size, fabs(p[i]));
                }
                const double gain = cur[0] - trial[0];
                for (int i = 0; i < NP; ++i) p[i] = sh.p[i];
                for (int i = 0; i < kS; ++i) cur[i] = trial[i];
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
        for (int i = 0; i < NP; ++i) params[(int64_t)roi * NP + i] = p[i];
        status[roi] = iters;
    }
}

}  // namespace
}  // namespace xpcs

using namespace xpcs;

extern "C" {

namespace {
xpcs_status fit_launch(xpcs_ctx *ctx, int np_, const double *g2, const int64_t *npairs, int64_t n, int32_t n_roi,
                       int64_t tau_lo, int64_t tau_hi, const double *p0, int32_t max_iter, double *params,
                       int32_t *status) {
    if (!ctx) return XPCS_EINVAL;
    if (!g2 || !params || !status) return fail(ctx, XPCS_EINVAL, "g2, params and status must not be NULL");
    if (n <= 0 || n_roi < 1) return fail(ctx, XPCS_EINVAL, "need n > 0 and n_roi >= 1");
    if (tau_lo < 0 || tau_hi <= tau_lo || tau_hi > n) return fail(ctx, XPCS_EINVAL, "need 0 <= tau_lo < tau_hi <= n");
    if (max_iter < 0 || max_iter > 10000) return fail(ctx, XPCS_EINVAL, "max_iter outside [0, 10000]");
    (void)hipSetDevice(ctx->device);
    Phase phase_(ctx, "fit_relaxation");
    if (np_ == 3)
        hipLaunchKernelGGL(fit_relaxation_kernel<3>, dim3((unsigned)n_roi), dim3(kFitThreads), 0, ctx->stream, g2,
                           npairs, n, tau_lo, tau_hi, p0, max_iter, params, status);
    else
        hipLaunchKernelGGL(fit_relaxation_kernel<4>, dim3((unsigned)n_roi), dim3(kFitThreads), 0, ctx->stream, g2,
                           npairs, n, tau_lo, tau_hi, p0, max_iter, params, status);
    XPCS_LAUNCH_CHECK(ctx, "fit_relaxation");
    return XPCS_OK;
}
}  // namespace

xpcs_status fit_relaxation(xpcs_ctx *ctx, const double *g2, const int64_t *npairs, int64_t n, int32_t n_roi,
                           int64_t tau_lo, int64_t tau_hi, const double *p0, int32_t max_iter, double *params,
                           int32_t *status) {
    return fit_launch(ctx, 3, g2, npairs, n, n_roi, tau_lo, tau_hi, p0, max_iter, params, status);
}

xpcs_status fit_relaxation_stretched(xpcs_ctx *ctx, const double *g2, const int64_t *npairs, int64_t n,
                                     int32_t n_roi, int64_t tau_lo, int64_t tau_hi, const double *p0,
                                     int32_t max_iter, double *params, int32_t *status) {
    return fit_launch(ctx, 4, g2, npairs, n, n_roi, tau_lo, tau_hi, p0, max_iter, params, status);
}

}  // extern "C"
