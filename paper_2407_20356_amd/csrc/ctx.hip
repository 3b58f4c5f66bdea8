// Context, workspace arena, stream binding and device-side error flags.
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "internal.hpp"

namespace xpcs {

// Scratch of the entry points that allocate nothing.  In host code `scratch` names a
// host-side stand-in, not device memory: its device address is looked up once per
// device (with that device current) and only that address is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`; the caller has made `device` current.
hipError_t static_scratch_address(int device, void **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

xpcs_status fail(xpcs_ctx *ctx, xpcs_status st, const std::string &msg) {
    if (ctx) ctx->last_error = msg;
    return st;
}

xpcs_status check_hip(xpcs_ctx *ctx, hipError_t err, const char *what) {
    if (err == hipSuccess) return XPCS_OK;
    std::string m = std::string(what) + ": " + hipGetErrorString(err);
    return fail(ctx, err == hipErrorOutOfMemory ? XPCS_ENOMEM : XPCS_EDEVICE, m);
}

void ws_begin(xpcs_ctx *ctx) { ctx->ws.used = 0; }

xpcs_status ws_reserve(xpcs_ctx *ctx, size_t total) {
    total = align_up(total, 256) + 256;
    if (ctx->ws.used + total <= ctx->ws.capacity) return XPCS_OK;
    size_t want = ctx->ws.used + total;
    if (ctx->budget && want + ctx->scratch.capacity + ctx->persistent > ctx->budget)
        return fail(ctx, XPCS_EBUDGET,
                    "workspace of " + std::to_string(want) + " bytes exceeds the HBM budget of " +
                        std::to_string(ctx->budget));
    if (ctx->ws.used != 0)
        return fail(ctx, XPCS_EDEVICE, "internal: workspace grown after pieces were taken");
    // The old arena may still be read by work in flight on the stream.
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    if (ctx->ws.base) {
        e = hipFree(ctx->ws.base);
        ctx->ws.base = nullptr;
        ctx->ws.capacity = 0;
        if (e != hipSuccess) return check_hip(ctx, e, "hipFree(workspace)");
    }
    size_t grow = want + want / 4;
    if (ctx->budget && grow + ctx->scratch.capacity + ctx->persistent > ctx->budget) grow = want;
    void *p = nullptr;
    e = hipMalloc(&p, grow);
    if (e != hipSuccess) return check_hip(ctx, e, "hipMalloc(workspace)");
    ctx->ws.base = static_cast<char *>(p);
    ctx->ws.capacity = grow;
    return XPCS_OK;
}

void *scratch_get(xpcs_ctx *ctx, size_t bytes, xpcs_status *st) {
    *st = XPCS_OK;
    bytes = align_up(bytes, 256);
    if (bytes <= ctx->scratch.capacity) return ctx->scratch.base;
    const size_t total = ctx->ws.capacity + ctx->persistent + bytes;
    if (ctx->budget && total > ctx->budget) {
        *st = fail(ctx, XPCS_EBUDGET, "scratch of " + std::to_string(bytes) + " bytes exceeds the HBM budget");
        return nullptr;
    }
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess && ctx->scratch.base) e = hipFree(ctx->scratch.base);
    ctx->scratch.base = nullptr;
    ctx->scratch.capacity = 0;
    void *p = nullptr;
    if (e == hipSuccess) e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        *st = check_hip(ctx, e, "scratch allocation");
        return nullptr;
    }
    ctx->scratch.base = static_cast<char *>(p);
    ctx->scratch.capacity = bytes;
    return p;
}

namespace {
__global__ void zero_kernel(unsigned int *p, size_t nwords) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nwords; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}
}  // namespace

xpcs_status launch_zero(xpcs_ctx *ctx, void *p, size_t bytes) {
    Phase phase_(ctx, "zero");
    if (bytes % 4) return fail(ctx, XPCS_EINVAL, "internal: zero fill of a size not a multiple of 4");
    size_t nw = bytes / 4;
    int grid = (int)((nw + 255) / 256);
    if (grid > 4096) grid = 4096;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(zero_kernel, dim3(grid), dim3(256), 0, ctx->stream, static_cast<unsigned int *>(p), nw);
    XPCS_LAUNCH_CHECK(ctx, "zero");
    return XPCS_OK;
}

void *ws_take(xpcs_ctx *ctx, size_t bytes) {
    size_t off = align_up(ctx->ws.used, 256);
    ctx->ws.used = off + align_up(bytes, 256);
    return ctx->ws.base + off;
}

static hipEvent_t pool_event(xpcs_ctx *ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

Phase::Phase(xpcs_ctx *ctx, const char *name) : ctx_(ctx) {
    if (!ctx_->timing) return;
    if (!ctx_->phase_only.empty()) {
        bool want = false;
        for (const auto &n : ctx_->phase_only) want = want || n == name;
        if (!want) return;
    }
    PhaseRecord r{name, pool_event(ctx_), pool_event(ctx_)};
    if (!r.start || !r.stop || hipEventRecord(r.start, ctx_->stream) != hipSuccess) return;
    ctx_->phases.push_back(r);
    idx_ = (int)ctx_->phases.size() - 1;
}

Phase::~Phase() {
    if (idx_ >= 0) (void)hipEventRecord(ctx_->phases[idx_].stop, ctx_->stream);
}

}  // namespace xpcs

using namespace xpcs;

extern "C" {

xpcs_status xpcs_create(int device, size_t hbm_budget_bytes, xpcs_ctx **out) {
    if (!out) return XPCS_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev || device >= kMaxDevices)
        return XPCS_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return XPCS_EDEVICE;
    void *sptr = nullptr;
    if (static_scratch_address(device, &sptr) != hipSuccess) return XPCS_EDEVICE;
    xpcs_ctx *ctx = new xpcs_ctx();
    ctx->device = device;
    ctx->budget = hbm_budget_bytes;
    ctx->static_scratch = sptr;
    void *p = nullptr;
    if (hipMalloc(&p, kNumFlags * sizeof(int)) != hipSuccess) {
        delete ctx;
        return XPCS_ENOMEM;
    }
    ctx->flags = static_cast<int *>(p);
    if (hipMemset(ctx->flags, 0, kNumFlags * sizeof(int)) != hipSuccess) {
        (void)hipFree(p);
        delete ctx;
        return XPCS_EDEVICE;
    }
    *out = ctx;
    return XPCS_OK;
}

void xpcs_destroy(xpcs_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &r : ctx->phases) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    if (ctx->ws.base) (void)hipFree(ctx->ws.base);
    if (ctx->scratch.base) (void)hipFree(ctx->scratch.base);
    if (ctx->flags) (void)hipFree(ctx->flags);
    delete ctx;
}

xpcs_status xpcs_set_stream(xpcs_ctx *ctx, void *hip_stream) {
    if (!ctx) return XPCS_EINVAL;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return XPCS_OK;
}

xpcs_status xpcs_sync(xpcs_ctx *ctx) {
    if (!ctx) return XPCS_EINVAL;
    (void)hipSetDevice(ctx->device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    int h[kNumFlags] = {0};
    e = hipMemcpy(h, ctx->flags, sizeof(h), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return check_hip(ctx, e, "read device flags");
    e = hipMemset(ctx->flags, 0, sizeof(h));
    if (e != hipSuccess) return check_hip(ctx, e, "clear device flags");
    if (h[kFlagLabel]) return fail(ctx, XPCS_EINVAL, "a ROI label is outside [-1, n_roi)");
    if (h[kFlagNumeric])
        return fail(ctx, XPCS_EDEVICE, "a numerically singular step (sketch of rank 0 or no eigen convergence)");
    return XPCS_OK;
}

xpcs_status xpcs_phase_filter(xpcs_ctx *ctx, const char *names) {
    if (!ctx) return XPCS_EINVAL;
    ctx->phase_only.clear();
    if (!names) return XPCS_OK;
    std::string cur;
    for (const char *c = names;; ++c) {
        if (*c == ',' || *c == 0) {
            if (!cur.empty()) ctx->phase_only.push_back(cur);
            cur.clear();
            if (*c == 0) break;
        } else {
            cur.push_back(*c);
        }
    }
    return XPCS_OK;
}

xpcs_status xpcs_enable_phase_timing(xpcs_ctx *ctx, int32_t enable) {
    if (!ctx) return XPCS_EINVAL;
    (void)hipSetDevice(ctx->device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    for (auto &r : ctx->phases) {
        ctx->event_pool.push_back(r.start);
        ctx->event_pool.push_back(r.stop);
    }
    ctx->phases.clear();
    ctx->timing = enable != 0;
    return XPCS_OK;
}

xpcs_status xpcs_phase_times(xpcs_ctx *ctx, int32_t cap, char *names, double *ms, int64_t *launches,
                             int32_t *n_out) {
    if (!ctx || cap < 0 || (cap > 0 && (!names || !ms || !launches)) || !n_out) return XPCS_EINVAL;
    (void)hipSetDevice(ctx->device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return check_hip(ctx, e, "hipStreamSynchronize");
    int n = 0;
    std::vector<std::string> seen;
    for (auto &r : ctx->phases) {
        float t = 0.f;
        e = hipEventElapsedTime(&t, r.start, r.stop);
        if (e != hipSuccess) return check_hip(ctx, e, "hipEventElapsedTime");
        int idx = -1;
        for (int i = 0; i < (int)seen.size(); ++i)
            if (seen[i] == r.name) idx = i;
        if (idx < 0) {
            if (n >= cap) continue;
            idx = n++;
            seen.push_back(r.name);
            strncpy(names + 32 * idx, r.name, 31);
            names[32 * idx + 31] = 0;
            ms[idx] = 0.0;
            launches[idx] = 0;
        }
        ms[idx] += t;
        launches[idx] += 1;
    }
    *n_out = n;
    return XPCS_OK;
}

const char *xpcs_last_error(const xpcs_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

size_t xpcs_workspace_bytes(const xpcs_ctx *ctx) { return ctx ? ctx->ws.capacity + ctx->scratch.capacity : 0; }

}  // extern "C"
