// Serving: many online streams (Sec. 2.2 online strategy, one per detector) on
// one GPU at once.  Each admitted stream is placed on one of a few lanes -- a
// context with its own HIP stream and workspace -- so that the blocks of
// streams on different lanes run concurrently on the device.  Admission follows
// the order of the requests and waits for a free slot and for HBM under the
// budget (stream state plus lane workspaces); a close admits the waiting
// requests that now fit, in order.  Every block is timed from the push call to
// the end of its work with device events: the start event is recorded on an
// idle stream, where it completes at once.
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "internal.hpp"

struct xpcs_server {
    struct Block {
        hipEvent_t start = nullptr, end = nullptr, dep = nullptr;
        int64_t frames = 0;
    };
    struct Entry {
        xpcs_stream_desc desc{};
        int32_t state = 0;
        int lane = -1;
        xpcs_stream *s = nullptr;
        size_t state_bytes = 0, ws_bytes = 0;
        std::deque<Block> blocks;
    };
    int device = 0;
    size_t budget = 0;
    int max_streams = 0;
    std::vector<xpcs_ctx *> lane_ctx;
    std::vector<hipStream_t> lane_stream;
    std::vector<int> lane_count;
    hipStream_t clock = nullptr;
    size_t state_used = 0;
    int admitted = 0;
    std::map<int64_t, Entry> entries;
    std::deque<int64_t> waiting;
    int64_t next_id = 1;
    std::vector<hipEvent_t> pool;
    std::string last_error;
};

namespace {

using xpcs::align_up;

xpcs_status srv_fail(xpcs_server *srv, xpcs_status st, const std::string &msg) {
    srv->last_error = msg;
    return st;
}
// Adopts the message a lane context recorded for a failed call.
xpcs_status lane_fail(xpcs_server *srv, int lane, xpcs_status st) {
    srv->last_error = srv->lane_ctx[lane]->last_error;
    return st;
}

size_t lanes_bytes(const xpcs_server *srv) {
    size_t b = 0;
    for (const xpcs_ctx *c : srv->lane_ctx) b += c->ws.capacity + c->scratch.capacity;
    return b;
}

// Capacity a lane's workspace reaches when `need` bytes are reserved on it
// (the arena grows by a quarter beyond what is asked).
size_t grown_capacity(size_t cap, size_t need) {
    const size_t want = align_up(need, 256) + 256;
    return want <= cap ? cap : want + want / 4;
}

hipEvent_t take_event(xpcs_server *srv) {
    if (!srv->pool.empty()) {
        hipEvent_t e = srv->pool.back();
        srv->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
void give_event(xpcs_server *srv, hipEvent_t e) {
    if (e) srv->pool.push_back(e);
}
void release_block(xpcs_server *srv, xpcs_server::Block &b) {
    give_event(srv, b.start);
    give_event(srv, b.end);
    give_event(srv, b.dep);
    b.start = b.end = b.dep = nullptr;
}

xpcs_status check_desc(xpcs_server *srv, const xpcs_stream_desc *d) {
    if (!d->roi_label || !d->basis) return srv_fail(srv, XPCS_EINVAL, "roi_label or basis is NULL");
    if (d->M <= 0) return srv_fail(srv, XPCS_EINVAL, "M must be positive");
    if (d->dtype != XPCS_U8 && d->dtype != XPCS_U16) return srv_fail(srv, XPCS_EINVAL, "dtype must be XPCS_U8 or XPCS_U16");
    if (d->n_roi < 1) return srv_fail(srv, XPCS_EINVAL, "n_roi must be >= 1");
    if (d->n_roi > 64) return srv_fail(srv, XPCS_EUNSUPPORTED, "a stream records at most 64 ROIs");
    if (d->k < 1 || d->k > d->M) return srv_fail(srv, XPCS_EINVAL, "k must be in 1..M");
    if (d->k > xpcs::kMaxRank) return srv_fail(srv, XPCS_EUNSUPPORTED, "basis wider than 1024");
    if (d->window < 1 || d->window > 65536) return srv_fail(srv, XPCS_EINVAL, "window must be in 1..65536");
    if (d->max_block < 1 || d->max_block > 4096) return srv_fail(srv, XPCS_EINVAL, "max_block must be in 1..4096");
    return XPCS_OK;
}

// Admits entry e now if a slot and the memory are free: returns 1 when admitted,
// 0 when it must wait, or an error status.
int try_admit(xpcs_server *srv, xpcs_server::Entry &e) {
    if (srv->admitted >= srv->max_streams) return 0;
    int lane = 0;
    for (int l = 1; l < (int)srv->lane_ctx.size(); ++l)
        if (srv->lane_count[l] < srv->lane_count[lane]) lane = l;
    xpcs_ctx *ctx = srv->lane_ctx[lane];
    const size_t cap_now = ctx->ws.capacity + ctx->scratch.capacity;
    const size_t cap_after = grown_capacity(ctx->ws.capacity, e.ws_bytes) + ctx->scratch.capacity;
    const size_t after = srv->state_used + e.state_bytes + lanes_bytes(srv) - cap_now + cap_after;
    if (srv->budget && after > srv->budget) return 0;
    (void)hipSetDevice(srv->device);
    xpcs::ws_begin(ctx);
    xpcs_status st = xpcs::ws_reserve(ctx, e.ws_bytes);
    if (st) return lane_fail(srv, lane, st);
    if ((st = xpcs_stream_open(ctx, &e.desc, &e.s))) return lane_fail(srv, lane, st);
    // the open reads the caller's labels and basis on the lane: finish it here
    hipError_t he = hipStreamSynchronize(srv->lane_stream[lane]);
    if (he != hipSuccess) {
        xpcs_stream_close(e.s);
        e.s = nullptr;
        return srv_fail(srv, XPCS_EDEVICE, std::string("stream open: ") + hipGetErrorString(he));
    }
    e.lane = lane;
    e.state = XPCS_STREAM_ADMITTED;
    srv->lane_count[lane] += 1;
    srv->admitted += 1;
    srv->state_used += e.state_bytes;
    return 1;
}

// Admits waiting requests in order while they fit; one that fails is dropped
// with state XPCS_STREAM_FAILED.
void admit_waiting(xpcs_server *srv) {
    while (!srv->waiting.empty()) {
        auto it = srv->entries.find(srv->waiting.front());
        if (it == srv->entries.end()) {
            srv->waiting.pop_front();
            continue;
        }
        const int r = try_admit(srv, it->second);
        if (r == 0) return;
        if (r < 0) it->second.state = XPCS_STREAM_FAILED;
        srv->waiting.pop_front();
    }
}

xpcs_server::Entry *find(xpcs_server *srv, int64_t id) {
    auto it = srv->entries.find(id);
    return it == srv->entries.end() ? nullptr : &it->second;
}

}  // namespace

extern "C" {

xpcs_status xpcs_server_create(int device, size_t hbm_budget_bytes, int32_t lanes, int32_t max_streams,
                               xpcs_server **out) {
    if (!out) return XPCS_EINVAL;
    *out = nullptr;
    if (lanes < 1 || lanes > 16 || max_streams < 1) return XPCS_EINVAL;
    auto *srv = new xpcs_server;
    srv->device = device;
    srv->budget = hbm_budget_bytes;
    srv->max_streams = max_streams;
    auto bail = [&](xpcs_status st) {
        xpcs_server_destroy(srv);
        return st;
    };
    for (int l = 0; l < lanes; ++l) {
        xpcs_ctx *ctx = nullptr;
        xpcs_status st = xpcs_create(device, 0, &ctx);
        if (st) return bail(st);
        srv->lane_ctx.push_back(ctx);
        srv->lane_count.push_back(0);
        hipStream_t hs = nullptr;
        if (hipStreamCreateWithFlags(&hs, hipStreamNonBlocking) != hipSuccess) return bail(XPCS_EDEVICE);
        srv->lane_stream.push_back(hs);
        xpcs_set_stream(ctx, hs);
    }
    if (hipStreamCreateWithFlags(&srv->clock, hipStreamNonBlocking) != hipSuccess) return bail(XPCS_EDEVICE);
    *out = srv;
    return XPCS_OK;
}

void xpcs_server_destroy(xpcs_server *srv) {
    if (!srv) return;
    (void)hipSetDevice(srv->device);
    for (auto &kv : srv->entries) {
        auto &e = kv.second;
        if (e.s) xpcs_stream_close(e.s);
        for (auto &b : e.blocks) release_block(srv, b);
    }
    for (hipStream_t hs : srv->lane_stream) (void)hipStreamSynchronize(hs);
    for (xpcs_ctx *c : srv->lane_ctx) xpcs_destroy(c);
    for (hipStream_t hs : srv->lane_stream) (void)hipStreamDestroy(hs);
    if (srv->clock) (void)hipStreamDestroy(srv->clock);
    for (hipEvent_t e : srv->pool) (void)hipEventDestroy(e);
    delete srv;
}

const char *xpcs_server_last_error(const xpcs_server *srv) { return srv ? srv->last_error.c_str() : "NULL server"; }

xpcs_status xpcs_server_open(xpcs_server *srv, const xpcs_stream_desc *desc, int64_t *id, int32_t *state) {
    if (!srv) return XPCS_EINVAL;
    if (!desc || !id) return srv_fail(srv, XPCS_EINVAL, "desc or id is NULL");
    xpcs_status st = check_desc(srv, desc);
    if (st) return st;
    xpcs_server::Entry e;
    e.desc = *desc;
    e.state_bytes = xpcs::stream_state_bytes(desc);
    e.ws_bytes = xpcs::stream_workspace_bytes(desc);
    if (srv->budget && e.state_bytes + grown_capacity(0, e.ws_bytes) > srv->budget)
        return srv_fail(srv, XPCS_EBUDGET, "the stream alone needs " + std::to_string(e.state_bytes) +
                                               " bytes of state and " + std::to_string(e.ws_bytes) +
                                               " of workspace, beyond the HBM budget");
    const int64_t my = srv->next_id++;
    auto &ent = srv->entries[my] = e;
    ent.state = XPCS_STREAM_QUEUED;
    if (srv->waiting.empty()) {
        const int r = try_admit(srv, ent);
        if (r < 0) {
            srv->entries.erase(my);
            return (xpcs_status)r;
        }
        if (r == 0) srv->waiting.push_back(my);
    } else {
        srv->waiting.push_back(my);
    }
    *id = my;
    if (state) *state = ent.state;
    return XPCS_OK;
}

xpcs_status xpcs_server_state(xpcs_server *srv, int64_t id, int32_t *state) {
    if (!srv || !state) return XPCS_EINVAL;
    auto *e = find(srv, id);
    if (!e) return srv_fail(srv, XPCS_EINVAL, "no such stream id");
    *state = e->state;
    return XPCS_OK;
}

xpcs_status xpcs_server_push(xpcs_server *srv, int64_t id, const void *frames, int64_t nframes, void *band,
                             int32_t c_dtype, void *producer) {
    if (!srv) return XPCS_EINVAL;
    auto *e = find(srv, id);
    if (!e) return srv_fail(srv, XPCS_EINVAL, "no such stream id");
    if (e->state == XPCS_STREAM_QUEUED) return srv_fail(srv, XPCS_EQUEUED, "the stream waits for admission");
    if (e->state != XPCS_STREAM_ADMITTED) return srv_fail(srv, XPCS_EINVAL, "the stream failed to open");
    (void)hipSetDevice(srv->device);
    hipStream_t lane = srv->lane_stream[e->lane];
    xpcs_server::Block b;
    b.frames = nframes;
    b.start = take_event(srv);
    b.end = take_event(srv);
    if (producer) b.dep = take_event(srv);
    if (!b.start || !b.end || (producer && !b.dep)) {
        release_block(srv, b);
        return srv_fail(srv, XPCS_EDEVICE, "hipEventCreate failed");
    }
    hipError_t he = hipEventRecord(b.start, srv->clock);
    if (he == hipSuccess && producer) {
        he = hipEventRecord(b.dep, static_cast<hipStream_t>(producer));
        if (he == hipSuccess) he = hipStreamWaitEvent(lane, b.dep, 0);
    }
    if (he != hipSuccess) {
        release_block(srv, b);
        return srv_fail(srv, XPCS_EDEVICE, std::string("push ordering: ") + hipGetErrorString(he));
    }
    xpcs_status st = xpcs_stream_push(e->s, frames, nframes, band, c_dtype);
    if (st) {
        release_block(srv, b);
        return lane_fail(srv, e->lane, st);
    }
    if ((he = hipEventRecord(b.end, lane)) != hipSuccess) {
        release_block(srv, b);
        return srv_fail(srv, XPCS_EDEVICE, std::string("hipEventRecord: ") + hipGetErrorString(he));
    }
    e->blocks.push_back(b);
    return XPCS_OK;
}

xpcs_status xpcs_server_poll(xpcs_server *srv, int64_t id, int32_t cap, double *latency_ms, int64_t *frames,
                             int32_t *count) {
    if (!srv || !count) return XPCS_EINVAL;
    *count = 0;
    auto *e = find(srv, id);
    if (!e) return srv_fail(srv, XPCS_EINVAL, "no such stream id");
    (void)hipSetDevice(srv->device);
    int32_t n = 0;
    while (n < cap && !e->blocks.empty()) {
        auto &b = e->blocks.front();
        const hipError_t q = hipEventQuery(b.end);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) return srv_fail(srv, XPCS_EDEVICE, std::string("block event: ") + hipGetErrorString(q));
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, b.start, b.end) != hipSuccess) ms = -1.f;
        if (latency_ms) latency_ms[n] = ms;
        if (frames) frames[n] = b.frames;
        ++n;
        release_block(srv, b);
        e->blocks.pop_front();
    }
    *count = n;
    return XPCS_OK;
}

xpcs_status xpcs_server_g2(xpcs_server *srv, int64_t id, double *g2, int64_t *npairs) {
    if (!srv) return XPCS_EINVAL;
    auto *e = find(srv, id);
    if (!e) return srv_fail(srv, XPCS_EINVAL, "no such stream id");
    if (e->state != XPCS_STREAM_ADMITTED) return srv_fail(srv, XPCS_EQUEUED, "the stream is not admitted");
    xpcs_status st = xpcs_stream_g2(e->s, g2, npairs);
    return st ? lane_fail(srv, e->lane, st) : XPCS_OK;
}

xpcs_status xpcs_server_wait(xpcs_server *srv, int64_t id) {
    if (!srv) return XPCS_EINVAL;
    std::vector<int> lanes;
    if (id == 0) {
        for (int l = 0; l < (int)srv->lane_ctx.size(); ++l) lanes.push_back(l);
    } else {
        auto *e = find(srv, id);
        if (!e) return srv_fail(srv, XPCS_EINVAL, "no such stream id");
        if (e->state != XPCS_STREAM_ADMITTED) return XPCS_OK;
        lanes.push_back(e->lane);
    }
    for (int l : lanes) {
        xpcs_status st = xpcs_sync(srv->lane_ctx[l]);
        if (st) return lane_fail(srv, l, st);
    }
    return XPCS_OK;
}

xpcs_status xpcs_server_close(xpcs_server *srv, int64_t id) {
    if (!srv) return XPCS_EINVAL;
    auto it = srv->entries.find(id);
    if (it == srv->entries.end()) return srv_fail(srv, XPCS_EINVAL, "no such stream id");
    auto &e = it->second;
    (void)hipSetDevice(srv->device);
    if (e.state == XPCS_STREAM_ADMITTED) {
        xpcs_stream_close(e.s);              // waits for the lane
        e.s = nullptr;
        srv->lane_count[e.lane] -= 1;
        srv->admitted -= 1;
        srv->state_used -= e.state_bytes;
    }
    for (auto &b : e.blocks) release_block(srv, b);
    for (auto w = srv->waiting.begin(); w != srv->waiting.end(); ++w)
        if (*w == id) {
            srv->waiting.erase(w);
            break;
        }
    srv->entries.erase(it);
    admit_waiting(srv);
    return XPCS_OK;
}

xpcs_status xpcs_server_stats(const xpcs_server *srv, size_t *bytes_used, int32_t *admitted, int32_t *queued) {
    if (!srv) return XPCS_EINVAL;
    if (bytes_used) *bytes_used = srv->state_used + lanes_bytes(srv);
    if (admitted) *admitted = srv->admitted;
    if (queued) *queued = (int32_t)srv->waiting.size();
    return XPCS_OK;
}

}  // extern "C"
