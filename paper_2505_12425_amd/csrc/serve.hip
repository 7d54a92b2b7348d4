// serve.hip -- the request server: continuous batching of resize / warp
// requests (serve_core.h) over `slots` HIP streams, with outputs in one
// device arena sized by the caller's HBM budget.
//
// Each slot owns a stream, a completion event, a pinned host staging buffer
// and a device buffer for its batch's work-list, all created once.  A slot's
// batch takes its class's batch configuration (one workgroup per tile unless
// the tuning table names a persistent grid), so that batches of different
// slots share the GPU.  A slot is reused only after its event has
// completed, so its staging and work-list buffers are never overwritten while
// in flight.  Output blocks stay allocated until released by the caller.
// One server object is driven by one host thread at a time.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <unordered_map>
#include <vector>

#include "batch_internal.h"
#include "kr_api_internal.h"
#include "serve_core.h"

namespace kr {

struct HipExec {
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        void *staging = nullptr;  // pinned host
        void *table = nullptr;    // device
    };
    std::vector<Slot> slots;
    uint8_t *arena_base = nullptr;
    int c = 3;
    kr_dtype dt = KR_U8;
    Epilogue e{};
    size_t table_cap = 0;  // bytes of one slot's table buffer

    bool launch(int s, const std::vector<serve::Admitted> &batch)
    {
        Slot &sl = slots[s];
        std::vector<ImageJob> imgs[2];
        for (const serve::Admitted &a : batch) {
            ImageJob j;
            std::memset(&j, 0, sizeof j);
            j.src = a.req.src;
            j.dst = arena_base + a.dst_off;
            j.sh = a.req.sh; j.sw = a.req.sw; j.dh = a.req.dh; j.dw = a.req.dw;
            j.sp = a.req.sw;  // contiguous source
            j.sk = 0;
            for (int i = 0; i < 6; i++)
                j.inv[i] = a.req.m[i];
            imgs[a.req.op == OP_WARP ? 1 : 0].push_back(j);
        }
        const TileCfg *const none[2] = {nullptr, nullptr};
        BatchBuild bb;
        build_batch(imgs, dt == KR_F32, c, none, bb);
        const size_t bytes = bb.bytes();
        if (bytes > table_cap)
            return false;
        bb.pack(static_cast<uint8_t *>(sl.staging));
        // On a failure after something was enqueued, the scheduler releases
        // the batch's output blocks and requeues its requests, and the slot's
        // staging buffer may be repacked at once: wait for what this slot
        // already has in flight before reporting it.
        bool ok = hipMemcpyAsync(sl.table, sl.staging, bytes, hipMemcpyHostToDevice, sl.stream) == hipSuccess;
        bb.bind(sl.table);
        for (size_t g = 0; ok && g < bb.groups.size(); g++)
            ok = launch_group(bb.groups[g], c, dt, e, sl.stream) == hipSuccess;
        ok = ok && hipEventRecord(sl.done, sl.stream) == hipSuccess;
        if (!ok)
            (void)hipStreamSynchronize(sl.stream);
        return ok;
    }

    bool done(int s) { return hipEventQuery(slots[s].done) == hipSuccess; }
};

}  // namespace kr

using namespace kr;

struct kr_server {
    kr_server_config cfg{};
    int c = 3;
    kr_dtype st = KR_U8, dt = KR_U8;
    HipExec exec;
    serve::Scheduler<HipExec> *sched = nullptr;
    void *arena = nullptr;
    uint64_t next_id = 0;
    std::unordered_map<uint64_t, size_t> done_off;  // completed, not yet released
    std::vector<serve::Completion> pending;
    std::chrono::steady_clock::time_point t0;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

static void server_free(kr_server *s)
{
    if (!s)
        return;
    for (auto &sl : s->exec.slots) {
        if (sl.stream)
            (void)hipStreamSynchronize(sl.stream);
        if (sl.done)
            (void)hipEventDestroy(sl.done);
        if (sl.stream)
            (void)hipStreamDestroy(sl.stream);
        if (sl.staging)
            (void)hipHostFree(sl.staging);
        if (sl.table)
            (void)hipFree(sl.table);
    }
    if (s->arena)
        (void)hipFree(s->arena);
    delete s->sched;
    delete s;
}

// Validate one request and turn it into a scheduler request (warp matrices
// are inverted here, once).
static kr_status make_request(const kr_server *s, const kr_request *r, serve::Request &out)
{
    if (!r)
        return fail(KR_ERR_INVALID_ARGUMENT, "request pointer is NULL");
    if (r->op != KR_OP_RESIZE && r->op != KR_OP_WARP)
        return fail(KR_ERR_INVALID_ARGUMENT, "unknown op %d", r->op);
    kr_status st = check_image("src", r->src, r->src_h, r->src_w, s->c);
    if (st != KR_OK)
        return st;
    if (r->dst_h < 1 || r->dst_w < 1 || r->dst_h > KR_MAX_DIM || r->dst_w > KR_MAX_DIM)
        return fail(KR_ERR_INVALID_ARGUMENT, "dst size %dx%d outside [1, %d]", r->dst_h, r->dst_w, KR_MAX_DIM);
    out = serve::Request{};
    out.op = r->op;
    out.src = r->src;
    out.sh = r->src_h; out.sw = r->src_w; out.dh = r->dst_h; out.dw = r->dst_w;
    if (r->op == KR_OP_WARP) {
        if (r->flags & ~KR_WARP_INVERSE_MAP)
            return fail(KR_ERR_INVALID_ARGUMENT, "unknown warp flags 0x%x", r->flags);
        st = check_matrix(r->m, r->flags, out.m);
        if (st != KR_OK)
            return st;
    }
    out.dst_bytes = (size_t)r->dst_h * r->dst_w * s->c * (s->dt == KR_U8 ? 1 : 4);
    return KR_OK;
}

static void harvest(kr_server *s, std::vector<serve::Completion> &comps)
{
    for (const auto &cpl : comps) {
        s->done_off[cpl.id] = cpl.dst_off;
        s->pending.push_back(cpl);
    }
}

extern "C" {

kr_status kr_server_create(const kr_server_config *cfg, int c, kr_dtype src_t, kr_dtype dst_t, kr_border border,
                           float border_value, const kr_normalize *norm, kr_server **out)
{
    clear_error();
    if (!out)
        return fail(KR_ERR_INVALID_ARGUMENT, "server pointer is NULL");
    *out = nullptr;
    if (!cfg)
        return fail(KR_ERR_INVALID_ARGUMENT, "config pointer is NULL");
    if (cfg->budget_bytes < 256 || cfg->slots < 1 || cfg->slots > 16 || cfg->max_batch < 1 || cfg->max_batch > 4096)
        return fail(KR_ERR_INVALID_ARGUMENT, "config out of range (budget >= 256 B, 1 <= slots <= 16, "
                                             "1 <= max_batch <= 4096)");
    if (c < 1 || c > 4)
        return fail(KR_ERR_UNSUPPORTED, "channel count %d not in [1, 4]", c);
    if (!tiled_image_supported(c, src_t) || !(dst_t == KR_U8 || dst_t == KR_F32))
        return fail(KR_ERR_UNSUPPORTED, "the server needs u8 sources");
    if (border != KR_BORDER_CONSTANT && border != KR_BORDER_REPLICATE)
        return fail(KR_ERR_UNSUPPORTED, "border mode %d not supported", (int)border);
    if (!std::isfinite(border_value) || border_value < 0.0f || border_value > 255.0f ||
        border_value != std::floor(border_value))
        return fail(KR_ERR_INVALID_ARGUMENT, "u8 border value %g is not an integer in [0, 255]", (double)border_value);
    if (norm && dst_t != KR_F32)
        return fail(KR_ERR_INVALID_ARGUMENT, "normalisation needs an f32 destination");
    kr_server *s = new (std::nothrow) kr_server();
    if (!s)
        return fail(KR_ERR_INVALID_ARGUMENT, "out of host memory");
    s->cfg = *cfg;
    s->c = c;
    s->st = src_t;
    s->dt = dst_t;
    s->exec.c = c;
    s->exec.dt = dst_t;
    s->exec.e = make_epilogue(c, border, border_value, norm);
    s->exec.table_cap = kr_resize_batch_workspace_size(cfg->max_batch);
    hipError_t err = hipMalloc(&s->arena, cfg->budget_bytes);
    s->exec.arena_base = static_cast<uint8_t *>(s->arena);
    s->exec.slots.resize(cfg->slots);
    for (int i = 0; i < cfg->slots && err == hipSuccess; i++) {
        auto &sl = s->exec.slots[i];
        err = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (err == hipSuccess)
            err = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (err == hipSuccess)
            err = hipHostMalloc(&sl.staging, s->exec.table_cap, hipHostMallocDefault);
        if (err == hipSuccess)
            err = hipMalloc(&sl.table, s->exec.table_cap);
    }
    if (err != hipSuccess) {
        server_free(s);
        return fail(KR_ERR_HIP, "server setup failed: %s", hipGetErrorString(err));
    }
    s->sched = new (std::nothrow) serve::Scheduler<HipExec>(s->exec, cfg->budget_bytes, cfg->slots, cfg->max_batch);
    if (!s->sched) {
        server_free(s);
        return fail(KR_ERR_INVALID_ARGUMENT, "out of host memory");
    }
    s->t0 = std::chrono::steady_clock::now();
    *out = s;
    return KR_OK;
}

double kr_server_now(const kr_server *s) { return s ? s->now() : 0.0; }

kr_status kr_server_submit(kr_server *s, const kr_request *req, uint64_t *id)
{
    clear_error();
    if (!s)
        return fail(KR_ERR_INVALID_ARGUMENT, "server is NULL");
    serve::Request r;
    kr_status st = make_request(s, req, r);
    if (st != KR_OK)
        return st;
    r.id = s->next_id;
    r.t_arrival = s->now();
    if (!s->sched->submit(r))
        return fail(KR_ERR_OUT_OF_BUDGET, "request output of %zu bytes exceeds the %zu-byte budget", r.dst_bytes,
                    s->cfg.budget_bytes);
    s->next_id++;
    if (id)
        *id = r.id;
    return KR_OK;
}

kr_status kr_server_poll(kr_server *s, kr_completion *out, int max_out, int *n_out)
{
    clear_error();
    if (!s || (max_out > 0 && !out) || !n_out)
        return fail(KR_ERR_INVALID_ARGUMENT, "NULL argument");
    std::vector<serve::Completion> comps;
    const bool ok = s->sched->step(s->now(), comps);
    harvest(s, comps);
    int n = 0;
    while (n < max_out && !s->pending.empty()) {
        const serve::Completion &cpl = s->pending.front();
        out[n].id = cpl.id;
        out[n].dst = static_cast<uint8_t *>(s->arena) + cpl.dst_off;
        out[n].dst_bytes = cpl.dst_bytes;
        out[n].t_done = cpl.t_done;
        n++;
        s->pending.erase(s->pending.begin());
    }
    *n_out = n;
    if (!ok)
        return fail(KR_ERR_HIP, "a batch launch failed");
    return KR_OK;
}

kr_status kr_server_release(kr_server *s, uint64_t id)
{
    clear_error();
    if (!s)
        return fail(KR_ERR_INVALID_ARGUMENT, "server is NULL");
    auto it = s->done_off.find(id);
    if (it == s->done_off.end())
        return fail(KR_ERR_INVALID_ARGUMENT, "request %llu is not completed or already released",
                    (unsigned long long)id);
    s->sched->release(it->second);
    s->done_off.erase(it);
    return KR_OK;
}

kr_status kr_server_stats(const kr_server *s, size_t *arena_used, size_t *queued, int *busy_slots)
{
    if (!s)
        return KR_ERR_INVALID_ARGUMENT;
    if (arena_used)
        *arena_used = s->sched->arena().used();
    if (queued)
        *queued = s->sched->queued();
    if (busy_slots)
        *busy_slots = s->sched->busy_slots();
    return KR_OK;
}

kr_status kr_server_run_trace(kr_server *s, const kr_request *reqs, const double *arrival_s, int n, double *latency_s)
{
    clear_error();
    if (!s || n < 0 || (n > 0 && (!reqs || !arrival_s || !latency_s)))
        return fail(KR_ERR_INVALID_ARGUMENT, "bad trace arguments");
    if (!s->sched->idle() || !s->pending.empty() || !s->done_off.empty())
        return fail(KR_ERR_INVALID_ARGUMENT, "run_trace needs an idle server with nothing unreleased");
    std::vector<serve::Request> rq(n);
    for (int i = 0; i < n; i++) {
        kr_status st = make_request(s, &reqs[i], rq[i]);
        if (st != KR_OK)
            return fail(st, "request %d: %s", i, kr_last_error());
        if (s->sched->arena().round(rq[i].dst_bytes) > s->cfg.budget_bytes)
            return fail(KR_ERR_OUT_OF_BUDGET, "request %d exceeds the budget", i);
        rq[i].id = (uint64_t)i;
        rq[i].t_arrival = arrival_s[i];
        latency_s[i] = -1.0;
    }
    const auto t_start = std::chrono::steady_clock::now();
    auto clock = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count(); };
    int next = 0, done = 0;
    std::vector<serve::Completion> comps;
    while (done < n) {
        const double t = clock();
        while (next < n && arrival_s[next] <= t)
            s->sched->submit(rq[next++]);
        comps.clear();
        if (!s->sched->step(clock(), comps))
            return fail(KR_ERR_HIP, "a batch launch failed");
        for (const auto &cpl : comps) {
            latency_s[cpl.id] = cpl.t_done - arrival_s[cpl.id];
            s->sched->release(cpl.dst_off);
            done++;
        }
    }
    return KR_OK;
}

void kr_server_destroy(kr_server *s) { server_free(s); }

}  // extern "C"
