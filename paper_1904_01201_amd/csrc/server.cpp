// Serving loop: scenes stay resident in HBM; callers submit single-view
// requests (scene, sensor, pose, output pointers) from any thread; one
// request thread admits them by memory footprint and packs them into
// batches that run on `num_streams` HIP streams at once (continuous
// batching: requests that arrive while batches are on the device are
// admitted as soon as a stream and memory free up).  The server's device
// scratch is one pool of memory_budget bytes allocated at creation; each
// launched batch works in a region of it (admission.h), so the budget
// bounds the memory actually held.  Each batch is an ordinary launch
// sequence, so a result is bitwise the same alone and in any mix.  Latency
// is stamped at submit, launch and observed completion.  Queued requests
// can be cancelled, and time out at their deadline.
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "admission.h"
#include "runtime.h"

using namespace habmi;

namespace {

uint64_t now_ns()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

struct Req {
    uint64_t ticket;
    ViewReq view;
    uint64_t submit_ns;
};

struct Batch {
    std::vector<Req> reqs;
    hipEvent_t ev = nullptr;
    uint64_t offset = 0, bytes = 0;   // region of the scratch pool
    uint64_t launch_ns = 0;
    uint32_t id = 0;
    bool active = false;
};

constexpr uint32_t kSkipAhead = 64;   // queued requests a batch may look at
constexpr uint32_t kMaxSkips = 8;     // batches that may pass one request over

}  // namespace

struct hab_server {
    hab_context *ctx = nullptr;
    hab_server_cfg cfg{};
    std::vector<Workspace *> ws;
    std::vector<hipStream_t> streams;
    std::vector<Batch> slots;
    void *pool = nullptr;             // memory_budget bytes of device scratch
    std::thread th;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    Admission *adm = nullptr;
    std::unordered_map<uint64_t, Req> queued;   // requests not launched yet
    std::unordered_map<uint64_t, hab_request_stats> done;
    std::unordered_map<uint64_t, hab_status> failed;
    std::unordered_map<uint64_t, uint8_t> pending;   // queued or in flight
    uint64_t next_ticket = 1;
    uint32_t next_batch = 0;
    bool stop = false;
    hab_server_stats st{};
    hab_status loop_error = HAB_OK;
};

static uint64_t req_bytes(hab_server *s, const ViewReq &v)
{
    PlanOpts o;
    return footprint(&v, 1, o, s->ctx).arena_bytes;
}

// Retire a batch (caller holds the lock): results or an error per ticket,
// its pool region returned.
static void retire(hab_server *s, Batch &b, hab_status e, uint64_t t)
{
    for (const Req &r : b.reqs) {
        if (e == HAB_OK) {
            hab_request_stats rs;
            rs.submit_ns = r.submit_ns;
            rs.launch_ns = b.launch_ns;
            rs.done_ns = t;
            rs.batch_size = (uint32_t)b.reqs.size();
            rs.batch_id = b.id;
            s->done[r.ticket] = rs;
        } else {
            s->failed[r.ticket] = e;
        }
        s->pending.erase(r.ticket);
    }
    if (e == HAB_OK) s->st.completed += b.reqs.size();
    else s->loop_error = e;
    s->adm->release(b.offset, b.bytes);
    b.offset = b.bytes = 0;
    b.reqs.clear();
    b.active = false;
    s->cv_done.notify_all();
}

static void run_loop(hab_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    std::vector<ViewReq> vr;
    std::vector<uint64_t> gone;
    Admission::Batch ab;
    const uint64_t hold_ns = 1000ull * s->cfg.max_wait_us;
    for (;;) {
        // 1. retire finished batches
        for (Batch &b : s->slots) {
            if (!b.active) continue;
            const hipError_t q = hipEventQuery(b.ev);
            if (q == hipErrorNotReady) continue;
            const uint64_t t = now_ns();
            std::lock_guard<std::mutex> g(s->mu);
            retire(s, b, q == hipSuccess ? HAB_OK : HAB_ERR_DEVICE, t);
        }
        // 2. queued requests past their deadline
        {
            std::lock_guard<std::mutex> g(s->mu);
            gone.clear();
            s->adm->expire(now_ns(), gone);
            for (uint64_t tk : gone) {
                s->queued.erase(tk);
                s->pending.erase(tk);
                s->failed[tk] = HAB_ERR_TIMEOUT;
                s->st.expired += 1;
            }
            if (!gone.empty()) s->cv_done.notify_all();
        }
        // 3. admit and launch on every free stream
        bool launched = false;
        for (size_t k = 0; k < s->slots.size(); ++k) {
            Batch &b = s->slots[k];
            if (b.active) continue;
            {
                std::lock_guard<std::mutex> g(s->mu);
                if (!s->adm->next(now_ns(), hold_ns, s->stop, ab)) break;
                b.reqs.clear();
                for (const AdmReq &a : ab.reqs) {
                    auto it = s->queued.find(a.ticket);
                    b.reqs.push_back(it->second);
                    s->queued.erase(it);
                }
                b.offset = ab.offset;
                b.bytes = ab.size;
                s->st.peak_inflight_bytes = std::max(s->st.peak_inflight_bytes, s->adm->in_use());
                s->st.peak_batch = std::max(s->st.peak_batch, (uint32_t)b.reqs.size());
                s->st.batches += 1;
                b.id = s->next_batch++;
            }
            vr.clear();
            for (const Req &r : b.reqs) vr.push_back(r.view);
            b.launch_ns = now_ns();
            // the batch's region of the pool is its workspace arena
            Workspace &w = *s->ws[k];
            w.arena = static_cast<char *>(s->pool) + b.offset;
            w.cap = b.bytes;
            PlanOpts o;
            hab_status e = render_all(s->ctx, w, vr.data(), (uint32_t)vr.size(), o, s->streams[k], nullptr);
            if (e == HAB_OK && hipEventRecord(b.ev, s->streams[k]) != hipSuccess) e = HAB_ERR_DEVICE;
            if (e != HAB_OK) {
                // the stream may still be running earlier work on this
                // region: wait before the region goes back to the pool
                (void)hipStreamSynchronize(s->streams[k]);
                std::lock_guard<std::mutex> g(s->mu);
                retire(s, b, e, now_ns());
                continue;
            }
            b.active = true;
            launched = true;
        }
        // 4. exit or wait for work / completions
        bool any_active = false;
        for (const Batch &b : s->slots) any_active |= b.active;
        std::unique_lock<std::mutex> g(s->mu);
        if (s->stop && s->adm->queued() == 0 && !any_active) break;
        if (!launched) {
            if (any_active || s->adm->queued() != 0) {
                g.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
            } else {
                s->cv_work.wait_for(g, std::chrono::milliseconds(5),
                                    [&] { return s->stop || s->adm->queued() != 0; });
            }
        }
    }
}

extern "C" {

static void destroy_server(hab_server *s)
{
    for (size_t k = 0; k < s->streams.size(); ++k) {
        (void)hipStreamSynchronize(s->streams[k]);
        (void)hipStreamDestroy(s->streams[k]);
    }
    for (Workspace *w : s->ws) delete w;
    for (Batch &b : s->slots)
        if (b.ev) (void)hipEventDestroy(b.ev);
    if (s->pool) dev_free(s->pool);
    delete s->adm;
    delete s;
}

hab_status hab_server_create(hab_context *ctx, const hab_server_cfg *cfg, hab_server **out)
{
    if (!ctx || !out) return HAB_ERR_INVALID_ARG;
    *out = nullptr;
    hab_server *s = nullptr;
    try {
        s = new hab_server();
        s->ctx = ctx;
        hab_server_cfg c{};
        if (cfg) c = *cfg;
        if (c.num_streams == 0) c.num_streams = 2;
        if (c.num_streams > 16) c.num_streams = 16;
        if (c.max_batch == 0) c.max_batch = 256;
        if (c.max_batch > kMaxViews) c.max_batch = kMaxViews;
        if (c.memory_budget == 0) c.memory_budget = 8ull << 30;
        if (c.max_queue == 0) c.max_queue = 65536;
        s->cfg = c;
        s->adm = new Admission(c.memory_budget, c.max_queue, c.max_batch, kSkipAhead, kMaxSkips);
        DeviceGuard g(ctx->device);
        if (!g.ok) {
            destroy_server(s);
            return HAB_ERR_DEVICE;
        }
        if (!dev_alloc(&s->pool, c.memory_budget)) {
            destroy_server(s);
            return HAB_ERR_OUT_OF_MEMORY;
        }
        s->st.scratch_bytes = c.memory_budget;
        s->slots.resize(c.num_streams);
        for (uint32_t k = 0; k < c.num_streams; ++k) {
            hipStream_t st = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
                destroy_server(s);
                return HAB_ERR_DEVICE;
            }
            s->streams.push_back(st);
            if (hipEventCreateWithFlags(&s->slots[k].ev, hipEventDisableTiming) != hipSuccess) {
                s->slots[k].ev = nullptr;
                destroy_server(s);
                return HAB_ERR_DEVICE;
            }
            Workspace *w = new Workspace();
            w->device = ctx->device;
            w->external = true;   // its arena is a region of the pool
            s->ws.push_back(w);
        }
        s->th = std::thread(run_loop, s);
        *out = s;
        return HAB_OK;
    } catch (const std::bad_alloc &) {
        if (s) destroy_server(s);
        return HAB_ERR_OUT_OF_MEMORY;
    }
}

hab_status hab_server_submit_ex(hab_server *s, const hab_view *view, uint32_t timeout_us, uint64_t *ticket)
{
    if (!s || !view || !ticket) return HAB_ERR_INVALID_ARG;
    try {
        Req r;
        hab_status e = to_view_req(*view, r.view);
        if (e != HAB_OK) return e;
        AdmReq a;
        a.bytes = req_bytes(s, r.view);
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) return HAB_ERR_INVALID_ARG;
        a.ticket = s->next_ticket;
        a.submit_ns = now_ns();
        a.deadline_ns = timeout_us ? a.submit_ns + 1000ull * timeout_us : 0;
        const Admission::Submit q = s->adm->submit(a);
        if (q != Admission::kQueued) {
            s->st.rejected += 1;
            return HAB_ERR_CAPACITY;
        }
        r.ticket = a.ticket;
        r.submit_ns = a.submit_ns;
        s->next_ticket += 1;
        s->queued.emplace(r.ticket, r);
        s->pending[r.ticket] = 1;
        s->st.submitted += 1;
        *ticket = r.ticket;
        s->cv_work.notify_one();
        return HAB_OK;
    } catch (const std::bad_alloc &) {
        return HAB_ERR_OUT_OF_MEMORY;
    }
}

hab_status hab_server_submit(hab_server *s, const hab_view *view, uint64_t *ticket)
{
    return hab_server_submit_ex(s, view, 0, ticket);
}

hab_status hab_server_cancel(hab_server *s, uint64_t ticket)
{
    if (!s) return HAB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    if (s->adm->cancel(ticket)) {
        s->queued.erase(ticket);
        s->pending.erase(ticket);
        s->failed[ticket] = HAB_ERR_CANCELLED;
        s->st.cancelled += 1;
        s->cv_done.notify_all();
        return HAB_OK;
    }
    // launched (it completes), or unknown / already collected
    return s->pending.count(ticket) ? HAB_ERR_NOT_READY : HAB_ERR_INVALID_ARG;
}

static hab_status take(hab_server *s, uint64_t ticket, hab_request_stats *out)
{
    auto it = s->done.find(ticket);
    if (it != s->done.end()) {
        if (out) *out = it->second;
        s->done.erase(it);
        return HAB_OK;
    }
    auto f = s->failed.find(ticket);
    if (f != s->failed.end()) {
        hab_status e = f->second;
        s->failed.erase(f);
        return e;
    }
    if (s->pending.count(ticket)) return HAB_ERR_NOT_READY;
    return HAB_ERR_INVALID_ARG;   // unknown, or already collected
}

hab_status hab_server_poll(hab_server *s, uint64_t ticket, hab_request_stats *out)
{
    if (!s) return HAB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    return take(s, ticket, out);
}

hab_status hab_server_wait(hab_server *s, uint64_t ticket, hab_request_stats *out)
{
    if (!s) return HAB_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> g(s->mu);
    for (;;) {
        hab_status e = take(s, ticket, out);
        if (e != HAB_ERR_NOT_READY) return e;
        s->cv_done.wait_for(g, std::chrono::milliseconds(10));
    }
}

hab_status hab_server_stats_get(hab_server *s, hab_server_stats *out)
{
    if (!s || !out) return HAB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->st;
    return HAB_OK;
}

hab_status hab_server_destroy(hab_server *s)
{
    if (!s) return HAB_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    DeviceGuard g(s->ctx->device);
    destroy_server(s);
    return HAB_OK;
}

}  // extern "C"
