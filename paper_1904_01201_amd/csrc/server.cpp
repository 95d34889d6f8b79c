// Serving loop: scenes stay resident in HBM; callers submit single-view
// requests (scene, sensor, pose, output pointers) from any thread; one
// request thread admits them by memory footprint and packs them into
// batches that run on `num_streams` HIP streams at once (continuous
// batching: requests that arrive while batches are on the device are
// admitted as soon as a stream and memory free up).  Each batch is an
// ordinary launch sequence, so a result is bitwise the same alone and in
// any mix.  Latency is stamped at submit, launch and observed completion.
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
    uint64_t bytes;    // admission footprint (upper bound of its scratch)
};

struct Batch {
    std::vector<Req> reqs;
    hipEvent_t ev = nullptr;
    int slot = -1;
    uint64_t bytes = 0;
    uint64_t launch_ns = 0;
    uint32_t id = 0;
    bool active = false;
};

constexpr uint32_t kSkipAhead = 64;   // queued requests a blocked head may be overtaken by

}  // namespace

struct hab_server {
    hab_context *ctx = nullptr;
    hab_server_cfg cfg{};
    std::vector<Workspace *> ws;
    std::vector<hipStream_t> streams;
    std::vector<Batch> slots;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req> queue;
    std::unordered_map<uint64_t, hab_request_stats> done;
    std::unordered_map<uint64_t, hab_status> failed;
    std::unordered_map<uint64_t, uint8_t> pending;   // queued or in flight
    uint64_t next_ticket = 1;
    uint64_t inflight_bytes = 0;
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

static void complete(hab_server *s, Batch &b)
{
    const uint64_t t = now_ns();
    std::lock_guard<std::mutex> g(s->mu);
    for (const Req &r : b.reqs) {
        hab_request_stats rs;
        rs.submit_ns = r.submit_ns;
        rs.launch_ns = b.launch_ns;
        rs.done_ns = t;
        rs.batch_size = (uint32_t)b.reqs.size();
        rs.batch_id = b.id;
        s->done[r.ticket] = rs;
        s->pending.erase(r.ticket);
    }
    s->st.completed += b.reqs.size();
    s->inflight_bytes -= b.bytes;
    b.bytes = 0;
    b.reqs.clear();
    b.active = false;
    s->cv_done.notify_all();
}

static void fail_batch(hab_server *s, Batch &b, hab_status e)
{
    std::lock_guard<std::mutex> g(s->mu);
    for (const Req &r : b.reqs) {
        s->failed[r.ticket] = e;
        s->pending.erase(r.ticket);
    }
    s->inflight_bytes -= b.bytes;
    b.bytes = 0;
    b.reqs.clear();
    b.active = false;
    s->loop_error = e;
    s->cv_done.notify_all();
}

static void run_loop(hab_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    std::vector<ViewReq> vr;
    for (;;) {
        // 1. retire finished batches
        for (Batch &b : s->slots) {
            if (!b.active) continue;
            const hipError_t q = hipEventQuery(b.ev);
            if (q == hipSuccess) complete(s, b);
            else if (q != hipErrorNotReady) fail_batch(s, b, HAB_ERR_DEVICE);
        }
        // 2. admit and launch on every free stream
        bool launched = false;
        for (size_t k = 0; k < s->slots.size(); ++k) {
            Batch &b = s->slots[k];
            if (b.active) continue;
            {
                std::unique_lock<std::mutex> g(s->mu);
                if (s->queue.empty()) break;
                // optionally hold a partial batch back to let it fill, up to
                // max_wait_us after its oldest request arrived
                if (s->cfg.max_wait_us && s->queue.size() < s->cfg.max_batch && !s->stop &&
                    now_ns() - s->queue.front().submit_ns < 1000ull * s->cfg.max_wait_us)
                    break;
                b.bytes = 0;
                b.reqs.clear();
                uint64_t room = s->cfg.memory_budget - s->inflight_bytes;
                uint32_t scanned = 0;
                for (auto it = s->queue.begin();
                     it != s->queue.end() && b.reqs.size() < s->cfg.max_batch && scanned < kSkipAhead;) {
                    ++scanned;
                    if (it->bytes <= room) {
                        room -= it->bytes;
                        b.bytes += it->bytes;
                        b.reqs.push_back(*it);
                        it = s->queue.erase(it);
                    } else {
                        ++it;
                    }
                }
                if (b.reqs.empty()) break;   // nothing fits until memory is released
                s->inflight_bytes += b.bytes;
                s->st.peak_inflight_bytes = std::max(s->st.peak_inflight_bytes, s->inflight_bytes);
                s->st.peak_batch = std::max(s->st.peak_batch, (uint32_t)b.reqs.size());
                s->st.batches += 1;
                b.id = s->next_batch++;
            }
            vr.clear();
            for (const Req &r : b.reqs) vr.push_back(r.view);
            b.slot = (int)k;
            b.launch_ns = now_ns();
            PlanOpts o;
            hab_status e = render_all(s->ctx, *s->ws[k], vr.data(), (uint32_t)vr.size(), o,
                                      s->streams[k], nullptr);
            if (e == HAB_OK && hipEventRecord(b.ev, s->streams[k]) != hipSuccess) e = HAB_ERR_DEVICE;
            if (e != HAB_OK) {
                fail_batch(s, b, e);
                continue;
            }
            b.active = true;
            launched = true;
        }
        // 3. exit or wait for work / completions
        bool any_active = false;
        for (const Batch &b : s->slots) any_active |= b.active;
        std::unique_lock<std::mutex> g(s->mu);
        if (s->stop && s->queue.empty() && !any_active) break;
        if (!launched) {
            if (any_active || !s->queue.empty()) {
                g.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
            } else {
                s->cv_work.wait_for(g, std::chrono::milliseconds(5),
                                    [&] { return s->stop || !s->queue.empty(); });
            }
        }
    }
}

extern "C" {

hab_status hab_server_create(hab_context *ctx, const hab_server_cfg *cfg, hab_server **out)
{
    if (!ctx || !out) return HAB_ERR_INVALID_ARG;
    *out = nullptr;
    try {
        hab_server *s = new hab_server();
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
        int prev = -1;
        (void)hipGetDevice(&prev);
        if (hipSetDevice(ctx->device) != hipSuccess) {
            delete s;
            return HAB_ERR_DEVICE;
        }
        s->slots.resize(c.num_streams);
        for (uint32_t k = 0; k < c.num_streams; ++k) {
            hipStream_t st = nullptr;
            hipEvent_t ev = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                for (auto x : s->streams) (void)hipStreamDestroy(x);
                delete s;
                return HAB_ERR_DEVICE;
            }
            s->streams.push_back(st);
            s->slots[k].ev = ev;
            Workspace *w = new Workspace();
            w->device = ctx->device;
            s->ws.push_back(w);
        }
        if (prev >= 0) (void)hipSetDevice(prev);
        s->th = std::thread(run_loop, s);
        *out = s;
        return HAB_OK;
    } catch (const std::bad_alloc &) {
        return HAB_ERR_OUT_OF_MEMORY;
    }
}

hab_status hab_server_submit(hab_server *s, const hab_view *view, uint64_t *ticket)
{
    if (!s || !view || !ticket) return HAB_ERR_INVALID_ARG;
    try {
        Req r;
        hab_status e = to_view_req(*view, r.view);
        if (e != HAB_OK) return e;
        r.bytes = req_bytes(s, r.view);
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) return HAB_ERR_INVALID_ARG;
        if (r.bytes > s->cfg.memory_budget || s->queue.size() >= s->cfg.max_queue) {
            s->st.rejected += 1;
            return HAB_ERR_CAPACITY;
        }
        r.ticket = s->next_ticket++;
        r.submit_ns = now_ns();
        s->queue.push_back(r);
        s->pending[r.ticket] = 1;
        s->st.submitted += 1;
        *ticket = r.ticket;
        s->cv_work.notify_one();
        return HAB_OK;
    } catch (const std::bad_alloc &) {
        return HAB_ERR_OUT_OF_MEMORY;
    }
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
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->ctx->device);
    for (size_t k = 0; k < s->streams.size(); ++k) {
        (void)hipStreamSynchronize(s->streams[k]);
        delete s->ws[k];
        (void)hipStreamDestroy(s->streams[k]);
        (void)hipEventDestroy(s->slots[k].ev);
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    delete s;
    return HAB_OK;
}

}  // extern "C"
