// Graph-captured step loop: a fixed batch composition (scenes, sensors,
// output pointers) is planned once and captured as a HIP graph (descriptor
// upload + the whole kernel sequence).  Each step only rewrites the poses in
// pinned host memory and replays the graph.  Two descriptor buffers and two
// graph instances alternate so the host can stage step k+1 while step k
// runs.  A batch of kSplitViews or more views is planned as two interleaved
// halves whose launch sequences the graph runs side by side (a fork to a
// second capture stream and a join back), as the eager path does.
#include <cstring>
#include <new>
#include <vector>

#include "runtime.h"

using namespace habmi;

// Device-pose steps: copy each view's pose (caller order) into its
// descriptor (planned order) after the descriptor upload; the poses'
// address arrives with the descriptors, in the plan's control slot.
__global__ void k_patch_poses(DView *__restrict__ views, const float *const *__restrict__ ctl,
                              const uint32_t *__restrict__ order, uint32_t n)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float *src = ctl[0] + 12ull * order[k];
    DView &v = views[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) v.p[a] = src[a];
#pragma unroll
    for (int a = 0; a < 9; ++a) v.R[a] = src[3 + a];
}

// One launch sequence of the stepper: views idx[0..) of the caller's list.
struct StepHalf {
    std::vector<ViewReq> req;
    std::vector<uint32_t> idx;   // caller index of each request
    Plan plan;
    std::vector<uint8_t> desc;
    void *arena = nullptr;
    void *host[2] = {nullptr, nullptr};
    uint32_t *dorder = nullptr;  // [n] planned position -> caller index
};

struct hab_stepper {
    hab_context *ctx = nullptr;
    int device = 0;
    uint32_t n = 0;
    int nh = 1;                  // launch sequences per step (1 or 2)
    StepHalf half[2];
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipGraphExec_t exec_dev[2] = {nullptr, nullptr};   // with the pose patch
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool pending[2] = {false, false};
    hipEvent_t last = nullptr;
    bool has_last = false;
    hipStream_t last_stream = nullptr;
    hipStream_t cap = nullptr, cap2 = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;   // capture-time fork and join
    int next = 0;
    uint64_t steps = 0;         // steps taken (advances the depth noise seeds)
};

static void destroy(hab_stepper *st)
{
    for (int b = 0; b < 2; ++b) {
        if (st->pending[b]) (void)hipEventSynchronize(st->ev[b]);
        if (st->exec[b]) (void)hipGraphExecDestroy(st->exec[b]);
        if (st->exec_dev[b]) (void)hipGraphExecDestroy(st->exec_dev[b]);
        if (st->ev[b]) (void)hipEventDestroy(st->ev[b]);
    }
    if (st->has_last) (void)hipEventSynchronize(st->last);
    if (st->last) (void)hipEventDestroy(st->last);
    if (st->fork_ev) (void)hipEventDestroy(st->fork_ev);
    if (st->join_ev) (void)hipEventDestroy(st->join_ev);
    if (st->cap) (void)hipStreamDestroy(st->cap);
    if (st->cap2) (void)hipStreamDestroy(st->cap2);
    for (StepHalf &h : st->half) {
        for (void *p : h.host)
            if (p) pinned_free(p);
        if (h.arena) dev_free(h.arena);
        if (h.dorder) dev_free(h.dorder);
    }
    delete st;
}

// Enqueue one half's descriptor upload (buffer b), the pose patch (dev)
// and its launch sequence on stream s (being captured).
static hipError_t capture_half(StepHalf &h, int b, bool dev, hipStream_t s)
{
    const uint32_t n = (uint32_t)h.req.size();
    hipError_t e = hipMemcpyAsync(h.arena, h.host[b], h.plan.desc_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && dev) {
        DView *views = reinterpret_cast<DView *>(static_cast<char *>(h.arena) + h.plan.off_views);
        const float *const *ctl =
            reinterpret_cast<const float *const *>(static_cast<char *>(h.arena) + h.plan.off_ctl);
        hipLaunchKernelGGL(k_patch_poses, dim3((n + 255) / 256), dim3(256), 0, s, views, ctl,
                           (const uint32_t *)h.dorder, n);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = launch_render(h.plan.L, s);
    return e;
}

extern "C" {

hab_status hab_stepper_create(hab_context *ctx, const hab_view *views, uint32_t n,
                              const hab_render_opts *opts, hipStream_t stream, hab_stepper **out)
{
    if (!ctx || !views || !out || n == 0 || n > kMaxViews) return HAB_ERR_INVALID_ARG;
    if (opts && opts->tile_size && opts->tile_size != 8 && opts->tile_size != 16 && opts->tile_size != 32)
        return HAB_ERR_INVALID_ARG;
    if (opts && (opts->bin_factor < 0.0f || (opts->flags & ~HAB_RENDER_FLAGS))) return HAB_ERR_INVALID_ARG;
    *out = nullptr;
    try {
        int prev = -1;
        (void)hipGetDevice(&prev);
        if (hipSetDevice(ctx->device) != hipSuccess) return HAB_ERR_DEVICE;
        hab_stepper *st = new hab_stepper();
        st->ctx = ctx;
        st->device = ctx->device;
        st->n = n;
        st->nh = n >= kSplitViews && !(opts && (opts->flags & HAB_RENDER_ONE_SEQUENCE)) ? 2 : 1;
        hab_status s = HAB_OK;
        for (uint32_t k = 0; k < n && s == HAB_OK; ++k) {
            StepHalf &h = st->half[st->nh == 2 ? k & 1u : 0u];
            h.req.emplace_back();
            h.idx.push_back(k);
            s = to_view_req(views[k], h.req.back());
        }
        PlanOpts o;
        if (opts) {
            o.tile_size = opts->tile_size;
            o.bin_factor = opts->bin_factor;
            o.tile_cap = opts->tile_cap;
            o.lane_owned_z = (opts->flags & HAB_RENDER_LANE_OWNED_Z) != 0;
        }
        auto fail = [&](hab_status e) {
            destroy(st);
            if (prev >= 0) (void)hipSetDevice(prev);
            return e;
        };
        if (s != HAB_OK) return fail(s);
        for (int hi = 0; hi < st->nh; ++hi) {
            StepHalf &h = st->half[hi];
            const uint32_t nh = (uint32_t)h.req.size();
            s = build_plan(ctx, ctx->ws, h.req.data(), nh, o, h.plan, h.desc);
            if (s != HAB_OK) return fail(s);
            if (!dev_alloc(&h.arena, h.plan.arena_bytes)) return fail(HAB_ERR_OUT_OF_MEMORY);
            bind_plan(h.plan, h.arena, ctx->err);
            std::vector<uint32_t> order(nh);
            for (uint32_t k = 0; k < nh; ++k) order[k] = h.idx[h.plan.order[k]];
            if (!dev_alloc((void **)&h.dorder, 4ull * nh)) return fail(HAB_ERR_OUT_OF_MEMORY);
            if (hipMemcpy(h.dorder, order.data(), 4ull * nh, hipMemcpyHostToDevice) != hipSuccess)
                return fail(HAB_ERR_DEVICE);
            for (int b = 0; b < 2; ++b) {
                if (!pinned_alloc(&h.host[b], h.plan.desc_bytes)) return fail(HAB_ERR_OUT_OF_MEMORY);
                std::memcpy(h.host[b], h.desc.data(), h.plan.desc_bytes);
            }
        }
        if (hipStreamCreateWithFlags(&st->cap, hipStreamNonBlocking) != hipSuccess)
            return fail(HAB_ERR_DEVICE);
        if (hipEventCreateWithFlags(&st->last, hipEventDisableTiming) != hipSuccess)
            return fail(HAB_ERR_DEVICE);
        if (st->nh == 2 && (hipStreamCreateWithFlags(&st->cap2, hipStreamNonBlocking) != hipSuccess ||
                            hipEventCreateWithFlags(&st->fork_ev, hipEventDisableTiming) != hipSuccess ||
                            hipEventCreateWithFlags(&st->join_ev, hipEventDisableTiming) != hipSuccess))
            return fail(HAB_ERR_DEVICE);
        for (int b = 0; b < 2; ++b) {
            if (hipEventCreateWithFlags(&st->ev[b], hipEventDisableTiming) != hipSuccess)
                return fail(HAB_ERR_DEVICE);
            for (int dev = 0; dev < 2; ++dev) {
                hipGraph_t g = nullptr;
                if (hipStreamBeginCapture(st->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
                    return fail(HAB_ERR_DEVICE);
                hipError_t e = hipSuccess;
                if (st->nh == 2) {
                    // fork: the second half on cap2, joined back into cap
                    e = hipEventRecord(st->fork_ev, st->cap);
                    if (e == hipSuccess) e = hipStreamWaitEvent(st->cap2, st->fork_ev, 0);
                    if (e == hipSuccess) e = capture_half(st->half[1], b, dev != 0, st->cap2);
                    if (e == hipSuccess) e = capture_half(st->half[0], b, dev != 0, st->cap);
                    if (e == hipSuccess) e = hipEventRecord(st->join_ev, st->cap2);
                    if (e == hipSuccess) e = hipStreamWaitEvent(st->cap, st->join_ev, 0);
                } else {
                    e = capture_half(st->half[0], b, dev != 0, st->cap);
                }
                hipError_t e2 = hipStreamEndCapture(st->cap, &g);
                if (e != hipSuccess || e2 != hipSuccess || !g) {
                    if (g) (void)hipGraphDestroy(g);
                    return fail(HAB_ERR_DEVICE);
                }
                e = hipGraphInstantiate(dev ? &st->exec_dev[b] : &st->exec[b], g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) return fail(HAB_ERR_DEVICE);
            }
        }
        (void)stream;
        if (prev >= 0) (void)hipSetDevice(prev);
        *out = st;
        return HAB_OK;
    } catch (const std::bad_alloc &) {
        return HAB_ERR_OUT_OF_MEMORY;
    }
}

}  // extern "C"

// One step: host poses (validated, staged with the descriptors) or device
// poses (their address staged in the control slot, patched into the
// descriptors by the graph).
static hab_status step_common(hab_stepper *st, const hab_pose *poses, const float *dposes,
                              hipStream_t stream)
{
    if (poses)
        for (int hi = 0; hi < st->nh; ++hi) {
            const StepHalf &h = st->half[hi];
            for (size_t k = 0; k < h.req.size(); ++k) {
                hab_status s = validate_pose(h.req[k].scene, &h.req[k].sensor, &poses[h.idx[k]]);
                if (s != HAB_OK) return s;
            }
        }
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(st->device) != hipSuccess) return HAB_ERR_DEVICE;
    const int b = st->next;
    st->next ^= 1;
    hab_status rc = HAB_OK;
    do {
        if (st->pending[b]) {
            if (hipEventSynchronize(st->ev[b]) != hipSuccess) { rc = HAB_ERR_DEVICE; break; }
            st->pending[b] = false;
        }
        for (int hi = 0; hi < st->nh; ++hi) {
            StepHalf &hf = st->half[hi];
            char *h = static_cast<char *>(hf.host[b]);
            if (dposes) std::memcpy(h + hf.plan.off_ctl, &dposes, sizeof dposes);
            for (size_t k = 0; k < hf.req.size(); ++k) {
                DView *d = reinterpret_cast<DView *>(h + hf.plan.off_views) + k;
                const uint32_t r = hf.plan.order[k];
                if (poses) {
                    const hab_pose &p = poses[hf.idx[r]];
                    std::memcpy(d->p, p.position, sizeof d->p);
                    std::memcpy(d->R, p.rotation, sizeof d->R);
                }
                d->noise_seed = hf.req[r].noise_seed + st->steps;
            }
        }
        if (st->has_last && st->last_stream != stream &&
            hipStreamWaitEvent(stream, st->last, 0) != hipSuccess) { rc = HAB_ERR_DEVICE; break; }
        if (hipGraphLaunch(dposes ? st->exec_dev[b] : st->exec[b], stream) != hipSuccess) { rc = HAB_ERR_DEVICE; break; }
        if (hipEventRecord(st->ev[b], stream) != hipSuccess) { rc = HAB_ERR_DEVICE; break; }
        st->pending[b] = true;
        ++st->steps;
        if (hipEventRecord(st->last, stream) != hipSuccess) { rc = HAB_ERR_DEVICE; break; }
        st->has_last = true;
        st->last_stream = stream;
    } while (0);
    if (prev >= 0) (void)hipSetDevice(prev);
    return rc;
}

extern "C" {

hab_status hab_stepper_step(hab_stepper *st, const hab_pose *poses, hipStream_t stream)
{
    if (!st || !poses) return HAB_ERR_INVALID_ARG;
    return step_common(st, poses, nullptr, stream);
}

hab_status hab_stepper_step_device(hab_stepper *st, const float *poses, hipStream_t stream)
{
    if (!st || !poses) return HAB_ERR_INVALID_ARG;
    return step_common(st, nullptr, poses, stream);
}

hab_status hab_stepper_destroy(hab_stepper *st)
{
    if (!st) return HAB_ERR_INVALID_ARG;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(st->device);
    destroy(st);
    if (prev >= 0) (void)hipSetDevice(prev);
    return HAB_OK;
}

}  // extern "C"
