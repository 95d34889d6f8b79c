// Graph-captured step loop: a fixed batch composition (scenes, sensors,
// output pointers) is planned once and captured as a HIP graph (descriptor
// upload + the whole kernel sequence).  Each step only rewrites the poses in
// pinned host memory and replays the graph.  Two descriptor buffers and two
// graph instances alternate so the host can stage step k+1 while step k
// runs.
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

struct hab_stepper {
    hab_context *ctx = nullptr;
    int device = 0;
    std::vector<ViewReq> req;
    Plan plan;
    std::vector<uint8_t> desc;
    void *arena = nullptr;
    void *host[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipGraphExec_t exec_dev[2] = {nullptr, nullptr};   // with the pose patch
    uint32_t *dorder = nullptr;   // [n] planned position -> caller index
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool pending[2] = {false, false};
    hipEvent_t last = nullptr;
    bool has_last = false;
    hipStream_t last_stream = nullptr;
    hipStream_t cap = nullptr;
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
        if (st->host[b]) pinned_free(st->host[b]);
    }
    if (st->has_last) (void)hipEventSynchronize(st->last);
    if (st->last) (void)hipEventDestroy(st->last);
    if (st->cap) (void)hipStreamDestroy(st->cap);
    if (st->arena) dev_free(st->arena);
    if (st->dorder) dev_free(st->dorder);
    delete st;
}

extern "C" {

hab_status hab_stepper_create(hab_context *ctx, const hab_view *views, uint32_t n,
                              const hab_render_opts *opts, hipStream_t stream, hab_stepper **out)
{
    if (!ctx || !views || !out || n == 0 || n > kMaxViews) return HAB_ERR_INVALID_ARG;
    if (opts && opts->tile_size && opts->tile_size != 8 && opts->tile_size != 16 && opts->tile_size != 32)
        return HAB_ERR_INVALID_ARG;
    *out = nullptr;
    try {
        int prev = -1;
        (void)hipGetDevice(&prev);
        if (hipSetDevice(ctx->device) != hipSuccess) return HAB_ERR_DEVICE;
        hab_stepper *st = new hab_stepper();
        st->ctx = ctx;
        st->device = ctx->device;
        st->req.resize(n);
        hab_status s = HAB_OK;
        for (uint32_t k = 0; k < n && s == HAB_OK; ++k) s = to_view_req(views[k], st->req[k]);
        PlanOpts o;
        if (opts) {
            o.tile_size = opts->tile_size;
            o.bin_factor = opts->bin_factor;
            o.tile_cap = opts->tile_cap;
        }
        if (s == HAB_OK) s = build_plan(ctx, ctx->ws, st->req.data(), n, o, st->plan, st->desc);
        auto fail = [&](hab_status e) {
            destroy(st);
            if (prev >= 0) (void)hipSetDevice(prev);
            return e;
        };
        if (s != HAB_OK) return fail(s);
        if (!dev_alloc(&st->arena, st->plan.arena_bytes)) return fail(HAB_ERR_OUT_OF_MEMORY);
        bind_plan(st->plan, st->arena, ctx->err);
        if (!dev_alloc((void **)&st->dorder, 4ull * n)) return fail(HAB_ERR_OUT_OF_MEMORY);
        if (hipMemcpy(st->dorder, st->plan.order.data(), 4ull * n, hipMemcpyHostToDevice) != hipSuccess)
            return fail(HAB_ERR_DEVICE);
        if (hipStreamCreateWithFlags(&st->cap, hipStreamNonBlocking) != hipSuccess)
            return fail(HAB_ERR_DEVICE);
        if (hipEventCreateWithFlags(&st->last, hipEventDisableTiming) != hipSuccess)
            return fail(HAB_ERR_DEVICE);
        for (int b = 0; b < 2; ++b) {
            if (!pinned_alloc(&st->host[b], st->plan.desc_bytes)) return fail(HAB_ERR_OUT_OF_MEMORY);
            std::memcpy(st->host[b], st->desc.data(), st->plan.desc_bytes);
            if (hipEventCreateWithFlags(&st->ev[b], hipEventDisableTiming) != hipSuccess)
                return fail(HAB_ERR_DEVICE);
            for (int dev = 0; dev < 2; ++dev) {
                hipGraph_t g = nullptr;
                if (hipStreamBeginCapture(st->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
                    return fail(HAB_ERR_DEVICE);
                hipError_t e = hipMemcpyAsync(st->arena, st->host[b], st->plan.desc_bytes,
                                              hipMemcpyHostToDevice, st->cap);
                if (e == hipSuccess && dev) {
                    DView *views = reinterpret_cast<DView *>(static_cast<char *>(st->arena) + st->plan.off_views);
                    const float *const *ctl =
                        reinterpret_cast<const float *const *>(static_cast<char *>(st->arena) + st->plan.off_ctl);
                    hipLaunchKernelGGL(k_patch_poses, dim3((n + 255) / 256), dim3(256), 0, st->cap, views, ctl,
                                       (const uint32_t *)st->dorder, n);
                    e = hipGetLastError();
                }
                if (e == hipSuccess) e = launch_render(st->plan.L, st->cap);
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
    const uint32_t n = (uint32_t)st->req.size();
    if (poses)
        for (uint32_t k = 0; k < n; ++k) {
            hab_status s = validate_pose(st->req[k].scene, &st->req[k].sensor, &poses[k]);
            if (s != HAB_OK) return s;
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
        char *h = static_cast<char *>(st->host[b]);
        if (dposes) std::memcpy(h + st->plan.off_ctl, &dposes, sizeof dposes);
        for (uint32_t k = 0; k < n; ++k) {
            DView *d = reinterpret_cast<DView *>(h + st->plan.off_views) + k;
            if (poses) {
                const hab_pose &p = poses[st->plan.order[k]];
                std::memcpy(d->p, p.position, sizeof d->p);
                std::memcpy(d->R, p.rotation, sizeof d->R);
            }
            d->noise_seed = st->req[st->plan.order[k]].noise_seed + st->steps;
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
