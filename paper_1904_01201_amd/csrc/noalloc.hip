// hab_render_noalloc: hab_render for callers that cannot allocate memory
// (code under stream capture, serving loops, harnesses that forbid it).
//
// The launch arena (descriptor block, per-view counters, visible-cluster
// lists, tile counts and offsets, survivor keys and boxes, tile lists, work
// items, per-item partial z-keys, queue heads) lives in one static device
// array per GPU instead of a workspace grown with hipMalloc.  Its address
// is looked up once per device while hab_init has that device current; the
// kernels take that address like any other arena base.  The pinned ring the
// descriptor block is staged through and the host planning buffers are
// reserved by hab_init as well, so a call allocates nothing.
#include <hip/hip_runtime.h>

#include <mutex>

#include "runtime.h"

namespace habmi {

// 64 MiB: one 256x256 view of a scene of up to about 1.3M triangles at
// 8-pixel tiles with four list entries per triangle (the largest tuned
// setting), or many views of smaller scenes.
constexpr size_t kNoAllocScratchBytes = 64ull << 20;
constexpr uint32_t kNoAllocMaxViews = 256;
// Descriptor block of kNoAllocMaxViews views: the view records, three
// per-tile-size view lists and prefixes, the control slot (256-byte aligned).
constexpr size_t kNoAllocDescBytes =
    ((sizeof(DView) * kNoAllocMaxViews + 255) & ~size_t(255)) + 6 * ((4 * kNoAllocMaxViews + 255) & ~size_t(255)) + 256;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// The array's address on each device (the name is only a host-side
// stand-in: every device holds its own copy at its own address).
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

hab_status noalloc_setup(hab_context *ctx)
{
    if (ctx->device < 0 || ctx->device >= kMaxDevices) return HAB_ERR_DEVICE;
    {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        void *&p = g_scratch_ptr[ctx->device];
        if (!p) {
            void *q = nullptr;
            if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) {
                (void)hipGetLastError();
                return HAB_ERR_DEVICE;
            }
            p = q;
        }
        ctx->na_scratch = p;
    }
    ctx->na_req.reserve(kNoAllocMaxViews);
    ctx->na_plan.order.reserve(kNoAllocMaxViews);
    ctx->na_ws.device = ctx->device;
    ctx->na_ws.reserve_planning(kNoAllocMaxViews, kNoAllocDescBytes);
    return ctx->na_ws.reserve_staging(kNoAllocDescBytes);
}

}  // namespace habmi

using namespace habmi;

extern "C" hab_status hab_render_noalloc(hab_context *ctx, const hab_scene *scene, const hab_sensor *sensor,
                                         const hab_pose *poses, uint32_t num_poses, uint8_t *out_rgb,
                                         float *out_depth, hipStream_t stream)
{
    if (!ctx || !scene || !sensor || (!poses && num_poses)) return HAB_ERR_INVALID_ARG;
    if (num_poses == 0) return HAB_OK;
    if (num_poses > kNoAllocMaxViews) return HAB_ERR_CAPACITY;
    hab_status st = validate_sensor(sensor);
    if (st != HAB_OK) return st;
    return guarded([&]() -> hab_status {
        std::vector<ViewReq> &req = ctx->na_req;   // reserved: resize does not allocate
        req.resize(num_poses);
        const size_t px = (size_t)sensor->width * sensor->height;
        for (uint32_t k = 0; k < num_poses; ++k) {
            hab_status s2 = validate_pose(scene, sensor, &poses[k]);
            if (s2 != HAB_OK) return s2;
            ViewReq &r = req[k];
            r.scene = scene;
            r.sensor = *sensor;
            r.pose = poses[k];
            r.rgb = (out_rgb && (sensor->outputs & HAB_OUT_RGB)) ? out_rgb + 3 * px * k : nullptr;
            r.depth = (out_depth && (sensor->outputs & HAB_OUT_DEPTH)) ? out_depth + px * k : nullptr;
            r.tri = nullptr;
            r.sem = nullptr;
            r.noise_seed = k;
        }
        DeviceGuard g(ctx->device);
        if (!g.ok) return HAB_ERR_DEVICE;
        if (!ctx->na_scratch) return HAB_ERR_DEVICE;
        Plan &plan = ctx->na_plan;
        hab_status s3 = build_plan(ctx, ctx->na_ws, req.data(), num_poses, PlanOpts{}, plan, ctx->na_ws.desc);
        if (s3 != HAB_OK) return s3;
        if (plan.arena_bytes > kNoAllocScratchBytes || plan.desc_bytes > kNoAllocDescBytes) return HAB_ERR_CAPACITY;
        return stage_and_launch(ctx, ctx->na_ws, plan, ctx->na_scratch, stream, true);
    });
}
