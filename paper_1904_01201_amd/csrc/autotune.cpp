// Autotuner: for each batch class (scene-size bucket, resolution bucket,
// output mix) present in a sample batch, time every tile size in {8, 16,
// 32} and bin capacity factor in {1, 2, 4} on that class's views, and keep
// the fastest in the context's table.  The choice cannot change any output
// (the rendering definition does not depend on tiling or capacity).
#include <algorithm>
#include <map>
#include <new>
#include <vector>

#include "runtime.h"

using namespace habmi;

extern "C" hab_status hab_autotune(hab_context *ctx, const hab_view *views, uint32_t n,
                                   hipStream_t stream, uint32_t *chosen_ts, float *chosen_bf)
{
    if (!ctx || !views || n == 0) return HAB_ERR_INVALID_ARG;
    try {
        std::vector<ViewReq> req(n);
        for (uint32_t k = 0; k < n; ++k) {
            hab_status s = to_view_req(views[k], req[k]);
            if (s != HAB_OK) return s;
        }
        std::map<uint32_t, std::vector<ViewReq>> classes;
        for (const ViewReq &r : req) classes[class_key(r.scene, &r.sensor)].push_back(r);
        int prev = -1;
        (void)hipGetDevice(&prev);
        if (hipSetDevice(ctx->device) != hipSuccess) return HAB_ERR_DEVICE;
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return HAB_ERR_DEVICE;
        const uint32_t first_key = class_key(req[0].scene, &req[0].sensor);
        hab_status rc = HAB_OK;
        for (auto &kv : classes) {
            float best_ms = 1e30f;
            Tuned best{kv.first, 16, 2.0f};
            for (uint32_t ts : {8u, 16u, 32u}) {
                for (float bf : {1.0f, 2.0f, 4.0f}) {
                    PlanOpts o;
                    o.tile_size = ts;
                    o.bin_factor = bf;
                    std::vector<ViewReq> &v = kv.second;
                    rc = render_all(ctx, ctx->ws, v.data(), (uint32_t)v.size(), o, stream, nullptr);
                    if (rc != HAB_OK) break;
                    float tot = 0.0f;
                    const int reps = 3;
                    if (hipEventRecord(e0, stream) != hipSuccess) { rc = HAB_ERR_DEVICE; break; }
                    for (int r = 0; r < reps && rc == HAB_OK; ++r)
                        rc = render_all(ctx, ctx->ws, v.data(), (uint32_t)v.size(), o, stream, nullptr);
                    if (rc != HAB_OK) break;
                    if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                        rc = HAB_ERR_DEVICE;
                        break;
                    }
                    if (hipEventElapsedTime(&tot, e0, e1) != hipSuccess) { rc = HAB_ERR_DEVICE; break; }
                    if (tot < best_ms) {
                        best_ms = tot;
                        best.ts = ts;
                        best.bin_factor = bf;
                    }
                }
                if (rc != HAB_OK) break;
            }
            if (rc != HAB_OK) break;
            {
                std::lock_guard<std::mutex> g(ctx->tune_mu);
                auto it = std::find_if(ctx->tuned.begin(), ctx->tuned.end(),
                                       [&](const Tuned &t) { return t.key == best.key; });
                if (it != ctx->tuned.end()) *it = best;
                else ctx->tuned.push_back(best);
            }
            if (kv.first == first_key) {
                if (chosen_ts) *chosen_ts = best.ts;
                if (chosen_bf) *chosen_bf = best.bin_factor;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (prev >= 0) (void)hipSetDevice(prev);
        return rc;
    } catch (const std::bad_alloc &) {
        return HAB_ERR_OUT_OF_MEMORY;
    }
}
