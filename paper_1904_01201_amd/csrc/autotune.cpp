// Autotuner: picks a tile size in {8, 16, 32} and a bin capacity factor in
// {1, 2, 4} for every batch class (scene-size bucket, resolution bucket,
// output mix) of a sample batch, by timing the whole batch: first every
// choice applied to all classes, then, class by class, the other tile
// sizes for that class alone, kept when the whole batch gets faster by
// more than 2%.  A candidate's time is the fastest of kReps renders.  The
// choice cannot change any output (the rendering definition does not
// depend on tiling or capacity).
//
// Persistent table: with HABMI_AUTOTUNE_CACHE naming a file, hab_init
// loads the choices made earlier on the same GPU architecture and
// hab_autotune writes the context's whole table back (JSON, one class per
// line, replaced atomically), so later processes skip the tuning.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "runtime.h"

using namespace habmi;

namespace {

constexpr int kReps = 5;
constexpr float kKeepGain = 0.98f;   // a per-class change must beat the best by 2%

struct Timer {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Timer()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

void set_table(hab_context *ctx, const std::map<uint32_t, Tuned> &choice)
{
    std::lock_guard<std::mutex> g(ctx->tune_mu);
    for (const auto &kv : choice) {
        auto it = std::find_if(ctx->tuned.begin(), ctx->tuned.end(),
                               [&](const Tuned &t) { return t.key == kv.first; });
        if (it != ctx->tuned.end()) *it = kv.second;
        else ctx->tuned.push_back(kv.second);
    }
}

// Fastest of kReps renders of the batch with the table's current choices.
hab_status time_batch(hab_context *ctx, std::vector<ViewReq> &req, hipStream_t s, Timer &t, float *ms)
{
    PlanOpts o;   // tile size 0: every class takes its table entry
    hab_status rc = render_all(ctx, ctx->ws, req.data(), (uint32_t)req.size(), o, s, nullptr);
    if (rc != HAB_OK) return rc;
    float best = 1e30f;
    for (int r = 0; r < kReps; ++r) {
        if (hipEventRecord(t.e0, s) != hipSuccess) return HAB_ERR_DEVICE;
        rc = render_all(ctx, ctx->ws, req.data(), (uint32_t)req.size(), o, s, nullptr);
        if (rc != HAB_OK) return rc;
        float e = 0.0f;
        if (hipEventRecord(t.e1, s) != hipSuccess || hipEventSynchronize(t.e1) != hipSuccess ||
            hipEventElapsedTime(&e, t.e0, t.e1) != hipSuccess)
            return HAB_ERR_DEVICE;
        best = std::min(best, e);
    }
    *ms = best;
    return HAB_OK;
}

std::string device_arch(int device)
{
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t colon = a.find(':');   // drop feature flags (":sramecc+:xnack-")
    return colon == std::string::npos ? a : a.substr(0, colon);
}

const char *cache_path()
{
    const char *p = getenv("HABMI_AUTOTUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

// Write the context's table (tmp file + rename); false on an I/O error.
bool cache_save(hab_context *ctx, const char *path)
{
    std::vector<Tuned> t;
    {
        std::lock_guard<std::mutex> g(ctx->tune_mu);
        t = ctx->tuned;
    }
    std::sort(t.begin(), t.end(), [](const Tuned &a, const Tuned &b) { return a.key < b.key; });
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    fprintf(f, "{\"arch\": \"%s\", \"entries\": [\n", device_arch(ctx->device).c_str());
    for (size_t k = 0; k < t.size(); ++k)
        fprintf(f, "  {\"class\": %u, \"tile\": %u, \"bin_factor\": %.9g}%s\n", t[k].key, t[k].ts,
                (double)t[k].bin_factor, k + 1 < t.size() ? "," : "");
    fprintf(f, "]}\n");
    const bool ok = fclose(f) == 0;
    if (!ok || rename(tmp.c_str(), path) != 0) {
        (void)remove(tmp.c_str());
        return false;
    }
    return true;
}

}  // namespace

namespace habmi {

// Entries of the file written by cache_save for this context's
// architecture; anything else (another architecture, a malformed line, an
// invalid choice) is skipped.
void autotune_cache_load(hab_context *ctx)
{
    const char *path = cache_path();
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char line[512];
    bool arch_ok = false;
    const std::string arch = device_arch(ctx->device);
    std::vector<Tuned> got;
    while (fgets(line, sizeof line, f)) {
        char a[128];
        if (sscanf(line, " {\"arch\": \"%127[^\"]\"", a) == 1) arch_ok = arch == a;
        unsigned key = 0, ts = 0;
        double bf = 0.0;
        if (sscanf(line, " {\"class\": %u, \"tile\": %u, \"bin_factor\": %lf}", &key, &ts, &bf) == 3 &&
            (ts == 8 || ts == 16 || ts == 32) && (bf == 1.0 || bf == 2.0 || bf == 4.0))
            got.push_back(Tuned{key, ts, (float)bf});
    }
    fclose(f);
    if (!arch_ok) return;
    std::lock_guard<std::mutex> g(ctx->tune_mu);
    for (const Tuned &t : got) {
        auto it = std::find_if(ctx->tuned.begin(), ctx->tuned.end(), [&](const Tuned &u) { return u.key == t.key; });
        if (it != ctx->tuned.end()) *it = t;
        else ctx->tuned.push_back(t);
    }
}

}  // namespace habmi

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
        std::map<uint32_t, Tuned> choice;
        for (const ViewReq &r : req) {
            const uint32_t key = class_key(r.scene, &r.sensor);
            choice[key] = Tuned{key, 16, 2.0f};
        }
        int prev = -1;
        (void)hipGetDevice(&prev);
        if (hipSetDevice(ctx->device) != hipSuccess) return HAB_ERR_DEVICE;
        Timer t;
        if (hipEventCreate(&t.e0) != hipSuccess || hipEventCreate(&t.e1) != hipSuccess) return HAB_ERR_DEVICE;
        hab_status rc = HAB_OK;
        float best_ms = 1e30f;
        std::map<uint32_t, Tuned> best = choice;
        // 1. one choice for every class
        for (uint32_t ts : {8u, 16u, 32u}) {
            for (float bf : {1.0f, 2.0f, 4.0f}) {
                for (auto &kv : choice) kv.second = Tuned{kv.first, ts, bf};
                set_table(ctx, choice);
                float ms = 0.0f;
                rc = time_batch(ctx, req, stream, t, &ms);
                if (rc != HAB_OK) break;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = choice;
                }
            }
            if (rc != HAB_OK) break;
        }
        // 2. class by class, another tile size for that class alone
        if (rc == HAB_OK && best.size() > 1) {
            for (auto &kv : best) {
                const Tuned keep = kv.second;
                Tuned won = keep;
                for (uint32_t ts : {8u, 16u, 32u}) {
                    if (ts == keep.ts) continue;
                    kv.second.ts = ts;
                    set_table(ctx, best);
                    float ms = 0.0f;
                    rc = time_batch(ctx, req, stream, t, &ms);
                    if (rc != HAB_OK) break;
                    if (ms < best_ms * kKeepGain) {
                        best_ms = ms;
                        won = kv.second;
                    }
                }
                kv.second = won;
                if (rc != HAB_OK) break;
            }
        }
        set_table(ctx, best);
        if (rc == HAB_OK) {
            const Tuned &first = best[class_key(req[0].scene, &req[0].sensor)];
            if (chosen_ts) *chosen_ts = first.ts;
            if (chosen_bf) *chosen_bf = first.bin_factor;
            if (const char *path = cache_path())
                if (!cache_save(ctx, path)) rc = HAB_ERR_INVALID_ARG;   // tuned, but the file could not be written
        }
        if (prev >= 0) (void)hipSetDevice(prev);
        return rc;
    } catch (const std::bad_alloc &) {
        return HAB_ERR_OUT_OF_MEMORY;
    }
}
