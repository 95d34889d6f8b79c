// Host runtime of the renderer: context, resident scenes, workspace arena,
// launch planner.  Internal; the public surface is include/hab.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <new>
#include <vector>

#include "../../include/hab.h"
#include "dtypes.h"
#include "kernels.h"

namespace habmi {

#define HAB_HIP(x)                                  \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return HAB_ERR_DEVICE; \
    } while (0)

// Every device and pinned host allocation of the library goes through
// these, so that a test can make an allocation fail on purpose
// (hab_test_fail_alloc) and count what is still allocated
// (hab_test_live_allocations).  false: out of memory (nothing allocated).
bool dev_alloc(void **p, size_t bytes);
void dev_free(void *p);
bool pinned_alloc(void **p, size_t bytes);
void pinned_free(void *p);
void alloc_fail_after(int64_t n);                // n < 0: no injected failure
void alloc_live(uint64_t *count, uint64_t *bytes);

// Make a context's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Run an entry point's body with no exception crossing the C boundary.
template <class F>
hab_status guarded(F &&f)
{
    try {
        return f();
    } catch (const std::bad_alloc &) {
        return HAB_ERR_OUT_OF_MEMORY;
    } catch (...) {
        return HAB_ERR_DEVICE;
    }
}

struct Scene {
    int device = 0;
    float *tpos = nullptr;      // [T][3][3] vertex positions per triangle
    uint32_t *col = nullptr;    // [V] packed
    uint32_t *idx = nullptr;    // [T][3]
    float4 *cbox = nullptr;     // [ceil(T/64)][2] cluster bounding boxes
    uint32_t *inst = nullptr;   // [T] instance id per triangle, or null
    float *uv = nullptr;        // [V][2] texture coordinates, or null
    uint32_t *tex = nullptr;    // [th][tw] packed RGB texels, or null
    uint32_t tw = 0, th = 0;
    uint32_t V = 0, T = 0;
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    uint64_t bytes = 0;
};

// One view after validation (host side).
struct ViewReq {
    const Scene *scene;
    hab_sensor sensor;
    hab_pose pose;
    uint8_t *rgb;
    float *depth;
    uint32_t *tri;
    uint32_t *sem;
    uint64_t noise_seed;
};

struct PlanOpts {
    uint32_t tile_size = 0;     // 0: per-class autotuned choice, else default
    float bin_factor = 0.0f;    // 0: default
    uint32_t tile_cap = 0;      // 0: unlimited
    bool count_work = false;    // accumulate bbox tests / covered fragments
    bool one_sequence = false;  // never split a batch into two launch sequences
    bool lane_owned_z = false;  // the atomic-free lane-owned z-test
};

// Sizes of one launch sequence; used for memory admission as well.
struct Footprint {
    uint64_t desc_bytes = 0;    // descriptors copied from the host
    uint64_t arena_bytes = 0;   // total device scratch incl. descriptors
};

// Device scratch of one launch sequence plus a ring of pinned staging
// buffers for the descriptors.  A workspace is used by one launch sequence
// at a time; `done` orders reuse across streams.
struct Workspace {
    int device = 0;
    void *arena = nullptr;
    size_t cap = 0;
    bool external = false;      // arena owned by someone else (a server pool region): never reallocated
    struct Slot {
        void *host = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
        bool pending = false;
    };
    static constexpr int kSlots = 4;
    Slot slots[kSlots];
    int next = 0;
    hipEvent_t done = nullptr;
    bool has_done = false;
    hipStream_t last_stream = nullptr;
    bool last_valid = false;
    // host-side planning buffers, kept to avoid reallocation
    std::vector<uint8_t> desc;
    std::vector<DView> dv;
    std::vector<uint32_t> lview[3], lpre[3];
    ~Workspace();
    hab_status ensure(size_t bytes);
    hab_status staging(size_t bytes, void **host, int *slot);
    // Pinned slots of at least `bytes` each and their events, made now so
    // that staging_reserved() never allocates.
    hab_status reserve_staging(size_t bytes);
    // The next slot if it holds `bytes` (else HAB_ERR_CAPACITY); waits for
    // the slot's previous copy; allocates nothing.
    hab_status staging_reserved(size_t bytes, void **host, int *slot);
    // Planning buffers with room for n views (reserved, not resized).
    void reserve_planning(uint32_t n, size_t desc_bytes);
};

// Everything one launch sequence needs, laid out in a workspace arena.
// Offsets are relative to the arena base; the descriptor block
// [0, desc_bytes) is copied from pinned host memory before the launch.
struct Plan {
    LaunchPlan L{};
    size_t desc_bytes = 0;
    size_t arena_bytes = 0;
    size_t off_views = 0, off_lview[3] = {0, 0, 0}, off_lpre[3] = {0, 0, 0};
    size_t off_ctr = 0, off_tcount = 0, off_toff = 0, off_tcur = 0;
    size_t off_skey = 0, off_sbox = 0, off_bins = 0;
    size_t off_titem = 0, off_queue = 0, off_items[3] = {0, 0, 0}, off_partial[3] = {0, 0, 0};
    size_t off_pairs = 0;
    size_t off_ctl = 0;              // 16 B control slot in the descriptor block
    std::vector<uint32_t> order;     // sorted position -> caller index
    uint32_t n = 0;
};

// Batches of at least this many views render as two interleaved halves,
// each its own launch sequence, on the caller's stream and a second stream
// of the context: the halves' kernels overlap, so one half's low-occupancy
// phases (the setup's tail, binning) run beside the other's raster.
constexpr uint32_t kSplitViews = 32;

struct Tuned {
    uint32_t key;
    uint32_t ts;
    float bin_factor;
};

}  // namespace habmi

struct hab_context {
    int device = 0;
    habmi::Workspace ws;
    // the second half of a split batch: its workspace and stream, and the
    // events that order it after the caller's stream and back (made on
    // first use)
    habmi::Workspace ws2;
    hipStream_t aux = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    uint32_t *err = nullptr;          // device error word
    std::vector<habmi::Scene *> scenes;
    std::vector<habmi::Tuned> tuned;  // autotune table
    std::mutex tune_mu;
    int cu_count = 256;
    // resident raster blocks per CU: [lane-owned z-test][tile 8/16/32]
    int raster_bpc[2][3] = {{1, 1, 1}, {1, 1, 1}};
    // per-phase event timing (hab_profile_enable)
    struct ProfSet {
        hipEvent_t ev[habmi::kProfEvents];
        uint32_t mask;            // phases recorded in this set
    };
    bool prof_on = false;
    uint32_t prof_phase_mask = 0x1FFu;   // phases timed while profiling is on
    std::vector<ProfSet> prof_sets;
    size_t prof_used = 0;
    // actuation: obstacle sets and the workspace of hab_actuate; the last
    // call's per-agent sets, whose descriptor table and per-agent indices
    // stay in act_ws's arena until a call with other sets (a release
    // clears it)
    std::vector<hab_nav *> navs;
    habmi::Workspace act_ws;
    std::vector<const hab_nav *> act_last;
    size_t act_last_off = 0;
    // hab_render_noalloc: the device's static scratch array (its address on
    // this context's device), planning buffers and pinned staging reserved
    // at hab_init
    void *na_scratch = nullptr;
    habmi::Workspace na_ws;
    habmi::Plan na_plan;
    std::vector<habmi::ViewReq> na_req;
};

struct hab_scene : habmi::Scene {};

namespace habmi {

hab_status validate_sensor(const hab_sensor *s);
void release_navs(hab_context *ctx);   // frees every obstacle set (shutdown)
hab_status validate_pose(const Scene *sc, const hab_sensor *s, const hab_pose *p);
uint32_t class_key(const Scene *sc, const hab_sensor *s);
uint32_t choose_tile(hab_context *ctx, const Scene *sc, const hab_sensor *s, const PlanOpts &o,
                     float *bin_factor);
// Lay out a plan for views [0, n) (validated) in workspace-relative offsets.
hab_status build_plan(hab_context *ctx, Workspace &ws, const ViewReq *v, uint32_t n,
                      const PlanOpts &o, Plan &plan, std::vector<uint8_t> &desc);
// Bind a plan to an arena base address.
void bind_plan(Plan &plan, void *arena, uint32_t *err);
// Plan, stage and enqueue one launch sequence on stream s (n <= kMaxViews,
// footprint checked by the caller).  If stats != NULL, synchronises and
// fills them (caller order).
hab_status render_views(hab_context *ctx, Workspace &ws, const ViewReq *v, uint32_t n,
                        const PlanOpts &o, hipStream_t s, hab_view_stats *stats);
// Copy a planned descriptor block through a pinned staging slot to the
// arena base, bind the plan there and enqueue its launch sequence (no
// profiling events, no statistics).  `reserved`: take only a slot reserved
// beforehand (allocates nothing).
hab_status stage_and_launch(hab_context *ctx, Workspace &ws, Plan &plan, void *arena, hipStream_t s,
                            bool reserved);
// Reserve what hab_render_noalloc uses on ctx's device (called by hab_init
// with that device current): the scratch array's address, planning buffers,
// pinned staging.
hab_status noalloc_setup(hab_context *ctx);
// Load the autotune choices saved in the HABMI_AUTOTUNE_CACHE file for this
// context's GPU architecture (nothing when unset, missing or another one).
void autotune_cache_load(hab_context *ctx);
// Split a request list into launch sequences that fit the limits and run
// them all.
hab_status render_all(hab_context *ctx, Workspace &ws, const ViewReq *v, uint32_t n,
                      const PlanOpts &o, hipStream_t s, hab_view_stats *stats);
// render_all on the context's workspace; a batch of kSplitViews or more
// views as two interleaved halves on s and the context's second stream
// (joined back into s before returning).
hab_status render_split(hab_context *ctx, const ViewReq *v, uint32_t n, const PlanOpts &o, hipStream_t s,
                        hab_view_stats *stats);
// The second stream and its events (once per context).
hab_status ensure_aux(hab_context *ctx);
Footprint footprint(const ViewReq *v, uint32_t n, const PlanOpts &o, hab_context *ctx);
hab_status to_view_req(const hab_view &hv, ViewReq &out);

}  // namespace habmi
