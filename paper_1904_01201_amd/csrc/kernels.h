// Launch interface between the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dtypes.h"

namespace habmi {

constexpr uint32_t kMaxViews = 4096;   // views per launch sequence
constexpr uint32_t kSegPerTile = 4;    // a work item covers <= 4 * TS^2 list entries
constexpr uint32_t kMaxSegments = 1u << 14;

// One raster + resolve launch pair: all views of a batch that use the same
// tile size.
struct RasterLaunch {
    int ts;                    // 8, 16 or 32
    const uint32_t *lview;     // [nl] view index (resolve: block -> view)
    const uint32_t *bpre;      // [nl] first resolve band of each view (32 x 2 pixels each)
    uint32_t nl;
    uint32_t blocks;           // total tiles
    uint32_t bands;            // total resolve bands (resolve grid)
    uint32_t grid;             // persistent raster blocks
    bool lane_owned;           // atomic-free lane-owned z-test (else balanced steps, z-keys in LDS)
    uint64_t item_cap;         // work items the scratch below can hold
    uint2 *items;              // [item_cap] (view, tile | segment << 18)
    uint2 *partial;            // [item_cap][TS*TS] per-pixel (1/w bits, key) of each item
};

// Device pointers and sizes of one launch sequence.
struct LaunchPlan {
    const DView *views;
    uint32_t nviews;
    uint32_t cull_blocks;      // cull blocks per view (256 clusters each, for the largest scene)
    uint32_t setup_grid;       // setup grid (waves stride over the visible cluster runs)
    uint32_t *pairs;           // visible clusters, one segment per view
    DViewCounters *ctr;
    uint32_t *skey;
    uint2 *sbox;
    uint32_t *tile_count;
    uint32_t *tile_off;
    uint32_t *tile_cursor;
    uint32_t ntiles;
    uint32_t *bins;
    uint32_t *tile_item;       // first work item of each tile
    DQueue *queue;
    uint2 *items[3];           // per tile size (null when unused)
    uint32_t *err;
    uint32_t bin_grid;
    RasterLaunch raster[3];
    int nraster;
    hipEvent_t *prof;          // null, or kProfEvents events recorded around the kernels
    uint32_t prof_mask;        // phases whose start/stop events are recorded
};

constexpr int kPhaseResolve = 8;
constexpr int kProfPhases = 9;
constexpr int kProfEvents = 2 * kProfPhases;   // start/stop per phase

// Resident k_raster<ts, lane_owned> blocks per compute unit (sizes the
// persistent grid).
int raster_blocks_per_cu(int ts, bool lane_owned);

// Enqueue the whole sequence on stream s.
hipError_t launch_render(const LaunchPlan &L, hipStream_t s);

// Compare recip_rn with the IEEE division 1/x for every float whose bits
// lie in [lo, hi) (lo < hi <= 0x7F800000), adding the number of differing
// results to *count (device memory, one 64-bit word), on stream s.
hipError_t launch_check_recip(uint32_t lo, uint32_t hi, unsigned long long *count, hipStream_t s);

}  // namespace habmi
