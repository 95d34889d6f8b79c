// Launch interface between the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dtypes.h"

namespace habmi {

constexpr uint32_t kMaxViews = 4096;   // views per launch sequence

// One raster launch: all views of a batch that use the same tile size.
struct RasterLaunch {
    int ts;                    // 8, 16 or 32
    const uint32_t *lview;     // [nl] view index
    const uint32_t *lpre;      // [nl] first block of each view (prefix of tile counts)
    uint32_t nl;
    uint32_t blocks;           // total tiles
};

// Device pointers and sizes of one launch sequence.
struct LaunchPlan {
    const DView *views;
    uint32_t nviews;
    const DGroup *groups;
    uint32_t ngroups;
    uint32_t setup_blocks;
    DViewCounters *ctr;
    uint32_t *skey;
    uint2 *sbox;
    uint32_t *tile_count;
    uint32_t *tile_off;
    uint32_t *tile_cursor;
    uint32_t ntiles;
    uint32_t *bins;
    uint32_t *err;
    uint32_t bin_grid;
    RasterLaunch raster[3];
    int nraster;
};

// Enqueue the whole sequence on stream s.
hipError_t launch_render(const LaunchPlan &L, hipStream_t s);

}  // namespace habmi
