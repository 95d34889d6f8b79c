// Plain structures shared by the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace habmi {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kOverflow = 0xFFFFFFFFu;   // tile offset marker: list not stored
constexpr int kSetupBlock = 256;              // threads per block in setup
constexpr int kSetupWavesPerSimd = 5;         // setup's register budget; its grid is one round of it
constexpr int kBinBlock = 256;                // threads per block in count/scatter
constexpr int kBinItems = 4;                  // survivors per thread in count/scatter
constexpr int kScanBlock = 1024;
constexpr int kCluster = 64;                  // triangles per culling cluster (one wave)

// Error bits of the sticky device error word.
constexpr uint32_t kErrRange = 1u;            // a vertex snapped outside |X|,|Y| < 2^29
constexpr uint32_t kErrResolve = 2u;          // a winning key could not be rebuilt

// One view of a launch.  16-byte aligned; 240 bytes.
struct alignas(16) DView {
    float p[3];
    float R[9];                 // row-major world-from-camera
    float fS, cxS, cyS, zn;     // f*256, W*128, H*128, near
    uint32_t W, H;
    uint32_t T;                 // triangles of the scene
    uint32_t ts_log2;           // tile size 8/16/32 -> 3/4/5
    const float *tpos;          // [T][3][3] vertex positions per triangle
    const uint32_t *col;        // [V] packed R | G<<8 | B<<16
    const uint32_t *idx;        // [T][3]
    uint8_t *rgb;               // [H][W][3] or null
    float *depth;               // [H][W] or null
    uint32_t *tri;              // [H][W] or null
    uint32_t tiles_x, tiles_y;
    uint32_t tile_base;         // first entry in the per-tile arrays
    uint32_t surv_base;         // first entry in the survivor arrays
    uint32_t surv_cap;          // 2 T
    uint32_t bin_base;          // first entry in the bin array
    uint32_t bin_cap;           // entries available to this view
    uint32_t tile_cap;          // entries one tile may hold (else overflow)
    uint32_t pair_base;         // first entry of this view's visible-cluster segment
    const float4 *cbox;         // per 64-triangle cluster: (min xyz, -) (max xyz, -)
    uint32_t count_work;        // 1: accumulate bbox tests and covered fragments
    uint32_t pad;
    const uint32_t *inst;       // [T] instance id per triangle (semantic output)
    uint32_t *sem;              // [H][W] or null
    float noise_sigma;          // depth noise in 1/m (0: ideal depth)
    uint32_t pad2;
    uint64_t noise_seed;        // key of the per-pixel depth noise
    const float *uv;            // [V][2] texture coordinates (textured scenes)
    const uint32_t *tex;        // [tex_h][tex_w] packed RGB texels, or null
    uint32_t tex_w, tex_h;      // powers of two
};
static_assert(sizeof(DView) == 240, "DView layout");

// Work queues of the raster stage, per tile size (8, 16, 32): `total`
// items were appended by the scan.  The items are dealt to kQueues queues
// in interleaved groups of kQueueGroup; each queue's head sits on its own
// cache line, so the blocks that drain different queues never contend for
// one atomic.
constexpr uint32_t kQueues = 8;       // one per XCD when blocks are dealt round-robin
constexpr uint32_t kQueueGroup = 4;   // consecutive items that go to one queue
struct alignas(128) DQueueHead {
    uint32_t next;
    uint32_t pad[31];
};
struct alignas(128) DQueue {
    uint32_t total[4];
    uint32_t pad[28];
    DQueueHead head[3][kQueues];
};

// Per-view counters (zeroed at the start of every launch sequence).
// Each view's counters take two cache lines: the first holds what atomics
// update, the second what is written once and read by many waves, so
// those reads never queue behind the atomics (nor do different views'
// atomics meet on one line).
struct alignas(128) DViewCounters {
    uint32_t surv_count;        // survivors appended by setup
    uint32_t bin_used;          // entries the scan assigned
    unsigned long long bbox_tests;
    unsigned long long covered;
    uint32_t pad[26];
    uint32_t vis_clusters;      // clusters that passed the view's frustum test
    uint32_t pad2[31];
};
static_assert(sizeof(DViewCounters) == 256, "counter lines");

}  // namespace habmi
