// HIP kernels of the renderer for gfx950 (CDNA4, wave64).
//
// One launch sequence renders a batch of views (any mix of scenes,
// resolutions and output sets):
//   k_reset      zero the per-view, per-tile and work-queue counters
//   k_cull       per (view, 64-triangle cluster): conservative frustum test
//                of the cluster's box; the visible clusters are listed
//   k_setup      per (view, run of visible clusters): fetch each triangle,
//                transform, clip, snap, orient and cull it; survivors (key,
//                pixel bbox) are appended to the view's list with
//                wave-level prefix-sum compaction (the views of a scene are
//                consecutive, so its triangles are re-read from L2/MALL)
//   k_bin<count> per chunk of survivors: LDS histogram of the screen tiles
//                their boxes touch, one global add per touched tile
//   k_bin_scan   per view: exclusive scans of the tile counts (list offsets;
//                tiles over capacity take the lossless overflow path) and of
//                the tiles' segment counts; the (tile, segment) work items
//                are appended to the queue of the view's tile size
//   k_bin<scatter> per chunk of survivors: write each key into every touched
//                tile's list (LDS ranks, one global reservation per tile)
//   k_raster<TS> persistent blocks pull (tile, segment) items from the queue
//                (an atomic counter used for work distribution only).  The
//                segment's triangles are staged through LDS (each lane
//                rebuilds one edge setup relative to the tile, with the
//                pixel blocks its box and edges leave), then the wave lists
//                the (triangle, block) pairs and each step gives every lane
//                group one pair: the group's lanes test that block's pixels
//                and keep the nearest candidate (largest 1/w, smaller key on
//                ties) by an LDS atomic max per pixel; the segment's
//                per-pixel winner goes to scratch
//   k_resolve<TS> per band of 32 x 2 pixels (one wave): merge the segments'
//                winners with the same rule, rebuild the winner, write
//                colour (through LDS, as words), planar depth and index:
//                whole 32-byte sectors.
// Coverage and visibility are decided by exact integer edge functions and
// one fixed sequence of fp32 operations (the key), so outputs do not depend
// on batching, tile size, capacity, segmenting or scheduling order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "dtypes.h"
#include "kernels.h"
#include "raster_math.h"

#pragma clang fp contract(off)

namespace habmi {

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// A value every lane of the wave holds alike, moved to a scalar register so
// that what it indexes is fetched through the scalar cache.
__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ unsigned long long lanemask_lt()
{
    return (1ull << lane_id()) - 1ull;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// Exclusive scan over the block (NT threads, wave64); *total gets the sum.
// wtot: LDS scratch of NT/64 words.  Contains two barriers.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t *wtot, uint32_t *total)
{
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t s = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(s, off);
        if (lane >= (uint32_t)off) s += y;
    }
    if (lane == 63) wtot[wave] = s;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        uint32_t v = wtot[w];
        pre += (w < (int)wave) ? v : 0u;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return pre + s - x;
}

// Add 1 to counters[key] for every lane with `has`, one atomic per distinct
// key in the wave.  Returns, per participating lane, the counter's value
// before the wave's additions plus the lane's rank among the lanes with the
// same key: a unique slot.
__device__ __forceinline__ uint32_t wave_aggregated_add(uint32_t *counters, uint32_t key, bool has)
{
    unsigned long long pending = __ballot(has);
    uint32_t mine = 0;
    const uint32_t lane = lane_id();
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const uint32_t lk = __shfl(key, leader);
        const unsigned long long peers = __ballot(has && key == lk);
        uint32_t base = 0;
        if (lane == (uint32_t)leader) base = atomicAdd(&counters[lk], (uint32_t)__popcll(peers));
        base = __shfl(base, leader);
        if (has && key == lk) mine = base + (uint32_t)__popcll(peers & lanemask_lt());
        pending &= ~peers;
    }
    return mine;
}

__device__ __forceinline__ uint2 pack_box(const PixBox &b)
{
    return make_uint2((uint32_t)b.i0 | ((uint32_t)b.j0 << 16), (uint32_t)b.i1 | ((uint32_t)b.j1 << 16));
}

// A pointer read out of a view record, known to point into device global
// memory: loads through it are global (vector memory only), not flat.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gmem(const T *p)
{
    return (const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gmem_out(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}

// Triangle t's vertex positions: nine consecutive floats of the
// per-triangle copy, independent loads (no dependent index -> position
// load).  With T up to 2^30, 9 t can exceed 32 bits: a 64-bit offset.
__device__ __forceinline__ void load_pos(const DView &v, uint32_t t, float P[9])
{
    const auto *p = gmem(v.tpos) + 9ull * t;
#pragma unroll
    for (int i = 0; i < 9; ++i) P[i] = p[i];
}

// Positions and the vertex indices (for per-vertex attributes).
__device__ __forceinline__ void load_tri(const DView &v, uint32_t t, float P[9], uint32_t vid[3])
{
    const auto *ix = gmem(v.idx) + 3u * t;
    vid[0] = ix[0];
    vid[1] = ix[1];
    vid[2] = ix[2];
    load_pos(v, t, P);
}

// ------------------------------------------------------------ k_reset
__global__ __launch_bounds__(256) void k_reset(DViewCounters *__restrict__ ctr, uint32_t nviews,
                                               uint32_t *__restrict__ tile_count,
                                               uint32_t *__restrict__ tile_cursor, uint32_t ntiles,
                                               DQueue *__restrict__ q)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < nviews) {
        ctr[i].vis_clusters = 0;
        ctr[i].surv_count = 0;
        ctr[i].bin_used = 0;
        ctr[i].bbox_tests = 0;
        ctr[i].covered = 0;
    }
    if (i < ntiles) {
        tile_count[i] = 0;
        tile_cursor[i] = 0;
    }
    if (i < 4) q->total[i] = 0;
    if (i < 3 * kQueues) q->head[i / kQueues][i % kQueues].next = 0;
}

// ------------------------------------------------------------ k_setup
// Survival of sub-triangles 0 and 1 of one triangle in view v, with their
// pixel boxes.  Deterministic: calling it twice gives the same answer.
__device__ __forceinline__ void survive(const DView &v, const float P[9], bool valid, bool &s0,
                                        bool &s1, PixBox &b0, PixBox &b1, bool &rerr)
{
    s0 = s1 = false;
    if (!valid) return;
    Vtx<0> c0, c1, c2;
    cam_xform(v, P[0], P[1], P[2], c0);
    cam_xform(v, P[3], P[4], P[5], c1);
    cam_xform(v, P[6], P[7], P[8], c2);
    const float zn = v.zn;
    const bool allin = c0.w >= zn && c1.w >= zn && c2.w >= zn;
    const bool anyin = c0.w >= zn || c1.w >= zn || c2.w >= zn;
    if (!anyin) return;
    if (allin) {
        // Conservative frustum rejection before any division: if all three
        // |Xc fS| exceed (cxS + 4 px)(1 + 2^-16) w on one side, the snapped
        // bbox is at least 3 px outside the viewport (three fp32 roundings
        // cost < 2^-22 relative), so the exact path would cull it too.
        const float Kx = (v.cxS + 1024.0f) * 1.0000152587890625f;
        const float Ky = (v.cyS + 1024.0f) * 1.0000152587890625f;
        const float x0 = c0.x * v.fS, x1 = c1.x * v.fS, x2 = c2.x * v.fS;
        const float y0 = c0.y * v.fS, y1 = c1.y * v.fS, y2 = c2.y * v.fS;
        const float kx0 = Kx * c0.w, kx1 = Kx * c1.w, kx2 = Kx * c2.w;
        const float ky0 = Ky * c0.w, ky1 = Ky * c1.w, ky2 = Ky * c2.w;
        if ((x0 > kx0 && x1 > kx1 && x2 > kx2) || (x0 < -kx0 && x1 < -kx1 && x2 < -kx2) ||
            (y0 > ky0 && y1 > ky1 && y2 > ky2) || (y0 < -ky0 && y1 < -ky1 && y2 < -ky2))
            return;
    }
    SVtx<0> a, bb, c;
    long long A;
    if (setup_sub(v, c0, c1, c2, 0, a, bb, c, A, rerr)) {
        b0 = pix_box(v, a, bb, c);
        s0 = b0.i0 <= b0.i1 && b0.j0 <= b0.j1;
    }
    if (!allin && setup_sub(v, c0, c1, c2, 1, a, bb, c, A, rerr)) {
        b1 = pix_box(v, a, bb, c);
        s1 = b1.i0 <= b1.i1 && b1.j0 <= b1.j1;
    }
}

// Conservative frustum test of a 64-triangle cluster's bounding box for
// view v, in fp64 over the box's eight corners.  The box counts as outside
// only when all corners lie beyond one side plane of the per-vertex
// rejection in `survive` by a margin (fS + K) 2^-18 |d|_1 that exceeds that
// test's fp32 error (< 2^-20 |d|_1 per camera coordinate), or all lie in
// front of the near plane by 2^-18 |d|_1: then every vertex of every
// triangle in the box fails in the same way, each triangle (and each
// near-clipped piece, a convex combination of its vertices) is culled by
// the exact path, and skipping the cluster changes nothing.
__device__ __forceinline__ bool box_outside(const DView &v, float4 mn, float4 mx)
{
    const double fS = (double)v.fS;
    const double Kx = (double)((v.cxS + 1024.0f) * 1.0000152587890625f);
    const double Ky = (double)((v.cyS + 1024.0f) * 1.0000152587890625f);
    double X[8], Y[8], W[8], l1 = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const double dx = (double)((c & 1) ? mx.x : mn.x) - (double)v.p[0];
        const double dy = (double)((c & 2) ? mx.y : mn.y) - (double)v.p[1];
        const double dz = (double)((c & 4) ? mx.z : mn.z) - (double)v.p[2];
        X[c] = (double)v.R[0] * dx + (double)v.R[3] * dy + (double)v.R[6] * dz;
        Y[c] = (double)v.R[1] * dx + (double)v.R[4] * dy + (double)v.R[7] * dz;
        W[c] = -((double)v.R[2] * dx + (double)v.R[5] * dy + (double)v.R[8] * dz);
        l1 = fmax(l1, fabs(dx) + fabs(dy) + fabs(dz));
    }
    const double mg = (fS + fmax(Kx, Ky)) * 0x1p-18 * l1, mz = 0x1p-18 * l1;
    bool r = true, l = true, u = true, d = true, n = true;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        r = r && X[c] * fS - Kx * W[c] > mg;
        l = l && -X[c] * fS - Kx * W[c] > mg;
        u = u && Y[c] * fS - Ky * W[c] > mg;
        d = d && -Y[c] * fS - Ky * W[c] > mg;
        n = n && W[c] < (double)v.zn - mz;
    }
    return r || l || u || d || n;
}

// Block (x, view): test kCullBlock consecutive 64-triangle clusters of the
// view's scene against the view's frustum, compact the visible ones with a
// block scan and append them to the view's segment of the visible-cluster
// list behind one reservation (their order there is immaterial: nothing
// downstream depends on it).
constexpr int kCullBlock = 256;

__global__ __launch_bounds__(kCullBlock) void k_cull(const DView *__restrict__ views,
                                                     DViewCounters *__restrict__ ctr,
                                                     uint32_t *__restrict__ vis_clusters)
{
    __shared__ uint32_t wtot[kCullBlock / 64];
    __shared__ uint32_t sbase;
    const uint32_t vi = blockIdx.y;
    const DView &v = views[vi];
    const uint32_t ncl = (v.T + kCluster - 1) / kCluster;
    const uint32_t c0 = blockIdx.x * kCullBlock;
    if (c0 >= ncl) return;
    const uint32_t c = c0 + threadIdx.x;
    bool vis = c < ncl;
    if (vis && v.cbox) {
        const auto *b = gmem(reinterpret_cast<const float *>(v.cbox)) + 8ull * c;
        vis = !box_outside(v, make_float4(b[0], b[1], b[2], b[3]), make_float4(b[4], b[5], b[6], b[7]));
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan<kCullBlock>(vis ? 1u : 0u, wtot, &tot);
    if (threadIdx.x == 0) sbase = tot ? atomicAdd(&ctr[vi].vis_clusters, tot) : 0u;
    __syncthreads();
    if (vis) vis_clusters[v.pair_base + sbase + ex] = c;
}

// Work items of k_setup: (view, run of kRun visible clusters).  Each block
// builds the prefix of item counts over the views in LDS; each wave then
// takes a contiguous range of items.  A wave sets up one triangle of each
// of the run's clusters per lane (independent loads in flight together),
// appends the survivors (key, box) to its LDS buffer, and copies the buffer
// out behind one slot reservation when the view changes or the buffer is
// full: device-wide atomics, not the arithmetic, bound this stage.
constexpr uint32_t kRun = 4;
constexpr uint32_t kSetupBuf = 2 * kRun * kCluster;   // survivors one wave buffers in LDS

// 5 waves per SIMD (at most 96 VGPRs; 85 used, none spilled): the four
// clusters' loads per lane are in flight together, and at 6 waves the
// spills cost about what the extra wave hides
__global__ __launch_bounds__(kSetupBlock) __attribute__((amdgpu_waves_per_eu(kSetupWavesPerSimd))) void k_setup(const DView *__restrict__ views,
                                                       uint32_t nviews,
                                                       DViewCounters *__restrict__ ctr,
                                                       const uint32_t *__restrict__ vis_clusters,
                                                       uint32_t *__restrict__ skey,
                                                       uint2 *__restrict__ sbox,
                                                       uint32_t *__restrict__ err)
{
    extern __shared__ uint32_t pre[];      // [nviews]: sized at launch
    __shared__ uint32_t bkey[kSetupBlock / 64][kSetupBuf];
    __shared__ uint2 bbox[kSetupBlock / 64][kSetupBuf];
    // the prologue scan's per-wave totals live in the first survivor buffer
    // (dead until the barrier below): 40 KiB per block, four blocks per CU
    uint32_t *const wtot = bkey[0];
    uint32_t total;
    {
        const uint32_t seg = (nviews + kSetupBlock - 1) / kSetupBlock;
        const uint32_t i0 = threadIdx.x * seg, i1 = min(i0 + seg, nviews);
        uint32_t local = 0;
        for (uint32_t i = i0; i < i1; ++i) local += (ctr[i].vis_clusters + kRun - 1) / kRun;
        uint32_t run = block_excl_scan<kSetupBlock>(local, wtot, &total);
        for (uint32_t i = i0; i < i1; ++i) {
            pre[i] = run;
            run += (ctr[i].vis_clusters + kRun - 1) / kRun;
        }
        __syncthreads();
    }
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    const unsigned long long lt = lanemask_lt();
    // each wave takes a contiguous range of items (mostly of one view)
    const uint32_t wave0 = uniform((blockIdx.x * kSetupBlock + threadIdx.x) >> 6);
    const uint32_t nwaves = (gridDim.x * kSetupBlock) >> 6;
    const uint32_t per = (total + nwaves - 1) / nwaves;
    const uint32_t i0 = min(total, wave0 * per), i1 = min(total, i0 + per);
    uint32_t *const wkey = bkey[w];
    uint2 *const wbox = bbox[w];
    uint32_t nbuf = 0, bview = 0;
    unsigned long long barea = 0;   // bbox pixels of the buffered survivors (lane 0)
    bool rerr = false;
    // copy the wave's buffered survivors of view bview out with one atomic
    auto flush = [&]() {
        if (!nbuf) return;
        uint32_t base = 0;
        if (lane == 0) {
            base = atomicAdd(&ctr[bview].surv_count, nbuf);
            if (barea) atomicAdd(&ctr[bview].bbox_tests, barea);
        }
        base = __shfl(base, 0) + views[bview].surv_base;
        __threadfence_block();
        for (uint32_t i = lane; i < nbuf; i += 64) {
            skey[base + i] = wkey[i];
            sbox[base + i] = wbox[i];
        }
        __threadfence_block();
        nbuf = 0;
        barea = 0;
    };
    for (uint32_t item = i0; item < i1; ++item) {
        uint32_t lo = 0, hi = nviews - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (pre[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        const uint32_t vi = uniform(lo);
        if (vi != bview) {
            flush();
            bview = vi;
        }
        const DView &v = views[vi];
        const uint32_t first = (item - pre[vi]) * kRun;
        const uint32_t nrun = min(kRun, ctr[vi].vis_clusters - first);
        uint32_t t[kRun];
        bool valid[kRun];
        float P[kRun][9];
#pragma unroll
        for (uint32_t j = 0; j < kRun; ++j) {
            t[j] = j < nrun ? vis_clusters[v.pair_base + first + j] * kCluster + lane : 0xFFFFFFFFu;
            valid[j] = j < nrun && t[j] < v.T;
        }
#pragma unroll
        for (uint32_t j = 0; j < kRun; ++j) {
            if (valid[j]) {
                load_pos(v, t[j], P[j]);
            } else {
#pragma unroll
                for (int k = 0; k < 9; ++k) P[j][k] = 0.0f;
            }
        }
        // set up the runs' triangles one cluster at a time, appending the
        // survivors in (cluster, sub, lane) order: only one cluster's boxes
        // are live at once
#pragma unroll
        for (uint32_t j = 0; j < kRun; ++j) {
            bool s0, s1;
            PixBox b0, b1;
            survive(v, P[j], valid[j], s0, s1, b0, b1, rerr);
            const unsigned long long m0 = __ballot(s0), m1 = __ballot(s1);
            const uint32_t c0 = (uint32_t)__popcll(m0), cnt = c0 + (uint32_t)__popcll(m1);
            if (!cnt) continue;
            if (nbuf + cnt > kSetupBuf) flush();   // cnt <= 2 * 64 <= kSetupBuf
            if (v.count_work) {
                uint32_t area = 0;
                if (s0) area += (uint32_t)(b0.i1 - b0.i0 + 1) * (uint32_t)(b0.j1 - b0.j0 + 1);
                if (s1) area += (uint32_t)(b1.i1 - b1.i0 + 1) * (uint32_t)(b1.j1 - b1.j0 + 1);
                // two boxes of at most 2^24 pixels per lane: the two halves
                // of the wave sum cannot overflow
                const uint32_t alo = wave_sum_u32(area & 0xFFFFu);
                const uint32_t ahi = wave_sum_u32(area >> 16);
                barea += (unsigned long long)alo + ((unsigned long long)ahi << 16);
            }
            if (s0) {
                const uint32_t k = nbuf + (uint32_t)__popcll(m0 & lt);
                wkey[k] = 2u * t[j];
                wbox[k] = pack_box(b0);
            }
            if (s1) {
                const uint32_t k = nbuf + c0 + (uint32_t)__popcll(m1 & lt);
                wkey[k] = 2u * t[j] + 1u;
                wbox[k] = pack_box(b1);
            }
            nbuf += cnt;
        }
    }
    flush();
    if (rerr) atomicOr(err, kErrRange);
}

// ------------------------------------------------------------ binning
// Items of the count/scatter kernels are (view, chunk of kBinChunk
// survivors); every block builds the prefix of chunk counts over the views
// from the device-side survivor counts, then strides over the items.
constexpr uint32_t kBinChunk = kBinBlock * kBinItems;
constexpr uint32_t kLdsTiles = 2048;   // views with more tiles bin through global atomics

__device__ __forceinline__ uint32_t build_item_prefix(const DViewCounters *ctr, uint32_t nviews,
                                                      uint32_t *pre, uint32_t *wtot)
{
    const uint32_t seg = (nviews + kBinBlock - 1) / kBinBlock;
    const uint32_t i0 = threadIdx.x * seg, i1 = min(i0 + seg, nviews);
    uint32_t local = 0;
    for (uint32_t i = i0; i < i1; ++i) local += (ctr[i].surv_count + kBinChunk - 1) / kBinChunk;
    uint32_t total;
    uint32_t run = block_excl_scan<kBinBlock>(local, wtot, &total);
    for (uint32_t i = i0; i < i1; ++i) {
        pre[i] = run;
        run += (ctr[i].surv_count + kBinChunk - 1) / kBinChunk;
    }
    __syncthreads();
    return total;
}

// LDS slot of tile i in the per-chunk tile arrays: the low five bits are
// XORed with the next five, a permutation within each aligned run of 32
// slots.  Vertically adjacent tiles (32 per row at 256 px / 8 px tiles) would
// otherwise share an LDS bank, and a wave's boxes touch such columns of tiles
// together; the arrays are cleared up to the next multiple of 32.
__device__ __forceinline__ uint32_t swz(uint32_t i) { return i ^ ((i >> 5) & 31u); }

__device__ __forceinline__ uint32_t find_view(const uint32_t *pre, uint32_t nviews, uint32_t item)
{
    uint32_t lo = 0, hi = nviews - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Tiles [tx0, tx1] x [ty0, ty1] that a survivor's pixel box touches.
struct TileRange {
    int tx0, ty0, tx1, ty1;
};

__device__ __forceinline__ TileRange tile_range(uint2 bb, uint32_t ts)
{
    TileRange r;
    r.tx0 = (int)(bb.x & 0xFFFFu) >> ts;
    r.ty0 = (int)(bb.x >> 16) >> ts;
    r.tx1 = (int)(bb.y & 0xFFFFu) >> ts;
    r.ty1 = (int)(bb.y >> 16) >> ts;
    return r;
}

template <bool SCATTER>
__global__ __launch_bounds__(kBinBlock) void k_bin(const DView *__restrict__ views, uint32_t nviews,
                                                   const DViewCounters *__restrict__ ctr,
                                                   const uint32_t *__restrict__ skey,
                                                   const uint2 *__restrict__ sbox,
                                                   uint32_t *__restrict__ tile_count,
                                                   const uint32_t *__restrict__ tile_off,
                                                   uint32_t *__restrict__ tile_cursor,
                                                   uint32_t *__restrict__ bins)
{
    extern __shared__ uint32_t pre[];      // [nviews]: sized at launch
    __shared__ uint32_t hist[kLdsTiles];   // low 16 bits: count, high 16 bits: rank cursor
    __shared__ uint32_t lbase[SCATTER ? kLdsTiles : 1];
    // the prefix scan's per-wave totals live in the histogram (first
    // written after the scan's closing barrier): 32 KiB per scatter block
    uint32_t *const wtot = hist;
    const uint32_t total = build_item_prefix(ctr, nviews, pre, wtot);
    const uint32_t tid = threadIdx.x;
    for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
        const uint32_t vi = uniform(find_view(pre, nviews, item));
        const DView &v = views[vi];
        const uint32_t cnt = ctr[vi].surv_count;
        const uint32_t s0 = (item - pre[vi]) * kBinChunk;
        // the view's fields in registers: the atomics below may not be
        // assumed to leave the view records alone
        const uint32_t ts = v.ts_log2, tiles_x = v.tiles_x, nt = v.tiles_x * v.tiles_y;
        const uint32_t tile_base = v.tile_base, bin_base = v.bin_base, surv_base = v.surv_base;
        if (nt <= kLdsTiles) {
            for (uint32_t i = tid; i < ((nt + 31u) & ~31u); i += kBinBlock) hist[i] = 0;
            __syncthreads();
            // count this chunk's entries per tile in LDS (at most kBinChunk
            // per tile: fits the 16-bit half)
#pragma unroll 1
            for (int r = 0; r < kBinItems; ++r) {
                const uint32_t s = s0 + (uint32_t)r * kBinBlock + tid;
                if (s >= cnt) break;
                const TileRange R = tile_range(sbox[surv_base + s], ts);
                for (int ty = R.ty0; ty <= R.ty1; ++ty)
                    for (int tx = R.tx0; tx <= R.tx1; ++tx) atomicAdd(&hist[swz((uint32_t)ty * tiles_x + (uint32_t)tx)], 1u);
            }
            __syncthreads();
            // one global operation per touched tile; a thread's tiles are
            // i, i + kBinBlock, ...: their loads and atomics are issued
            // together, not one tile after another
            if (!SCATTER) {
                for (uint32_t i = tid; i < nt; i += kBinBlock) {
                    const uint32_t c = hist[swz(i)] & 0xFFFFu;
                    if (c) atomicAdd(&tile_count[tile_base + i], c);
                }
            } else {
                constexpr int kPer = kLdsTiles / kBinBlock;
                uint32_t c[kPer], off[kPer], got[kPer];
#pragma unroll
                for (int k = 0; k < kPer; ++k) {
                    const uint32_t i = tid + (uint32_t)k * kBinBlock;
                    c[k] = i < nt ? hist[swz(i)] & 0xFFFFu : 0u;
                }
                // list offsets of the tiles this chunk touches only (a chunk
                // of consecutive survivors touches a small part of the view)
#pragma unroll
                for (int k = 0; k < kPer; ++k) {
                    const uint32_t i = tid + (uint32_t)k * kBinBlock;
                    off[k] = c[k] ? tile_off[tile_base + i] : kOverflow;
                }
#pragma unroll
                for (int k = 0; k < kPer; ++k) {
                    const uint32_t i = tid + (uint32_t)k * kBinBlock;
                    got[k] = (c[k] && off[k] != kOverflow) ? atomicAdd(&tile_cursor[tile_base + i], c[k]) : 0u;
                }
#pragma unroll
                for (int k = 0; k < kPer; ++k) {
                    const uint32_t i = tid + (uint32_t)k * kBinBlock;
                    if (c[k]) lbase[swz(i)] = off[k] == kOverflow ? kOverflow : off[k] + got[k];
                }
            }
            if (SCATTER) {
                __syncthreads();
#pragma unroll 1
                for (int r = 0; r < kBinItems; ++r) {
                    const uint32_t s = s0 + (uint32_t)r * kBinBlock + tid;
                    if (s >= cnt) break;
                    const TileRange R = tile_range(sbox[surv_base + s], ts);
                    const uint32_t key = skey[surv_base + s];
                    for (int ty = R.ty0; ty <= R.ty1; ++ty)
                        for (int tx = R.tx0; tx <= R.tx1; ++tx) {
                            const uint32_t tl = (uint32_t)ty * tiles_x + (uint32_t)tx;
                            const uint32_t b = lbase[swz(tl)];
                            if (b == kOverflow) continue;
                            const uint32_t rank = atomicAdd(&hist[swz(tl)], 1u << 16) >> 16;
                            bins[bin_base + b + rank] = key;
                        }
                }
            }
            __syncthreads();
        } else {
            // large views: wave-aggregated global atomics
#pragma unroll 1
            for (int r = 0; r < kBinItems; ++r) {
                const uint32_t s = s0 + (uint32_t)r * kBinBlock + tid;
                const bool has = s < cnt;
                TileRange R = {0, 0, -1, -1};   // empty
                uint32_t key = 0;
                if (has) {
                    R = tile_range(sbox[v.surv_base + s], ts);
                    if (SCATTER) key = skey[v.surv_base + s];
                }
                // every lane walks its box's tiles row by row
                int tx = R.tx0, ty = R.ty0;
                while (__ballot(ty <= R.ty1)) {
                    bool act = ty <= R.ty1;
                    uint32_t tile = 0;
                    if (act) tile = v.tile_base + (uint32_t)ty * v.tiles_x + (uint32_t)tx;
                    if (!SCATTER) {
                        wave_aggregated_add(tile_count, tile, act);
                    } else {
                        const uint32_t off = act ? tile_off[tile] : kOverflow;
                        const bool put = act && off != kOverflow;
                        const uint32_t slot = wave_aggregated_add(tile_cursor, tile, put);
                        if (put) bins[v.bin_base + off + slot] = key;
                    }
                    if (act && ++tx > R.tx1) {
                        tx = R.tx0;
                        ++ty;
                    }
                }
            }
        }
    }
}

__device__ __forceinline__ uint32_t seg_size(uint32_t ts_log2) { return kSegPerTile << (2 * ts_log2); }

// Number of (tile, segment) work items of a tile: none when empty, one for
// an overflow tile (it scans the whole survivor list), else one per
// segment of at most kSegPerTile * TS^2 list entries.
__device__ __forceinline__ uint32_t tile_segments(uint32_t c, uint32_t off, uint32_t ts_log2)
{
    if (c == 0) return 0;
    if (off == kOverflow) return 1;
    const uint32_t S = seg_size(ts_log2);
    return (c + S - 1) / S;
}

// Per view: exclusive scan of tile counts into list offsets.  A tile whose
// count exceeds tile_cap, or whose list would end beyond the view's bin
// capacity, is marked kOverflow.  Then the view's work items are reserved
// in its tile size's queue and written out; tile_item gets each tile's
// first item.
__global__ __launch_bounds__(kScanBlock) void k_bin_scan(const DView *__restrict__ views,
                                                         DViewCounters *__restrict__ ctr,
                                                         const uint32_t *__restrict__ tile_count,
                                                         uint32_t *__restrict__ tile_off,
                                                         uint32_t *__restrict__ tile_item,
                                                         DQueue *__restrict__ q,
                                                         uint2 *__restrict__ items8,
                                                         uint2 *__restrict__ items16,
                                                         uint2 *__restrict__ items32)
{
    __shared__ uint32_t wtot[kScanBlock / 64];
    __shared__ uint32_t sbase;
    const uint32_t vi = blockIdx.x;
    const DView &v = views[vi];
    const uint32_t n = v.tiles_x * v.tiles_y;
    const uint32_t cls = v.ts_log2 - 3;
    uint32_t run = 0, srun = 0;
    for (uint32_t base = 0; base < n; base += kScanBlock) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t c = i < n ? tile_count[v.tile_base + i] : 0u;
        const uint32_t e = c <= v.tile_cap ? c : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kScanBlock>(e, wtot, &tot);
        const unsigned long long P = (unsigned long long)run + ex;
        // a tile with more segments than the item encoding holds also takes
        // the (single-item) overflow path
        const bool over = c > v.tile_cap || P + e > v.bin_cap ||
                          c > (kMaxSegments - 1) * seg_size(v.ts_log2);
        const uint32_t off = (c == 0) ? 0u : (over ? kOverflow : (uint32_t)P);
        const uint32_t ns = tile_segments(c, off, v.ts_log2);
        uint32_t stot;
        const uint32_t sex = block_excl_scan<kScanBlock>(ns, wtot, &stot);
        if (i < n) {
            tile_off[v.tile_base + i] = off;
            tile_item[v.tile_base + i] = srun + sex;
        }
        run += tot;
        srun += stot;
    }
    if (threadIdx.x == 0) {
        ctr[vi].bin_used = min(run, v.bin_cap);
        sbase = srun ? atomicAdd(&q->total[cls], srun) : 0u;
    }
    __syncthreads();
    const uint32_t qb = sbase;
    uint2 *items = cls == 0 ? items8 : cls == 1 ? items16 : items32;
    for (uint32_t i = threadIdx.x; i < n; i += kScanBlock) {
        const uint32_t c = tile_count[v.tile_base + i];
        const uint32_t ns = tile_segments(c, tile_off[v.tile_base + i], v.ts_log2);
        const uint32_t first = qb + tile_item[v.tile_base + i];
        tile_item[v.tile_base + i] = first;
        for (uint32_t sgm = 0; sgm < ns; ++sgm) items[first + sgm] = make_uint2(vi, i | (sgm << 18));
    }
}

// ------------------------------------------------------------ k_raster
// LDS record of one (sub-triangle, tile) pair: edge functions relative to
// the tile's first pixel centre, E_k(P, Q) = C_k + dx_k Q - dy_k P with
// (P, Q) the pixel offset from that centre in 1/256 px.  Everything a visit
// needs for the common (packed) case sits in one 48-byte block laid out as
// three naturally aligned 16-byte words (three LDS loads); unpacked and
// int64 records keep their extra words in a second array.
struct alignas(16) LRec {
    int c0, c1, c2;    // C_k (slow: its low word)
    uint32_t flags;
    int e0, e1, e2;    // packed: (dx_k, -dy_k) as 16-bit pairs; else dx_k
    uint32_t nkey;     // ~key: the low word of the z-key
    float rw0, rw1, rw2, invA;
};
struct alignas(8) LExt {
    int ny0, ny1, ny2; // -dy_k (unpacked records)
    int hi0, hi1, hi2; // slow: high words of C_k
};
static_assert(sizeof(LRec) == 48 && sizeof(LExt) == 24, "LDS records");

// One record as three 16-byte LDS loads, at a byte offset from the array.
__device__ __forceinline__ LRec lds_rec_at(const char *base, uint32_t off)
{
    const uint4 *p = reinterpret_cast<const uint4 *>(base + off);
    const uint4 a = p[0], b = p[1], c = p[2];
    LRec r;
    r.c0 = (int)a.x;
    r.c1 = (int)a.y;
    r.c2 = (int)a.z;
    r.flags = a.w;
    r.e0 = (int)b.x;
    r.e1 = (int)b.y;
    r.e2 = (int)b.z;
    r.nkey = b.w;
    r.rw0 = __uint_as_float(c.x);
    r.rw1 = __uint_as_float(c.y);
    r.rw2 = __uint_as_float(c.z);
    r.invA = __uint_as_float(c.w);
    return r;
}

// flags: byte k (k = 0, 1, 2) is 1 when edge k is not owned (the pixel needs
// E_k > 0; a byte of its own lets a compare read it directly), bit 24 slow
// (int64 edge values), bit 25 packed (every edge delta fits int16)
constexpr uint32_t kSlow = 1u << 24;
constexpr uint32_t kPacked = 1u << 25;

typedef short short2_t __attribute__((ext_vector_type(2)));

// The raster's lanes test their pixels block by block: an 8-pixel tile
// (one wave) is cut into eight blocks of 4 columns x 2 rows, larger tiles
// into 4x4-pixel quarters.  A record carries the mask of the tile's blocks
// (row-major, NX per row) that its pixel box touches: 8, 16 or 64 bits.
template <int TS>
struct Blk {
    static constexpr int WL = 2, HL = TS == 8 ? 1 : 2;   // log2 of the block's width, height
    static constexpr int W = 1 << WL, H = 1 << HL, NX = TS / W, NY = TS / H;
};
template <int TS>
using QMask = typename std::conditional<TS == 32, unsigned long long,
                                        typename std::conditional<TS == 8, uint8_t, uint32_t>::type>::type;

// The bits a raster pair entry carries for block b of a wave's 8 x 8 pixels
// (bx = b % 2, by = b / 2): the block's offset in the packed (Q, P) pair of
// 1/256-pixel coordinates (Q in the low half, P in the high half) and in
// the wave's z-keys (8 bytes per pixel, row-major), both placed so that an
// OR with the lane's own offsets adds them; the record's offset sits in bits
// 12..23 and touches neither.
template <int TS>
__host__ __device__ constexpr uint32_t pair_bits(int b)
{
    using B = Blk<TS>;
    const uint32_t bx = (uint32_t)(b & 1), by = (uint32_t)(b >> 1);
    return (by * B::H * 256u) | ((bx * B::W * 256u) << 16) | ((by * B::H * 8u + bx * B::W) * 8u);
}
template <int TS>
__host__ __device__ constexpr uint32_t pair_bits_all()
{
    uint32_t m = 0;
    for (int b = 0; b < 2 * (8 / Blk<TS>::H); ++b) m |= pair_bits<TS>(b);
    return m;
}
// the z-key offsets are below 512 bytes, the (Q, P) offsets at or above
template <int TS>
constexpr uint32_t kPairZ = pair_bits_all<TS>() & 0x1FFu;
template <int TS>
constexpr uint32_t kPairQP = pair_bits_all<TS>() & ~0x1FFu;
static_assert(kPairZ<8> == 0x1A0u && kPairQP<8> == 0x04000600u, "pair bits, 8-pixel tiles");
static_assert(kPairZ<16> == 0x120u && kPairQP<16> == 0x04000400u, "pair bits, larger tiles");
static_assert(((kPairZ<8> | kPairQP<8>) & 0x00FFF000u) == 0 && ((kPairZ<32> | kPairQP<32>) & 0x00FFF000u) == 0,
              "record offset bits");

template <int TS>
__device__ __forceinline__ bool build_rec(const DView &v, uint32_t key, int ti0, int tj0, LRec &r, LExt &x,
                                          QMask<TS> &qm, bool &rerr)
{
    const uint32_t t = key >> 1;
    const int sub = (int)(key & 1u);
    float P[9];
    load_pos(v, t, P);
    Vtx<0> c0, c1, c2;
    cam_xform(v, P[0], P[1], P[2], c0);
    cam_xform(v, P[3], P[4], P[5], c1);
    cam_xform(v, P[6], P[7], P[8], c2);
    SVtx<0> a, b, c;
    long long A;
    if (c0.w >= v.zn && c1.w >= v.zn && c2.w >= v.zn) {
        // all three vertices in front of the near plane (the common case):
        // clipping returns them unchanged and there is no second
        // sub-triangle, so this is the setup of sub-triangle 0 without the
        // polygon bookkeeping
        if (sub != 0) return false;
        bool ok = snap(v, c0, a);
        ok &= snap(v, c1, b);
        ok &= snap(v, c2, c);
        if (!ok) {
            rerr = true;
            return false;
        }
        A = area2(a, b, c);
        if (A == 0) return false;
        if (A < 0) {
            const SVtx<0> tmp = b;
            b = c;
            c = tmp;
            A = -A;
        }
    } else if (!setup_sub(v, c0, c1, c2, sub, a, b, c, A, rerr)) {
        return false;
    }
    const PixBox pb = pix_box(v, a, b, c);
    const int bi0 = max(pb.i0 - ti0, 0), bi1 = min(pb.i1 - ti0, TS - 1);
    const int bj0 = max(pb.j0 - tj0, 0), bj1 = min(pb.j1 - tj0, TS - 1);
    if (bi0 > bi1 || bj0 > bj1) return false;
    using B = Blk<TS>;
    using Q = QMask<TS>;
    const int qx0 = bi0 >> B::WL, qx1 = bi1 >> B::WL, qy0 = bj0 >> B::HL, qy1 = bj1 >> B::HL;
    const Q row = (Q)(((Q)2 << qx1) - ((Q)1 << qx0));
    qm = 0;
#pragma unroll
    for (int qy = 0; qy < B::NY; ++qy)
        if (qy >= qy0 && qy <= qy1) qm |= row << (qy * B::NX);

    // edge k runs from vertex k+1 to vertex k+2
    const int dx[3] = {c.X - b.X, a.X - c.X, b.X - a.X};
    const int dy[3] = {c.Y - b.Y, a.Y - c.Y, b.Y - a.Y};
    const int ax[3] = {b.X, c.X, a.X};
    const int ay[3] = {b.Y, c.Y, a.Y};
    uint32_t notown = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (!owned(dx[k], dy[k])) notown |= 1u << (8 * k);
    // C_k = E_k at the tile's first pixel centre, as low and high words
    int clo[3], chi[3];
    bool fast = true, packed = true;
    // edge start points relative to that centre (|X| < 2^29: fits int32)
    const int Ox = 256 * ti0 + 128, Oy = 256 * tj0 + 128;
    const int rx[3] = {ax[0] - Ox, ax[1] - Ox, ax[2] - Ox};
    const int ry[3] = {ay[0] - Oy, ay[1] - Oy, ay[2] - Oy};
    constexpr int kNear = 1 << 14;
    const bool small = abs(rx[0]) < kNear && abs(rx[1]) < kNear && abs(rx[2]) < kNear && abs(ry[0]) < kNear &&
                       abs(ry[1]) < kNear && abs(ry[2]) < kNear;
    if (small) {
        // every vertex within 64 px of the tile: |d| < 2^15, 24-bit products,
        // |C| < 2^30, every pixel value of the tile < 2^31 in magnitude:
        // the packed form, without 64-bit arithmetic
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            clo[k] = __mul24(dy[k], rx[k]) - __mul24(dx[k], ry[k]);
            chi[k] = clo[k] >> 31;
        }
    } else {
        constexpr unsigned long long PM = 256ull * (TS - 1);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            // C_k = dy r_x - dx r_y from 32 x 32 -> 64-bit products (|r| < 2^30)
            const long long C = (long long)dy[k] * rx[k] - (long long)dx[k] * ry[k];
            clo[k] = (int)(uint32_t)(unsigned long long)C;
            chi[k] = (int)(C >> 32);
            // the largest and smallest E_k over the tile's pixel centres: C_k
            // plus PM times the positive (negative) parts of dx_k and -dy_k
            // (each part below 2^30 in magnitude, their sum below 2^31)
            const uint32_t up = (uint32_t)max(dx[k], 0) + (uint32_t)(-min(dy[k], 0));
            const uint32_t dn = (uint32_t)(-min(dx[k], 0)) + (uint32_t)max(dy[k], 0);
            const long long emax = C + (long long)((unsigned long long)up * PM);
            const long long emin = C - (long long)((unsigned long long)dn * PM);
            // every pixel value of the tile within +-2^29, so each product
            // term (a difference of two such values) stays within +-2^30: no
            // int32 intermediate can overflow
            fast = fast && emax <= (1ll << 29) && emin >= -(1ll << 29) && dx[k] < (1 << 22) &&
                   dx[k] > -(1 << 22) && dy[k] < (1 << 22) && dy[k] > -(1 << 22);
        }
        packed = fast;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            packed = packed && dx[k] < 32768 && dx[k] > -32768 && dy[k] < 32768 && dy[k] > -32768;
    }
    r.c0 = clo[0];
    r.c1 = clo[1];
    r.c2 = clo[2];
    x.hi0 = chi[0];
    x.hi1 = chi[1];
    x.hi2 = chi[2];
    if (packed) {
        r.e0 = (int)(((uint32_t)dx[0] & 0xFFFFu) | ((uint32_t)(-dy[0]) << 16));
        r.e1 = (int)(((uint32_t)dx[1] & 0xFFFFu) | ((uint32_t)(-dy[1]) << 16));
        r.e2 = (int)(((uint32_t)dx[2] & 0xFFFFu) | ((uint32_t)(-dy[2]) << 16));
    } else {
        r.e0 = dx[0];
        r.e1 = dx[1];
        r.e2 = dx[2];
    }
    x.ny0 = -dy[0];
    x.ny1 = -dy[1];
    x.ny2 = -dy[2];
    if constexpr (TS == 8) {
        // Drop the blocks that hold no pixel centre the triangle can cover:
        // an edge whose largest value over a block's centres is below its
        // threshold (1 if not owned, else 0) excludes the block.  E_k peaks
        // at the block corner that dx_k and -dy_k favour; g_k is that peak
        // for block (0, 0) less the threshold, and moves by dx_k 256 H per
        // block row and by -dy_k 256 W per block column.  A block stays
        // while every such value is >= 0, i.e. while the sign bit of their
        // OR is clear.  Every value is E_k at a pixel centre of the tile,
        // minus 0 or 1: exact in int32 for packed records (|E| < 2^31).
        if (packed) {
            constexpr int PW = 256 * (B::W - 1), QH = 256 * (B::H - 1);
            int g[3], sp[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                g[k] = clo[k] + (dx[k] > 0 ? __mul24(dx[k], QH) : 0) - (dy[k] < 0 ? __mul24(dy[k], PW) : 0) -
                       (int)((notown >> (8 * k)) & 1u);
                sp[k] = dy[k] * (256 * B::W);
            }
            QMask<TS> keep = 0;
#pragma unroll
            for (int qy = 0; qy < B::NY; ++qy) {
#pragma unroll
                for (int qx = 0; qx < B::NX; ++qx) {
                    const int e = (g[0] - qx * sp[0]) | (g[1] - qx * sp[1]) | (g[2] - qx * sp[2]);
                    keep |= (QMask<TS>)((uint32_t)~e >> 31) << (qy * B::NX + qx);
                }
                if (qy + 1 < B::NY) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) g[k] += dx[k] * (256 * B::H);
                }
            }
            qm &= keep;
            if (!qm) return false;
        }
    }
    // (float)A: from int32 when A fits (always for small records), which is
    // the same rounding as the int64 conversion
    float fA;
    if (A == (long long)(int)A) fA = (float)(int)A;
    else fA = (float)A;
    r.invA = recip_rn(fA);
    r.rw0 = a.rw;
    r.rw1 = b.rw;
    r.rw2 = c.rw;
    r.nkey = ~key;
    r.flags = notown | (fast ? 0u : kSlow) | (packed ? kPacked : 0u);
    return true;
}

__device__ __forceinline__ long long join64(int hi, int lo)
{
    return (long long)(((unsigned long long)(uint32_t)hi << 32) | (unsigned long long)(uint32_t)lo);
}

// Colour, depth and index of the winning sub-triangle at pixel (i, j):
// the winner's setup is rebuilt with colours, its three edge functions at
// the pixel centre give the perspective-correct weights.
// Colour of the winner at pixel (i, j): the triangle's setup rebuilt with
// the same arithmetic as the raster's (the depth comes from the winning
// key's 1/w, the same value).
__device__ __forceinline__ bool resolve(const DView &v, uint32_t key, int i, int j, uint32_t rgb[3])
{
    const uint32_t t = key >> 1;
    const int sub = (int)(key & 1u);
    float P[9];
    uint32_t vid[3];
    load_tri(v, t, P, vid);
    Vtx<3> c0, c1, c2;
    cam_xform(v, P[0], P[1], P[2], c0);
    cam_xform(v, P[3], P[4], P[5], c1);
    cam_xform(v, P[6], P[7], P[8], c2);
    const uint32_t k0 = v.col ? gmem(v.col)[vid[0]] : 0xFFFFFFu;
    const uint32_t k1 = v.col ? gmem(v.col)[vid[1]] : 0xFFFFFFu;
    const uint32_t k2 = v.col ? gmem(v.col)[vid[2]] : 0xFFFFFFu;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        c0.a[ch] = (float)unpack_rgb(k0, ch);
        c1.a[ch] = (float)unpack_rgb(k1, ch);
        c2.a[ch] = (float)unpack_rgb(k2, ch);
    }
    SVtx<3> a = {}, b = {}, c = {};
    long long A = 1;
    bool rerr = false;
    if (!setup_sub(v, c0, c1, c2, sub, a, b, c, A, rerr)) {
        // unreachable: the key came from a successful setup of the same
        // arithmetic; report it as a device fault rather than guess
        rgb[0] = rgb[1] = rgb[2] = 0;
        return false;
    }
    const long long px = 256ll * i + 128, py = 256ll * j + 128;
    const long long E0 = edge_at(b.X, b.Y, c.X, c.Y, px, py);
    const long long E1 = edge_at(c.X, c.Y, a.X, a.Y, px, py);
    const long long E2 = edge_at(a.X, a.Y, b.X, b.Y, px, py);
    const float w0 = (float)E0 * a.rw, w1 = (float)E1 * b.rw, w2 = (float)E2 * c.rw;
    const float num = (w0 + w1) + w2;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float val = ((w0 * a.a[ch] + w1 * b.a[ch]) + w2 * c.a[ch]) / num;
        val = rintf(val);
        val = fminf(fmaxf(val, 0.0f), 255.0f);
        rgb[ch] = (uint32_t)val;
    }
    return true;
}

// Textured colour: the texture coordinates ride through the clip and the
// perspective-correct interpolation exactly as colours do (same fp32
// sequence), then a bilinear fetch with texel centres at (k + 1/2) / size,
// coordinates repeating.  For a power-of-two size and |u| size < 2^22,
// u * size - 1/2 and its fraction are exact in fp32, so only the blend's
// rounding differs from an fp64 evaluation.
__device__ __forceinline__ void tex_bilinear(const DView &v, float u, float t, uint32_t rgb[3])
{
    const float x = u * (float)v.tex_w - 0.5f, y = t * (float)v.tex_h - 0.5f;
    const float xf = floorf(x), yf = floorf(y);
    const float fx = x - xf, fy = y - yf;
    const int xi = (int)xf, yi = (int)yf;
    const uint32_t wm = v.tex_w - 1u, hm = v.tex_h - 1u;
    const uint32_t i0 = (uint32_t)xi & wm, i1 = (uint32_t)(xi + 1) & wm;
    const uint32_t r0 = ((uint32_t)yi & hm) * v.tex_w, r1 = ((uint32_t)(yi + 1) & hm) * v.tex_w;
    const auto *tex = gmem(v.tex);
    const uint32_t t00 = tex[r0 + i0], t10 = tex[r0 + i1], t01 = tex[r1 + i0], t11 = tex[r1 + i1];
    const float gx = 1.0f - fx, gy = 1.0f - fy;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float c00 = (float)unpack_rgb(t00, ch), c10 = (float)unpack_rgb(t10, ch);
        const float c01 = (float)unpack_rgb(t01, ch), c11 = (float)unpack_rgb(t11, ch);
        float val = gy * (gx * c00 + fx * c10) + fy * (gx * c01 + fx * c11);
        val = rintf(val);
        rgb[ch] = (uint32_t)fminf(fmaxf(val, 0.0f), 255.0f);
    }
}

// resolve() for a textured scene: the same rebuild of the winner with the
// texture coordinates as its two attributes.
__device__ __forceinline__ bool resolve_tex(const DView &v, uint32_t key, int i, int j,
                                            uint32_t rgb[3])
{
    const uint32_t t = key >> 1;
    const int sub = (int)(key & 1u);
    float P[9];
    uint32_t vid[3];
    load_tri(v, t, P, vid);
    Vtx<2> c0, c1, c2;
    cam_xform(v, P[0], P[1], P[2], c0);
    cam_xform(v, P[3], P[4], P[5], c1);
    cam_xform(v, P[6], P[7], P[8], c2);
    const auto *uv = gmem(v.uv);
    c0.a[0] = uv[2u * vid[0]];
    c0.a[1] = uv[2u * vid[0] + 1u];
    c1.a[0] = uv[2u * vid[1]];
    c1.a[1] = uv[2u * vid[1] + 1u];
    c2.a[0] = uv[2u * vid[2]];
    c2.a[1] = uv[2u * vid[2] + 1u];
    SVtx<2> a = {}, b = {}, c = {};
    long long A = 1;
    bool rerr = false;
    if (!setup_sub(v, c0, c1, c2, sub, a, b, c, A, rerr)) {
        rgb[0] = rgb[1] = rgb[2] = 0;
        return false;
    }
    const long long px = 256ll * i + 128, py = 256ll * j + 128;
    const long long E0 = edge_at(b.X, b.Y, c.X, c.Y, px, py);
    const long long E1 = edge_at(c.X, c.Y, a.X, a.Y, px, py);
    const long long E2 = edge_at(a.X, a.Y, b.X, b.Y, px, py);
    const float w0 = (float)E0 * a.rw, w1 = (float)E1 * b.rw, w2 = (float)E2 * c.rw;
    const float num = (w0 + w1) + w2;
    const float u = ((w0 * a.a[0] + w1 * b.a[0]) + w2 * c.a[0]) / num;
    const float tv = ((w0 * a.a[1] + w1 * b.a[1]) + w2 * c.a[1]) / num;
    tex_bilinear(v, u, tv, rgb);
    return true;
}

// LO: lane-owned pixels with an atomic-free z-test in registers; else
// balanced steps over (record, block) pairs with the z-keys in LDS.
template <int TS, bool LO>
// 6 waves per SIMD: the register budget (80 VGPRs) that lets enough
// waves hide the LDS and staging latency (the LDS of an 8-pixel tile,
// 7.3 KB, allows 22 blocks per CU); a 32-pixel tile's LDS allows 4.
__global__ __launch_bounds__(TS *TS) __attribute__((amdgpu_waves_per_eu(TS == 32 ? 4 : 6))) void k_raster(const DView *__restrict__ views,
                                                   const uint2 *__restrict__ items,
                                                   DQueue *__restrict__ q,
                                                   DViewCounters *__restrict__ ctr,
                                                   const uint32_t *__restrict__ skey,
                                                   const uint2 *__restrict__ sbox,
                                                   const uint32_t *__restrict__ tile_count,
                                                   const uint32_t *__restrict__ tile_off,
                                                   const uint32_t *__restrict__ bins,
                                                   uint2 *__restrict__ partial,
                                                   uint32_t *__restrict__ err)
{
    constexpr int NT = TS * TS;
    constexpr int NS = TS / 8;
    constexpr uint32_t cls = TS == 8 ? 0u : TS == 16 ? 1u : 2u;
    constexpr uint32_t S = kSegPerTile * NT;
    using B = Blk<TS>;
    // a wave's 8x8 pixels hold NL blocks: 2 columns of 8 / H rows
    constexpr int NL = 2 * (8 / B::H);
    using QM = QMask<TS>;
    __shared__ LRec srec[NT];
    __shared__ LExt sext[NT];
    __shared__ QM sqm[NT];
    // lane groups of one block's size; a step gives each group one (record,
    // block) pair
    constexpr uint32_t GS = B::W * B::H, NG = 64 / GS;
    static_assert(NG == NL, "one lane group per block of a wave");
    // per wave, lane-owned pixels: per block, byte offsets in srec of the
    // chunk's records that touch the block ([NL][64]); balanced steps: the
    // chunk's (record, block) pairs, record by record, padded for the last
    // double step's read (zeroed once, so a stale entry is still a record
    // or a pair)
    constexpr uint32_t kList = LO ? NL * 64 : NL * 64 + 2 * NG;
    __shared__ __align__(8) uint32_t slist[NT / 64][kList];
    // per wave, balanced steps: the best z-key of each of its 64 pixels
    // (row-major 8 x 8)
    __shared__ unsigned long long szb[NT / 64][LO ? 1 : 64];
    __shared__ uint32_t s_item;

    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const unsigned long long lt = lanemask_lt();
    for (uint32_t i = lane; i < kList; i += 64) slist[wave][i] = 0;
    const int sx = (int)(wave % NS), sy = (int)(wave / NS);
    // lane-owned pixels: lane (li, lj) of the wave's 8 x 8 pixels, at (P, Q)
    // in 1/256 pixel from the tile's first pixel centre; (Q, P) as a 16-bit
    // pair for the packed edge records (dot2 gives dx Q - dy P)
    const int li = (int)(lane & 7u), lj = (int)(lane >> 3);
    const int P = 256 * (sx * 8 + li), Q = 256 * (sy * 8 + lj);
    const short2_t QP = __builtin_bit_cast(short2_t, (uint32_t)Q | ((uint32_t)P << 16));
    // balanced steps: a lane's place in its group's block: (pxl, pyl); the
    // group's block b (bx = b % 2, by = b / 2 in the wave's 8 x 8 pixels)
    // comes with the pair.  QPl: (Q, P) of that place in block 0 as a
    // 16-bit pair; zl: its byte offset in the wave's z-keys.
    const uint32_t pxl = lane % B::W, pyl = (lane % GS) / B::W;
    const uint32_t QPl = (256u * (uint32_t)(sy * 8 + (int)pyl)) | ((256u * (uint32_t)(sx * 8 + (int)pxl)) << 16);
    const uint32_t zl = (pyl * 8 + pxl) * 8;
    unsigned long long *const zw = &szb[wave][0];
    const uint32_t total = q->total[cls];
    bool rerr = false;

    // nq queues (at most one per block); this block drains queue x, whose
    // k-th grab is item ((k / G) nq + x) G + k % G with G = kQueueGroup:
    // every item belongs to exactly one (queue, grab), in increasing order
    const uint32_t nq = min(kQueues, gridDim.x), x = blockIdx.x % nq;
    for (;;) {
        if (tid == 0) {
            const uint32_t k = atomicAdd(&q->head[cls][x].next, 1u);
            s_item = ((k / kQueueGroup) * nq + x) * kQueueGroup + k % kQueueGroup;
        }
        __syncthreads();
        const uint32_t item = uniform(s_item);
        __syncthreads();
        if (item >= total) break;
        const uint2 it = items[item];
        const uint32_t vi = it.x;
        const uint32_t tile = it.y & 0x3FFFFu, sgm = it.y >> 18;
        const DView &v = views[vi];
        const int tx = (int)(tile % v.tiles_x), ty = (int)(tile / v.tiles_x);
        const int ti0 = tx * TS, tj0 = ty * TS;
        const bool count = v.count_work != 0;
        // lane-owned pixels: the lanes whose pixel is in view
        unsigned long long inmask = 0ull;
        if constexpr (LO) inmask = __ballot(ti0 + sx * 8 + li < (int)v.W && tj0 + sy * 8 + lj < (int)v.H);

        const uint32_t tglob = v.tile_base + tile;
        const uint32_t cnt = tile_count[tglob];
        const uint32_t off = tile_off[tglob];
        const bool over = off == kOverflow;
        const uint32_t begin = over ? 0u : sgm * S;
        const uint32_t end = over ? ctr[vi].surv_count : min(begin + S, cnt);
        const uint32_t *list = bins + v.bin_base + (over ? 0u : off);

        // z-key of the best fragment so far: 1/w bits above the complemented
        // triangle key.  A covered fragment has 1/w > 0 (positive weights,
        // positive twice-area), so one unsigned max orders by largest 1/w,
        // then smaller key; 0 means no fragment.  Lane-owned pixels keep it
        // in the owning lane's registers (atomic-free); balanced steps, where
        // any lane group may test any pixel block, keep it in LDS and merge
        // by atomic max.
        unsigned long long best = 0ull;
        if constexpr (!LO) {
            zw[lane] = 0ull;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
        uint32_t ncov = 0;

        for (uint32_t base = begin; base < end; base += NT) {
            // stage: each thread rebuilds one list entry's edge setup for this tile
            {
                const uint32_t e = base + tid;
                QM qm = 0;
                LRec r;
                LExt rx;
                if (e < end) {
                    bool go = true;
                    uint32_t key;
                    if (over) {
                        const uint2 bb = sbox[v.surv_base + e];
                        const int i0 = (int)(bb.x & 0xFFFFu), j0 = (int)(bb.x >> 16);
                        const int i1 = (int)(bb.y & 0xFFFFu), j1 = (int)(bb.y >> 16);
                        go = i1 >= ti0 && i0 < ti0 + TS && j1 >= tj0 && j0 < tj0 + TS;
                        key = skey[v.surv_base + e];
                    } else {
                        key = list[e];
                    }
                    if (go && !build_rec<TS>(v, key, ti0, tj0, r, rx, qm, rerr)) qm = 0;
                }
                sqm[tid] = qm;
                if (qm) {
                    srec[tid] = r;
                    if (!(r.flags & kPacked)) sext[tid] = rx;
                }
            }
            __syncthreads();
            const uint32_t m = min((uint32_t)NT, end - base);
            if constexpr (LO) {
                // z-test of this lane's pixel against fragment weights w_k where
                // covered (cov) and the wave's coverage ballot cm
                auto zkeep = [&](const LRec &R, bool cov, float w0, float w1, float w2) {
                    const float num = (w0 + w1) + w2;
                    const float rho = num * R.invA;
                    const unsigned long long cand =
                        ((unsigned long long)__float_as_uint(rho) << 32) | (unsigned long long)R.nkey;
                    if (count) ncov += (uint32_t)__popcll(__ballot(cov) & inmask);
                    best = (cov && cand > best) ? cand : best;
                };
                // one step: every active lane tests its pixel against record R
                // (index k) of its block under the top-left rule (an edge not
                // owned needs E > 0)
                auto visit = [&](const LRec &R, uint32_t k, bool act, auto allpk) {
                    const uint32_t fl = R.flags;
                    const int n0 = (int)(fl & 0xFFu), n1 = (int)((fl >> 8) & 0xFFu), n2 = (int)((fl >> 16) & 0xFFu);
                    if (decltype(allpk)::value || !__ballot(act && !(fl & kPacked))) {
                        // every active lane's record is packed
                        const int F0 = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, R.e0), QP, R.c0, false);
                        const int F1 = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, R.e1), QP, R.c1, false);
                        const int F2 = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, R.e2), QP, R.c2, false);
                        const bool cov = act && F0 >= n0 && F1 >= n1 && F2 >= n2;
                        if (!__ballot(cov)) return;
                        zkeep(R, cov, (float)F0 * R.rw0, (float)F1 * R.rw1, (float)F2 * R.rw2);
                        return;
                    }
                    bool cov = false;
                    float w0 = 0.0f, w1 = 0.0f, w2 = 0.0f;
                    if (act && (fl & kPacked)) {
                        const int F0 = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, R.e0), QP, R.c0, false);
                        const int F1 = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, R.e1), QP, R.c1, false);
                        const int F2 = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, R.e2), QP, R.c2, false);
                        cov = F0 >= n0 && F1 >= n1 && F2 >= n2;
                        w0 = (float)F0 * R.rw0;
                        w1 = (float)F1 * R.rw1;
                        w2 = (float)F2 * R.rw2;
                    } else if (act && !(fl & kSlow)) {
                        const LExt &X = sext[k];
                        const int F0 = (int)((uint32_t)R.c0 + (uint32_t)__mul24(R.e0, Q) + (uint32_t)__mul24(X.ny0, P));
                        const int F1 = (int)((uint32_t)R.c1 + (uint32_t)__mul24(R.e1, Q) + (uint32_t)__mul24(X.ny1, P));
                        const int F2 = (int)((uint32_t)R.c2 + (uint32_t)__mul24(R.e2, Q) + (uint32_t)__mul24(X.ny2, P));
                        cov = F0 >= n0 && F1 >= n1 && F2 >= n2;
                        w0 = (float)F0 * R.rw0;
                        w1 = (float)F1 * R.rw1;
                        w2 = (float)F2 * R.rw2;
                    } else if (act) {
                        const LExt &X = sext[k];
                        const long long E0 = join64(X.hi0, R.c0) + (long long)R.e0 * Q + (long long)X.ny0 * P;
                        const long long E1 = join64(X.hi1, R.c1) + (long long)R.e1 * Q + (long long)X.ny1 * P;
                        const long long E2 = join64(X.hi2, R.c2) + (long long)R.e2 * Q + (long long)X.ny2 * P;
                        cov = E0 >= (long long)n0 && E1 >= (long long)n1 && E2 >= (long long)n2;
                        w0 = (float)E0 * R.rw0;
                        w1 = (float)E1 * R.rw1;
                        w2 = (float)E2 * R.rw2;
                    }
                    if (!__ballot(cov)) return;
                    zkeep(R, cov, w0, w1, w2);
                };
                // the wave's NL blocks (8 or 16 lanes each) walk their own lists
                // of records whose box touches them: one step tests up to NL
                // records.  Block b of this wave is bit qb + (b / 2) NX + b % 2
                // of a record's block mask.  Per chunk of 64 records, each
                // block's relevant records are compacted into its LDS list; step
                // i then tests entry i of every block's list.
                const uint32_t qb = (uint32_t)(sy * (8 / B::H) * B::NX + 2 * sx);
                const uint32_t lq = ((lane >> (3 + B::HL)) << 1) | ((lane >> 2) & 1u);
                uint32_t *const wl = &slist[wave][0];
                for (uint32_t g = 0; g < m; g += 64) {
                    const bool in = g + lane < m;
                    const QM qm = in ? sqm[g + lane] : (QM)0;
                    bool rl[NL];
                    unsigned long long mk[NL], any = 0;
#pragma unroll
                    for (int b = 0; b < NL; ++b) {
                        rl[b] = (qm >> (qb + (uint32_t)((b >> 1) * B::NX + (b & 1)))) & 1u;
                        mk[b] = __ballot(rl[b]);
                        any |= mk[b];
                    }
                    if (!any) continue;
                    const uint32_t off = (g + lane) * (uint32_t)sizeof(LRec);
                    bool rel = false;
                    uint32_t nsteps = 0, myc = 0;
#pragma unroll
                    for (int b = 0; b < NL; ++b) {
                        if (rl[b]) wl[b * 64 + __popcll(mk[b] & lt)] = off;
                        rel = rel || rl[b];
                        const uint32_t c = (uint32_t)__popcll(mk[b]);
                        nsteps = max(nsteps, c);
                        myc = lq == (uint32_t)b ? c : myc;
                    }
                    nsteps = uniform(nsteps);
                    // does every record this wave will test have the packed form?
                    const bool allpk = !__ballot(rel && !(srec[g + lane].flags & kPacked));
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    const uint32_t *const myl = wl + lq * 64;
                    const char *const rb = reinterpret_cast<const char *>(srec);
                    if (allpk) {
                        // two steps per list read (one 8-byte LDS load)
                        uint32_t i = 0;
                        for (; i + 1 < nsteps; i += 2) {
                            const uint2 o2 = *reinterpret_cast<const uint2 *>(myl + i);
                            visit(lds_rec_at(rb, o2.x), o2.x / (uint32_t)sizeof(LRec), i < myc, std::true_type());
                            visit(lds_rec_at(rb, o2.y), o2.y / (uint32_t)sizeof(LRec), i + 1 < myc, std::true_type());
                        }
                        if (i < nsteps) {
                            const uint32_t o = myl[i];
                            visit(lds_rec_at(rb, o), o / (uint32_t)sizeof(LRec), i < myc, std::true_type());
                        }
                    } else {
                        for (uint32_t i = 0; i < nsteps; ++i) {
                            const uint32_t o = myl[i];
                            visit(lds_rec_at(rb, o), o / (uint32_t)sizeof(LRec), i < myc, std::false_type());
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                }
            } else {
                // z-test of the pixel of pair entry `en` against fragment weights
                // w_k where covered (cov)
                auto zkeep = [&](const LRec &R, uint32_t en, uint32_t qp, bool cov, float w0, float w1, float w2) {
                    const float num = (w0 + w1) + w2;
                    const float rho = num * R.invA;
                    const unsigned long long cand =
                        ((unsigned long long)__float_as_uint(rho) << 32) | (unsigned long long)R.nkey;
                    if (count) {
                        // pixels outside the view do not count
                        const bool inv = ti0 + (int)(qp >> 24) < (int)v.W && tj0 + (int)((qp & 0xFFFFu) >> 8) < (int)v.H;
                        ncov += (uint32_t)__popcll(__ballot(cov && inv));
                    }
                    if (cov) {
                        unsigned long long *z = reinterpret_cast<unsigned long long *>(
                            reinterpret_cast<char *>(zw) + ((en & kPairZ<TS>) | zl));
                        atomicMax(z, cand);
                    }
                };
                // one step: every active lane tests the pixel its pair entry
                // names against the pair's record under the top-left rule (an
                // edge not owned needs E > 0)
                const char *const rb = reinterpret_cast<const char *>(srec);
                auto visit = [&](uint32_t en, bool act, auto allpk) {
                    const uint32_t off = ((en >> 12) & 0xFFFu) << 4;
                    const LRec R = lds_rec_at(rb, off);
                    const uint32_t qp = (en & kPairQP<TS>) | QPl;
                    const short2_t QPq = __builtin_bit_cast(short2_t, qp);
                    const uint32_t fl = R.flags;
                    const int n0 = (int)(fl & 0xFFu), n1 = (int)((fl >> 8) & 0xFFu), n2 = (int)((fl >> 16) & 0xFFu);
                    if (decltype(allpk)::value || !__ballot(act && !(fl & kPacked))) {
                        // every active lane's record is packed
                        const int F0 = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, R.e0), QPq, R.c0, false);
                        const int F1 = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, R.e1), QPq, R.c1, false);
                        const int F2 = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, R.e2), QPq, R.c2, false);
                        const bool cov = act && F0 >= n0 && F1 >= n1 && F2 >= n2;
                        if (!__ballot(cov)) return;
                        zkeep(R, en, qp, cov, (float)F0 * R.rw0, (float)F1 * R.rw1, (float)F2 * R.rw2);
                        return;
                    }
                    const int Pq = (int)(qp >> 16), Qq = (int)(qp & 0xFFFFu);
                    bool cov = false;
                    float w0 = 0.0f, w1 = 0.0f, w2 = 0.0f;
                    if (act && (fl & kPacked)) {
                        const int F0 = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, R.e0), QPq, R.c0, false);
                        const int F1 = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, R.e1), QPq, R.c1, false);
                        const int F2 = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, R.e2), QPq, R.c2, false);
                        cov = F0 >= n0 && F1 >= n1 && F2 >= n2;
                        w0 = (float)F0 * R.rw0;
                        w1 = (float)F1 * R.rw1;
                        w2 = (float)F2 * R.rw2;
                    } else if (act && !(fl & kSlow)) {
                        const LExt &X = sext[off / (uint32_t)sizeof(LRec)];
                        const int F0 = (int)((uint32_t)R.c0 + (uint32_t)__mul24(R.e0, Qq) + (uint32_t)__mul24(X.ny0, Pq));
                        const int F1 = (int)((uint32_t)R.c1 + (uint32_t)__mul24(R.e1, Qq) + (uint32_t)__mul24(X.ny1, Pq));
                        const int F2 = (int)((uint32_t)R.c2 + (uint32_t)__mul24(R.e2, Qq) + (uint32_t)__mul24(X.ny2, Pq));
                        cov = F0 >= n0 && F1 >= n1 && F2 >= n2;
                        w0 = (float)F0 * R.rw0;
                        w1 = (float)F1 * R.rw1;
                        w2 = (float)F2 * R.rw2;
                    } else if (act) {
                        const LExt &X = sext[off / (uint32_t)sizeof(LRec)];
                        const long long E0 = join64(X.hi0, R.c0) + (long long)R.e0 * Qq + (long long)X.ny0 * Pq;
                        const long long E1 = join64(X.hi1, R.c1) + (long long)R.e1 * Qq + (long long)X.ny1 * Pq;
                        const long long E2 = join64(X.hi2, R.c2) + (long long)R.e2 * Qq + (long long)X.ny2 * Pq;
                        cov = E0 >= (long long)n0 && E1 >= (long long)n1 && E2 >= (long long)n2;
                        w0 = (float)E0 * R.rw0;
                        w1 = (float)E1 * R.rw1;
                        w2 = (float)E2 * R.rw2;
                    }
                    if (!__ballot(cov)) return;
                    zkeep(R, en, qp, cov, w0, w1, w2);
                };
                // Per 64 records, the wave lists the (record, block) pairs of the
                // records whose block mask has its blocks (block b of this wave
                // is bit qb + (b / 2) NX + b % 2 of the mask), record by record;
                // step i gives lane group g pair i NG + g, so every step tests
                // NG pairs whatever blocks they fall in.  A pair entry carries
                // the record's offset in srec (in 16-byte units, bits 12..23)
                // and its block's pixel offsets: for the packed (Q, P) pair and
                // for the z-keys (kPairQP, kPairZ bits).
                const uint32_t qb = (uint32_t)(sy * (8 / B::H) * B::NX + 2 * sx);
                uint32_t *const wl = &slist[wave][0];
                const uint32_t gi = lane / GS;
                for (uint32_t g = 0; g < m; g += 64) {
                    const bool in = g + lane < m;
                    const QM qm = in ? sqm[g + lane] : (QM)0;
                    uint32_t mb = 0;
#pragma unroll
                    for (int b = 0; b < NL; ++b)
                        mb |= (uint32_t)((qm >> (qb + (uint32_t)((b >> 1) * B::NX + (b & 1)))) & 1u) << b;
                    // exclusive prefix of the pair counts over the wave, by bit
                    // planes (a count is at most NL <= 8)
                    const uint32_t np = (uint32_t)__popc(mb);
                    uint32_t pos = 0, tot = 0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const unsigned long long bk = __ballot((np >> k) & 1u);
                        pos += (uint32_t)__popcll(bk & lt) << k;
                        tot += (uint32_t)__popcll(bk) << k;
                    }
                    tot = uniform(tot);
                    if (!tot) continue;
                    const uint32_t eb = ((g + lane) * (uint32_t)(sizeof(LRec) / 16)) << 12;
#pragma unroll
                    for (int b = 0; b < NL; ++b) {
                        if ((mb >> b) & 1u) wl[pos++] = eb | pair_bits<TS>(b);
                    }
                    // does every record this wave will test have the packed form?
                    const bool allpk = !__ballot(mb && !(srec[g + lane].flags & kPacked));
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    uint32_t p = 0;
                    if (allpk) {
                        // two steps per list read (one 8-byte LDS load) while
                        // more than NG pairs remain
                        for (; p + NG < tot; p += 2 * NG) {
                            const uint32_t pi = p + 2 * gi;
                            const uint2 e2 = *reinterpret_cast<const uint2 *>(wl + pi);
                            visit(e2.x, pi < tot, std::true_type());
                            visit(e2.y, pi + 1 < tot, std::true_type());
                        }
                        if (p < tot) visit(wl[p + gi], p + gi < tot, std::true_type());
                    } else {
                        for (; p < tot; p += NG) visit(wl[p + gi], p + gi < tot, std::false_type());
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                }
            }
            __syncthreads();
        }
        if constexpr (!LO) {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            best = zw[lane];
        }
        partial[(size_t)item * NT + tid] = make_uint2((uint32_t)(best >> 32), ~(uint32_t)best);
        if (v.count_work && lane == 0 && ncov) atomicAdd(&ctr[vi].covered, (unsigned long long)ncov);
    }
    if (rerr) atomicOr(err, kErrRange);
}

// Depth noise (the appendix's noise study): a standard normal deviate per
// pixel, added to the inverse depth times the sensor's sigma.  Philox4x64
// with 10 rounds (Salmon, Moraes, Dror and Shaw, SC 2011) keyed by (view
// seed, stream tag), counter (pixel index, 0, 0, 0), so each pixel draws on
// its own, whatever thread renders it; the top 24 bits of the first two
// words feed the Box-Muller transform.
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;   // Weyl key increments
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;
constexpr uint64_t kDepthNoiseTag = 0x6465707468ull;    // "depth"

__device__ __forceinline__ float depth_noise_normal(uint64_t seed, uint64_t pixel)
{
    uint64_t c0 = pixel, c1 = 0, c2 = 0, c3 = 0;
    uint64_t k0 = seed, k1 = kDepthNoiseTag;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
        const uint64_t hi1 = __umul64hi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    const float u1 = (float)((uint32_t)(c0 >> 40) + 1u) * 0x1p-24f;   // (0, 1]
    const float u2 = (float)(uint32_t)(c1 >> 40) * 0x1p-24f;          // [0, 1)
    return sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
}

// Resolve bands: 32 x 2 pixels of one view per wave (one lane per pixel,
// four 8-pixel tiles side by side).  Each lane merges its pixel's segment
// winners (largest 1/w, smaller key on a tie: the same order-free rule) and
// shades it.  A band row is 96 bytes of RGB at a multiple of 96 (three
// whole 32-byte sectors) and 128 bytes of depth, index or instance (one
// whole line): the RGB bytes go through LDS so that the wave stores them as
// words, and every sector the band writes is written once and whole.
constexpr int kBandW = 32, kBandH = 2;
constexpr int kBandThreads = kBandW * kBandH;   // one wave

template <int TS>
__global__ __launch_bounds__(kBandThreads) void k_resolve(const DView *__restrict__ views,
                                                          const uint32_t *__restrict__ lview,
                                                          const uint32_t *__restrict__ bpre, uint32_t nl,
                                                          const uint32_t *__restrict__ tile_count,
                                                          const uint32_t *__restrict__ tile_off,
                                                          const uint32_t *__restrict__ tile_item,
                                                          const uint2 *__restrict__ partial,
                                                          uint32_t *__restrict__ err)
{
    constexpr int NT = TS * TS;
    constexpr int NS = TS / 8;
    __shared__ __align__(16) uint8_t s_rgb[kBandH * kBandW * 3];
    uint32_t lo = 0, hi = nl - 1;
    const uint32_t blk = blockIdx.x;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (bpre[mid] <= blk) lo = mid;
        else hi = mid - 1;
    }
    const uint32_t vi = uniform(lview[uniform(lo)]);
    const DView &v = views[vi];
    const uint32_t W = v.W, H = v.H;
    const uint32_t nbx = (W + kBandW - 1) / kBandW;
    const uint32_t band = blk - bpre[lo];
    const uint32_t x0 = (band % nbx) * kBandW, y0 = (band / nbx) * kBandH;
    const uint32_t lane = lane_id();
    const uint32_t cx = lane % kBandW, cy = lane / kBandW;   // position in the band
    const int pi = (int)(x0 + cx), pj = (int)(y0 + cy);
    const bool in = pi < (int)W && pj < (int)H;
    uint32_t rgb[3] = {0, 0, 0};
    if (in) {
        const uint32_t tile = (uint32_t)(pj / TS) * v.tiles_x + (uint32_t)(pi / TS);
        const uint32_t sub = (uint32_t)(((pj % TS) / 8) * NS + (pi % TS) / 8);
        const uint32_t tglob = v.tile_base + tile;
        const uint32_t ns = tile_segments(tile_count[tglob], tile_off[tglob], v.ts_log2);
        const uint32_t first = tile_item[tglob];
        const uint32_t slot = sub * 64u + (uint32_t)((pj % 8) * 8 + (pi % 8));
        float best_rho = 0.0f;
        uint32_t best_key = kNone;
        for (uint32_t s = 0; s < ns; ++s) {
            const uint2 pr = partial[(size_t)(first + s) * NT + slot];
            const float rho = __uint_as_float(pr.x);
            if (pr.y != kNone && (rho > best_rho || (rho == best_rho && pr.y < best_key))) {
                best_rho = rho;
                best_key = pr.y;
            }
        }
        float depth = 0.0f;
        if (best_key != kNone) {
            // the depth is the reciprocal of the winning key's 1/w (the value
            // a rebuild of the triangle would compute again); colour needs
            // the rebuild
            depth = 1.0f / best_rho;
            if (v.rgb && !(v.tex ? resolve_tex(v, best_key, pi, pj, rgb) : resolve(v, best_key, pi, pj, rgb)))
                atomicOr(err, kErrResolve);
        }
        const size_t p = (size_t)pj * W + (size_t)pi;
        if (v.noise_sigma > 0.0f && best_key != kNone) {
            const float rp = best_rho + v.noise_sigma * depth_noise_normal(v.noise_seed, (uint64_t)p);
            depth = rp > 0.0f ? 1.0f / rp : 0.0f;
        }
        if (v.depth) gmem_out(v.depth)[p] = depth;
        if (v.tri) gmem_out(v.tri)[p] = best_key == kNone ? kNone : (best_key >> 1);
        if (v.sem) gmem_out(v.sem)[p] = best_key == kNone ? kNone : gmem(v.inst)[best_key >> 1];
    }
    if (!v.rgb) return;
    auto *o = gmem_out(v.rgb);
    const uint32_t wpx = min((uint32_t)kBandW, W - x0), rows = min((uint32_t)kBandH, H - y0);
    if ((W % 4u) == 0 && (reinterpret_cast<uintptr_t>(v.rgb) % 4u) == 0) {
        // rows of 3 wpx bytes start on a word (the image does, W and x0 are
        // multiples of 4): stage the band's bytes, store words
        constexpr uint32_t kRowWords = kBandW * 3u / 4u;   // 24
        s_rgb[3 * lane] = (uint8_t)rgb[0];
        s_rgb[3 * lane + 1] = (uint8_t)rgb[1];
        s_rgb[3 * lane + 2] = (uint8_t)rgb[2];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const uint32_t r = lane / kRowWords, d = lane % kRowWords;
        if (lane < kBandH * kRowWords && r < rows && d < wpx * 3u / 4u) {
            auto *dst = reinterpret_cast<__attribute__((address_space(1))) uint32_t *>(
                o + ((size_t)(y0 + r) * W + x0) * 3u);
            dst[d] = reinterpret_cast<const uint32_t *>(s_rgb)[lane];
        }
    } else if (in) {
        auto *q = o + 3 * ((size_t)pj * W + (size_t)pi);
        q[0] = (uint8_t)rgb[0];
        q[1] = (uint8_t)rgb[1];
        q[2] = (uint8_t)rgb[2];
    }
}

// ------------------------------------------------------------ host side
static inline uint32_t cdiv(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

static inline void mark(const LaunchPlan &L, int ev, hipStream_t s)
{
    if (L.prof && ((L.prof_mask >> (ev >> 1)) & 1u)) (void)hipEventRecord(L.prof[ev], s);
}

template <int TS>
static void launch_raster(const LaunchPlan &L, const RasterLaunch &R, hipStream_t s)
{
    if (R.lane_owned)
        hipLaunchKernelGGL((k_raster<TS, true>), dim3(R.grid), dim3(TS * TS), 0, s, L.views, R.items, L.queue,
                           L.ctr, L.skey, L.sbox, L.tile_count, L.tile_off, L.bins, R.partial, L.err);
    else
        hipLaunchKernelGGL((k_raster<TS, false>), dim3(R.grid), dim3(TS * TS), 0, s, L.views, R.items, L.queue,
                           L.ctr, L.skey, L.sbox, L.tile_count, L.tile_off, L.bins, R.partial, L.err);
}

template <int TS>
static void launch_resolve(const LaunchPlan &L, const RasterLaunch &R, hipStream_t s)
{
    hipLaunchKernelGGL(k_resolve<TS>, dim3(R.bands), dim3(kBandThreads), 0, s, L.views, R.lview, R.bpre,
                       R.nl, L.tile_count, L.tile_off, L.tile_item, R.partial, L.err);
}

int raster_blocks_per_cu(int ts, bool lane_owned)
{
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (ts * 2 + (lane_owned ? 1 : 0)) {
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_raster<8, false>, 64, 0); break;
    case 17: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_raster<8, true>, 64, 0); break;
    case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_raster<16, false>, 256, 0); break;
    case 33: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_raster<16, true>, 256, 0); break;
    case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_raster<32, false>, 1024, 0); break;
    case 65: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_raster<32, true>, 1024, 0); break;
    default: break;
    }
    if (e != hipSuccess) (void)hipGetLastError();
    return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_render(const LaunchPlan &L, hipStream_t s)
{
    const uint32_t nreset = L.nviews > L.ntiles ? L.nviews : L.ntiles;
    mark(L, 0, s);
    hipLaunchKernelGGL(k_reset, dim3(cdiv(nreset > 4 ? nreset : 4, 256)), dim3(256), 0, s, L.ctr,
                       L.nviews, L.tile_count, L.tile_cursor, L.ntiles, L.queue);
    mark(L, 1, s);
    mark(L, 2, s);
    hipLaunchKernelGGL(k_cull, dim3(L.cull_blocks, L.nviews), dim3(kCullBlock), 0, s, L.views, L.ctr, L.pairs);
    const size_t pre_bytes = 4u * (size_t)L.nviews;   // the per-view prefix in LDS
    hipLaunchKernelGGL(k_setup, dim3(L.setup_grid), dim3(kSetupBlock), pre_bytes, s, L.views, L.nviews, L.ctr,
                       L.pairs, L.skey, L.sbox, L.err);
    mark(L, 3, s);
    mark(L, 4, s);
    hipLaunchKernelGGL(k_bin<false>, dim3(L.bin_grid), dim3(kBinBlock), pre_bytes, s, L.views, L.nviews,
                       L.ctr, L.skey, L.sbox, L.tile_count, L.tile_off, L.tile_cursor, L.bins);
    mark(L, 5, s);
    mark(L, 6, s);
    hipLaunchKernelGGL(k_bin_scan, dim3(L.nviews), dim3(kScanBlock), 0, s, L.views, L.ctr,
                       L.tile_count, L.tile_off, L.tile_item, L.queue, L.items[0], L.items[1],
                       L.items[2]);
    mark(L, 7, s);
    mark(L, 8, s);
    hipLaunchKernelGGL(k_bin<true>, dim3(L.bin_grid), dim3(kBinBlock), pre_bytes, s, L.views, L.nviews,
                       L.ctr, L.skey, L.sbox, L.tile_count, L.tile_off, L.tile_cursor, L.bins);
    mark(L, 9, s);
    for (int k = 0; k < L.nraster; ++k) {
        const RasterLaunch &R = L.raster[k];
        if (!R.blocks) continue;
        const int ph = R.ts == 8 ? 5 : R.ts == 16 ? 6 : 7;
        mark(L, 2 * ph, s);
        switch (R.ts) {
        case 8: launch_raster<8>(L, R, s); break;
        case 16: launch_raster<16>(L, R, s); break;
        case 32: launch_raster<32>(L, R, s); break;
        default: return hipErrorInvalidValue;
        }
        mark(L, 2 * ph + 1, s);
    }
    mark(L, 2 * kPhaseResolve, s);
    for (int k = 0; k < L.nraster; ++k) {
        const RasterLaunch &R = L.raster[k];
        if (!R.blocks) continue;
        switch (R.ts) {
        case 8: launch_resolve<8>(L, R, s); break;
        case 16: launch_resolve<16>(L, R, s); break;
        case 32: launch_resolve<32>(L, R, s); break;
        default: return hipErrorInvalidValue;
        }
    }
    mark(L, 2 * kPhaseResolve + 1, s);
    return hipGetLastError();
}

// ------------------------------------------------------------ self-check
__global__ __launch_bounds__(256) void k_check_recip(uint32_t lo, uint32_t hi, unsigned long long *count)
{
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    uint32_t bad = 0;
    for (unsigned long long b = lo + (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; b < hi; b += stride) {
        const float x = __uint_as_float((uint32_t)b);
        bad += __float_as_uint(recip_rn(x)) != __float_as_uint(1.0f / x) ? 1u : 0u;
    }
    const uint32_t tot = wave_sum_u32(bad);
    if (lane_id() == 0 && tot) atomicAdd(count, (unsigned long long)tot);
}

hipError_t launch_check_recip(uint32_t lo, uint32_t hi, unsigned long long *count, hipStream_t s)
{
    if (!count || lo >= hi || hi > 0x7F800000u) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_check_recip, dim3(2048), dim3(256), 0, s, lo, hi, count);
    return hipGetLastError();
}

}  // namespace habmi
