// HIP kernels of the renderer for gfx950 (CDNA4, wave64).
//
// One launch sequence renders a batch of views (any mix of scenes,
// resolutions and output sets):
//   k_reset      zero the per-view counters and per-tile counters
//   k_setup      per (scene group, triangle): fetch the triangle once, then
//                for every view of the group transform, clip, snap, orient
//                and cull; survivors (key, pixel bbox) are appended to the
//                view's list with wave-level prefix-sum compaction
//   k_bin_count  per survivor, count the screen tiles its bbox touches
//                (wave-aggregated atomics)
//   k_bin_scan   per view, exclusive scan of the tile counts into list
//                offsets; tiles over capacity are marked for the overflow
//                path (lossless)
//   k_bin_scatter per survivor, write its key into each touched tile list
//   k_raster<TS> per (view, tile): stage the tile's triangles through LDS
//                (each lane rebuilds one triangle's edge setup relative to
//                the tile), then every lane owns one pixel and keeps the
//                nearest (largest 1/w, smaller key on ties) in registers:
//                an atomic-free z-test that does not depend on list order;
//                finally the winner is resolved to colour, depth and index.
// The arithmetic that decides coverage and visibility is exact integer
// (edge functions) or one fixed sequence of fp32 operations (the key), so
// the output is the same for every batching, tile size and capacity.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dtypes.h"
#include "kernels.h"
#include "raster_math.h"

#pragma clang fp contract(off)

namespace habmi {

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

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

// Add `inc` to counters[key] for every lane with `has`, one atomic per
// distinct key in the wave.  Returns, per participating lane, the value
// the counter had before the wave's additions plus the lane's rank among
// the lanes with the same key (i.e. a unique slot when inc == 1).
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

__device__ __forceinline__ void load_tri(const DView &v, uint32_t t, float P[9], uint32_t vid[3])
{
    const uint32_t *ix = v.idx + 3ull * t;
    vid[0] = ix[0];
    vid[1] = ix[1];
    vid[2] = ix[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float *p = v.pos + 3ull * vid[k];
        P[3 * k + 0] = p[0];
        P[3 * k + 1] = p[1];
        P[3 * k + 2] = p[2];
    }
}

// ------------------------------------------------------------ k_reset
__global__ __launch_bounds__(256) void k_reset(DViewCounters *__restrict__ ctr, uint32_t nviews,
                                               uint32_t *__restrict__ tile_count,
                                               uint32_t *__restrict__ tile_cursor, uint32_t ntiles)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < nviews) {
        ctr[i].surv_count = 0;
        ctr[i].bin_used = 0;
        ctr[i].bbox_tests = 0;
        ctr[i].covered = 0;
    }
    if (i < ntiles) {
        tile_count[i] = 0;
        tile_cursor[i] = 0;
    }
}

// ------------------------------------------------------------ k_setup
__global__ __launch_bounds__(kSetupBlock) void k_setup(const DView *__restrict__ views,
                                                       const DGroup *__restrict__ groups,
                                                       int ngroups, DViewCounters *__restrict__ ctr,
                                                       uint32_t *__restrict__ skey,
                                                       uint2 *__restrict__ sbox,
                                                       uint32_t *__restrict__ err)
{
    int lo = 0, hi = ngroups - 1;
    const int b = (int)blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int)groups[mid].block_start <= b) lo = mid;
        else hi = mid - 1;
    }
    const DGroup G = groups[lo];
    const uint32_t t = (uint32_t)(b - (int)G.block_start) * kSetupBlock + threadIdx.x;
    const bool valid = t < G.T;
    const DView &vg = views[G.first_view];
    float P[9];
    uint32_t vid[3];
    if (valid) {
        load_tri(vg, t, P, vid);
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) P[k] = 0.0f;
    }
    const uint32_t lane = lane_id();
    const unsigned long long lt = lanemask_lt();
    bool rerr = false;

    for (uint32_t k = 0; k < G.num_views; ++k) {
        const uint32_t vi = G.first_view + k;
        const DView &v = views[vi];
        Vtx<0> c0, c1, c2;
        cam_xform(v, P[0], P[1], P[2], c0);
        cam_xform(v, P[3], P[4], P[5], c1);
        cam_xform(v, P[6], P[7], P[8], c2);
        bool s0 = false, s1 = false;
        PixBox b0 = {0, -1, 0, -1}, b1 = {0, -1, 0, -1};
        if (valid) {
            const float zn = v.zn;
            const bool allin = c0.w >= zn && c1.w >= zn && c2.w >= zn;
            const bool anyin = c0.w >= zn || c1.w >= zn || c2.w >= zn;
            bool cull = !anyin;
            if (allin) {
                // Conservative frustum rejection before any division: if all
                // three |Xc fS| exceed (cxS + 4 px)(1 + 2^-16) w on one side,
                // the snapped bbox is at least 3 px outside the viewport
                // (three fp32 roundings cost < 2^-22 relative), so the exact
                // path would cull it too.
                const float Kx = (v.cxS + 1024.0f) * 1.0000152587890625f;
                const float Ky = (v.cyS + 1024.0f) * 1.0000152587890625f;
                const float x0 = c0.x * v.fS, x1 = c1.x * v.fS, x2 = c2.x * v.fS;
                const float y0 = c0.y * v.fS, y1 = c1.y * v.fS, y2 = c2.y * v.fS;
                const float kx0 = Kx * c0.w, kx1 = Kx * c1.w, kx2 = Kx * c2.w;
                const float ky0 = Ky * c0.w, ky1 = Ky * c1.w, ky2 = Ky * c2.w;
                cull = (x0 > kx0 && x1 > kx1 && x2 > kx2) || (x0 < -kx0 && x1 < -kx1 && x2 < -kx2) ||
                       (y0 > ky0 && y1 > ky1 && y2 > ky2) || (y0 < -ky0 && y1 < -ky1 && y2 < -ky2);
            }
            if (!cull) {
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
        }
        const unsigned long long m0 = __ballot(s0), m1 = __ballot(s1);
        if (m0 | m1) {
            const uint32_t tot = (uint32_t)(__popcll(m0) + __popcll(m1));
            const uint32_t pre = (uint32_t)(__popcll(m0 & lt) + __popcll(m1 & lt));
            uint32_t area = 0;
            if (s0) area += (uint32_t)(b0.i1 - b0.i0 + 1) * (uint32_t)(b0.j1 - b0.j0 + 1);
            if (s1) area += (uint32_t)(b1.i1 - b1.i0 + 1) * (uint32_t)(b1.j1 - b1.j0 + 1);
            // two boxes per lane of at most 2^24 pixels each: the wave sum
            // of the low and high halves cannot overflow separately
            const uint32_t alo = wave_sum_u32(area & 0xFFFFu);
            const uint32_t ahi = wave_sum_u32(area >> 16);
            uint32_t base = 0;
            if (lane == 0) {
                base = atomicAdd(&ctr[vi].surv_count, tot);
                atomicAdd(&ctr[vi].bbox_tests, (unsigned long long)alo + ((unsigned long long)ahi << 16));
            }
            base = __shfl(base, 0);
            uint32_t o = v.surv_base + base + pre;
            if (s0) {
                skey[o] = 2u * t;
                sbox[o] = pack_box(b0);
                ++o;
            }
            if (s1) {
                skey[o] = 2u * t + 1u;
                sbox[o] = pack_box(b1);
            }
        }
    }
    if (rerr) atomicOr(err, kErrRange);
}

// ------------------------------------------------------------ binning
// Items of the count/scatter kernels are (view, chunk of kBinChunk
// survivors); every block builds the prefix of chunk counts over the views
// from the device-side survivor counts, then strides over the items.
constexpr uint32_t kBinChunk = kBinBlock * kBinItems;

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
    __shared__ uint32_t pre[kMaxViews];
    __shared__ uint32_t wtot[kBinBlock / 64];
    const uint32_t total = build_item_prefix(ctr, nviews, pre, wtot);
    for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
        const uint32_t vi = find_view(pre, nviews, item);
        const DView &v = views[vi];
        const uint32_t cnt = ctr[vi].surv_count;
        const uint32_t s0 = (item - pre[vi]) * kBinChunk;
        const uint32_t ts = v.ts_log2;
#pragma unroll 1
        for (int r = 0; r < kBinItems; ++r) {
            const uint32_t s = s0 + (uint32_t)r * kBinBlock + threadIdx.x;
            const bool has = s < cnt;
            int tx0 = 0, tx1 = -1, ty0 = 0, ty1 = -1;
            uint32_t key = 0;
            if (has) {
                const uint2 bb = sbox[v.surv_base + s];
                tx0 = (int)(bb.x & 0xFFFFu) >> ts;
                ty0 = (int)(bb.x >> 16) >> ts;
                tx1 = (int)(bb.y & 0xFFFFu) >> ts;
                ty1 = (int)(bb.y >> 16) >> ts;
                if (SCATTER) key = skey[v.surv_base + s];
            }
            const int nx = tx1 - tx0 + 1;
            const int n = has ? nx * (ty1 - ty0 + 1) : 0;
            for (int k = 0; __ballot(k < n); ++k) {
                bool act = k < n;
                uint32_t tile = 0;
                if (act) {
                    const int ty = ty0 + k / nx, tx = tx0 + k % nx;
                    tile = v.tile_base + (uint32_t)ty * v.tiles_x + (uint32_t)tx;
                }
                if (!SCATTER) {
                    wave_aggregated_add(tile_count, tile, act);
                } else {
                    const uint32_t off = act ? tile_off[tile] : kOverflow;
                    act = act && off != kOverflow;
                    const uint32_t slot = wave_aggregated_add(tile_cursor, tile, act);
                    if (act) bins[v.bin_base + off + slot] = key;
                }
            }
        }
    }
}

// Per view: exclusive scan of tile counts into list offsets.  A tile whose
// count exceeds tile_cap, or whose list would end beyond the view's bin
// capacity, is marked kOverflow and rasterised from the full survivor list.
__global__ __launch_bounds__(kScanBlock) void k_bin_scan(const DView *__restrict__ views,
                                                         DViewCounters *__restrict__ ctr,
                                                         const uint32_t *__restrict__ tile_count,
                                                         uint32_t *__restrict__ tile_off)
{
    __shared__ uint32_t wtot[kScanBlock / 64];
    const uint32_t vi = blockIdx.x;
    const DView &v = views[vi];
    const uint32_t n = v.tiles_x * v.tiles_y;
    uint32_t run = 0;
    for (uint32_t base = 0; base < n; base += kScanBlock) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t c = i < n ? tile_count[v.tile_base + i] : 0u;
        const uint32_t e = c <= v.tile_cap ? c : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kScanBlock>(e, wtot, &tot);
        const unsigned long long P = (unsigned long long)run + ex;
        if (i < n) {
            const bool over = c > v.tile_cap || P + e > v.bin_cap;
            tile_off[v.tile_base + i] = (c == 0) ? 0u : (over ? kOverflow : (uint32_t)P);
        }
        run += tot;
    }
    if (threadIdx.x == 0) ctr[vi].bin_used = min(run, v.bin_cap);
}

// ------------------------------------------------------------ k_raster
// LDS record of one (sub-triangle, tile) pair: edge functions relative to
// the tile's first pixel centre, E_k(P, Q) = C_k + dx_k Q - dy_k P with
// (P, Q) the pixel offset from that centre in 1/256 px.
struct alignas(16) LRec {
    uint32_t flags;   // bits 0..15 sub-tiles touched, 16..18 edge k not owned, 19 slow
    int c0, c1, c2;   // fast: C_k - notowned_k; slow: low words of C_k
    int dx0, dx1, dx2;
    int ny0, ny1, ny2; // -dy_k
    uint32_t key;
    float invA;
    float rw0, rw1, rw2;
    uint32_t pad;
};
static_assert(sizeof(LRec) == 64, "LRec");

constexpr uint32_t kSlow = 1u << 19;

__device__ __forceinline__ long long join64(int hi, int lo)
{
    return (long long)(((unsigned long long)(uint32_t)hi << 32) | (unsigned long long)(uint32_t)lo);
}

template <int TS>
__device__ __forceinline__ void build_rec(const DView &v, uint32_t key, int ti0, int tj0, LRec &r,
                                          int hi3[3], bool &rerr)
{
    r.flags = 0;
    const uint32_t t = key >> 1;
    const int sub = (int)(key & 1u);
    float P[9];
    uint32_t vid[3];
    load_tri(v, t, P, vid);
    Vtx<0> c0, c1, c2;
    cam_xform(v, P[0], P[1], P[2], c0);
    cam_xform(v, P[3], P[4], P[5], c1);
    cam_xform(v, P[6], P[7], P[8], c2);
    SVtx<0> a, b, c;
    long long A;
    if (!setup_sub(v, c0, c1, c2, sub, a, b, c, A, rerr)) return;
    const PixBox pb = pix_box(v, a, b, c);
    const int bi0 = max(pb.i0 - ti0, 0), bi1 = min(pb.i1 - ti0, TS - 1);
    const int bj0 = max(pb.j0 - tj0, 0), bj1 = min(pb.j1 - tj0, TS - 1);
    if (bi0 > bi1 || bj0 > bj1) return;
    constexpr int NS = TS / 8;
    uint32_t mask = 0;
    const int sx0 = bi0 >> 3, sx1 = bi1 >> 3, sy0 = bj0 >> 3, sy1 = bj1 >> 3;
#pragma unroll
    for (int sy = 0; sy < NS; ++sy)
#pragma unroll
        for (int sx = 0; sx < NS; ++sx)
            if (sx >= sx0 && sx <= sx1 && sy >= sy0 && sy <= sy1) mask |= 1u << (sy * NS + sx);

    // edge k runs from vertex k+1 to vertex k+2
    const int dx[3] = {c.X - b.X, a.X - c.X, b.X - a.X};
    const int dy[3] = {c.Y - b.Y, a.Y - c.Y, b.Y - a.Y};
    const int ax[3] = {b.X, c.X, a.X};
    const int ay[3] = {b.Y, c.Y, a.Y};
    const long long Ox = 256ll * ti0 + 128, Oy = 256ll * tj0 + 128;
    constexpr long long PM = 256ll * (TS - 1);
    long long C[3];
    uint32_t notown = 0;
    bool fast = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        C[k] = (long long)dx[k] * (Oy - ay[k]) - (long long)dy[k] * (Ox - ax[k]);
        if (!owned(dx[k], dy[k])) notown |= 1u << k;
        const long long qx = (long long)dx[k] * PM, px = -(long long)dy[k] * PM;
        const long long emax = C[k] + (qx > 0 ? qx : 0) + (px > 0 ? px : 0);
        const long long emin = C[k] + (qx < 0 ? qx : 0) + (px < 0 ? px : 0);
        // every pixel value of the tile within +-2^29, so each product term
        // (a difference of two such values) stays within +-2^30: no int32
        // intermediate can overflow
        fast = fast && emax <= (1ll << 29) && emin >= -(1ll << 29) &&
               dx[k] < (1 << 22) && dx[k] > -(1 << 22) && dy[k] < (1 << 22) && dy[k] > -(1 << 22);
    }
    if (fast) {
        r.c0 = (int)(C[0] - (long long)(notown & 1u));
        r.c1 = (int)(C[1] - (long long)((notown >> 1) & 1u));
        r.c2 = (int)(C[2] - (long long)((notown >> 2) & 1u));
    } else {
        r.c0 = (int)(uint32_t)(unsigned long long)C[0];
        r.c1 = (int)(uint32_t)(unsigned long long)C[1];
        r.c2 = (int)(uint32_t)(unsigned long long)C[2];
    }
    hi3[0] = (int)(C[0] >> 32);
    hi3[1] = (int)(C[1] >> 32);
    hi3[2] = (int)(C[2] >> 32);
    r.dx0 = dx[0];
    r.dx1 = dx[1];
    r.dx2 = dx[2];
    r.ny0 = -dy[0];
    r.ny1 = -dy[1];
    r.ny2 = -dy[2];
    r.key = key;
    r.invA = 1.0f / (float)A;
    r.rw0 = a.rw;
    r.rw1 = b.rw;
    r.rw2 = c.rw;
    r.flags = mask | (notown << 16) | (fast ? 0u : kSlow);
}

// Colour, depth and index of the winning sub-triangle at pixel (i, j):
// the winner's setup is rebuilt with colours, its three edge functions at
// the pixel centre give the perspective-correct weights.
__device__ __forceinline__ bool resolve(const DView &v, uint32_t key, int i, int j, uint32_t rgb[3],
                                        float &depth)
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
    const uint32_t k0 = v.col ? v.col[vid[0]] : 0xFFFFFFu;
    const uint32_t k1 = v.col ? v.col[vid[1]] : 0xFFFFFFu;
    const uint32_t k2 = v.col ? v.col[vid[2]] : 0xFFFFFFu;
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
        depth = 0.0f;
        return false;
    }
    const long long px = 256ll * i + 128, py = 256ll * j + 128;
    const long long E0 = edge_at(b.X, b.Y, c.X, c.Y, px, py);
    const long long E1 = edge_at(c.X, c.Y, a.X, a.Y, px, py);
    const long long E2 = edge_at(a.X, a.Y, b.X, b.Y, px, py);
    const float w0 = (float)E0 * a.rw, w1 = (float)E1 * b.rw, w2 = (float)E2 * c.rw;
    const float num = (w0 + w1) + w2;
    const float invA = 1.0f / (float)A;
    const float rho = num * invA;
    depth = 1.0f / rho;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float val = ((w0 * a.a[ch] + w1 * b.a[ch]) + w2 * c.a[ch]) / num;
        val = rintf(val);
        val = fminf(fmaxf(val, 0.0f), 255.0f);
        rgb[ch] = (uint32_t)val;
    }
    return true;
}

template <int TS>
__global__ __launch_bounds__(TS *TS) void k_raster(const DView *__restrict__ views,
                                                   const uint32_t *__restrict__ lview,
                                                   const uint32_t *__restrict__ lpre, uint32_t nl,
                                                   DViewCounters *__restrict__ ctr,
                                                   const uint32_t *__restrict__ skey,
                                                   const uint2 *__restrict__ sbox,
                                                   const uint32_t *__restrict__ tile_count,
                                                   const uint32_t *__restrict__ tile_off,
                                                   const uint32_t *__restrict__ bins,
                                                   uint32_t *__restrict__ err)
{
    constexpr int NT = TS * TS;
    constexpr int NS = TS / 8;
    __shared__ LRec rec[NT];
    __shared__ int rhi[3][NT];

    // block -> (view, tile)
    uint32_t lo = 0, hi = nl - 1;
    const uint32_t blk = blockIdx.x;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (lpre[mid] <= blk) lo = mid;
        else hi = mid - 1;
    }
    const uint32_t vi = lview[lo];
    const DView &v = views[vi];
    const uint32_t tile = blk - lpre[lo];
    const int tx = (int)(tile % v.tiles_x), ty = (int)(tile / v.tiles_x);
    const int ti0 = tx * TS, tj0 = ty * TS;

    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const int sx = (int)(wave % NS), sy = (int)(wave / NS);
    const int li = (int)(lane & 7u), lj = (int)(lane >> 3);
    const int pi = ti0 + sx * 8 + li, pj = tj0 + sy * 8 + lj;
    const int P = 256 * (sx * 8 + li), Q = 256 * (sy * 8 + lj);
    const bool inview = pi < (int)v.W && pj < (int)v.H;
    const unsigned long long inmask = __ballot(inview);
    const uint32_t mybit = 1u << wave;

    const uint32_t tglob = v.tile_base + tile;
    const uint32_t cnt = tile_count[tglob];
    const uint32_t off = tile_off[tglob];
    const bool over = cnt != 0 && off == kOverflow;
    const uint32_t n = over ? ctr[vi].surv_count : cnt;
    const uint32_t *list = bins + v.bin_base + (over ? 0u : off);

    float best_rho = 0.0f;
    uint32_t best_key = kNone;
    uint32_t ncov = 0;
    bool rerr = false;

    for (uint32_t base = 0; base < n; base += NT) {
        const uint32_t e = base + tid;
        LRec r;
        r.flags = 0;
        int h3[3] = {0, 0, 0};
        if (e < n) {
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
            if (go) build_rec<TS>(v, key, ti0, tj0, r, h3, rerr);
        }
        rec[tid] = r;
        rhi[0][tid] = h3[0];
        rhi[1][tid] = h3[1];
        rhi[2][tid] = h3[2];
        __syncthreads();
        const uint32_t m = min((uint32_t)NT, n - base);
        for (uint32_t k = 0; k < m; ++k) {
            const uint32_t fl = __builtin_amdgcn_readfirstlane(rec[k].flags);
            if (!(fl & mybit)) continue;
            const LRec &R = rec[k];
            const uint32_t nt = (fl >> 16) & 7u;
            bool cov;
            float w0, w1, w2;
            if (!(fl & kSlow)) {
                const int F0 = R.c0 + __mul24(R.dx0, Q) + __mul24(R.ny0, P);
                const int F1 = R.c1 + __mul24(R.dx1, Q) + __mul24(R.ny1, P);
                const int F2 = R.c2 + __mul24(R.dx2, Q) + __mul24(R.ny2, P);
                cov = (F0 | F1 | F2) >= 0;
                if (!__ballot(cov)) continue;
                w0 = (float)(F0 + (int)(nt & 1u)) * R.rw0;
                w1 = (float)(F1 + (int)((nt >> 1) & 1u)) * R.rw1;
                w2 = (float)(F2 + (int)(nt >> 2)) * R.rw2;
            } else {
                const long long C0 = join64(rhi[0][k], R.c0);
                const long long C1 = join64(rhi[1][k], R.c1);
                const long long C2 = join64(rhi[2][k], R.c2);
                const long long E0 = C0 + (long long)R.dx0 * Q + (long long)R.ny0 * P;
                const long long E1 = C1 + (long long)R.dx1 * Q + (long long)R.ny1 * P;
                const long long E2 = C2 + (long long)R.dx2 * Q + (long long)R.ny2 * P;
                cov = E0 >= (long long)(nt & 1u) && E1 >= (long long)((nt >> 1) & 1u) &&
                      E2 >= (long long)(nt >> 2);
                if (!__ballot(cov)) continue;
                w0 = (float)E0 * R.rw0;
                w1 = (float)E1 * R.rw1;
                w2 = (float)E2 * R.rw2;
            }
            const float num = (w0 + w1) + w2;
            const float rho = num * R.invA;
            const uint32_t key = R.key;
            ncov += (uint32_t)__popcll(__ballot(cov) & inmask);
            const bool better = cov && (rho > best_rho || (rho == best_rho && key < best_key));
            best_rho = better ? rho : best_rho;
            best_key = better ? key : best_key;
        }
        __syncthreads();
    }
    if (lane == 0 && ncov) atomicAdd(&ctr[vi].covered, (unsigned long long)ncov);
    if (rerr) atomicOr(err, kErrRange);

    if (!inview) return;
    uint32_t rgb[3] = {0, 0, 0};
    float depth = 0.0f;
    if (best_key != kNone && !resolve(v, best_key, pi, pj, rgb, depth)) atomicOr(err, kErrResolve);
    const size_t p = (size_t)pj * v.W + (size_t)pi;
    if (v.rgb) {
        v.rgb[3 * p + 0] = (uint8_t)rgb[0];
        v.rgb[3 * p + 1] = (uint8_t)rgb[1];
        v.rgb[3 * p + 2] = (uint8_t)rgb[2];
    }
    if (v.depth) v.depth[p] = depth;
    if (v.tri) v.tri[p] = best_key == kNone ? kNone : (best_key >> 1);
}

// ------------------------------------------------------------ host side
static inline uint32_t cdiv(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

hipError_t launch_render(const LaunchPlan &L, hipStream_t s)
{
    const uint32_t nreset = L.nviews > L.ntiles ? L.nviews : L.ntiles;
    if (nreset)
        hipLaunchKernelGGL(k_reset, dim3(cdiv(nreset, 256)), dim3(256), 0, s, L.ctr, L.nviews,
                           L.tile_count, L.tile_cursor, L.ntiles);
    if (L.setup_blocks)
        hipLaunchKernelGGL(k_setup, dim3(L.setup_blocks), dim3(kSetupBlock), 0, s, L.views, L.groups,
                           (int)L.ngroups, L.ctr, L.skey, L.sbox, L.err);
    hipLaunchKernelGGL(k_bin<false>, dim3(L.bin_grid), dim3(kBinBlock), 0, s, L.views, L.nviews,
                       L.ctr, L.skey, L.sbox, L.tile_count, L.tile_off, L.tile_cursor, L.bins);
    hipLaunchKernelGGL(k_bin_scan, dim3(L.nviews), dim3(kScanBlock), 0, s, L.views, L.ctr,
                       L.tile_count, L.tile_off);
    hipLaunchKernelGGL(k_bin<true>, dim3(L.bin_grid), dim3(kBinBlock), 0, s, L.views, L.nviews,
                       L.ctr, L.skey, L.sbox, L.tile_count, L.tile_off, L.tile_cursor, L.bins);
    for (int k = 0; k < L.nraster; ++k) {
        const RasterLaunch &R = L.raster[k];
        if (!R.blocks) continue;
        switch (R.ts) {
        case 8:
            hipLaunchKernelGGL(k_raster<8>, dim3(R.blocks), dim3(64), 0, s, L.views, R.lview, R.lpre,
                               R.nl, L.ctr, L.skey, L.sbox, L.tile_count, L.tile_off, L.bins, L.err);
            break;
        case 16:
            hipLaunchKernelGGL(k_raster<16>, dim3(R.blocks), dim3(256), 0, s, L.views, R.lview,
                               R.lpre, R.nl, L.ctr, L.skey, L.sbox, L.tile_count, L.tile_off, L.bins,
                               L.err);
            break;
        case 32:
            hipLaunchKernelGGL(k_raster<32>, dim3(R.blocks), dim3(1024), 0, s, L.views, R.lview,
                               R.lpre, R.nl, L.ctr, L.skey, L.sbox, L.tile_count, L.tile_off, L.bins,
                               L.err);
            break;
        default:
            return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

}  // namespace habmi
