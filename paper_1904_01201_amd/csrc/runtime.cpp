// Host runtime: validation, workspace arena, launch planning and staging.
#include "runtime.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>

namespace habmi {

static constexpr float kDefaultBinFactor = 2.0f;
static constexpr uint32_t kDefaultTile = 16;
static constexpr uint64_t kIndexLimit = 1ull << 31; // per launch: survivors, bins, tiles

static inline uint32_t cdiv(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

// Stable sort that allocates nothing for short ranges (insertion sort; the
// allocation-free render entry plans at most 256 views); longer ranges use
// std::stable_sort.
template <class It, class Cmp>
static void stable_sort_views(It b, It e, Cmp less)
{
    if (e - b > 256) {
        std::stable_sort(b, e, less);
        return;
    }
    for (It i = b + (e > b ? 1 : 0); i < e; ++i) {
        auto x = *i;
        It j = i;
        for (; j > b && less(x, *(j - 1)); --j) *j = *(j - 1);
        *j = x;
    }
}
static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ---------------------------------------------------------------- allocation
namespace {
std::mutex g_alloc_mu;
int64_t g_fail_after = -1;                      // allocations left before one fails (-1: never)
std::unordered_map<void *, size_t> g_live;      // pointer -> bytes

// After g_fail_after more successes every allocation fails, until reset.
bool inject_failure()
{
    if (g_fail_after < 0) return false;
    if (g_fail_after == 0) return true;
    --g_fail_after;
    return false;
}
}  // namespace

bool dev_alloc(void **p, size_t bytes)
{
    std::lock_guard<std::mutex> g(g_alloc_mu);
    *p = nullptr;
    if (inject_failure()) return false;
    if (hipMalloc(p, std::max<size_t>(bytes, 1)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return false;
    }
    g_live[*p] = bytes;
    return true;
}

void dev_free(void *p)
{
    if (!p) return;
    std::lock_guard<std::mutex> g(g_alloc_mu);
    g_live.erase(p);
    (void)hipFree(p);
}

bool pinned_alloc(void **p, size_t bytes)
{
    std::lock_guard<std::mutex> g(g_alloc_mu);
    *p = nullptr;
    if (inject_failure()) return false;
    if (hipHostMalloc(p, std::max<size_t>(bytes, 1), hipHostMallocDefault) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return false;
    }
    g_live[*p] = bytes;
    return true;
}

void pinned_free(void *p)
{
    if (!p) return;
    std::lock_guard<std::mutex> g(g_alloc_mu);
    g_live.erase(p);
    (void)hipHostFree(p);
}

void alloc_fail_after(int64_t n)
{
    std::lock_guard<std::mutex> g(g_alloc_mu);
    g_fail_after = n;
}

void alloc_live(uint64_t *count, uint64_t *bytes)
{
    std::lock_guard<std::mutex> g(g_alloc_mu);
    uint64_t b = 0;
    for (const auto &e : g_live) b += e.second;
    *count = g_live.size();
    *bytes = b;
}

// ---------------------------------------------------------------- workspace
Workspace::~Workspace()
{
    if (has_done) (void)hipEventSynchronize(done);
    for (auto &s : slots) {
        if (s.pending) (void)hipEventSynchronize(s.ev);
        if (s.host) pinned_free(s.host);
        if (s.ev) (void)hipEventDestroy(s.ev);
    }
    if (arena && !external) dev_free(arena);
    if (done) (void)hipEventDestroy(done);
}

hab_status Workspace::ensure(size_t bytes)
{
    if (!done) HAB_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    if (bytes <= cap) return HAB_OK;
    if (external) return HAB_ERR_CAPACITY;
    if (has_done) HAB_HIP(hipEventSynchronize(done));
    const size_t old = cap;
    if (arena) {
        dev_free(arena);
        arena = nullptr;
        cap = 0;
    }
    size_t want = std::max(bytes, old + old / 2);
    if (!dev_alloc(&arena, want)) {
        if (!dev_alloc(&arena, bytes)) return HAB_ERR_OUT_OF_MEMORY;
        want = bytes;
    }
    cap = want;
    return HAB_OK;
}

hab_status Workspace::staging(size_t bytes, void **host, int *slot)
{
    Slot &s = slots[next];
    *slot = next;
    next = (next + 1) % kSlots;
    if (!s.ev) HAB_HIP(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
    if (s.pending) {
        HAB_HIP(hipEventSynchronize(s.ev));
        s.pending = false;
    }
    if (s.cap < bytes) {
        if (s.host) pinned_free(s.host);
        s.host = nullptr;
        s.cap = 0;
        size_t want = std::max(bytes, (size_t)64 << 10);
        if (!pinned_alloc(&s.host, want)) return HAB_ERR_OUT_OF_MEMORY;
        s.cap = want;
    }
    *host = s.host;
    return HAB_OK;
}

hab_status Workspace::reserve_staging(size_t bytes)
{
    for (int k = 0; k < kSlots; ++k) {
        Slot &s = slots[k];
        if (!s.ev) HAB_HIP(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
        if (s.cap >= bytes) continue;
        if (s.pending) {
            HAB_HIP(hipEventSynchronize(s.ev));
            s.pending = false;
        }
        if (s.host) pinned_free(s.host);
        s.host = nullptr;
        s.cap = 0;
        if (!pinned_alloc(&s.host, bytes)) return HAB_ERR_OUT_OF_MEMORY;
        s.cap = bytes;
    }
    return HAB_OK;
}

hab_status Workspace::staging_reserved(size_t bytes, void **host, int *slot)
{
    Slot &s = slots[next];
    if (!s.ev || !s.host || s.cap < bytes) return HAB_ERR_CAPACITY;
    *slot = next;
    next = (next + 1) % kSlots;
    if (s.pending) {
        HAB_HIP(hipEventSynchronize(s.ev));
        s.pending = false;
    }
    *host = s.host;
    return HAB_OK;
}

void Workspace::reserve_planning(uint32_t n, size_t desc_bytes)
{
    desc.reserve(desc_bytes);
    dv.reserve(n);
    for (int c = 0; c < 3; ++c) {
        lview[c].reserve(n);
        lpre[c].reserve(n);
    }
}

// ---------------------------------------------------------------- validation
static double focal_of(uint32_t W, double hfov_deg)
{
    return (double)W / (2.0 * std::tan(hfov_deg * 3.14159265358979323846 / 360.0));
}

hab_status validate_sensor(const hab_sensor *s)
{
    if (!s) return HAB_ERR_INVALID_ARG;
    if (s->width == 0 || s->height == 0 || s->width > HAB_MAX_DIM || s->height > HAB_MAX_DIM)
        return HAB_ERR_INVALID_ARG;
    if (!(s->hfov_deg > 0.0f && s->hfov_deg < 180.0f)) return HAB_ERR_INVALID_ARG;
    if (!(s->near_m > 0.0f) || !std::isfinite(s->near_m)) return HAB_ERR_INVALID_ARG;
    if (s->outputs == 0 ||
        (s->outputs & ~(uint32_t)(HAB_OUT_RGB | HAB_OUT_DEPTH | HAB_OUT_TRI | HAB_OUT_SEMANTIC)))
        return HAB_ERR_INVALID_ARG;
    if (s->f != (float)focal_of(s->width, s->hfov_deg)) return HAB_ERR_INVALID_ARG;
    if (!(s->depth_noise_sigma >= 0.0f) || !std::isfinite(s->depth_noise_sigma)) return HAB_ERR_INVALID_ARG;
    return HAB_OK;
}

// Static fixed-point domain check: with D the largest distance from the
// camera to a corner of the scene's bounding box, every vertex at w >= near
// projects to at most D f 256 / near + max(W, H) 128 in 1/256 px; requiring
// that below 2^28 keeps |X|, |Y| < 2^29 with a factor-two margin for fp32
// rounding.  The rotation must be orthonormal to 1e-4.
hab_status validate_pose(const Scene *sc, const hab_sensor *s, const hab_pose *p)
{
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(p->position[k])) return HAB_ERR_INVALID_ARG;
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(p->rotation[k])) return HAB_ERR_INVALID_ARG;
    const float *R = p->rotation;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double d = 0.0;
            for (int k = 0; k < 3; ++k) d += (double)R[3 * k + a] * (double)R[3 * k + b];
            if (std::fabs(d - (a == b ? 1.0 : 0.0)) > 1e-4) return HAB_ERR_INVALID_ARG;
        }
    double D2 = 0.0;
    for (int c = 0; c < 8; ++c) {
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double x = ((c >> a) & 1) ? sc->hi[a] : sc->lo[a];
            double d = x - (double)p->position[a];
            d2 += d * d;
        }
        D2 = std::max(D2, d2);
    }
    double reach = std::sqrt(D2) * (double)s->f * 256.0 / (double)s->near_m +
                   (double)std::max(s->width, s->height) * 128.0;
    if (!(reach < 268435456.0)) return HAB_ERR_RANGE;
    return HAB_OK;
}

hab_status to_view_req(const hab_view &hv, ViewReq &out)
{
    if (!hv.scene || !hv.sensor) return HAB_ERR_INVALID_ARG;
    hab_status st = validate_sensor(hv.sensor);
    if (st != HAB_OK) return st;
    const Scene *sc = hv.scene;
    st = validate_pose(sc, hv.sensor, &hv.pose);
    if (st != HAB_OK) return st;
    out.scene = sc;
    out.sensor = *hv.sensor;
    out.pose = hv.pose;
    out.rgb = (hv.sensor->outputs & HAB_OUT_RGB) ? hv.out_rgb : nullptr;
    out.depth = (hv.sensor->outputs & HAB_OUT_DEPTH) ? hv.out_depth : nullptr;
    out.tri = hv.out_tri;
    out.sem = (hv.sensor->outputs & HAB_OUT_SEMANTIC) ? hv.out_semantic : nullptr;
    out.noise_seed = hv.noise_seed;
    if (out.sem && !sc->inst) return HAB_ERR_INVALID_ARG;
    return HAB_OK;
}

// ---------------------------------------------------------------- autotune table
uint32_t class_key(const Scene *sc, const hab_sensor *s)
{
    uint32_t tlog = 0;
    while ((1u << tlog) < std::max<uint32_t>(sc->T, 1)) ++tlog;
    uint32_t wlog = 0;
    while ((1u << wlog) < std::max(s->width, s->height)) ++wlog;
    return (tlog << 9) | (wlog << 4) | (s->outputs & 15u);
}

uint32_t choose_tile(hab_context *ctx, const Scene *sc, const hab_sensor *s, const PlanOpts &o,
                     float *bin_factor)
{
    *bin_factor = o.bin_factor > 0.0f ? o.bin_factor : kDefaultBinFactor;
    if (o.tile_size) return o.tile_size;
    if (ctx) {
        const uint32_t key = class_key(sc, s);
        std::lock_guard<std::mutex> g(ctx->tune_mu);
        for (const Tuned &t : ctx->tuned)
            if (t.key == key) {
                if (o.bin_factor <= 0.0f) *bin_factor = t.bin_factor;
                return t.ts;
            }
    }
    return kDefaultTile;
}

// ---------------------------------------------------------------- planning
static inline uint32_t ts_log2(uint32_t ts) { return ts == 8 ? 3u : ts == 16 ? 4u : 5u; }

hab_status build_plan(hab_context *ctx, Workspace &ws, const ViewReq *v, uint32_t n,
                      const PlanOpts &o, Plan &plan, std::vector<uint8_t> &desc)
{
    if (n == 0 || n > kMaxViews) return HAB_ERR_INVALID_ARG;
    plan.n = n;
    plan.order.resize(n);
    std::iota(plan.order.begin(), plan.order.end(), 0u);
    stable_sort_views(plan.order.begin(), plan.order.end(),
                      [&](uint32_t a, uint32_t b) { return v[a].scene < v[b].scene; });

    // the workspace's buffers: no allocation once they have grown to n views
    std::vector<DView> &dv = ws.dv;
    dv.resize(n);
    std::vector<uint32_t> *lview = ws.lview, *lpre = ws.lpre;
    for (int c = 0; c < 3; ++c) {
        lview[c].clear();
        lpre[c].clear();
    }
    uint64_t tile_total = 0, surv_total = 0, bin_total = 0, pair_total = 0;
    for (uint32_t k = 0; k < n; ++k) {
        const ViewReq &r = v[plan.order[k]];
        float bf;
        uint32_t ts = choose_tile(ctx, r.scene, &r.sensor, o, &bf);
        if (ts != 8 && ts != 16 && ts != 32) return HAB_ERR_INVALID_ARG;
        DView &d = dv[k];
        std::memset(&d, 0, sizeof d);
        for (int a = 0; a < 3; ++a) d.p[a] = r.pose.position[a];
        for (int a = 0; a < 9; ++a) d.R[a] = r.pose.rotation[a];
        d.fS = r.sensor.f * 256.0f;
        d.cxS = (float)r.sensor.width * 128.0f;
        d.cyS = (float)r.sensor.height * 128.0f;
        d.zn = r.sensor.near_m;
        d.W = r.sensor.width;
        d.H = r.sensor.height;
        d.T = r.scene->T;
        d.ts_log2 = ts_log2(ts);
        d.tpos = r.scene->tpos;
        d.col = r.scene->col;
        d.idx = r.scene->idx;
        d.cbox = r.scene->cbox;
        d.rgb = r.rgb;
        d.depth = r.depth;
        d.tri = r.tri;
        d.inst = r.scene->inst;
        d.sem = r.sem;
        d.noise_sigma = r.sensor.depth_noise_sigma;
        d.noise_seed = r.noise_seed;
        d.uv = r.scene->uv;
        d.tex = r.scene->tex;
        d.tex_w = r.scene->tw;
        d.tex_h = r.scene->th;
        d.tiles_x = cdiv(d.W, ts);
        d.tiles_y = cdiv(d.H, ts);
        d.tile_base = (uint32_t)tile_total;
        tile_total += (uint64_t)d.tiles_x * d.tiles_y;
        d.surv_base = (uint32_t)surv_total;
        d.surv_cap = 2u * d.T;
        surv_total += d.surv_cap;
        uint64_t bc = (uint64_t)std::ceil((double)bf * (double)d.T);
        bc = std::max<uint64_t>(bc, 1024);
        bc = std::min<uint64_t>(bc, kIndexLimit / 4);
        d.bin_base = (uint32_t)bin_total;
        d.bin_cap = (uint32_t)bc;
        bin_total += bc;
        d.tile_cap = o.tile_cap ? o.tile_cap : 0xFFFFFFFFu;
        d.count_work = o.count_work ? 1u : 0u;
        d.pair_base = (uint32_t)pair_total;
        pair_total += cdiv(d.T, kCluster);
        const int c = ts == 8 ? 0 : ts == 16 ? 1 : 2;
        lview[c].push_back(k);
    }
    // Raster blocks are dispatched roughly in block order: put the views of
    // the largest scenes (the longest tile lists) first so that their tiles
    // do not form the tail of the launch.
    for (int c = 0; c < 3; ++c) {
        stable_sort_views(lview[c].begin(), lview[c].end(),
                          [&](uint32_t a, uint32_t b) { return dv[a].T > dv[b].T; });
        // lpre: each view's first resolve band (32 x 2 pixels)
        uint32_t pre = 0;
        for (uint32_t k : lview[c]) {
            lpre[c].push_back(pre);
            pre += cdiv(dv[k].W, 32u) * cdiv(dv[k].H, 2u);
        }
    }
    if (tile_total >= kIndexLimit || surv_total >= kIndexLimit || bin_total >= kIndexLimit ||
        pair_total >= kIndexLimit)
        return HAB_ERR_CAPACITY;

    const uint64_t npairs = pair_total;

    // descriptor block
    size_t off = 0;
    plan.off_views = off;
    off = align256(off + sizeof(DView) * n);
    for (int c = 0; c < 3; ++c) {
        plan.off_lview[c] = off;
        off = align256(off + 4 * lview[c].size());
        plan.off_lpre[c] = off;
        off = align256(off + 4 * lpre[c].size());
    }
    plan.off_ctl = off;          // control slot (the stepper's device-pose pointer)
    off = align256(off + 16);
    plan.desc_bytes = off;
    desc.resize(off);
    std::memcpy(desc.data() + plan.off_views, dv.data(), sizeof(DView) * n);

    for (int c = 0; c < 3; ++c) {
        if (!lview[c].empty()) {
            std::memcpy(desc.data() + plan.off_lview[c], lview[c].data(), 4 * lview[c].size());
            std::memcpy(desc.data() + plan.off_lpre[c], lpre[c].data(), 4 * lpre[c].size());
        }
    }
    // scratch
    plan.off_ctr = off;
    off = align256(off + sizeof(DViewCounters) * n);
    plan.off_tcount = off;
    off = align256(off + 4 * tile_total);
    plan.off_toff = off;
    off = align256(off + 4 * tile_total);
    plan.off_tcur = off;
    off = align256(off + 4 * tile_total);
    plan.off_skey = off;
    off = align256(off + 4 * surv_total);
    plan.off_sbox = off;
    off = align256(off + 8 * surv_total);
    plan.off_bins = off;
    off = align256(off + 4 * bin_total);
    plan.off_pairs = off;
    off = align256(off + 4 * std::max<uint64_t>(npairs, 1));
    plan.off_titem = off;
    off = align256(off + 4 * tile_total);
    plan.off_queue = off;
    off = align256(off + sizeof(DQueue));
    // raster work items: a tile holds at most one item per kSegPerTile*TS^2
    // list entries (plus one), so a view needs at most tiles + bin_cap / S
    uint64_t item_cap[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c) {
        const uint64_t S = (uint64_t)kSegPerTile << (6 + 2 * c);
        for (uint32_t k : lview[c])
            item_cap[c] += (uint64_t)dv[k].tiles_x * dv[k].tiles_y + (dv[k].bin_cap + S - 1) / S;
        plan.off_items[c] = off;
        off = align256(off + 8 * item_cap[c]);
        plan.off_partial[c] = off;
        off = align256(off + 8 * item_cap[c] * (64ull << (2 * c)));
    }
    plan.arena_bytes = off;

    LaunchPlan &L = plan.L;
    L = LaunchPlan{};
    L.nviews = n;
    uint32_t max_t = 0;
    for (uint32_t k = 0; k < n; ++k) max_t = std::max(max_t, dv[k].T);
    L.cull_blocks = std::max<uint32_t>(1, cdiv(cdiv(max_t, kCluster), 256));
    // one round of resident setup blocks (the waves take static shares of
    // the work, so a second partial round would only add a tail)
    const uint64_t setup_resident = (uint64_t)kSetupWavesPerSimd * 4 / (kSetupBlock / 64);
    L.setup_grid = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>((npairs + 15) / 16, setup_resident * (ctx ? ctx->cu_count : 256)));
    L.ntiles = (uint32_t)tile_total;
    uint64_t ub = 0;
    for (uint32_t k = 0; k < n; ++k) ub += cdiv(dv[k].surv_cap, kBinBlock * kBinItems);
    L.bin_grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(ub, 8ull * (ctx ? ctx->cu_count : 256)));
    L.nraster = 0;
    const uint32_t cus = ctx ? (uint32_t)ctx->cu_count : 256u;
    const int lo = o.lane_owned_z ? 1 : 0;
    const uint32_t kBlocksPerCu[3] = {ctx ? (uint32_t)ctx->raster_bpc[lo][0] : 1u,
                                      ctx ? (uint32_t)ctx->raster_bpc[lo][1] : 1u,
                                      ctx ? (uint32_t)ctx->raster_bpc[lo][2] : 1u};
    for (int c = 0; c < 3; ++c) {
        if (lview[c].empty()) continue;
        RasterLaunch &R = L.raster[L.nraster++];
        R.ts = c == 0 ? 8 : c == 1 ? 16 : 32;
        R.nl = (uint32_t)lview[c].size();
        const DView &last = dv[lview[c].back()];
        R.blocks = 0;
        for (uint32_t k : lview[c]) R.blocks += dv[k].tiles_x * dv[k].tiles_y;
        R.bands = lpre[c].back() + cdiv(last.W, 32u) * cdiv(last.H, 2u);
        R.item_cap = item_cap[c];
        R.grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(item_cap[c], (uint64_t)cus * kBlocksPerCu[c]));
        R.lane_owned = o.lane_owned_z;
    }
    return HAB_OK;
}

void bind_plan(Plan &plan, void *arena, uint32_t *err)
{
    char *b = static_cast<char *>(arena);
    LaunchPlan &L = plan.L;
    L.views = reinterpret_cast<const DView *>(b + plan.off_views);
    L.ctr = reinterpret_cast<DViewCounters *>(b + plan.off_ctr);
    L.tile_count = reinterpret_cast<uint32_t *>(b + plan.off_tcount);
    L.tile_off = reinterpret_cast<uint32_t *>(b + plan.off_toff);
    L.tile_cursor = reinterpret_cast<uint32_t *>(b + plan.off_tcur);
    L.skey = reinterpret_cast<uint32_t *>(b + plan.off_skey);
    L.sbox = reinterpret_cast<uint2 *>(b + plan.off_sbox);
    L.bins = reinterpret_cast<uint32_t *>(b + plan.off_bins);
    L.tile_item = reinterpret_cast<uint32_t *>(b + plan.off_titem);
    L.queue = reinterpret_cast<DQueue *>(b + plan.off_queue);
    L.pairs = reinterpret_cast<uint32_t *>(b + plan.off_pairs);
    L.err = err;
    for (int c = 0; c < 3; ++c) L.items[c] = reinterpret_cast<uint2 *>(b + plan.off_items[c]);
    for (int k = 0; k < L.nraster; ++k) {
        RasterLaunch &R = L.raster[k];
        const int c = R.ts == 8 ? 0 : R.ts == 16 ? 1 : 2;
        R.lview = reinterpret_cast<const uint32_t *>(b + plan.off_lview[c]);
        R.bpre = reinterpret_cast<const uint32_t *>(b + plan.off_lpre[c]);
        R.items = reinterpret_cast<uint2 *>(b + plan.off_items[c]);
        R.partial = reinterpret_cast<uint2 *>(b + plan.off_partial[c]);
    }
}

Footprint footprint(const ViewReq *v, uint32_t n, const PlanOpts &o, hab_context *ctx)
{
    Footprint f;
    uint64_t bytes = 0, tiles = 0;
    for (uint32_t k = 0; k < n; ++k) {
        float bf;
        uint32_t ts = choose_tile(ctx, v[k].scene, &v[k].sensor, o, &bf);
        uint64_t nt = (uint64_t)cdiv(v[k].sensor.width, ts) * cdiv(v[k].sensor.height, ts);
        tiles += nt;
        uint64_t bc = std::max<uint64_t>((uint64_t)std::ceil((double)bf * v[k].scene->T), 1024);
        const uint64_t S = (uint64_t)kSegPerTile * ts * ts;
        const uint64_t items = nt + (bc + S - 1) / S;
        bytes += 2ull * v[k].scene->T * 12ull + bc * 4ull + nt * 16ull + sizeof(DView) + sizeof(DViewCounters) + 64 +
                 4ull * cdiv(v[k].scene->T, kCluster) +
                 items * 8ull * (1 + (uint64_t)ts * ts);
    }
    f.desc_bytes = n * (sizeof(DView) + 32) + 4096;
    // + the work queues and the padding of the plan's 24 aligned arrays
    f.arena_bytes = bytes + f.desc_bytes + sizeof(DQueue) + 32 * 256;
    (void)tiles;
    return f;
}

// ---------------------------------------------------------------- launching
hab_status render_views(hab_context *ctx, Workspace &ws, const ViewReq *v, uint32_t n,
                        const PlanOpts &opts, hipStream_t s, hab_view_stats *stats)
{
    PlanOpts o = opts;
    o.count_work = stats != nullptr;
    Plan plan;
    hab_status st = build_plan(ctx, ws, v, n, o, plan, ws.desc);
    if (st != HAB_OK) return st;
    st = ws.ensure(plan.arena_bytes);
    if (st != HAB_OK) return st;
    if (ws.has_done && ws.last_stream != s) HAB_HIP(hipStreamWaitEvent(s, ws.done, 0));
    void *host;
    int slot;
    st = ws.staging(plan.desc_bytes, &host, &slot);
    if (st != HAB_OK) return st;
    std::memcpy(host, ws.desc.data(), plan.desc_bytes);
    HAB_HIP(hipMemcpyAsync(ws.arena, host, plan.desc_bytes, hipMemcpyHostToDevice, s));
    HAB_HIP(hipEventRecord(ws.slots[slot].ev, s));
    ws.slots[slot].pending = true;
    bind_plan(plan, ws.arena, ctx->err);
    hab_context::ProfSet *ps = nullptr;
    if (ctx->prof_on) {
        if (ctx->prof_used == ctx->prof_sets.size()) {
            hab_context::ProfSet fresh{};
            for (int e = 0; e < kProfEvents; ++e) HAB_HIP(hipEventCreate(&fresh.ev[e]));
            ctx->prof_sets.push_back(fresh);
        }
        ps = &ctx->prof_sets[ctx->prof_used++];
        ps->mask = 0x1Fu | (1u << kPhaseResolve);
        for (int k = 0; k < plan.L.nraster; ++k)
            if (plan.L.raster[k].blocks)
                ps->mask |= 1u << (plan.L.raster[k].ts == 8 ? 5 : plan.L.raster[k].ts == 16 ? 6 : 7);
        ps->mask &= ctx->prof_phase_mask;
        plan.L.prof = ps->ev;
        plan.L.prof_mask = ps->mask;
    }
    HAB_HIP(launch_render(plan.L, s));
    HAB_HIP(hipEventRecord(ws.done, s));
    ws.has_done = true;
    ws.last_stream = s;
    if (stats) {
        std::vector<DViewCounters> c(n);
        HAB_HIP(hipMemcpyAsync(c.data(), plan.L.ctr, sizeof(DViewCounters) * n, hipMemcpyDeviceToHost, s));
        HAB_HIP(hipStreamSynchronize(s));
        for (uint32_t k = 0; k < n; ++k) {
            hab_view_stats &o2 = stats[plan.order[k]];
            o2.survivors = c[k].surv_count;
            o2.bbox_tests = c[k].bbox_tests;
            o2.covered = c[k].covered;
        }
    }
    return HAB_OK;
}

hab_status stage_and_launch(hab_context *ctx, Workspace &ws, Plan &plan, void *arena, hipStream_t s,
                            bool reserved)
{
    void *host;
    int slot;
    hab_status st = reserved ? ws.staging_reserved(plan.desc_bytes, &host, &slot)
                             : ws.staging(plan.desc_bytes, &host, &slot);
    if (st != HAB_OK) return st;
    std::memcpy(host, ws.desc.data(), plan.desc_bytes);
    HAB_HIP(hipMemcpyAsync(arena, host, plan.desc_bytes, hipMemcpyHostToDevice, s));
    HAB_HIP(hipEventRecord(ws.slots[slot].ev, s));
    ws.slots[slot].pending = true;
    bind_plan(plan, arena, ctx->err);
    HAB_HIP(launch_render(plan.L, s));
    return HAB_OK;
}

hab_status render_all(hab_context *ctx, Workspace &ws, const ViewReq *v, uint32_t n,
                      const PlanOpts &o, hipStream_t s, hab_view_stats *stats)
{
    uint32_t k = 0;
    while (k < n) {
        uint32_t e = k;
        uint64_t surv = 0, bins = 0;
        while (e < n && e - k < kMaxViews) {
            float bf;
            (void)choose_tile(ctx, v[e].scene, &v[e].sensor, o, &bf);
            const uint64_t s2 = 2ull * v[e].scene->T;
            const uint64_t b2 = std::max<uint64_t>((uint64_t)std::ceil((double)bf * v[e].scene->T), 1024);
            if (e > k && (surv + s2 >= kIndexLimit / 2 || bins + b2 >= kIndexLimit / 2)) break;
            surv += s2;
            bins += b2;
            ++e;
        }
        hab_status st = render_views(ctx, ws, v + k, e - k, o, s, stats ? stats + k : nullptr);
        if (st != HAB_OK) return st;
        k = e;
    }
    return HAB_OK;
}

hab_status ensure_aux(hab_context *ctx)
{
    if (!ctx->aux) HAB_HIP(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
    if (!ctx->fork_ev) HAB_HIP(hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
    if (!ctx->join_ev) HAB_HIP(hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming));
    return HAB_OK;
}

hab_status render_split(hab_context *ctx, const ViewReq *v, uint32_t n, const PlanOpts &o, hipStream_t s,
                        hab_view_stats *stats)
{
    if (n < kSplitViews || o.one_sequence) return render_all(ctx, ctx->ws, v, n, o, s, stats);
    hab_status st = ensure_aux(ctx);
    if (st != HAB_OK) return st;
    // views 0, 2, 4, ... and 1, 3, 5, ...: halves of like composition
    std::vector<ViewReq> half[2];
    std::vector<hab_view_stats> hs[2];
    for (int h = 0; h < 2; ++h) {
        half[h].reserve((n + 1) / 2);
        if (stats) hs[h].resize((n + 1 - (uint32_t)h) / 2);
    }
    for (uint32_t k = 0; k < n; ++k) half[k & 1u].push_back(v[k]);
    HAB_HIP(hipEventRecord(ctx->fork_ev, s));
    HAB_HIP(hipStreamWaitEvent(ctx->aux, ctx->fork_ev, 0));
    st = render_all(ctx, ctx->ws, half[0].data(), (uint32_t)half[0].size(), o, s,
                    stats ? hs[0].data() : nullptr);
    if (st == HAB_OK)
        st = render_all(ctx, ctx->ws2, half[1].data(), (uint32_t)half[1].size(), o, ctx->aux,
                        stats ? hs[1].data() : nullptr);
    // the join is enqueued whatever happened, so that s is ordered after
    // everything the call put on the second stream
    HAB_HIP(hipEventRecord(ctx->join_ev, ctx->aux));
    HAB_HIP(hipStreamWaitEvent(s, ctx->join_ev, 0));
    if (st != HAB_OK) return st;
    if (stats)
        for (uint32_t k = 0; k < n; ++k) stats[k] = hs[k & 1u][k >> 1];
    return HAB_OK;
}

}  // namespace habmi
