// Agent actuation and collision (Sec. 4 "Agent embodiment and action
// space", "Collision dynamics"): one action per agent, forward moves by
// collide-and-slide of a disc against line-segment obstacles on the floor
// plane, in fp64.  The definition (contact rule, skin, passes, tie order)
// is stated with hab_actuate in hab.h.
//
// Layout: each obstacle set carries a uniform grid built at upload (cells
// of 0.1-0.5 m sized to the segments; a cell lists every segment whose
// bounding box overlaps it).  A
// group of G lanes moves one agent (G = 64 for small batches, where one
// lane per agent would leave the chip idle and expose the dependent
// cell -> list -> segment loads; fewer for large ones): per pass each lane
// takes every G-th entry of the cells under the box swept by the disc
// (grown by the radius and a 0.1 mm margin), runs the fp64 contact test on
// the segments whose own box meets the swept box, and the group reduces
// the lanes' earliest contacts with shuffles.
// A segment outside that box cannot be touched during the move, and the
// winning contact is chosen by an explicit order (time, then segment index,
// then interior before first before second endpoint), so the result is the
// same as testing every segment in index order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <unordered_map>
#include <vector>

#include "runtime.h"

#pragma clang fp contract(off)

namespace {

constexpr double kNavCellMax = 0.5;    // grid cell edge, metres: at most
constexpr double kNavCellMin = 0.1;    //   and at least (see nav_build)
constexpr uint32_t kNavMaxDim = 1024;  // cells per axis (the cell grows beyond)

// What the kernel needs of one obstacle set.
struct alignas(16) NavDesc {
    const float4 *seg;          // [n] (x0, z0, x1, z1)
    const uint32_t *cell_start; // [gx * gz + 1]
    const uint32_t *items;      // segment indices, per cell
    float ox, oz;               // grid origin
    float inv_h, h;             // 1 / cell edge, cell edge
    uint32_t gx, gz;            // cells per axis (0: no segments)
};

}  // namespace

struct hab_nav {
    int device = 0;
    uint32_t n = 0;
    void *mem = nullptr;        // segments, cell starts and items in one allocation
    NavDesc d{};
};

namespace habmi {
namespace {

constexpr int kActBlock = 256;
constexpr int kSlidePasses = 4;
constexpr double kSkin = 1e-6;

struct ActParams {
    double radius, step, tc, ts;
    float cam_h;
};

// Contact of the disc at p moving by d (a = |d|^2 > 0) with segment j;
// keeps the first contact in the order (t, 3 j + kind), kind 0 for the
// interior, 1 and 2 for the endpoints.
__device__ __forceinline__ void seg_contact(float4 sg, uint32_t j, double r, double px, double pz,
                                            double dx, double dz, double a, bool &found, double &bt,
                                            uint32_t &bcode, double &bnx, double &bnz)
{
    const double ax = sg.x, az = sg.y, bx = sg.z, bz = sg.w;
    const double ex = bx - ax, ez = bz - az;
    const double L2 = ex * ex + ez * ez;
    if (L2 > 0.0) {
        const double L = sqrt(L2);
        double nx = -ez / L, nz = ex / L;
        double d0 = (px - ax) * nx + (pz - az) * nz;
        double rate = dx * nx + dz * nz;
        if (d0 < 0.0) {
            d0 = -d0;
            rate = -rate;
            nx = -nx;
            nz = -nz;
        }
        if (rate < 0.0) {
            double t = (d0 - r) / -rate;
            if (t < 0.0) t = 0.0;
            if (t <= 1.0) {
                const double cx = px + t * dx, cz = pz + t * dz;
                const double s = ((cx - ax) * ex + (cz - az) * ez) / L2;
                const uint32_t code = 3u * j;
                if (s >= 0.0 && s <= 1.0 && (!found || t < bt || (t == bt && code < bcode))) {
                    found = true;
                    bt = t;
                    bcode = code;
                    bnx = nx;
                    bnz = nz;
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const double qx = e ? bx : ax, qz = e ? bz : az;
        const double gx = px - qx, gz = pz - qz;
        const double b = gx * dx + gz * dz;
        if (!(b < 0.0)) continue;
        const double c = gx * gx + gz * gz - r * r;
        double t;
        if (c <= 0.0) {
            t = 0.0;
        } else {
            const double disc = b * b - a * c;
            if (disc < 0.0) continue;
            t = (-b - sqrt(disc)) / a;
        }
        if (t > 1.0) continue;
        const double cx = px + t * dx - qx, cz = pz + t * dz - qz;
        const double len = sqrt(cx * cx + cz * cz);
        if (!(len > 0.0)) continue;
        const uint32_t code = 3u * j + 1u + (uint32_t)e;
        if (!found || t < bt || (t == bt && code < bcode)) {
            found = true;
            bt = t;
            bcode = code;
            bnx = cx / len;
            bnz = cz / len;
        }
    }
}

__device__ __forceinline__ int cell_of(float q, float o, float inv_h, uint32_t g)
{
    const float c = floorf((q - o) * inv_h);
    return (int)fminf(fmaxf(c, 0.0f), (float)(g - 1u));
}

// Lexicographic minimum of the group's contacts (found first, then t, then
// code): every lane ends with the group's winner.
template <int G>
__device__ __forceinline__ void group_min(bool &found, double &bt, uint32_t &bcode, double &bnx, double &bnz)
{
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
        const int of = __shfl_xor((int)found, off, G);
        const double ot = __shfl_xor(bt, off, G);
        const uint32_t oc = (uint32_t)__shfl_xor((int)bcode, off, G);
        const double ox = __shfl_xor(bnx, off, G), oz = __shfl_xor(bnz, off, G);
        if (of && (!found || ot < bt || (ot == bt && oc < bcode))) {
            found = true;
            bt = ot;
            bcode = oc;
            bnx = ox;
            bnz = oz;
        }
    }
}

template <int G>
__global__ __launch_bounds__(kActBlock) void k_actuate(const NavDesc *__restrict__ navs,
                                                       const uint32_t *__restrict__ nav_of,
                                                       uint32_t n, hab_agent *__restrict__ agents,
                                                       const uint8_t *__restrict__ actions,
                                                       uint8_t *__restrict__ collided,
                                                       float *__restrict__ poses, ActParams P)
{
    const uint32_t gid = blockIdx.x * kActBlock + threadIdx.x;
    const uint32_t k = gid / G, lane = gid % G;
    // whole groups leave together (n agents fill n * G lanes; groups never
    // straddle a wave), so the shuffles below see only live lanes
    if (k >= n) return;
    hab_agent g = agents[k];
    const uint32_t act = actions[k];
    if (act == HAB_ACT_LEFT || act == HAB_ACT_RIGHT) {
        const double s = act == HAB_ACT_LEFT ? P.ts : -P.ts;
        const double fx = g.fx * P.tc + g.fz * s;
        const double fz = g.fz * P.tc - g.fx * s;
        g.fx = fx;
        g.fz = fz;
    }
    bool hit = false;
    if (act == HAB_ACT_FORWARD) {
        const NavDesc D = navs[nav_of[k]];
        double px = g.x, pz = g.z;
        double dx = P.step * g.fx, dz = P.step * g.fz;
        const float grow = (float)P.radius + 1e-4f;
        for (int pass = 0; pass < kSlidePasses; ++pass) {
            const double a = dx * dx + dz * dz;
            if (!(a > 0.0)) break;
            bool found = false;
            double bt = 0.0, bnx = 0.0, bnz = 0.0;
            uint32_t bcode = 0;
            const float qx0 = (float)fmin(px, px + dx) - grow, qx1 = (float)fmax(px, px + dx) + grow;
            const float qz0 = (float)fmin(pz, pz + dz) - grow, qz1 = (float)fmax(pz, pz + dz) + grow;
            const bool inside = D.gx && qx1 >= D.ox && qz1 >= D.oz && qx0 <= D.ox + D.h * (float)D.gx &&
                                qz0 <= D.oz + D.h * (float)D.gz;
            if (inside) {
                const int cx0 = cell_of(qx0, D.ox, D.inv_h, D.gx), cx1 = cell_of(qx1, D.ox, D.inv_h, D.gx);
                const int cz0 = cell_of(qz0, D.oz, D.inv_h, D.gz), cz1 = cell_of(qz1, D.oz, D.inv_h, D.gz);
                for (int cz = cz0; cz <= cz1; ++cz)
                    for (int cx = cx0; cx <= cx1; ++cx) {
                        const uint32_t c = (uint32_t)cz * D.gx + (uint32_t)cx;
                        const uint32_t i1 = D.cell_start[c + 1];
                        for (uint32_t i = D.cell_start[c] + lane; i < i1; i += G) {
                            const uint32_t j = D.items[i];
                            const float4 sg = D.seg[j];
                            if (fminf(sg.x, sg.z) > qx1 || fmaxf(sg.x, sg.z) < qx0 ||
                                fminf(sg.y, sg.w) > qz1 || fmaxf(sg.y, sg.w) < qz0)
                                continue;
                            seg_contact(sg, j, P.radius, px, pz, dx, dz, a, found, bt, bcode, bnx, bnz);
                        }
                    }
            }
            if (G > 1) group_min<G>(found, bt, bcode, bnx, bnz);
            if (!found) {
                px += dx;
                pz += dz;
                break;
            }
            hit = true;
            double ts = bt - kSkin / sqrt(a);
            if (ts < 0.0) ts = 0.0;
            px += ts * dx;
            pz += ts * dz;
            double rx = (1.0 - ts) * dx, rz = (1.0 - ts) * dz;
            const double dn = rx * bnx + rz * bnz;
            rx -= dn * bnx;
            rz -= dn * bnz;
            dx = rx;
            dz = rz;
        }
        g.x = px;
        g.z = pz;
    }
    if (lane != 0) return;
    agents[k] = g;
    if (collided) collided[k] = hit ? 1 : 0;
    if (poses) {
        float *o = poses + 12ull * k;
        const float fx = (float)g.fx, fz = (float)g.fz;
        o[0] = (float)g.x;
        o[1] = P.cam_h;
        o[2] = (float)g.z;
        o[3] = -fz;
        o[4] = 0.0f;
        o[5] = -fx;
        o[6] = 0.0f;
        o[7] = 1.0f;
        o[8] = 0.0f;
        o[9] = fx;
        o[10] = 0.0f;
        o[11] = -fz;
    }
}

// ------------------------------------------------------------ obstacles from the mesh
// Horizontal cross-sections of the scene's triangles at K heights (the
// agent's body between just above the floor and its top; the definition is
// stated with hab_nav_from_scene in hab.h): per triangle, the mask of the
// heights whose plane separates its vertices; a block scan of the counts
// gives each triangle's first output slot, so the segments come out in
// (triangle, height) order.
constexpr int kSliceBlock = 256;

struct SliceParams {
    double h[HAB_NAV_MAX_HEIGHTS];
    uint32_t K;
};

__device__ __forceinline__ void load_tri_pos(const float *__restrict__ tpos, uint32_t t, double P[3][3])
{
    const float *p = tpos + 9ull * t;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) P[k][a] = (double)p[3 * k + a];
}

// Heights (bit h) whose plane has vertices of the triangle on both sides
// (a vertex at exactly the height counts as above).
__device__ __forceinline__ uint32_t slice_mask(const double P[3][3], const SliceParams &S)
{
    uint32_t m = 0;
    for (uint32_t h = 0; h < S.K; ++h) {
        const double y = S.h[h];
        const bool u0 = P[0][1] >= y, u1 = P[1][1] >= y, u2 = P[2][1] >= y;
        if (!(u0 == u1 && u1 == u2)) m |= 1u << h;
    }
    return m;
}

// Exclusive scan of x over the block (wave64 shuffles + one LDS word per
// wave); *total gets the block's sum.
__device__ __forceinline__ uint32_t slice_block_scan(uint32_t x, uint32_t *total)
{
    __shared__ uint32_t wsum[kSliceBlock / 64];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    uint32_t s = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(s, off);
        if (lane >= (uint32_t)off) s += y;
    }
    if (lane == 63) wsum[wave] = s;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kSliceBlock / 64; ++w) {
        const uint32_t v = wsum[w];
        pre += (w < (int)wave) ? v : 0u;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return pre + s - x;
}

__global__ __launch_bounds__(kSliceBlock) void k_slice_count(const float *__restrict__ tpos, uint32_t T,
                                                             SliceParams S, uint32_t *__restrict__ block_total)
{
    const uint32_t t = blockIdx.x * kSliceBlock + threadIdx.x;
    uint32_t c = 0;
    if (t < T) {
        double P[3][3];
        load_tri_pos(tpos, t, P);
        c = (uint32_t)__popc(slice_mask(P, S));
    }
    uint32_t tot;
    (void)slice_block_scan(c, &tot);
    if (threadIdx.x == 0) block_total[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kSliceBlock) void k_slice_write(const float *__restrict__ tpos, uint32_t T,
                                                             SliceParams S,
                                                             const uint32_t *__restrict__ block_base,
                                                             float4 *__restrict__ seg)
{
    const uint32_t t = blockIdx.x * kSliceBlock + threadIdx.x;
    double P[3][3] = {};
    uint32_t m = 0;
    if (t < T) {
        load_tri_pos(tpos, t, P);
        m = slice_mask(P, S);
    }
    uint32_t tot;
    uint32_t o = block_base[blockIdx.x] + slice_block_scan((uint32_t)__popc(m), &tot);
    for (uint32_t h = 0; h < S.K; ++h) {
        if (!((m >> h) & 1u)) continue;
        const double y = S.h[h];
        bool up[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) up[k] = P[k][1] >= y;
        // the two edges (walked v0->v1, v1->v2, v2->v0) that change side,
        // each cut by interpolation from its lower end to its upper end
        double cx[2] = {0.0, 0.0}, cz[2] = {0.0, 0.0};
        int nc = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int k1 = (k + 1) % 3;
            if (up[k] == up[k1]) continue;
            const double *lo = up[k] ? P[k1] : P[k];
            const double *hi = up[k] ? P[k] : P[k1];
            const double s = (y - lo[1]) / (hi[1] - lo[1]);
            cx[nc] = lo[0] + s * (hi[0] - lo[0]);
            cz[nc] = lo[2] + s * (hi[2] - lo[2]);
            ++nc;
        }
        seg[o++] = make_float4((float)cx[0], (float)cz[0], (float)cx[1], (float)cz[1]);
    }
}

// Free-space query: is a disc of radius r at (x, z) clear of every segment
// (each at least r away)?  One lane per point, over the grid cells under
// the disc's box grown by a 0.1 mm margin (a segment that comes within r
// has its box meet the disc's, so it is listed in one of those cells);
// the per-segment test is the fp64 point-segment distance with the
// parameter clamped to the segment.
__global__ __launch_bounds__(kActBlock) void k_nav_free(NavDesc D, const double2 *__restrict__ pts, uint32_t n,
                                                        double r, uint8_t *__restrict__ out)
{
    const uint32_t i = blockIdx.x * kActBlock + threadIdx.x;
    if (i >= n) return;
    const double2 p = pts[i];
    const double px = p.x, pz = p.y, r2 = r * r;
    bool blocked = false;
    const float grow = (float)r + 1e-4f;
    const float qx0 = (float)px - grow, qx1 = (float)px + grow;
    const float qz0 = (float)pz - grow, qz1 = (float)pz + grow;
    const bool inside = D.gx && qx1 >= D.ox && qz1 >= D.oz && qx0 <= D.ox + D.h * (float)D.gx &&
                        qz0 <= D.oz + D.h * (float)D.gz;
    if (inside) {
        const int cx0 = cell_of(qx0, D.ox, D.inv_h, D.gx), cx1 = cell_of(qx1, D.ox, D.inv_h, D.gx);
        const int cz0 = cell_of(qz0, D.oz, D.inv_h, D.gz), cz1 = cell_of(qz1, D.oz, D.inv_h, D.gz);
        for (int cz = cz0; cz <= cz1 && !blocked; ++cz)
            for (int cx = cx0; cx <= cx1 && !blocked; ++cx) {
                const uint32_t c = (uint32_t)cz * D.gx + (uint32_t)cx;
                const uint32_t i1 = D.cell_start[c + 1];
                for (uint32_t k = D.cell_start[c]; k < i1; ++k) {
                    const float4 sg = D.seg[D.items[k]];
                    if (fminf(sg.x, sg.z) > qx1 || fmaxf(sg.x, sg.z) < qx0 || fminf(sg.y, sg.w) > qz1 ||
                        fmaxf(sg.y, sg.w) < qz0)
                        continue;
                    const double ax = sg.x, az = sg.y;
                    const double ex = (double)sg.z - ax, ez = (double)sg.w - az;
                    const double L2 = ex * ex + ez * ez;
                    double s = 0.0;
                    if (L2 > 0.0) {
                        s = ((px - ax) * ex + (pz - az) * ez) / L2;
                        s = s < 0.0 ? 0.0 : s;
                        s = s > 1.0 ? 1.0 : s;
                    }
                    const double qx = ax + s * ex - px, qz = az + s * ez - pz;
                    if (qx * qx + qz * qz < r2) {
                        blocked = true;
                        break;
                    }
                }
            }
    }
    out[i] = blocked ? 0 : 1;
}

}  // namespace

void release_navs(hab_context *ctx)
{
    for (hab_nav *n : ctx->navs) {
        dev_free(n->mem);
        delete n;
    }
    ctx->navs.clear();
    ctx->act_last.clear();
}

}  // namespace habmi

using namespace habmi;

namespace habmi {

// An obstacle set from host segments: the grid built here, segments, cell
// starts and cell lists copied to one device allocation.
static hab_status nav_build(hab_context *ctx, const float *segments, uint32_t num_segments, hab_nav **out)
{
    {
        // the grid over the segments' bounding box: cells of four times the
        // mean segment length within [kNavCellMin, kNavCellMax] (a few
        // segments per occupied cell whether the obstacles are whole walls
        // or a tessellated mesh's short cross-section pieces), larger when
        // the extent needs more than kNavMaxDim cells per axis
        NavDesc d{};
        std::vector<uint32_t> start, items;
        if (num_segments) {
            double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
            for (uint32_t j = 0; j < num_segments; ++j)
                for (int e = 0; e < 2; ++e)
                    for (int a = 0; a < 2; ++a) {
                        lo[a] = std::min(lo[a], (double)segments[4ull * j + 2 * e + a]);
                        hi[a] = std::max(hi[a], (double)segments[4ull * j + 2 * e + a]);
                    }
            double len = 0.0;
            for (uint32_t j = 0; j < num_segments; ++j) {
                const float *q = segments + 4ull * j;
                len += std::hypot((double)q[2] - q[0], (double)q[3] - q[1]);
            }
            double h = std::min(kNavCellMax, std::max(kNavCellMin, 4.0 * len / num_segments));
            const double ext = std::max(hi[0] - lo[0], hi[1] - lo[1]);
            if (ext / h + 1.0 > kNavMaxDim) h = ext / (kNavMaxDim - 1);
            d.gx = (uint32_t)((hi[0] - lo[0]) / h) + 1u;
            d.gz = (uint32_t)((hi[1] - lo[1]) / h) + 1u;
            d.ox = (float)lo[0];
            d.oz = (float)lo[1];
            d.h = (float)h;
            d.inv_h = (float)(1.0 / h);
            auto cell = [&](double q, double o, uint32_t gdim) {
                const double c = std::floor((q - o) / h);
                return (uint32_t)std::min(std::max(c, 0.0), (double)(gdim - 1));
            };
            std::vector<std::vector<uint32_t>> lists((size_t)d.gx * d.gz);
            for (uint32_t j = 0; j < num_segments; ++j) {
                const float *s = segments + 4ull * j;
                const uint32_t x0 = cell(std::min(s[0], s[2]), d.ox, d.gx);
                const uint32_t x1 = cell(std::max(s[0], s[2]), d.ox, d.gx);
                const uint32_t z0 = cell(std::min(s[1], s[3]), d.oz, d.gz);
                const uint32_t z1 = cell(std::max(s[1], s[3]), d.oz, d.gz);
                for (uint32_t cz = z0; cz <= z1; ++cz)
                    for (uint32_t cx = x0; cx <= x1; ++cx) lists[(size_t)cz * d.gx + cx].push_back(j);
            }
            start.assign(lists.size() + 1, 0);
            for (size_t c = 0; c < lists.size(); ++c) {
                start[c + 1] = start[c] + (uint32_t)lists[c].size();
                items.insert(items.end(), lists[c].begin(), lists[c].end());
            }
        }
        const size_t bseg = 16ull * num_segments, bstart = 4ull * start.size(), bitems = 4ull * items.size();
        const size_t o_start = (bseg + 255) & ~(size_t)255, o_items = (o_start + bstart + 255) & ~(size_t)255;
        DeviceGuard g(ctx->device);
        if (!g.ok) return HAB_ERR_DEVICE;
        hab_nav *n = new hab_nav();
        n->device = ctx->device;
        n->n = num_segments;
        if (num_segments) {
            if (!dev_alloc(&n->mem, o_items + bitems)) {
                delete n;
                return HAB_ERR_OUT_OF_MEMORY;
            }
            char *m = static_cast<char *>(n->mem);
            if (hipMemcpy(m, segments, bseg, hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(m + o_start, start.data(), bstart, hipMemcpyHostToDevice) != hipSuccess ||
                (bitems && hipMemcpy(m + o_items, items.data(), bitems, hipMemcpyHostToDevice) != hipSuccess)) {
                dev_free(n->mem);
                delete n;
                return HAB_ERR_DEVICE;
            }
            d.seg = reinterpret_cast<const float4 *>(m);
            d.cell_start = reinterpret_cast<const uint32_t *>(m + o_start);
            d.items = reinterpret_cast<const uint32_t *>(m + o_items);
        }
        n->d = d;
        ctx->navs.push_back(n);
        *out = n;
        return HAB_OK;
    }
}

}  // namespace habmi

extern "C" {

hab_status hab_nav_upload(hab_context *ctx, const float *segments, uint32_t num_segments, hab_nav **out)
{
    if (!ctx || !out || (num_segments && !segments)) return HAB_ERR_INVALID_ARG;
    *out = nullptr;
    return guarded([&]() -> hab_status {
        for (uint64_t k = 0; k < 4ull * num_segments; ++k)
            if (!std::isfinite(segments[k])) return HAB_ERR_INVALID_ARG;
        return nav_build(ctx, segments, num_segments, out);
    });
}

hab_status hab_nav_release(hab_context *ctx, hab_nav *nav)
{
    if (!ctx || !nav) return HAB_ERR_INVALID_ARG;
    return guarded([&]() -> hab_status {
        auto it = std::find(ctx->navs.begin(), ctx->navs.end(), nav);
        if (it == ctx->navs.end()) return HAB_ERR_INVALID_ARG;
        DeviceGuard g(ctx->device);
        // work that still reads the segments must finish first
        HAB_HIP(hipDeviceSynchronize());
        dev_free(nav->mem);
        ctx->navs.erase(it);
        delete nav;
        ctx->act_last.clear();
        return HAB_OK;
    });
}

hab_status hab_actuate(hab_context *ctx, const hab_nav *const *navs, uint32_t n, hab_agent *agents,
                       const uint8_t *actions, uint8_t *collided, float *poses, float camera_height,
                       const hab_actuation *params, hipStream_t stream)
{
    if (!ctx || !params || (n && (!navs || !agents || !actions))) return HAB_ERR_INVALID_ARG;
    if (!(params->radius > 0.0) || !std::isfinite(params->radius) || !(params->forward_m >= 0.0) ||
        !std::isfinite(params->forward_m) || !std::isfinite(params->turn_cos) ||
        !std::isfinite(params->turn_sin) || !std::isfinite(camera_height))
        return HAB_ERR_INVALID_ARG;
    if (n == 0) return HAB_OK;
    return guarded([&]() -> hab_status {
        Workspace &ws = ctx->act_ws;
        DeviceGuard dg(ctx->device);
        if (!dg.ok) return HAB_ERR_DEVICE;
        const bool same = ctx->act_last.size() == n && ws.arena &&
                          std::memcmp(ctx->act_last.data(), navs, sizeof(const hab_nav *) * n) == 0;
        if (!same) {
            // the distinct obstacle sets (first-seen order) and each agent's
            // index among them, staged and copied to the arena; kept for the
            // next call with the same sets
            ctx->act_last.clear();
            std::unordered_map<const hab_nav *, uint32_t> id;
            std::vector<NavDesc> table;
            for (uint32_t k = 0; k < n; ++k)
                if (!id.count(navs[k])) {
                    if (std::find(ctx->navs.begin(), ctx->navs.end(), navs[k]) == ctx->navs.end())
                        return HAB_ERR_INVALID_ARG;
                    id.emplace(navs[k], (uint32_t)table.size());
                    table.push_back(navs[k]->d);
                }
            const size_t off_idx = (sizeof(NavDesc) * table.size() + 255) & ~(size_t)255;
            const size_t bytes = off_idx + 4ull * n;
            hab_status st = ws.ensure(bytes);
            if (st != HAB_OK) return st;
            if (ws.has_done && ws.last_stream != stream) HAB_HIP(hipStreamWaitEvent(stream, ws.done, 0));
            void *host;
            int slot;
            st = ws.staging(bytes, &host, &slot);
            if (st != HAB_OK) return st;
            std::memcpy(host, table.data(), sizeof(NavDesc) * table.size());
            uint32_t *hi = reinterpret_cast<uint32_t *>(static_cast<char *>(host) + off_idx);
            for (uint32_t k = 0; k < n; ++k) hi[k] = id[navs[k]];
            HAB_HIP(hipMemcpyAsync(ws.arena, host, bytes, hipMemcpyHostToDevice, stream));
            HAB_HIP(hipEventRecord(ws.slots[slot].ev, stream));
            ws.slots[slot].pending = true;
            ctx->act_last.assign(navs, navs + n);
            ctx->act_last_off = off_idx;
        } else if (ws.has_done && ws.last_stream != stream) {
            HAB_HIP(hipStreamWaitEvent(stream, ws.done, 0));
        }
        ActParams P{params->radius, params->forward_m, params->turn_cos, params->turn_sin, camera_height};
        const NavDesc *dt = static_cast<const NavDesc *>(ws.arena);
        const uint32_t *di = reinterpret_cast<const uint32_t *>(static_cast<char *>(ws.arena) + ctx->act_last_off);
        // lanes per agent: enough groups to fill the chip (~64k lanes)
        const uint32_t G = n <= 1024 ? 64u : n <= 4096 ? 16u : n <= 16384 ? 4u : 1u;
        const dim3 grid((uint32_t)((uint64_t(n) * G + kActBlock - 1) / kActBlock));
        if (G == 64)
            hipLaunchKernelGGL(k_actuate<64>, grid, dim3(kActBlock), 0, stream, dt, di, n, agents, actions,
                               collided, poses, P);
        else if (G == 16)
            hipLaunchKernelGGL(k_actuate<16>, grid, dim3(kActBlock), 0, stream, dt, di, n, agents, actions,
                               collided, poses, P);
        else if (G == 4)
            hipLaunchKernelGGL(k_actuate<4>, grid, dim3(kActBlock), 0, stream, dt, di, n, agents, actions,
                               collided, poses, P);
        else
            hipLaunchKernelGGL(k_actuate<1>, grid, dim3(kActBlock), 0, stream, dt, di, n, agents, actions,
                               collided, poses, P);
        HAB_HIP(hipGetLastError());
        HAB_HIP(hipEventRecord(ws.done, stream));
        ws.has_done = true;
        ws.last_stream = stream;
        return HAB_OK;
    });
}


hab_status hab_nav_from_scene(hab_context *ctx, const hab_scene *scene, const double *heights, uint32_t num_heights,
                              hipStream_t stream, hab_nav **out)
{
    if (!ctx || !scene || !out || !heights || num_heights == 0 || num_heights > HAB_NAV_MAX_HEIGHTS)
        return HAB_ERR_INVALID_ARG;
    *out = nullptr;
    for (uint32_t h = 0; h < num_heights; ++h)
        if (!std::isfinite(heights[h])) return HAB_ERR_INVALID_ARG;
    if (std::find(ctx->scenes.begin(), ctx->scenes.end(), static_cast<const Scene *>(scene)) == ctx->scenes.end())
        return HAB_ERR_INVALID_ARG;
    return guarded([&]() -> hab_status {
        DeviceGuard g(ctx->device);
        if (!g.ok) return HAB_ERR_DEVICE;
        const uint32_t T = scene->T;
        std::vector<float> segs;
        if (T) {
            SliceParams S{};
            for (uint32_t h = 0; h < num_heights; ++h) S.h[h] = heights[h];
            S.K = num_heights;
            const uint32_t nb = (T + kSliceBlock - 1) / kSliceBlock;
            uint32_t *dtot = nullptr;
            if (!dev_alloc((void **)&dtot, 8ull * nb)) return HAB_ERR_OUT_OF_MEMORY;
            uint32_t *dbase = dtot + nb;
            std::vector<uint32_t> tot(nb), base(nb);
            float4 *dseg = nullptr;
            auto fail = [&](hab_status st) {
                dev_free(dtot);
                if (dseg) dev_free(dseg);
                return st;
            };
            hipLaunchKernelGGL(k_slice_count, dim3(nb), dim3(kSliceBlock), 0, stream, scene->tpos, T, S, dtot);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(tot.data(), dtot, 4ull * nb, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                hipStreamSynchronize(stream) != hipSuccess)
                return fail(HAB_ERR_DEVICE);
            uint64_t nseg = 0;
            for (uint32_t b = 0; b < nb; ++b) {
                base[b] = (uint32_t)nseg;
                nseg += tot[b];
            }
            if (nseg >= (1ull << 31)) return fail(HAB_ERR_CAPACITY);
            if (nseg) {
                if (!dev_alloc((void **)&dseg, 16ull * nseg)) return fail(HAB_ERR_OUT_OF_MEMORY);
                segs.resize(4ull * nseg);
                if (hipMemcpyAsync(dbase, base.data(), 4ull * nb, hipMemcpyHostToDevice, stream) != hipSuccess)
                    return fail(HAB_ERR_DEVICE);
                hipLaunchKernelGGL(k_slice_write, dim3(nb), dim3(kSliceBlock), 0, stream, scene->tpos, T, S, dbase,
                                   dseg);
                if (hipGetLastError() != hipSuccess ||
                    hipMemcpyAsync(segs.data(), dseg, 16ull * nseg, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                    hipStreamSynchronize(stream) != hipSuccess)
                    return fail(HAB_ERR_DEVICE);
            }
            (void)fail(HAB_OK);
        }
        return nav_build(ctx, segs.data(), (uint32_t)(segs.size() / 4), out);
    });
}

hab_status hab_nav_segments(hab_context *ctx, const hab_nav *nav, float *out, uint32_t capacity, uint32_t *num_segments)
{
    if (!ctx || !nav || !num_segments || (capacity && !out)) return HAB_ERR_INVALID_ARG;
    return guarded([&]() -> hab_status {
        if (std::find(ctx->navs.begin(), ctx->navs.end(), nav) == ctx->navs.end()) return HAB_ERR_INVALID_ARG;
        *num_segments = nav->n;
        const uint32_t m = std::min(capacity, nav->n);
        if (!m) return HAB_OK;
        DeviceGuard g(ctx->device);
        if (!g.ok) return HAB_ERR_DEVICE;
        HAB_HIP(hipMemcpy(out, nav->d.seg, 16ull * m, hipMemcpyDeviceToHost));
        return HAB_OK;
    });
}

hab_status hab_nav_free(hab_context *ctx, const hab_nav *nav, const double *points, uint32_t n, double radius,
                        uint8_t *out_free, hipStream_t stream)
{
    if (!ctx || !nav || (n && (!points || !out_free))) return HAB_ERR_INVALID_ARG;
    if (!(radius > 0.0) || !std::isfinite(radius)) return HAB_ERR_INVALID_ARG;
    if (n == 0) return HAB_OK;
    return guarded([&]() -> hab_status {
        if (std::find(ctx->navs.begin(), ctx->navs.end(), nav) == ctx->navs.end()) return HAB_ERR_INVALID_ARG;
        DeviceGuard g(ctx->device);
        if (!g.ok) return HAB_ERR_DEVICE;
        hipLaunchKernelGGL(k_nav_free, dim3((n + kActBlock - 1) / kActBlock), dim3(kActBlock), 0, stream, nav->d,
                           reinterpret_cast<const double2 *>(points), n, radius, out_free);
        HAB_HIP(hipGetLastError());
        return HAB_OK;
    });
}

}  // extern "C"
