// extern "C" entry points: argument checks, device selection, no exceptions
// across the boundary.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "runtime.h"

using namespace habmi;


extern "C" {

const char *hab_status_string(hab_status s)
{
    switch (s) {
    case HAB_OK: return "ok";
    case HAB_ERR_INVALID_ARG: return "invalid argument";
    case HAB_ERR_OUT_OF_MEMORY: return "out of memory";
    case HAB_ERR_RANGE: return "outside the fixed-point domain";
    case HAB_ERR_DEVICE: return "device error";
    case HAB_ERR_NOT_READY: return "not ready";
    case HAB_ERR_CAPACITY: return "capacity exceeded";
    case HAB_ERR_CANCELLED: return "cancelled";
    case HAB_ERR_TIMEOUT: return "timed out";
    case HAB_STATUS_MAX_: break;
    }
    return "unknown status";
}

hab_status hab_init(int device, hab_context **out)
{
    if (!out) return HAB_ERR_INVALID_ARG;
    *out = nullptr;
    return guarded([&]() -> hab_status {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
            return HAB_ERR_INVALID_ARG;
        DeviceGuard g(device);
        if (!g.ok) return HAB_ERR_DEVICE;
        hab_context *ctx = new hab_context();
        ctx->device = device;
        ctx->ws.device = device;
        ctx->ws2.device = device;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
            ctx->cu_count = prop.multiProcessorCount;
        for (int lo = 0; lo < 2; ++lo)
            for (int c = 0; c < 3; ++c) ctx->raster_bpc[lo][c] = raster_blocks_per_cu(8 << c, lo != 0);
        if (!dev_alloc((void **)&ctx->err, 256)) {
            delete ctx;
            return HAB_ERR_OUT_OF_MEMORY;
        }
        if (hipMemset(ctx->err, 0, 256) != hipSuccess) {
            dev_free(ctx->err);
            delete ctx;
            return HAB_ERR_DEVICE;
        }
        const hab_status na = noalloc_setup(ctx);
        if (na != HAB_OK) {
            dev_free(ctx->err);
            delete ctx;   // frees whatever the reservation got (its staging slots)
            return na;
        }
        autotune_cache_load(ctx);
        *out = ctx;
        return HAB_OK;
    });
}

// Device memory of a scene (every pointer may be null).
static void free_scene_mem(Scene *s)
{
    dev_free(s->tpos);
    dev_free(s->col);
    dev_free(s->idx);
    dev_free(s->cbox);
    dev_free(s->inst);
    dev_free(s->uv);
    dev_free(s->tex);
}

hab_status hab_shutdown(hab_context *ctx)
{
    if (!ctx) return HAB_ERR_INVALID_ARG;
    return guarded([&]() -> hab_status {
        DeviceGuard g(ctx->device);
        (void)hipDeviceSynchronize();
        for (Scene *s : ctx->scenes) {
            free_scene_mem(s);
            delete static_cast<hab_scene *>(s);
        }
        ctx->scenes.clear();
        release_navs(ctx);
        for (auto &ps : ctx->prof_sets)
            for (auto &e : ps.ev) (void)hipEventDestroy(e);
        if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
        if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
        if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
        if (ctx->err) dev_free(ctx->err);
        delete ctx;
        return HAB_OK;
    });
}

hab_status hab_get_error(hab_context *ctx)
{
    if (!ctx) return HAB_ERR_INVALID_ARG;
    return guarded([&]() -> hab_status {
        DeviceGuard g(ctx->device);
        uint32_t e = 0;
        HAB_HIP(hipMemcpy(&e, ctx->err, 4, hipMemcpyDeviceToHost));
        if (e) HAB_HIP(hipMemset(ctx->err, 0, 4));
        if (e & kErrRange) return HAB_ERR_RANGE;
        return e ? HAB_ERR_DEVICE : HAB_OK;
    });
}

hab_status hab_scene_upload(hab_context *ctx, const hab_mesh_desc *m, hipStream_t stream,
                            hab_scene **out)
{
    if (!ctx || !m || !out) return HAB_ERR_INVALID_ARG;
    *out = nullptr;
    if (!m->positions || m->num_vertices == 0 || m->num_vertices >= (1u << 30)) return HAB_ERR_INVALID_ARG;
    if (m->num_triangles >= (1u << 30)) return HAB_ERR_INVALID_ARG;
    if (m->num_triangles && !m->indices) return HAB_ERR_INVALID_ARG;
    return guarded([&]() -> hab_status {
        const uint32_t V = m->num_vertices, T = m->num_triangles;
        for (uint64_t k = 0; k < 3ull * T; ++k)
            if (m->indices[k] >= V) return HAB_ERR_INVALID_ARG;
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (uint64_t k = 0; k < V; ++k)
            for (int a = 0; a < 3; ++a) {
                const float x = m->positions[3 * k + a];
                if (!std::isfinite(x)) return HAB_ERR_INVALID_ARG;
                lo[a] = std::min(lo[a], x);
                hi[a] = std::max(hi[a], x);
            }
        // bounding box of every 64 consecutive triangles (one setup wave):
        // exact float min/max of the vertex coordinates
        const uint32_t ncl = (T + kCluster - 1) / kCluster;
        std::vector<float4> cbox(2 * (size_t)std::max<uint32_t>(ncl, 1));
        for (uint32_t c = 0; c < ncl; ++c) {
            float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
            const uint32_t t1 = std::min<uint32_t>(T, (c + 1) * kCluster);
            for (uint32_t t = c * kCluster; t < t1; ++t)
                for (int k = 0; k < 3; ++k) {
                    const float *q = m->positions + 3ull * m->indices[3ull * t + k];
                    for (int a = 0; a < 3; ++a) {
                        mn[a] = std::min(mn[a], q[a]);
                        mx[a] = std::max(mx[a], q[a]);
                    }
                }
            cbox[2 * c] = make_float4(mn[0], mn[1], mn[2], 0.0f);
            cbox[2 * c + 1] = make_float4(mx[0], mx[1], mx[2], 0.0f);
        }
        // texture: both parts or neither, power-of-two sizes, coordinates
        // inside the range where u * tex_width keeps sub-texel precision
        const bool textured = m->uvs || m->texture;
        std::vector<uint32_t> texels;
        if (textured) {
            const uint32_t tw = m->tex_width, th = m->tex_height;
            const bool pow2 = tw && th && !(tw & (tw - 1)) && !(th & (th - 1));
            if (!m->uvs || !m->texture || !pow2 || tw > 16384 || th > 16384) return HAB_ERR_INVALID_ARG;
            for (uint64_t k = 0; k < V; ++k) {
                const double a = std::fabs((double)m->uvs[2 * k] * tw);
                const double b = std::fabs((double)m->uvs[2 * k + 1] * th);
                if (!(a < 4194304.0 && b < 4194304.0)) return HAB_ERR_INVALID_ARG;
            }
            texels.resize((size_t)tw * th);
            for (size_t k = 0; k < texels.size(); ++k)
                texels[k] = (uint32_t)m->texture[3 * k] | ((uint32_t)m->texture[3 * k + 1] << 8) |
                            ((uint32_t)m->texture[3 * k + 2] << 16);
        }
        std::vector<uint32_t> col(V);
        for (uint64_t k = 0; k < V; ++k) {
            if (m->colors)
                col[k] = (uint32_t)m->colors[3 * k] | ((uint32_t)m->colors[3 * k + 1] << 8) |
                         ((uint32_t)m->colors[3 * k + 2] << 16);
            else
                col[k] = 0xFFFFFFu;
        }
        DeviceGuard g(ctx->device);
        if (!g.ok) return HAB_ERR_DEVICE;
        hab_scene *s = new hab_scene();
        s->device = ctx->device;
        s->V = V;
        s->T = T;
        for (int a = 0; a < 3; ++a) {
            s->lo[a] = lo[a];
            s->hi[a] = hi[a];
        }
        // positions are stored per triangle (nine floats per triangle) so
        // that kernels load a triangle without the index -> position hop
        std::vector<float> tri(9 * (size_t)std::max<uint32_t>(T, 1), 0.0f);
        for (uint64_t t = 0; t < T; ++t)
            for (int k = 0; k < 3; ++k) {
                const float *q = m->positions + 3ull * m->indices[3ull * t + k];
                for (int a = 0; a < 3; ++a) tri[9 * t + 3 * k + a] = q[a];
            }
        const size_t bp = sizeof(float) * tri.size(), bc = 4ull * V, bi = std::max<size_t>(12ull * T, 12);
        const size_t bb = sizeof(float4) * cbox.size();
        const size_t bs = m->instances ? std::max<size_t>(4ull * T, 4) : 0;
        const size_t buv = textured ? 8ull * V : 0;
        const size_t btex = textured ? 4ull * m->tex_width * m->tex_height : 0;
        auto drop = [&]() {
            free_scene_mem(s);
            delete s;
        };
        bool ok = dev_alloc((void **)&s->tpos, bp) && dev_alloc((void **)&s->col, bc) &&
                  dev_alloc((void **)&s->idx, bi) && dev_alloc((void **)&s->cbox, bb) &&
                  (!bs || dev_alloc((void **)&s->inst, bs)) && (!buv || dev_alloc((void **)&s->uv, buv)) &&
                  (!btex || dev_alloc((void **)&s->tex, btex));
        if (!ok) {
            drop();
            return HAB_ERR_OUT_OF_MEMORY;
        }
        s->bytes = bp + bc + bi + bb + bs + buv + btex;
        if (textured) {
            s->tw = m->tex_width;
            s->th = m->tex_height;
        }
        hipError_t e = hipMemcpyAsync(s->tpos, tri.data(), bp, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(s->col, col.data(), bc, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess && T)
            e = hipMemcpyAsync(s->idx, m->indices, 12ull * T, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(s->cbox, cbox.data(), bb, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess && bs && T)
            e = hipMemcpyAsync(s->inst, m->instances, 4ull * T, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess && buv) e = hipMemcpyAsync(s->uv, m->uvs, buv, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess && btex)
            e = hipMemcpyAsync(s->tex, texels.data(), btex, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            drop();
            return HAB_ERR_DEVICE;
        }
        ctx->scenes.push_back(s);
        *out = s;
        return HAB_OK;
    });
}

hab_status hab_scene_release(hab_context *ctx, hab_scene *scene)
{
    if (!ctx || !scene) return HAB_ERR_INVALID_ARG;
    return guarded([&]() -> hab_status {
        auto it = std::find(ctx->scenes.begin(), ctx->scenes.end(), static_cast<Scene *>(scene));
        if (it == ctx->scenes.end()) return HAB_ERR_INVALID_ARG;
        DeviceGuard g(ctx->device);
        // work that still reads the scene must finish first
        HAB_HIP(hipDeviceSynchronize());
        free_scene_mem(scene);
        ctx->scenes.erase(it);
        delete scene;
        return HAB_OK;
    });
}

hab_status hab_scene_info(const hab_scene *s, uint32_t *nv, uint32_t *nt, uint64_t *bytes,
                          float lo[3], float hi[3])
{
    if (!s) return HAB_ERR_INVALID_ARG;
    if (nv) *nv = s->V;
    if (nt) *nt = s->T;
    if (bytes) *bytes = s->bytes;
    for (int a = 0; a < 3; ++a) {
        if (lo) lo[a] = s->lo[a];
        if (hi) hi[a] = s->hi[a];
    }
    return HAB_OK;
}

hab_status hab_sensor_spec(const hab_sensor_desc *d, hab_sensor *out)
{
    if (!d || !out) return HAB_ERR_INVALID_ARG;
    if (d->width == 0 || d->height == 0 || d->width > HAB_MAX_DIM || d->height > HAB_MAX_DIM)
        return HAB_ERR_INVALID_ARG;
    if (!(d->hfov_deg > 0.0f && d->hfov_deg < 180.0f)) return HAB_ERR_INVALID_ARG;
    const float near_m = d->near_m == 0.0f ? 0.01f : d->near_m;
    if (!(near_m > 0.0f) || !std::isfinite(near_m)) return HAB_ERR_INVALID_ARG;
    const uint32_t outputs = d->outputs ? d->outputs : (HAB_OUT_RGB | HAB_OUT_DEPTH);
    if (outputs & ~(uint32_t)(HAB_OUT_RGB | HAB_OUT_DEPTH | HAB_OUT_TRI | HAB_OUT_SEMANTIC))
        return HAB_ERR_INVALID_ARG;
    if (!(d->depth_noise_sigma >= 0.0f) || !std::isfinite(d->depth_noise_sigma)) return HAB_ERR_INVALID_ARG;
    hab_sensor s;
    s.width = d->width;
    s.height = d->height;
    s.outputs = outputs;
    s.hfov_deg = d->hfov_deg;
    s.f = (float)((double)d->width / (2.0 * std::tan((double)d->hfov_deg * 3.14159265358979323846 / 360.0)));
    s.near_m = near_m;
    s.depth_noise_sigma = d->depth_noise_sigma;
    if (!(s.f > 0.0f) || !std::isfinite(s.f)) return HAB_ERR_INVALID_ARG;
    *out = s;
    return HAB_OK;
}

static hab_status render_common(hab_context *ctx, const hab_scene *scene, const hab_sensor *sensor,
                                const hab_pose *poses, uint32_t n, uint8_t *rgb, float *depth,
                                uint32_t *tri, const hab_render_opts *opts, hipStream_t stream)
{
    if (!ctx || !scene || !sensor || (!poses && n)) return HAB_ERR_INVALID_ARG;
    if (n == 0) return HAB_OK;
    hab_status st = validate_sensor(sensor);
    if (st != HAB_OK) return st;
    if (opts && opts->tile_size && opts->tile_size != 8 && opts->tile_size != 16 && opts->tile_size != 32)
        return HAB_ERR_INVALID_ARG;
    if (opts && (opts->bin_factor < 0.0f || (opts->flags & ~HAB_RENDER_FLAGS))) return HAB_ERR_INVALID_ARG;
    return guarded([&]() -> hab_status {
        std::vector<ViewReq> req(n);
        const size_t px = (size_t)sensor->width * sensor->height;
        for (uint32_t k = 0; k < n; ++k) {
            hab_status s2 = validate_pose(scene, sensor, &poses[k]);
            if (s2 != HAB_OK) return s2;
            ViewReq &r = req[k];
            r.scene = scene;
            r.sensor = *sensor;
            r.pose = poses[k];
            r.rgb = (rgb && (sensor->outputs & HAB_OUT_RGB)) ? rgb + 3 * px * k : nullptr;
            r.depth = (depth && (sensor->outputs & HAB_OUT_DEPTH)) ? depth + px * k : nullptr;
            r.tri = tri ? tri + px * k : nullptr;
            r.noise_seed = k;
        }
        PlanOpts o;
        if (opts) {
            o.tile_size = opts->tile_size;
            o.bin_factor = opts->bin_factor;
            o.tile_cap = opts->tile_cap;
            o.one_sequence = (opts->flags & HAB_RENDER_ONE_SEQUENCE) != 0;
            o.lane_owned_z = (opts->flags & HAB_RENDER_LANE_OWNED_Z) != 0;
        }
        DeviceGuard g(ctx->device);
        if (!g.ok) return HAB_ERR_DEVICE;
        return render_split(ctx, req.data(), n, o, stream, opts ? opts->stats : nullptr);
    });
}

hab_status hab_render(hab_context *ctx, const hab_scene *scene, const hab_sensor *sensor,
                      const hab_pose *poses, uint32_t num_poses, uint8_t *out_rgb, float *out_depth,
                      hipStream_t stream)
{
    return render_common(ctx, scene, sensor, poses, num_poses, out_rgb, out_depth, nullptr, nullptr,
                         stream);
}

hab_status hab_render_ex(hab_context *ctx, const hab_scene *scene, const hab_sensor *sensor,
                         const hab_pose *poses, uint32_t num_poses, uint8_t *out_rgb,
                         float *out_depth, uint32_t *out_tri, const hab_render_opts *opts,
                         hipStream_t stream)
{
    return render_common(ctx, scene, sensor, poses, num_poses, out_rgb, out_depth, out_tri, opts,
                         stream);
}

hab_status hab_render_batch(hab_context *ctx, const hab_view *views, uint32_t n,
                            const hab_render_opts *opts, hipStream_t stream)
{
    if (!ctx || (!views && n)) return HAB_ERR_INVALID_ARG;
    if (n == 0) return HAB_OK;
    if (opts && opts->tile_size && opts->tile_size != 8 && opts->tile_size != 16 && opts->tile_size != 32)
        return HAB_ERR_INVALID_ARG;
    if (opts && (opts->bin_factor < 0.0f || (opts->flags & ~HAB_RENDER_FLAGS))) return HAB_ERR_INVALID_ARG;
    return guarded([&]() -> hab_status {
        std::vector<ViewReq> req(n);
        for (uint32_t k = 0; k < n; ++k) {
            hab_status s2 = to_view_req(views[k], req[k]);
            if (s2 != HAB_OK) return s2;
        }
        PlanOpts o;
        if (opts) {
            o.tile_size = opts->tile_size;
            o.bin_factor = opts->bin_factor;
            o.tile_cap = opts->tile_cap;
            o.one_sequence = (opts->flags & HAB_RENDER_ONE_SEQUENCE) != 0;
            o.lane_owned_z = (opts->flags & HAB_RENDER_LANE_OWNED_Z) != 0;
        }
        DeviceGuard g(ctx->device);
        if (!g.ok) return HAB_ERR_DEVICE;
        return render_split(ctx, req.data(), n, o, stream, opts ? opts->stats : nullptr);
    });
}

hab_status hab_profile_enable(hab_context *ctx, int on)
{
    if (!ctx) return HAB_ERR_INVALID_ARG;
    ctx->prof_on = on != 0;
    return HAB_OK;
}

hab_status hab_profile_phases(hab_context *ctx, uint32_t phase_mask)
{
    if (!ctx || !(phase_mask & ((1u << HAB_NUM_PHASES) - 1u))) return HAB_ERR_INVALID_ARG;
    ctx->prof_phase_mask = phase_mask & ((1u << HAB_NUM_PHASES) - 1u);
    return HAB_OK;
}

hab_status hab_profile_read(hab_context *ctx, hab_phase_times *out)
{
    if (!ctx || !out) return HAB_ERR_INVALID_ARG;
    return guarded([&]() -> hab_status {
        DeviceGuard g(ctx->device);
        std::memset(out, 0, sizeof *out);
        for (size_t k = 0; k < ctx->prof_used; ++k) {
            const hab_context::ProfSet &ps = ctx->prof_sets[k];
            for (int ph = 0; ph < HAB_NUM_PHASES; ++ph) {
                if (!(ps.mask & (1u << ph))) continue;
                HAB_HIP(hipEventSynchronize(ps.ev[2 * ph + 1]));
                float ms = 0.0f;
                HAB_HIP(hipEventElapsedTime(&ms, ps.ev[2 * ph], ps.ev[2 * ph + 1]));
                out->ms[ph] += ms;
                out->launches[ph] += 1;
            }
        }
        out->sequences = ctx->prof_used;
        ctx->prof_used = 0;
        return HAB_OK;
    });
}

hab_status hab_selfcheck_reciprocal(hab_context *ctx, uint32_t lo_bits, uint32_t hi_bits, hipStream_t stream,
                                    uint64_t *mismatches)
{
    if (!ctx || !mismatches || lo_bits >= hi_bits || hi_bits > 0x7F800000u) return HAB_ERR_INVALID_ARG;
    return guarded([&]() -> hab_status {
        DeviceGuard g(ctx->device);
        if (!g.ok) return HAB_ERR_DEVICE;
        unsigned long long *d = nullptr;
        if (!dev_alloc((void **)&d, sizeof *d)) return HAB_ERR_OUT_OF_MEMORY;
        unsigned long long h = 0;
        hipError_t e = hipMemsetAsync(d, 0, sizeof *d, stream);
        if (e == hipSuccess) e = launch_check_recip(lo_bits, hi_bits, d, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof h, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        dev_free(d);
        if (e != hipSuccess) return HAB_ERR_DEVICE;
        *mismatches = h;
        return HAB_OK;
    });
}

hab_status hab_test_fail_alloc(int64_t after)
{
    alloc_fail_after(after < 0 ? -1 : after);
    return HAB_OK;
}

hab_status hab_test_live_allocations(uint64_t *count, uint64_t *bytes)
{
    if (!count || !bytes) return HAB_ERR_INVALID_ARG;
    alloc_live(count, bytes);
    return HAB_OK;
}

}  // extern "C"
