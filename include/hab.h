/*
 * hab.h -- C ABI of the MI355X (gfx950) RGB + depth sensor renderer.
 *
 * The library renders colour and depth observations of static triangle
 * meshes from camera poses, the sensor model of the Habitat simulator
 * (arXiv:1904.01201): Sec. 3 "Design overview" (the simulator returns the
 * sensory data of an agent's sensors), Sec. 3 "Rendering engine" (one pass
 * produces colour, depth and the per-pixel visible triangle), Sec. 4
 * "Sensory input" (pinhole sensor with a resolution and a field of view,
 * depth sharing the colour sensor's pose and intrinsics), Appendix A "Key
 * abstractions" (given the agents' state the Simulator provides the
 * observations of all active sensors) and Sec. 3 "Efficient GPU
 * throughput" (frames handed to the learning framework as GPU tensors,
 * without a copy through host memory).
 *
 * Rendering definition (identical for every entry point, batch size, tile
 * size or bin capacity):
 *   - world is right-handed, metres, +Y up; a pose is the camera position
 *     p[3] and the row-major world-from-camera rotation R[9]; the camera
 *     looks along its -Z axis with +Y up and +X right;
 *   - f = W / (2 tan(hfov/2)) px (rounded once to fp32), principal point at
 *     (W/2, H/2), pixel (i, j) centred at (i + 1/2, j + 1/2), row 0 on top;
 *   - geometry with planar depth w < near is clipped away (no far plane);
 *   - vertices snap to 1/256 px (round half to even); coverage uses edge
 *     functions with the top-left fill rule; both faces are drawn;
 *   - the visible triangle has the largest interpolated 1/w, ties going to
 *     the smaller triangle index; depth is planar (distance along the view
 *     axis) in metres; colour is the perspective-correct interpolation of
 *     the vertex colours rounded to uint8;
 *   - no hit: depth 0, colour (0, 0, 0), triangle index HAB_NO_HIT.
 * The same pass can also write the semantic instance mask, shade from a
 * texture instead of the vertex colours, and add depth noise (see
 * hab_mesh_desc and hab_sensor_desc); hab_actuate moves agents (turns and
 * forward moves with collide-and-slide) and writes the camera poses that
 * hab_stepper_step_device renders from.
 *
 * Memory: every output pointer is caller-owned device memory, contiguous,
 * row-major: rgb [N][H][W][3] uint8, depth [N][H][W] float, tri and
 * semantic [N][H][W] uint32.  The library never keeps an output pointer
 * after the call returns, except inside a stepper (which keeps the
 * pointers it was created with until it is destroyed).  Host arrays passed
 * in are read during the call only; device inputs (agent states, actions,
 * device poses) are read when the enqueued work runs.
 *
 * Errors: every function returns a hab_status; nothing throws across the
 * boundary.  Argument errors are detected before any work is enqueued.
 * Rendering is asynchronous on the given HIP stream; a device-side fault
 * report (a vertex outside the fixed-point range: unreachable for poses
 * checked on the host, possible for device poses) is sticky and read with
 * hab_get_error after synchronising.
 *
 * Threading: a context is externally synchronised (one thread at a time);
 * scenes are immutable after upload and may be used by any stream.  Work
 * enqueued through one context on different streams is ordered by the
 * context (each call waits for the previous call's use of the context's
 * scratch memory).
 */
#ifndef HAB_H
#define HAB_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HAB_OK = 0,
    HAB_ERR_INVALID_ARG = 1,   /* bad pointer, size, index, sensor or pose          */
    HAB_ERR_OUT_OF_MEMORY = 2, /* device or pinned host allocation failed           */
    HAB_ERR_RANGE = 3,         /* pose/scene outside the fixed-point domain          */
    HAB_ERR_DEVICE = 4,        /* a HIP call failed                                  */
    HAB_ERR_NOT_READY = 5,     /* poll: the request has not completed yet            */
    HAB_ERR_CAPACITY = 6,      /* queue full, request over budget, or beyond a limit */
    HAB_ERR_CANCELLED = 7,     /* server: the request was cancelled before launch    */
    HAB_ERR_TIMEOUT = 8,       /* server: the request was not launched by its deadline */
    HAB_STATUS_MAX_ = 0x7FFFFFFF /* (not a status: makes every non-negative int a valid value) */
} hab_status;

#define HAB_NO_HIT 0xFFFFFFFFu
#define HAB_MAX_DIM 4096u

/* Outputs of a sensor.  HAB_OUT_SEMANTIC: the instance id of the visible
 * triangle (the semantic attachment of the paper's single render pass,
 * Sec. 3 "Rendering engine"), from the scene's per-triangle instance table. */
enum { HAB_OUT_RGB = 1, HAB_OUT_DEPTH = 2, HAB_OUT_TRI = 4, HAB_OUT_SEMANTIC = 8 };

typedef struct hab_context hab_context;
typedef struct hab_scene hab_scene;
typedef struct hab_stepper hab_stepper;
typedef struct hab_server hab_server;

/* Triangle mesh on the host.  positions [V][3] float (metres), colors
 * [V][3] uint8 RGB (NULL: all white), indices [T][3] uint32 (each < V),
 * instances [T] uint32 instance id per triangle (NULL: the scene has no
 * semantic table and cannot feed HAB_OUT_SEMANTIC).  1 <= V < 2^30,
 * T < 2^30 (HAB_ERR_INVALID_ARG otherwise).
 *
 * Texture (scanned scenes are textured meshes, Sec. 4 "Episode dataset
 * preparation"): uvs [V][2] float and texture [tex_height][tex_width][3]
 * uint8 RGB, both or neither.  With a texture the colour output is the
 * texture, not the vertex colours: texture coordinates are interpolated
 * perspective-correctly like the colours (the same fp32 sequence, through
 * the near clip), then fetched bilinearly with texel centres at
 * ((k + 1/2) / tex_width, (l + 1/2) / tex_height), v = 0 at the first row,
 * coordinates repeating.  tex_width and tex_height are powers of two in
 * [1, 16384] and every vertex has |u| tex_width, |v| tex_height < 2^22
 * (HAB_ERR_INVALID_ARG otherwise). */
typedef struct {
    const float *positions;
    uint32_t num_vertices;
    const uint8_t *colors;
    const uint32_t *indices;
    uint32_t num_triangles;
    const uint32_t *instances;
    const float *uvs;
    const uint8_t *texture;
    uint32_t tex_width, tex_height;
} hab_mesh_desc;

/* Sensor request.  width, height in [1, 4096]; hfov_deg in (0, 180);
 * near_m > 0 (0 selects the default 0.01 m); outputs = OR of HAB_OUT_*
 * (0 selects RGB | DEPTH).
 *
 * depth_noise_sigma (1/m, finite, >= 0; 0 = the ideal depth sensor): the
 * noisy depth of the appendix's noise study ("Noisy Depth"): iid Gaussian
 * noise of standard deviation sigma added to each pixel's inverse depth,
 * rho' = rho + sigma n; the depth output is 1/rho' where rho' > 0 and 0
 * where rho' <= 0 or nothing is visible.  n is drawn per pixel from
 * Philox4x64-10 (Salmon et al., SC 2011) with key (view noise seed,
 * 0x6465707468) and counter (j W + i, 0, 0, 0): u1 = ((x0 >> 40) + 1) 2^-24,
 * u2 = (x1 >> 40) 2^-24, n = sqrt(-2 ln u1) cos(2 pi u2) (Box-Muller),
 * evaluated in fp32.  The seed comes with each view (hab_view.noise_seed). */
typedef struct {
    uint32_t width, height;
    float hfov_deg;
    float near_m;
    uint32_t outputs;
    float depth_noise_sigma;
} hab_sensor_desc;

/* Validated sensor (plain data, filled by hab_sensor_spec). */
typedef struct {
    uint32_t width, height, outputs;
    float hfov_deg;
    float f;       /* focal length in px, fp32 */
    float near_m;
    float depth_noise_sigma;
} hab_sensor;

/* Camera pose: world_from_camera.  position in metres, rotation row-major,
 * orthonormal to 1e-4 (max |R^T R - I|). */
typedef struct {
    float position[3];
    float rotation[9];
} hab_pose;

/* Per-view work-counters, filled on request (hab_render_opts.stats):
 * survivors = sub-triangles whose snapped bounding box meets the viewport,
 * bbox_tests = pixel centres inside those boxes, covered = (sub-triangle,
 * pixel) pairs that pass the coverage test. */
typedef struct {
    uint64_t survivors;
    uint64_t bbox_tests;
    uint64_t covered;
} hab_view_stats;

/* Launch options.  Zero-initialised = defaults.  tile_size in {0, 8, 16,
 * 32} (0: autotuned/default); bin_factor: per-view bin capacity as a
 * multiple of the triangle count (0: default); tile_cap: entries a tile
 * list may hold before the tile takes the overflow path (0: unlimited);
 * flags: HAB_RENDER_* bits (others: HAB_ERR_INVALID_ARG).  None of these
 * changes any output bit.
 *
 * A batch of 32 or more views is rendered as two launch sequences over
 * interleaved halves (views 0, 2, 4, ... and 1, 3, 5, ...): one on the
 * caller's stream, one on a second stream of the context that waits for the
 * caller's stream first, and the caller's stream then waits for it, so the
 * call orders like one launch on the caller's stream.  The halves' kernels
 * overlap on the GPU.  HAB_RENDER_ONE_SEQUENCE keeps the batch in one
 * launch sequence. */
#define HAB_RENDER_ONE_SEQUENCE 1u
/* Test each pixel in the lane that owns it for the whole tile, keeping its
 * nearest fragment in that lane's registers: the atomic-free z-test (one
 * record per pixel block per step, so a step lasts as long as the busiest
 * block's list).  By default a wave deals (triangle, pixel block) pairs to
 * its lane groups evenly and merges each pixel's nearest fragment in LDS by
 * an atomic 64-bit max, the same order-free rule.  Outputs are identical. */
#define HAB_RENDER_LANE_OWNED_Z 2u
#define HAB_RENDER_FLAGS (HAB_RENDER_ONE_SEQUENCE | HAB_RENDER_LANE_OWNED_Z)
typedef struct {
    uint32_t tile_size;
    float bin_factor;
    uint32_t tile_cap;
    uint32_t flags;
    hab_view_stats *stats; /* host array [N] or NULL; written after completion */
} hab_render_opts;

/* One view of a heterogeneous batch: any scene, any sensor, own outputs
 * (device pointers sized for that sensor; NULL for unwanted outputs).
 * out_semantic ([H][W] uint32, HAB_NO_HIT where nothing is visible) is
 * written when the sensor has HAB_OUT_SEMANTIC; the scene must then have an
 * instance table (else HAB_ERR_INVALID_ARG).  noise_seed keys the depth
 * noise of a sensor with depth_noise_sigma > 0 (the same seed and pose give
 * the same noise; vary it per frame for fresh noise). */
typedef struct {
    const hab_scene *scene;
    const hab_sensor *sensor;
    hab_pose pose;
    uint8_t *out_rgb;
    float *out_depth;
    uint32_t *out_tri;
    uint32_t *out_semantic;
    uint64_t noise_seed;
} hab_view;

/* ---------------------------------------------------------- lifetime */
/* Create a context on HIP device `device` (its ordinal). */
hab_status hab_init(int device, hab_context **out);
/* Synchronise and free everything the context owns (scenes and obstacle
 * sets included). */
hab_status hab_shutdown(hab_context *ctx);
const char *hab_status_string(hab_status s);
/* Sticky device-side error of this context (HAB_OK if none); call after
 * the stream has been synchronised.  Reading it clears it. */
hab_status hab_get_error(hab_context *ctx);

/* ---------------------------------------------------------- scenes */
/* Copy a mesh into device memory (HBM-resident until released).  The host
 * arrays may be freed when the call returns (the copy is synchronous with
 * respect to the host).  Fails with HAB_ERR_INVALID_ARG on an index >= V,
 * a non-finite position, V == 0 or T >= 2^30. */
hab_status hab_scene_upload(hab_context *ctx, const hab_mesh_desc *mesh, hipStream_t stream,
                            hab_scene **out);
hab_status hab_scene_release(hab_context *ctx, hab_scene *scene);
/* Device bytes held by a scene, its counts and its bounding box. */
hab_status hab_scene_info(const hab_scene *scene, uint32_t *num_vertices,
                          uint32_t *num_triangles, uint64_t *device_bytes, float bbox_lo[3],
                          float bbox_hi[3]);

/* ---------------------------------------------------------- sensors */
/* Validate a sensor request and fill the plain-data sensor. */
hab_status hab_sensor_spec(const hab_sensor_desc *desc, hab_sensor *out);

/* ---------------------------------------------------------- rendering */
/* Render num_poses views of one scene with one sensor.  poses: host array.
 * out_rgb / out_depth: device [N][H][W][3] uint8 / [N][H][W] float, or
 * NULL.  Poses outside the fixed-point domain of this scene and sensor
 * fail with HAB_ERR_RANGE before anything is enqueued. */
hab_status hab_render(hab_context *ctx, const hab_scene *scene, const hab_sensor *sensor,
                      const hab_pose *poses, uint32_t num_poses, uint8_t *out_rgb,
                      float *out_depth, hipStream_t stream);
/* As hab_render, plus the visible-triangle output (device [N][H][W]
 * uint32 or NULL) and options (NULL = defaults).  With opts->stats set
 * the call synchronises the stream before returning.  hab_render and
 * hab_render_ex have no semantic output: they ignore HAB_OUT_SEMANTIC
 * (hab_view carries it, for hab_render_batch, the stepper and the server).
 * Their depth noise seed is the pose index k. */
hab_status hab_render_ex(hab_context *ctx, const hab_scene *scene, const hab_sensor *sensor,
                         const hab_pose *poses, uint32_t num_poses, uint8_t *out_rgb,
                         float *out_depth, uint32_t *out_tri, const hab_render_opts *opts,
                         hipStream_t stream);
/* Render a heterogeneous batch (different scenes, resolutions and output
 * sets) in one launch sequence.  Views are ordered by scene, so the views
 * of one scene read its geometry while it is in cache. */
hab_status hab_render_batch(hab_context *ctx, const hab_view *views, uint32_t num_views,
                            const hab_render_opts *opts, hipStream_t stream);
/* hab_render for callers that cannot allocate memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * arguments, kernels and outputs as hab_render (default options; depth
 * noise seed = pose index), but the launch's scratch memory is one static
 * device array of 64 MiB per GPU, held from the library's load until the
 * process ends, and the pinned staging and host planning buffers are
 * reserved by hab_init.  The call allocates no device, pinned or host
 * memory.
 *
 * Limits: num_poses <= 256 and the launch's scratch (about 50 MB for one
 * 256x256 view of a 1M-triangle scene at the largest tuned capacity) must
 * fit the array: beyond either, HAB_ERR_CAPACITY before anything is
 * enqueued.  Every call on one GPU shares that GPU's array (whatever the
 * context) and finds it holding the previous call's contents (each launch
 * clears what must start at zero itself); calls that overlap on one GPU
 * race, so order them (e.g. one stream, or events between streams).
 * Outputs, poses and errors as hab_render. */
hab_status hab_render_noalloc(hab_context *ctx, const hab_scene *scene, const hab_sensor *sensor,
                              const hab_pose *poses, uint32_t num_poses, uint8_t *out_rgb,
                              float *out_depth, hipStream_t stream);

/* ---------------------------------------------------------- actuation */
/* The agent step before rendering (Sec. 4 "Agent embodiment and action
 * space", "Collision dynamics"): an agent is a vertical cylinder (a disc of
 * radius r on the floor plane) that stops, turns left or right, or moves
 * forward in a continuous state space; a forward move that meets an
 * obstacle makes partial or no progress and may slide along it.
 *
 * Obstacles are line segments on the floor plane (x0, z0, x1, z1), made
 * once per scene: from the scene's own mesh (hab_nav_from_scene) or given
 * by the caller (hab_nav_upload). */
typedef struct hab_nav hab_nav;

/* segments: host [num_segments][4] float, metres (finite; a zero-length
 * segment is a point obstacle); num_segments may be 0.  The segments are
 * copied. */
hab_status hab_nav_upload(hab_context *ctx, const float *segments, uint32_t num_segments,
                          hab_nav **out);

/* Obstacles from the scene's own geometry, so that agents collide with what
 * is rendered (Sec. 4 "Collision dynamics": the agent slides along the
 * scene's walls and obstacles; the paper gives no navigability
 * representation).  The obstacles are the mesh's horizontal cross-sections
 * at num_heights (1..HAB_NAV_MAX_HEIGHTS) heights across the agent's body
 * (heights: host array, metres, finite; e.g. 0.1 and 1.5 for the paper's
 * 1.5 m agent: just above the floor, where every piece of furniture
 * stands, and its top): for each triangle in index order and each height h
 * in the given order, a vertex is above when its y >= h; when the three
 * vertices are not all on one side, the two edges (walked v0->v1, v1->v2,
 * v2->v0) that change side are cut at y = h by interpolating from the
 * edge's lower end to its upper end, s = (h - lo.y) / (hi.y - lo.y),
 * x = lo.x + s (hi.x - lo.x) (z alike), and the segment from the first cut
 * to the second is one obstacle, computed in fp64 and rounded once to fp32
 * per coordinate.  The cross-sections are computed on the device from the
 * scene's resident geometry (one kernel pass counting, one writing); the
 * lookup grid is built as by hab_nav_upload.  Synchronous with respect to
 * the host (stream is used for the kernels and copies). */
#define HAB_NAV_MAX_HEIGHTS 16
hab_status hab_nav_from_scene(hab_context *ctx, const hab_scene *scene, const double *heights,
                              uint32_t num_heights, hipStream_t stream, hab_nav **out);
/* Copy an obstacle set's segments (in their order) to host [capacity][4]
 * floats; *num_segments gets the set's count (the first capacity are
 * written).  Synchronous. */
hab_status hab_nav_segments(hab_context *ctx, const hab_nav *nav, float *out, uint32_t capacity,
                            uint32_t *num_segments);
hab_status hab_nav_release(hab_context *ctx, hab_nav *nav);

/* Free-space query (navigability, Sec. 4 "Agent embodiment and action
 * space"): out_free[i] = 1 when a disc of radius at points[i] = (x, z) is
 * clear of every segment of nav (each at least radius away: with
 * e = b - a, L2 = |e|^2, s = ((p - a).e) / L2 clamped to [0, 1] (0 when
 * L2 = 0), q = a + s e - p, blocked when |q|^2 < radius^2; fp64), else 0.
 * points: device [n][2] double; out_free: device [n] uint8; radius > 0 and
 * finite.  Asynchronous on the stream. */
hab_status hab_nav_free(hab_context *ctx, const hab_nav *nav, const double *points, uint32_t n,
                        double radius, uint8_t *out_free, hipStream_t stream);

/* Agent state: position on the floor plane and the unit forward vector
 * (yaw 0 looks along -z: (fx, fz) = (-sin yaw, -cos yaw)). */
typedef struct {
    double x, z;
    double fx, fz;
} hab_agent;

enum { HAB_ACT_STOP = 0, HAB_ACT_FORWARD = 1, HAB_ACT_LEFT = 2, HAB_ACT_RIGHT = 3 };

/* radius > 0 (the paper's agent: 0.1 m), forward_m >= 0 (0.25 m), and the
 * rotation of one turn, (turn_cos, turn_sin) = (cos, sin) of the turn angle
 * (10 degrees), all finite. */
typedef struct {
    double radius;
    double forward_m;
    double turn_cos, turn_sin;
} hab_actuation;

/* Apply one action to each of num_agents agents, in fp64:
 *   - left / right: (fx, fz) <- (fx c + fz s, fz c - fx s), s = +-turn_sin;
 *   - forward: the motion D = forward_m (fx, fz) runs through at most 4
 *     passes of collide-and-slide against the agent's segments: the earliest
 *     contact time t in [0, 1] at which the moving disc reaches distance
 *     radius from a segment while approaching it (its interior or an
 *     endpoint; earliest t, then lower segment index, then interior before
 *     first before second endpoint); without one the disc moves by D; with
 *     one it moves by max(0, t - 1e-6 / |D|) D, the rest of the motion loses
 *     its component along the contact normal and the next pass continues
 *     with it; motion left after the last pass is dropped;
 *   - stop, and any action value above 3: no change.
 * navs: host array [num_agents], the obstacles of each agent's scene.
 * agents [num_agents] (in/out), actions [num_agents] uint8, collided
 * [num_agents] uint8 (1 when a forward move met an obstacle; or NULL) and
 * poses [num_agents][12] float (the camera pose after the step: position
 * (x, camera_height, z), rotation with columns right (-fz, 0, fx), up and
 * back (-fx, 0, -fz); or NULL) are device pointers; the call is
 * asynchronous on the stream. */
hab_status hab_actuate(hab_context *ctx, const hab_nav *const *navs, uint32_t num_agents,
                       hab_agent *agents, const uint8_t *actions, uint8_t *collided,
                       float *poses, float camera_height, const hab_actuation *params,
                       hipStream_t stream);

/* ---------------------------------------------------------- stepper */
/* A fixed batch composition captured once as a HIP graph.  Each step
 * takes new poses (host array [num_views]), validates them, stages them
 * in pinned memory and replays the graph on the stream.  The views'
 * output pointers are those given at creation.  Step s (counted from 0 at
 * creation) renders view k with depth noise seed views[k].noise_seed + s. */
hab_status hab_stepper_create(hab_context *ctx, const hab_view *views, uint32_t num_views,
                              const hab_render_opts *opts, hipStream_t stream,
                              hab_stepper **out);
hab_status hab_stepper_step(hab_stepper *st, const hab_pose *poses, hipStream_t stream);
/* As hab_stepper_step with the poses already on the device: poses is a
 * device array [num_views][12] float (position, then the row-major
 * rotation, in the order of the views given at creation), e.g. the poses
 * output of hab_actuate, so an agent step and its render run without a host
 * round trip.  The poses are read when the step runs on the stream, so
 * they must stay valid (and unchanged) until then.  No host-side pose check
 * is possible: a pose whose scene leaves the fixed-point domain drops the
 * affected triangles and sets the sticky HAB_ERR_RANGE bit of hab_get_error
 * instead. */
hab_status hab_stepper_step_device(hab_stepper *st, const float *poses, hipStream_t stream);
hab_status hab_stepper_destroy(hab_stepper *st);

/* ---------------------------------------------------------- serving */
typedef struct {
    uint32_t num_streams;      /* concurrent batches in flight (default 2)       */
    uint32_t max_batch;        /* views per launched batch (default 256)         */
    uint64_t memory_budget;    /* scratch bytes for admitted work (default 8 GiB) */
    uint32_t max_queue;        /* queued requests before submit refuses (64k)    */
    uint32_t max_wait_us;      /* how long the batcher waits to fill a batch (0) */
} hab_server_cfg;

typedef struct {
    uint64_t submit_ns;   /* host clock (CLOCK_MONOTONIC) at submit   */
    uint64_t launch_ns;   /* batch launched                           */
    uint64_t done_ns;     /* completion observed                      */
    uint32_t batch_size;  /* views in the batch this request rode in  */
    uint32_t batch_id;
} hab_request_stats;

typedef struct {
    uint64_t submitted, completed, batches, rejected;
    uint64_t peak_inflight_bytes;   /* largest footprint of the batches in flight at once */
    uint32_t peak_batch;
    uint32_t pad;
    uint64_t cancelled, expired;    /* requests cancelled / timed out before launch */
    uint64_t scratch_bytes;         /* device scratch the server holds (= memory_budget) */
} hab_server_stats;

/* Start the request loop (one host thread) on a context the caller then
 * no longer uses directly until hab_server_destroy.  The server's device
 * scratch is one allocation of memory_budget bytes made here; every batch
 * works in a region of it, so the budget bounds the memory held.
 *
 * Admission (deterministic, in arrival order): a request's footprint is an
 * upper bound of its launch scratch (survivor and setup-record slots, tile
 * lists, work items and partial results for its scene, sensor and tile
 * size); a batch takes queued requests in order, among the first 64, while
 * their summed footprint fits the largest free region of the scratch; a
 * request passed over by 8 launched batches blocks those behind it until
 * it is admitted (it waits at most for the batches in flight). */
hab_status hab_server_create(hab_context *ctx, const hab_server_cfg *cfg, hab_server **out);
/* Non-blocking: queue one view (its pointers must stay valid until the
 * request completes).  Returns a ticket.  HAB_ERR_CAPACITY when the queue
 * is full or the request's footprint exceeds the budget. */
hab_status hab_server_submit(hab_server *srv, const hab_view *view, uint64_t *ticket);
/* As hab_server_submit with a deadline: a request not launched within
 * timeout_us microseconds of submission is dropped and its ticket reports
 * HAB_ERR_TIMEOUT (0: no deadline). */
hab_status hab_server_submit_ex(hab_server *srv, const hab_view *view, uint32_t timeout_us,
                                uint64_t *ticket);
/* Cancel a queued request: HAB_OK (its ticket then reports
 * HAB_ERR_CANCELLED); HAB_ERR_NOT_READY when it is already launched (it
 * completes normally); HAB_ERR_INVALID_ARG for a ticket that is done,
 * collected or unknown. */
hab_status hab_server_cancel(hab_server *srv, uint64_t ticket);
/* HAB_ERR_NOT_READY until the ticket's outputs are complete in device
 * memory; then HAB_OK and, if stats is non-NULL, its timestamps (or the
 * request's error: HAB_ERR_CANCELLED, HAB_ERR_TIMEOUT, a launch error). */
hab_status hab_server_poll(hab_server *srv, uint64_t ticket, hab_request_stats *stats);
hab_status hab_server_wait(hab_server *srv, uint64_t ticket, hab_request_stats *stats);
hab_status hab_server_stats_get(hab_server *srv, hab_server_stats *out);
/* Drain outstanding work, stop the loop, free server resources. */
hab_status hab_server_destroy(hab_server *srv);

/* ---------------------------------------------------------- profiling */
/* Per-phase device time, from HIP events recorded on the launch stream
 * around every kernel while profiling is on (hab_profile_enable).  Phases:
 * 0 reset, 1 setup, 2 bin count, 3 bin scan, 4 bin scatter, 5..7 raster
 * with tile size 8, 16, 32, 8 resolve.  Graph replays (stepper) are not
 * timed. */
#define HAB_NUM_PHASES 9
typedef struct {
    double ms[HAB_NUM_PHASES];        /* summed device time per phase        */
    uint64_t launches[HAB_NUM_PHASES]; /* kernel launches per phase           */
    uint64_t sequences;                /* launch sequences that were timed    */
} hab_phase_times;
hab_status hab_profile_enable(hab_context *ctx, int on);
/* Restrict the timed phases to bit set `phase_mask` (bit k = phase k; the
 * default is all): fewer events are recorded, so timing perturbs the rest
 * of the step less.  HAB_ERR_INVALID_ARG for a mask with no phase. */
hab_status hab_profile_phases(hab_context *ctx, uint32_t phase_mask);
/* Synchronise, add up every timed sequence since the last read, reset. */
hab_status hab_profile_read(hab_context *ctx, hab_phase_times *out);

/* ---------------------------------------------------------- self-check */
/* The setup and raster take 1/w at the snap and 1/A of a triangle's twice
 * area with a reciprocal-and-Newton-step sequence instead of a division;
 * it must return the IEEE quotient (what a division gives) bit for bit.
 * This counts the positive floats x whose bit patterns lie in
 * [lo_bits, hi_bits) for which it does not, on ctx's device and `stream`
 * (synchronised before returning), into *mismatches.  Requires
 * lo_bits < hi_bits <= 0x7F800000, else HAB_ERR_INVALID_ARG.  The range the
 * sequence serves, [0x00800000, 0x7E800000) (2^-126 to 2^126; other inputs
 * take the division), is about 2.1e9 values and a fraction of a second. */
hab_status hab_selfcheck_reciprocal(hab_context *ctx, uint32_t lo_bits, uint32_t hi_bits,
                                    hipStream_t stream, uint64_t *mismatches);

/* ---------------------------------------------------------- autotune */
/* Pick a tile size (8, 16, 32) and bin capacity factor (1, 2, 4) for every
 * batch class (scene-size bucket, resolution bucket, output mix) of a
 * sample batch by timing the whole batch: every choice for all classes,
 * then other tile sizes class by class.  The context remembers the choices;
 * later calls with opts->tile_size == 0 (and the stepper and server) use
 * them.  *chosen_tile_size / *chosen_bin_factor (may be NULL) receive the
 * first view's class's choice.  Renders on `stream` and synchronises it.
 * Results are identical for every choice.
 *
 * With the environment variable HABMI_AUTOTUNE_CACHE naming a file, the
 * context's whole table is written there (JSON: the GPU architecture and
 * one {"class", "tile", "bin_factor"} entry per class, replaced atomically;
 * HAB_ERR_INVALID_ARG if it cannot be written, the choices still made), and
 * hab_init loads the entries saved for the same architecture. */
hab_status hab_autotune(hab_context *ctx, const hab_view *views, uint32_t num_views,
                        hipStream_t stream, uint32_t *chosen_tile_size, float *chosen_bin_factor);

/* ---------------------------------------------------------- testing */
/* For tests of failure handling: every device and pinned host allocation
 * of the library goes through one place; after `after` more successful
 * allocations every further one fails as if out of memory, until this is
 * called with after < 0.  Process-wide. */
hab_status hab_test_fail_alloc(int64_t after);
/* Device and pinned host allocations of the library still held (count and
 * bytes), process-wide: an entry point that fails must leave them as they
 * were. */
hab_status hab_test_live_allocations(uint64_t *count, uint64_t *bytes);

#ifdef __cplusplus
}
#endif
#endif /* HAB_H */
