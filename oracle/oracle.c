/*
 * oracle.c -- plain, slow CPU reference renderer.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this file's library.  The rendering library never links, calls or
 * falls back to it, and the two share no code.
 *
 * What it computes (the paper's sensor model, Sec. 4 "Sensory input" and
 * Sec. 3 "Rendering engine"): for a static triangle mesh with per-vertex
 * colours and a pinhole camera of given resolution and horizontal field of
 * view, the colour image and the "idealized" depth image seen from a camera
 * pose, in one pass that also yields the visible triangle per pixel.  The
 * paper gives no rasterisation rules; the written definition below fixes
 * them (camera convention, planar depth, near plane, 8-bit sub-pixel snap,
 * top-left fill rule, nearest-wins with a smaller-id tie break, perspective
 * correct colour).  Every floating point step is fp32 with one rounding per
 * operation, in the order written (compile with -ffp-contract=off, SSE math).
 *
 * Published methods restated here: Pineda edge functions (1988); the
 * top-left fill rule with 8 sub-pixel bits; Sutherland-Hodgman clipping
 * against one plane (1974); perspective-correct interpolation through 1/w
 * (Heckbert & Moreton 1991); z-buffer visibility.
 *
 * Steps, per view, for each triangle in index order:
 *   1. transform to camera space          (pose -> Xc, Yc, w = -Zc)
 *   2. clip against w >= near              (0, 1 or 2 sub-triangles)
 *   3. project and snap to 1/256 px        (X, Y int64, rw = 1/w)
 *   4. orient (A > 0), drop A == 0, bbox   (pixel range in the viewport)
 *   5. for each pixel centre in the bbox: coverage by three edge functions
 *      with the top-left rule, key rho = interpolated 1/w, keep the largest
 *      rho (smaller key on ties)
 * and finally resolve each pixel: depth = 1/rho, colour interpolated with
 * perspective-correct weights, triangle index.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_INVALID_ARG 1
#define OR_ERR_RANGE 3

#define OR_NONE 0xFFFFFFFFu
#define OR_DOMAIN 536870912.0f /* 2^29: |X|, |Y| in 1/256 px must stay below */

typedef struct {
    uint64_t bbox_tests; /* pixel centres examined (sum of clipped bbox areas) */
    uint64_t covered;    /* (sub-triangle, pixel) pairs that pass coverage    */
    uint64_t survivors;  /* sub-triangles with a non-empty viewport bbox      */
    uint64_t clipped;    /* triangles that straddle the near plane            */
} or_stats;

/* Vertex attributes carried through clipping and interpolation: colour
 * (0..255 as float) in 0..2, texture coordinates (u, v) in 3..4. */
#define OR_NA 5

/* camera-space vertex with its attributes */
typedef struct {
    float x, y, w;
    float c[OR_NA];
} cvert;

/* snapped screen vertex */
typedef struct {
    int64_t X, Y;
    float rw;
    float c[OR_NA];
} svert;

/* ------------------------------------------------------------------ a1 */
/* Sensor constants.  The paper's sensor has a square 256^2 image with a
 * 90-degree field of view (Sec. 4 "Sensory input"); the focal length in
 * pixels is W / (2 tan(HFOV/2)), evaluated in double and rounded once. */
float or_focal(uint32_t W, double hfov_deg)
{
    double f = (double)W / (2.0 * tan(hfov_deg * 3.14159265358979323846 / 360.0));
    return (float)f;
}

/* Static fixed-point domain check for one pose: every vertex of the scene
 * (inside the given axis-aligned box) that lies at w >= near must project
 * to |X|, |Y| < 2^29 with a factor-two margin.  In double: the largest
 * distance D from the camera to a box corner bounds |Xc| and |Yc|, and the
 * projection is at most D * f * 256 / near + (W or H) * 128.  The rotation
 * must be orthonormal to 1e-4 (max abs entry of R^T R - I). */
int or_pose_check(const float *lo, const float *hi, const float *pose, uint32_t W,
                  uint32_t H, double hfov_deg, float near_m)
{
    const float *R = pose + 3;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += (double)R[3 * k + a] * (double)R[3 * k + b];
            if (fabs(s - (a == b ? 1.0 : 0.0)) > 1e-4) return OR_ERR_INVALID_ARG;
        }
    for (int k = 0; k < 12; ++k)
        if (!isfinite(pose[k])) return OR_ERR_INVALID_ARG;
    double D = 0.0;
    for (int c = 0; c < 8; ++c) {
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double v = (c >> a) & 1 ? hi[a] : lo[a];
            double d = v - (double)pose[a];
            d2 += d * d;
        }
        if (d2 > D) D = d2;
    }
    D = sqrt(D);
    double fS = (double)or_focal(W, hfov_deg) * 256.0;
    double m = (double)(W > H ? W : H) * 128.0;
    if (D * fS / (double)near_m + m >= 268435456.0 /* 2^28 */) return OR_ERR_RANGE;
    return OR_OK;
}

/* ------------------------------------------------------------------ a2 */
/* world -> camera: d = P - p, camera coordinates are R^T d with R the
 * row-major world-from-camera rotation; the camera looks along -Z so the
 * depth coordinate is w = -Zc. */
static void to_camera(const float *P, const float *pose, cvert *v)
{
    const float *R = pose + 3;
    float dx = P[0] - pose[0];
    float dy = P[1] - pose[1];
    float dz = P[2] - pose[2];
    float xc = (R[0] * dx + R[3] * dy) + R[6] * dz;
    float yc = (R[1] * dx + R[4] * dy) + R[7] * dz;
    float zc = (R[2] * dx + R[5] * dy) + R[8] * dz;
    v->x = xc;
    v->y = yc;
    v->w = -zc;
}

/* ------------------------------------------------------------------ a3 */
/* Sutherland-Hodgman against the single plane w >= near.  Walk the edges
 * v0->v1, v1->v2, v2->v0; emit the start vertex when inside, then the
 * crossing point when the edge crosses the plane.  The crossing is always
 * interpolated from the inside end towards the outside end, so two
 * triangles that share the edge produce the same point.  Returns the
 * polygon size (0, 3 or 4). */
static int clip_near(const cvert in[3], float zn, cvert out[4])
{
    int n = 0;
    for (int k = 0; k < 3; ++k) {
        const cvert *a = &in[k];
        const cvert *b = &in[(k + 1) % 3];
        int ia = a->w >= zn;
        int ib = b->w >= zn;
        if (ia) out[n++] = *a;
        if (ia != ib) {
            const cvert *s = ia ? a : b; /* inside end */
            const cvert *o = ia ? b : a; /* outside end */
            float t = (s->w - zn) / (s->w - o->w);
            cvert q;
            q.x = s->x + t * (o->x - s->x);
            q.y = s->y + t * (o->y - s->y);
            for (int c = 0; c < OR_NA; ++c) q.c[c] = s->c[c] + t * (o->c[c] - s->c[c]);
            q.w = zn;
            out[n++] = q;
        }
    }
    return n;
}

/* ------------------------------------------------------------------ a4 */
/* Perspective projection and snap to 8 sub-pixel bits (1/256 px), rounding
 * half to even.  Pixel (i, j) has its centre at (i + 1/2, j + 1/2) px, i.e.
 * (256 i + 128, 256 j + 128) in fixed point; image row 0 is the top, so
 * camera +Y maps to decreasing rows. */
static int project(const cvert *v, float fS, float cxS, float cyS, svert *s)
{
    float rw = 1.0f / v->w;
    float xs = rintf(cxS + (v->x * fS) * rw);
    float ys = rintf(cyS - (v->y * fS) * rw);
    if (!(fabsf(xs) < OR_DOMAIN && fabsf(ys) < OR_DOMAIN)) return OR_ERR_RANGE;
    s->X = (int64_t)xs;
    s->Y = (int64_t)ys;
    s->rw = rw;
    for (int c = 0; c < OR_NA; ++c) s->c[c] = v->c[c];
    return OR_OK;
}

static int64_t floor_div256(int64_t a)
{
    /* floor(a / 256) for any sign */
    int64_t q = a / 256;
    if ((a % 256) != 0 && (a < 0)) q -= 1;
    return q;
}

/* Edge k runs from vertex k+1 to vertex k+2 (mod 3); its function at
 * (px, py) is dx*(py - ay) - dy*(px - ax), positive inside once A > 0.
 * An edge is owned ("top-left") when dy < 0, or dy == 0 and dx > 0. */
static int64_t edge_fn(const svert *a, const svert *b, int64_t px, int64_t py)
{
    int64_t dx = b->X - a->X, dy = b->Y - a->Y;
    return dx * (py - a->Y) - dy * (px - a->X);
}

static int edge_owned(const svert *a, const svert *b)
{
    int64_t dx = b->X - a->X, dy = b->Y - a->Y;
    return dy < 0 || (dy == 0 && dx > 0);
}

/* Per-pixel state while the scene is drawn (the z-buffer). */
typedef struct {
    float rho;       /* interpolated 1/w of the current winner, 0 = empty   */
    uint32_t key;    /* 2 * triangle index + sub-triangle, OR_NONE = empty  */
    float wgt[3];    /* b_k * rw_k of the winner at this pixel              */
    float num;       /* (wgt0 + wgt1) + wgt2                                */
    float col[3][OR_NA]; /* the winner's vertex attributes                  */
} zpix;

typedef struct {
    const float *pos;
    uint32_t V;
    const uint8_t *col;
    const uint32_t *idx;
    uint32_t T;
    const float *uv;      /* [V][2] texture coordinates, or NULL            */
    const uint8_t *tex;   /* [th][tw][3] RGB texture, or NULL               */
    uint32_t tw, th;
    uint32_t W, H;
    float fS, cxS, cyS, zn;
    const float *pose;
} view_in;

/* Rasterise one snapped sub-triangle into the z-buffer, or, with count !=
 * NULL, only count covering triangles per pixel. */
static void raster_tri(const view_in *in, svert v[3], uint32_t key, zpix *zb,
                       uint32_t *count, or_stats *st)
{
    int64_t A = (v[1].X - v[0].X) * (v[2].Y - v[0].Y) - (v[1].Y - v[0].Y) * (v[2].X - v[0].X);
    if (A == 0) return;
    if (A < 0) {
        svert t = v[1];
        v[1] = v[2];
        v[2] = t;
        A = -A;
    }
    int64_t minX = v[0].X, maxX = v[0].X, minY = v[0].Y, maxY = v[0].Y;
    for (int k = 1; k < 3; ++k) {
        if (v[k].X < minX) minX = v[k].X;
        if (v[k].X > maxX) maxX = v[k].X;
        if (v[k].Y < minY) minY = v[k].Y;
        if (v[k].Y > maxY) maxY = v[k].Y;
    }
    /* pixel centres 256 i + 128 inside [minX, maxX] */
    int64_t i0 = floor_div256(minX - 128 + 255), i1 = floor_div256(maxX - 128);
    int64_t j0 = floor_div256(minY - 128 + 255), j1 = floor_div256(maxY - 128);
    if (i0 < 0) i0 = 0;
    if (j0 < 0) j0 = 0;
    if (i1 > (int64_t)in->W - 1) i1 = (int64_t)in->W - 1;
    if (j1 > (int64_t)in->H - 1) j1 = (int64_t)in->H - 1;
    if (i0 > i1 || j0 > j1) return;
    st->survivors += 1;
    st->bbox_tests += (uint64_t)((i1 - i0 + 1) * (j1 - j0 + 1));

    int owned[3];
    for (int k = 0; k < 3; ++k) owned[k] = edge_owned(&v[(k + 1) % 3], &v[(k + 2) % 3]);
    float invA = 1.0f / (float)A;

    for (int64_t j = j0; j <= j1; ++j) {
        for (int64_t i = i0; i <= i1; ++i) {
            int64_t px = 256 * i + 128, py = 256 * j + 128;
            int64_t E[3];
            int cov = 1;
            for (int k = 0; k < 3; ++k) {
                E[k] = edge_fn(&v[(k + 1) % 3], &v[(k + 2) % 3], px, py);
                if (!(E[k] > 0 || (E[k] == 0 && owned[k]))) cov = 0;
            }
            if (!cov) continue;
            st->covered += 1;
            size_t p = (size_t)j * in->W + (size_t)i;
            if (count) {
                count[p] += 1;
                continue;
            }
            float b0 = (float)E[0], b1 = (float)E[1], b2 = (float)E[2];
            float w0 = b0 * v[0].rw, w1 = b1 * v[1].rw, w2 = b2 * v[2].rw;
            float num = (w0 + w1) + w2;
            float rho = num * invA;
            zpix *z = &zb[p];
            if (rho > z->rho || (rho == z->rho && key < z->key)) {
                z->rho = rho;
                z->key = key;
                z->wgt[0] = w0;
                z->wgt[1] = w1;
                z->wgt[2] = w2;
                z->num = num;
                for (int k = 0; k < 3; ++k)
                    for (int c = 0; c < OR_NA; ++c) z->col[k][c] = v[k].c[c];
            }
        }
    }
}

static int draw_view(const view_in *in, zpix *zb, uint32_t *count, or_stats *st)
{
    for (uint32_t t = 0; t < in->T; ++t) {
        cvert cv[3];
        for (int k = 0; k < 3; ++k) {
            uint32_t vi = in->idx[3 * (size_t)t + k];
            to_camera(in->pos + 3 * (size_t)vi, in->pose, &cv[k]);
            for (int c = 0; c < 3; ++c)
                cv[k].c[c] = in->col ? (float)in->col[3 * (size_t)vi + c] : 255.0f;
            cv[k].c[3] = in->uv ? in->uv[2 * (size_t)vi] : 0.0f;
            cv[k].c[4] = in->uv ? in->uv[2 * (size_t)vi + 1] : 0.0f;
        }
        cvert poly[4];
        int n = clip_near(cv, in->zn, poly);
        if (n == 0) continue;
        if (!(cv[0].w >= in->zn && cv[1].w >= in->zn && cv[2].w >= in->zn)) st->clipped += 1;
        svert sp[4];
        for (int k = 0; k < n; ++k)
            if (project(&poly[k], in->fS, in->cxS, in->cyS, &sp[k]) != OR_OK) return OR_ERR_RANGE;
        /* fan: (q0, q1, q2) and, for a quad, (q0, q2, q3) */
        for (int s = 0; s + 2 < n; ++s) {
            svert tri[3] = {sp[0], sp[s + 1], sp[s + 2]};
            raster_tri(in, tri, 2u * t + (uint32_t)s, zb, count, st);
        }
    }
    return OR_OK;
}

static int setup_view(view_in *in, const float *pos, uint32_t V, const uint8_t *col,
                      const uint32_t *idx, uint32_t T, uint32_t W, uint32_t H,
                      double hfov_deg, float near_m, const float *pose)
{
    if (W == 0 || H == 0 || W > 4096 || H > 4096) return OR_ERR_INVALID_ARG;
    if (!(hfov_deg > 0.0 && hfov_deg < 180.0) || !(near_m > 0.0f)) return OR_ERR_INVALID_ARG;
    if (T >= 0x7FFFFFFFu) return OR_ERR_INVALID_ARG;
    for (size_t k = 0; k < 3 * (size_t)T; ++k)
        if (idx[k] >= V) return OR_ERR_INVALID_ARG;
    in->pos = pos;
    in->V = V;
    in->col = col;
    in->idx = idx;
    in->T = T;
    in->uv = NULL;
    in->tex = NULL;
    in->tw = in->th = 0;
    in->W = W;
    in->H = H;
    in->fS = or_focal(W, hfov_deg) * 256.0f;
    in->cxS = (float)W * 128.0f;
    in->cyS = (float)H * 128.0f;
    in->zn = near_m;
    in->pose = pose;
    return OR_OK;
}

/* ------------------------------------------------------------------ f2 */
/* Textured shading.  Scanned scenes carry textures (Sec. 4 "Episode
 * dataset preparation": textured meshes); the paper does not say how they
 * are filtered, so the written definition is the classic one: texture
 * coordinates interpolated perspective-correctly exactly as the colours
 * are, then a bilinear fetch with the texel centres at ((k + 1/2) / tw,
 * (l + 1/2) / th), v = 0 at the texture's first row, coordinates wrapping
 * (repeat).  The texture size is a power of two and |u| tw, |v| th < 2^22
 * at every vertex.  The fetch is evaluated in fp64 and rounded half to even
 * into 0..255. */
static uint32_t wrap(int64_t k, uint32_t n)
{
    int64_t m = k % (int64_t)n;
    return (uint32_t)(m < 0 ? m + (int64_t)n : m);
}

static void tex_bilinear(const uint8_t *tex, uint32_t tw, uint32_t th, float u, float v,
                         uint8_t out[3])
{
    const double x = (double)u * (double)tw - 0.5, y = (double)v * (double)th - 0.5;
    const double xf = floor(x), yf = floor(y);
    const double fx = x - xf, fy = y - yf;
    const uint32_t i0 = wrap((int64_t)xf, tw), i1 = wrap((int64_t)xf + 1, tw);
    const uint32_t j0 = wrap((int64_t)yf, th), j1 = wrap((int64_t)yf + 1, th);
    for (int c = 0; c < 3; ++c) {
        const double t00 = tex[((size_t)j0 * tw + i0) * 3 + c], t10 = tex[((size_t)j0 * tw + i1) * 3 + c];
        const double t01 = tex[((size_t)j1 * tw + i0) * 3 + c], t11 = tex[((size_t)j1 * tw + i1) * 3 + c];
        const double val = (1.0 - fy) * ((1.0 - fx) * t00 + fx * t10) + fy * ((1.0 - fx) * t01 + fx * t11);
        double r = rint(val);
        if (r < 0.0) r = 0.0;
        if (r > 255.0) r = 255.0;
        out[c] = (uint8_t)r;
    }
}

static int pow2(uint32_t n) { return n != 0 && (n & (n - 1)) == 0; }

static int render_core(view_in *in, uint8_t *rgb, float *depth, uint32_t *tri, float *rho_out,
                       uint32_t *key_out, or_stats *st);

/* Render one view.  Outputs (any may be NULL): rgb [H][W][3] uint8,
 * depth [H][W] float (planar metres, 0 = no hit), tri [H][W] uint32 (index
 * of the visible triangle, OR_NONE = no hit), rho [H][W] float and key
 * [H][W] uint32 (the raw z-buffer).  Positions [V][3] float, colours
 * [V][3] uint8 (NULL = white), indices [T][3] uint32. */
int or_render_view(const float *pos, uint32_t V, const uint8_t *col, const uint32_t *idx,
                   uint32_t T, uint32_t W, uint32_t H, double hfov_deg, float near_m,
                   const float *pose, uint8_t *rgb, float *depth, uint32_t *tri,
                   float *rho_out, uint32_t *key_out, or_stats *st)
{
    view_in in;
    int rc = setup_view(&in, pos, V, col, idx, T, W, H, hfov_deg, near_m, pose);
    if (rc != OR_OK) return rc;
    return render_core(&in, rgb, depth, tri, rho_out, key_out, st);
}

/* As or_render_view, with the colour taken from a texture: uv [V][2]
 * float, tex [th][tw][3] uint8 (tw, th powers of two). */
int or_render_view_tex(const float *pos, uint32_t V, const uint32_t *idx, uint32_t T,
                       const float *uv, const uint8_t *tex, uint32_t tw, uint32_t th,
                       uint32_t W, uint32_t H, double hfov_deg, float near_m, const float *pose,
                       uint8_t *rgb, float *depth, uint32_t *tri, float *rho_out,
                       uint32_t *key_out, or_stats *st)
{
    view_in in;
    if (!uv || !tex || !pow2(tw) || !pow2(th) || tw > 16384 || th > 16384) return OR_ERR_INVALID_ARG;
    for (size_t k = 0; k < V; ++k) {
        const double a = fabs((double)uv[2 * k] * tw), b = fabs((double)uv[2 * k + 1] * th);
        if (!(a < 4194304.0 && b < 4194304.0)) return OR_ERR_INVALID_ARG;
    }
    int rc = setup_view(&in, pos, V, NULL, idx, T, W, H, hfov_deg, near_m, pose);
    if (rc != OR_OK) return rc;
    in.uv = uv;
    in.tex = tex;
    in.tw = tw;
    in.th = th;
    return render_core(&in, rgb, depth, tri, rho_out, key_out, st);
}

static int render_core(view_in *in_, uint8_t *rgb, float *depth, uint32_t *tri, float *rho_out,
                       uint32_t *key_out, or_stats *st)
{
    view_in in = *in_;
    const uint32_t W = in.W, H = in.H;
    int rc;
    or_stats local;
    memset(&local, 0, sizeof local);
    size_t np = (size_t)W * H;
    zpix *zb = (zpix *)calloc(np, sizeof(zpix));
    if (!zb) return OR_ERR_INVALID_ARG;
    for (size_t p = 0; p < np; ++p) {
        zb[p].rho = 0.0f;
        zb[p].key = OR_NONE;
    }
    rc = draw_view(&in, zb, NULL, &local);
    if (rc != OR_OK) {
        free(zb);
        return rc;
    }
    /* ------------------------------------------------------------ a7 */
    for (size_t p = 0; p < np; ++p) {
        const zpix *z = &zb[p];
        int hit = z->key != OR_NONE;
        if (rho_out) rho_out[p] = z->rho;
        if (key_out) key_out[p] = z->key;
        if (tri) tri[p] = hit ? (z->key >> 1) : OR_NONE;
        if (depth) depth[p] = hit ? 1.0f / z->rho : 0.0f;
        if (rgb && in.tex) {
            uint8_t t[3] = {0, 0, 0};
            if (hit) {
                const float u = ((z->wgt[0] * z->col[0][3] + z->wgt[1] * z->col[1][3]) +
                                 z->wgt[2] * z->col[2][3]) / z->num;
                const float v = ((z->wgt[0] * z->col[0][4] + z->wgt[1] * z->col[1][4]) +
                                 z->wgt[2] * z->col[2][4]) / z->num;
                tex_bilinear(in.tex, in.tw, in.th, u, v, t);
            }
            for (int c = 0; c < 3; ++c) rgb[3 * p + c] = t[c];
        } else if (rgb) {
            for (int c = 0; c < 3; ++c) {
                uint8_t u = 0;
                if (hit) {
                    float val = ((z->wgt[0] * z->col[0][c] + z->wgt[1] * z->col[1][c]) +
                                 z->wgt[2] * z->col[2][c]) / z->num;
                    val = rintf(val);
                    if (val < 0.0f) val = 0.0f;
                    if (val > 255.0f) val = 255.0f;
                    u = (uint8_t)val;
                }
                rgb[3 * p + c] = u;
            }
        }
    }
    free(zb);
    if (st) *st = local;
    return OR_OK;
}

/* Coverage-count mode: count[p] = number of sub-triangles whose coverage
 * test accepts pixel p (no depth test).  Used for the watertightness
 * invariant. */
int or_coverage_count(const float *pos, uint32_t V, const uint32_t *idx, uint32_t T,
                      uint32_t W, uint32_t H, double hfov_deg, float near_m,
                      const float *pose, uint32_t *count, or_stats *st)
{
    view_in in;
    int rc = setup_view(&in, pos, V, NULL, idx, T, W, H, hfov_deg, near_m, pose);
    if (rc != OR_OK) return rc;
    or_stats local;
    memset(&local, 0, sizeof local);
    memset(count, 0, sizeof(uint32_t) * (size_t)W * H);
    rc = draw_view(&in, NULL, count, &local);
    if (st) *st = local;
    return rc;
}

/* Projection of a single point (closed-form checks): snapped fixed-point
 * X, Y for a world point seen from a pose, or OR_ERR_RANGE / behind-camera
 * (returns 1 when w < near). */
int or_project_point(const float *P, const float *pose, uint32_t W, uint32_t H,
                     double hfov_deg, float near_m, int64_t *X, int64_t *Y, float *rw)
{
    cvert v;
    to_camera(P, pose, &v);
    if (!(v.w >= near_m)) return 1;
    svert s;
    float fS = or_focal(W, hfov_deg) * 256.0f;
    int rc = project(&v, fS, (float)W * 128.0f, (float)H * 128.0f, &s);
    if (rc != OR_OK) return rc;
    *X = s.X;
    *Y = s.Y;
    *rw = s.rw;
    return OR_OK;
}

/* ------------------------------------------------------------------------
 * Noisy depth (the appendix's noise study, "Noisy Depth"): iid Gaussian
 * noise of mean 0 and standard deviation sigma added to each pixel's
 * inverse depth, so the error in depth grows with depth.  The paper states
 * no generator and gives two inconsistent sigma values; the reading taken
 * here: sigma is a sensor parameter in 1/m, the noisy inverse depth is
 * rho' = rho + sigma * n, the noisy depth is 1/rho' when rho' > 0 and 0
 * (no return) otherwise, and pixels with nothing visible stay 0.
 *
 * n comes from a counter-based generator so that any pixel's noise can be
 * drawn on its own: Philox4x64 with 10 rounds (Salmon, Moraes, Dror and
 * Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011), keyed by
 * (view seed, depth-noise stream tag), counter (pixel index j*W + i, 0, 0,
 * 0).  Of its four 64-bit words, the top 24 bits of word 0 and of word 1
 * give u1 = (a + 1) / 2^24 in (0, 1] and u2 = b / 2^24 in [0, 1), and the
 * Box-Muller transform (1958) gives n = sqrt(-2 ln u1) cos(2 pi u2).  The
 * oracle evaluates n and rho' in fp64.
 * ---------------------------------------------------------------------- */
#define OR_PHILOX_M0 0xD2E7470EE14C6C93ull
#define OR_PHILOX_M1 0xCA5A826395121157ull
#define OR_PHILOX_W0 0x9E3779B97F4A7C15ull /* golden ratio */
#define OR_PHILOX_W1 0xBB67AE8584CAA73Bull /* sqrt(3) - 1 */
#define OR_DEPTH_NOISE_TAG 0x6465707468ull  /* "depth" */

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += OR_PHILOX_W0;
            k1 += OR_PHILOX_W1;
        }
        const unsigned __int128 p0 = (unsigned __int128)OR_PHILOX_M0 * c0;
        const unsigned __int128 p1 = (unsigned __int128)OR_PHILOX_M1 * c2;
        const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* The standard normal deviate of one pixel (fp64). */
double or_depth_noise_normal(uint64_t seed, uint64_t pixel)
{
    const uint64_t ctr[4] = {pixel, 0, 0, 0};
    const uint64_t key[2] = {seed, OR_DEPTH_NOISE_TAG};
    uint64_t x[4];
    or_philox4x64_10(ctr, key, x);
    const double u1 = (double)((x[0] >> 40) + 1) / 16777216.0;
    const double u2 = (double)(x[1] >> 40) / 16777216.0;
    return sqrt(-2.0 * log(u1)) * cos(2.0 * 3.14159265358979323846 * u2);
}

/* Noisy inverse depth and depth of a W x H view from its per-pixel key rho
 * (fp32, as the render's raw output) and visible triangle (OR_NONE: none).
 * rho_out / depth_out: fp64 [H][W]; nothing visible gives 0 in both. */
int or_depth_noise(const float *rho, const uint32_t *tri, uint32_t W, uint32_t H, double sigma,
                   uint64_t seed, double *rho_out, double *depth_out)
{
    if (!rho || !tri || !rho_out || !depth_out || !(sigma >= 0.0)) return OR_ERR_INVALID_ARG;
    for (uint32_t j = 0; j < H; ++j)
        for (uint32_t i = 0; i < W; ++i) {
            const size_t p = (size_t)j * W + i;
            if (tri[p] == OR_NONE) {
                rho_out[p] = 0.0;
                depth_out[p] = 0.0;
                continue;
            }
            const double rp = (double)rho[p] + sigma * or_depth_noise_normal(seed, (uint64_t)p);
            rho_out[p] = rp;
            depth_out[p] = rp > 0.0 ? 1.0 / rp : 0.0;
        }
    return OR_OK;
}

/* ------------------------------------------------------------------------
 * Actuation and collision (Sec. 4 "Agent embodiment and action space" and
 * "Collision dynamics"): the agent is a vertical cylinder of 0.2 m diameter
 * that turns by 10 degrees or moves 0.25 m forward in a continuous state
 * space; a move that meets an obstacle makes partial or no progress and may
 * slide along it.  The paper gives no algorithm; the written definition:
 *
 *   - the agent is a disc of radius r on the floor plane (x, z); its heading
 *     is the unit forward vector (fx, fz) (yaw 0 looks along -z);
 *   - obstacles are line segments in that plane (the boundary of the free
 *     floor: walls and furniture footprints);
 *   - turn left / right: (fx, fz) <- (fx c + fz s, fz c - fx s) with
 *     (c, s) = (cos, +-sin) of the turn angle, given by the caller;
 *   - forward: the motion D = step (fx, fz) runs through at most 4 passes of
 *     collide-and-slide: find the earliest contact time t in [0, 1] at which
 *     the moving disc reaches distance r from a segment while approaching it
 *     (the segment's interior or an endpoint; earliest t, then the lower
 *     segment index, then interior before first before second endpoint);
 *     without one the disc moves by D and stops; with one it moves by
 *     max(0, t - skin / |D|) D (skin = 1e-6 m), the rest of the motion
 *     loses its component along the contact normal, and the next pass
 *     continues with what is left.  Motion left after the last pass is
 *     dropped.
 * Everything is fp64, one IEEE rounding per operation in the order written.
 * ---------------------------------------------------------------------- */
#define OR_SLIDE_PASSES 4
#define OR_SKIN 1e-6

typedef struct {
    double x, z;   /* position on the floor plane, metres */
    double fx, fz; /* unit forward vector */
} or_agent;

/* Earliest approach contact of the disc at (px, pz) moving by (dx, dz)
 * (not zero) against the segments; returns 1 and (t, contact normal) if
 * there is one with t <= 1. */
static int first_contact(const float *seg, uint32_t nseg, double r, double px, double pz,
                         double dx, double dz, double *t_out, double *nx_out, double *nz_out)
{
    const double a = dx * dx + dz * dz;
    int found = 0;
    double bt = 0.0, bnx = 0.0, bnz = 0.0;
    for (uint32_t k = 0; k < nseg; ++k) {
        const double ax = seg[4 * (size_t)k], az = seg[4 * (size_t)k + 1];
        const double bx = seg[4 * (size_t)k + 2], bz = seg[4 * (size_t)k + 3];
        const double ex = bx - ax, ez = bz - az;
        const double L2 = ex * ex + ez * ez;
        if (L2 > 0.0) {
            /* the segment's interior: the disc's centre reaches distance r
             * from the line with its foot inside the segment */
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
                    if (s >= 0.0 && s <= 1.0 && (!found || t < bt)) {
                        found = 1;
                        bt = t;
                        bnx = nx;
                        bnz = nz;
                    }
                }
            }
        }
        for (int e = 0; e < 2; ++e) {
            /* an endpoint: |p + t D - q| = r, first root, approaching */
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
            if (!found || t < bt) {
                found = 1;
                bt = t;
                bnx = cx / len;
                bnz = cz / len;
            }
        }
    }
    *t_out = bt;
    *nx_out = bnx;
    *nz_out = bnz;
    return found;
}

/* One action of one agent.  action: 0 stop, 1 forward, 2 turn left, 3 turn
 * right.  *collided is set to 1 when a forward move met an obstacle. */
int or_actuate(const float *seg, uint32_t nseg, double radius, double step, double turn_cos,
               double turn_sin, uint32_t action, or_agent *ag, uint32_t *collided)
{
    if (!ag || !collided || (nseg && !seg) || action > 3) return OR_ERR_INVALID_ARG;
    *collided = 0;
    if (action == 2 || action == 3) {
        const double s = action == 2 ? turn_sin : -turn_sin;
        const double fx = ag->fx * turn_cos + ag->fz * s;
        const double fz = ag->fz * turn_cos - ag->fx * s;
        ag->fx = fx;
        ag->fz = fz;
        return OR_OK;
    }
    if (action == 0) return OR_OK;
    double px = ag->x, pz = ag->z;
    double dx = step * ag->fx, dz = step * ag->fz;
    for (int pass = 0; pass < OR_SLIDE_PASSES; ++pass) {
        const double a = dx * dx + dz * dz;
        if (!(a > 0.0)) break;
        double t, nx, nz;
        if (!first_contact(seg, nseg, radius, px, pz, dx, dz, &t, &nx, &nz)) {
            px += dx;
            pz += dz;
            break;
        }
        *collided = 1;
        double ts = t - OR_SKIN / sqrt(a);
        if (ts < 0.0) ts = 0.0;
        px += ts * dx;
        pz += ts * dz;
        double rx = (1.0 - ts) * dx, rz = (1.0 - ts) * dz;
        const double dn = rx * nx + rz * nz;
        rx -= dn * nx;
        rz -= dn * nz;
        dx = rx;
        dz = rz;
    }
    ag->x = px;
    ag->z = pz;
    return OR_OK;
}

/* Camera pose of an agent state (Sec. 4 "Sensory input": the sensor sits at
 * a fixed height above the agent's base and faces the way the agent does).
 * The camera looks along its -Z axis with +Y up, so its axes in the world
 * are right = (-fz, 0, fx), up = (0, 1, 0) and back = (-fx, 0, -fz), the
 * columns of the row-major world-from-camera rotation.  Each entry is the
 * fp64 value rounded once to fp32; no trigonometry is involved. */
void or_agent_pose(const or_agent *ag, float height, float pose[12])
{
    const double right[3] = {-ag->fz, 0.0, ag->fx};
    const double up[3] = {0.0, 1.0, 0.0};
    const double back[3] = {-ag->fx, 0.0, -ag->fz};
    pose[0] = (float)ag->x;
    pose[1] = height;
    pose[2] = (float)ag->z;
    for (int r = 0; r < 3; ++r) {
        pose[3 + 3 * r + 0] = (float)right[r];
        pose[3 + 3 * r + 1] = (float)up[r];
        pose[3 + 3 * r + 2] = (float)back[r];
    }
}

/* ------------------------------------------------------------------------
 * Obstacles from the scene's own geometry and free space (Sec. 4 "Agent
 * embodiment and action space": the agent is a 0.2 m-diameter, 1.5 m-tall
 * cylinder; "Collision dynamics": it slides along the scene's walls and
 * obstacles).  The paper describes no navigability representation; the
 * written definition:
 *
 *   - the obstacles of a mesh are its horizontal cross-sections at K given
 *     heights across the agent's body (above the floor, up to its height):
 *     for each triangle in index order and each height h in the given order,
 *     classify the vertices as above (y >= h) or below; when the classes
 *     differ, exactly two edges (walked v0->v1, v1->v2, v2->v0) change class,
 *     each is cut at y = h by interpolating from its lower end towards its
 *     upper end, t = (h - lo.y) / (hi.y - lo.y), x = lo.x + t (hi.x - lo.x)
 *     (the same for z), and the segment from the first cut to the second is
 *     one obstacle (x0, z0, x1, z1), computed in fp64 and rounded once to
 *     fp32 per coordinate;
 *   - a disc of radius r at (x, z) is free when every obstacle segment is at
 *     least r away: with e = b - a, L2 = |e|^2, s = ((p - a).e) / L2 clamped
 *     to [0, 1] (s = 0 when L2 = 0), q = a + s e - p, the disc is blocked by
 *     the segment when |q|^2 < r^2 (fp64, in that order).
 * ---------------------------------------------------------------------- */

/* Cross-section obstacles of a mesh.  seg_out [cap][4] (may be NULL when cap
 * is 0); returns the number of segments (written up to cap), or -1 for an
 * index out of range. */
int64_t or_nav_slice(const float *pos, uint32_t V, const uint32_t *idx, uint32_t T, const double *heights,
                     uint32_t K, float *seg_out, uint64_t cap)
{
    uint64_t n = 0;
    for (uint32_t t = 0; t < T; ++t) {
        double P[3][3];
        for (int k = 0; k < 3; ++k) {
            const uint32_t vi = idx[3 * (size_t)t + k];
            if (vi >= V) return -1;
            for (int a = 0; a < 3; ++a) P[k][a] = (double)pos[3 * (size_t)vi + a];
        }
        for (uint32_t h = 0; h < K; ++h) {
            const double y = heights[h];
            int up[3];
            for (int k = 0; k < 3; ++k) up[k] = P[k][1] >= y;
            if (up[0] == up[1] && up[1] == up[2]) continue;
            double cut[2][2];
            int nc = 0;
            for (int k = 0; k < 3; ++k) {
                const double *a = P[k], *b = P[(k + 1) % 3];
                if (up[k] == up[(k + 1) % 3]) continue;
                const double *lo = up[k] ? b : a, *hi = up[k] ? a : b;
                const double s = (y - lo[1]) / (hi[1] - lo[1]);
                cut[nc][0] = lo[0] + s * (hi[0] - lo[0]);
                cut[nc][1] = lo[2] + s * (hi[2] - lo[2]);
                ++nc;
            }
            if (n < cap) {
                float *o = seg_out + 4 * n;
                o[0] = (float)cut[0][0];
                o[1] = (float)cut[0][1];
                o[2] = (float)cut[1][0];
                o[3] = (float)cut[1][1];
            }
            ++n;
        }
    }
    return (int64_t)n;
}

/* 1 when a disc of radius r at (px, pz) is free of every segment. */
int or_nav_free(const float *seg, uint32_t nseg, double px, double pz, double r)
{
    for (uint32_t k = 0; k < nseg; ++k) {
        const double ax = seg[4 * (size_t)k], az = seg[4 * (size_t)k + 1];
        const double ex = (double)seg[4 * (size_t)k + 2] - ax, ez = (double)seg[4 * (size_t)k + 3] - az;
        const double L2 = ex * ex + ez * ez;
        double s = 0.0;
        if (L2 > 0.0) {
            s = ((px - ax) * ex + (pz - az) * ez) / L2;
            if (s < 0.0) s = 0.0;
            if (s > 1.0) s = 1.0;
        }
        const double qx = ax + s * ex - px, qz = az + s * ez - pz;
        if (qx * qx + qz * qz < r * r) return 0;
    }
    return 1;
}
