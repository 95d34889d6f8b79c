// Device-side arithmetic of the renderer: camera transform, near-plane
// clip, projection + snap, triangle setup.  Every fp32 step is one IEEE
// operation in the written order (contraction is off for this file), so
// the same inputs give the same bits in the setup, raster and resolve
// kernels and in any batch, tile size or launch order.
//
// What is computed follows the paper's sensor model (Sec. 4 "Sensory
// input": pinhole colour sensor and an idealized depth sensor sharing its
// pose and intrinsics; Sec. 3 "Rendering engine": one pass yields every
// output) with these rules: planar depth, near plane, no far plane,
// vertices snapped to 1/256 px with round-half-even, double-sided,
// top-left fill rule, nearest (largest 1/w) wins with the smaller key on a
// tie, perspective-correct colour through 1/w.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dtypes.h"

#pragma clang fp contract(off)

namespace habmi {

constexpr float kDomain = 536870912.0f;   // 2^29: |X|, |Y| bound in 1/256 px

// Correctly rounded 1/x, the value of the IEEE division.  For x in
// [2^-126, 2^126) the hardware reciprocal (within one ulp) refined by one
// Newton step, e = 1 - x y exact in a fused multiply-add and y + e y
// rounded once, gives that value (checked for every float of the range by
// launch_check_recip); elsewhere the division itself.
constexpr uint32_t kRecipLo = 0x00800000u;   // 2^-126
constexpr uint32_t kRecipHi = 0x7E800000u;   // 2^126
__device__ __forceinline__ float recip_rn(float x)
{
    if (__builtin_expect(__float_as_uint(x) - kRecipLo < kRecipHi - kRecipLo, 1)) {
        const float y = __builtin_amdgcn_rcpf(x);
        return __builtin_fmaf(__builtin_fmaf(-x, y, 1.0f), y, y);
    }
    return 1.0f / x;
}

// Camera-space vertex with NA interpolated attributes (colour channels).
template <int NA>
struct Vtx {
    float x, y, w;
    float a[NA > 0 ? NA : 1];
};

// Snapped screen vertex.
template <int NA>
struct SVtx {
    int X, Y;
    float rw;
    float a[NA > 0 ? NA : 1];
};

// World -> camera for a row-major world-from-camera rotation R: camera
// coordinates are R^T (P - p); the view axis is -Z, so w = -Zc.
template <int NA>
__device__ __forceinline__ void cam_xform(const DView &v, float Px, float Py, float Pz, Vtx<NA> &o)
{
    float dx = Px - v.p[0];
    float dy = Py - v.p[1];
    float dz = Pz - v.p[2];
    o.x = (v.R[0] * dx + v.R[3] * dy) + v.R[6] * dz;
    o.y = (v.R[1] * dx + v.R[4] * dy) + v.R[7] * dz;
    float zc = (v.R[2] * dx + v.R[5] * dy) + v.R[8] * dz;
    o.w = -zc;
}

// Crossing of edge (s inside, o outside) with the plane w = near,
// interpolated from the inside end so that neighbouring triangles that
// share the edge produce the same point.
template <int NA>
__device__ __forceinline__ Vtx<NA> isect(const Vtx<NA> &s, const Vtx<NA> &o, float zn)
{
    float t = (s.w - zn) / (s.w - o.w);
    Vtx<NA> q;
    q.x = s.x + t * (o.x - s.x);
    q.y = s.y + t * (o.y - s.y);
#pragma unroll
    for (int k = 0; k < NA; ++k) q.a[k] = s.a[k] + t * (o.a[k] - s.a[k]);
    q.w = zn;
    return q;
}

// Sutherland-Hodgman against w >= near, edges walked v0->v1, v1->v2,
// v2->v0 (emit the start vertex if inside, then the crossing if the edge
// crosses), written out per inside-mask so that no array is indexed at run
// time.  Returns the polygon size: 0, 3 or 4.
template <int NA>
__device__ __forceinline__ int clip_poly(const Vtx<NA> &v0, const Vtx<NA> &v1, const Vtx<NA> &v2,
                                         float zn, Vtx<NA> &q0, Vtx<NA> &q1, Vtx<NA> &q2,
                                         Vtx<NA> &q3)
{
    int m = (v0.w >= zn ? 1 : 0) | (v1.w >= zn ? 2 : 0) | (v2.w >= zn ? 4 : 0);
    switch (m) {
    case 7: q0 = v0; q1 = v1; q2 = v2; return 3;
    case 1: q0 = v0; q1 = isect(v0, v1, zn); q2 = isect(v0, v2, zn); return 3;
    case 2: q0 = isect(v1, v0, zn); q1 = v1; q2 = isect(v1, v2, zn); return 3;
    case 4: q0 = isect(v2, v1, zn); q1 = v2; q2 = isect(v2, v0, zn); return 3;
    case 3: q0 = v0; q1 = v1; q2 = isect(v1, v2, zn); q3 = isect(v0, v2, zn); return 4;
    case 5: q0 = v0; q1 = isect(v0, v1, zn); q2 = isect(v2, v1, zn); q3 = v2; return 4;
    case 6: q0 = isect(v1, v0, zn); q1 = v1; q2 = v2; q3 = isect(v2, v0, zn); return 4;
    default: return 0;
    }
}

// Perspective projection and snap to 1/256 px, round half to even.  Returns
// false if the snapped point leaves |X|, |Y| < 2^29.
template <int NA>
__device__ __forceinline__ bool snap(const DView &v, const Vtx<NA> &c, SVtx<NA> &s)
{
    float rw = recip_rn(c.w);
    float xs = rintf(v.cxS + (c.x * v.fS) * rw);
    float ys = rintf(v.cyS - (c.y * v.fS) * rw);
    bool ok = fabsf(xs) < kDomain && fabsf(ys) < kDomain;
    s.X = ok ? (int)xs : 0;
    s.Y = ok ? (int)ys : 0;
    s.rw = rw;
#pragma unroll
    for (int k = 0; k < NA; ++k) s.a[k] = c.a[k];
    return ok;
}

// Twice the signed area in 1/256^2 px^2 (|.| < 2^61 in the domain).
template <int NA>
__device__ __forceinline__ long long area2(const SVtx<NA> &a, const SVtx<NA> &b, const SVtx<NA> &c)
{
    return (long long)(b.X - a.X) * (long long)(c.Y - a.Y) -
           (long long)(b.Y - a.Y) * (long long)(c.X - a.X);
}

// Pixel range [i0, i1] x [j0, j1] of centres inside the snapped bbox,
// clipped to the viewport; empty when i0 > i1 or j0 > j1.
struct PixBox {
    int i0, i1, j0, j1;
};

template <int NA>
__device__ __forceinline__ PixBox pix_box(const DView &v, const SVtx<NA> &a, const SVtx<NA> &b,
                                          const SVtx<NA> &c)
{
    int mnx = min(a.X, min(b.X, c.X)), mxx = max(a.X, max(b.X, c.X));
    int mny = min(a.Y, min(b.Y, c.Y)), mxy = max(a.Y, max(b.Y, c.Y));
    PixBox r;
    r.i0 = max((mnx + 127) >> 8, 0);            // ceil((minX - 128) / 256)
    r.i1 = min((mxx - 128) >> 8, (int)v.W - 1); // floor((maxX - 128) / 256)
    r.j0 = max((mny + 127) >> 8, 0);
    r.j1 = min((mxy - 128) >> 8, (int)v.H - 1);
    return r;
}

// Full setup of sub-triangle `sub` (0 or 1) of triangle `t` for view v:
// transform, clip, snap, orient.  On success a, b, c are the oriented
// vertices (A > 0) and A is twice the area.  Returns false if the
// sub-triangle does not exist, is degenerate, or leaves the fixed-point
// domain (then *range_err is set).
template <int NA>
__device__ __forceinline__ bool setup_sub(const DView &v, const Vtx<NA> &v0, const Vtx<NA> &v1,
                                          const Vtx<NA> &v2, int sub, SVtx<NA> &a, SVtx<NA> &b,
                                          SVtx<NA> &c, long long &A, bool &range_err)
{
    Vtx<NA> q0, q1, q2, q3;
    int n = clip_poly(v0, v1, v2, v.zn, q0, q1, q2, q3);
    if (n == 0 || (sub == 1 && n != 4)) return false;
    bool ok = snap(v, q0, a);
    if (sub == 0) {
        ok &= snap(v, q1, b);
        ok &= snap(v, q2, c);
    } else {
        ok &= snap(v, q2, b);
        ok &= snap(v, q3, c);
    }
    if (!ok) {
        range_err = true;
        return false;
    }
    A = area2(a, b, c);
    if (A == 0) return false;
    if (A < 0) {
        SVtx<NA> t = b;
        b = c;
        c = t;
        A = -A;
    }
    return true;
}

// Edge function of the directed edge a -> b at fixed-point point (px, py).
__device__ __forceinline__ long long edge_at(int ax, int ay, int bx, int by, long long px, long long py)
{
    long long dx = (long long)(bx - ax), dy = (long long)(by - ay);
    return dx * (py - ay) - dy * (px - ax);
}

__device__ __forceinline__ bool owned(int dx, int dy) { return dy < 0 || (dy == 0 && dx > 0); }

__device__ __forceinline__ uint32_t unpack_rgb(uint32_t c, int k) { return (c >> (8 * k)) & 0xFFu; }

}  // namespace habmi
