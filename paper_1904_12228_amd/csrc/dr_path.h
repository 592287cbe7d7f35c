// Light transport on the device (forward values): hit points, shading
// normals, next-event estimation and the radiance of a path suffix, with the
// thesis's setting (Ch. 5): Lambertian surfaces, triangle area lights.
// Readings where the thesis is silent: one light triangle picked by area and
// a point by the square-root warp; next-event estimation only (emission found
// by continuation rays is not added); cosine-weighted continuation around the
// shading normal; emitters radiate along their geometric normal.
#pragma once
#include "dr_trace.h"

namespace dr {

struct TriGeom { v3 p0, e1, e2; };

__device__ inline TriGeom tri_geom(const SceneView& s, int id) {
    TriRec r = load_tri(s.tri, id);
    return {{r.a.x, r.a.y, r.a.z}, {r.a.w, r.b.x, r.b.y}, {r.b.z, r.b.w, r.c.x}};
}

// Point where the ray meets the triangle's plane (moves with the ray and the
// triangle under differentiation).
__device__ inline v3 hit_point(const TriGeom& g, v3 o, v3 d) {
    v3 n = cross(g.e1, g.e2);
    float t = dot(g.p0 - o, n) / dot(d, n);
    return o + d * t;
}

// Shading normal at x (unoriented): interpolated vertex normals, or the
// geometric normal for flat scenes.
__device__ inline v3 shading_normal(const SceneView& s, int id, const TriGeom& g, v3 x) {
    v3 n = cross(g.e1, g.e2);
    if (!s.N) return nrm(n);
    v3 w = x - g.p0;
    float nn = dot(n, n);
    float b1 = dot(cross(w, g.e2), n) / nn;
    float b2 = dot(cross(g.e1, w), n) / nn;
    int i0 = s.I[3 * id], i1 = s.I[3 * id + 1], i2 = s.I[3 * id + 2];
    v3 N0 = ld3(s.N, i0), N1 = ld3(s.N, i1), N2 = ld3(s.N, i2);
    return nrm(N0 * (1.0f - b1 - b2) + N1 * b1 + N2 * b2);
}

__device__ inline float emitted(const SceneView& s, int id, bool front) {
    float e = s.emi[id];
    if (e <= 0.0f) return 0.0f;
    return (front || s.two_sided) ? e : 0.0f;
}

// first index with cdf[i] > u
__device__ inline int pick_cdf_d(const double* cdf, int n, double ud) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (cdf[mid] > ud) hi = mid; else lo = mid + 1;
    }
    return lo;
}

__device__ inline int pick_cdf(const double* cdf, int n, float u) {
    int lo = 0, hi = n - 1;
    double ud = (double)u;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (cdf[mid] > ud) hi = mid; else lo = mid + 1;
    }
    return lo;
}

struct NeeSample {
    v3 w;        // unit direction towards the light point
    float K;     // radiance * solid-angle factor / pi (0: no contribution)
    float r;     // distance to the light point
};

// Light sample for NEE at x with shading normal ns; visibility not tested.
__device__ inline NeeSample nee_sample(const SceneView& s, float4 u, v3 x, v3 ns) {
    NeeSample q{{0, 0, 0}, 0.0f, 0.0f};
    if (s.L == 0) return q;
    int li = pick_cdf(s.lcdf, s.L, u.x);
    int lt = s.lights[li];
    TriGeom g = tri_geom(s, lt);
    float su = sqrtf(u.y);
    v3 y = g.p0 + g.e1 * (su * (1.0f - u.z)) + g.e2 * (su * u.z);
    v3 w = y - x;
    float r2 = dot(w, w), r = sqrtf(r2);
    v3 wh = w * (1.0f / r);
    v3 nl = nrm(cross(g.e1, g.e2));
    float cy = -dot(nl, wh);
    if (s.two_sided) cy = fabsf(cy);
    float cp = dot(ns, wh);
    q.w = wh;
    q.r = r;
    if (cp <= 0.0f || cy <= 0.0f) return q;
    q.K = s.emi[lt] * cy / r2 * s.atot[0] / kPi;
    return q;
}

__device__ inline v3 cosine_dir(v3 n, float u0, float u1) {
    v3 t1, t2;
    onb(n, t1, t2);
    float r = sqrtf(u0), ph = 2.0f * kPi * u1;
    float sp, cp;
    sincosf(ph, &sp, &cp);
    return t1 * (r * cp) + t2 * (r * sp) + n * sqrtf(1.0f - u0);
}

// Radiance arriving along the ray o + t d whose first hit is h: emission at
// the hit, then NEE at path vertices 1..budget with cosine continuation
// between them. camera: a miss returns the background.
template <class W>
__device__ inline float radiance_hit(const SceneView& s, const Rng& rng, int base, v3 o, v3 d, const Hit& h, bool camera,
                                     int budget, int* stk, int stride, W& wk) {
    if (h.tri < 0) return camera ? s.background : 0.0f;
    int tri = h.tri;
    TriGeom g = tri_geom(s, tri);
    v3 x = hit_point(g, o, d);
    bool front = dot(d, cross(g.e1, g.e2)) < 0.0f;
    float L = emitted(s, tri, front);
    float beta = 1.0f;
    for (int k = 1; k <= budget; ++k) {
        v3 ns = shading_normal(s, tri, g, x);
        if (!front) ns = -ns;
        float rho = s.alb[tri];
        if (rho == 0.0f) break;
        NeeSample q = nee_sample(s, rng.block(base + 2 * k - 1), x, ns);
        if (q.K > 0.0f && !trace_any(s, x, q.w, s.tmin, q.r * (1.0f - kShadowEnd), stk, stride, wk))
            L += beta * rho * dot(ns, q.w) * q.K;
        if (k == budget) break;
        float4 ub = rng.block(base + 2 * k);
        v3 w = cosine_dir(ns, ub.x, ub.y);
        if (dot(ns, w) <= 0.0f) break;
        Hit h2 = trace_closest(s, x, w, s.tmin, 3.0e38f, stk, stride, wk);
        if (h2.tri < 0) break;
        beta *= rho;
        tri = h2.tri;
        g = tri_geom(s, tri);
        x = hit_point(g, x, w);
        front = dot(w, cross(g.e1, g.e2)) < 0.0f;
    }
    return L;
}

// Radiance arriving at o from direction d (ray from o, first hit in (tmin, inf)).
template <class W>
__device__ inline float radiance(const SceneView& s, const Rng& rng, int base, v3 o, v3 d, float tmin, bool camera,
                                 int budget, int* stk, int stride, W& wk) {
    Hit h = trace_closest(s, o, d, tmin, 3.0e38f, stk, stride, wk);
    return radiance_hit(s, rng, base, o, d, h, camera, budget, stk, stride, wk);
}

// The two one-sided radiances of a boundary sample, along d+ and d- just off
// the edge. When both rays first hit the same triangle (or both escape), the
// edge is not a visible discontinuity there: the one-sided limits coincide and
// both values are returned as 0 without tracing the paths further.
template <class W>
__device__ inline void radiance_pair(const SceneView& s, const Rng& rng, int base, v3 o, v3 dp, v3 dm, float tmin,
                                     bool camera, int budget, int* stk, int stride, W& wk, float& Lp, float& Lm) {
    Hit hp, hm;
    trace_closest2(s, o, dp, dm, tmin, 3.0e38f, stk, stride, wk, hp, hm);
    if (hp.tri == hm.tri) {
        Lp = Lm = 0.0f;
        return;
    }
    Lp = radiance_hit(s, rng, base, o, dp, hp, camera, budget, stk, stride, wk);
    Lm = radiance_hit(s, rng, base, o, dm, hm, camera, budget, stk, stride, wk);
}

// Whether the ray o + t d, t > tmin, may meet an emitter: a test against
// every light triangle with margins far above the FP32 rounding of the
// traversal's own triangle test (half of tmin in distance; 1e-4 in
// barycentric units divided by the incidence cosine, since the rounding of
// the barycentrics grows as the ray grazes the plane), so that when it fails
// the traversal's closest hit is no emitter. A side path with no bounce left
// then carries no radiance on that side. With more than kLightScan light
// triangles it answers true.
constexpr int kLightScan = 16;

__device__ inline bool may_reach_light(const SceneView& s, v3 o, v3 d, float tmin) {
    if (s.L > kLightScan) return true;
    for (int i = 0; i < s.L; ++i) {
        TriRec T = load_tri(s.tri, s.lights[i]);
        v3 v0 = {T.a.x, T.a.y, T.a.z}, e1 = {T.a.w, T.b.x, T.b.y}, e2 = {T.b.z, T.b.w, T.c.x};
        v3 pv = cross(d, e2);
        float det = dot(e1, pv);
        if (det == 0.0f) continue;
        float inv = 1.0f / det;
        v3 tv = o - v0;
        float u = dot(tv, pv) * inv;
        v3 qv = cross(tv, e1);
        float v = dot(d, qv) * inv;
        float t = dot(e2, qv) * inv;
        float eps = 1e-4f / fmaxf(fabsf(det) / (len(cross(e1, e2)) * len(d)), 1e-6f);
        if (u >= -eps && v >= -eps && u + v <= 1.0f + eps && t > 0.5f * tmin) return true;
    }
    return false;
}

// Geometry-buffer channel at the first hit x of triangle tri along d (Ch. 5,
// Results: G-buffers): 1..3 position, 4..6 shading normal facing the ray,
// 7 albedo; aov = 8 asks for all seven (aov_values).
__device__ inline float aov_value(const SceneView& s, int aov, int tri, const TriGeom& g, v3 x, v3 d) {
    if (aov <= 3) return aov == 1 ? x.x : (aov == 2 ? x.y : x.z);
    if (aov <= 6) {
        v3 n = shading_normal(s, tri, g, x);
        if (!(dot(d, cross(g.e1, g.e2)) < 0.0f)) n = -n;
        return aov == 4 ? n.x : (aov == 5 ? n.y : n.z);
    }
    return s.alb[tri];
}

// All seven channels at once (aov = 8): v[c - 1] = channel c.
__device__ inline void aov_values(const SceneView& s, int tri, const TriGeom& g, v3 x, v3 d, float (&v)[7]) {
    v3 n = shading_normal(s, tri, g, x);
    if (!(dot(d, cross(g.e1, g.e2)) < 0.0f)) n = -n;
    v[0] = x.x; v[1] = x.y; v[2] = x.z;
    v[3] = n.x; v[4] = n.y; v[5] = n.z;
    v[6] = s.alb[tri];
}

// Loss-weighted jump of the buffer across a primary boundary sample:
// sum over the channels of dI[channel] * (value on the + side - value on the
// - side), a ray that escapes giving 0. dI points at the sample's pixel in the
// first channel's loss gradient; channels are npix floats apart. Zero when
// the two rays hit the same triangle, as for radiance.
template <class W>
__device__ inline float aov_jump(const SceneView& s, int aov, v3 o, v3 dp, v3 dm, float tmin, const float* dI, int npix,
                                 int* stk, int stride, W& wk) {
    Hit hp, hm;
    trace_closest2(s, o, dp, dm, tmin, 3.0e38f, stk, stride, wk, hp, hm);
    if (hp.tri == hm.tri) return 0.0f;
    if (aov != 8) {
        float Fp = 0.0f, Fm = 0.0f;
        if (hp.tri >= 0) {
            TriGeom g = tri_geom(s, hp.tri);
            Fp = aov_value(s, aov, hp.tri, g, hit_point(g, o, dp), dp);
        }
        if (hm.tri >= 0) {
            TriGeom g = tri_geom(s, hm.tri);
            Fm = aov_value(s, aov, hm.tri, g, hit_point(g, o, dm), dm);
        }
        return dI[0] * (Fp - Fm);
    }
    float vp[7] = {0, 0, 0, 0, 0, 0, 0}, vm[7] = {0, 0, 0, 0, 0, 0, 0};
    if (hp.tri >= 0) {
        TriGeom g = tri_geom(s, hp.tri);
        aov_values(s, hp.tri, g, hit_point(g, o, dp), dp, vp);
    }
    if (hm.tri >= 0) {
        TriGeom g = tri_geom(s, hm.tri);
        aov_values(s, hm.tri, g, hit_point(g, o, dm), dm, vm);
    }
    float j = 0.0f;
#pragma unroll
    for (int c = 0; c < 7; ++c) j += dI[(size_t)c * npix] * (vp[c] - vm[c]);
    return j;
}

__device__ inline void project(const Cam& k, v3 P, float& sx, float& sy) {
    v3 q = P - k.c;
    float z = dot(q, k.f), xc = dot(q, k.r), yc = dot(q, k.u);
    sx = (1.0f + xc / (z * (k.asp * k.th))) * (k.W * 0.5f);
    sy = (1.0f - yc / (z * k.th)) * (k.H * 0.5f);
}

// Points defining the edge equation alpha (eq. edge_equation): the endpoints,
// except that an endpoint behind the near plane is replaced by the edge point
// at depth zd = max(near, half the other endpoint's depth). Any two points of
// the edge in front of the camera give the same projected line, hence the same
// boundary term; this choice keeps the projection well conditioned (a point at
// depth `near` projects far off screen with a 1/near^2 Jacobian).
__device__ inline v3 alpha_point(const Cam& k, v3 a, v3 b, float za, float zb) {
    float zd = fmaxf(k.nearc, 0.5f * zb);
    return a + (b - a) * ((zd - za) / (zb - za));
}

// An edge is a silhouette from q when its two faces lie on opposite sides of q.
__device__ inline bool silhouette_from(const SceneView& s, int4 e, v3 q) {
    v3 pa = ld3(s.P, e.x);
    v3 w = q - pa;
    TriGeom g0 = tri_geom(s, e.z), g1 = tri_geom(s, e.w);
    float s0 = dot(cross(g0.e1, g0.e2), w), s1 = dot(cross(g1.e1, g1.e2), w);
    return (s0 > 0.0f) != (s1 > 0.0f);
}

}  // namespace dr
