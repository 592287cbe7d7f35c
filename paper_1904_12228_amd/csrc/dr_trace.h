// Ray casting on the binary triangle BVH: Moller-Trumbore intersection in
// FP32, closest-hit (ties in t go to the smaller triangle id) and any-hit
// traversal. Each lane keeps its traversal stack in LDS, strided by the
// block size so that the 64 lanes of a wave touch 64 consecutive words.
#pragma once
#include "dr_common.h"

namespace dr {

// One triangle record (v0 | e1 | e2 in three 16-byte words), loaded whole.
struct TriRec { float4 a, b, c; };

__device__ inline TriRec load_tri(const float4* __restrict__ tri, int id) {
    const float4* p = reinterpret_cast<const float4*>(reinterpret_cast<const char*>(tri) + (uint32_t)id * 48u);
    return {p[0], p[1], p[2]};
}

// Moller-Trumbore without early exits: every word of the record is used on
// every path, so its three loads issue together and the lane waits for memory
// once. A zero determinant or a barycentric outside the triangle gives false.
// The same test with early exits, for a record already in registers:
// `tri_wait` makes the lane wait for the whole record at once, so the exits
// cannot move a part of its loads behind a branch.
__device__ inline void tri_wait(const TriRec& T) {
    asm volatile("" ::"v"(T.a.x), "v"(T.a.y), "v"(T.a.z), "v"(T.a.w), "v"(T.b.x), "v"(T.b.y), "v"(T.b.z), "v"(T.b.w),
                 "v"(T.c.x));
}

__device__ inline bool tri_hit_exit(const TriRec& T, v3 o, v3 d, float& t, float& u, float& v) {
    v3 v0 = {T.a.x, T.a.y, T.a.z}, e1 = {T.a.w, T.b.x, T.b.y}, e2 = {T.b.z, T.b.w, T.c.x};
    v3 pv = cross(d, e2);
    float det = dot(e1, pv);
    if (det == 0.0f) return false;
    float inv = 1.0f / det;
    v3 tv = o - v0;
    u = dot(tv, pv) * inv;
    if (!(u >= 0.0f && u <= 1.0f)) return false;
    v3 qv = cross(tv, e1);
    v = dot(d, qv) * inv;
    if (!(v >= 0.0f && u + v <= 1.0f)) return false;
    t = dot(e2, qv) * inv;
    return true;
}

__device__ inline bool tri_hit(const TriRec& T, v3 o, v3 d, float& t, float& u, float& v) {
    v3 v0 = {T.a.x, T.a.y, T.a.z}, e1 = {T.a.w, T.b.x, T.b.y}, e2 = {T.b.z, T.b.w, T.c.x};
    v3 pv = cross(d, e2);
    float det = dot(e1, pv);
    float inv = 1.0f / det;
    v3 tv = o - v0;
    u = dot(tv, pv) * inv;
    v3 qv = cross(tv, e1);
    v = dot(d, qv) * inv;
    t = dot(e2, qv) * inv;
    return (det != 0.0f) & (u >= 0.0f) & (u <= 1.0f) & (v >= 0.0f) & (u + v <= 1.0f);
}

// Ray with reciprocal direction and the origin pre-scaled by it: a slab
// plane's distance is then one fused multiply-add.
struct RayInv { v3 id, noid; };

__device__ inline RayInv ray_inv(v3 o, v3 d) {
    auto inv = [](float x) { return fabsf(x) > 1e-30f ? 1.0f / x : copysignf(1e30f, x); };
    v3 id = {inv(d.x), inv(d.y), inv(d.z)};
    return {id, {-o.x * id.x, -o.y * id.y, -o.z * id.z}};
}

// Widening of a box's exit distance that covers the rounding of the fused
// plane distances (a few ulps of the distances involved), so a box that the
// exact test enters is always entered (Ize, Robust BVH ray traversal, 2013);
// the cost is an occasional extra node visit.
constexpr float kSlabWiden = 1.0f + 4.0f * 1.1920929e-7f;

// slab test of [lo, hi] against the ray over [t0, t1]; returns entry distance
__device__ inline bool slab(const RayInv& r, float lx, float ly, float lz, float hx, float hy, float hz, float t0, float t1,
                            float& tent) {
    float ax = fmaf(lx, r.id.x, r.noid.x), bx = fmaf(hx, r.id.x, r.noid.x);
    float ay = fmaf(ly, r.id.y, r.noid.y), by = fmaf(hy, r.id.y, r.noid.y);
    float az = fmaf(lz, r.id.z, r.noid.z), bz = fmaf(hz, r.id.z, r.noid.z);
    float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), t0));
    float tx = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fmaxf(az, bz));
    float tf = fminf(tx * kSlabWiden, t1);
    tent = tn;
    return tn <= tf;
}

struct Hit { int tri; float t, u, v; };

// Node i as four 16-byte loads at a 32-bit byte offset from the tree's base
// (one address add per visit instead of 64-bit index arithmetic).
__device__ inline BvhNode load_bvh(const BvhNode* __restrict__ b, int i) {
    const float4* p = reinterpret_cast<const float4*>(reinterpret_cast<const char*>(b) + (uint32_t)i * 64u);
    BvhNode n;
    n.a = p[0];
    n.b = p[1];
    n.c = p[2];
    float4 d = p[3];
    n.d = make_int4(__float_as_int(d.x), __float_as_int(d.y), __float_as_int(d.z), __float_as_int(d.w));
    return n;
}

// Closest hit in (tmin, tmax). `stk` points at this lane's first LDS slot;
// consecutive entries are `stride` words apart.
template <class W>
__device__ inline Hit trace_closest(const SceneView& s, v3 o, v3 d, float tmin, float tmax, int* stk, int stride, W& wk) {
    Hit h{-1, tmax, 0.0f, 0.0f};
    uint32_t nn = 0, nt = 0;
    auto consider_rec = [&](const TriRec& T, int id) {
        ++nt;
        float t, u, v;
        if (tri_hit(T, o, d, t, u, v) && t > tmin && (t < h.t || (t == h.t && id < h.tri))) h = {id, t, u, v};
    };
    if (s.T == 1) {
        consider_rec(load_tri(s.tri, 0), 0);
        wk.ray(0, nt);
        return h;
    }
    RayInv r = ray_inv(o, d);
    int sp = 0;
    int node = 0;
    int guard = 2 * s.T + 8;    // a valid tree visits each node at most once
    while (true) {
        if (--guard < 0) { atomicOr(s.err, kErrStack); break; }
        ++nn;
        BvhNode n = load_bvh(s.bvh, node);
        float tl, tr;
        bool hl = slab(r, n.a.x, n.a.y, n.a.z, n.a.w, n.b.x, n.b.y, tmin, h.t, tl);
        bool hr = slab(r, n.b.z, n.b.w, n.c.x, n.c.y, n.c.z, n.c.w, tmin, h.t, tr);
        int l = n.d.x, rr = n.d.y;
        // leaf children: both triangles are fetched before either is tested
        // (the closest-hit rule is symmetric in the order of the tests)
        bool la = hl && l < 0, lb = hr && rr < 0;
        if (la || lb) {
            int ia = la ? ~l : ~rr;
            TriRec A = load_tri(s.tri, ia), B;
            if (la && lb) B = load_tri(s.tri, ~rr);
            consider_rec(A, ia);
            if (la && lb) consider_rec(B, ~rr);
            if (la) hl = false;
            if (lb) hr = false;
        }
        if (hl && hr) {
            int nearc = tl <= tr ? l : rr, farc = tl <= tr ? rr : l;
            if (sp < s.stk_cap) stk[(sp++) * stride] = farc;
            else atomicOr(s.err, kErrStack);
            node = nearc;
        } else if (hl) {
            node = l;
        } else if (hr) {
            node = rr;
        } else {
            if (sp == 0) break;
            node = stk[(--sp) * stride];
        }
    }
    wk.ray(nn, nt);
    return h;
}

// Closest hits of two rays from one origin (the two sides of a boundary
// sample, a tiny angle apart) in one traversal: a node is entered when either
// ray meets one of its boxes (each against its own closest hit so far), a
// leaf's triangle is fetched once and tested against the rays whose box test
// passed, and each ray keeps its own closest hit with the same tie rule, so
// each result equals that ray's own trace_closest.
template <class W>
__device__ inline void trace_closest2(const SceneView& s, v3 o, v3 da, v3 db, float tmin, float tmax, int* stk, int stride,
                                      W& wk, Hit& ha, Hit& hb) {
    ha = {-1, tmax, 0.0f, 0.0f};
    hb = {-1, tmax, 0.0f, 0.0f};
    uint32_t nn = 0, nt = 0;
    auto consider = [&](const TriRec& T, int id, bool ta, bool tb) {
        ++nt;
        tri_wait(T);
        auto test = [&](v3 d, Hit& h) {
            float t, u, v;
            if (tri_hit_exit(T, o, d, t, u, v) && t > tmin && (t < h.t || (t == h.t && id < h.tri))) h = {id, t, u, v};
        };
        if (ta) test(da, ha);
        if (tb) test(db, hb);
    };
    if (s.T == 1) {
        consider(load_tri(s.tri, 0), 0, true, true);
        wk.ray(0, nt);
        wk.ray(0, 0);
        return;
    }
    const float kInf = __builtin_huge_valf();
    RayInv ra = ray_inv(o, da), rb = ray_inv(o, db);
    int sp = 0;
    int node = 0;
    int guard = 2 * s.T + 8;
    while (true) {
        if (--guard < 0) { atomicOr(s.err, kErrStack); break; }
        ++nn;
        BvhNode n = load_bvh(s.bvh, node);
        float tla, tra, tlb, trb;
        bool hla = slab(ra, n.a.x, n.a.y, n.a.z, n.a.w, n.b.x, n.b.y, tmin, ha.t, tla);
        bool hra = slab(ra, n.b.z, n.b.w, n.c.x, n.c.y, n.c.z, n.c.w, tmin, ha.t, tra);
        bool hlb = slab(rb, n.a.x, n.a.y, n.a.z, n.a.w, n.b.x, n.b.y, tmin, hb.t, tlb);
        bool hrb = slab(rb, n.b.z, n.b.w, n.c.x, n.c.y, n.c.z, n.c.w, tmin, hb.t, trb);
        int l = n.d.x, rr = n.d.y;
        bool la = (hla || hlb) && l < 0, lb = (hra || hrb) && rr < 0;
        if (la || lb) {
            int ia = la ? ~l : ~rr;
            TriRec A = load_tri(s.tri, ia), B;
            if (la && lb) B = load_tri(s.tri, ~rr);
            if (la) consider(A, ia, hla, hlb);
            else consider(A, ia, hra, hrb);
            if (la && lb) consider(B, ~rr, hra, hrb);
            if (la) hla = hlb = false;
            if (lb) hra = hrb = false;
        }
        bool hl = hla || hlb, hr = hra || hrb;
        if (hl && hr) {
            float tl = fminf(hla ? tla : kInf, hlb ? tlb : kInf), tr = fminf(hra ? tra : kInf, hrb ? trb : kInf);
            int nearc = tl <= tr ? l : rr, farc = tl <= tr ? rr : l;
            if (sp < s.stk_cap) stk[(sp++) * stride] = farc;
            else atomicOr(s.err, kErrStack);
            node = nearc;
        } else if (hl) {
            node = l;
        } else if (hr) {
            node = rr;
        } else {
            if (sp == 0) break;
            node = stk[(--sp) * stride];
        }
    }
    // one traversal, two rays
    wk.ray(nn, nt);
    wk.ray(0, 0);
}

// Any hit in (tmin, tmax).
template <class W>
__device__ inline bool trace_any(const SceneView& s, v3 o, v3 d, float tmin, float tmax, int* stk, int stride, W& wk) {
    uint32_t nn = 0, nt = 0;
    auto test_rec = [&](const TriRec& T) {
        ++nt;
        float t, u, v;
        return tri_hit(T, o, d, t, u, v) && t > tmin && t < tmax;
    };
    if (s.T == 1) {
        bool r0 = test_rec(load_tri(s.tri, 0));
        wk.ray(0, nt);
        return r0;
    }
    RayInv r = ray_inv(o, d);
    int sp = 0;
    int node = 0;
    int guard = 2 * s.T + 8;
    bool hit = false;
    while (true) {
        if (--guard < 0) { atomicOr(s.err, kErrStack); break; }
        ++nn;
        BvhNode n = load_bvh(s.bvh, node);
        float tl, tr;
        bool hl = slab(r, n.a.x, n.a.y, n.a.z, n.a.w, n.b.x, n.b.y, tmin, tmax, tl);
        bool hr = slab(r, n.b.z, n.b.w, n.c.x, n.c.y, n.c.z, n.c.w, tmin, tmax, tr);
        int l = n.d.x, rr = n.d.y;
        bool la = hl && l < 0, lb = hr && rr < 0;
        if (la || lb) {
            int ia = la ? ~l : ~rr;
            TriRec A = load_tri(s.tri, ia), B;
            if (la && lb) B = load_tri(s.tri, ~rr);
            bool any = test_rec(A);
            if (la && lb) any |= test_rec(B);
            if (any) { hit = true; break; }
            if (la) hl = false;
            if (lb) hr = false;
        }
        if (hl && hr) {
            if (sp < s.stk_cap) stk[(sp++) * stride] = rr;
            else atomicOr(s.err, kErrStack);
            node = l;
        } else if (hl) {
            node = l;
        } else if (hr) {
            node = rr;
        } else {
            if (sp == 0) break;
            node = stk[(--sp) * stride];
        }
    }
    wk.ray(nn, nt);
    return hit;
}

}  // namespace dr
