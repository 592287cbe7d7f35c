// Ray casting on the triangle LBVH: Moller-Trumbore intersection in FP32,
// closest-hit (ties in t go to the smaller triangle id) and any-hit
// traversal. Each lane keeps its traversal stack in LDS, strided by the
// block size so that the 64 lanes of a wave touch 64 consecutive words.
#pragma once
#include "dr_common.h"

namespace dr {

__device__ inline bool tri_test(const float4* __restrict__ tri, int id, v3 o, v3 d, float& t, float& u, float& v) {
    float4 a = tri[3 * id], b = tri[3 * id + 1], c = tri[3 * id + 2];
    v3 v0 = {a.x, a.y, a.z}, e1 = {a.w, b.x, b.y}, e2 = {b.z, b.w, c.x};
    v3 pv = cross(d, e2);
    float det = dot(e1, pv);
    if (det == 0.0f) return false;
    float inv = 1.0f / det;
    v3 tv = o - v0;
    u = dot(tv, pv) * inv;
    if (u < 0.0f || u > 1.0f) return false;
    v3 qv = cross(tv, e1);
    v = dot(d, qv) * inv;
    if (v < 0.0f || u + v > 1.0f) return false;
    t = dot(e2, qv) * inv;
    return true;
}

struct RayInv { v3 o, id; };

__device__ inline RayInv ray_inv(v3 o, v3 d) {
    auto inv = [](float x) { return fabsf(x) > 1e-30f ? 1.0f / x : copysignf(1e30f, x); };
    return {o, {inv(d.x), inv(d.y), inv(d.z)}};
}

// slab test of [lo, hi] against the ray over [t0, t1]; returns entry distance
__device__ inline bool slab(const RayInv& r, float lx, float ly, float lz, float hx, float hy, float hz, float t0, float t1,
                            float& tent) {
    float ax = (lx - r.o.x) * r.id.x, bx = (hx - r.o.x) * r.id.x;
    float ay = (ly - r.o.y) * r.id.y, by = (hy - r.o.y) * r.id.y;
    float az = (lz - r.o.z) * r.id.z, bz = (hz - r.o.z) * r.id.z;
    float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), t0));
    float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), t1));
    tent = tn;
    return tn <= tf;
}

struct Hit { int tri; float t, u, v; };

// Closest hit in (tmin, tmax). `stk` points at this lane's first LDS slot;
// consecutive entries are `stride` words apart.
template <class W>
__device__ inline Hit trace_closest(const SceneView& s, v3 o, v3 d, float tmin, float tmax, int* stk, int stride, W& wk) {
    Hit h{-1, tmax, 0.0f, 0.0f};
    uint32_t nn = 0, nt = 0;
    auto consider = [&](int id) {
        ++nt;
        float t, u, v;
        if (tri_test(s.tri, id, o, d, t, u, v) && t > tmin && (t < h.t || (t == h.t && id < h.tri))) h = {id, t, u, v};
    };
    if (s.T == 1) {
        consider(0);
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
        BvhNode n = s.bvh[node];
        float tl, tr;
        bool hl = slab(r, n.a.x, n.a.y, n.a.z, n.a.w, n.b.x, n.b.y, tmin, h.t, tl);
        bool hr = slab(r, n.b.z, n.b.w, n.c.x, n.c.y, n.c.z, n.c.w, tmin, h.t, tr);
        int l = n.d.x, rr = n.d.y;
        if (hl && l < 0) { consider(~l); hl = false; }
        if (hr && rr < 0) { consider(~rr); hr = false; }
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
    auto consider = [&](int id, bool ta, bool tb) {
        ++nt;
        float4 a = s.tri[3 * id], b = s.tri[3 * id + 1], c = s.tri[3 * id + 2];
        v3 v0 = {a.x, a.y, a.z}, e1 = {a.w, b.x, b.y}, e2 = {b.z, b.w, c.x};
        auto test = [&](v3 d, Hit& h) {
            v3 pv = cross(d, e2);
            float det = dot(e1, pv);
            if (det == 0.0f) return;
            float inv = 1.0f / det;
            v3 tv = o - v0;
            float u = dot(tv, pv) * inv;
            if (u < 0.0f || u > 1.0f) return;
            v3 qv = cross(tv, e1);
            float v = dot(d, qv) * inv;
            if (v < 0.0f || u + v > 1.0f) return;
            float t = dot(e2, qv) * inv;
            if (t > tmin && (t < h.t || (t == h.t && id < h.tri))) h = {id, t, u, v};
        };
        if (ta) test(da, ha);
        if (tb) test(db, hb);
    };
    if (s.T == 1) {
        consider(0, true, true);
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
        BvhNode n = s.bvh[node];
        float tla, tra, tlb, trb;
        bool hla = slab(ra, n.a.x, n.a.y, n.a.z, n.a.w, n.b.x, n.b.y, tmin, ha.t, tla);
        bool hra = slab(ra, n.b.z, n.b.w, n.c.x, n.c.y, n.c.z, n.c.w, tmin, ha.t, tra);
        bool hlb = slab(rb, n.a.x, n.a.y, n.a.z, n.a.w, n.b.x, n.b.y, tmin, hb.t, tlb);
        bool hrb = slab(rb, n.b.z, n.b.w, n.c.x, n.c.y, n.c.z, n.c.w, tmin, hb.t, trb);
        int l = n.d.x, rr = n.d.y;
        if ((hla || hlb) && l < 0) { consider(~l, hla, hlb); hla = hlb = false; }
        if ((hra || hrb) && rr < 0) { consider(~rr, hra, hrb); hra = hrb = false; }
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
    auto test = [&](int id) {
        ++nt;
        float t, u, v;
        return tri_test(s.tri, id, o, d, t, u, v) && t > tmin && t < tmax;
    };
    if (s.T == 1) {
        bool r0 = test(0);
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
        BvhNode n = s.bvh[node];
        float tl, tr;
        bool hl = slab(r, n.a.x, n.a.y, n.a.z, n.a.w, n.b.x, n.b.y, tmin, tmax, tl);
        bool hr = slab(r, n.b.z, n.b.w, n.c.x, n.c.y, n.c.z, n.c.w, tmin, tmax, tr);
        int l = n.d.x, rr = n.d.y;
        if (hl && l < 0) { if (test(~l)) { hit = true; break; } hl = false; }
        if (hr && rr < 0) { if (test(~rr)) { hit = true; break; } hr = false; }
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
