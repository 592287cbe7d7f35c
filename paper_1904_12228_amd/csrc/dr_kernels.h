// Forward and backward kernels of the edge-sampling differentiable path
// tracer (thesis Ch. 5), shared by the translation units that instantiate and
// launch them (dr_render*.hip; each compiles only the variants it launches).
// One lane per unit: a unit is one pixel sample (its
// path, interior adjoint and one secondary edge sample per path vertex) plus
// one primary edge sample. Blocks are one 64-lane wave; each lane's BVH
// traversal stack lives in LDS.
//
// Measure convention of the interior term: the screen sample, every sampled
// world direction and every sampling pdf are held fixed (the integrals are
// over screen space and over the sphere of directions at each vertex); hit
// points move by ray-plane intersection with their triangles. The boundary
// terms use the matching measures: screen-space edges (eq. mc) and
// direction-space edges at each vertex (eq. dirac_3d_edge in the solid-angle
// measure; its endpoint terms equal the thesis's area form exactly).
#pragma once
#include <cstdlib>
#include <type_traits>

#include "dr_args.h"
#include "dr_host.h"
#include "dr_path.h"

#pragma clang diagnostic ignored "-Wunused-function"
// Per-sample device printf of the unit RenderArgs::debug_unit names (primary
// edge sample, edge-tree levels, secondary samples) is compiled only with
// -DDIFFRT_DEVICE_PRINTF: the printf machinery costs the kernels registers.

namespace dr {

__device__ inline void unit_pixel(const Cam& k, const RenderArgs& a, int m, int& pix, int& px, int& py, uint32_t& sid) {
    pix = m / a.spp;
    int smp = m - pix * a.spp;
    int pxr = pix % a.Ww, pyr = pix / a.Ww;
    px = k.x0 + pxr;
    py = k.y0 + pyr;
    sid = ((uint32_t)py * (uint32_t)k.W + (uint32_t)px) * (uint32_t)a.spp + (uint32_t)smp;
}

__device__ inline void flush_work(const NoWork&, unsigned long long*) {}

__device__ inline void flush_work(const Work& w, unsigned long long* c) {
    if (!c) return;
    uint32_t v[5] = {w.nodes, w.tris, w.tnodes, w.atom, w.rays};
    for (int i = 0; i < 5; ++i) {
        uint32_t t = v[i];
        for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, BS);
        if (threadIdx.x == 0 && t) atomicAdd(&c[i], (unsigned long long)t);
    }
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
// One wave of units [mbase, mbase + 64) of one view; stk: the block's LDS
// traversal stacks.
template <int STK, bool CNT>
__device__ __forceinline__ void forward_body(const SceneView& s, const Cam& k, const RenderArgs& a, float* __restrict__ image,
                                             int reduce, int mbase, int* stk) {
    int lane = threadIdx.x;
    int* my = stk + lane;
    int m = mbase + lane;
    float L = 0.0f;
    int pix = 0;
    typename std::conditional<CNT, Work, NoWork>::type wk;
    if (m < a.M) {
        int px, py;
        uint32_t sid;
        unit_pixel(k, a, m, pix, px, py, sid);
        bool act = !a.mask || a.mask[m];
        int ckt0 = -1, ckt1 = -1, ckt2 = -1;
        v3 ckx0 = {0, 0, 0}, ckx1 = {0, 0, 0}, ckx2 = {0, 0, 0};
        uint8_t vis = 0;
        if (act) {
            Rng rc{sid, a.view, kTagCam, a.k0, a.k1};
            float4 j = rc.block(0);
            v3 d = cam_dir(k, px + j.x, py + j.y);
            Hit h = trace_closest(s, k.c, d, k.nearc, 3.0e38f, my, BS, wk);
            if (h.tri < 0) {
                L = s.background;
            } else {
                int tri = h.tri;
                TriGeom g = tri_geom(s, tri);
                v3 x = hit_point(g, k.c, d);
                bool front = dot(d, cross(g.e1, g.e2)) < 0.0f;
                L = emitted(s, tri, front);
                ckt0 = tri;
                ckx0 = x;
                float beta = 1.0f;
                for (int kk = 1; kk <= a.depth; ++kk) {
                    v3 ns = shading_normal(s, tri, g, x);
                    if (!front) ns = -ns;
                    float rho = s.alb[tri];
                    if (rho == 0.0f) break;
                    NeeSample q = nee_sample(s, rc.block(2 * kk - 1), x, ns);
                    if (q.K > 0.0f && !trace_any(s, x, q.w, s.tmin, q.r * (1.0f - kShadowEnd), my, BS, wk)) {
                        L += beta * rho * dot(ns, q.w) * q.K;
                        vis |= (uint8_t)(1u << (kk - 1));
                    }
                    if (kk == a.depth) break;
                    float4 ub = rc.block(2 * kk);
                    v3 w = cosine_dir(ns, ub.x, ub.y);
                    if (dot(ns, w) <= 0.0f) break;
                    Hit h2 = trace_closest(s, x, w, s.tmin, 3.0e38f, my, BS, wk);
                    if (h2.tri < 0) break;
                    beta *= rho;
                    tri = h2.tri;
                    g = tri_geom(s, tri);
                    x = hit_point(g, x, w);
                    front = dot(w, cross(g.e1, g.e2)) < 0.0f;
                    if (kk == 1) { ckt1 = tri; ckx1 = x; }
                    if (kk == 2) { ckt2 = tri; ckx2 = x; }
                }
            }
        }
        if (a.ck_tri) {
            a.ck_tri[m] = ckt0;
            a.ck_tri[a.M + m] = ckt1;
            a.ck_tri[2 * (size_t)a.M + m] = ckt2;
            float* cx = a.ck_x + 3 * (size_t)m;
            cx[0] = ckx0.x; cx[1] = ckx0.y; cx[2] = ckx0.z;
            float* cy = a.ck_x + 3 * ((size_t)a.M + m);
            cy[0] = ckx1.x; cy[1] = ckx1.y; cy[2] = ckx1.z;
            float* cz = a.ck_x + 3 * (2 * (size_t)a.M + m);
            cz[0] = ckx2.x; cz[1] = ckx2.y; cz[2] = ckx2.z;
            a.ck_vis[m] = vis;
        }
    }
    flush_work(wk, a.counters);
    float v = L / (float)a.spp;
    if (reduce) {
        // a.spp divides 64: lanes of one pixel are consecutive, reduce in-wave
        for (int off = a.spp >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, BS);
        if (m < a.M && (lane % a.spp) == 0) image[pix] = v;
    } else if (m < a.M) {
        atomicAdd(&image[pix], v);
    }
}

// Six waves per SIMD (at most 80 VGPRs, a few spilled) measured faster than
// five; the side-path and edge-sampling kernels lose more to their spills.
template <int STK, bool CNT>
__global__ __launch_bounds__(BS, 6) void k_forward(SceneView s, Cam k, RenderArgs a, float* __restrict__ image, int reduce) {
    __shared__ int stk[STK * BS];
    forward_body<STK, CNT>(s, k, a, image, reduce, blockIdx.x * BS, stk);
}

// ---------------------------------------------------------------------------
// Wavefront forward (max_depth 2 or 3): the camera paths of k_forward split
// at their continuation rays. k_fwd_hit traces every camera ray, does the
// first vertex's next-event estimation, stores the first checkpoint and, for
// the paths that continue, appends (unit, direction) to the queue of bounce 1
// (wave ballot + popcount, one atomic per wave). k_fwd_bounce<k> drains the
// queue of bounce k on a persistent grid: it traces the continuation ray
// from checkpoint k - 1, stores checkpoint k, adds vertex k + 1's
// next-event estimation to the unit's radiance and queues the next bounce.
// Every unit's arithmetic is k_forward's, step for step (beta is rebuilt as
// the same product of checkpointed albedos), so radiance, checkpoints and
// visibility bits are bit-identical; k_fwd_image reduces the radiance to
// pixels as k_forward does.
// ---------------------------------------------------------------------------
struct FwdQueue {
    int4* q;        // [2][M]: unit, direction bits (bounce k at offset (k - 1) M)
    int* count;     // [2]
    float* L;       // [M] radiance of each unit
};

__device__ inline void fwd_push(const FwdQueue& fq, int M, int k, bool push, int m, v3 w) {
    int lane = threadIdx.x;
    unsigned long long bal = __ballot(push);
    if (!bal) return;
    int leader = __ffsll(bal) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(&fq.count[k - 1], __popcll(bal));
    base = __shfl(base, leader, BS);
    if (push)
        fq.q[(size_t)(k - 1) * M + base + __popcll(bal & ((1ull << lane) - 1ull))] =
            make_int4(m, __float_as_int(w.x), __float_as_int(w.y), __float_as_int(w.z));
}

// Next-event estimation at path vertex kk (x on triangle tri, facing ns), and
// the continuation direction when kk < depth; returns whether the path goes
// on (k_forward's loop body up to its continuation ray).
template <class W>
__device__ inline bool fwd_vertex(const SceneView& s, const RenderArgs& a, const Rng& rc, int kk, int tri, v3 x, v3 ns,
                                  float beta, float& L, uint8_t& vis, v3& w, int* my, W& wk) {
    float rho = s.alb[tri];
    if (rho == 0.0f) return false;
    NeeSample q = nee_sample(s, rc.block(2 * kk - 1), x, ns);
    if (q.K > 0.0f && !trace_any(s, x, q.w, s.tmin, q.r * (1.0f - kShadowEnd), my, BS, wk)) {
        L += beta * rho * dot(ns, q.w) * q.K;
        vis |= (uint8_t)(1u << (kk - 1));
    }
    if (kk == a.depth) return false;
    float4 ub = rc.block(2 * kk);
    w = cosine_dir(ns, ub.x, ub.y);
    return dot(ns, w) > 0.0f;
}

template <int STK>
__global__ __launch_bounds__(BS, 6) void k_fwd_hit(SceneView s, Cam k, RenderArgs a, FwdQueue fq) {
    __shared__ int stk[STK * BS];
    int lane = threadIdx.x;
    int* my = stk + lane;
    int m = blockIdx.x * BS + lane;
    NoWork wk;
    bool push = false;
    v3 w = {0, 0, 0};
    if (m < a.M) {
        int pix, px, py;
        uint32_t sid;
        unit_pixel(k, a, m, pix, px, py, sid);
        float L = 0.0f;
        uint8_t vis = 0;
        int ckt0 = -1;
        v3 ckx0 = {0, 0, 0};
        if (!a.mask || a.mask[m]) {
            Rng rc{sid, a.view, kTagCam, a.k0, a.k1};
            float4 j = rc.block(0);
            v3 d = cam_dir(k, px + j.x, py + j.y);
            Hit h = trace_closest(s, k.c, d, k.nearc, 3.0e38f, my, BS, wk);
            if (h.tri < 0) {
                L = s.background;
            } else {
                TriGeom g = tri_geom(s, h.tri);
                v3 x = hit_point(g, k.c, d);
                bool front = dot(d, cross(g.e1, g.e2)) < 0.0f;
                L = emitted(s, h.tri, front);
                ckt0 = h.tri;
                ckx0 = x;
                v3 ns = shading_normal(s, h.tri, g, x);
                if (!front) ns = -ns;
                push = fwd_vertex(s, a, rc, 1, h.tri, x, ns, 1.0f, L, vis, w, my, wk);
            }
        }
        a.ck_tri[m] = ckt0;
        a.ck_tri[a.M + m] = -1;
        a.ck_tri[2 * (size_t)a.M + m] = -1;
        float* cx = a.ck_x + 3 * (size_t)m;
        cx[0] = ckx0.x; cx[1] = ckx0.y; cx[2] = ckx0.z;
        float* cy = a.ck_x + 3 * ((size_t)a.M + m);
        cy[0] = 0.0f; cy[1] = 0.0f; cy[2] = 0.0f;
        float* cz = a.ck_x + 3 * (2 * (size_t)a.M + m);
        cz[0] = 0.0f; cz[1] = 0.0f; cz[2] = 0.0f;
        a.ck_vis[m] = vis;
        fq.L[m] = L;
    }
    fwd_push(fq, a.M, 1, push, m, w);
}

template <int STK, int K>
__global__ __launch_bounds__(BS, 6) void k_fwd_bounce(SceneView s, Cam k, RenderArgs a, FwdQueue fq) {
    __shared__ int stk[STK * BS];
    int lane = threadIdx.x;
    int* my = stk + lane;
    NoWork wk;
    int n = fq.count[K - 1];
    for (int base = blockIdx.x * BS; base < n; base += gridDim.x * BS) {
        bool in = base + lane < n;
        bool push = false;
        int m = 0;
        v3 w = {0, 0, 0};
        if (in) {
            int4 e = fq.q[(size_t)(K - 1) * a.M + base + lane];
            m = e.x;
            v3 d = {__int_as_float(e.y), __int_as_float(e.z), __int_as_float(e.w)};
            const float* cp = a.ck_x + 3 * ((size_t)(K - 1) * a.M + m);
            v3 x = {cp[0], cp[1], cp[2]};
            Hit h = trace_closest(s, x, d, s.tmin, 3.0e38f, my, BS, wk);
            if (h.tri >= 0) {
                // the albedos of the vertices left so far, multiplied in path order
                float beta = 1.0f;
                for (int j = 0; j < K; ++j) beta *= s.alb[a.ck_tri[(size_t)j * a.M + m]];
                TriGeom g = tri_geom(s, h.tri);
                v3 x2 = hit_point(g, x, d);
                bool front = dot(d, cross(g.e1, g.e2)) < 0.0f;
                a.ck_tri[(size_t)K * a.M + m] = h.tri;
                float* cq = a.ck_x + 3 * ((size_t)K * a.M + m);
                cq[0] = x2.x; cq[1] = x2.y; cq[2] = x2.z;
                int pix, px, py;
                uint32_t sid;
                unit_pixel(k, a, m, pix, px, py, sid);
                Rng rc{sid, a.view, kTagCam, a.k0, a.k1};
                v3 ns = shading_normal(s, h.tri, g, x2);
                if (!front) ns = -ns;
                float L = fq.L[m];
                uint8_t vis = a.ck_vis[m];
                push = fwd_vertex(s, a, rc, K + 1, h.tri, x2, ns, beta, L, vis, w, my, wk);
                fq.L[m] = L;
                a.ck_vis[m] = vis;
            }
        }
        if (K + 1 < 3) fwd_push(fq, a.M, K + 1, push, m, w);
    }
}

// Pixels from the units' radiance, as k_forward ends.
static __global__ __launch_bounds__(BS) void k_fwd_image(RenderArgs a, const float* __restrict__ L,
                                                         float* __restrict__ image, int reduce) {
    int lane = threadIdx.x;
    int m = blockIdx.x * BS + lane;
    int pix = m / a.spp;
    float v = (m < a.M ? L[m] : 0.0f) / (float)a.spp;
    if (reduce) {
        for (int off = a.spp >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, BS);
        if (m < a.M && (lane % a.spp) == 0) image[pix] = v;
    } else if (m < a.M) {
        atomicAdd(&image[pix], v);
    }
}

// Geometry buffers (Ch. 5, Results): channel a.aov (1..7) of the first hit of
// each camera ray, or all seven (a.aov = 8; image [7][Hw][Ww]); 0 where the
// ray escapes. Stores the first-hit checkpoint the backward pass reuses.
template <int STK>
__global__ __launch_bounds__(BS) void k_forward_aov(SceneView s, Cam k, RenderArgs a, float* __restrict__ image,
                                                    int reduce) {
    __shared__ int stk[STK * BS];
    int lane = threadIdx.x;
    int* my = stk + lane;
    int m = blockIdx.x * BS + lane;
    NoWork wk;
    float v[7] = {0, 0, 0, 0, 0, 0, 0};
    int pix = 0;
    if (m < a.M) {
        int px, py;
        uint32_t sid;
        unit_pixel(k, a, m, pix, px, py, sid);
        int ckt = -1;
        v3 ckx = {0, 0, 0};
        if (!a.mask || a.mask[m]) {
            Rng rc{sid, a.view, kTagCam, a.k0, a.k1};
            float4 j = rc.block(0);
            v3 d = cam_dir(k, px + j.x, py + j.y);
            Hit h = trace_closest(s, k.c, d, k.nearc, 3.0e38f, my, BS, wk);
            if (h.tri >= 0) {
                TriGeom g = tri_geom(s, h.tri);
                v3 x = hit_point(g, k.c, d);
                if (a.aov == 8) aov_values(s, h.tri, g, x, d, v);
                else v[0] = aov_value(s, a.aov, h.tri, g, x, d);
                ckt = h.tri;
                ckx = x;
            }
        }
        if (a.ck_tri) {
            a.ck_tri[m] = ckt;
            a.ck_tri[a.M + m] = -1;
            a.ck_tri[2 * (size_t)a.M + m] = -1;
            float* cx = a.ck_x + 3 * (size_t)m;
            cx[0] = ckx.x; cx[1] = ckx.y; cx[2] = ckx.z;
            a.ck_vis[m] = 0;
        }
    }
    int nch = a.aov == 8 ? 7 : 1;
    long npix = (long)a.Ww * (k.y1 - k.y0);
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        if (c >= nch) break;
        float val = v[c] / (float)a.spp;
        if (reduce) {
            for (int off = a.spp >> 1; off > 0; off >>= 1) val += __shfl_xor(val, off, BS);
            if (m < a.M && (lane % a.spp) == 0) image[c * npix + pix] = val;
        } else if (m < a.M) {
            atomicAdd(&image[c * npix + pix], val);
        }
    }
}

// ---------------------------------------------------------------------------
// adjoint helpers
// ---------------------------------------------------------------------------
struct CamAcc { v3 f, r, u, c; };

__device__ inline void atomic_add3(float* p, int i, v3 v) {
    if (v.x != 0.0f) atomicAdd(&p[3 * i], v.x);
    if (v.y != 0.0f) atomicAdd(&p[3 * i + 1], v.y);
    if (v.z != 0.0f) atomicAdd(&p[3 * i + 2], v.z);
}

// Adjoint of the projection to pixels.
__device__ inline v3 project_adj(const Cam& k, v3 P, float gsx, float gsy, CamAcc& ca) {
    v3 q = P - k.c;
    float z = dot(q, k.f), xc = dot(q, k.r), yc = dot(q, k.u);
    float ax = k.W * 0.5f / (k.asp * k.th), ay = k.H * 0.5f / k.th;
    float gxc = gsx * ax / z;
    float gyc = -gsy * ay / z;
    float gz = -gsx * ax * xc / (z * z) + gsy * ay * yc / (z * z);
    v3 gq = k.f * gz + k.r * gxc + k.u * gyc;
    ca.f += q * gz;
    ca.r += q * gxc;
    ca.u += q * gyc;
    ca.c -= gq;
    return gq;
}

// Adjoint of a* = a + (b - a) s, s = (zd - za)/(zb - za), zd = max(near, zb/2).
__device__ inline void nearclip_adj(const Cam& k, v3 a, v3 b, v3 g, v3& ga, v3& gb, CamAcc& ca) {
    float za = dot(a - k.c, k.f), zb = dot(b - k.c, k.f);
    float D = zb - za;
    bool half = 0.5f * zb > k.nearc;
    float zd = half ? 0.5f * zb : k.nearc;
    float s = (zd - za) / D;
    ga += g * (1.0f - s);
    gb += g * s;
    float gs = dot(g, b - a);
    float gza = gs * (s - 1.0f) / D, gzb = gs * ((half ? 0.5f : 0.0f) - s) / D;
    ga += k.f * gza;
    gb += k.f * gzb;
    ca.c -= k.f * (gza + gzb);
    ca.f += (a - k.c) * gza + (b - k.c) * gzb;
}

// Adjoint of x = o + d t, t = (p0 - o).n / (d.n), n = e1 x e2.
__device__ inline void ray_plane_adj(const TriGeom& g, v3 o, v3 d, v3 gx, v3& go, v3& gd, v3& gp0, v3& gp1, v3& gp2) {
    v3 n = cross(g.e1, g.e2);
    float den = dot(d, n);
    float num = dot(g.p0 - o, n);
    float t = num / den;
    go += gx;
    gd += gx * t;
    float gt = dot(gx, d);
    float gnum = gt / den, gden = -gt * t / den;
    gp0 += n * gnum;
    go -= n * gnum;
    v3 gn = (g.p0 - o) * gnum + d * gden;
    gd += n * gden;
    v3 ge1 = cross(g.e2, gn), ge2 = cross(gn, g.e1);
    gp1 += ge1;
    gp2 += ge2;
    gp0 -= ge1 + ge2;
}

// Adjoint of the shading normal (unoriented) w.r.t. the hit point and the
// triangle vertices; gns is dL/d(normal before orientation).
__device__ inline void shading_normal_adj(const SceneView& s, int id, const TriGeom& g, v3 x, v3 gns, v3& gx, v3& gp0, v3& gp1,
                                          v3& gp2) {
    v3 n = cross(g.e1, g.e2);
    v3 gn = {0, 0, 0}, ge1 = {0, 0, 0}, ge2 = {0, 0, 0};
    if (!s.N) {
        gn = nrm_adj(n, gns);
    } else {
        v3 w = x - g.p0;
        float nn = dot(n, n);
        v3 c1 = cross(w, g.e2), c2 = cross(g.e1, w);
        float b1 = dot(c1, n) / nn, b2 = dot(c2, n) / nn;
        int i0 = s.I[3 * id], i1 = s.I[3 * id + 1], i2 = s.I[3 * id + 2];
        v3 N0 = ld3(s.N, i0), N1 = ld3(s.N, i1), N2 = ld3(s.N, i2);
        v3 mv = N0 * (1.0f - b1 - b2) + N1 * b1 + N2 * b2;
        v3 gm = nrm_adj(mv, gns);
        float gb1 = dot(gm, N1 - N0), gb2 = dot(gm, N2 - N0);
        float gq1 = gb1 / nn, gq2 = gb2 / nn;
        float gnn = -(gb1 * b1 + gb2 * b2) / nn;
        v3 gc1 = n * gq1, gc2 = n * gq2;
        gn += c1 * gq1 + c2 * gq2 + n * (2.0f * gnn);
        v3 gw = cross(g.e2, gc1) + cross(gc2, g.e1);
        ge2 += cross(gc1, w);
        ge1 += cross(w, gc2);
        gx += gw;
        gp0 -= gw;
    }
    ge1 += cross(g.e2, gn);
    ge2 += cross(gn, g.e1);
    gp1 += ge1;
    gp2 += ge2;
    gp0 -= ge1 + ge2;
}

__device__ inline float wave_sum(float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, BS);
    return v;
}

__device__ inline float wave_sum_all(float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, BS);
    return v;
}

// Gradient scatter with in-wave pre-reduction. Lanes holding the same key
// (an edge or a triangle) are summed with cross-lane shuffles and one lane
// issues the atomics, which removes same-address atomic contention when the
// lanes of a wave work on the same primitive (all samples of a pixel, or the
// stratified primary edge samples). After `max_groups` distinct keys the
// remaining lanes add their values directly. Must be called by all lanes.
template <int N, class Dest>
__device__ inline void scatter_grouped(bool valid, int key, const float (&vals)[N], int max_groups, Dest dest) {
    const int lane = threadIdx.x;
    unsigned long long active = __ballot(valid);
    for (int it = 0; active; ++it) {
        if (it == max_groups) {
            if ((active >> lane) & 1ull)
#pragma unroll
                for (int i = 0; i < N; ++i)
                    if (vals[i] != 0.0f) atomicAdd(dest(key, i), vals[i]);
            break;
        }
        int leader = __ffsll(active) - 1;
        int lkey = __shfl(key, leader, BS);
        bool mine = ((active >> lane) & 1ull) && key == lkey;
        unsigned long long grp = __ballot(mine);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            float v = wave_sum_all(mine ? vals[i] : 0.0f);
            if (lane == leader && v != 0.0f) atomicAdd(dest(lkey, i), v);
        }
        active &= ~grp;
    }
}

__device__ inline void flush_cam(const CamAcc& ca, float* camacc) {
    float v[12] = {ca.f.x, ca.f.y, ca.f.z, ca.r.x, ca.r.y, ca.r.z, ca.u.x, ca.u.y, ca.u.z, ca.c.x, ca.c.y, ca.c.z};
    for (int i = 0; i < 12; ++i) {
        float t = wave_sum(v[i]);
        if (threadIdx.x == 0 && t != 0.0f) atomicAdd(&camacc[i], t);
    }
}

// ---------------------------------------------------------------------------
// primary edge samples (eq. mc): one per unit
// ---------------------------------------------------------------------------
// Geometry of unit m's primary edge sample: the edge (stratified choice by
// the CDF), the point on its clipped screen segment, the edge equation's two
// defining points (near-clipped alpha points), the two side rays and the
// pixel whose loss gradient weights the sample.
struct PrimGeom {
    int ei;
    bool live;
    double inv_p, p_edge;    // 1 / (P(edge) p(point | edge)); P(edge)
    float x, y, Ax, Ay, Bx, By, nl;
    float za, zb;
    v3 va, vb, ac, bc, du, dl;
    int pix;                 // offset of the sample's pixel in the window
};

template <bool MIX>
__device__ inline PrimGeom prim_geom(const SceneView& s, const Cam& k, const RenderArgs& a, const PEdge* __restrict__ pe,
                                     const double* __restrict__ cdf, const MixArgs& mx, int m, const float4& b0) {
    PrimGeom G;
    double total = cdf[s.E];
    // stratified edge choice: unit m draws its uniform in [m/M, (m+1)/M), so
    // the lanes of a wave take neighbouring edges in CDF order
    bool mixp = MIX && mx.prim;
    G.ei = pick_cdf_d(mixp ? mx.mcdf : cdf, s.E, ((double)m + (double)b0.x) / (double)a.M);
    // 1 / (P(edge) p(point | edge)), the point uniform on the clipped segment
    G.inv_p = total;
    G.p_edge = 0.0;
    G.live = true;
    if (MIX) {
        double l = mx.plen[G.ei];
        G.p_edge = mixp ? ((1.0 - (double)mx.mix) * l / total + (double)mx.mix * (double)mx.q[G.ei]) / mx.mcdf[s.E]
                        : l / total;
        G.live = l > 0.0;
        if (G.live) G.inv_p = l / G.p_edge;
    }
    if (!G.live) return G;
    PEdge p = pe[G.ei];
    float t = b0.y;
    G.x = p.Ac[0] + (p.Bc[0] - p.Ac[0]) * t;
    G.y = p.Ac[1] + (p.Bc[1] - p.Ac[1]) * t;
    int4 e = s.edges[G.ei];
    G.va = ld3(s.P, e.x);
    G.vb = ld3(s.P, e.y);
    G.za = dot(G.va - k.c, k.f);
    G.zb = dot(G.vb - k.c, k.f);
    G.ac = G.za < k.nearc ? alpha_point(k, G.va, G.vb, G.za, G.zb) : G.va;
    G.bc = G.zb < k.nearc ? alpha_point(k, G.vb, G.va, G.zb, G.za) : G.vb;
    project(k, G.ac, G.Ax, G.Ay);
    project(k, G.bc, G.Bx, G.By);
    float dx = G.Ax - G.Bx, dy = G.Ay - G.By;
    G.nl = sqrtf(dx * dx + dy * dy);
    float nx = (G.Ay - G.By) / G.nl, ny = (G.Bx - G.Ax) / G.nl;
    G.du = cam_dir(k, G.x + kEpsPx * nx, G.y + kEpsPx * ny);
    G.dl = cam_dir(k, G.x - kEpsPx * nx, G.y - kEpsPx * ny);
    int ix = min(max((int)floorf(G.x), k.x0), k.x1 - 1);
    int iy = min(max((int)floorf(G.y), k.y0), k.y1 - 1);
    G.pix = (iy - k.y0) * a.Ww + (ix - k.x0);
    return G;
}

// Gradient of the edge's two endpoints (6 numbers) and the camera frame
// (accumulated into ca) from the sample's loss-weighted jump.
__device__ inline void prim_contrib(const Cam& k, const RenderArgs& a, const PrimGeom& G, float jump, float (&gv)[6],
                                    CamAcc& ca) {
    float w = jump * (float)(G.inv_p / (double)a.M) / G.nl;
    // d alpha / d(a, b) (eq. redner_dirac_jacobian) at the sample point
    float gax = w * (G.By - G.y), gay = w * (G.x - G.Bx);
    float gbx = w * (G.y - G.Ay), gby = w * (G.Ax - G.x);
    v3 gac = project_adj(k, G.ac, gax, gay, ca);
    v3 gbc = project_adj(k, G.bc, gbx, gby, ca);
    v3 ga = {0, 0, 0}, gb = {0, 0, 0};
    if (G.za < k.nearc) nearclip_adj(k, G.va, G.vb, gac, ga, gb, ca);
    else ga += gac;
    if (G.zb < k.nearc) nearclip_adj(k, G.vb, G.va, gbc, gb, ga, ca);
    else gb += gbc;
    gv[0] = ga.x; gv[1] = ga.y; gv[2] = ga.z;
    gv[3] = gb.x; gv[4] = gb.y; gv[5] = gb.z;
}

template <int STK, bool CNT, bool MIX, bool AOV = false>
__device__ __forceinline__ void primary_body(const SceneView& s, const Cam& k, const RenderArgs& a, const PEdge* __restrict__ pe,
                                             const double* __restrict__ cdf, const float* __restrict__ d_image,
                                             float* __restrict__ dV, float* __restrict__ camacc, const MixArgs& mx,
                                             int mbase, int* stk) {
    int lane = threadIdx.x;
    int* my = stk + lane;
    int m = mbase + lane;
    CamAcc ca = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    typename std::conditional<CNT, Work, NoWork>::type wk;
    double total = cdf[s.E];
    bool have = false;
    int key = -1;
    float gv[6] = {0, 0, 0, 0, 0, 0};
    if (m < a.M && (!a.mask || a.mask[m]) && total > 0.0) {
        Rng rp{(uint32_t)m, a.view, kTagPedge, a.k0, a.k1};
        float4 b0 = rp.block(0);
        PrimGeom G = prim_geom<MIX>(s, k, a, pe, cdf, mx, m, b0);
        if (G.live) {
            const float* dI = d_image + G.pix;
            // loss gradient times the jump of the pixel function across the edge
            float jump = 0.0f;
            bool jumps;
            if (AOV) {
                jump = aov_jump(s, a.aov, k.c, G.du, G.dl, k.nearc, dI, a.Ww * (k.y1 - k.y0), my, BS, wk);
                jumps = jump != 0.0f;
            } else {
                float fu, fl;
                radiance_pair(s, rp, 0, k.c, G.du, G.dl, k.nearc, true, a.depth, my, BS, wk, fu, fl);
                jumps = fu != fl;
                if (jumps) jump = dI[0] * (fu - fl);
            }
#ifdef DIFFRT_DEVICE_PRINTF
            if (m == a.debug_unit)
                printf("punit %d edge %d x %.9g y %.9g A %.9g %.9g B %.9g %.9g jump %.9g total %.9g\n", m, G.ei, G.x,
                       G.y, G.Ax, G.Ay, G.Bx, G.By, jump, total);
#endif
            if (jumps) {
                prim_contrib(k, a, G, jump, gv, ca);
                have = true;
                key = G.ei;
                wk.atomics(6);
                if (MIX && mx.estats) {
                    float c2 = 0.0f;
#pragma unroll
                    for (int i = 0; i < 6; ++i) c2 += gv[i] * gv[i];
                    atomicAdd(&mx.estats[G.ei], (float)G.p_edge * c2);
                }
            }
        }
    }
    scatter_grouped(have, key, gv, 4, [&](int ek, int i) {
        int4 e = s.edges[ek];
        return &dV[3 * (i < 3 ? e.x : e.y) + (i % 3)];
    });
    flush_work(wk, a.counters);
    flush_cam(ca, camacc);
}

// Split primary pass (the production path), 1 of 2: every unit's edge sample
// and the first hits of its two side rays (one traversal for both); samples
// whose sides hit the same triangle contribute nothing and stop here, the
// others are appended to a compact queue (one atomic per wave).
template <int STK, bool MIX>
__global__ __launch_bounds__(BS) void k_prim_sample(SceneView s, Cam k, RenderArgs a, const PEdge* __restrict__ pe,
                                                    const double* __restrict__ cdf, int3* __restrict__ q,
                                                    int* __restrict__ count, MixArgs mx) {
    __shared__ int stk[STK * BS];
    int lane = threadIdx.x;
    int* my = stk + lane;
    int m = blockIdx.x * BS + lane;
    NoWork wk;
    bool push = false;
    Hit hu, hl;
    if (m < a.M && (!a.mask || a.mask[m]) && cdf[s.E] > 0.0) {
        Rng rp{(uint32_t)m, a.view, kTagPedge, a.k0, a.k1};
        float4 b0 = rp.block(0);
        PrimGeom G = prim_geom<MIX>(s, k, a, pe, cdf, mx, m, b0);
        if (G.live) {
            trace_closest2(s, k.c, G.du, G.dl, k.nearc, 3.0e38f, my, BS, wk, hu, hl);
            push = hu.tri != hl.tri;
        }
    }
    unsigned long long bal = __ballot(push);
    if (bal == 0ull) return;
    int leader = __ffsll(bal) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(count, __popcll(bal));
    base = __shfl(base, leader, BS);
    if (push) q[base + __popcll(bal & ((1ull << lane) - 1ull))] = make_int3(m, hu.tri, hl.tri);
}

// Split primary pass, 2 of 2: the queued samples, densely: both sides'
// camera paths from their first hits (same random numbers), the jump, and
// the endpoint and camera gradients (lanes drawing the same edge summed in
// the wave before the atomics). MIX: the learned-proposal mixture's edge
// choice and, when asked, the per-edge harvest statistic. Five waves per SIMD
// (at most 96 VGPRs, some spilled) measured faster than four.
template <int STK, bool MIX>
__global__ __launch_bounds__(BS, 5) void k_prim_paths(SceneView s, Cam k, RenderArgs a, const PEdge* __restrict__ pe,
                                                   const double* __restrict__ cdf, const int3* __restrict__ q,
                                                   const int* __restrict__ count, const float* __restrict__ d_image,
                                                   float* __restrict__ dV, float* __restrict__ camacc, MixArgs mx) {
    __shared__ int stk[STK * BS];
    int lane = threadIdx.x;
    int* my = stk + lane;
    NoWork wk;
    CamAcc ca = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    int sh = blockIdx.x & (a.gshards - 1);
    dV += sh * a.gstride;
    camacc += 12 * sh;
    int n = *count;
    for (int base = blockIdx.x * BS; base < n; base += gridDim.x * BS) {
        bool have = false;
        int key = -1;
        float gv[6] = {0, 0, 0, 0, 0, 0};
        if (base + lane < n) {
            int3 Q = q[base + lane];
            int m = Q.x;
            Rng rp{(uint32_t)m, a.view, kTagPedge, a.k0, a.k1};
            float4 b0 = rp.block(0);
            v3 du, dl;
            {
                // only the two ray directions stay live across the paths; the
                // rest of the sample's geometry is recomputed afterwards
                PrimGeom G = prim_geom<MIX>(s, k, a, pe, cdf, mx, m, b0);
                du = G.du;
                dl = G.dl;
            }
            Hit hu{Q.y, 0.0f, 0.0f, 0.0f}, hl{Q.z, 0.0f, 0.0f, 0.0f};
            float fu = radiance_hit(s, rp, 0, k.c, du, hu, true, a.depth, my, BS, wk);
            float fl = radiance_hit(s, rp, 0, k.c, dl, hl, true, a.depth, my, BS, wk);
            if (fu != fl) {
                PrimGeom G = prim_geom<MIX>(s, k, a, pe, cdf, mx, m, b0);
                float jump = d_image[G.pix] * (fu - fl);
                prim_contrib(k, a, G, jump, gv, ca);
                have = true;
                key = G.ei;
                if (MIX && mx.estats) {
                    float c2 = 0.0f;
#pragma unroll
                    for (int i = 0; i < 6; ++i) c2 += gv[i] * gv[i];
                    atomicAdd(&mx.estats[G.ei], (float)G.p_edge * c2);
                }
            }
        }
        scatter_grouped(have, key, gv, 4, [&](int ek, int i) {
            int4 e = s.edges[ek];
            return &dV[3 * (i < 3 ? e.x : e.y) + (i % 3)];
        });
    }
    flush_cam(ca, camacc);
}

// Five waves per SIMD (at most 96 VGPRs, a few spilled): measured faster
// than four for this kernel, unlike for the path backward kernels.
template <int STK, bool CNT, bool MIX, bool AOV = false>
__global__ __launch_bounds__(BS, 5) void k_primary(SceneView s, Cam k, RenderArgs a, const PEdge* __restrict__ pe,
                                                const double* __restrict__ cdf, const float* __restrict__ d_image,
                                                float* __restrict__ dV, float* __restrict__ camacc, MixArgs mx) {
    __shared__ int stk[STK * BS];
    int sh = blockIdx.x & (a.gshards - 1);
    primary_body<STK, CNT, MIX, AOV>(s, k, a, pe, cdf, d_image, dV + sh * a.gstride, camacc + 12 * sh, mx, blockIdx.x * BS, stk);
}

// ---------------------------------------------------------------------------
// edge hierarchy descent (Edge selection): one uniform per level, explicit pdf
// ---------------------------------------------------------------------------
__device__ inline bool vsphere_prune(const ETChild& c, v3 pc) {
    v3 sc = pc * 0.5f;
    float r2 = dot(pc, pc) * 0.25f;
    const float sv[3] = {sc.x, sc.y, sc.z};
    bool out[2], in[2];
    for (int f = 0; f < 2; ++f) {
        const float* lo = f == 0 ? c.hlo0 : c.hlo1;
        const float* hi = f == 0 ? c.hhi0 : c.hhi1;
        float d2 = 0.0f, far2 = 0.0f;
        for (int k = 0; k < 3; ++k) {
            // distance of the centre to the box along k (0 inside) and to its far face
            float a = lo[k] - sv[k], b = sv[k] - hi[k];
            float d = fmaxf(fmaxf(a, b), 0.0f);
            d2 += d * d;
            float fa = fmaxf(fabsf(a), fabsf(b));
            far2 += fa * fa;
        }
        out[f] = d2 > r2 * (1.0f + kVsphereMargin);
        in[f] = far2 < r2 * (1.0f - kVsphereMargin);
    }
    return (out[0] && out[1]) || (in[0] && in[1]);
}

// Walter et al.'s bound on the cosine between the normal n and the direction
// from p to any point of the box [lo, hi], in the frame (t1, t2, n): the box's
// extent along each frame axis is its centre's projection plus or minus the
// half-extents projected by the axis' absolute components.
__device__ inline float cos_bound(const float lo[3], const float hi[3], v3 p, v3 n, v3 t1, v3 t2, float hz) {
    v3 c = {(lo[0] + hi[0]) * 0.5f - p.x, (lo[1] + hi[1]) * 0.5f - p.y, (lo[2] + hi[2]) * 0.5f - p.z};
    v3 h = {(hi[0] - lo[0]) * 0.5f, (hi[1] - lo[1]) * 0.5f, (hi[2] - lo[2]) * 0.5f};
    float cx = dot(t1, c), ex = fabsf(t1.x) * h.x + fabsf(t1.y) * h.y + fabsf(t1.z) * h.z;
    float cy = dot(t2, c), ey = fabsf(t2.x) * h.x + fabsf(t2.y) * h.y + fabsf(t2.z) * h.z;
    float zh = dot(n, c) + fabsf(n.x) * h.x + fabsf(n.y) * h.y + fabsf(n.z) * h.z;
    float xl = cx - ex, xh = cx + ex, yl = cy - ey, yh = cy + ey;
    // distance of [l, h] from 0: l when above it, -h when below, 0 when it spans 0
    float dx = fmaxf(fmaxf(xl, -xh), 0.0f);
    float dy = fmaxf(fmaxf(yl, -yh), 0.0f);
    float dxy2 = dx * dx + dy * dy;
    if (zh <= hz) return 0.0f;
    if (dxy2 == 0.0f) return 1.0f;
    return zh * rsqrtf(dxy2 + zh * zh);
}

struct TreeCtx {
    const SceneView* s;
    v3 p, n, cam;
    int tri;
    float hz, pad;
    v3 t1, t2;     // tangent frame of n (Duff et al.)
};

__device__ inline TreeCtx tree_ctx(const SceneView* s, v3 p, v3 n, v3 cam, int tri, float hz, float pad) {
    TreeCtx q{s, p, n, cam, tri, hz, pad, {0, 0, 0}, {0, 0, 0}};
    onb(n, q.t1, q.t2);
    return q;
}

// Whether the shading point lies in the parent's box grown by the pad: then
// both children get importance one. Evaluated once per node.
__device__ inline bool in_parent(const TreeCtx& q, const float* plo, const float* phi) {
    const float pv[3] = {q.p.x, q.p.y, q.p.z};
    bool in = true;
    for (int k = 0; k < 3; ++k)
        if (pv[k] < plo[k] - q.pad || pv[k] > phi[k] + q.pad) in = false;
    return in;
}

__device__ inline float importance(const TreeCtx& q, const ETChild& c, int ref, int h2, bool inpar) {
    if (ref == 0) return 0.0f;
    if (ref < 0) {
        // both faces of the leaf's edge in one 8-byte load
        const int2 f = *reinterpret_cast<const int2*>(&q.s->edges[~ref].z);
        if ((f.x == q.tri) | (f.y == q.tri)) return 0.0f;
    }
    if (h2 && vsphere_prune(c, q.p - q.cam)) return 0.0f;
    float b = cos_bound(c.lo, c.hi, q.p, q.n, q.t1, q.t2, q.hz);
    if (b <= 0.0f) return 0.0f;
    if (inpar) return 1.0f;
    v3 ctr = {(c.lo[0] + c.hi[0]) * 0.5f, (c.lo[1] + c.hi[1]) * 0.5f, (c.lo[2] + c.hi[2]) * 0.5f};
    v3 dc = ctr - q.p;
    return c.len * b * rsqrtf(dot(dc, dc));
}

// A whole node in registers: its eleven 16-byte words are loaded together,
// so a level waits for memory once instead of once per field it reads.
__device__ inline ETNode load_node(const ETNode* __restrict__ nodes, int i) {
    const float4* p = reinterpret_cast<const float4*>(nodes + i);
    float4 w[11];
#pragma unroll
    for (int k = 0; k < 11; ++k) w[k] = p[k];
    ETNode n;
    __builtin_memcpy(&n, w, sizeof(ETNode));
    return n;
}

template <class W>
__device__ inline int tree_sample(const TreeView& tv, const TreeCtx& q, const Rng& rk, float u_root, float& pdf, W& wk,
                                  bool dbg = false) {
    const ETNode* nodes = tv.nodes;
    int node = 0;
    float plo[3], phi[3];
    {
        const ETNode& r = nodes[0];
        for (int k = 0; k < 3; ++k) { plo[k] = 3e38f; phi[k] = -3e38f; }
        for (int c = 0; c < 2; ++c)
            if (r.child[c] != 0)
                for (int k = 0; k < 3; ++k) { plo[k] = fminf(plo[k], r.ch[c].lo[k]); phi[k] = fmaxf(phi[k], r.ch[c].hi[k]); }
    }
    pdf = 1.0f;
    int level = -1;
    float4 ub = make_float4(0, 0, 0, 0);
    while (true) {
        const ETNode N = load_node(nodes, node);
        wk.tree();
        int h2a = node == 0 ? 0 : N.h2, h2b = node == 0 ? 1 : N.h2;
        bool inpar = in_parent(q, plo, phi);
        float w0 = importance(q, N.ch[0], N.child[0], h2a, inpar);
        float w1 = importance(q, N.ch[1], N.child[1], h2b, inpar);
        float tot = w0 + w1;
        if (!(tot > 0.0f)) return -1;
        float u;
        if (level < 0) u = u_root;
        else {
            if (level >= kMaxLevels) { atomicOr(q.s->err, kErrTreeDepth); return -1; }
            if ((level & 3) == 0) ub = rk.block(1 + (level >> 2));
            int c = level & 3;
            u = c == 0 ? ub.x : (c == 1 ? ub.y : (c == 2 ? ub.z : ub.w));
        }
        float p0 = w0 / tot;
        int side = u < p0 ? 0 : 1;
        pdf *= side == 0 ? p0 : w1 / tot;
#ifdef DIFFRT_DEVICE_PRINTF
        if (dbg) printf("  level %d node %d w0 %.9g w1 %.9g u %.9g side %d\n", level, node, w0, w1, u, side);
#endif
        int ref = N.child[side];
        if (ref < 0) return ~ref;
        for (int k = 0; k < 3; ++k) { plo[k] = N.ch[side].lo[k]; phi[k] = N.ch[side].hi[k]; }
        node = ref;
        ++level;
    }
}

// Probability that one descent ends at edge e: the product of the branch
// probabilities along its leaf-to-root path (root choice included).
template <class W>
__device__ inline float tree_pdf_edge(const TreeView& tv, const TreeCtx& q, int e, W& wk) {
    int code = tv.eleaf[e];
    if (code < 0) return 0.0f;
    const ETNode* nodes = tv.nodes;
    int node = code >> 1, side = code & 1;
    float pdf = 1.0f;
    for (int guard = 0; guard <= kMaxLevels + 1; ++guard) {
        const ETNode N = load_node(nodes, node);
        wk.tree();
        int pcode = node == 0 ? -1 : tv.enpar[node];
        float plo[3], phi[3];
        if (node == 0) {
            for (int k = 0; k < 3; ++k) { plo[k] = 3e38f; phi[k] = -3e38f; }
            for (int c = 0; c < 2; ++c)
                if (N.child[c] != 0)
                    for (int k = 0; k < 3; ++k) { plo[k] = fminf(plo[k], N.ch[c].lo[k]); phi[k] = fmaxf(phi[k], N.ch[c].hi[k]); }
        } else {
            const ETChild& pc = nodes[pcode >> 1].ch[pcode & 1];
            for (int k = 0; k < 3; ++k) { plo[k] = pc.lo[k]; phi[k] = pc.hi[k]; }
        }
        int h2a = node == 0 ? 0 : N.h2, h2b = node == 0 ? 1 : N.h2;
        bool inpar = in_parent(q, plo, phi);
        float w0 = importance(q, N.ch[0], N.child[0], h2a, inpar);
        float w1 = importance(q, N.ch[1], N.child[1], h2b, inpar);
        float tot = w0 + w1;
        if (!(tot > 0.0f)) return 0.0f;
        pdf *= (side == 0 ? w0 : w1) / tot;
        if (node == 0) return pdf;
        node = pcode >> 1;
        side = pcode & 1;
    }
    atomicOr(q.s->err, kErrTreeDepth);
    return 0.0f;
}

// Stratified multi-sample descent with weighted reservoir selection (Edge
// selection). M samples enter at the root; the n samples that reach a node are
// divided between its children, the first receiving floor(n p0 + xi) (p0 its
// share of the two importances, xi uniform), so a leaf e receives M pdf_e in
// expectation, pdf_e being the probability that one descent ends there. The
// leaves reached are visited depth first, first child first; a leaf holding
// n_e samples has weight n_e imp_e / pdf_e (imp_e: its importance at its
// parent) and one is kept by weighted reservoir sampling. Returns the kept
// edge (or -1) and, in `pdf`, M imp_z / W (W: total weight), which takes the
// place of the descent pdf in the sample's weight: resampled importance
// sampling, unbiased since sum_e E[n_e] f(e) / (M pdf_e) = sum_e f(e).
// Uniforms from `rs` in visiting order: one per split, one per leaf reached.
// `stk`: this lane's first LDS word, kSelectMax entries of 4 words, strided
// by `stride`: the deferred second children (their sample groups are
// disjoint and non-empty, so at most M - 1 are pending).
template <class W>
__device__ inline int tree_select(const TreeView& tv, const TreeCtx& q, const Rng& rs, int M, float& pdf, int* stk,
                                  int stride, W& wk) {
    const ETNode* nodes = tv.nodes;
    uint32_t c = 0;
    float4 ub = make_float4(0, 0, 0, 0);
    auto next_u = [&]() {
        if ((c & 3) == 0) ub = rs.block(c >> 2);
        int k = c & 3;
        ++c;
        return k == 0 ? ub.x : (k == 1 ? ub.y : (k == 2 ? ub.z : ub.w));
    };
    float Wt = 0.0f, impz = 0.0f;
    int z = -1;
    auto candidate = [&](int edge, int n, float pd, float imp) {
        float om = (float)n * imp / pd;
        Wt += om;
        float r = om / Wt;
        if (next_u() < r) {
            z = edge;
            impz = imp;
        }
    };
    int sp = 0;
    int node = 0, n = M;
    float pd = 1.0f;
    for (int guard = 0; guard <= M * (kMaxLevels + 1); ++guard) {
        bool descend = false;
        {
            const ETNode N = load_node(nodes, node);
            wk.tree();
            // the node's box: the union of its children's (of the non-empty
            // ones at the virtual root), as its parent stores it
            float plo[3], phi[3];
            for (int k = 0; k < 3; ++k) { plo[k] = 3e38f; phi[k] = -3e38f; }
            for (int ci = 0; ci < 2; ++ci)
                if (node != 0 || N.child[ci] != 0)
                    for (int k = 0; k < 3; ++k) {
                        plo[k] = fminf(plo[k], N.ch[ci].lo[k]);
                        phi[k] = fmaxf(phi[k], N.ch[ci].hi[k]);
                    }
            int h2a = node == 0 ? 0 : N.h2, h2b = node == 0 ? 1 : N.h2;
            bool inpar = in_parent(q, plo, phi);
            float w0 = importance(q, N.ch[0], N.child[0], h2a, inpar);
            float w1 = importance(q, N.ch[1], N.child[1], h2b, inpar);
            float tot = w0 + w1;
            if (tot > 0.0f) {
                float p0 = w0 / tot;
                int n0 = min(max((int)floorf((float)n * p0 + next_u()), 0), n);
                int n1 = n - n0;
                if (n1 > 0) {
                    // the second child waits until the first one's subtree is done
                    int* e = stk + 4 * sp * stride;
                    e[0] = N.child[1];
                    e[stride] = n1;
                    e[2 * stride] = __float_as_int(pd * (w1 / tot));
                    e[3 * stride] = __float_as_int(w1);
                    ++sp;
                }
                if (n0 > 0) {
                    int ref = N.child[0];
                    if (ref < 0) {
                        candidate(~ref, n0, pd * p0, w0);
                    } else {
                        node = ref;
                        n = n0;
                        pd = pd * p0;
                        descend = true;
                    }
                }
            }
        }
        if (descend) continue;
        // next deferred child; leaves among them are candidates at once
        bool found = false;
        while (sp > 0) {
            --sp;
            const int* e = stk + 4 * sp * stride;
            int ref = e[0], ne = e[stride];
            float pe = __int_as_float(e[2 * stride]), ie = __int_as_float(e[3 * stride]);
            if (ref < 0) {
                candidate(~ref, ne, pe, ie);
            } else {
                node = ref;
                n = ne;
                pd = pe;
                found = true;
                break;
            }
        }
        if (!found) {
            if (z >= 0) pdf = (float)M * impz / Wt;
            return z;
        }
    }
    atomicOr(q.s->err, kErrTreeDepth);
    return -1;
}

// ---------------------------------------------------------------------------
// Point on a secondary edge in proportion to the clamped cosine (Importance
// sampling on an edge, Lambertian lobe). Seen from p the edge is a great-
// circle arc of directions w(phi) = cos(phi) a + sin(phi) b', phi in [0, Phi];
// along it n . w = R cos(phi - phi0), whose positive part integrates to
// R (sin(phi - phi0) - sin(lo - phi0)) and is inverted by an arcsine. The
// density in the edge parameter is p(t) = max(n . w^, 0) |e x w^| / (T |w|),
// T the integral of the positive part over the whole arc. Returns false when
// there is no sample (degenerate arc, no positive part).
// ---------------------------------------------------------------------------
constexpr float kArcMin = 1e-6f;

__device__ inline bool cosine_edge_t(v3 p, v3 n, v3 pa, v3 pb, float u, float& t, float& T) {
    v3 a = nrm(pa - p), b = nrm(pb - p);
    float cab = dot(a, b);
    v3 bo = b - a * cab;
    float sb = len(bo);
    if (!(sb > kArcMin)) return false;
    bo = bo * (1.0f / sb);
    float Phi = atan2f(sb, cab);
    float A = dot(n, a), B = dot(n, bo);
    float phi0 = atan2f(B, A);
    if (phi0 < -0.5f * kPi) phi0 += 2.0f * kPi;
    float lo = fmaxf(0.0f, phi0 - 0.5f * kPi), hi = fminf(Phi, phi0 + 0.5f * kPi);
    if (!(hi > lo)) return false;
    float slo = sinf(lo - phi0), shi = sinf(hi - phi0);
    T = sqrtf(A * A + B * B) * (shi - slo);
    float sv = slo + u * (shi - slo);
    float phi = phi0 + asinf(fmaxf(-1.0f, fminf(1.0f, sv)));
    v3 wd = a * cosf(phi) + bo * sinf(phi);
    v3 e = pb - pa;
    v3 ew = cross(e, wd);
    t = -dot(cross(pa - p, wd), ew) / dot(ew, ew);
    t = fmaxf(0.0f, fminf(1.0f, t));
    return true;
}

__device__ inline float cosine_edge_pdf(v3 p, v3 n, v3 pa, v3 pb, float t, float T) {
    v3 e = pb - pa;
    v3 w = pa + e * t - p;
    float wl = len(w);
    v3 wh = w * (1.0f / wl);
    float c = dot(n, wh);
    if (!(c > 0.0f) || !(T > 0.0f)) return 0.0f;
    return c * len(cross(e, wh)) / (T * wl);
}

// ---------------------------------------------------------------------------
// Next event estimation for edges (Ch. 5, Next event estimation for edges):
// a second strategy for the secondary edge sample. A light point y is drawn
// as next-event estimation draws it; every edge is widened into a strip of
// width w that faces the shading point x, { pa + t (pb - pa) + s v :
// t in [0, 1], |s| <= w/2 }, v the unit vector orthogonal to the edge and to
// pa - x; among the strips the segment x -> y crosses, one is chosen in
// proportion to the edge's importance (an exponential race: edge e's key
// -log(1 - u_e) / imp_e with u_e from its own Philox block, the smallest key
// wins, so the choice does not depend on the order of the BVH walk
// that finds the crossings), and the crossing's parameter t is the point on
// the edge. Its density in (t, s): the ray from x through the strip point b
// meets the lights at y = x + mu (b - x), mu > 1, each drawn with area
// density 1 / A_lights; with the Jacobian from light area to strip area and
// the choice among the strips crossed by x -> y,
//   p_N = |pb - pa| / A_lights * sum_y mu^2 |cos_b| / |cos_y| * imp_e / sum_crossed imp.
// The strategy is mixed with the hierarchy by one-sample multiple importance
// sampling (probability alpha for the strips, a uniform s across the strip
// for hierarchy draws): the sample's density in (e, t) is
// alpha w p_N + (1 - alpha) p_H. Importance: that of a hierarchy leaf
// without the parent-box rule, zero for the shading triangle's own edges,
// emitter edges and edges that are no discontinuity as seen from x. Light
// points behind x's tangent plane or on a one-sided emitter's back are not
// used.
// ---------------------------------------------------------------------------
struct Strip {
    v3 pa, ah, v, nb;    // edge start, unit edge direction, unit width direction, unit normal
    float L;             // edge length
    bool ok;
};

__device__ inline Strip strip_of(const SceneView& s, int4 e, v3 x) {
    Strip B;
    B.pa = ld3(s.P, e.x);
    v3 a = ld3(s.P, e.y) - B.pa;
    B.L = len(a);
    B.ok = false;
    if (!(B.L > 0.0f)) return B;
    B.ah = a * (1.0f / B.L);
    v3 c = cross(B.ah, B.pa - x);
    float cl = len(c);
    if (!(cl > 0.0f)) return B;
    B.v = c * (1.0f / cl);
    B.nb = cross(B.ah, B.v);
    B.ok = true;
    return B;
}

// Crossing of the segment x -> x + d (both ends excluded) with the strip.
__device__ inline bool strip_cross(const Strip& B, v3 x, v3 d, float w, float& t, float& sv) {
    if (!B.ok) return false;
    float den = dot(d, B.nb);
    if (den == 0.0f) return false;
    float lam = dot(B.pa - x, B.nb) / den;
    v3 r = x + d * lam - B.pa;
    t = dot(r, B.ah) / B.L;
    sv = dot(r, B.v);
    return t >= 0.0f && t <= 1.0f && fabsf(sv) <= 0.5f * w && lam > 0.0f && lam < 1.0f;
}

__device__ inline float strip_importance(const SceneView& s, int ei, const TreeCtx& q) {
    if (s.ekind[ei] == 0) return 0.0f;
    int4 e = s.edges[ei];
    if (e.z == q.tri || e.w == q.tri) return 0.0f;
    if (s.emi[e.z] > 0.0f || (e.w >= 0 && s.emi[e.w] > 0.0f)) return 0.0f;
    if (s.ekind[ei] == 2 && !silhouette_from(s, e, q.p)) return 0.0f;
    v3 a = ld3(s.P, e.x), b = ld3(s.P, e.y);
    float lo[3] = {fminf(a.x, b.x), fminf(a.y, b.y), fminf(a.z, b.z)};
    float hi[3] = {fmaxf(a.x, b.x), fmaxf(a.y, b.y), fmaxf(a.z, b.z)};
    float cb = cos_bound(lo, hi, q.p, q.n, q.t1, q.t2, q.hz);
    if (cb <= 0.0f) return 0.0f;
    v3 dc = (a + b) * 0.5f - q.p;
    return len(b - a) * cb * rsqrtf(dot(dc, dc));
}

// Segment x -> x + d (parameter in [0, 1]) against a box grown by pad (inv:
// the reciprocals of d's components). A zero component of d on a grown face
// gives NaN, which fminf / fmaxf drop; such a segment lies outside the
// ungrown box by the pad's margin beyond the strip, so the test cannot lose
// a crossing either way.
__device__ inline bool seg_box(v3 x, v3 inv, float pad, float lx, float ly, float lz, float hx, float hy, float hz) {
    float a0 = (lx - pad - x.x) * inv.x, b0 = (hx + pad - x.x) * inv.x;
    float a1 = (ly - pad - x.y) * inv.y, b1 = (hy + pad - x.y) * inv.y;
    float a2 = (lz - pad - x.z) * inv.z, b2 = (hz + pad - x.z) * inv.z;
    float t0 = fmaxf(fmaxf(fminf(a0, b0), fminf(a1, b1)), fmaxf(fminf(a2, b2), 0.0f));
    float t1 = fminf(fminf(fmaxf(a0, b0), fmaxf(a1, b1)), fminf(fmaxf(a2, b2), 1.0f));
    return t0 <= t1;
}

// Visits every edge of the triangles whose BVH boxes, grown by pad, meet the
// segment x -> x + d (a strip lies within half its width of its edge, and an
// edge within its faces' boxes); each edge once, through its first face.
// stk: this lane's LDS stack (entries `stride` words apart, s.stk_cap of
// them), as the ray traversals use it.
template <class F, class W>
__device__ inline void strip_walk(const SceneView& s, v3 x, v3 d, float pad, int* stk, int stride, W& wk, F&& visit) {
    auto leaf = [&](int tr) {
        int4 o = s.towned[tr];
        if (o.x >= 0) visit(o.x);
        if (o.y >= 0) visit(o.y);
        if (o.z >= 0) visit(o.z);
    };
    if (s.T == 1) {
        leaf(0);
        return;
    }
    v3 inv = {1.0f / d.x, 1.0f / d.y, 1.0f / d.z};
    int sp = 0, node = 0;
    for (int guard = 2 * s.T + 8; guard > 0; --guard) {
        wk.tree();
        BvhNode n = load_bvh(s.bvh, node);
        bool hl = seg_box(x, inv, pad, n.a.x, n.a.y, n.a.z, n.a.w, n.b.x, n.b.y);
        bool hr = seg_box(x, inv, pad, n.b.z, n.b.w, n.c.x, n.c.y, n.c.z, n.c.w);
        int l = n.d.x, r = n.d.y;
        if (hl && l < 0) {
            leaf(~l);
            hl = false;
        }
        if (hr && r < 0) {
            leaf(~r);
            hr = false;
        }
        if (hl && hr) {
            if (sp < s.stk_cap) stk[(sp++) * stride] = r;
            else atomicOr(s.err, kErrStack);
            node = l;
        } else if (hl) {
            node = l;
        } else if (hr) {
            node = r;
        } else {
            if (sp == 0) return;
            node = stk[(--sp) * stride];
        }
    }
    atomicOr(s.err, kErrStack);
}

// Sum of the importances of the strips crossed by x -> y, edge `skip` left out.
template <class W>
__device__ inline float strip_crossed_sum(const SceneView& s, const TreeCtx& q, float w, v3 y, int skip, int* stk,
                                          int stride, W& wk) {
    float sum = 0.0f;
    v3 d = y - q.p;
    strip_walk(s, q.p, d, kStripPad * w + kWalkPad * s.diag, stk, stride, wk, [&](int ei) {
        if (ei == skip) return;
        float t, sv;
        if (!strip_cross(strip_of(s, s.edges[ei], q.p), q.p, d, w, t, sv)) return;
        sum += strip_importance(s, ei, q);
    });
    return sum;
}

// Whether the direction dh towards a point of light triangle g is used: above
// the tangent plane and, for one-sided emitters, on the emitting side.
__device__ inline bool strip_light_usable(const SceneView& s, const TreeCtx& q, v3 dh, const TriGeom& g) {
    if (!(dot(q.n, dh) > 0.0f)) return false;
    if (s.two_sided) return true;
    return -dot(nrm(cross(g.e1, g.e2)), dh) > 0.0f;
}

// Density of the strip strategy at (edge ei, t, sv), in dt ds. known_lt /
// known_sum: the light triangle of the draw's own light point (-1: none) and
// the crossed-importance sum along the segment to it. The ray through the
// strip point meets that triangle by construction, at the light point up to
// rounding, so its hit is taken without the inside and side tests (a rounding
// miss would drop the strategy's own density from the sample's weight) and
// the sum is not walked again.
template <class W>
__device__ inline float strip_pdf(const SceneView& s, const TreeCtx& q, float w, int ei, float t, float sv, int known_lt,
                                  float known_sum, int* stk, int stride, W& wk) {
    float imp = strip_importance(s, ei, q);
    if (!(imp > 0.0f) || s.L == 0) return 0.0f;
    Strip B = strip_of(s, s.edges[ei], q.p);
    if (!B.ok) return 0.0f;
    v3 b = B.pa + B.ah * (B.L * t) + B.v * sv;
    v3 d = b - q.p;
    v3 dh = nrm(d);
    float cb = fabsf(dot(dh, B.nb));
    float acc = 0.0f;
    for (int i = 0; i < s.L; ++i) {
        int lt = s.lights[i];
        TriGeom g = tri_geom(s, lt);
        v3 nl = nrm(cross(g.e1, g.e2));
        float mu;
        if (lt == known_lt) {
            float dn = dot(d, nl);
            if (dn == 0.0f) continue;
            mu = dot(g.p0 - q.p, nl) / dn;
        } else {
            // Moller-Trumbore on the ray x + mu d, both faces, mu > 1
            v3 pv = cross(d, g.e2);
            float det = dot(g.e1, pv);
            if (det == 0.0f) continue;
            float inv = 1.0f / det;
            v3 tq = q.p - g.p0;
            float u = dot(tq, pv) * inv;
            v3 qv = cross(tq, g.e1);
            float vv = dot(d, qv) * inv;
            mu = dot(g.e2, qv) * inv;
            if (!(u >= 0.0f && vv >= 0.0f && u + vv <= 1.0f && mu > 1.0f)) continue;
            if (!strip_light_usable(s, q, dh, g)) continue;
        }
        float cy = fabsf(dot(nl, dh));
        if (!(cy > 0.0f)) continue;
        float sum = lt == known_lt ? known_sum : imp + strip_crossed_sum(s, q, w, q.p + d * mu, ei, stk, stride, wk);
        acc += mu * mu * cb / cy * imp / sum;
    }
    return acc * B.L / s.atot[0];
}

// One draw of the strip strategy: light point from c0.y (light), c0.z, c0.w
// (point), the race's uniforms from rn's blocks 2 + edge id. Returns the
// edge (or -1), the crossing's strip coordinates, the light triangle and the
// sum of the crossed strips' importances.
template <class W>
__device__ inline int strip_sample(const SceneView& s, const TreeCtx& q, float w, float4 c0, const Rng& rn, float& t,
                                   float& sv, int& lt, float& sum, int* stk, int stride, W& wk) {
    if (s.L == 0) return -1;
    lt = s.lights[pick_cdf(s.lcdf, s.L, c0.y)];
    TriGeom g = tri_geom(s, lt);
    float su = sqrtf(c0.z);
    v3 y = g.p0 + g.e1 * (su * (1.0f - c0.w)) + g.e2 * (su * c0.w);
    v3 d = y - q.p;
    if (!strip_light_usable(s, q, nrm(d), g)) return -1;
    int best = -1;
    float kbest = 3e38f;
    sum = 0.0f;
    strip_walk(s, q.p, d, kStripPad * w + kWalkPad * s.diag, stk, stride, wk, [&](int ei) {
        float te, se;
        if (!strip_cross(strip_of(s, s.edges[ei], q.p), q.p, d, w, te, se)) return;
        float imp = strip_importance(s, ei, q);
        if (!(imp > 0.0f)) return;
        sum += imp;
        float key = -logf(1.0f - rn.block(2u + (uint32_t)ei).x) / imp;
        if (key < kbest) {
            kbest = key;
            best = ei;
            t = te;
            sv = se;
        }
    });
    return best;
}

// The mixture draw: with probability a.nee the strips, else the hierarchy
// (root uniform b0.x, t = b0.y, s from rn's block 1). Returns the edge (or
// -1), its parameter t and the density in (e, t).
template <class W>
__device__ inline int strip_mix_draw(const SceneView& s, const TreeView& tv, const TreeCtx& q, const RenderArgs& a,
                                     const Rng& rk, float4 b0, const Rng& rn, float& t, float& pdf, int* stk, int stride,
                                     W& wk) {
    float4 c0 = rn.block(0);
    float w = a.nee_w;
    int ei, lt = -1;
    float sv, ph, sum = 0.0f;
    if (c0.x < a.nee) {
        ei = strip_sample(s, q, w, c0, rn, t, sv, lt, sum, stk, stride, wk);
        if (ei < 0) return -1;
        ph = tree_pdf_edge(tv, q, ei, wk);
    } else {
        ei = tree_sample(tv, q, rk, b0.x, ph, wk);
        if (ei < 0) return -1;
        t = b0.y;
        sv = (rn.block(1).x - 0.5f) * w;
    }
    pdf = a.nee * w * strip_pdf(s, q, w, ei, t, sv, lt, sum, stk, stride, wk) + (1.0f - a.nee) * ph;
    return pdf > 0.0f ? ei : -1;
}

// ---------------------------------------------------------------------------
// backward over paths: secondary edges at every vertex + interior adjoint
// ---------------------------------------------------------------------------
// PH: 0 = all in one pass; 1 = rebuild the path, sample the secondary edges and
// queue their side-path queries; 2 = rebuild the path, read the side
// radiances of its queries and run the adjoint sweep.
// AOV (with MAXD = 1, PH = 0): gradient of the geometry-buffer channel a.aov;
// only the first hit, no NEE, no secondary term.
// NEE (with PH = 1): secondary edge samples from the strip strategy mixed with
// the hierarchy (next event estimation for edges); its walks use the lane's
// traversal stack, idle while an edge is drawn.
template <int MAXD, int STK, bool CNT, bool MIX, int PH = 0, bool AOV = false, bool NEE = false>
__device__ __forceinline__ void backward_body(const SceneView& s, const Cam& k, const RenderArgs& a, const TreeView& tv,
                                              const float* __restrict__ d_image, float* __restrict__ dV,
                                              float* __restrict__ dA, float* __restrict__ camacc, const MixArgs& mx,
                                              int mbase, int* stk, const SplitArgs& sp = SplitArgs{}) {
    int lane = threadIdx.x;
    int* my = stk + lane;
    int m = mbase + lane;
    CamAcc ca = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    typename std::conditional<CNT, Work, NoWork>::type wk;
    bool have0 = false;          // vertex-1 triangle gradients, scattered per wave group
    int key0 = -1;
    float g0[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (PH == 1 && m < a.M)
#pragma unroll
        for (int kk = 0; kk < MAXD; ++kk) sp.qidx[(size_t)kk * a.M + m] = -1;
    const int depth = AOV ? 1 : a.depth;
    if (m < a.M && (!a.mask || a.mask[m]) && depth >= 1 && a.ck_tri[m] >= 0) {
        int pix, px, py;
        uint32_t sid;
        unit_pixel(k, a, m, pix, px, py, sid);
        float W0 = PH == 1 ? 0.0f : d_image[pix] / (float)a.spp;
        Rng rc{sid, a.view, kTagCam, a.k0, a.k1};
        float4 j = rc.block(0);
        float sx = px + j.x, sy = py + j.y;
        float ndx = 2.0f * sx / k.W - 1.0f, ndy = 1.0f - 2.0f * sy / k.H;
        v3 d0 = k.f + k.r * (ndx * k.asp * k.th) + k.u * (ndy * k.th);
        uint8_t vis = a.ck_vis[m];
        // ---- rebuild the path's vertices
        // per vertex: the ray reaching vertex k starts at vertex k-1 (camera for
        // k = 0) along wc[k-1] (camera direction d0 for k = 0)
        int tri[MAXD];
        v3 xs[MAXD], ns[MAXD], wc[MAXD];
        float sg[MAXD], rho[MAXD], beta[MAXD], cc[MAXD];
        int nv = 0;
        {
            int t = a.ck_tri[m];
            v3 o = k.c, d = d0;
            v3 x = {a.ck_x[3 * (size_t)m], a.ck_x[3 * (size_t)m + 1], a.ck_x[3 * (size_t)m + 2]};
            float b = 1.0f;
#pragma unroll
            for (int kk = 0; kk < MAXD; ++kk) {
                if (kk >= depth) break;
                TriGeom g = tri_geom(s, t);
                float sgn = dot(d, cross(g.e1, g.e2)) < 0.0f ? 1.0f : -1.0f;
                v3 n = shading_normal(s, t, g, x) * sgn;
                float r = s.alb[t];
                if (r == 0.0f && !AOV) break;
                tri[kk] = t; xs[kk] = x; ns[kk] = n; sg[kk] = sgn; rho[kk] = r; beta[kk] = b;
                cc[kk] = 0.0f;
                wc[kk] = {0, 0, 0};
                nv = kk + 1;
                if (kk + 1 >= depth) break;
                float4 ub = rc.block(2 * kk + 2);
                v3 w = cosine_dir(n, ub.x, ub.y);
                float c = dot(n, w);
                if (c <= 0.0f) break;
                int t2;
                v3 x2;
                if (kk + 1 < 3) {
                    // vertices 1 and 2 were stored by the forward pass
                    t2 = a.ck_tri[(size_t)(kk + 1) * a.M + m];
                    if (t2 < 0) break;
                    const float* cx = a.ck_x + 3 * ((size_t)(kk + 1) * a.M + m);
                    x2 = {cx[0], cx[1], cx[2]};
                } else if (PH == 2) {
                    // the sampling pass traced this vertex: take its hit
                    size_t slot = (size_t)(kk - 1) * a.M + m;
                    t2 = sp.vtri[slot];
                    if (t2 < 0) break;
                    x2 = {sp.vx[3 * slot], sp.vx[3 * slot + 1], sp.vx[3 * slot + 2]};
                } else {
                    Hit h = trace_closest(s, x, w, s.tmin, 3.0e38f, my, BS, wk);
                    if (PH == 1) {
                        size_t slot = (size_t)(kk - 1) * a.M + m;
                        sp.vtri[slot] = h.tri;
                        if (h.tri >= 0) {
                            v3 xh = hit_point(tri_geom(s, h.tri), x, w);
                            sp.vx[3 * slot] = xh.x; sp.vx[3 * slot + 1] = xh.y; sp.vx[3 * slot + 2] = xh.z;
                        }
                    }
                    if (h.tri < 0) break;
                    t2 = h.tri;
                    x2 = hit_point(tri_geom(s, t2), x, w);
                }
                if (s.alb[t2] == 0.0f) break;     // the next vertex would end the path before contributing
                wc[kk] = w;
                cc[kk] = c;
                b *= r;
                o = x; d = w; t = t2; x = x2;
            }
        }
        v3 xbar[MAXD];
#pragma unroll
        for (int kk = 0; kk < MAXD; ++kk) xbar[kk] = {0, 0, 0};
        // ---- secondary boundary term: one edge sample per vertex
        if ((a.terms & DR_TERM_SECONDARY) && tv.valid && !AOV) {
            // adjoint pass: a vertex's edge-endpoint contributions (edge id, 6
            // numbers) are scattered at the end of its iteration, where lanes
            // of a converged wave that drew the same edge are summed first
            auto edge_dest = [&](int ek, int i) {
                int4 e = s.edges[ek];
                return &dV[3 * (i < 3 ? e.x : e.y) + (i % 3)];
            };
#pragma unroll
            for (int kk = 0; kk < MAXD; ++kk) {
                int bedge = -1;
                float bval[6] = {0, 0, 0, 0, 0, 0};
                do {
                    if (kk >= nv) break;
                    Rng rk{sid, a.view, kTagSedge + (uint32_t)(kk + 1), a.k0, a.k1};
                    float4 b0 = rk.block(0);
                    v3 p = xs[kk], n = ns[kk];
                    float pdf;
                    bool dbg = m == a.debug_unit;
                    int ei;
                    int qi = -1;
                    float te_draw = 0.0f;
                    if (PH == 2) {
                        qi = sp.qidx[(size_t)kk * a.M + m];
                        if (qi < 0) break;
                        ei = sp.q[qi].edge;
                        pdf = sp.q[qi].pdf;
                    } else if (NEE) {
                        TreeCtx q = tree_ctx(&s, p, n, tv.cam, tri[kk], kHorizon * s.diag, kInsidePad * s.diag);
                        Rng rn{sid, a.view, kTagEnee + (uint32_t)(kk + 1), a.k0, a.k1};
                        ei = strip_mix_draw(s, tv, q, a, rk, b0, rn, te_draw, pdf, my, BS, wk);
                    } else if (MIX && mx.sec) {
                        TreeCtx q = tree_ctx(&s, p, n, tv.cam, tri[kk], kHorizon * s.diag, kInsidePad * s.diag);
                        // proposal mixture: component from the third uniform of the
                        // block, proposal draw from the fourth
                        float pt;
                        if (b0.z < mx.mix) {
                            ei = pick_cdf_d(mx.qcdf, s.E, (double)b0.w);
                            pt = tree_pdf_edge(tv, q, ei, wk);
                        } else {
                            ei = tree_sample(tv, q, rk, b0.x, pt, wk, dbg);
                            if (ei < 0) break;
                        }
                        pdf = mx.mix * mx.q[ei] + (1.0f - mx.mix) * pt;
                        if (!(pdf > 0.0f) || s.ekind[ei] == 0) break;
                    } else {
                        TreeCtx q = tree_ctx(&s, p, n, tv.cam, tri[kk], kHorizon * s.diag, kInsidePad * s.diag);
                        ei = tree_sample(tv, q, rk, b0.x, pdf, wk, dbg);
                    }
                    if (ei < 0) break;
                    int4 e = s.edges[ei];
                    if (PH != 2) {
                        if (e.z == tri[kk] || e.w == tri[kk]) break;
                        if (s.ekind[ei] == 2 && !silhouette_from(s, e, p)) break;
                    }
                    v3 pa = ld3(s.P, e.x), pb = ld3(s.P, e.y);
                    // the point on the edge: uniform in t, or by the clamped cosine
                    float te = NEE ? te_draw : b0.y, pdf_t = 1.0f;
                    if (PH == 2) {
                        // the sampling pass's point (no transcendentals here)
                        te = sp.q[qi].te;
                        pdf_t = sp.q[qi].pdf_t;
                    } else if (a.edge_t == 1) {
                        float Tc;
                        if (!cosine_edge_t(p, n, pa, pb, b0.y, te, Tc)) break;
                        pdf_t = cosine_edge_pdf(p, n, pa, pb, te, Tc);
                        if (!(pdf_t > 0.0f)) break;
                    }
                    v3 w = pa + (pb - pa) * te - p;
                    if (PH != 2 && dot(n, w) <= kHorizon * s.diag) break;
                    v3 v0p = pa - p, v1p = pb - p;
                    v3 c = cross(v0p, v1p);
                    float cn = len(c);
                    if (PH != 2 && cn == 0.0f) break;
                    v3 nh = c * (1.0f / cn);
                    float wl = len(w);
                    v3 wh = w * (1.0f / wl);
                    v3 wp = nrm(wh + nh * kEps3), wm = nrm(wh - nh * kEps3);
                    int rem = a.depth - (kk + 1);
                    // no bounce left and no light along either side: both
                    // radiances are zero, and so is the sample
                    if (PH != 2 && rem == 0 && !may_reach_light(s, p, wp, s.tmin) && !may_reach_light(s, p, wm, s.tmin))
                        break;
                    float Lp, Lm;
                    if (PH == 1) {
                        // queue the side paths: one atomic per wave
                        unsigned long long bal = __ballot(1);
                        int leader = __ffsll(bal) - 1;
                        int base = 0;
                        // one queue segment of a.M slots per path vertex, so that
                        // the side paths of a segment all have the same length
                        if (lane == leader) base = atomicAdd(&sp.count[kk], __popcll(bal));
                        base = __shfl(base, leader, BS);
                        int slot = kk * a.M + base + __popcll(bal & ((1ull << lane) - 1ull));
                        SideQuery Q;
                        Q.p[0] = p.x; Q.p[1] = p.y; Q.p[2] = p.z;
                        Q.wp[0] = wp.x; Q.wp[1] = wp.y; Q.wp[2] = wp.z;
                        Q.wm[0] = wm.x; Q.wm[1] = wm.y; Q.wm[2] = wm.z;
                        Q.sid = sid;
                        Q.edge = ei;
                        Q.pdf = pdf;
                        Q.k = kk;
                        Q.te = te;
                        Q.pdf_t = pdf_t;
                        sp.q[slot] = Q;
                        sp.qidx[(size_t)kk * a.M + m] = slot;
                        break;
                    } else if (PH == 2) {
                        float2 L = sp.res[qi];
                        Lp = L.x;
                        Lm = L.y;
                    } else {
                        radiance_pair(s, rk, kSideBlockBase, p, wp, wm, s.tmin, false, rem, my, BS, wk, Lp, Lm);
                    }
                    // the cosine is continuous across the edge; only the radiance jumps
                    float cosw = dot(n, wh);
                    float Fp = rho[kk] / kPi * cosw * Lp;
                    float Fm = rho[kk] / kPi * cosw * Lm;
                    if (Fp == Fm) break;
                    float Wk = d_image[pix] * beta[kk] / (float)a.spp;
                    float wgt = Wk * (Fp - Fm) * len(cross(pb - pa, wh)) / (cn * wl * pdf * pdf_t);
#ifdef DIFFRT_DEVICE_PRINTF
                    if (dbg)
                        printf("unit %d vertex %d tri %d p=(%.9g %.9g %.9g) n=(%.9g %.9g %.9g) edge %d pdf %.9g t %.9g Lp %.9g "
                               "Lm %.9g cos %.9g W %.9g wgt %.9g\n",
                               m, kk + 1, tri[kk], p.x, p.y, p.z, n.x, n.y, n.z, ei, pdf, te, Lp, Lm, cosw, Wk, wgt);
#endif
                    if (PH == 2) {
                        v3 c0 = cross(v1p, wh) * wgt, c1 = cross(wh, v0p) * wgt;
                        bedge = ei;
                        bval[0] = c0.x; bval[1] = c0.y; bval[2] = c0.z;
                        bval[3] = c1.x; bval[4] = c1.y; bval[5] = c1.z;
                    } else {
                        atomic_add3(dV, e.x, cross(v1p, wh) * wgt);
                        atomic_add3(dV, e.y, cross(wh, v0p) * wgt);
                    }
                    wk.atomics(6);
                    if (MIX && mx.estats) {
                        v3 c0 = cross(v1p, wh), c1 = cross(wh, v0p);
                        atomicAdd(&mx.estats[ei], pdf * pdf_t * wgt * wgt * (dot(c0, c0) + dot(c1, c1)));
                    }
                    xbar[kk] += (cross(wh, v1p) + cross(v0p, wh)) * wgt;
                } while (false);
                if (PH == 2) {
                    if (__ballot(1) == ~0ull) {
                        scatter_grouped(bedge >= 0, bedge, bval, 4, edge_dest);
                    } else if (bedge >= 0) {
#pragma unroll
                        for (int i = 0; i < 6; ++i)
                            if (bval[i] != 0.0f) atomicAdd(edge_dest(bedge, i), bval[i]);
                    }
                }
            }
        }
        // ---- reverse sweep: interior term and propagation of vertex adjoints
        if (PH == 1) nv = 0;
        bool interior = (a.terms & DR_TERM_INTERIOR) != 0;
        float Aft = 0.0f;          // radiance from later vertices per unit throughput there
        v3 carry = {0, 0, 0};      // adjoint of this vertex's position from the next ray-plane
        v3 gd0 = {0, 0, 0};
        float grho_k = 0.0f;       // albedo adjoint of vertices 2.. (scattered with their vertices)
#pragma unroll
        for (int kk = MAXD - 1; kk >= 0; --kk) {
            if (kk >= nv) continue;
            int t = tri[kk];
            TriGeom g = tri_geom(s, t);
            v3 gns = {0, 0, 0};
            v3 gx = xbar[kk] + carry;
            float Nk = 0.0f;
            bool cont = false;
            float Ab = 0.0f;
            if (AOV) {
                // d(buffer)/d(position, oriented normal, albedo) at the first hit;
                // with all channels (aov = 8) their loss gradients are npix apart
                if (interior) {
                    float wc7[7];
                    long npix = (long)a.Ww * (k.y1 - k.y0);
#pragma unroll
                    for (int c = 0; c < 7; ++c)
                        wc7[c] = a.aov == 8 ? d_image[c * npix + pix] / (float)a.spp : (a.aov == c + 1 ? W0 : 0.0f);
                    gx += v3{wc7[0], wc7[1], wc7[2]};
                    gns = v3{wc7[3], wc7[4], wc7[5]};
                    g0[9] = wc7[6];
                }
            } else {
            // NEE of this vertex, recomputed from its random numbers; the
            // visibility comes from the forward pass
            NeeSample q = nee_sample(s, rc.block(2 * kk + 1), xs[kk], ns[kk]);
            float Kk = ((vis >> kk) & 1) ? q.K : 0.0f;
            float nee_cos = dot(ns[kk], q.w);
            Nk = rho[kk] * nee_cos * Kk;
            cont = cc[kk] > 0.0f;
            Ab = cont ? Aft : 0.0f;
            if (interior) {
                float gN = W0 * beta[kk];
                float gw = cont ? W0 * beta[kk] * Ab : 0.0f;
                float grho = gN * nee_cos * Kk + gw;
                if (kk == 0) g0[9] = grho;
                else grho_k = grho;
                gns = q.w * (gN * rho[kk] * Kk);
                if (cont) gns += wc[kk] * (gw * rho[kk] / cc[kk]);
            }
            }
            v3 gp0 = {0, 0, 0}, gp1 = {0, 0, 0}, gp2 = {0, 0, 0};
            if (gns.x != 0.0f || gns.y != 0.0f || gns.z != 0.0f)
                shading_normal_adj(s, t, g, xs[kk], gns * sg[kk], gx, gp0, gp1, gp2);
            v3 go = {0, 0, 0}, gd = {0, 0, 0};
            v3 org = kk == 0 ? k.c : xs[kk == 0 ? 0 : kk - 1];
            v3 dir = kk == 0 ? d0 : wc[kk == 0 ? 0 : kk - 1];
            ray_plane_adj(g, org, dir, gx, go, gd, gp0, gp1, gp2);
            if (kk == 0) {
                have0 = true;
                key0 = t;
                g0[0] = gp0.x; g0[1] = gp0.y; g0[2] = gp0.z;
                g0[3] = gp1.x; g0[4] = gp1.y; g0[5] = gp1.z;
                g0[6] = gp2.x; g0[7] = gp2.y; g0[8] = gp2.z;
            } else if (__ballot(1) == ~0ull) {
                // every lane of the wave is at this vertex: lanes that hit the
                // same triangle (large walls, say) are summed before the atomics
                const float gv[10] = {gp0.x, gp0.y, gp0.z, gp1.x, gp1.y, gp1.z, gp2.x, gp2.y, gp2.z, grho_k};
                scatter_grouped(true, t, gv, 4, [&](int tt, int i) {
                    return i == 9 ? &dA[tt] : &dV[3 * s.I[3 * tt + i / 3] + (i % 3)];
                });
                grho_k = 0.0f;
            } else {
                int i0 = s.I[3 * t], i1 = s.I[3 * t + 1], i2 = s.I[3 * t + 2];
                atomic_add3(dV, i0, gp0);
                atomic_add3(dV, i1, gp1);
                atomic_add3(dV, i2, gp2);
                if (grho_k != 0.0f) atomicAdd(&dA[t], grho_k);
                grho_k = 0.0f;
            }
            wk.atomics(10);
            if (kk == 0) {
                ca.c += go;
                gd0 = gd;
            } else {
                carry = go;        // the ray of vertex kk starts at vertex kk-1; its direction is held fixed
            }
            Aft = Nk + (cont ? rho[kk] * Ab : 0.0f);
        }
        // camera ray direction d = f + a r + b u
        ca.f += gd0;
        ca.r += gd0 * (ndx * k.asp * k.th);
        ca.u += gd0 * (ndy * k.th);
    }
    scatter_grouped(have0, key0, g0, 4, [&](int t, int i) {
        return i == 9 ? &dA[t] : &dV[3 * s.I[3 * t + i / 3] + (i % 3)];
    });
    flush_work(wk, a.counters);
    flush_cam(ca, camacc);
}

// dL/d(position, look_at, up) from the frame adjoints (f, r, u, c).
template <int MAXD, int STK, bool CNT, bool MIX, bool AOV = false>
__global__ __launch_bounds__(BS) void k_backward(SceneView s, Cam k, RenderArgs a, TreeView tv, const float* __restrict__ d_image,
                                                 float* __restrict__ dV, float* __restrict__ dA, float* __restrict__ camacc,
                                                 MixArgs mx) {
    __shared__ int stk[STK * BS];
    int sh = blockIdx.x & (a.gshards - 1);
    backward_body<MAXD, STK, CNT, MIX, 0, AOV>(s, k, a, tv, d_image, dV + sh * a.gstride, dA + sh * a.gstride, camacc + 12 * sh,
                                       mx, blockIdx.x * BS, stk);
}

// Split backward, pass 1: secondary edge samples of every path vertex, their
// side-path queries appended to a compact queue.
template <int MAXD, int STK, bool NEE = false>
__global__ __launch_bounds__(BS) void k_bwd_sample(SceneView s, Cam k, RenderArgs a, TreeView tv, SplitArgs sp) {
    __shared__ int stk[STK * BS];
    MixArgs mx{};
    backward_body<MAXD, STK, false, false, 1, false, NEE>(s, k, a, tv, nullptr, nullptr, nullptr, nullptr, mx,
                                                           blockIdx.x * BS, stk, sp);
}

// Split backward, pass 1, one lane per (path vertex, unit) when every vertex
// the pass needs is checkpointed (kernel depth <= 3): items are vertex-major
// (item = kk * M + m), so a unit's edge-tree descents, each a chain of
// dependent node fetches, run in parallel lanes instead of one after another.
// Each lane rebuilds its unit's path up to its vertex with the adjoint pass's
// arithmetic (same operations in the same order) and appends its side-path
// query to segment kk of the queue.
template <int STK, bool MIX, bool SEL = false, bool NEE = false>
__global__ __launch_bounds__(BS) void k_bwd_sample_v(SceneView s, Cam k, RenderArgs a, TreeView tv, SplitArgs sp,
                                                     int nvert, MixArgs mx) {
    // no rays are traced here: no traversal stack (STK only names the variant);
    // SEL: the multi-sample edge selection and its LDS stack of deferred children;
    // NEE: the strip strategy (next event estimation for edges) mixed with the
    // hierarchy, and the LDS stack of its walks through the triangle BVH
    __shared__ int sel_stk[SEL ? kSelectMax * 4 * BS : 1];
    __shared__ int walk_stk[NEE ? STK * BS : 1];
    int lane = threadIdx.x;
    NoWork wk;
    long item = (long)blockIdx.x * BS + lane;
    int kk = (int)(item / a.M);
    int m = (int)(item - (long)kk * a.M);
    bool in = kk < nvert;
    if (in) sp.qidx[(size_t)kk * a.M + m] = -1;
    bool push = false;
    SideQuery Q;
    if (in && (!a.mask || a.mask[m]) && a.depth >= kk + 1 && a.ck_tri[m] >= 0 && tv.valid &&
        (a.terms & DR_TERM_SECONDARY)) {
        int pix, px, py;
        uint32_t sid;
        unit_pixel(k, a, m, pix, px, py, sid);
        Rng rc{sid, a.view, kTagCam, a.k0, a.k1};
        float4 j = rc.block(0);
        float sx = px + j.x, sy = py + j.y;
        float ndx = 2.0f * sx / k.W - 1.0f, ndy = 1.0f - 2.0f * sy / k.H;
        v3 d = k.f + k.r * (ndx * k.asp * k.th) + k.u * (ndy * k.th);
        // the path up to vertex kk, as the adjoint pass rebuilds it
        int t = a.ck_tri[m];
        v3 x = {a.ck_x[3 * (size_t)m], a.ck_x[3 * (size_t)m + 1], a.ck_x[3 * (size_t)m + 2]};
        v3 n = {0, 0, 0};
        bool alive = false;
        for (int jj = 0; jj <= kk; ++jj) {
            TriGeom g = tri_geom(s, t);
            float sgn = dot(d, cross(g.e1, g.e2)) < 0.0f ? 1.0f : -1.0f;
            n = shading_normal(s, t, g, x) * sgn;
            if (s.alb[t] == 0.0f) break;
            if (jj == kk) {
                alive = true;
                break;
            }
            float4 ub = rc.block(2 * jj + 2);
            v3 w = cosine_dir(n, ub.x, ub.y);
            if (dot(n, w) <= 0.0f) break;
            int t2 = a.ck_tri[(size_t)(jj + 1) * a.M + m];
            if (t2 < 0) break;
            const float* cx = a.ck_x + 3 * ((size_t)(jj + 1) * a.M + m);
            v3 x2 = {cx[0], cx[1], cx[2]};
            if (s.alb[t2] == 0.0f) break;
            d = w;
            t = t2;
            x = x2;
        }
        if (alive) {
            Rng rk{sid, a.view, kTagSedge + (uint32_t)(kk + 1), a.k0, a.k1};
            float4 b0 = rk.block(0);
            v3 p = x;
            float pdf;
            TreeCtx q = tree_ctx(&s, p, n, tv.cam, t, kHorizon * s.diag, kInsidePad * s.diag);
            int ei;
            float te_draw = 0.0f;
            do {
                if (NEE) {
                    Rng rn{sid, a.view, kTagEnee + (uint32_t)(kk + 1), a.k0, a.k1};
                    ei = strip_mix_draw(s, tv, q, a, rk, b0, rn, te_draw, pdf, walk_stk + lane, BS, wk);
                } else if (MIX && mx.sec) {
                    // proposal mixture: component from the third uniform of the
                    // block, proposal draw from the fourth
                    float pt;
                    if (b0.z < mx.mix) {
                        ei = pick_cdf_d(mx.qcdf, s.E, (double)b0.w);
                        pt = tree_pdf_edge(tv, q, ei, wk);
                    } else {
                        ei = tree_sample(tv, q, rk, b0.x, pt, wk, m == a.debug_unit);
                        if (ei < 0) break;
                    }
                    pdf = mx.mix * mx.q[ei] + (1.0f - mx.mix) * pt;
                    if (!(pdf > 0.0f) || s.ekind[ei] == 0) break;
                } else if (SEL) {
                    Rng rs{sid, a.view, kTagSelect + (uint32_t)(kk + 1), a.k0, a.k1};
                    ei = tree_select(tv, q, rs, a.cands, pdf, sel_stk + lane, BS, wk);
                } else {
                    ei = tree_sample(tv, q, rk, b0.x, pdf, wk, m == a.debug_unit);
                }
                if (ei < 0) break;
                int4 e = s.edges[ei];
                if (e.z == t || e.w == t) break;
                if (s.ekind[ei] == 2 && !silhouette_from(s, e, p)) break;
                v3 pa = ld3(s.P, e.x), pb = ld3(s.P, e.y);
                float te = NEE ? te_draw : b0.y, pdf_t = 1.0f;
                if (!NEE && a.edge_t == 1) {
                    float Tc;
                    if (!cosine_edge_t(p, n, pa, pb, b0.y, te, Tc)) break;
                    pdf_t = cosine_edge_pdf(p, n, pa, pb, te, Tc);
                    if (!(pdf_t > 0.0f)) break;
                }
                v3 w = pa + (pb - pa) * te - p;
                if (dot(n, w) <= kHorizon * s.diag) break;
                v3 c = cross(pa - p, pb - p);
                float cn = len(c);
                if (cn == 0.0f) break;
                v3 nh = c * (1.0f / cn);
                v3 wh = w * (1.0f / len(w));
                v3 wp = nrm(wh + nh * kEps3), wm = nrm(wh - nh * kEps3);
                // the last vertex's side paths end at their first hit: with no
                // light along either side, both radiances and the sample are zero
                if (kk + 1 == a.depth && !may_reach_light(s, p, wp, s.tmin) && !may_reach_light(s, p, wm, s.tmin))
                    break;
                Q.p[0] = p.x; Q.p[1] = p.y; Q.p[2] = p.z;
                Q.wp[0] = wp.x; Q.wp[1] = wp.y; Q.wp[2] = wp.z;
                Q.wm[0] = wm.x; Q.wm[1] = wm.y; Q.wm[2] = wm.z;
                Q.sid = sid;
                Q.edge = ei;
                Q.pdf = pdf;
                Q.k = kk;
                Q.te = te;
                Q.pdf_t = pdf_t;
                push = true;
            } while (false);
        }
    }
    // append to the queue segment of each lane's vertex: one atomic per
    // (wave, vertex); a wave spans more than one vertex only at segment ends
    unsigned long long left = __ballot(push);
    while (left) {
        int leader = __ffsll(left) - 1;
        int kl = __shfl(kk, leader, BS);
        bool mine = push && kk == kl;
        unsigned long long bal = __ballot(mine);
        int base = 0;
        if (lane == leader) base = atomicAdd(&sp.count[kl], __popcll(bal));
        base = __shfl(base, leader, BS);
        if (mine) {
            int slot = kl * a.M + base + __popcll(bal & ((1ull << lane) - 1ull));
            sp.q[slot] = Q;
            sp.qidx[(size_t)kk * a.M + m] = slot;
        }
        left &= ~bal;
    }
}

// Split backward, pass 2: both one-sided radiances of every queued query, one
// query per lane (no idle lanes), with the query's own Philox stream.
template <int STK>
__global__ __launch_bounds__(BS) void k_side(SceneView s, RenderArgs a, SplitArgs sp, int kk) {
    __shared__ int stk[STK * BS];
    int lane = threadIdx.x;
    int* my = stk + lane;
    NoWork wk;
    int n = sp.count[kk];
    for (int base = blockIdx.x * BS; base < n; base += gridDim.x * BS) {
        int i = kk * a.M + base + lane;
        if (base + lane < n) {
            SideQuery Q = sp.q[i];
            Rng rk{Q.sid, a.view, kTagSedge + (uint32_t)(Q.k + 1), a.k0, a.k1};
            int rem = a.depth - (Q.k + 1);
            v3 p = {Q.p[0], Q.p[1], Q.p[2]};
            v3 wp = {Q.wp[0], Q.wp[1], Q.wp[2]}, wm = {Q.wm[0], Q.wm[1], Q.wm[2]};
            float Lp, Lm;
            radiance_pair(s, rk, kSideBlockBase, p, wp, wm, s.tmin, false, rem, my, BS, wk, Lp, Lm);
            sp.res[i] = make_float2(Lp, Lm);
        }
    }
}

// Split backward, pass 3: boundary contributions from the queued radiances and
// the adjoint sweep. Six waves per SIMD (at most 80 VGPRs) hide more of its
// dependent loads than four (7.4 -> 6.8 ms at config 3).
template <int MAXD, int STK, bool MIX>
__global__ __launch_bounds__(BS, 6) void k_bwd_adjoint(SceneView s, Cam k, RenderArgs a, TreeView tv,
                                                    const float* __restrict__ d_image, float* __restrict__ dV,
                                                    float* __restrict__ dA, float* __restrict__ camacc, SplitArgs sp,
                                                    MixArgs mx) {
    __shared__ int stk[STK * BS];
    int sh = blockIdx.x & (a.gshards - 1);
    backward_body<MAXD, STK, false, MIX, 2>(s, k, a, tv, d_image, dV + sh * a.gstride, dA + sh * a.gstride,
                                            camacc + 12 * sh, mx, blockIdx.x * BS, stk, sp);
}

__device__ inline void cam_finalize(const Cam& k, const float* __restrict__ acc, float* __restrict__ d_camera) {
    v3 gf = {acc[0], acc[1], acc[2]}, gr = {acc[3], acc[4], acc[5]}, gu = {acc[6], acc[7], acc[8]}, gc = {acc[9], acc[10], acc[11]};
    v3 look = k.look, up = k.upv;
    // u = r x f
    gr += cross(k.f, gu);
    gf += cross(gu, k.r);
    // r = normalize(f x up)
    v3 gg = nrm_adj(cross(k.f, up), gr);
    gf += cross(up, gg);
    v3 gup = cross(gg, k.f);
    // f = normalize(look - c)
    v3 gh = nrm_adj(look - k.c, gf);
    v3 gl = gh;
    gc -= gh;
    d_camera[0] = gc.x; d_camera[1] = gc.y; d_camera[2] = gc.z;
    d_camera[3] = gl.x; d_camera[4] = gl.y; d_camera[5] = gl.z;
    d_camera[6] = gup.x; d_camera[7] = gup.y; d_camera[8] = gup.z;
}

// One wave: lane j sums copies j, j + 64, ...; the wave then adds the lanes.
static __global__ void k_cam_finalize(Cam k, const float* __restrict__ acc, int shards, float* __restrict__ d_camera) {
    if (blockIdx.x != 0) return;
    float sum[12];
    for (int i = 0; i < 12; ++i) {
        float v = 0.0f;
        for (int h = threadIdx.x; h < shards; h += BS) v += acc[12 * h + i];
        sum[i] = wave_sum(v);
    }
    if (threadIdx.x == 0) cam_finalize(k, sum, d_camera);
}

// out[i] = sum over the copies of shard[h * stride + i], i < n. A block of
// 256 threads takes 32 consecutive entries: eight groups of 32 lanes read
// copies g, g + 8, ... of them (coalesced within a group), and the eight
// partial sums meet in LDS, so that small arrays still spread over many waves.
// Launch with 256 threads and ceil(n / 32) blocks.
constexpr int kReduceEntries = 32;
static __global__ __launch_bounds__(256) void k_reduce_shards(const float* __restrict__ shard, int shards, long stride,
                                                            long n, float* __restrict__ out) {
    __shared__ float part[256];
    int e = threadIdx.x % kReduceEntries, g = threadIdx.x / kReduceEntries;
    long i = (long)blockIdx.x * kReduceEntries + e;
    float v = 0.0f;
    if (i < n)
        for (int h = g; h < shards; h += 256 / kReduceEntries) v += shard[h * stride + i];
    part[threadIdx.x] = v;
    __syncthreads();
    if (g == 0 && i < n) {
        float t = 0.0f;
        for (int k = 0; k < 256 / kReduceEntries; ++k) t += part[k * kReduceEntries + e];
        out[i] = t;
    }
}

// ---------------------------------------------------------------------------
// batches of views: one launch per kernel for every view. Each block of 64
// units lies in one view, so the view's arguments are uniform per block.
// Work items of `chunk` blocks are taken in grid order, or from an atomic
// counter when the grid is persistent (smaller than the work list).
// ---------------------------------------------------------------------------
__device__ inline int batch_view(const BatchLaunch& L, int b) {
    int lo = 0, hi = L.nviews - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (L.boff[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline int batch_next(const BatchLaunch& L, int it, int* slot) {
    int item;
    if (L.queue) {
        if (threadIdx.x == 0) *slot = atomicAdd(L.queue, 1);
        __syncthreads();
        item = *slot;
        __syncthreads();
    } else {
        item = blockIdx.x + it * gridDim.x;
    }
    return __builtin_amdgcn_readfirstlane(item);
}

template <int STK>
__global__ __launch_bounds__(BS) void k_forward_batch(SceneView s, BatchLaunch L) {
    __shared__ int stk[STK * BS];
    __shared__ int slot;
    for (int it = 0;; ++it) {
        int item = batch_next(L, it, &slot);
        if (item >= (L.total + L.chunk - 1) / L.chunk) break;
        for (int c = 0; c < L.chunk; ++c) {
            int b = item * L.chunk + c;
            if (b >= L.total) break;
            int v = __builtin_amdgcn_readfirstlane(batch_view(L, b));
            const BatchView& bv = L.views[v];
            forward_body<STK, false>(s, bv.k, bv.a, bv.image, bv.reduce, (b - L.boff[v]) * BS, stk);
        }
    }
}

template <int STK>
__global__ __launch_bounds__(BS) void k_primary_batch(SceneView s, BatchLaunch L, float* __restrict__ dV) {
    __shared__ int stk[STK * BS];
    __shared__ int slot;
    MixArgs mx{};
    for (int it = 0;; ++it) {
        int item = batch_next(L, it, &slot);
        if (item >= (L.total + L.chunk - 1) / L.chunk) break;
        for (int c = 0; c < L.chunk; ++c) {
            int b = item * L.chunk + c;
            if (b >= L.total) break;
            int v = __builtin_amdgcn_readfirstlane(batch_view(L, b));
            const BatchView& bv = L.views[v];
            int sh = blockIdx.x & (L.gshards - 1);
            primary_body<STK, false, false>(s, bv.k, bv.a, bv.pe, bv.pcdf, bv.d_image, dV + sh * L.gstride,
                                            bv.camacc + 12 * sh, mx, (b - L.boff[v]) * BS, stk);
        }
    }
}

template <int MAXD, int STK>
__global__ __launch_bounds__(BS) void k_backward_batch(SceneView s, BatchLaunch L, float* __restrict__ dV,
                                                       float* __restrict__ dA) {
    __shared__ int stk[STK * BS];
    __shared__ int slot;
    MixArgs mx{};
    for (int it = 0;; ++it) {
        int item = batch_next(L, it, &slot);
        if (item >= (L.total + L.chunk - 1) / L.chunk) break;
        for (int c = 0; c < L.chunk; ++c) {
            int b = item * L.chunk + c;
            if (b >= L.total) break;
            int v = __builtin_amdgcn_readfirstlane(batch_view(L, b));
            const BatchView& bv = L.views[v];
            int sh = blockIdx.x & (L.gshards - 1);
            backward_body<MAXD, STK, false, false>(s, bv.k, bv.a, bv.tv, bv.d_image, dV + sh * L.gstride,
                                                   dA + sh * L.gstride, bv.camacc + 12 * sh, mx, (b - L.boff[v]) * BS,
                                                   stk);
        }
    }
}

static __global__ void k_cam_finalize_batch(const BatchView* __restrict__ views, int n, int shards, float* __restrict__ d_cameras) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    float sum[12];
    for (int i = 0; i < 12; ++i) {
        sum[i] = 0.0f;
        for (int h = 0; h < shards; ++h) sum[i] += views[v].camacc[12 * h + i];
    }
    cam_finalize(views[v].k, sum, d_cameras + 9 * v);
}

static __global__ void k_batch_zero(const BatchView* __restrict__ views, int n, int image, int shards) {
    // zeroes each view's image (image = 1) or camera accumulator (image = 0)
    int v = blockIdx.y;
    if (v >= n) return;
    const BatchView& bv = views[v];
    if (image) {
        int npix = bv.a.M / bv.a.spp;
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += gridDim.x * blockDim.x) bv.image[i] = 0.0f;
    } else if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < 12 * shards; i += blockDim.x) bv.camacc[i] = 0.0f;
    }
}

static __global__ void k_batch_seed(BatchView* __restrict__ views, int n, uint32_t add) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) views[v].a.k0 += add;
}

static __global__ void k_fill_i32(int* __restrict__ p, int v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}

static __global__ void k_fill_count(int* __restrict__ c, int n) {
    if (blockIdx.x == 0 && (int)threadIdx.x < n) c[threadIdx.x] = 0;
}

static __global__ void k_fill(float* __restrict__ p, long n, float v) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline int nblk(long n, int bs) { return (int)((n + bs - 1) / bs); }

// Brackets one kernel launch with HIP events when profiling is on.
struct EvScope {
    drScene_t* s;
    int kind;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    EvScope(drScene_t* s_, int kind_, hipStream_t st_) : s(s_), kind(kind_), st(st_) {
        s->launches[kind]++;
        if (!s->prof_events) return;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        (void)hipEventRecord(a, st);
    }
    ~EvScope() {
        if (!a) return;
        (void)hipEventRecord(b, st);
        s->evs.push_back({a, b, kind});
    }
};

static RenderArgs make_args(drScene_t* s, const Cam& cam, const drRenderOptions& o) {
    RenderArgs a;
    a.spp = o.spp;
    a.depth = o.max_depth;
    a.Ww = cam.x1 - cam.x0;
    a.M = a.Ww * (cam.y1 - cam.y0) * o.spp;
    a.k0 = (uint32_t)(o.seed & 0xffffffffu);
    a.k1 = (uint32_t)(o.seed >> 32);
    a.view = o.view_id;
    a.terms = o.terms ? o.terms : DR_TERM_ALL;
    a.mask = o.unit_mask;
    const char* du = std::getenv("DIFFRT_DEBUG_UNIT");
    a.debug_unit = du ? std::atoi(du) : -1;
    a.counters = s->prof_counters ? s->counters.as<unsigned long long>() : nullptr;
    a.ck_tri = s->ck_tri.as<int>();
    a.ck_x = s->ck_x.as<float>();
    a.ck_vis = s->ck_vis.as<uint8_t>();
    a.gshards = 1;
    a.gstride = 0;
    a.aov = o.aov;
    a.edge_t = o.edge_t_mode;
    a.cands = o.edge_candidates;
    a.nee = o.edge_nee;
    a.nee_w = o.edge_nee_width > 0.0f ? o.edge_nee_width : s->nee_w;
    return a;
}

// Traversal stack per lane: kSmallStack entries when the BVH is at most that
// many internal nodes deep (then the stack can never overflow: a near-first
// descent pushes at most one entry per level), kStackDepth otherwise.
static inline bool small_stack(const drScene_t* s) { return s->bvh_depth <= kSmallStack; }

}  // namespace dr
