// FP64 CPU oracle of the differentiable edge-sampling path tracer.
//
// TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
// benchmark's CPU-baseline leg. It shares no code with the HIP library.
//
// Plain and slow on purpose: exact FP64 arithmetic, brute-force or
// median-split-BVH intersection, and a generic tape-based reverse-mode
// differentiator (thesis Ch. 2, Reverse-mode) for the interior term, so that
// the hand-written GPU adjoints are checked against a mechanism that has no
// hand-derived derivative in it. The boundary terms are written out from the
// thesis's formulas (Ch. 5, Method):
//   primary   eq. edge_equation, eq. dirac_rewrite, eq. redner_dirac_jacobian, eq. mc
//   secondary eq. 3d_half_space / eq. dirac_3d_edge in the direction measure
// and the edge hierarchy from Importance Sampling the Edges, Edge selection.
//
// Readings where the thesis is silent (random-number layout, constants, light
// transport details, measure convention) follow the written specification of
// the project; each one is named where it is used.
#include "oracle.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <unordered_map>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

const double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Near-tie thresholds. A unit (one pixel sample plus its primary edge sample)
// is flagged when one of its discrete decisions lies this close to a tie, so
// that an FP32 implementation may legitimately decide the other way.
// ---------------------------------------------------------------------------
const double kTieWorld = 2.5e-7;  // ray-to-triangle-edge distance, relative to the scene diagonal
const double kTieT = 1e-6;        // relative distance between hit distances
const double kTieCos = 1e-5;      // |cos| of grazing hits
const double kTieU = 1e-5;        // uniform vs. branch probability
const double kTieCdf = 5e-7;      // uniform vs. FP64 CDF built from FP32 lengths/areas
const double kTieSign = 1e-5;     // relative plane-side tests
const double kTiePx = 1e-3;       // edge point vs. pixel boundary (pixels)
const double kTieCond = 1e-3;     // sin(angle(v0', v1')) of secondary edges
const double kTieBox = 1e-6;      // relative point-in-box / sphere tests
const double kTieDepart = 1e-6;   // FP32 error of a surface point, relative to max(1, |x|) (rays leaving a surface)
const double kTieRes = 1e-4;      // reservoir uniform vs. its FP32 keep probability (relative): weights are
                                  // importance / descent pdf, a chain of some 25 operations per level

// Constants of the estimator (shared by specification with the GPU path).
const double kEpsPx = 1e-3;       // primary: offset of the two sides, pixels
const double kEps3 = 1e-4;        // secondary: angular offset of the two sides
const double kTminRel = 1e-4;     // secondary ray t_min, relative to scene diagonal
const double kShadowEnd = 1e-4;   // shadow rays stop at (1 - this) * distance
const double kInsidePad = 1e-4;   // "point inside the parent box" uses the box grown by this * diagonal
const double kVsphereMargin = 1e-5;  // v-sphere pruning only beyond this relative margin (conservative)
const double kHorizon = 1e-5;     // edge points within this * diagonal of the tangent plane are skipped

// Philox counter tags.
// SEDGE_k = 1 + k, SELECT_k = 16 + k, ENEE_k = 32 + k (billboard strategy of the secondary edge sample)
enum : uint32_t { TAG_CAM = 0, TAG_PEDGE = 1, TAG_SEDGE = 1, TAG_SELECT = 16, TAG_ENEE = 32 };
const int kSideBlockBase = 32;    // side-path blocks of secondary edge samples
const int kMaxLevels = 64;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), from its definition.
// ---------------------------------------------------------------------------
void philox(const uint32_t ci[4], const uint32_t ki[2], uint32_t out[4]) {
    uint32_t c0 = ci[0], c1 = ci[1], c2 = ci[2], c3 = ci[3];
    uint32_t k0 = ki[0], k1 = ki[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// One stream = (sample id, view id, tag); block b gives four uniforms
// u = (x >> 8) * 2^-24, exact in both FP32 and FP64.
struct Stream {
    uint32_t sid, view, tag, k0, k1;
    void block(uint32_t b, double u[4]) const {
        uint32_t c[4] = {sid, view, tag, b}, k[2] = {k0, k1}, o[4];
        philox(c, k, o);
        for (int i = 0; i < 4; ++i) u[i] = (double)(o[i] >> 8) * (1.0 / 16777216.0);
    }
};

// ---------------------------------------------------------------------------
// Tape for reverse-mode differentiation (thesis Ch. 2, Reverse-mode): every
// operation on a differentiated value records its operands and local
// partials; a backward sweep from an output accumulates adjoints.
// ---------------------------------------------------------------------------
struct Tape {
    std::vector<int32_t> pa, pb;
    std::vector<double> ga, gb;
    std::vector<double> adj;
    int32_t push(int32_t a, double da, int32_t b, double db) {
        pa.push_back(a); ga.push_back(da); pb.push_back(b); gb.push_back(db);
        return (int32_t)pa.size() - 1;
    }
    void clear() { pa.clear(); pb.clear(); ga.clear(); gb.clear(); }
};
thread_local Tape TP;

struct D { double v; int32_t i; };
inline D mk(double v, int32_t a, double da, int32_t b, double db) {
    if (a < 0 && b < 0) return D{v, -1};
    return D{v, TP.push(a, da, b, db)};
}
inline D leafD(double v) { return D{v, TP.push(-1, 0.0, -1, 0.0)}; }
inline D operator+(D a, D b) { return mk(a.v + b.v, a.i, 1.0, b.i, 1.0); }
inline D operator-(D a, D b) { return mk(a.v - b.v, a.i, 1.0, b.i, -1.0); }
inline D operator*(D a, D b) { return mk(a.v * b.v, a.i, b.v, b.i, a.v); }
inline D operator/(D a, D b) { double q = a.v / b.v; return mk(q, a.i, 1.0 / b.v, b.i, -q / b.v); }
inline D operator-(D a) { return mk(-a.v, a.i, -1.0, -1, 0.0); }
inline D operator+(D a, double b) { return mk(a.v + b, a.i, 1.0, -1, 0.0); }
inline D operator+(double a, D b) { return b + a; }
inline D operator-(D a, double b) { return mk(a.v - b, a.i, 1.0, -1, 0.0); }
inline D operator-(double a, D b) { return mk(a - b.v, b.i, -1.0, -1, 0.0); }
inline D operator*(D a, double b) { return mk(a.v * b, a.i, b, -1, 0.0); }
inline D operator*(double a, D b) { return b * a; }
inline D operator/(D a, double b) { return mk(a.v / b, a.i, 1.0 / b, -1, 0.0); }
inline D operator/(double a, D b) { double q = a / b.v; return mk(q, b.i, -q / b.v, -1, 0.0); }
inline D sqrt(D a) { double s = std::sqrt(a.v); return mk(s, a.i, 0.5 / s, -1, 0.0); }

inline double val(double x) { return x; }
inline double val(D x) { return x.v; }
template <class S> S cst(double x);
template <> double cst<double>(double x) { return x; }
template <> D cst<D>(double x) { return D{x, -1}; }

template <class S> struct V3 { S x, y, z; };
using V3d = V3<double>;
template <class S> inline V3<S> operator+(const V3<S>& a, const V3<S>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class S> inline V3<S> operator-(const V3<S>& a, const V3<S>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class S> inline V3<S> operator-(const V3<S>& a) { return {-a.x, -a.y, -a.z}; }
template <class S, class T> inline V3<S> operator*(const V3<S>& a, T s) { return {a.x * s, a.y * s, a.z * s}; }
template <class S, class T> inline V3<S> operator/(const V3<S>& a, T s) { return {a.x / s, a.y / s, a.z / s}; }
template <class S> inline S dot(const V3<S>& a, const V3<S>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class S> inline V3<S> cross(const V3<S>& a, const V3<S>& b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class S> inline S length(const V3<S>& a) { using std::sqrt; return sqrt(dot(a, a)); }
template <class S> inline V3<S> normalize(const V3<S>& a) { return a / length(a); }
template <class S> inline V3d valv(const V3<S>& a) { return {val(a.x), val(a.y), val(a.z)}; }
template <class S> inline V3<S> lift(const V3d& a) { return {cst<S>(a.x), cst<S>(a.y), cst<S>(a.z)}; }
inline double comp(const V3d& a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

// Orthonormal basis around a unit normal (Duff et al. 2017, "Building an
// Orthonormal Basis, Revisited"). Used for cosine sampling and the cosine
// bound of the edge hierarchy; the GPU uses the same published formula.
void onb(const V3d& n, V3d& t1, V3d& t2) {
    double sign = std::copysign(1.0, n.z);
    double a = -1.0 / (sign + n.z);
    double b = n.x * n.y * a;
    t1 = {1.0 + sign * n.x * n.x * a, sign * b, -sign * n.x};
    t2 = {b, sign + n.y * n.y * a, -n.y};
}

// ---------------------------------------------------------------------------
// Scene
// ---------------------------------------------------------------------------
struct Edge { int va, vb, f0, f1; int kind; };  // kind: 0 never, 1 always, 2 silhouette-only

struct BNode { double lo[3], hi[3]; int left, right, first, count; };

struct Scn {
    int V = 0, T = 0;
    std::vector<double> P;        // [V][3]
    std::vector<int> I;           // [T][3]
    std::vector<double> alb, emi; // [T]
    std::vector<double> N;        // [V][3] if smooth
    bool smooth = false, two_sided = false;
    double bg = 0, diag = 0, tmin = 0;
    std::vector<Edge> edges;
    std::vector<int> lights;
    std::vector<double> lcdf;
    double atot = 0;
    std::vector<BNode> bvh;
    std::vector<int> border;
    std::vector<double> tie_bary;   // per triangle: near-edge threshold in barycentric units
    bool use_bvh = true;

    V3d p(int v) const { return {P[3 * v], P[3 * v + 1], P[3 * v + 2]}; }
    V3d nrm(int v) const { return {N[3 * v], N[3 * v + 1], N[3 * v + 2]}; }
    V3d face_n(int f) const {   // unnormalised geometric normal (e1 x e2)
        V3d a = p(I[3 * f]), b = p(I[3 * f + 1]), c = p(I[3 * f + 2]);
        return cross(b - a, c - a);
    }
};

int build_edges(Scn& s) {
    struct K { int a, b, f; };
    std::vector<K> ks;
    ks.reserve(3 * s.T);
    for (int f = 0; f < s.T; ++f)
        for (int j = 0; j < 3; ++j) {
            int a = s.I[3 * f + j], b = s.I[3 * f + (j + 1) % 3];
            ks.push_back({std::min(a, b), std::max(a, b), f});
        }
    std::sort(ks.begin(), ks.end(), [](const K& x, const K& y) {
        if (x.a != y.a) return x.a < y.a;
        if (x.b != y.b) return x.b < y.b;
        return x.f < y.f;
    });
    s.edges.clear();
    for (size_t i = 0; i < ks.size();) {
        size_t j = i;
        while (j < ks.size() && ks[j].a == ks[i].a && ks[j].b == ks[i].b) ++j;
        if (j - i > 2) return ORC_ENONMANIFOLD;
        Edge e{ks[i].a, ks[i].b, ks[i].f, j - i == 2 ? ks[i + 1].f : -1, 0};
        // Static classification of discontinuities (thesis: only silhouette
        // edges matter under smooth shading; boundaries, material changes and
        // flat creases are discontinuous from every viewpoint).
        if (e.f1 < 0) e.kind = 1;
        else if (s.alb[e.f0] != s.alb[e.f1] || s.emi[e.f0] != s.emi[e.f1]) e.kind = 1;
        else if (!s.smooth) {
            V3d n0 = s.face_n(e.f0), n1 = s.face_n(e.f1);
            V3d c = cross(n0, n1);
            bool coplanar = c.x == 0 && c.y == 0 && c.z == 0 && dot(n0, n1) > 0;
            e.kind = coplanar ? 0 : 1;
        } else e.kind = 2;
        s.edges.push_back(e);
        i = j;
    }
    return ORC_OK;
}

// Median-split BVH (oracle's own acceleration structure; leaves of <= 4).
void build_bvh(Scn& s) {
    s.border.resize(s.T);
    for (int i = 0; i < s.T; ++i) s.border[i] = i;
    std::vector<double> cen(3 * s.T);
    for (int f = 0; f < s.T; ++f)
        for (int k = 0; k < 3; ++k)
            cen[3 * f + k] = (s.P[3 * s.I[3 * f] + k] + s.P[3 * s.I[3 * f + 1] + k] + s.P[3 * s.I[3 * f + 2] + k]) / 3.0;
    s.bvh.clear();
    struct Job { int node, first, count; };
    s.bvh.push_back(BNode{});
    std::vector<Job> st{{0, 0, s.T}};
    while (!st.empty()) {
        Job j = st.back(); st.pop_back();
        BNode nd;
        for (int k = 0; k < 3; ++k) { nd.lo[k] = 1e300; nd.hi[k] = -1e300; }
        double clo[3] = {1e300, 1e300, 1e300}, chi[3] = {-1e300, -1e300, -1e300};
        for (int i = j.first; i < j.first + j.count; ++i) {
            int f = s.border[i];
            for (int v = 0; v < 3; ++v)
                for (int k = 0; k < 3; ++k) {
                    double x = s.P[3 * s.I[3 * f + v] + k];
                    nd.lo[k] = std::min(nd.lo[k], x); nd.hi[k] = std::max(nd.hi[k], x);
                }
            for (int k = 0; k < 3; ++k) { clo[k] = std::min(clo[k], cen[3 * f + k]); chi[k] = std::max(chi[k], cen[3 * f + k]); }
        }
        nd.first = j.first; nd.count = j.count; nd.left = nd.right = -1;
        if (j.count > 4) {
            int ax = 0;
            for (int k = 1; k < 3; ++k) if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
            int mid = j.first + j.count / 2;
            std::nth_element(s.border.begin() + j.first, s.border.begin() + mid, s.border.begin() + j.first + j.count,
                             [&](int a, int b) {
                                 if (cen[3 * a + ax] != cen[3 * b + ax]) return cen[3 * a + ax] < cen[3 * b + ax];
                                 return a < b;
                             });
            nd.left = (int)s.bvh.size(); s.bvh.push_back(BNode{});
            nd.right = (int)s.bvh.size(); s.bvh.push_back(BNode{});
            st.push_back({nd.left, j.first, mid - j.first});
            st.push_back({nd.right, mid, j.first + j.count - mid});
        }
        s.bvh[j.node] = nd;
    }
}

int prepare(const orc_scene* d, Scn& s) {
    if (!d || d->num_vertices <= 0 || d->num_triangles <= 0 || !d->vertices || !d->indices || !d->albedo || !d->emission)
        return ORC_EINVAL;
    s.V = d->num_vertices; s.T = d->num_triangles;
    if (d->vertices64) s.P.assign(d->vertices64, d->vertices64 + 3 * s.V);
    else s.P.assign(d->vertices, d->vertices + 3 * s.V);
    s.I.assign(d->indices, d->indices + 3 * s.T);
    for (int i = 0; i < 3 * s.T; ++i) if (s.I[i] < 0 || s.I[i] >= s.V) return ORC_EINVAL;
    if (d->albedo64) s.alb.assign(d->albedo64, d->albedo64 + s.T);
    else s.alb.assign(d->albedo, d->albedo + s.T);
    s.emi.assign(d->emission, d->emission + s.T);
    s.smooth = d->normals != nullptr;
    if (s.smooth) s.N.assign(d->normals, d->normals + 3 * s.V);
    s.two_sided = d->emission_two_sided != 0;
    s.bg = d->background;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int v = 0; v < s.V; ++v)
        for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], s.P[3 * v + k]); hi[k] = std::max(hi[k], s.P[3 * v + k]); }
    s.diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) + (hi[2] - lo[2]) * (hi[2] - lo[2]));
    s.tmin = kTminRel * s.diag;
    int rc = build_edges(s);
    if (rc) return rc;
    // Light selection proportional to area (reading: NEE picks one light
    // triangle by area, then a uniform point by the square-root warp).
    s.lights.clear(); s.lcdf.clear(); s.atot = 0;
    for (int f = 0; f < s.T; ++f)
        if (s.emi[f] > 0) {
            s.lights.push_back(f);
            s.atot += 0.5 * length(s.face_n(f));
            s.lcdf.push_back(s.atot);
        }
    for (double& c : s.lcdf) c /= s.atot;
    s.tie_bary.resize(s.T);
    for (int f = 0; f < s.T; ++f) {
        V3d a = s.p(s.I[3 * f]), b = s.p(s.I[3 * f + 1]), c = s.p(s.I[3 * f + 2]);
        double e = std::min(length(b - a), std::min(length(c - b), length(a - c)));
        s.tie_bary[f] = kTieWorld * s.diag / e;
    }
    build_bvh(s);
    return ORC_OK;
}

// ---------------------------------------------------------------------------
// Ray casting with near-tie detection
// ---------------------------------------------------------------------------
// Per-reason counters of near-tie flags (diagnostics for the tests).
int64_t g_reason[24];
#define TIE(U, r) do { (U).flag = true; __atomic_add_fetch(&g_reason[r], 1, __ATOMIC_RELAXED); } while (0)

struct Unit {
    bool flag = false;
    int64_t rays = 0;
    int dir_mode = 0;            // 0 off, 1 record, 2 replay (main path only)
    double* dir = nullptr;       // 64 slots: per vertex k, NEE (dir[3], factor, valid), BSDF (dir[3], cos)
};
const int kDirSlots = 64;

struct TriHit { bool ok; double t, u, v, m; bool valid; };

TriHit tri_test(const Scn& s, int f, const V3d& o, const V3d& d, double tmin, double tmax) {
    V3d a = s.p(s.I[3 * f]), b = s.p(s.I[3 * f + 1]), c = s.p(s.I[3 * f + 2]);
    V3d e1 = b - a, e2 = c - a;
    V3d pv = cross(d, e2);
    double det = dot(e1, pv);
    TriHit h{false, 0, 0, 0, 0, false};
    if (det == 0) return h;
    double inv = 1.0 / det;
    V3d tv = o - a;
    h.u = dot(tv, pv) * inv;
    V3d qv = cross(tv, e1);
    h.v = dot(d, qv) * inv;
    h.t = dot(e2, qv) * inv;
    h.m = std::min(std::min(h.u, h.v), 1.0 - h.u - h.v);
    h.valid = true;
    h.ok = h.u >= 0 && h.v >= 0 && h.u + h.v <= 1 && h.t > tmin && h.t < tmax;
    return h;
}

bool slab(const BNode& n, const V3d& o, const V3d& d, double pad, double t0, double t1) {
    const double ov[3] = {o.x, o.y, o.z}, dv[3] = {d.x, d.y, d.z};
    for (int k = 0; k < 3; ++k) {
        double lo = n.lo[k] - pad, hi = n.hi[k] + pad;
        if (dv[k] == 0) {
            if (ov[k] < lo || ov[k] > hi) return false;
            continue;
        }
        double a = (lo - ov[k]) / dv[k], b = (hi - ov[k]) / dv[k];
        if (a > b) std::swap(a, b);
        t0 = std::max(t0, a); t1 = std::min(t1, b);
        if (t0 > t1) return false;
    }
    return true;
}

template <class F>
void for_candidates(const Scn& s, const V3d& o, const V3d& d, double tmin, double tmax, F&& fn) {
    if (!s.use_bvh) {
        for (int f = 0; f < s.T; ++f) fn(f);
        return;
    }
    double pad = kTieWorld * s.diag + 1e-12;
    double dl = length(d);
    std::vector<int> st{0};
    while (!st.empty()) {
        int ni = st.back(); st.pop_back();
        const BNode& n = s.bvh[ni];
        if (!slab(n, o, d, pad, tmin - pad / dl, tmax * (1 + kTieT) + pad / dl)) continue;
        if (n.left < 0) {
            for (int i = n.first; i < n.first + n.count; ++i) fn(s.border[i]);
        } else {
            st.push_back(n.left);
            st.push_back(n.right);
        }
    }
}

struct Hit { int tri; double t, u, v; };

// Near-edge threshold of triangle f for a ray along d, in barycentric units:
// an FP32 ray's crossing of the triangle's plane is off by its across-ray
// error divided by the incidence cosine, so grazing rays get a wider margin.
double edge_tie(const Scn& s, int f, const V3d& d) {
    double c = std::fabs(dot(normalize(s.face_n(f)), normalize(d)));
    return s.tie_bary[f] / std::max(c, kTieCos);
}

// Closest hit in (tmin, tmax); ties in t go to the smaller triangle id.
Hit closest(const Scn& s, const V3d& o, const V3d& d, double tmin, double tmax, Unit& U) {
    U.rays++;
    Hit best{-1, tmax, 0, 0};
    struct Near { int f; double t; bool hit; };
    std::vector<Near> nears;
    for_candidates(s, o, d, tmin, tmax, [&](int f) {
        TriHit h = tri_test(s, f, o, d, tmin, tmax);
        if (!h.valid) return;
        if (h.ok && (h.t < best.t || (h.t == best.t && f < best.tri))) best = {f, h.t, h.u, h.v};
        bool near_edge = std::fabs(h.m) < edge_tie(s, f, d);
        bool in_range = h.t > tmin * (1 - kTieT) - 1e-300 && h.t < tmax * (1 + kTieT);
        if ((near_edge && in_range) || h.ok) nears.push_back({f, h.t, h.ok});
    });
    double tb = best.tri >= 0 ? best.t : tmax;
    for (const Near& n : nears) {
        if (n.f == best.tri) continue;
        if (n.t <= tb * (1 + kTieT) + 1e-300) {
            if (!n.hit) TIE(U, 0);                                      // barely missed, in front
            else if (std::fabs(n.t - tb) <= kTieT * tb) TIE(U, 1);      // two hits at ~equal t
        }
    }
    if (best.tri >= 0) {
        double m = std::min(std::min(best.u, best.v), 1 - best.u - best.v);
        if (m < edge_tie(s, best.tri, d)) TIE(U, 2);
        if (std::fabs(best.t - tmin) <= kTieT * std::max(best.t, tmin)) TIE(U, 3);
        V3d n = normalize(s.face_n(best.tri));
        if (std::fabs(dot(n, normalize(d))) < kTieCos) TIE(U, 4);
    }
    return best;
}

// Any hit in (tmin, tmax).
bool occluded(const Scn& s, const V3d& o, const V3d& d, double tmin, double tmax, Unit& U) {
    U.rays++;
    bool any = false;
    for_candidates(s, o, d, tmin, tmax, [&](int f) {
        TriHit h = tri_test(s, f, o, d, tmin, tmax);
        if (!h.valid) return;
        if (h.ok) any = true;
        bool in_range = h.t > tmin * (1 - kTieT) && h.t < tmax * (1 + kTieT);
        double tie = edge_tie(s, f, d);
        if (in_range && std::fabs(h.m) < tie) TIE(U, 5);
        if (h.ok || std::fabs(h.m) < tie) {
            if (std::fabs(h.t - tmin) <= kTieT * std::max(h.t, tmin) || std::fabs(h.t - tmax) <= kTieT * tmax)
                TIE(U, 6);
        }
    });
    return any;
}

// ---------------------------------------------------------------------------
// Camera: pinhole look-at; screen in pixels, y down; ray direction
// d = f + ndc_x*aspect*tan(fov/2)*r + ndc_y*tan(fov/2)*u, so d.f = 1 and the
// ray parameter equals camera-space depth (near clip = t_min of camera rays).
// ---------------------------------------------------------------------------
template <class S> struct Cam {
    V3<S> c, f, r, u;
    double th, asp, W, H, near;
};

template <class S> Cam<S> make_cam(const V3<S>& c, const V3<S>& l, const V3<S>& up, const orc_camera& oc) {
    Cam<S> k;
    k.c = c;
    k.f = normalize(l - c);
    k.r = normalize(cross(k.f, up));
    k.u = cross(k.r, k.f);
    k.th = std::tan((double)oc.fov_y_deg * kPi / 360.0);
    k.W = oc.width; k.H = oc.height;
    k.asp = k.W / k.H;
    k.near = oc.near_clip;
    return k;
}

template <class S> V3<S> cam_dir(const Cam<S>& k, double sx, double sy) {
    double nx = 2.0 * sx / k.W - 1.0, ny = 1.0 - 2.0 * sy / k.H;
    return k.f + k.r * (nx * k.asp * k.th) + k.u * (ny * k.th);
}

template <class S> void project(const Cam<S>& k, const V3<S>& P, S& sx, S& sy) {
    V3<S> q = P - k.c;
    S z = dot(q, k.f), xc = dot(q, k.r), yc = dot(q, k.u);
    sx = (1.0 + xc / (z * (k.asp * k.th))) * (k.W / 2);
    sy = (1.0 - yc / (z * k.th)) * (k.H / 2);
}

// ---------------------------------------------------------------------------
// Edge discontinuity test from a viewpoint q (silhouette: the two faces lie
// on opposite sides of q).
// ---------------------------------------------------------------------------
bool disc_from(const Scn& s, const Edge& e, const V3d& q, bool* tie) {
    if (e.kind == 1) return true;
    if (e.kind == 0) return false;
    V3d pa = s.p(e.va);
    V3d w = q - pa;
    V3d n0 = s.face_n(e.f0), n1 = s.face_n(e.f1);
    double s0 = dot(n0, w), s1 = dot(n1, w);
    double wl = length(w);
    if (tie && (std::fabs(s0) < kTieSign * length(n0) * wl || std::fabs(s1) < kTieSign * length(n1) * wl)) {
        *tie = true;
        __atomic_add_fetch(&g_reason[14], 1, __ATOMIC_RELAXED);
    }
    return (s0 > 0) != (s1 > 0);
}

// ---------------------------------------------------------------------------
// Primary edge table (per view): candidates, near clip, projection, screen
// clip, screen length, FP64 CDF (Primary Visibility; edge chosen with
// probability proportional to clipped screen length, point uniform on it).
// ---------------------------------------------------------------------------
struct PEdge { double A[2], B[2], Ac[2], Bc[2], Aa[2], Ba[2], len; };  // Aa, Ba: alpha points

struct View {
    Cam<double> cam;
    int x0, y0, x1, y1;
    std::vector<PEdge> pe;
    std::vector<double> pcdf;
    double psum = 0;
    bool tie = false;
    // proposal mixture of the primary edge choice: P(e) = (1 - mix) len_e / psum + mix q_e
    std::vector<double> mprob, mcdf;
};

// Window clip of the screen segment A + l (B - A), l in [t0, t1].
bool clip_segment(double A[2], double B[2], double t0, double t1, double x0, double y0, double x1, double y1,
                  double out0[2], double out1[2]) {
    double dx = B[0] - A[0], dy = B[1] - A[1];
    double p[4] = {-dx, dx, -dy, dy}, qv[4] = {A[0] - x0, x1 - A[0], A[1] - y0, y1 - A[1]};
    for (int i = 0; i < 4; ++i) {
        if (p[i] == 0) {
            if (qv[i] < 0) return false;
        } else {
            double r = qv[i] / p[i];
            if (p[i] < 0) { if (r > t1) return false; if (r > t0) t0 = r; }
            else { if (r < t0) return false; if (r < t1) t1 = r; }
        }
    }
    out0[0] = A[0] + t0 * dx; out0[1] = A[1] + t0 * dy;
    out1[0] = A[0] + t1 * dx; out1[1] = A[1] + t1 * dy;
    return true;
}

// Near-clipped endpoints of an edge (camera-space depth >= near): the part of
// the edge that can be sampled on screen.
template <class S> bool near_clip(const Cam<S>& k, V3<S> a, V3<S> b, V3<S>& ao, V3<S>& bo) {
    S za = dot(a - k.c, k.f), zb = dot(b - k.c, k.f);
    if (val(za) < k.near && val(zb) < k.near) return false;
    ao = a; bo = b;
    if (val(za) < k.near) ao = a + (b - a) * ((k.near - za) / (zb - za));
    if (val(zb) < k.near) bo = b + (a - b) * ((k.near - zb) / (za - zb));
    return true;
}

// Two points of the edge whose projections define the edge equation alpha
// (eq. edge_equation). The projected line, and hence the boundary term
// d alpha/d Phi / |grad_xy alpha|, is the same for any two points of the edge
// in front of the camera; an endpoint behind the near plane is replaced by the
// edge point at depth max(near, half the other endpoint's depth), which keeps
// the projection well conditioned (a point at depth `near` projects far off
// screen with a 1/near^2 Jacobian).
template <class S> void alpha_points(const Cam<S>& k, V3<S> a, V3<S> b, V3<S>& ao, V3<S>& bo) {
    S za = dot(a - k.c, k.f), zb = dot(b - k.c, k.f);
    ao = a; bo = b;
    if (val(za) < k.near) {
        S zd = val(zb) * 0.5 > k.near ? zb * 0.5 : cst<S>(k.near);
        ao = a + (b - a) * ((zd - za) / (zb - za));
    }
    if (val(zb) < k.near) {
        S zd = val(za) * 0.5 > k.near ? za * 0.5 : cst<S>(k.near);
        bo = b + (a - b) * ((zd - zb) / (za - zb));
    }
}

double cam_param(const orc_camera& oc, int k) {
    if (oc.params64) return oc.params64[k];
    const float* f[3] = {oc.position, oc.look_at, oc.up};
    return f[k / 3][k % 3];
}

void build_view(const Scn& s, const orc_camera& oc, View& vw) {
    V3d c{cam_param(oc, 0), cam_param(oc, 1), cam_param(oc, 2)};
    V3d l{cam_param(oc, 3), cam_param(oc, 4), cam_param(oc, 5)};
    V3d up{cam_param(oc, 6), cam_param(oc, 7), cam_param(oc, 8)};
    vw.cam = make_cam<double>(c, l, up, oc);
    vw.x0 = oc.win_x0; vw.y0 = oc.win_y0; vw.x1 = oc.win_x1; vw.y1 = oc.win_y1;
    vw.pe.assign(s.edges.size(), PEdge{});
    vw.pcdf.assign(s.edges.size(), 0.0);
    double acc = 0;
    for (size_t i = 0; i < s.edges.size(); ++i) {
        const Edge& e = s.edges[i];
        PEdge& p = vw.pe[i];
        p.len = 0;
        if (disc_from(s, e, c, &vw.tie)) {
            V3d a, b;
            if (near_clip(vw.cam, s.p(e.va), s.p(e.vb), a, b)) {
                // the visible (near-clipped) segment, as a parameter range on the
                // line through the projections of the alpha points
                project(vw.cam, a, p.A[0], p.A[1]);
                project(vw.cam, b, p.B[0], p.B[1]);
                V3d aa, ba;
                alpha_points(vw.cam, s.p(e.va), s.p(e.vb), aa, ba);
                project(vw.cam, aa, p.Aa[0], p.Aa[1]);
                project(vw.cam, ba, p.Ba[0], p.Ba[1]);
                double dx = p.Ba[0] - p.Aa[0], dy = p.Ba[1] - p.Aa[1], dd = dx * dx + dy * dy;
                double l0 = ((p.A[0] - p.Aa[0]) * dx + (p.A[1] - p.Aa[1]) * dy) / dd;
                double l1 = ((p.B[0] - p.Aa[0]) * dx + (p.B[1] - p.Aa[1]) * dy) / dd;
                if (dd > 0 && clip_segment(p.Aa, p.Ba, l0, l1, vw.x0, vw.y0, vw.x1, vw.y1, p.Ac, p.Bc))
                    p.len = std::hypot(p.Bc[0] - p.Ac[0], p.Bc[1] - p.Ac[1]);
            }
        }
        acc += p.len;
        vw.pcdf[i] = acc;
    }
    vw.psum = acc;
    if (acc > 0) for (double& x : vw.pcdf) x /= acc;
}

// Mixture of the screen-length edge pdf with a given distribution q over all
// edges (the learned proposal): weights, running sum, normalised CDF.
void build_view_mix(const View& vwc, const double* q, double mix, View& vw) {
    size_t E = vwc.pe.size();
    vw.mprob.assign(E, 0.0);
    vw.mcdf.assign(E, 0.0);
    if (!(vwc.psum > 0)) return;
    double acc = 0;
    for (size_t i = 0; i < E; ++i) {
        vw.mprob[i] = (1.0 - mix) * (vwc.pe[i].len / vwc.psum) + mix * q[i];
        acc += vw.mprob[i];
        vw.mcdf[i] = acc;
    }
    for (size_t i = 0; i < E; ++i) { vw.mprob[i] /= acc; vw.mcdf[i] /= acc; }
}

// Index of the first CDF entry greater than u; flags near ties.
int cdf_pick(const std::vector<double>& cdf, double u, Unit& U) {
    int i = (int)(std::upper_bound(cdf.begin(), cdf.end(), u) - cdf.begin());
    if (i >= (int)cdf.size()) i = (int)cdf.size() - 1;
    if (std::fabs(cdf[i] - u) < kTieCdf) TIE(U, 7);
    if (i > 0 && std::fabs(cdf[i - 1] - u) < kTieCdf) TIE(U, 7);
    return i;
}

// ---------------------------------------------------------------------------
// Edge hierarchy (Importance Sampling the Edges, Edge selection): two binary
// radix trees over edge midpoints (Morton order). H1 holds the edges that are
// discontinuities from every viewpoint and the silhouettes w.r.t. the camera;
// H2 the remaining smooth edges, whose nodes also bound the two face planes in
// Hough space (foot points d*n, camera at the origin) for the v-sphere test.
// ---------------------------------------------------------------------------
struct ENode {
    double lo[3], hi[3], len;
    double hlo[2][3], hhi[2][3];
    int left = -1, right = -1, edge = -1;
};

struct ETree {
    std::vector<ENode> nodes;
    int root[2] = {-1, -1};
    V3d cam;
    int max_depth = 0;
    std::vector<int> parent;    // per node (-1 at the two roots)
    std::vector<int> leaf_of;   // per edge: its leaf node, -1 if in neither hierarchy
    std::vector<int> which;     // per node: 0 = H1, 1 = H2
};

uint32_t spread10(uint32_t x) {
    uint32_t r = 0;
    for (int b = 0; b < 10; ++b) r |= ((x >> b) & 1u) << (3 * b);
    return r;
}

#pragma GCC push_options
#pragma GCC optimize("fp-contract=off")
uint32_t quantize(double c, double lo, double hi) {
    if (!(hi > lo)) return 0;
    double q = (c - lo) / (hi - lo);
    q = q * 1024.0;
    double f = std::floor(q);
    if (f < 0) f = 0;
    if (f > 1023) f = 1023;
    return (uint32_t)f;
}
#pragma GCC pop_options

int build_tree_rec(ETree& t, const std::vector<uint64_t>& keys, const std::vector<int>& ids, int lo, int hi,
                   const std::vector<ENode>& leaves, int depth) {
    t.max_depth = std::max(t.max_depth, depth);
    if (lo == hi) {
        t.nodes.push_back(leaves[lo]);
        return (int)t.nodes.size() - 1;
    }
    // Split at the highest bit where the first and last keys differ.
    uint64_t x = keys[lo] ^ keys[hi];
    int bit = 63;
    while (!((x >> bit) & 1ull)) --bit;
    int split = lo;
    for (int i = lo; i < hi; ++i)
        if (((keys[i] ^ keys[lo]) >> bit) == 0) split = i;
    int me = (int)t.nodes.size();
    t.nodes.push_back(ENode{});
    int l = build_tree_rec(t, keys, ids, lo, split, leaves, depth + 1);
    int r = build_tree_rec(t, keys, ids, split + 1, hi, leaves, depth + 1);
    ENode& n = t.nodes[me];
    const ENode& a = t.nodes[l];
    const ENode& b = t.nodes[r];
    for (int k = 0; k < 3; ++k) {
        n.lo[k] = std::min(a.lo[k], b.lo[k]); n.hi[k] = std::max(a.hi[k], b.hi[k]);
        for (int f = 0; f < 2; ++f) {
            n.hlo[f][k] = std::min(a.hlo[f][k], b.hlo[f][k]);
            n.hhi[f][k] = std::max(a.hhi[f][k], b.hhi[f][k]);
        }
    }
    n.len = a.len + b.len;
    n.left = l; n.right = r;
    return me;
}

int build_etree(const Scn& s, const V3d& cam, ETree& t) {
    t.nodes.clear();
    t.cam = cam;
    t.max_depth = 0;
    for (int h = 0; h < 2; ++h) {
        std::vector<int> ids;
        for (int i = 0; i < (int)s.edges.size(); ++i) {
            const Edge& e = s.edges[i];
            if (e.kind == 0) continue;
            bool h1 = e.kind == 1 || disc_from(s, e, cam, nullptr);
            if ((h == 0) == h1) ids.push_back(i);
        }
        if (ids.empty()) { t.root[h] = -1; continue; }
        // Morton codes of midpoints, quantised in FP64 from the FP32 inputs.
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        std::vector<double> mid(3 * ids.size());
        for (size_t j = 0; j < ids.size(); ++j) {
            const Edge& e = s.edges[ids[j]];
            for (int k = 0; k < 3; ++k) {
                double m = (s.P[3 * e.va + k] + s.P[3 * e.vb + k]) / 2.0;
                mid[3 * j + k] = m;
                lo[k] = std::min(lo[k], m); hi[k] = std::max(hi[k], m);
            }
        }
        std::vector<std::pair<uint32_t, int>> ord(ids.size());
        for (size_t j = 0; j < ids.size(); ++j) {
            uint32_t q[3];
            for (int k = 0; k < 3; ++k) q[k] = quantize(mid[3 * j + k], lo[k], hi[k]);
            uint32_t code = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
            ord[j] = {code, ids[j]};
        }
        std::sort(ord.begin(), ord.end());
        std::vector<uint64_t> keys(ord.size());
        std::vector<int> sid(ord.size());
        std::vector<ENode> leaves(ord.size());
        for (size_t j = 0; j < ord.size(); ++j) {
            keys[j] = ((uint64_t)ord[j].first << 32) | (uint64_t)j;   // ties broken by sorted position
            sid[j] = ord[j].second;
            const Edge& e = s.edges[ord[j].second];
            ENode& n = leaves[j];
            V3d a = s.p(e.va), b = s.p(e.vb);
            for (int k = 0; k < 3; ++k) {
                n.lo[k] = std::min(comp(a, k), comp(b, k));
                n.hi[k] = std::max(comp(a, k), comp(b, k));
            }
            n.len = length(b - a);
            n.edge = ord[j].second;
            for (int f = 0; f < 2; ++f) {
                V3d h3{0, 0, 0};
                if (h == 1) {
                    int face = f == 0 ? e.f0 : e.f1;
                    V3d nn = normalize(s.face_n(face));
                    double dd = dot(nn, s.p(s.I[3 * face]) - cam);
                    h3 = nn * dd;
                }
                for (int k = 0; k < 3; ++k) n.hlo[f][k] = n.hhi[f][k] = comp(h3, k);
            }
        }
        t.root[h] = build_tree_rec(t, keys, sid, 0, (int)ord.size() - 1, leaves, 0);
    }
    t.parent.assign(t.nodes.size(), -1);
    t.which.assign(t.nodes.size(), 0);
    t.leaf_of.assign(s.edges.size(), -1);
    for (int h = 0; h < 2; ++h) {
        if (t.root[h] < 0) continue;
        std::vector<int> todo{t.root[h]};
        while (!todo.empty()) {
            int n = todo.back();
            todo.pop_back();
            t.which[n] = h;
            const ENode& nd = t.nodes[n];
            if (nd.edge >= 0) { t.leaf_of[nd.edge] = n; continue; }
            t.parent[nd.left] = n; t.parent[nd.right] = n;
            todo.push_back(nd.left); todo.push_back(nd.right);
        }
    }
    return t.max_depth + 1 > kMaxLevels ? ORC_EDEPTH : ORC_OK;
}

bool in_box(const double lo[3], const double hi[3], const V3d& p, Unit* U, double scale) {
    const double pv[3] = {p.x, p.y, p.z};
    const double pad = kInsidePad * scale;
    bool in = true;
    for (int k = 0; k < 3; ++k) {
        double l = lo[k] - pad, h = hi[k] + pad;
        if (pv[k] < l || pv[k] > h) in = false;
        if (U && (std::fabs(pv[k] - l) < kTieBox * scale || std::fabs(pv[k] - h) < kTieBox * scale)) TIE(*U, 8);
    }
    return in;
}

// Conservative bound of the clamped cosine between n and directions from p to
// the box (Walter et al. 2005's cone-box bound in the frame of n).
double cos_bound(const double lo[3], const double hi[3], const V3d& p, const V3d& n, Unit* U, double scale) {
    V3d t1, t2;
    onb(n, t1, t2);
    double xl = 1e300, xh = -1e300, yl = 1e300, yh = -1e300, zh = -1e300;
    for (int c = 0; c < 8; ++c) {
        V3d q{(c & 1 ? hi[0] : lo[0]) - p.x, (c & 2 ? hi[1] : lo[1]) - p.y, (c & 4 ? hi[2] : lo[2]) - p.z};
        double x = dot(t1, q), y = dot(t2, q), z = dot(n, q);
        xl = std::min(xl, x); xh = std::max(xh, x);
        yl = std::min(yl, y); yh = std::max(yh, y);
        zh = std::max(zh, z);
    }
    double dx = (xl <= 0 && xh >= 0) ? 0 : std::min(std::fabs(xl), std::fabs(xh));
    double dy = (yl <= 0 && yh >= 0) ? 0 : std::min(std::fabs(yl), std::fabs(yh));
    double dxy2 = dx * dx + dy * dy;
    double hz = kHorizon * scale;
    if (U && dxy2 == 0 && std::fabs(zh - hz) < kTieBox * scale) TIE(*U, 9);
    if (zh <= hz) return 0;
    if (dxy2 == 0) return 1;
    return zh / std::sqrt(dxy2 + zh * zh);
}

// v-sphere test: sphere with diameter [camera, p]; a face plane flips between
// the camera and p iff its Hough foot point lies inside the sphere.
bool vsphere_prune(const ENode& n, const V3d& pc /* p - camera */, Unit* U) {
    V3d s = pc * 0.5;
    double r2 = dot(pc, pc) * 0.25;
    bool out[2], in[2];
    for (int f = 0; f < 2; ++f) {
        double d2 = 0, far2 = 0;
        const double sv[3] = {s.x, s.y, s.z};
        for (int k = 0; k < 3; ++k) {
            double lo = n.hlo[f][k], hi = n.hhi[f][k];
            double d = sv[k] < lo ? lo - sv[k] : (sv[k] > hi ? sv[k] - hi : 0);
            d2 += d * d;
            double fa = std::max(std::fabs(lo - sv[k]), std::fabs(hi - sv[k]));
            far2 += fa * fa;
        }
        double ro = r2 * (1 + kVsphereMargin), ri = r2 * (1 - kVsphereMargin);
        out[f] = d2 > ro;
        in[f] = far2 < ri;
        if (U && (std::fabs(d2 - ro) < kTieBox * r2 || std::fabs(far2 - ri) < kTieBox * r2)) TIE(*U, 10);
    }
    return (out[0] && out[1]) || (in[0] && in[1]);
}

struct TreeQuery {
    const Scn* s;
    const ETree* t;
    V3d p, n;
    int tri;      // triangle the shading point lies on (-1: none)
};

// Importance of a child node (thesis: total length x inverse distance to the
// box centre x cosine bound; zero without a possible silhouette; one for both
// children when the point lies inside the parent's box).
double importance(const TreeQuery& q, const ENode& c, bool h2, const double plo[3], const double phi[3], Unit* U) {
    double scale = q.s->diag;
    // Edges of the shading point's own triangle contribute nothing (the point
    // lies in their face plane); they get zero importance.
    if (c.edge >= 0 && q.tri >= 0) {
        const Edge& e = q.s->edges[c.edge];
        if (e.f0 == q.tri || e.f1 == q.tri) return 0;
    }
    if (h2 && vsphere_prune(c, q.p - q.t->cam, U)) return 0;
    double b = cos_bound(c.lo, c.hi, q.p, q.n, U, scale);
    if (b <= 0) return 0;
    if (in_box(plo, phi, q.p, U, scale)) return 1;
    V3d ctr{(c.lo[0] + c.hi[0]) / 2, (c.lo[1] + c.hi[1]) / 2, (c.lo[2] + c.hi[2]) / 2};
    return c.len * b / length(ctr - q.p);
}

void root_box(const ETree& t, double lo[3], double hi[3]) {
    for (int k = 0; k < 3; ++k) { lo[k] = 1e300; hi[k] = -1e300; }
    for (int h = 0; h < 2; ++h)
        if (t.root[h] >= 0)
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], t.nodes[t.root[h]].lo[k]);
                hi[k] = std::max(hi[k], t.nodes[t.root[h]].hi[k]);
            }
}

// Single descent with one uniform per level. Returns the edge or -1.
template <class LevelU>
int tree_sample(const TreeQuery& q, double u_root, LevelU&& ulev, double& pdf, Unit* U, bool dbg = false) {
    const ETree& t = *q.t;
    double lo[3], hi[3];
    root_box(t, lo, hi);
    double w[2] = {0, 0};
    for (int h = 0; h < 2; ++h)
        if (t.root[h] >= 0) w[h] = importance(q, t.nodes[t.root[h]], h == 1, lo, hi, U);
    if (w[0] + w[1] <= 0) return -1;
    double p0 = w[0] / (w[0] + w[1]);
    if (U && std::fabs(u_root - p0) < kTieU) TIE(*U, 11);
    int h = u_root < p0 ? 0 : 1;
    pdf = h == 0 ? p0 : 1 - p0;
    if (h == 1) pdf = w[1] / (w[0] + w[1]);
    int node = t.root[h];
    int level = 0;
    while (t.nodes[node].edge < 0) {
        const ENode& n = t.nodes[node];
        double wl = importance(q, t.nodes[n.left], h == 1, n.lo, n.hi, U);
        double wr = importance(q, t.nodes[n.right], h == 1, n.lo, n.hi, U);
        if (wl + wr <= 0) return -1;
        double pl = wl / (wl + wr);
        double u = ulev(level);
        if (U && std::fabs(u - pl) < kTieU) TIE(*U, 11);
        if (dbg) std::fprintf(stderr, "  level %d w0 %.9g w1 %.9g u %.9g side %d\n", level, wl, wr, u, u < pl ? 0 : 1);
        if (u < pl) { pdf *= pl; node = n.left; }
        else { pdf *= wr / (wl + wr); node = n.right; }
        ++level;
    }
    return t.nodes[node].edge;
}

void tree_enumerate(const TreeQuery& q, int node, bool h2, double prob, std::vector<double>& pdf, double& fail) {
    const ETree& t = *q.t;
    const ENode& n = t.nodes[node];
    if (n.edge >= 0) { pdf[n.edge] += prob; return; }
    double wl = importance(q, t.nodes[n.left], h2, n.lo, n.hi, nullptr);
    double wr = importance(q, t.nodes[n.right], h2, n.lo, n.hi, nullptr);
    if (wl + wr <= 0) { fail += prob; return; }
    if (wl > 0) tree_enumerate(q, n.left, h2, prob * (wl / (wl + wr)), pdf, fail);
    if (wr > 0) tree_enumerate(q, n.right, h2, prob * (wr / (wl + wr)), pdf, fail);
}

// Probability that the descent of tree_sample ends at edge e: the product of
// the branch probabilities along the unique root-to-leaf path of e (root choice
// included), with the same near-tie flags as a descent along that path.
double tree_pdf_edge(const TreeQuery& q, int e, Unit* U) {
    const ETree& t = *q.t;
    int leaf = t.leaf_of[e];
    if (leaf < 0) return 0.0;
    std::vector<int> path;
    for (int n = leaf; n >= 0; n = t.parent[n]) path.push_back(n);
    std::reverse(path.begin(), path.end());
    int h = t.which[leaf];
    double lo[3], hi[3];
    root_box(t, lo, hi);
    double w[2] = {0, 0};
    for (int r = 0; r < 2; ++r)
        if (t.root[r] >= 0) w[r] = importance(q, t.nodes[t.root[r]], r == 1, lo, hi, U);
    if (w[0] + w[1] <= 0) return 0.0;
    double pdf = w[h] / (w[0] + w[1]);
    for (size_t i = 0; i + 1 < path.size(); ++i) {
        const ENode& n = t.nodes[path[i]];
        double wl = importance(q, t.nodes[n.left], h == 1, n.lo, n.hi, U);
        double wr = importance(q, t.nodes[n.right], h == 1, n.lo, n.hi, U);
        if (wl + wr <= 0) return 0.0;
        pdf *= (path[i + 1] == n.left ? wl : wr) / (wl + wr);
    }
    return pdf;
}

// Stratified multi-sample descent with weighted reservoir selection (Ch. 5,
// Edge selection: a number of samples start at the root and are distributed
// to the two children of every node in proportion to their importance; one
// edge is finally kept by weighted reservoir sampling with the leaves'
// importance as weight).
//
// M samples enter at the root. The n samples that reach a node are divided
// between its children: child 0 receives floor(n p0 + xi) of them (p0 its
// share of the two importances, xi uniform), so each child receives n p_c in
// expectation and a leaf e receives M pdf_e, pdf_e being the probability that
// one descent (tree_sample) ends at e. The leaves reached form the candidates,
// visited depth first with child 0 before child 1; a leaf holding n_e samples
// has weight n_e imp_e / pdf_e (imp_e: its importance at its parent), and one
// candidate z is kept by weighted reservoir sampling. In place of 1 / pdf,
// the kept edge carries W / (M imp_z), W the total weight: resampled
// importance sampling, whose expectation is sum_e E[n_e] f(e) / (M pdf_e) =
// sum_e f(e). Uniforms: next_u() is called once per split and once per
// candidate, in visiting order. Returns -1 when no leaf was reached.
template <class NextU>
int tree_select(const TreeQuery& q, int M, NextU&& next_u, double& weight, Unit* U) {
    const ETree& t = *q.t;
    double W = 0, impz = 0;
    int z = -1;
    auto split = [&](int n, double wl, double wr) {
        double p0 = wl / (wl + wr);
        double x = n * p0 + next_u();
        if (U && p0 > 0 && p0 < 1 && std::fabs(x - std::round(x)) < kTieU * n) TIE(*U, 17);
        return std::min(std::max((int)std::floor(x), 0), n);
    };
    std::function<void(int, bool, int, double, double)> child = [&](int node, bool h2, int n, double pdf,
                                                                      double imp) {
        if (n == 0) return;
        const ENode& nd = t.nodes[node];
        if (nd.edge >= 0) {
            double om = n * imp / pdf;
            W += om;
            double r = om / W;
            double u = next_u();
            if (U && std::fabs(u - r) < kTieRes * r) TIE(*U, 18);
            if (u < r) { z = nd.edge; impz = imp; }
            return;
        }
        double wl = importance(q, t.nodes[nd.left], h2, nd.lo, nd.hi, U);
        double wr = importance(q, t.nodes[nd.right], h2, nd.lo, nd.hi, U);
        if (wl + wr <= 0) return;
        int n0 = split(n, wl, wr);
        child(nd.left, h2, n0, pdf * (wl / (wl + wr)), wl);
        child(nd.right, h2, n - n0, pdf * (wr / (wl + wr)), wr);
    };
    double lo[3], hi[3];
    root_box(t, lo, hi);
    double w[2] = {0, 0};
    for (int h = 0; h < 2; ++h)
        if (t.root[h] >= 0) w[h] = importance(q, t.nodes[t.root[h]], h == 1, lo, hi, U);
    if (w[0] + w[1] <= 0) return -1;
    int n0 = split(M, w[0], w[1]);
    if (t.root[0] >= 0) child(t.root[0], false, n0, w[0] / (w[0] + w[1]), w[0]);
    if (t.root[1] >= 0) child(t.root[1], true, M - n0, w[1] / (w[0] + w[1]), w[1]);
    if (z < 0) return -1;
    weight = W / (M * impz);
    return z;
}

// ---------------------------------------------------------------------------
// Differentiation environment: vertex positions, albedos and camera as
// tape leaves (created on first use within a unit).
// ---------------------------------------------------------------------------
struct Leaves {
    std::unordered_map<int, std::array<int32_t, 3>> v;
    std::unordered_map<int, int32_t> a;
    int32_t cam[9];
    void clear() { v.clear(); a.clear(); }
};

template <class S> struct Env;
template <> struct Env<double> {
    const Scn* s;
    V3d P(int i) const { return s->p(i); }
    double albedo(int f) const { return s->alb[f]; }
};
template <> struct Env<D> {
    const Scn* s;
    Leaves* L;
    V3<D> P(int i) const {
        auto it = L->v.find(i);
        if (it == L->v.end()) {
            std::array<int32_t, 3> ids;
            for (int k = 0; k < 3; ++k) ids[k] = leafD(s->P[3 * i + k]).i;
            it = L->v.emplace(i, ids).first;
        }
        return {D{s->P[3 * i], it->second[0]}, D{s->P[3 * i + 1], it->second[1]}, D{s->P[3 * i + 2], it->second[2]}};
    }
    D albedo(int f) const {
        auto it = L->a.find(f);
        if (it == L->a.end()) it = L->a.emplace(f, leafD(s->alb[f]).i).first;
        return D{s->alb[f], it->second};
    }
};

template <class S> struct PathVtx {
    V3<S> x, ns;
    S rho, beta;
    int tri;
    double dx;      // first-order FP32 position error bound of x, in units of u32 (absolute)
    double kappa;   // relative sensitivity of this vertex's contributions, in units of u32
};

// First-order rounding-error model of an FP32 evaluation of the same path
// (used only to scale the parity tolerance): positions carry an absolute
// error dx, directions a relative error dw (both in units of u32). A hit at
// distance t inherits dx + t*dw; the barycentric coordinates of a hit on a
// triangle with shortest edge e are then off by dx/e, which moves an
// interpolated normal by dx*g (g = normal variation / e) and the next sampled
// direction with it.
struct Cond {
    double dx = 0, dw = 4, kmax = 0;   // kmax: accumulated sensitivity along the path
};
const double kOpsU32 = 650;   // FP32 operations budget of one contribution (tolerance floor)
const double kCondSafety = 8; // the first-order model above underestimates compounded sensitivities

double min_edge(const Scn& s, int f) {
    V3d a = s.p(s.I[3 * f]), b = s.p(s.I[3 * f + 1]), c = s.p(s.I[3 * f + 2]);
    return std::min(length(b - a), std::min(length(c - b), length(a - c)));
}

double normal_spread(const Scn& s, int f) {
    if (!s.smooth) return 0;
    V3d n0 = s.nrm(s.I[3 * f]), n1 = s.nrm(s.I[3 * f + 1]), n2 = s.nrm(s.I[3 * f + 2]);
    return std::max(length(n1 - n0), std::max(length(n2 - n1), length(n0 - n2)));
}

// Ray-plane intersection of a ray with the plane of a triangle; moves with the
// ray origin, its direction and the triangle vertices.
template <class S> V3<S> ray_plane(const V3<S>& o, const V3<S>& d, const V3<S>& p0, const V3<S>& p1, const V3<S>& p2) {
    V3<S> n = cross(p1 - p0, p2 - p0);
    S t = dot(p0 - o, n) / dot(d, n);
    return o + d * t;
}

template <class S> V3<S> shading_normal(const Scn& s, int tri, const V3<S>& x, const V3<S>& p0, const V3<S>& p1, const V3<S>& p2) {
    V3<S> e1 = p1 - p0, e2 = p2 - p0;
    V3<S> n = cross(e1, e2);
    if (!s.smooth) return normalize(n);
    V3<S> w = x - p0;
    S nn = dot(n, n);
    S b1 = dot(cross(w, e2), n) / nn;
    S b2 = dot(cross(e1, w), n) / nn;
    S b0 = 1.0 - b1 - b2;
    V3<S> N0 = lift<S>(s.nrm(s.I[3 * tri])), N1 = lift<S>(s.nrm(s.I[3 * tri + 1])), N2 = lift<S>(s.nrm(s.I[3 * tri + 2]));
    return normalize(N0 * b0 + N1 * b1 + N2 * b2);
}

double emitted(const Scn& s, int tri, bool front) {
    if (s.emi[tri] <= 0) return 0;
    return (front || s.two_sided) ? s.emi[tri] : 0;
}

// Next-event estimation at x: one light triangle by area, a point by the
// square-root warp, one shadow ray. The sampled direction is held fixed and
// its solid-angle pdf is a constant under differentiation, so only the
// albedo and the shading cosine carry derivatives.
// A ray leaving a point x of triangle `tri` along w rises t |n . w| off the
// triangle's plane at distance t. An FP32 implementation places x within a
// few ulps of that plane, so when the rise at t_min is within that error it
// may hit its own triangle or miss it: a near tie.
void departure_tie(const Scn& s, int tri, const V3d& x, const V3d& w, Unit& U) {
    double c = std::fabs(dot(normalize(s.face_n(tri)), normalize(w)));
    if (c * s.tmin < kTieDepart * std::max(1.0, length(x))) TIE(U, 16);
}

template <class S> S nee(const Env<S>& E, Unit& U, const Stream& rs, int blk, const V3<S>& x, const V3<S>& ns, const S& rho,
                         double* log, int tri) {
    const Scn& s = *E.s;
    if (s.lights.empty()) return cst<S>(0);
    if (log && U.dir_mode == 2) {
        // replay: same world direction and solid-angle factor as recorded
        if (log[4] == 0) return cst<S>(0);
        V3d wh{log[0], log[1], log[2]};
        S cp = dot(ns, lift<S>(wh));
        if (val(cp) <= 0) return cst<S>(0);
        return rho * cp * log[3];
    }
    if (log) log[4] = 0;
    double u[4];
    rs.block(blk, u);
    int li = cdf_pick(s.lcdf, u[0], U);
    int lt = s.lights[li];
    V3d a = s.p(s.I[3 * lt]), b = s.p(s.I[3 * lt + 1]), c = s.p(s.I[3 * lt + 2]);
    double su = std::sqrt(u[1]);
    V3d y = a * (1 - su) + b * (su * (1 - u[2])) + c * (su * u[2]);
    V3d xv = valv(x);
    V3d w = y - xv;
    double r2 = dot(w, w), r = std::sqrt(r2);
    V3d wh = w / r;
    V3d nl = normalize(cross(b - a, c - a));
    double cy = -dot(nl, wh);
    if (s.two_sided) cy = std::fabs(cy);
    S cp = dot(ns, lift<S>(wh));
    if (val(cp) <= 0 || cy <= 0) return cst<S>(0);
    departure_tie(s, tri, xv, wh, U);
    if (occluded(s, xv, wh, s.tmin, r * (1 - kShadowEnd), U)) return cst<S>(0);
    double k = s.emi[lt] * cy / r2 * s.atot / kPi;
    if (log) { log[0] = wh.x; log[1] = wh.y; log[2] = wh.z; log[3] = k; log[4] = 1; }
    return rho * cp * k;
}

V3d cosine_dir(const V3d& n, double u0, double u1) {
    V3d t1, t2;
    onb(n, t1, t2);
    double r = std::sqrt(u0), ph = 2 * kPi * u1;
    return t1 * (r * std::cos(ph)) + t2 * (r * std::sin(ph)) + n * std::sqrt(1 - u0);
}

// Radiance along a ray (O4): emission at the first hit; then for path
// vertices 1..budget, next-event estimation, and cosine-sampled continuation
// between them (emission found by continuation rays is not added: NEE only).
// camera = true: t_min = near clip, misses return the background radiance.
template <class S>
S radiance_impl(const Env<S>& E, Unit& U, const Stream& rs, int base, const V3<S>& o, const V3<S>& d0, double tmin,
                bool camera, int budget, std::vector<PathVtx<S>>* log, Cond* cond = nullptr) {
    const Scn& s = *E.s;
    V3d dv = valv(d0);
    Hit h = closest(s, valv(o), dv, tmin, 1e300, U);
    if (h.tri < 0) return cst<S>(camera ? s.bg : 0.0);
    int tri = h.tri;
    V3<S> p0 = E.P(s.I[3 * tri]), p1 = E.P(s.I[3 * tri + 1]), p2 = E.P(s.I[3 * tri + 2]);
    V3<S> x = ray_plane(o, d0, p0, p1, p2);
    bool front = dot(dv, s.face_n(tri)) < 0;
    S L = cst<S>(emitted(s, tri, front));
    S beta = cst<S>(1.0);
    double seg = h.t * length(dv);
    for (int k = 1; k <= budget; ++k) {
        V3<S> ns = shading_normal(s, tri, x, p0, p1, p2);
        if (!front) ns = -ns;
        S rho = E.albedo(tri);
        if (val(rho) == 0) break;
        double kap = 0, dxv = 0;
        if (cond) {
            // incidence cosine: errors across the ray are stretched by 1/c on the
            // surface, and the ray-plane adjoint carries t/(d.n)
            double c = std::max(std::fabs(dot(normalize(dv), normalize(s.face_n(tri)))), 1e-6);
            cond->dx = (cond->dx + seg * cond->dw) / c + 4 * length(valv(x));
            double e = min_edge(s, tri);
            double dn = 4 + cond->dx * normal_spread(s, tri) / e;
            // adjoints flowing back to earlier vertices pass through every
            // ray-plane intersection on the way: sensitivities add up
            kap = cond->kmax + 4 + cond->dx / e + dn + cond->dw / c;
            cond->kmax = kap;
            cond->dw = 8 + dn;
            dxv = cond->dx;
        }
        if (log) log->push_back(PathVtx<S>{x, ns, rho, beta, tri, dxv, kap});
        double* dl = (log && U.dir_mode && k <= 6) ? U.dir + 10 * (k - 1) : nullptr;
        L = L + beta * nee(E, U, rs, base + 2 * k - 1, x, ns, rho, dl, tri);
        if (k == budget) break;
        double u[4];
        rs.block(base + 2 * k, u);
        V3d nsv = valv(ns);
        V3d w = cosine_dir(nsv, u[0], u[1]);
        double cv = dot(nsv, w);
        if (dl && U.dir_mode == 2) { w = V3d{dl[5], dl[6], dl[7]}; cv = dl[8]; }
        if (dl && U.dir_mode == 1) { dl[5] = w.x; dl[6] = w.y; dl[7] = w.z; dl[8] = cv; }
        if (cv <= 0) break;
        departure_tie(s, tri, valv(x), w, U);
        Hit h2 = closest(s, valv(x), w, s.tmin, 1e300, U);
        if (h2.tri < 0) break;
        // Continuation weight f*cos/pdf with the pdf held constant.
        beta = beta * (rho * dot(ns, lift<S>(w)) / cv);
        seg = h2.t;
        tri = h2.tri;
        p0 = E.P(s.I[3 * tri]); p1 = E.P(s.I[3 * tri + 1]); p2 = E.P(s.I[3 * tri + 2]);
        x = ray_plane(x, lift<S>(w), p0, p1, p2);
        front = dot(w, s.face_n(tri)) < 0;
        dv = w;
    }
    return L;
}

// Geometry buffers (Results, G-buffer / AOV outputs): one channel of the
// first camera hit: 1-3 world position, 4-6 shading normal facing the ray,
// 7 albedo; 0 on a miss. `cond` gets the first-vertex rounding model of
// radiance_impl.
template <class S>
S aov_impl(const Env<S>& E, Unit& U, int aov, const V3<S>& o, const V3<S>& d0, double tmin, Cond* cond) {
    const Scn& s = *E.s;
    V3d dv = valv(d0);
    Hit h = closest(s, valv(o), dv, tmin, 1e300, U);
    if (h.tri < 0) return cst<S>(0.0);
    int tri = h.tri;
    V3<S> p0 = E.P(s.I[3 * tri]), p1 = E.P(s.I[3 * tri + 1]), p2 = E.P(s.I[3 * tri + 2]);
    V3<S> x = ray_plane(o, d0, p0, p1, p2);
    if (cond) {
        double c = std::max(std::fabs(dot(normalize(dv), normalize(s.face_n(tri)))), 1e-6);
        cond->dx = (cond->dx + h.t * length(dv) * cond->dw) / c + 4 * length(valv(x));
        double e = min_edge(s, tri);
        double dn = 4 + cond->dx * normal_spread(s, tri) / e;
        cond->kmax = cond->kmax + 4 + cond->dx / e + dn + cond->dw / c;
    }
    if (aov <= 3) return aov == 1 ? x.x : (aov == 2 ? x.y : x.z);
    if (aov <= 6) {
        V3<S> ns = shading_normal(s, tri, x, p0, p1, p2);
        if (!(dot(dv, s.face_n(tri)) < 0)) ns = -ns;
        return aov == 4 ? ns.x : (aov == 5 ? ns.y : ns.z);
    }
    return E.albedo(tri);
}

// ---------------------------------------------------------------------------
// Point on a secondary edge drawn in proportion to the clamped cosine (Ch. 5,
// Importance sampling on an edge: the thesis samples an edge point by the
// shading lobe integrated along the edge; for a Lambertian surface the lobe is
// the clamped cosine itself).
//
// Seen from p the edge is a great-circle arc of directions: w(phi) = cos(phi)
// a + sin(phi) b', phi in [0, Phi], a toward v0, b' the unit vector in the
// arc's plane orthogonal to a, Phi the angle between the directions to v0 and
// v1. Along it n . w(phi) = R cos(phi - phi0), so the integral of its positive
// part over [lo, phi] is R (sin(phi - phi0) - sin(lo - phi0)), with [lo, hi]
// the part of [0, Phi] where the cosine is positive; the inverse of its
// normalised integral is an arcsine. The drawn direction is mapped to the edge
// parameter t (the point of the edge line along it), and the density in t is
// the density in phi times the arc-length Jacobian |e x w^| / |w|:
//   p(t) = max(n . w^(t), 0) |e x w^(t)| / (T |w(t)|),  T = integral of the
//   positive part of the cosine over the whole arc.
// Returns false (no sample) when T is zero or the arc degenerate.
// ---------------------------------------------------------------------------
const double kArcMin = 1e-6;      // sin of the smallest arc the cosine sampler handles
const double kTieArc = 1e-5;      // relative closeness of the arc test and of T to zero

bool cosine_edge_t(V3d p, V3d n, V3d pa, V3d pb, double u, double& t, bool* flag) {
    V3d a = normalize(pa - p), b = normalize(pb - p);
    double cab = dot(a, b);
    V3d bo = b - a * cab;
    double sb = length(bo);
    if (flag && std::fabs(sb - kArcMin) < kTieArc * kArcMin) *flag = true;
    if (!(sb > kArcMin)) return false;
    bo = bo / sb;
    double Phi = std::atan2(sb, cab);
    double A = dot(n, a), B = dot(n, bo);
    double phi0 = std::atan2(B, A);
    if (phi0 < -kPi / 2) phi0 += 2 * kPi;
    double lo = std::max(0.0, phi0 - kPi / 2), hi = std::min(Phi, phi0 + kPi / 2);
    if (flag && std::fabs(hi - lo) < kTieArc) *flag = true;
    if (!(hi > lo)) return false;
    double slo = std::sin(lo - phi0), shi = std::sin(hi - phi0);
    double sv = slo + u * (shi - slo);
    double phi = phi0 + std::asin(std::max(-1.0, std::min(1.0, sv)));
    V3d wd = a * std::cos(phi) + bo * std::sin(phi);
    V3d e = pb - pa, v0p = pa - p;
    V3d ew = cross(e, wd);
    t = -dot(cross(v0p, wd), ew) / dot(ew, ew);
    t = std::max(0.0, std::min(1.0, t));
    return true;
}

// T of cosine_edge_t: the integral over the arc of the positive part of the cosine.
double cosine_arc_integral(V3d p, V3d n, V3d pa, V3d pb) {
    V3d a = normalize(pa - p), b = normalize(pb - p);
    double cab = dot(a, b);
    V3d bo = b - a * cab;
    double sb = length(bo);
    if (!(sb > kArcMin)) return 0;
    bo = bo / sb;
    double Phi = std::atan2(sb, cab);
    double A = dot(n, a), B = dot(n, bo);
    double R = std::hypot(A, B);
    double phi0 = std::atan2(B, A);
    if (phi0 < -kPi / 2) phi0 += 2 * kPi;
    double lo = std::max(0.0, phi0 - kPi / 2), hi = std::min(Phi, phi0 + kPi / 2);
    if (!(hi > lo)) return 0;
    return R * (std::sin(hi - phi0) - std::sin(lo - phi0));
}

// Density in t of cosine_edge_t at edge parameter t.
double cosine_edge_pdf(V3d p, V3d n, V3d pa, V3d pb, double t, double T) {
    V3d e = pb - pa;
    V3d w = pa + e * t - p;
    double wl = length(w);
    V3d wh = w / wl;
    double c = dot(n, wh);
    if (!(c > 0) || !(T > 0)) return 0;
    return c * length(cross(e, wh)) / (T * wl);
}

// ---------------------------------------------------------------------------
// Next event estimation for edges (Ch. 5, Next event estimation for edges).
//
// A second strategy for the secondary edge sample at a shading point x: a
// light point y is drawn as for next-event estimation, every edge is widened
// into a billboard facing x, and among the billboards the segment x -> y
// crosses one is chosen in proportion to the edge's importance; the crossing,
// projected onto the edge, is the sample. Readings (the thesis gives the
// construction, not its density):
//  * the billboard of edge (pa, pb) seen from x is the planar strip
//    { pa + t a + s v : t in [0, 1], |s| <= w/2 }, a = pb - pa, v the unit
//    vector orthogonal to the edge and to pa - x. Its plane contains the edge
//    and its normal points along the perpendicular from the edge's line to x,
//    so it faces every ray leaving x; a crossing at (t, s) projects onto the
//    edge point of parameter t;
//  * w is the strip's full width, the L2 norm over the three coordinates of
//    2% of the mean absolute deviation of the scene's vertex positions;
//  * the light point is drawn afresh (the same light distribution as the
//    forward pass's next-event estimation: a light triangle by area, a
//    uniform point in it), and light points behind x's tangent plane or, for
//    one-sided emitters, on an emitter's back are not used;
//  * the importance of an edge is that of a leaf of the edge hierarchy
//    without the parent-box rule: length x cosine bound of its box / distance
//    of the box centre, zero for x's own triangle's edges and for edges that
//    are not discontinuities as seen from x; the choice among the crossed
//    billboards is an exponential race (edge e's key -log(1 - u_e) / imp_e
//    with u_e its own uniform, the smallest key wins), which picks e with
//    probability imp_e / sum of the crossed importances in any visiting order;
//  * the strategy is combined with the hierarchy by one-sample multiple
//    importance sampling: with probability alpha the billboard strategy,
//    otherwise the hierarchy (plus a uniform s across the strip), every sample
//    weighted by the balance-heuristic mixture density
//    alpha p_N(e, t, s) + (1 - alpha) p_H(e) / w in the space (e, t, s). Since
//    the integrand does not depend on s, dividing by 1/w turns that into the
//    density alpha w p_N + (1 - alpha) p_H in (e, t) that the estimator uses.
//
// The density of the billboard strategy at (e, t, s): the ray from x through
// b = pa + t a + s v meets the lights at points y = x + mu (b - x), mu > 1;
// each such y was drawn with area density 1 / A_lights, the map from light
// area to strip area has Jacobian |y - x|^2 cos_b / (|b - x|^2 cos_y), the
// strip's area element is |a| dt ds, and e was chosen among the billboards
// crossed by x -> y with probability imp_e / sum_crossed imp:
//   p_N = |a| / A_lights * sum_y mu^2 |cos_b| / |cos_y| * imp_e / sum_crossed(x, y) imp.
// ---------------------------------------------------------------------------
const double kNeeMadFrac = 0.02;  // billboard width: this fraction of the mean absolute deviation
const double kTieBB = 1e-4;       // crossing parameters vs. the strip's borders (t, and s relative to w)
const double kTieRace = 1e-4;     // relative gap between the two smallest race keys
const double kTieLight = 1e-4;    // barycentric margin of a light hit, relative distance of the light to b

double nee_width_default(const Scn& s) {
    double mean[3] = {0, 0, 0}, mad[3] = {0, 0, 0};
    for (int v = 0; v < s.V; ++v)
        for (int k = 0; k < 3; ++k) mean[k] += s.P[3 * v + k];
    for (int k = 0; k < 3; ++k) mean[k] /= s.V;
    for (int v = 0; v < s.V; ++v)
        for (int k = 0; k < 3; ++k) mad[k] += std::fabs(s.P[3 * v + k] - mean[k]);
    double w2 = 0;
    for (int k = 0; k < 3; ++k) {
        double m = kNeeMadFrac * mad[k] / s.V;
        w2 += m * m;
    }
    return std::sqrt(w2);
}

struct Billboard {
    V3d pa, ah, v, nb;   // edge start, unit edge direction, unit width direction, unit normal
    double L;            // edge length
    bool ok;
};

Billboard billboard(const Scn& s, const Edge& e, const V3d& x) {
    Billboard B;
    B.pa = s.p(e.va);
    V3d a = s.p(e.vb) - B.pa;
    B.L = length(a);
    B.ok = false;
    if (!(B.L > 0)) return B;
    B.ah = a / B.L;
    V3d c = cross(B.ah, B.pa - x);
    double cl = length(c);
    if (!(cl > 0)) return B;
    B.v = c / cl;
    B.nb = cross(B.ah, B.v);
    B.ok = true;
    return B;
}

// Crossing of the segment x -> y (excluding both ends) with the strip of
// width w; (t, sv) the crossing's strip coordinates; *near: one of the three
// tests was within rounding of its border.
bool bb_cross(const Billboard& B, const V3d& x, const V3d& y, double w, double& t, double& sv, bool* near) {
    *near = false;
    if (!B.ok) return false;
    V3d d = y - x;
    double den = dot(d, B.nb);
    if (den == 0) return false;
    double lam = dot(B.pa - x, B.nb) / den;
    V3d r = x + d * lam - B.pa;
    t = dot(r, B.ah) / B.L;
    sv = dot(r, B.v);
    bool in_t = t >= 0 && t <= 1, in_s = std::fabs(sv) <= 0.5 * w, in_l = lam > 0 && lam < 1;
    if (in_l && in_s && (std::fabs(t) < kTieBB || std::fabs(t - 1) < kTieBB)) *near = true;
    if (in_l && in_t && std::fabs(std::fabs(sv) - 0.5 * w) < kTieBB * w) *near = true;
    if (in_t && in_s && std::fabs(lam - 1) < kTieLight) *near = true;
    return in_t && in_s && in_l;
}

// Importance of edge ei at (p, n) on triangle tri (a hierarchy leaf's, no
// parent-box rule). Edges of emitters are left to the hierarchy: their strips
// reach the light's own plane, where the segment to a light point ends.
double nee_importance(const Scn& s, int ei, const V3d& p, const V3d& n, int tri, Unit* U) {
    const Edge& e = s.edges[ei];
    if (e.kind == 0 || (tri >= 0 && (e.f0 == tri || e.f1 == tri))) return 0;
    if (s.emi[e.f0] > 0 || (e.f1 >= 0 && s.emi[e.f1] > 0)) return 0;
    if (!disc_from(s, e, p, U ? &U->flag : nullptr)) return 0;
    V3d a = s.p(e.va), b = s.p(e.vb);
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) { lo[k] = std::min(comp(a, k), comp(b, k)); hi[k] = std::max(comp(a, k), comp(b, k)); }
    double cb = cos_bound(lo, hi, p, n, U, s.diag);
    if (cb <= 0) return 0;
    return length(b - a) * cb / length((a + b) * 0.5 - p);
}

struct NeeQuery {
    const Scn* s;
    V3d p, n;
    int tri;
    double w;
};

// Whether x -> y crosses edge ei's strip, and the edge's importance. Near
// ties are flagged only for edges at or near a crossing, and crossing ties
// only for edges of positive importance: only those decisions change a result.
bool nee_cross(const NeeQuery& q, int ei, const V3d& y, double& t, double& sv, double& imp, Unit* U) {
    bool near;
    bool c = bb_cross(billboard(*q.s, q.s->edges[ei], q.p), q.p, y, q.w, t, sv, &near);
    if (!c && !near) return false;
    imp = nee_importance(*q.s, ei, q.p, q.n, q.tri, U);
    if (!(imp > 0)) return false;
    if (near && U) TIE(*U, 19);
    return c;
}

// Sum of the importances of the billboards crossed by x -> y, edge `skip`
// left out.
double nee_crossed_sum(const NeeQuery& q, const V3d& y, int skip, Unit* U) {
    double sum = 0;
    for (int ei = 0; ei < (int)q.s->edges.size(); ++ei) {
        if (ei == skip || q.s->edges[ei].kind == 0) continue;
        double t, sv, imp;
        if (nee_cross(q, ei, y, t, sv, imp, U)) sum += imp;
    }
    return sum;
}

// Whether a light point direction is used by the strategy (above x's tangent
// plane; for one-sided emitters, on the emitting side); with near-tie flags.
bool nee_usable(const NeeQuery& q, const V3d& dh, int lt, Unit* U) {
    double cp = dot(q.n, dh);
    if (U && std::fabs(cp) < kTieSign) TIE(*U, 19);
    if (!(cp > 0)) return false;
    if (q.s->two_sided) return true;
    double cy = -dot(normalize(q.s->face_n(lt)), dh);
    if (U && std::fabs(cy) < kTieCos) TIE(*U, 19);
    return cy > 0;
}

// Density p_N of the billboard strategy at (edge ei, t, sv), in dt ds.
// known_lt: the light triangle of the draw's own light point (-1: none). The
// ray through the strip point meets that triangle by construction (the strip
// point lies on the segment to the light point), so its hit is taken without
// the inside and side tests: a rounding miss there would drop the strategy's
// own density from the sample's weight.
double nee_pdf(const NeeQuery& q, int ei, double t, double sv, int known_lt, Unit* U) {
    const Scn& s = *q.s;
    double imp = nee_importance(s, ei, q.p, q.n, q.tri, U);
    if (!(imp > 0) || s.atot <= 0) return 0;
    Billboard B = billboard(s, s.edges[ei], q.p);
    if (!B.ok) return 0;
    V3d b = B.pa + B.ah * (B.L * t) + B.v * sv;
    V3d d = b - q.p;
    V3d dh = normalize(d);
    double cb = std::fabs(dot(dh, B.nb));
    double acc = 0;
    for (int lt : s.lights) {
        double mu;
        V3d nl = normalize(s.face_n(lt));
        if (lt == known_lt) {
            double dn = dot(d, nl);
            if (dn == 0) continue;
            mu = dot(s.p(s.I[3 * lt]) - q.p, nl) / dn;
        } else {
            TriHit h = tri_test(s, lt, q.p, d, 1.0, 1e300);
            if (!h.valid) continue;
            if (U && h.t > 1 - kTieLight && std::fabs(h.m) < kTieLight) TIE(*U, 21);
            if (U && h.m > -kTieLight && std::fabs(h.t - 1) < kTieLight) TIE(*U, 21);
            if (!h.ok) continue;
            if (!nee_usable(q, dh, lt, U)) continue;
            mu = h.t;
        }
        double cy = std::fabs(dot(nl, dh));
        if (!(cy > 0)) continue;
        V3d y = q.p + d * mu;
        double sum = imp + nee_crossed_sum(q, y, ei, U);
        acc += mu * mu * cb / cy * imp / sum;
    }
    return acc * B.L / s.atot;
}

// One draw of the billboard strategy from uniforms ul = (light pick, two
// point uniforms) and the race uniforms of stream rs (edge e: block 2 + e,
// first uniform). Returns the edge (or -1), its strip coordinates and the
// light triangle of the light point.
int nee_sample(const NeeQuery& q, const double ul[3], const Stream& rs, double& t, double& sv, int& lt, Unit* U) {
    const Scn& s = *q.s;
    if (s.lights.empty()) return -1;
    Unit dummy;
    int li = cdf_pick(s.lcdf, ul[0], U ? *U : dummy);
    lt = s.lights[li];
    V3d a = s.p(s.I[3 * lt]), b = s.p(s.I[3 * lt + 1]), c = s.p(s.I[3 * lt + 2]);
    double su = std::sqrt(ul[1]);
    V3d y = a * (1 - su) + b * (su * (1 - ul[2])) + c * (su * ul[2]);
    if (!nee_usable(q, normalize(y - q.p), lt, U)) return -1;
    int best = -1;
    double k1 = 1e300, k2 = 1e300;
    for (int ei = 0; ei < (int)s.edges.size(); ++ei) {
        if (s.edges[ei].kind == 0) continue;
        double te, se, imp;
        if (!nee_cross(q, ei, y, te, se, imp, U)) continue;
        double u[4];
        rs.block(2u + (uint32_t)ei, u);
        double key = -std::log(1.0 - u[0]) / imp;
        if (key < k1) { k2 = k1; k1 = key; best = ei; t = te; sv = se; }
        else if (key < k2) k2 = key;
    }
    if (U && best >= 0 && k2 < 1e300 && k2 - k1 <= kTieRace * k2) TIE(*U, 20);
    return best;
}

// One-sample mixture of the billboard strategy (probability alpha) and the
// hierarchy. rk: the vertex's secondary-edge stream (root uniform and t in
// block 0, level uniforms from block 1); rn: its billboard stream (block 0:
// strategy choice and light uniforms, block 1: s of hierarchy draws, race
// uniforms from block 2). Returns the edge (or -1), its parameter t and the
// mixture density in (e, t).
int nee_mix_draw(const TreeQuery& tq, double w, double alpha, const Stream& rk, const Stream& rn, double& t, double& pdf,
                 Unit* U) {
    NeeQuery q{tq.s, tq.p, tq.n, tq.tri, w};
    double c0[4], c1[4];
    rn.block(0, c0);
    rn.block(1, c1);
    if (U && std::fabs(c0[0] - alpha) < kTieU) TIE(*U, 22);
    int ei, lt = -1;
    double sv, ph;
    if (c0[0] < alpha) {
        ei = nee_sample(q, c0 + 1, rn, t, sv, lt, U);
        if (ei < 0) return -1;
        ph = tree_pdf_edge(tq, ei, U);
    } else {
        double b0[4], cache[4];
        rk.block(0, b0);
        int cached = -1;
        auto level_u = [&](int lev) {
            int blk = 1 + lev / 4;
            if (blk != cached) { rk.block((uint32_t)blk, cache); cached = blk; }
            return cache[lev % 4];
        };
        ei = tree_sample(tq, b0[0], level_u, ph, U);
        if (ei < 0) return -1;
        t = b0[1];
        sv = (c1[0] - 0.5) * w;
    }
    pdf = alpha * w * nee_pdf(q, ei, t, sv, lt, U) + (1 - alpha) * ph;
    return pdf > 0 ? ei : -1;
}

// ---------------------------------------------------------------------------
// Per-unit evaluation
// ---------------------------------------------------------------------------
struct Ctx {
    const Scn* s;
    const orc_camera* oc;
    const orc_options* o;
    const View* vw;
    const ETree* et;
    const double* d_image;
    int Ww, Hw, spp, M, V, T;
    uint32_t k0, k1;
    std::vector<double> qcdf;   // CDF of the proposal distribution over all edges (secondary mixture)
    bool mix_p = false, mix_s = false, harvest = false;
    double nee_w = 0;           // billboard width of the secondary billboard strategy
};

struct Acc {
    std::vector<double> img, g, mass, es, esm;
    int64_t rays = 0, flagged = 0, pedge = 0, sedge = 0;
};

// Reverse sweep from one output; appends (parameter, adjoint) pairs.
void sweep(const Ctx& C, const Leaves& L, int32_t out, double seed, std::vector<std::pair<int, double>>& res) {
    if (out < 0 || seed == 0) return;
    std::vector<double>& adj = TP.adj;
    adj.assign((size_t)out + 1, 0.0);
    adj[out] = seed;
    for (int32_t i = out; i >= 0; --i) {
        double g = adj[i];
        if (g == 0) continue;
        if (TP.pa[i] >= 0) adj[TP.pa[i]] += TP.ga[i] * g;
        if (TP.pb[i] >= 0) adj[TP.pb[i]] += TP.gb[i] * g;
    }
    for (const auto& kv : L.v)
        for (int k = 0; k < 3; ++k)
            if (kv.second[k] <= out && adj[kv.second[k]] != 0) res.push_back({3 * kv.first + k, adj[kv.second[k]]});
    for (const auto& kv : L.a)
        if (kv.second <= out && adj[kv.second] != 0) res.push_back({3 * C.V + kv.first, adj[kv.second]});
    for (int k = 0; k < 9; ++k)
        if (L.cam[k] <= out && adj[L.cam[k]] != 0) res.push_back({3 * C.V + C.T + k, adj[L.cam[k]]});
}

int debug_unit() {
    static int u = [] {
        const char* e = std::getenv("ORC_DEBUG_UNIT");
        return e ? std::atoi(e) : -1;
    }();
    return u;
}

void run_unit(const Ctx& C, int m, Acc& acc) {
    const Scn& s = *C.s;
    const orc_options& o = *C.o;
    const bool dbg = m == debug_unit();
    if (o.unit_mask && !o.unit_mask[m]) return;
    TP.clear();
    Leaves L;
    Unit U;
    if (o.dir_mode && o.dir_log) {
        U.dir_mode = o.dir_mode;
        U.dir = o.dir_log + (size_t)m * kDirSlots;
    }
    int pix = m / C.spp, smp = m % C.spp;
    int pxr = pix % C.Ww, pyr = pix / C.Ww;
    int px = C.oc->win_x0 + pxr, py = C.oc->win_y0 + pyr;
    uint32_t sid = (uint32_t)(((uint32_t)py * (uint32_t)C.oc->width + (uint32_t)px) * (uint32_t)C.spp + (uint32_t)smp);
    Stream rc{sid, o.view_id, TAG_CAM, C.k0, C.k1};
    double j[4];
    rc.block(0, j);
    double sx = px + j[0], sy = py + j[1];
    // camera leaves
    D cp[9];
    for (int k = 0; k < 9; ++k) { cp[k] = leafD(cam_param(*C.oc, k)); L.cam[k] = cp[k].i; }
    Cam<D> cam = make_cam<D>(V3<D>{cp[0], cp[1], cp[2]}, V3<D>{cp[3], cp[4], cp[5]}, V3<D>{cp[6], cp[7], cp[8]}, *C.oc);
    Env<D> Ed{&s, &L};
    Env<double> Ev{&s};
    std::vector<PathVtx<D>> verts;
    V3<D> dir = cam_dir(cam, sx, sy);
    Cond cmain;
    cmain.dx = 4 * length(valv(cam.c));
    D Lr = o.aov ? aov_impl<D>(Ed, U, o.aov, cam.c, dir, C.oc->near_clip, &cmain)
                 : radiance_impl<D>(Ed, U, rc, 0, cam.c, dir, C.oc->near_clip, true, o.max_depth, &verts, &cmain);
    std::vector<std::pair<int, double>> contrib;
    std::vector<double> sweep_mass_keys;
    std::vector<std::vector<std::pair<int, double>>> parts;
    // Rounding scale of each part: a boundary sample's weight is a difference
    // of two radiances, whose rounding error scales with |a| + |b|.
    std::vector<double> scales;
    struct Harvest { int e; double v, mass; };
    std::vector<Harvest> harvest;   // (edge, P |c|^2, its rounding scale)
    int64_t used_p = 0, used_s = 0;
    if (C.d_image) {
        double wimg = C.d_image[pix] / C.spp;
        if (o.interior) {
            parts.emplace_back();
            scales.push_back(1.0 + kCondSafety * cmain.kmax / kOpsU32);
            sweep(C, L, Lr.i, wimg, parts.back());
        }
        // Secondary boundary term at every path vertex (one edge sample each).
        if (o.secondary_edges && C.et && !o.aov) {
            for (size_t kv = 0; kv < verts.size(); ++kv) {
                int k = (int)kv + 1;
                const PathVtx<D>& pv = verts[kv];
                Stream rk{sid, o.view_id, TAG_SEDGE + (uint32_t)k, C.k0, C.k1};
                double b0[4];
                rk.block(0, b0);
                V3d p = valv(pv.x), nsv = valv(pv.ns);
                TreeQuery q{&s, C.et, p, nsv, pv.tri};
                double pdf = 0;
                double cache[4];
                int cached = -1;
                auto level_u = [&](int lev) {
                    int blk = 1 + lev / 4;
                    if (blk != cached) { rk.block((uint32_t)blk, cache); cached = blk; }
                    return cache[lev % 4];
                };
                int ei;
                double te_draw = -1;
                if (o.enee > 0) {
                    // the billboard strategy mixed with the hierarchy: the
                    // draw carries its own edge parameter and mixture density
                    Stream rn{sid, o.view_id, TAG_ENEE + (uint32_t)k, C.k0, C.k1};
                    ei = nee_mix_draw(q, C.nee_w, o.enee, rk, rn, te_draw, pdf, &U);
                } else if (C.mix_s) {
                    // proposal mixture: the component from the block's third
                    // uniform, a proposal draw from its fourth
                    if (std::fabs(b0[2] - o.mix) < kTieU) TIE(U, 15);
                    double pt;
                    if (b0[2] < o.mix) {
                        ei = cdf_pick(C.qcdf, b0[3], U);
                        pt = tree_pdf_edge(q, ei, &U);
                    } else {
                        ei = tree_sample(q, b0[0], level_u, pt, &U, dbg);
                        if (ei < 0) continue;
                    }
                    pdf = o.mix * o.edge_pdf[ei] + (1.0 - o.mix) * pt;
                    if (!(pdf > 0)) continue;
                } else if (o.edge_candidates > 1) {
                    // several samples through the hierarchy, one kept: the
                    // kept edge's weight W / (M imp) stands in for 1 / pdf
                    Stream rs{sid, o.view_id, TAG_SELECT + (uint32_t)k, C.k0, C.k1};
                    double sc[4];
                    uint32_t cnt = 0;
                    auto next_u = [&]() {
                        if ((cnt & 3) == 0) rs.block(cnt >> 2, sc);
                        return sc[cnt++ & 3];
                    };
                    double wsel = 0;
                    ei = tree_select(q, o.edge_candidates, next_u, wsel, &U);
                    if (ei >= 0) pdf = 1.0 / wsel;
                } else {
                    ei = tree_sample(q, b0[0], level_u, pdf, &U, dbg);
                }
                if (ei < 0) continue;
                const Edge& e = s.edges[ei];
                if (e.f0 == pv.tri || e.f1 == pv.tri) continue;
                if (!disc_from(s, e, p, &U.flag)) continue;
                V3d pa = s.p(e.va), pb = s.p(e.vb);
                // the point on the edge: uniform in t, or by the clamped cosine
                double te = te_draw >= 0 ? te_draw : b0[1], pdf_t = 1.0;
                if (o.edge_t_mode == 1) {
                    if (!cosine_edge_t(p, nsv, pa, pb, b0[1], te, &U.flag)) continue;
                    double Tc = cosine_arc_integral(p, nsv, pa, pb);
                    pdf_t = cosine_edge_pdf(p, nsv, pa, pb, te, Tc);
                    if (!(pdf_t > 0)) continue;
                }
                V3d vt = pa + (pb - pa) * te;
                V3d w = vt - p;
                if (dot(nsv, w) <= kHorizon * s.diag) continue;
                V3d v0p = pa - p, v1p = pb - p;
                V3d c = cross(v0p, v1p);
                double cn = length(c);
                if (cn == 0) continue;
                if (cn < kTieCond * length(v0p) * length(v1p)) TIE(U, 12);
                V3d nh = c / cn;
                double wl = length(w);
                V3d wh = w / wl;
                V3d wp = normalize(wh + nh * kEps3), wm = normalize(wh - nh * kEps3);
                int rem = o.max_depth - k;
                Cond cp, cm;
                cp.dx = cm.dx = pv.dx;
                cp.dw = cm.dw = 8 + pv.dx / wl;
                cp.kmax = cm.kmax = pv.kappa;
                departure_tie(s, pv.tri, p, wp, U);
                departure_tie(s, pv.tri, p, wm, U);
                // the same limit rule as for primary edges
                bool same = closest(s, p, wp, s.tmin, 1e300, U).tri == closest(s, p, wm, s.tmin, 1e300, U).tri;
                double Lp = same ? 0.0 : radiance_impl<double>(Ev, U, rk, kSideBlockBase, p, wp, s.tmin, false, rem, nullptr, &cp);
                double Lm = same ? 0.0 : radiance_impl<double>(Ev, U, rk, kSideBlockBase, p, wm, s.tmin, false, rem, nullptr, &cm);
                double kap_s = std::max(pv.kappa, std::max(cp.kmax, cm.kmax)) + pv.dx / wl;
                // The cosine factor is continuous across the edge: both one-sided
                // limits share the cosine at the edge point; only L jumps.
                double cosw = dot(nsv, wh);
                double Fp = val(pv.rho) / kPi * cosw * Lp;
                double Fm = val(pv.rho) / kPi * cosw * Lm;
                used_s++;
                if (Fp == Fm) continue;
                double W = C.d_image[pix] * val(pv.beta) / C.spp;
                double wgt = W * (Fp - Fm) * length(cross(pb - pa, wh)) / (cn * wl * pdf * pdf_t);
                if (dbg)
                    std::fprintf(stderr, "unit %d vertex %d tri %d p=(%.9g %.9g %.9g) n=(%.9g %.9g %.9g) edge %d pdf %.9g "
                                 "t %.9g pdf_t %.9g Lp %.9g Lm %.9g cos %.9g W %.9g wgt %.9g kappa %.3g\n",
                                 m, k, pv.tri, p.x, p.y, p.z, nsv.x, nsv.y, nsv.z, ei, pdf, te, pdf_t, Lp, Lm, cosw, W, wgt,
                                 kap_s);
                V3<D> A = Ed.P(e.va), B = Ed.P(e.vb);
                D beta = dot(lift<D>(wh), cross(A - pv.x, B - pv.x));
                parts.emplace_back();
                scales.push_back((1.0 + kCondSafety * kap_s / kOpsU32) * (std::fabs(Fp) + std::fabs(Fm)) / std::fabs(Fp - Fm));
                sweep(C, L, beta.i, wgt, parts.back());
                if (C.harvest) {
                    double c2 = (dot(cross(v1p, wh), cross(v1p, wh)) + dot(cross(wh, v0p), cross(wh, v0p))) * wgt * wgt;
                    // P(edge) p(t) |c|^2: its expectation does not depend on either density
                    harvest.push_back({ei, pdf * pdf_t * c2, pdf * pdf_t * c2 * scales.back()});
                }
            }
        }
        // Primary boundary term: one screen-space edge sample for this unit.
        if (o.primary_edges && C.vw->psum > 0) {
            const View& vw = *C.vw;
            Stream rp{(uint32_t)m, o.view_id, TAG_PEDGE, C.k0, C.k1};
            double b0[4];
            rp.block(0, b0);
            // stratified edge choice: unit m draws its uniform in [m/M, (m+1)/M)
            double us = ((double)m + b0[0]) / (double)C.M;
            int ei = cdf_pick(C.mix_p ? vw.mcdf : vw.pcdf, us, U);
            const PEdge& pe = vw.pe[ei];
            // 1 / (P(edge) p(point | edge)), p uniform on the clipped segment
            double inv_p = C.mix_p ? pe.len / vw.mprob[ei] : vw.psum;
            double p_edge = C.mix_p ? vw.mprob[ei] : pe.len / vw.psum;
            if (pe.len > 0) {
            double t = b0[1];
            double x = pe.Ac[0] + (pe.Bc[0] - pe.Ac[0]) * t, y = pe.Ac[1] + (pe.Bc[1] - pe.Ac[1]) * t;
            double nl = std::hypot(pe.Aa[0] - pe.Ba[0], pe.Aa[1] - pe.Ba[1]);
            double nx = (pe.Aa[1] - pe.Ba[1]) / nl, ny = (pe.Ba[0] - pe.Aa[0]) / nl;
            V3d cpos = vw.cam.c;
            Cond cu, cl;
            cu.dx = cl.dx = 4 * length(cpos);
            V3d du = cam_dir(vw.cam, x + kEpsPx * nx, y + kEpsPx * ny), dl = cam_dir(vw.cam, x - kEpsPx * nx, y - kEpsPx * ny);
            // Both one-sided rays on the same triangle (or both escaping): the
            // edge is no visible discontinuity at this point, the one-sided
            // limits coincide and the sample contributes nothing.
            bool same = closest(s, cpos, du, C.oc->near_clip, 1e300, U).tri == closest(s, cpos, dl, C.oc->near_clip, 1e300, U).tri;
            double fu = same ? 0.0 : o.aov ? aov_impl<double>(Ev, U, o.aov, cpos, du, C.oc->near_clip, &cu)
                                     : radiance_impl<double>(Ev, U, rp, 0, cpos, du, C.oc->near_clip, true, o.max_depth, nullptr, &cu);
            double fl = same ? 0.0 : o.aov ? aov_impl<double>(Ev, U, o.aov, cpos, dl, C.oc->near_clip, &cl)
                                     : radiance_impl<double>(Ev, U, rp, 0, cpos, dl, C.oc->near_clip, true, o.max_depth, nullptr, &cl);
            double kap_p = std::max(cu.kmax, cl.kmax);
            {
                // a near-clipped endpoint sits at depth `near`: its projection and
                // the clip parameter amplify FP32 position errors by ~distance/near
                const Edge& ce = s.edges[ei];
                V3d pa = s.p(ce.va), pb = s.p(ce.vb);
                double za = dot(pa - vw.cam.c, vw.cam.f), zb = dot(pb - vw.cam.c, vw.cam.f);
                if (za < vw.cam.near || zb < vw.cam.near)
                    kap_p += 4 * (length(pa - vw.cam.c) + length(pb - vw.cam.c)) /
                             std::max(vw.cam.near, 0.5 * std::max(za, zb));
            }
            if (dbg)
                std::fprintf(stderr, "punit %d edge %d x %.9g y %.9g A %.9g %.9g B %.9g %.9g n %.9g %.9g fu %.9g fl %.9g total %.9g\n",
                             m, ei, x, y, pe.Aa[0], pe.Aa[1], pe.Ba[0], pe.Ba[1], nx, ny, fu, fl, vw.psum);
            int ix = (int)std::floor(x), iy = (int)std::floor(y);
            ix = std::min(std::max(ix, vw.x0), vw.x1 - 1);
            iy = std::min(std::max(iy, vw.y0), vw.y1 - 1);
            double rx = std::round(x), ry = std::round(y);
            if ((std::fabs(x - rx) < kTiePx && rx > vw.x0 && rx < vw.x1) || (std::fabs(y - ry) < kTiePx && ry > vw.y0 && ry < vw.y1))
                TIE(U, 13);
            used_p++;
            if (fu != fl) {
                int ppix = (iy - vw.y0) * C.Ww + (ix - vw.x0);
                double wgt = C.d_image[ppix] * (fu - fl) * inv_p / ((double)C.M * nl);
                const Edge& e = s.edges[ei];
                V3<D> a3, b3;
                alpha_points(cam, Ed.P(e.va), Ed.P(e.vb), a3, b3);
                D ax, ay, bx, by;
                project(cam, a3, ax, ay);
                project(cam, b3, bx, by);
                D alpha = (ay - by) * x + (bx - ax) * y + (ax * by - bx * ay);
                parts.emplace_back();
                scales.push_back((1.0 + kCondSafety * kap_p / kOpsU32) * (std::fabs(fu) + std::fabs(fl)) / std::fabs(fu - fl));
                sweep(C, L, alpha.i, wgt, parts.back());
                if (C.harvest) {
                    double c2 = 0;
                    for (const auto& pr : parts.back())
                        if (pr.first / 3 == e.va || pr.first / 3 == e.vb)
                            if (pr.first < 3 * C.V) c2 += pr.second * pr.second;
                    harvest.push_back({ei, p_edge * c2, p_edge * c2 * scales.back()});
                }
            }
            }
        }
    }
    acc.rays += U.rays;
    if (U.flag) {
        acc.flagged++;
        if (o.exclude_flagged) return;
    }
    acc.pedge += used_p;
    acc.sedge += used_s;
    if (!acc.img.empty()) acc.img[pix] += Lr.v / C.spp;
    for (size_t i = 0; i < parts.size(); ++i)
        for (const auto& pr : parts[i]) {
            acc.g[pr.first] += pr.second;
            acc.mass[pr.first] += std::fabs(pr.second) * scales[i];
        }
    for (const auto& h : harvest) { acc.es[h.e] += h.v; acc.esm[h.e] += h.mass; }
}

}  // namespace

// ---------------------------------------------------------------------------
// C API
// ---------------------------------------------------------------------------
extern "C" {

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) { philox(ctr, key, out); }

int orc_edge_t_cosine(const double p[3], const double n[3], const double v0[3], const double v1[3], int32_t count,
                      const double* u, double* t, double* pdf_t) {
    V3d P{p[0], p[1], p[2]}, N{n[0], n[1], n[2]}, A{v0[0], v0[1], v0[2]}, B{v1[0], v1[1], v1[2]};
    double T = cosine_arc_integral(P, N, A, B);
    for (int i = 0; i < count; ++i) {
        double te = -1;
        if (!cosine_edge_t(P, N, A, B, u[i], te, nullptr)) {
            t[i] = -1;
            pdf_t[i] = 0;
            continue;
        }
        t[i] = te;
        pdf_t[i] = cosine_edge_pdf(P, N, A, B, te, T);
    }
    return ORC_OK;
}

double orc_edge_t_cosine_pdf(const double p[3], const double n[3], const double v0[3], const double v1[3], double t) {
    V3d P{p[0], p[1], p[2]}, N{n[0], n[1], n[2]}, A{v0[0], v0[1], v0[2]}, B{v1[0], v1[1], v1[2]};
    return cosine_edge_pdf(P, N, A, B, t, cosine_arc_integral(P, N, A, B));
}

void orc_tie_reasons(int64_t out[24], int32_t reset) {
    for (int i = 0; i < 24; ++i) {
        out[i] = g_reason[i];
        if (reset) g_reason[i] = 0;
    }
}

int orc_edges(const orc_scene* sd, int32_t* num_edges, int32_t* rows) {
    Scn s;
    int rc = prepare(sd, s);
    if (rc) return rc;
    *num_edges = (int32_t)s.edges.size();
    if (rows)
        for (size_t i = 0; i < s.edges.size(); ++i) {
            rows[4 * i] = s.edges[i].va; rows[4 * i + 1] = s.edges[i].vb;
            rows[4 * i + 2] = s.edges[i].f0; rows[4 * i + 3] = s.edges[i].f1;
        }
    return ORC_OK;
}

int orc_closest_hit(const orc_scene* sd, int32_t n, const double* o, const double* d, double tmin, double tmax,
                    int32_t use_bvh, int32_t* tri, double* t) {
    Scn s;
    int rc = prepare(sd, s);
    if (rc) return rc;
    s.use_bvh = use_bvh != 0;
    for (int i = 0; i < n; ++i) {
        Unit U;
        Hit h = closest(s, V3d{o[3 * i], o[3 * i + 1], o[3 * i + 2]}, V3d{d[3 * i], d[3 * i + 1], d[3 * i + 2]}, tmin, tmax, U);
        tri[i] = h.tri;
        t[i] = h.tri >= 0 ? h.t : 0;
    }
    return ORC_OK;
}

static int tree_setup(const orc_scene* sd, const orc_camera* c, Scn& s, ETree& t) {
    int rc = prepare(sd, s);
    if (rc) return rc;
    return build_etree(s, V3d{cam_param(*c, 0), cam_param(*c, 1), cam_param(*c, 2)}, t);
}

int orc_edge_tree_pdf(const orc_scene* sd, const orc_camera* c, const double p[3], const double n[3], double* pdf,
                      double* p_fail) {
    Scn s;
    ETree t;
    int rc = tree_setup(sd, c, s, t);
    if (rc) return rc;
    TreeQuery q{&s, &t, V3d{p[0], p[1], p[2]}, V3d{n[0], n[1], n[2]}, -1};
    std::vector<double> pd(s.edges.size(), 0.0);
    double fail = 0;
    double lo[3], hi[3];
    root_box(t, lo, hi);
    double w[2] = {0, 0};
    for (int h = 0; h < 2; ++h)
        if (t.root[h] >= 0) w[h] = importance(q, t.nodes[t.root[h]], h == 1, lo, hi, nullptr);
    if (w[0] + w[1] <= 0) fail = 1;
    else
        for (int h = 0; h < 2; ++h)
            if (w[h] > 0) tree_enumerate(q, t.root[h], h == 1, w[h] / (w[0] + w[1]), pd, fail);
    for (size_t i = 0; i < pd.size(); ++i) pdf[i] = pd[i];
    *p_fail = fail;
    return ORC_OK;
}

int orc_edge_tree_pdf_of(const orc_scene* sd, const orc_camera* c, const double p[3], const double n[3],
                         int32_t count, const int32_t* edges, double* pdf) {
    Scn s;
    ETree t;
    int rc = tree_setup(sd, c, s, t);
    if (rc) return rc;
    TreeQuery q{&s, &t, V3d{p[0], p[1], p[2]}, V3d{n[0], n[1], n[2]}, -1};
    for (int i = 0; i < count; ++i) pdf[i] = tree_pdf_edge(q, edges[i], nullptr);
    return ORC_OK;
}

int orc_edge_tree_sample(const orc_scene* sd, const orc_camera* c, const double p[3], const double n[3], int32_t count,
                         const double* u, int32_t* edge, double* pdf) {
    Scn s;
    ETree t;
    int rc = tree_setup(sd, c, s, t);
    if (rc) return rc;
    TreeQuery q{&s, &t, V3d{p[0], p[1], p[2]}, V3d{n[0], n[1], n[2]}, -1};
    for (int i = 0; i < count; ++i) {
        const double* ui = u + (size_t)i * (kMaxLevels + 1);
        double pd = 0;
        edge[i] = tree_sample(q, ui[0], [&](int lev) { return ui[1 + lev]; }, pd, nullptr);
        pdf[i] = edge[i] >= 0 ? pd : 0;
    }
    return ORC_OK;
}

int orc_edge_tree_select(const orc_scene* sd, const orc_camera* c, const double p[3], const double n[3], int32_t M,
                         int32_t count, const double* u, int32_t ustride, int32_t* edge, double* weight) {
    Scn s;
    ETree t;
    int rc = tree_setup(sd, c, s, t);
    if (rc) return rc;
    if (M < 1 || ustride < 1) return ORC_EINVAL;
    TreeQuery q{&s, &t, V3d{p[0], p[1], p[2]}, V3d{n[0], n[1], n[2]}, -1};
    for (int i = 0; i < count; ++i) {
        const double* ui = u + (size_t)i * ustride;
        int k = 0;
        bool over = false;
        auto next_u = [&]() {
            if (k >= ustride) { over = true; return 0.5; }
            return ui[k++];
        };
        double w = 0;
        edge[i] = tree_select(q, M, next_u, w, nullptr);
        if (over) return ORC_EINVAL;
        weight[i] = edge[i] >= 0 ? w : 0;
    }
    return ORC_OK;
}

double orc_edge_nee_width(const orc_scene* sd) {
    Scn s;
    if (prepare(sd, s)) return -1;
    return nee_width_default(s);
}

int orc_edge_nee_sample(const orc_scene* sd, const double p[3], const double n[3], int32_t tri, double width,
                        int32_t count, uint64_t seed, int32_t* edge, double* t, double* sv, uint8_t* flags) {
    Scn s;
    int rc = prepare(sd, s);
    if (rc) return rc;
    if (!(width > 0) || tri < -1 || tri >= s.T) return ORC_EINVAL;
    NeeQuery q{&s, V3d{p[0], p[1], p[2]}, V3d{n[0], n[1], n[2]}, tri, width};
    for (int i = 0; i < count; ++i) {
        Stream rn{(uint32_t)i, 0, TAG_ENEE, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
        double c0[4];
        rn.block(0, c0);
        Unit U;
        t[i] = sv[i] = 0;
        int lt;
        edge[i] = nee_sample(q, c0 + 1, rn, t[i], sv[i], lt, &U);
        if (flags) flags[i] = U.flag;
    }
    return ORC_OK;
}

int orc_edge_nee_pdf(const orc_scene* sd, const double p[3], const double n[3], int32_t tri, double width,
                     int32_t count, const int32_t* edge, const double* t, const double* sv, double* pdf) {
    Scn s;
    int rc = prepare(sd, s);
    if (rc) return rc;
    if (!(width > 0) || tri < -1 || tri >= s.T) return ORC_EINVAL;
    NeeQuery q{&s, V3d{p[0], p[1], p[2]}, V3d{n[0], n[1], n[2]}, tri, width};
    for (int i = 0; i < count; ++i) {
        if (edge[i] < 0 || edge[i] >= (int)s.edges.size()) return ORC_EINVAL;
        pdf[i] = nee_pdf(q, edge[i], t[i], sv[i], -1, nullptr);
    }
    return ORC_OK;
}

int orc_edge_nee_mix_sample(const orc_scene* sd, const orc_camera* c, const double p[3], const double n[3],
                            int32_t tri, double width, double alpha, int32_t count, uint64_t seed, int32_t* edge,
                            double* t, double* pdf) {
    Scn s;
    ETree et;
    int rc = tree_setup(sd, c, s, et);
    if (rc) return rc;
    if (!(width > 0) || !(alpha >= 0 && alpha < 1) || tri < -1 || tri >= s.T) return ORC_EINVAL;
    TreeQuery q{&s, &et, V3d{p[0], p[1], p[2]}, V3d{n[0], n[1], n[2]}, tri};
    uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
    for (int i = 0; i < count; ++i) {
        Stream rk{(uint32_t)i, 0, TAG_SEDGE + 1, k0, k1};
        Stream rn{(uint32_t)i, 0, TAG_ENEE + 1, k0, k1};
        t[i] = pdf[i] = 0;
        edge[i] = nee_mix_draw(q, width, alpha, rk, rn, t[i], pdf[i], nullptr);
    }
    return ORC_OK;
}

void orc_secondary_forms(const double p_[3], const double v0_[3], const double v1_[3], double t, const double m0_[3],
                         const double nm_[3], double area_form[9], double dir_form[9]) {
    V3d p{p_[0], p_[1], p_[2]}, v0{v0_[0], v0_[1], v0_[2]}, v1{v1_[0], v1_[1], v1_[2]};
    V3d m0{m0_[0], m0_[1], m0_[2]}, nm{nm_[0], nm_[1], nm_[2]};
    nm = normalize(nm);
    V3d e = v1 - v0;
    V3d w = v0 + e * t - p;                       // omega(t), unnormalised
    V3d v0p = v0 - p, v1p = v1 - p;
    V3d c = cross(v0p, v1p);
    double cn = length(c);
    V3d nh = c / cn;
    // thesis form: m on the plane behind the edge, alpha(p,m) = (m-p).(v0-p)x(v1-p)
    double tau = dot(m0 - p, nm) / dot(w, nm);
    V3d mp = w * tau;                             // m - p
    V3d Jm = (e - w * (dot(e, nm) / dot(w, nm))) * tau;
    double sc = length(Jm) / (cn * length(cross(nm, nh)));
    V3d g0 = cross(v1p, mp), g1 = cross(mp, v0p);
    V3d gp = cross(v0p, v1p) * -1.0 + cross(mp, v1p) + cross(v0p, mp);   // m held fixed
    V3d af[3] = {g0 * sc, g1 * sc, gp * sc};
    // direction form: beta(w^) = w^.(v0-p)x(v1-p)
    double wl = length(w);
    V3d wh = w / wl;
    double sd = length(cross(e, wh)) / (cn * wl);
    V3d h0 = cross(v1p, wh), h1 = cross(wh, v0p), hp = cross(wh, v1p) + cross(v0p, wh);
    V3d df[3] = {h0 * sd, h1 * sd, hp * sd};
    for (int i = 0; i < 3; ++i) {
        area_form[3 * i] = af[i].x; area_form[3 * i + 1] = af[i].y; area_form[3 * i + 2] = af[i].z;
        dir_form[3 * i] = df[i].x; dir_form[3 * i + 1] = df[i].y; dir_form[3 * i + 2] = df[i].z;
    }
}

int orc_render(const orc_scene* sd, const orc_camera* oc, const orc_options* o, orc_outputs* out) {
    if (!oc || !o || !out) return ORC_EINVAL;
    if (o->aov < 0 || o->aov > 7) return ORC_EINVAL;
    if (o->spp <= 0 || o->max_depth < 0 || o->max_depth > 8) return ORC_EINVAL;
    if (oc->width <= 0 || oc->height <= 0 || oc->win_x0 < 0 || oc->win_y0 < 0 || oc->win_x1 > oc->width ||
        oc->win_y1 > oc->height || oc->win_x0 >= oc->win_x1 || oc->win_y0 >= oc->win_y1)
        return ORC_EINVAL;
    Scn s;
    int rc = prepare(sd, s);
    if (rc) return rc;
    s.use_bvh = o->use_bvh != 0;
    View vw;
    build_view(s, *oc, vw);
    ETree et;
    bool need_tree = o->secondary_edges && o->max_depth >= 1 && out->d_image && !o->aov;
    if (need_tree) {
        rc = build_etree(s, vw.cam.c, et);
        if (rc) return rc;
    }
    Ctx C;
    C.s = &s; C.oc = oc; C.o = o; C.vw = &vw; C.et = need_tree ? &et : nullptr;
    bool mix = o->edge_pdf && o->mix > 0;
    if (mix && !(o->mix < 1)) return ORC_EINVAL;
    // several samples per descent: up to 64, not with the proposal mixture
    // (the kept edge has no closed-form probability to mix with)
    if (o->edge_candidates < 0 || o->edge_candidates > 64) return ORC_EINVAL;
    if (o->edge_candidates > 1 && mix && (o->mix_terms & 2)) return ORC_EINVAL;
    // billboard strategy: alpha in [0, 1), uniform edge points, one descent
    if (!(o->enee >= 0 && o->enee < 1) || !(o->enee_width >= 0)) return ORC_EINVAL;
    if (o->enee > 0 && (o->edge_t_mode != 0 || o->edge_candidates > 1 || (mix && (o->mix_terms & 2))))
        return ORC_EINVAL;
    C.nee_w = o->enee_width > 0 ? o->enee_width : nee_width_default(s);
    C.mix_p = mix && (o->mix_terms & 1);
    C.mix_s = mix && (o->mix_terms & 2) && need_tree;
    if (C.mix_p) build_view_mix(vw, o->edge_pdf, o->mix, vw);
    if (C.mix_s) {
        C.qcdf.assign(s.edges.size(), 0.0);
        double acc = 0;
        for (size_t i = 0; i < s.edges.size(); ++i) { acc += o->edge_pdf[i]; C.qcdf[i] = acc; }
        for (double& x : C.qcdf) x /= acc;
    }
    C.harvest = out->edge_stats != nullptr && out->d_image != nullptr;
    C.d_image = out->d_image;
    C.Ww = oc->win_x1 - oc->win_x0; C.Hw = oc->win_y1 - oc->win_y0;
    C.spp = o->spp;
    C.M = C.Ww * C.Hw * C.spp;
    C.V = s.V; C.T = s.T;
    C.k0 = (uint32_t)(o->seed & 0xffffffffu); C.k1 = (uint32_t)(o->seed >> 32);
    int np = 3 * s.V + s.T + 9;
    int nth = o->num_threads > 0 ? o->num_threads : 1;
    std::vector<Acc> accs(nth);
    for (Acc& a : accs) {
        if (out->image) a.img.assign((size_t)C.Ww * C.Hw, 0.0);
        a.g.assign(np, 0.0);
        a.mass.assign(np, 0.0);
        if (C.harvest) { a.es.assign(s.edges.size(), 0.0); a.esm.assign(s.edges.size(), 0.0); }
    }
#ifdef _OPENMP
#pragma omp parallel for num_threads(nth) schedule(dynamic, 64)
#endif
    for (int m = 0; m < C.M; ++m) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        if (out->unit_flags) {
            Acc& a = accs[tid];
            int64_t before = a.flagged;
            run_unit(C, m, a);
            out->unit_flags[m] = a.flagged != before ? 1 : 0;
        } else {
            run_unit(C, m, accs[tid]);
        }
    }
    Acc tot;
    tot.img.assign(out->image ? (size_t)C.Ww * C.Hw : 0, 0.0);
    tot.g.assign(np, 0.0);
    tot.mass.assign(np, 0.0);
    for (Acc& a : accs) {
        for (size_t i = 0; i < tot.img.size(); ++i) tot.img[i] += a.img[i];
        for (int i = 0; i < np; ++i) { tot.g[i] += a.g[i]; tot.mass[i] += a.mass[i]; }
        tot.rays += a.rays; tot.flagged += a.flagged; tot.pedge += a.pedge; tot.sedge += a.sedge;
    }
    if (C.harvest) {
        for (size_t i = 0; i < s.edges.size(); ++i) out->edge_stats[i] = 0;
        if (out->edge_stats_mass) for (size_t i = 0; i < s.edges.size(); ++i) out->edge_stats_mass[i] = 0;
        for (Acc& a : accs)
            for (size_t i = 0; i < s.edges.size(); ++i) {
                out->edge_stats[i] += a.es[i];
                if (out->edge_stats_mass) out->edge_stats_mass[i] += a.esm[i];
            }
    }
    if (out->image) for (size_t i = 0; i < tot.img.size(); ++i) out->image[i] = tot.img[i];
    if (out->d_image) {
        if (out->d_vertices) for (int i = 0; i < 3 * s.V; ++i) out->d_vertices[i] = tot.g[i];
        if (out->d_albedo) for (int i = 0; i < s.T; ++i) out->d_albedo[i] = tot.g[3 * s.V + i];
        if (out->d_camera) for (int i = 0; i < 9; ++i) out->d_camera[i] = tot.g[3 * s.V + s.T + i];
        if (out->mass_vertices) for (int i = 0; i < 3 * s.V; ++i) out->mass_vertices[i] = tot.mass[i];
        if (out->mass_albedo) for (int i = 0; i < s.T; ++i) out->mass_albedo[i] = tot.mass[3 * s.V + i];
        if (out->mass_camera) for (int i = 0; i < 9; ++i) out->mass_camera[i] = tot.mass[3 * s.V + s.T + i];
    }
    if (out->stats) {
        out->stats[0] = tot.rays; out->stats[1] = tot.flagged; out->stats[2] = tot.pedge; out->stats[3] = tot.sedge;
        out->stats[4] = vw.tie ? 1 : 0; out->stats[5] = (int64_t)s.edges.size();
        out->stats[6] = need_tree ? et.max_depth : 0; out->stats[7] = 0;
    }
    return ORC_OK;
}

}  // extern "C"
