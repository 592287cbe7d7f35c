// Device-side building blocks of the gfx950 path tracer: small vector math,
// Philox4x32-10, the scene/view structures the kernels read, and the
// constants of the estimator.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dr {

// ---------------------------------------------------------------------------
// Constants of the estimator (thesis Ch. 5 leaves these open; the values are
// a fixed reading shared with the CPU oracle by specification).
// ---------------------------------------------------------------------------
constexpr float kEpsPx = 1e-3f;       // primary: offset of the two sides, pixels
constexpr float kEps3 = 1e-4f;        // secondary: angular offset of the two sides
constexpr float kTminRel = 1e-4f;     // secondary rays start at this * scene diagonal
constexpr float kShadowEnd = 1e-4f;   // shadow rays stop at (1 - this) * distance
constexpr float kInsidePad = 1e-4f;   // edge tree: parent box grown by this * diagonal
constexpr float kHorizon = 1e-5f;     // edge points this * diagonal below/at the tangent plane are skipped
constexpr float kVsphereMargin = 1e-5f;  // v-sphere pruning only beyond this relative margin
constexpr float kPi = 3.14159265358979323846f;
constexpr int kMaxDepth = 6;
constexpr int kMaxTriangles = 1 << 26;  // 64 B tree nodes and 48 B triangle records stay below 4 GiB
constexpr int kQueueBlocks = 10240;     // persistent grid of the kernels that drain a work queue: two rounds of
                                        // the 5,120 one-wave blocks resident at five waves per SIMD
constexpr int kSmallStack = 24;        // short traversal stack (entries per lane), for BVHs at most 24 deep:
                                        // 6 KB of LDS per one-wave block
constexpr int kStackDepth = 64;       // largest BVH traversal stack (entries per lane)
constexpr int kMaxLevels = 64;        // edge-tree descent levels (16 Philox blocks x 4)
constexpr int kSideBlockBase = 32;    // Philox block base of secondary side paths
constexpr uint32_t kTagCam = 0, kTagPedge = 1, kTagSedge = 1;  // SEDGE_k = 1 + k
constexpr uint32_t kTagSelect = 16;     // SELECT_k = 16 + k: uniforms of the multi-sample edge selection
constexpr int kSelectMax = 16;          // largest number of samples of the multi-sample edge selection
constexpr uint32_t kTagEnee = 32;       // ENEE_k = 32 + k: uniforms of next event estimation for edges
constexpr float kStripPad = 0.5005f;    // hierarchy boxes grown by this x strip width when walking a segment
constexpr float kWalkPad = 1e-5f;       // ... plus this x scene diagonal (FP32 rounding of the boxes)

// ---------------------------------------------------------------------------
// vector math
// ---------------------------------------------------------------------------
struct v3 { float x, y, z; };
__host__ __device__ inline v3 mk(float x, float y, float z) { return {x, y, z}; }
__host__ __device__ inline v3 operator+(v3 a, v3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__host__ __device__ inline v3 operator-(v3 a, v3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__host__ __device__ inline v3 operator-(v3 a) { return {-a.x, -a.y, -a.z}; }
__host__ __device__ inline v3 operator*(v3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__host__ __device__ inline v3 operator*(float s, v3 a) { return {a.x * s, a.y * s, a.z * s}; }
__host__ __device__ inline v3& operator+=(v3& a, v3 b) { a.x += b.x; a.y += b.y; a.z += b.z; return a; }
__host__ __device__ inline v3& operator-=(v3& a, v3 b) { a.x -= b.x; a.y -= b.y; a.z -= b.z; return a; }
__host__ __device__ inline float dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__host__ __device__ inline v3 cross(v3 a, v3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline float len(v3 a) { return sqrtf(dot(a, a)); }
__device__ inline v3 nrm(v3 a) { return a * (1.0f / sqrtf(dot(a, a))); }
// adjoint of y = v/|v|: returns dL/dv given dL/dy
__device__ inline v3 nrm_adj(v3 v, v3 gy) {
    float il = 1.0f / sqrtf(dot(v, v));
    v3 y = v * il;
    return (gy - y * dot(y, gy)) * il;
}
__device__ inline v3 ld3(const float* p, int i) { return {p[3 * i], p[3 * i + 1], p[3 * i + 2]}; }
__device__ inline float vmin(v3 a) { return fminf(a.x, fminf(a.y, a.z)); }

// Orthonormal basis around unit n (Duff et al. 2017, "Building an
// Orthonormal Basis, Revisited").
__device__ inline void onb(v3 n, v3& t1, v3& t2) {
    float sign = copysignf(1.0f, n.z);
    float a = -1.0f / (sign + n.z);
    float b = n.x * n.y * a;
    t1 = {1.0f + sign * n.x * n.x * a, sign * b, -sign * n.x};
    t2 = {b, sign + n.y * n.y * a, -n.y};
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11). Counter = (sample id, view, tag,
// block), key = seed. Uniforms u = (x >> 8) * 2^-24.
// ---------------------------------------------------------------------------
__device__ inline uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

struct Rng {
    uint32_t sid, view, tag, k0, k1;
    __device__ inline float4 block(uint32_t b) const {
        uint4 o = philox(make_uint4(sid, view, tag, b), k0, k1);
        const float s = 1.0f / 16777216.0f;
        return make_float4((o.x >> 8) * s, (o.y >> 8) * s, (o.z >> 8) * s, (o.w >> 8) * s);
    }
};

// ---------------------------------------------------------------------------
// Device views of the scene and of one camera view
// ---------------------------------------------------------------------------
struct BvhNode {          // 64 B: both children's boxes + child links
    float4 a;             // lo_l.xyz, hi_l.x
    float4 b;             // hi_l.yz, lo_r.xy
    float4 c;             // lo_r.z, hi_r.xyz
    int4 d;               // left, right (leaf: ~triangle id), unused
};

struct SceneView {
    int V, T, E, L;
    const float* P;          // [V][3]
    const int* I;            // [T][3]
    const float* N;          // [V][3] or null
    const float* alb;        // [T]
    const float* emi;        // [T]
    const float4* tri;       // [T][3] v0.xyz e1.x | e1.yz e2.xy | e2.z - - -
    const BvhNode* bvh;      // [T-1] (T == 1: unused)
    const int4* edges;       // [E] va, vb, f0, f1
    const int4* towned;      // [T] up to three edges whose first face is the triangle, -1 padded
    const uint8_t* ekind;    // [E] 0 never, 1 always, 2 silhouette-only
    const int* lights;       // [L]
    const double* lcdf;      // [L]
    const float* atot;       // total light area (device; updated by vertex refits)
    float diag, tmin;
    int two_sided;
    float background;
    int* err;                // sticky device error flags
    int stk_cap;             // traversal stack entries per lane in this launch (>= BVH depth)
};

struct Cam {
    v3 c, f, r, u;
    v3 look, upv;            // look-at point and up vector (for the camera adjoint)
    float th, asp, W, H, nearc;
    int x0, y0, x1, y1;      // window
};

__device__ inline v3 cam_dir(const Cam& k, float sx, float sy) {
    float nx = 2.0f * sx / k.W - 1.0f, ny = 1.0f - 2.0f * sy / k.H;
    return k.f + k.r * (nx * k.asp * k.th) + k.u * (ny * k.th);
}

// Primary edge record: A, B = projections of the two points defining the edge
// equation; Ac, Bc = the sampled segment (visible part, clipped to the window).
struct PEdge { float A[2], B[2], Ac[2], Bc[2]; };

// Edge hierarchy node: both children's data, so one fetch evaluates a split.
struct ETChild {
    float lo[3], hi[3], len;
    float hlo0[3], hhi0[3], hlo1[3], hhi1[3];
};
struct alignas(16) ETNode {
    ETChild ch[2];
    int child[2];            // >= 0: internal node index; < 0: ~edge id (leaf)
    int h2;                  // 1 if this node belongs to the Hough-space hierarchy
    int pad[3];              // 176 bytes: eleven 16-byte loads fetch a node
};
static_assert(sizeof(ETNode) == 176, "edge hierarchy node layout");

struct TreeView {
    const ETNode* nodes;     // [0] = virtual root whose children are the H1 and H2 roots
    int valid;               // 0: no edges at all
    v3 cam;
    const int* eleaf;        // [E] (node << 1 | side) holding the edge's leaf, -1 if in neither tree
    const int* enpar;        // [nodes] (parent << 1 | side) of each internal node; -1 at the virtual root
};

enum : int { kErrStack = 1, kErrTreeDepth = 2 };

// Per-lane work counters (measurement only): BVH nodes, triangles, edge-tree
// nodes, atomics, rays.
struct Work {
    uint32_t nodes = 0, tris = 0, tnodes = 0, atom = 0, rays = 0;
    __device__ void ray(uint32_t n, uint32_t t) { nodes += n; tris += t; rays += 1; }
    __device__ void tree() { ++tnodes; }
    __device__ void atomics(uint32_t n) { atom += n; }
};
// The same interface with no state: the production kernels count nothing.
struct NoWork {
    __device__ void ray(uint32_t, uint32_t) {}
    __device__ void tree() {}
    __device__ void atomics(uint32_t) {}
};

}  // namespace dr
