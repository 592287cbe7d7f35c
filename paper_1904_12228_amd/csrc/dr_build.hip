// Scene setup and per-view edge data on the device:
//  - static edge classification (FP64), light area CDF (FP64), triangle SoA;
//  - triangle LBVH: Morton codes, radix sort, binary radix tree (Karras 2012),
//    bottom-up box refit with one atomic counter per node;
//  - primary edge table (Primary Visibility: candidates, near and screen
//    clipping, screen lengths) and its FP64 CDF;
//  - the two-part edge hierarchy of "Importance Sampling the Edges, Edge
//    selection": H1 = edges discontinuous from every viewpoint plus camera
//    silhouettes, H2 = the other smooth edges with Hough-space face bounds,
//    each a radix tree over Morton-ordered edge midpoints.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "dr_host.h"
#include "dr_path.h"

namespace dr {

#define DR_CHECK(x)                                  \
    do {                                             \
        hipError_t e_ = (x);                         \
        if (e_ != hipSuccess) return DR_ERROR_DEVICE; \
    } while (0)
#define DR_ALLOC(buf, n)                                        \
    do {                                                        \
        if ((buf).ensure(n) != hipSuccess) return DR_ERROR_OUT_OF_MEMORY; \
    } while (0)

static inline int blocks(long n, int bs) { return (int)((n + bs - 1) / bs); }

// ---------------------------------------------------------------------------
// static scene data
// ---------------------------------------------------------------------------

// Discontinuity class of each edge, independent of the viewpoint: 1 = always
// (boundary, albedo or emission change, flat crease), 0 = never (coplanar flat
// faces), 2 = only where it is a silhouette (smooth shading). FP64 from the
// FP32 inputs with no contraction, so the decision is reproducible.
__global__ void k_edge_kind(const int4* __restrict__ edges, int E, const float* __restrict__ P, const int* __restrict__ I,
                            const float* __restrict__ alb, const float* __restrict__ emi, int smooth,
                            uint8_t* __restrict__ kind) {
#pragma clang fp contract(off)
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E) return;
    int4 e = edges[i];
    uint8_t k;
    if (e.w < 0) k = 1;
    else if (alb[e.z] != alb[e.w] || emi[e.z] != emi[e.w]) k = 1;
    else if (!smooth) {
        double n[2][3];
        for (int f = 0; f < 2; ++f) {
            int t = f == 0 ? e.z : e.w;
            double a[3], b[3], c[3];
            for (int j = 0; j < 3; ++j) {
                a[j] = P[3 * I[3 * t] + j];
                b[j] = P[3 * I[3 * t + 1] + j];
                c[j] = P[3 * I[3 * t + 2] + j];
            }
            double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
            double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
            n[f][0] = u[1] * v[2] - u[2] * v[1];
            n[f][1] = u[2] * v[0] - u[0] * v[2];
            n[f][2] = u[0] * v[1] - u[1] * v[0];
        }
        double cx = n[0][1] * n[1][2] - n[0][2] * n[1][1];
        double cy = n[0][2] * n[1][0] - n[0][0] * n[1][2];
        double cz = n[0][0] * n[1][1] - n[0][1] * n[1][0];
        double d = n[0][0] * n[1][0] + n[0][1] * n[1][1] + n[0][2] * n[1][2];
        k = (cx == 0.0 && cy == 0.0 && cz == 0.0 && d > 0.0) ? 0 : 1;
    } else k = 2;
    kind[i] = k;
}

// Light selection CDF proportional to area (FP64), total area.
__global__ void k_light_cdf(const int* __restrict__ lights, int L, const float* __restrict__ P, const int* __restrict__ I,
                            double* __restrict__ cdf, float* __restrict__ scal) {
#pragma clang fp contract(off)
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double acc = 0.0;
    for (int i = 0; i < L; ++i) {
        int t = lights[i];
        double a[3], b[3], c[3];
        for (int j = 0; j < 3; ++j) {
            a[j] = P[3 * I[3 * t] + j];
            b[j] = P[3 * I[3 * t + 1] + j];
            c[j] = P[3 * I[3 * t + 2] + j];
        }
        double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double nx = u[1] * v[2] - u[2] * v[1], ny = u[2] * v[0] - u[0] * v[2], nz = u[0] * v[1] - u[1] * v[0];
        acc += 0.5 * sqrt(nx * nx + ny * ny + nz * nz);
        cdf[i] = acc;
    }
    for (int i = 0; i < L; ++i) cdf[i] /= acc;
    scal[12] = (float)acc;
}

__global__ void k_tri_prep(const float* __restrict__ P, const int* __restrict__ I, int T, float4* __restrict__ tri) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    v3 a = ld3(P, I[3 * t]), b = ld3(P, I[3 * t + 1]), c = ld3(P, I[3 * t + 2]);
    v3 e1 = b - a, e2 = c - a;
    tri[3 * t] = make_float4(a.x, a.y, a.z, e1.x);
    tri[3 * t + 1] = make_float4(e1.y, e1.z, e2.x, e2.y);
    tri[3 * t + 2] = make_float4(e2.z, 0.0f, 0.0f, 0.0f);
}

// Single-block reduction: centroid bounds [0..5] and vertex bounds [6..11].
__global__ void k_bounds(const float* __restrict__ P, int V, const int* __restrict__ I, int T, float* __restrict__ scal) {
    __shared__ float sh[12][256];
    float r[12];
    for (int k = 0; k < 3; ++k) { r[k] = 3e38f; r[3 + k] = -3e38f; r[6 + k] = 3e38f; r[9 + k] = -3e38f; }
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
        v3 c = (ld3(P, I[3 * t]) + ld3(P, I[3 * t + 1]) + ld3(P, I[3 * t + 2])) * (1.0f / 3.0f);
        float cv[3] = {c.x, c.y, c.z};
        for (int k = 0; k < 3; ++k) { r[k] = fminf(r[k], cv[k]); r[3 + k] = fmaxf(r[3 + k], cv[k]); }
    }
    for (int v = threadIdx.x; v < V; v += blockDim.x)
        for (int k = 0; k < 3; ++k) { r[6 + k] = fminf(r[6 + k], P[3 * v + k]); r[9 + k] = fmaxf(r[9 + k], P[3 * v + k]); }
    for (int k = 0; k < 12; ++k) sh[k][threadIdx.x] = r[k];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 12; ++k) {
                float a = sh[k][threadIdx.x], b = sh[k][threadIdx.x + s];
                bool mn = (k % 6) < 3;
                sh[k][threadIdx.x] = mn ? fminf(a, b) : fmaxf(a, b);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 12; ++k) scal[k] = sh[k][0];
}

__device__ inline uint32_t spread10(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__global__ void k_morton_tri(const float* __restrict__ P, const int* __restrict__ I, int T, const float* __restrict__ scal,
                             uint32_t* __restrict__ codes, int* __restrict__ ids) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    v3 c = (ld3(P, I[3 * t]) + ld3(P, I[3 * t + 1]) + ld3(P, I[3 * t + 2])) * (1.0f / 3.0f);
    float cv[3] = {c.x, c.y, c.z};
    uint32_t q[3];
    for (int k = 0; k < 3; ++k) {
        float ext = scal[3 + k] - scal[k];
        float f = ext > 0.0f ? (cv[k] - scal[k]) / ext * 1024.0f : 0.0f;
        q[k] = (uint32_t)fminf(fmaxf(f, 0.0f), 1023.0f);
    }
    codes[t] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    ids[t] = t;
}

__global__ void k_keys64(const uint32_t* __restrict__ codes, int n, uint64_t* __restrict__ keys) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = ((uint64_t)codes[i] << 32) | (uint64_t)i;   // ties broken by sorted position
}

__device__ inline int kdelta(const uint64_t* __restrict__ k, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    return __clzll((long long)(k[i] ^ k[j]));
}

// Binary radix tree over n unique sorted keys (Karras 2012). Internal node i
// in [0, n-2]; child refs >= 0 are internal nodes, < 0 are ~(sorted leaf
// position). parent[] holds (node << 1 | side) for internal nodes [0, n-1) and
// leaves [n-1, 2n-1); the root's entry is -1.
__global__ void k_karras(const uint64_t* __restrict__ k, int n, int2* __restrict__ child, int* __restrict__ parent) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int d = (kdelta(k, n, i, i + 1) - kdelta(k, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = kdelta(k, n, i, i - d);
    int lmax = 2;
    while (kdelta(k, n, i, i + lmax * d) > dmin) lmax *= 2;
    int l = 0;
    for (int t = lmax / 2; t >= 1; t /= 2)
        if (kdelta(k, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dn = kdelta(k, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (kdelta(k, n, i, i + (s + t) * d) > dn) s += t;
    } while (t > 1);
    int g = i + s * d + min(d, 0);
    int lc = (min(i, j) == g) ? ~g : g;
    int rc = (max(i, j) == g + 1) ? ~(g + 1) : g + 1;
    child[i] = make_int2(lc, rc);
    parent[lc < 0 ? (n - 1 + ~lc) : lc] = (i << 1) | 0;
    parent[rc < 0 ? (n - 1 + ~rc) : rc] = (i << 1) | 1;
    if (i == 0) parent[0] = -1;
}

__device__ inline float coherent_load(const float* p) {
    return __int_as_float(__atomic_load_n(reinterpret_cast<const int*>(p), __ATOMIC_RELAXED));
}

// Triangle BVH: translate child refs to triangle ids and refit boxes bottom-up.
__global__ void k_bvh_links(const int2* __restrict__ child, int n, const int* __restrict__ ids_s, BvhNode* __restrict__ nodes,
                            int* __restrict__ counter) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int2 c = child[i];
    int l = c.x < 0 ? ~ids_s[~c.x] : c.x;
    int r = c.y < 0 ? ~ids_s[~c.y] : c.y;
    nodes[i].d = make_int4(l, r, 0, 0);
    counter[i] = 0;
}

__device__ inline void bvh_slot_store(BvhNode* nd, int side, const float b[6]) {
    float* f = reinterpret_cast<float*>(nd);
    int o = side * 6;
    for (int k = 0; k < 6; ++k) f[o + k] = b[k];   // layout: lo_l.xyz hi_l.xyz lo_r.xyz hi_r.xyz
}

__global__ void k_bvh_refit(const float* __restrict__ P, const int* __restrict__ I, int n, const int* __restrict__ ids_s,
                            const int* __restrict__ parent, BvhNode* __restrict__ nodes, int* __restrict__ counter) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    int t = ids_s[g];
    v3 a = ld3(P, I[3 * t]), b = ld3(P, I[3 * t + 1]), c = ld3(P, I[3 * t + 2]);
    float box[6] = {fminf(a.x, fminf(b.x, c.x)), fminf(a.y, fminf(b.y, c.y)), fminf(a.z, fminf(b.z, c.z)),
                    fmaxf(a.x, fmaxf(b.x, c.x)), fmaxf(a.y, fmaxf(b.y, c.y)), fmaxf(a.z, fmaxf(b.z, c.z))};
    int pp = parent[n - 1 + g];
    for (int guard = 0; pp >= 0 && guard < n; ++guard) {
        int node = pp >> 1, side = pp & 1;
        bvh_slot_store(&nodes[node], side, box);
        __threadfence();
        if (atomicAdd(&counter[node], 1) == 0) return;
        __threadfence();
        const float* f = reinterpret_cast<const float*>(&nodes[node]) + (1 - side) * 6;
        for (int k = 0; k < 3; ++k) {
            box[k] = fminf(box[k], coherent_load(f + k));
            box[3 + k] = fmaxf(box[3 + k], coherent_load(f + 3 + k));
        }
        pp = parent[node];
    }
}

// Internal nodes above each leaf (the traversal stack never holds more).
__global__ void k_tree_depth(const int* __restrict__ parent, int n, float* __restrict__ out) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    int dep = 0;
    for (int q = parent[n - 1 + g]; q >= 0 && dep <= n; q = parent[q >> 1]) ++dep;
    atomicMax(reinterpret_cast<int*>(out), dep);
}

// Binned-SAH topology of the triangle BVH, built on the host: at each node the
// centroids of its triangles go into 16 bins per axis and the split between
// bins with the least surface-area cost (area x count of each child) wins;
// leaves hold one triangle. Below depth `lim`, and wherever no bin boundary
// separates the centroids, a node splits at the object median of its widest
// centroid axis instead, which bounds the depth by lim + log2(T) for any
// input. Output in the layout of the Morton path: child refs (internal node
// index, or ~leaf position), parent links (node << 1 | side; internal nodes
// [0, T-1), leaves [T-1, 2T-1); the root's is -1), triangle per leaf position.
static void sah_topology(const float* P, const int* I, int T, int lim, std::vector<int>& child,
                         std::vector<int>& parent, std::vector<int>& order) {
    constexpr int NB = 16;
    struct Tb { float lo[3], hi[3], c[3]; };
    std::vector<Tb> tb(T);
    for (int t = 0; t < T; ++t) {
        for (int k = 0; k < 3; ++k) {
            float a = P[3 * I[3 * t] + k], b = P[3 * I[3 * t + 1] + k], c = P[3 * I[3 * t + 2] + k];
            tb[t].lo[k] = std::min(a, std::min(b, c));
            tb[t].hi[k] = std::max(a, std::max(b, c));
            tb[t].c[k] = (a + b + c) * (1.0f / 3.0f);
        }
    }
    auto area = [](const float lo[3], const float hi[3]) {
        float d0 = std::max(hi[0] - lo[0], 0.0f), d1 = std::max(hi[1] - lo[1], 0.0f), d2 = std::max(hi[2] - lo[2], 0.0f);
        return d0 * d1 + d1 * d2 + d2 * d0;
    };
    child.assign(2 * (size_t)(T - 1), 0);
    parent.assign(2 * (size_t)T, -1);
    order.assign(T, 0);
    std::vector<int> ids(T);
    for (int t = 0; t < T; ++t) ids[t] = t;
    struct Task { int b0, b1, node, depth; };
    std::vector<Task> stack{{0, T, 0, 0}};
    int next_node = 1, next_leaf = 0;
    while (!stack.empty()) {
        Task k = stack.back();
        stack.pop_back();
        int n = k.b1 - k.b0;
        float clo[3] = {3e38f, 3e38f, 3e38f}, chi[3] = {-3e38f, -3e38f, -3e38f};
        for (int i = k.b0; i < k.b1; ++i)
            for (int a = 0; a < 3; ++a) {
                clo[a] = std::min(clo[a], tb[ids[i]].c[a]);
                chi[a] = std::max(chi[a], tb[ids[i]].c[a]);
            }
        auto bin = [&](int t, int a) {
            // (c - lo) / extent lies in [0, 1]: no overflow however small the extent
            float e = chi[a] - clo[a];
            int q = (int)((tb[t].c[a] - clo[a]) / e * (float)NB);
            return std::min(std::max(q, 0), NB - 1);
        };
        int mid = -1;
        if (k.depth < lim) {
            int best_a = -1, best_q = -1;
            float best = 3e38f;
            for (int a = 0; a < 3; ++a) {
                if (!(chi[a] > clo[a])) continue;
                float blo[NB][3], bhi[NB][3];
                int cnt[NB];
                for (int q = 0; q < NB; ++q) {
                    cnt[q] = 0;
                    for (int j = 0; j < 3; ++j) { blo[q][j] = 3e38f; bhi[q][j] = -3e38f; }
                }
                for (int i = k.b0; i < k.b1; ++i) {
                    int t = ids[i], q = bin(t, a);
                    ++cnt[q];
                    for (int j = 0; j < 3; ++j) {
                        blo[q][j] = std::min(blo[q][j], tb[t].lo[j]);
                        bhi[q][j] = std::max(bhi[q][j], tb[t].hi[j]);
                    }
                }
                float right[NB];
                int rc[NB];
                float lo[3] = {3e38f, 3e38f, 3e38f}, hi[3] = {-3e38f, -3e38f, -3e38f};
                int c = 0;
                for (int q = NB - 1; q >= 1; --q) {
                    for (int j = 0; j < 3; ++j) { lo[j] = std::min(lo[j], blo[q][j]); hi[j] = std::max(hi[j], bhi[q][j]); }
                    c += cnt[q];
                    right[q] = area(lo, hi);
                    rc[q] = c;
                }
                for (int j = 0; j < 3; ++j) { lo[j] = 3e38f; hi[j] = -3e38f; }
                c = 0;
                for (int q = 0; q < NB - 1; ++q) {
                    for (int j = 0; j < 3; ++j) { lo[j] = std::min(lo[j], blo[q][j]); hi[j] = std::max(hi[j], bhi[q][j]); }
                    c += cnt[q];
                    if (c == 0 || rc[q + 1] == 0) continue;
                    float cost = area(lo, hi) * (float)c + right[q + 1] * (float)rc[q + 1];
                    if (cost < best) { best = cost; best_a = a; best_q = q; }
                }
            }
            if (best_a >= 0) {
                auto it = std::partition(ids.begin() + k.b0, ids.begin() + k.b1,
                                         [&](int t) { return bin(t, best_a) <= best_q; });
                mid = (int)(it - ids.begin());
                if (mid == k.b0 || mid == k.b1) mid = -1;
            }
        }
        if (mid < 0) {
            int a = 0;
            for (int j = 1; j < 3; ++j)
                if (chi[j] - clo[j] > chi[a] - clo[a]) a = j;
            mid = k.b0 + n / 2;
            std::nth_element(ids.begin() + k.b0, ids.begin() + mid, ids.begin() + k.b1, [&](int x, int y) {
                return tb[x].c[a] < tb[y].c[a] || (tb[x].c[a] == tb[y].c[a] && x < y);
            });
        }
        int range[2][2] = {{k.b0, mid}, {mid, k.b1}};
        for (int side = 0; side < 2; ++side) {
            int a = range[side][0], b = range[side][1];
            int ref;
            if (b - a == 1) {
                int pos = next_leaf++;
                order[pos] = ids[a];
                parent[T - 1 + pos] = (k.node << 1) | side;
                ref = ~pos;
            } else {
                int nd = next_node++;
                parent[nd] = (k.node << 1) | side;
                ref = nd;
                stack.push_back({a, b, nd, k.depth + 1});
            }
            child[2 * (size_t)k.node + side] = ref;
        }
    }
}

// Default strip width of next event estimation for edges (Ch. 5, Next event
// estimation for edges): the L2 norm over the three coordinates of 2% of the
// mean absolute deviation of the vertex positions.
static float strip_width(const float* P, int V) {
    double w2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        double mean = 0.0, dev = 0.0;
        for (int v = 0; v < V; ++v) mean += P[3 * (size_t)v + k];
        mean /= V;
        for (int v = 0; v < V; ++v) dev += std::fabs(P[3 * (size_t)v + k] - mean);
        double m = 0.02 * dev / V;
        w2 += m * m;
    }
    return (float)std::sqrt(w2);
}

drStatus build_scene_static(drScene_t* s, hipStream_t st) {
    const int BS = 256;
    int T = s->T, V = s->V;
    k_edge_kind<<<blocks(s->E, BS), BS, 0, st>>>(s->edges.as<int4>(), s->E, s->P.as<float>(), s->I.as<int>(),
                                                 s->alb.as<float>(), s->emi.as<float>(), s->smooth ? 1 : 0,
                                                 s->ekind.as<uint8_t>());
    if (s->L > 0)
        k_light_cdf<<<1, 64, 0, st>>>(s->lights.as<int>(), s->L, s->P.as<float>(), s->I.as<int>(), s->lcdf.as<double>(),
                                      s->scal.as<float>());
    k_tri_prep<<<blocks(T, BS), BS, 0, st>>>(s->P.as<float>(), s->I.as<int>(), T, s->tri.as<float4>());
    k_bounds<<<1, 256, 0, st>>>(s->P.as<float>(), V, s->I.as<int>(), T, s->scal.as<float>());
    // host copy of the vertices: the SAH topology and the default strip width
    s->hP.resize(3 * (size_t)V);
    DR_CHECK(hipMemcpyAsync(s->hP.data(), s->P.p, sizeof(float) * 3 * V, hipMemcpyDeviceToHost, st));
    DR_CHECK(hipStreamSynchronize(st));
    for (float x : s->hP)
        if (!std::isfinite(x)) return DR_ERROR_INVALID_VALUE;   // no meaningful bounds or splits
    s->nee_w = strip_width(s->hP.data(), V);
    if (T > 1 && s->sah_bvh) {
        // topology on the host from the current vertices; links and boxes on the device
        int lg = 0;
        while ((1 << lg) < T) ++lg;
        sah_topology(s->hP.data(), s->hI.data(), T, std::max(56 - lg, 0), s->hchild, s->hparent, s->horder);
        DR_CHECK(hipMemcpyAsync(s->counter.p, s->hchild.data(), sizeof(int) * s->hchild.size(), hipMemcpyHostToDevice, st));
        DR_CHECK(hipMemcpyAsync(s->parent.p, s->hparent.data(), sizeof(int) * (2 * (size_t)T - 1), hipMemcpyHostToDevice,
                                st));
        DR_CHECK(hipMemcpyAsync(s->ids_s.p, s->horder.data(), sizeof(int) * T, hipMemcpyHostToDevice, st));
    } else if (T > 1) {
        k_morton_tri<<<blocks(T, BS), BS, 0, st>>>(s->P.as<float>(), s->I.as<int>(), T, s->scal.as<float>(),
                                                   s->codes.as<uint32_t>(), s->ids.as<int>());
        size_t tmp = 0;
        DR_CHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, s->codes.as<uint32_t>(), s->codes_s.as<uint32_t>(),
                                                    s->ids.as<int>(), s->ids_s.as<int>(), T, 0, 30, st));
        DR_ALLOC(s->sort_tmp, tmp);
        DR_CHECK(hipcub::DeviceRadixSort::SortPairs(s->sort_tmp.p, tmp, s->codes.as<uint32_t>(), s->codes_s.as<uint32_t>(),
                                                    s->ids.as<int>(), s->ids_s.as<int>(), T, 0, 30, st));
        k_keys64<<<blocks(T, BS), BS, 0, st>>>(s->codes_s.as<uint32_t>(), T, s->keys64.as<uint64_t>());
        // child links go to `counter` (int2 per node), then into the nodes; `ids` is reused as refit counters
        k_karras<<<blocks(T - 1, BS), BS, 0, st>>>(s->keys64.as<uint64_t>(), T, s->counter.as<int2>(), s->parent.as<int>());
    }
    if (T > 1) {
        k_bvh_links<<<blocks(T - 1, BS), BS, 0, st>>>(s->counter.as<int2>(), T, s->ids_s.as<int>(), s->bvh.as<BvhNode>(),
                                                     s->ids.as<int>());
        k_bvh_refit<<<blocks(T, BS), BS, 0, st>>>(s->P.as<float>(), s->I.as<int>(), T, s->ids_s.as<int>(),
                                                  s->parent.as<int>(), s->bvh.as<BvhNode>(), s->ids.as<int>());
        DR_CHECK(hipMemsetAsync(s->scal.as<float>() + 13, 0, sizeof(int), st));
        k_tree_depth<<<blocks(T, BS), BS, 0, st>>>(s->parent.as<int>(), T, s->scal.as<float>() + 13);
    }
    float sc[14];
    DR_CHECK(hipMemcpyAsync(sc, s->scal.p, sizeof(sc), hipMemcpyDeviceToHost, st));
    DR_CHECK(hipStreamSynchronize(st));
    float dx = sc[9] - sc[6], dy = sc[10] - sc[7], dz = sc[11] - sc[8];
    s->diag = std::sqrt(dx * dx + dy * dy + dz * dz);
    s->tmin = kTminRel * s->diag;
    s->atot = s->L > 0 ? sc[12] : 0.0f;
    int dep = 0;
    if (T > 1) std::memcpy(&dep, &sc[13], sizeof(int));
    s->bvh_depth = dep;
    return DR_SUCCESS;
}

// ---------------------------------------------------------------------------
// per-view camera
// ---------------------------------------------------------------------------
Cam make_cam(const drCamera& c) {
    Cam k;
    v3 pos = {c.position[0], c.position[1], c.position[2]};
    v3 look = {c.look_at[0], c.look_at[1], c.look_at[2]};
    v3 up = {c.up[0], c.up[1], c.up[2]};
    auto hnrm = [](v3 a) {
        float l = std::sqrt(a.x * a.x + a.y * a.y + a.z * a.z);
        return v3{a.x / l, a.y / l, a.z / l};
    };
    k.c = pos;
    k.look = look;
    k.upv = up;
    k.f = hnrm(look - pos);
    k.r = hnrm(cross(k.f, up));
    k.u = cross(k.r, k.f);
    k.th = std::tan((double)c.fov_y_deg * 3.14159265358979323846 / 360.0);
    k.W = (float)c.width;
    k.H = (float)c.height;
    k.asp = k.W / k.H;
    k.nearc = c.near_clip;
    bool full = c.window[0] == 0 && c.window[1] == 0 && c.window[2] == 0 && c.window[3] == 0;
    k.x0 = full ? 0 : c.window[0];
    k.y0 = full ? 0 : c.window[1];
    k.x1 = full ? c.width : c.window[2];
    k.y1 = full ? c.height : c.window[3];
    return k;
}

// ---------------------------------------------------------------------------
// primary edge table
// ---------------------------------------------------------------------------
// Clips the screen segment P(l) = A + l (B - A), l in [l0, l1], to the window
// (Liang-Barsky in the parameter). Points are formed from A, a point of
// moderate screen coordinates, so their FP32 error stays at the ulp of the
// window coordinates even when the segment extends far off screen.
__device__ inline bool clip_param(const float A[2], const float B[2], float l0, float l1, float x0, float y0, float x1,
                                  float y1, float o0[2], float o1[2]) {
    float dx = B[0] - A[0], dy = B[1] - A[1];
    float p[4] = {-dx, dx, -dy, dy}, q[4] = {A[0] - x0, x1 - A[0], A[1] - y0, y1 - A[1]};
    for (int i = 0; i < 4; ++i) {
        if (p[i] == 0.0f) {
            if (q[i] < 0.0f) return false;
        } else {
            float r = q[i] / p[i];
            if (p[i] < 0.0f) { if (r > l1) return false; if (r > l0) l0 = r; }
            else { if (r < l0) return false; if (r < l1) l1 = r; }
        }
    }
    o0[0] = A[0] + l0 * dx; o0[1] = A[1] + l0 * dy;
    o1[0] = A[0] + l1 * dx; o1[1] = A[1] + l1 * dy;
    return true;
}

__global__ void k_pedge(SceneView s, Cam k, PEdge* __restrict__ pe, double* __restrict__ plen) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.E) return;
    int4 e = s.edges[i];
    uint8_t kind = s.ekind[i];
    PEdge r = {};
    float len = 0.0f;
    bool disc = kind == 1 || (kind == 2 && silhouette_from(s, e, k.c));
    if (disc) {
        v3 a = ld3(s.P, e.x), b = ld3(s.P, e.y);
        float za = dot(a - k.c, k.f), zb = dot(b - k.c, k.f);
        if (!(za < k.nearc && zb < k.nearc)) {
            // the line through the projections of the alpha points (A, B) ...
            v3 aa = za < k.nearc ? alpha_point(k, a, b, za, zb) : a;
            v3 ba = zb < k.nearc ? alpha_point(k, b, a, zb, za) : b;
            project(k, aa, r.A[0], r.A[1]);
            project(k, ba, r.B[0], r.B[1]);
            // ... restricted to the part in front of the near plane
            float dx = r.B[0] - r.A[0], dy = r.B[1] - r.A[1];
            float dd = dx * dx + dy * dy;
            float l0 = 0.0f, l1 = 1.0f;
            if (za < k.nearc) {
                float px, py;
                project(k, a + (b - a) * ((k.nearc - za) / (zb - za)), px, py);
                l0 = ((px - r.A[0]) * dx + (py - r.A[1]) * dy) / dd;
            }
            if (zb < k.nearc) {
                float px, py;
                project(k, b + (a - b) * ((k.nearc - zb) / (za - zb)), px, py);
                l1 = ((px - r.A[0]) * dx + (py - r.A[1]) * dy) / dd;
            }
            if (dd > 0.0f && clip_param(r.A, r.B, l0, l1, (float)k.x0, (float)k.y0, (float)k.x1, (float)k.y1, r.Ac, r.Bc))
                len = sqrtf((r.Bc[0] - r.Ac[0]) * (r.Bc[0] - r.Ac[0]) + (r.Bc[1] - r.Ac[1]) * (r.Bc[1] - r.Ac[1]));
        }
    }
    pe[i] = r;
    plen[i] = (double)len;
}

// cdf[n] holds the total (written before); entries [0, n) become cum / total.
__global__ void k_normalize_cdf(double* __restrict__ cdf, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double tot = cdf[n];
    if (i < n && tot > 0.0) cdf[i] = cdf[i] / tot;
}

__global__ void k_store_total(const double* __restrict__ cum, int n, double* __restrict__ dst) {
    if (blockIdx.x == 0 && threadIdx.x == 0) dst[0] = cum[n - 1];
}

// ---------------------------------------------------------------------------
// edge hierarchy
// ---------------------------------------------------------------------------
__global__ void k_edge_class(SceneView s, v3 cam, int* __restrict__ f1, int* __restrict__ f2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.E) return;
    uint8_t kind = s.ekind[i];
    int c = 0;
    if (kind == 1) c = 1;
    else if (kind == 2) c = silhouette_from(s, s.edges[i], cam) ? 1 : 2;
    f1[i] = c == 1;
    f2[i] = c == 2;
}

// Class of every edge of every batch view (0 in no hierarchy, 1 first, 2
// second), computed as k_edge_class does. check = 0 stores it; check = 1
// compares with the stored class and raises *stale where the kept hierarchy
// cannot represent the current one: an edge now in the first class but kept
// outside it (missing, or pruned by the second hierarchy's test, which
// assumes a non-silhouette from the camera), or an edge now in the second
// class but in no hierarchy. Edges that left a class only waste samples.
__global__ void k_batch_class(SceneView s, const BatchView* __restrict__ views, int n, uint8_t* __restrict__ cls, int check,
                              int* __restrict__ stale) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int v = blockIdx.y;
    if (i >= s.E || v >= n) return;
    uint8_t kind = s.ekind[i];
    uint8_t c = 0;
    if (kind == 1) c = 1;
    else if (kind == 2) c = silhouette_from(s, s.edges[i], views[v].k.c) ? 1 : 2;
    uint8_t* slot = cls + (size_t)v * s.E + i;
    if (!check) {
        *slot = c;
        return;
    }
    uint8_t kept = *slot;
    if ((c == 1 && kept != 1) || (c == 2 && kept == 0)) *stale = 1;
}

__global__ void k_edge_compact(const int* __restrict__ f1, const int* __restrict__ f2, const int* __restrict__ p1,
                               const int* __restrict__ p2, int E, int* __restrict__ l1, int* __restrict__ l2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E) return;
    if (f1[i]) l1[p1[i]] = i;
    if (f2[i]) l2[p2[i]] = i;
}

// FP64 bounds of edge midpoints of one list (single block).
__global__ void k_emid_bounds(const float* __restrict__ P, const int4* __restrict__ edges, const int* __restrict__ list, int n,
                              double* __restrict__ out) {
#pragma clang fp contract(off)
    __shared__ double sh[6][256];
    double r[6] = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300};
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        int4 e = edges[list[j]];
        for (int k = 0; k < 3; ++k) {
            double m = ((double)P[3 * e.x + k] + (double)P[3 * e.y + k]) / 2.0;
            r[k] = fmin(r[k], m);
            r[3 + k] = fmax(r[3 + k], m);
        }
    }
    for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] = r[k];
    __syncthreads();
    for (int s2 = blockDim.x / 2; s2 > 0; s2 >>= 1) {
        if ((int)threadIdx.x < s2)
            for (int k = 0; k < 6; ++k) {
                double a = sh[k][threadIdx.x], b = sh[k][threadIdx.x + s2];
                sh[k][threadIdx.x] = k < 3 ? fmin(a, b) : fmax(a, b);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 6; ++k) out[k] = sh[k][0];
}

// Morton code of an edge midpoint, quantised in FP64 without contraction so
// the code is reproducible bit for bit.
__device__ inline uint32_t quantize64(double c, double lo, double hi) {
#pragma clang fp contract(off)
    if (!(hi > lo)) return 0;
    double q = (c - lo) / (hi - lo);
    q = q * 1024.0;
    double f = floor(q);
    if (f < 0.0) f = 0.0;
    if (f > 1023.0) f = 1023.0;
    return (uint32_t)f;
}

__global__ void k_emorton(const float* __restrict__ P, const int4* __restrict__ edges, const int* __restrict__ list, int n,
                          const double* __restrict__ bnd, uint32_t* __restrict__ codes) {
#pragma clang fp contract(off)
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int4 e = edges[list[j]];
    uint32_t q[3];
    for (int k = 0; k < 3; ++k) {
        double m = ((double)P[3 * e.x + k] + (double)P[3 * e.y + k]) / 2.0;
        q[k] = quantize64(m, bnd[k], bnd[3 + k]);
    }
    codes[j] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
}

// Node numbering: 0 = virtual root (children: H1 root, H2 root; 0 = empty),
// H1 internal i -> base1 + i, H2 internal i -> base2 + i.
__global__ void k_etree_links(const int2* __restrict__ child, int n, int base, int is_h2, const int* __restrict__ list_s,
                              ETNode* __restrict__ nodes, int* __restrict__ counter) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int2 c = child[i];
    ETNode* nd = &nodes[base + i];
    nd->child[0] = c.x < 0 ? ~list_s[~c.x] : base + c.x;
    nd->child[1] = c.y < 0 ? ~list_s[~c.y] : base + c.y;
    nd->h2 = is_h2;
    nd->pad[0] = nd->pad[1] = nd->pad[2] = 0;
    counter[i] = 0;
}

__device__ inline void leaf_child(const SceneView& s, int edge, int is_h2, v3 cam, ETChild& c) {
    int4 e = s.edges[edge];
    v3 a = ld3(s.P, e.x), b = ld3(s.P, e.y);
    c.lo[0] = fminf(a.x, b.x); c.lo[1] = fminf(a.y, b.y); c.lo[2] = fminf(a.z, b.z);
    c.hi[0] = fmaxf(a.x, b.x); c.hi[1] = fmaxf(a.y, b.y); c.hi[2] = fmaxf(a.z, b.z);
    c.len = len(b - a);
    for (int f = 0; f < 2; ++f) {
        v3 h = {0.0f, 0.0f, 0.0f};
        if (is_h2) {
            int face = f == 0 ? e.z : e.w;
            TriGeom g = tri_geom(s, face);
            v3 nn = nrm(cross(g.e1, g.e2));
            h = nn * dot(nn, g.p0 - cam);
        }
        float* lo = f == 0 ? c.hlo0 : c.hlo1;
        float* hi = f == 0 ? c.hhi0 : c.hhi1;
        lo[0] = hi[0] = h.x; lo[1] = hi[1] = h.y; lo[2] = hi[2] = h.z;
    }
}

__global__ void k_etree_refit(SceneView s, v3 cam, int n, int base, int root_slot, int is_h2, const int* __restrict__ list_s,
                              const int* __restrict__ parent, ETNode* __restrict__ nodes, int* __restrict__ counter,
                              int* __restrict__ depth_out) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    ETChild c;
    leaf_child(s, list_s[g], is_h2, cam, c);
    const int NF = (int)(sizeof(ETChild) / sizeof(float));
    if (n == 1) {
        nodes[0].ch[root_slot] = c;
        nodes[0].child[root_slot] = ~list_s[0];
        return;
    }
    // depth of this leaf (internal nodes above it)
    int dep = 0;
    for (int q = parent[n - 1 + g]; q >= 0 && dep <= n; q = parent[q >> 1]) ++dep;
    atomicMax(depth_out, dep);
    int pp = parent[n - 1 + g];
    for (int guard = 0; guard < n; ++guard) {
        int node = pp >> 1, side = pp & 1;
        nodes[base + node].ch[side] = c;
        __threadfence();
        if (atomicAdd(&counter[node], 1) == 0) return;
        __threadfence();
        const float* o = reinterpret_cast<const float*>(&nodes[base + node].ch[1 - side]);
        float v[NF];
        for (int k = 0; k < NF; ++k) v[k] = coherent_load(o + k);
        const ETChild& sb = *reinterpret_cast<const ETChild*>(v);
        for (int k = 0; k < 3; ++k) {
            c.lo[k] = fminf(c.lo[k], sb.lo[k]); c.hi[k] = fmaxf(c.hi[k], sb.hi[k]);
            c.hlo0[k] = fminf(c.hlo0[k], sb.hlo0[k]); c.hhi0[k] = fmaxf(c.hhi0[k], sb.hhi0[k]);
            c.hlo1[k] = fminf(c.hlo1[k], sb.hlo1[k]); c.hhi1[k] = fmaxf(c.hhi1[k], sb.hhi1[k]);
        }
        c.len = c.len + sb.len;
        pp = parent[node];
        if (pp < 0) {
            nodes[0].ch[root_slot] = c;
            nodes[0].child[root_slot] = base + node;
            return;
        }
    }
}

__global__ void k_fill_int(int* __restrict__ x, int n, int v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// Parent links of the edge hierarchy: for every child slot of every node,
// (node << 1 | side) into the child's entry (internal nodes) or the edge's
// entry (leaves). Child 0 marks an absent root.
__global__ void k_etree_parents(const ETNode* __restrict__ nodes, int nnodes, int* __restrict__ enpar,
                                int* __restrict__ eleaf) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nnodes) return;
    if (n == 0) enpar[0] = -1;
    for (int side = 0; side < 2; ++side) {
        int ch = nodes[n].child[side];
        if (ch > 0) enpar[ch] = (n << 1) | side;
        else if (ch < 0) eleaf[~ch] = (n << 1) | side;
    }
}

__global__ void k_copy_f32(const float* __restrict__ a, int n, float* __restrict__ b) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ void k_mix_weights(const double* __restrict__ plen, const double* __restrict__ ptot, const float* __restrict__ q,
                              double mix, int E, double* __restrict__ w) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E) return;
    double tot = ptot[0];
    w[i] = (1.0 - mix) * (tot > 0.0 ? plen[i] / tot : 0.0) + mix * (double)q[i];
}

__global__ void k_to_double(const float* __restrict__ q, int E, double* __restrict__ w) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < E) w[i] = (double)q[i];
}

__global__ void k_etree_root_init(ETNode* nodes) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ETNode r = {};
        r.child[0] = 0;
        r.child[1] = 0;
        r.h2 = 0;
        nodes[0] = r;
    }
}

bool ViewKey::operator==(const ViewKey& o) const {
    for (int i = 0; i < 9; ++i)
        if (cam[i] != o.cam[i]) return false;
    return fov == o.fov && nearc == o.nearc && w == o.w && h == o.h && win[0] == o.win[0] && win[1] == o.win[1] &&
           win[2] == o.win[2] && win[3] == o.win[3] && spp == o.spp && depth == o.depth && seed == o.seed &&
           view == o.view && mask == o.mask && aov == o.aov && version == o.version;
}

drStatus build_view_edges(drScene_t* s, const Cam& cam, const ViewKey& key, bool need_tree, hipStream_t st) {
    const int BS = 256;
    int E = s->E;
    SceneView sv = s->view();
    // primary edge table + CDF (cdf[E] holds the total screen length)
    DR_ALLOC(s->pe, sizeof(PEdge) * E);
    DR_ALLOC(s->plen, sizeof(double) * E);
    DR_ALLOC(s->pcdf, sizeof(double) * (E + 1));
    k_pedge<<<blocks(E, BS), BS, 0, st>>>(sv, cam, s->pe.as<PEdge>(), s->plen.as<double>());
    size_t tmp = 0;
    DR_CHECK(hipcub::DeviceScan::InclusiveSum(nullptr, tmp, s->plen.as<double>(), s->pcdf.as<double>(), E, st));
    size_t tmp2 = 0;
    DR_CHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp2, s->ecls.as<int>(), s->epos.as<int>(), E, st));
    DR_ALLOC(s->scan_tmp, std::max(tmp, tmp2) + 256);
    DR_CHECK(hipcub::DeviceScan::InclusiveSum(s->scan_tmp.p, tmp, s->plen.as<double>(), s->pcdf.as<double>(), E, st));
    k_store_total<<<1, 1, 0, st>>>(s->pcdf.as<double>(), E, s->pcdf.as<double>() + E);
    k_normalize_cdf<<<blocks(E, BS), BS, 0, st>>>(s->pcdf.as<double>(), E);
    if (!need_tree) return DR_SUCCESS;
    if (s->tree_valid && s->tree_key == key) return DR_SUCCESS;
    // classification and compaction (lists keep edge-id order)
    DR_ALLOC(s->ecls, sizeof(int) * 2 * E);
    DR_ALLOC(s->epos, sizeof(int) * 2 * (E + 1));
    DR_ALLOC(s->elist, sizeof(int) * 2 * E);
    int* f1 = s->ecls.as<int>();
    int* f2 = f1 + E;
    int* p1 = s->epos.as<int>();
    int* p2 = p1 + E + 1;
    k_edge_class<<<blocks(E, BS), BS, 0, st>>>(sv, cam.c, f1, f2);
    DR_CHECK(hipcub::DeviceScan::ExclusiveSum(s->scan_tmp.p, tmp2, f1, p1, E, st));
    DR_CHECK(hipcub::DeviceScan::ExclusiveSum(s->scan_tmp.p, tmp2, f2, p2, E, st));
    int cnt[4];
    DR_CHECK(hipMemcpyAsync(&cnt[0], p1 + E - 1, sizeof(int), hipMemcpyDeviceToHost, st));
    DR_CHECK(hipMemcpyAsync(&cnt[1], f1 + E - 1, sizeof(int), hipMemcpyDeviceToHost, st));
    DR_CHECK(hipMemcpyAsync(&cnt[2], p2 + E - 1, sizeof(int), hipMemcpyDeviceToHost, st));
    DR_CHECK(hipMemcpyAsync(&cnt[3], f2 + E - 1, sizeof(int), hipMemcpyDeviceToHost, st));
    DR_CHECK(hipStreamSynchronize(st));
    int n[2] = {cnt[0] + cnt[1], cnt[2] + cnt[3]};
    s->n1 = n[0];
    s->n2 = n[1];
    int* l1 = s->elist.as<int>();
    int* l2 = l1 + E;
    k_edge_compact<<<blocks(E, BS), BS, 0, st>>>(f1, f2, p1, p2, E, l1, l2);
    int nnodes = 1 + std::max(n[0] - 1, 0) + std::max(n[1] - 1, 0);
    DR_ALLOC(s->etree, sizeof(ETNode) * nnodes);
    DR_ALLOC(s->ecode, sizeof(uint32_t) * E);
    DR_ALLOC(s->ecode_s, sizeof(uint32_t) * E);
    DR_ALLOC(s->elist_s, sizeof(int) * 2 * E);      // per hierarchy: sorted leaves (kept for refits)
    DR_ALLOC(s->ekeys, sizeof(uint64_t) * E);
    DR_ALLOC(s->eparent, sizeof(int) * 4 * E);      // per hierarchy: parent links of 2m - 1 nodes
    DR_ALLOC(s->ecounter, sizeof(int2) * E);
    DR_ALLOC(s->ebounds, sizeof(double) * 6);
    DR_ALLOC(s->edepth, sizeof(int));
    k_etree_root_init<<<1, 1, 0, st>>>(s->etree.as<ETNode>());
    DR_CHECK(hipMemsetAsync(s->edepth.p, 0, sizeof(int), st));
    int base = 1;
    for (int h = 0; h < 2; ++h) {
        int m = n[h];
        s->tree_m[h] = m;
        s->tree_base[h] = base;
        if (m == 0) continue;
        const int* list = h == 0 ? l1 : l2;
        int* list_s = s->elist_s.as<int>() + (size_t)h * E;
        int* parent = s->eparent.as<int>() + (size_t)h * 2 * E;
        k_emid_bounds<<<1, 256, 0, st>>>(s->P.as<float>(), s->edges.as<int4>(), list, m, s->ebounds.as<double>());
        k_emorton<<<blocks(m, BS), BS, 0, st>>>(s->P.as<float>(), s->edges.as<int4>(), list, m, s->ebounds.as<double>(),
                                                s->ecode.as<uint32_t>());
        size_t stmp = 0;
        DR_CHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, stmp, s->ecode.as<uint32_t>(), s->ecode_s.as<uint32_t>(), list,
                                                    list_s, m, 0, 30, st));
        DR_ALLOC(s->sort_tmp, stmp);
        DR_CHECK(hipcub::DeviceRadixSort::SortPairs(s->sort_tmp.p, stmp, s->ecode.as<uint32_t>(), s->ecode_s.as<uint32_t>(),
                                                    list, list_s, m, 0, 30, st));
        if (m > 1) {
            k_keys64<<<blocks(m, BS), BS, 0, st>>>(s->ecode_s.as<uint32_t>(), m, s->ekeys.as<uint64_t>());
            k_karras<<<blocks(m - 1, BS), BS, 0, st>>>(s->ekeys.as<uint64_t>(), m, s->ecounter.as<int2>(), parent);
            k_etree_links<<<blocks(m - 1, BS), BS, 0, st>>>(s->ecounter.as<int2>(), m, base, h, list_s,
                                                            s->etree.as<ETNode>(), s->ecode.as<int>());
        }
        k_etree_refit<<<blocks(m, BS), BS, 0, st>>>(sv, cam.c, m, base, h, h, list_s, parent, s->etree.as<ETNode>(),
                                                    s->ecode.as<int>(), s->edepth.as<int>());
        base += std::max(m - 1, 0);
    }
    s->etree_nodes = nnodes;
    DR_ALLOC(s->eleaf, sizeof(int) * E);
    DR_ALLOC(s->enpar, sizeof(int) * nnodes);
    k_fill_int<<<blocks(E, BS), BS, 0, st>>>(s->eleaf.as<int>(), E, -1);
    k_etree_parents<<<blocks(nnodes, BS), BS, 0, st>>>(s->etree.as<ETNode>(), nnodes, s->enpar.as<int>(),
                                                       s->eleaf.as<int>());
    s->tree_key = key;
    s->tree_valid = true;
    return DR_SUCCESS;
}

// Per-view tables again from the current geometry, with the hierarchy's
// topology kept (leaf order and parent links from the last build): primary
// edge table and CDF, then the hierarchy's bounds bottom-up. Kernel launches
// only (no host synchronisation, no allocation). counter: m - 1 ints of scratch.
drStatus refit_view(drScene_t* s, const Cam& cam, PEdge* pe, double* plen, double* pcdf, ETNode* nodes,
                    const int* list_s, const int* parent, const int m[2], const int base[2], int* counter, int* depth,
                    void* scan_tmp, size_t scan_bytes, hipStream_t st) {
    const int BS = 256;
    int E = s->E;
    if (E == 0) return DR_SUCCESS;
    SceneView sv = s->view();
    k_pedge<<<blocks(E, BS), BS, 0, st>>>(sv, cam, pe, plen);
    DR_CHECK(hipcub::DeviceScan::InclusiveSum(scan_tmp, scan_bytes, plen, pcdf, E, st));
    k_store_total<<<1, 1, 0, st>>>(pcdf, E, pcdf + E);
    k_normalize_cdf<<<blocks(E, BS), BS, 0, st>>>(pcdf, E);
    if (!nodes) return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
    for (int h = 0; h < 2; ++h) {
        int mh = m[h];
        if (mh == 0) continue;
        if (mh > 1) k_fill_int<<<blocks(mh - 1, BS), BS, 0, st>>>(counter, mh - 1, 0);
        k_etree_refit<<<blocks(mh, BS), BS, 0, st>>>(sv, cam.c, mh, base[h], h, h, list_s + (size_t)h * E,
                                                     parent + (size_t)h * 2 * E, nodes, counter, depth);
    }
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}

drStatus launch_batch_class(drScene_t* s, const BatchView* views, int n, uint8_t* cls, int check, int* stale,
                            hipStream_t st) {
    if (s->E == 0 || n == 0) return DR_SUCCESS;
    dim3 g(blocks(s->E, 256), n);
    k_batch_class<<<g, 256, 0, st>>>(s->view(), views, n, cls, check, stale);
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}

size_t refit_scan_bytes(int E) {
    size_t tmp = 0;
    (void)hipcub::DeviceScan::InclusiveSum(nullptr, tmp, (double*)nullptr, (double*)nullptr, E, (hipStream_t)0);
    return tmp + 256;
}

// Vertex update without topology changes: triangle records, edge kinds,
// light CDF and area, BVH bounds over the existing tree. Kernel launches only.
drStatus refit_scene(drScene_t* s, const float* vertices, hipStream_t st) {
    const int BS = 256;
    int T = s->T, V = s->V;
    k_copy_f32<<<blocks(3 * V, BS), BS, 0, st>>>(vertices, 3 * V, s->P.as<float>());
    k_edge_kind<<<blocks(s->E, BS), BS, 0, st>>>(s->edges.as<int4>(), s->E, s->P.as<float>(), s->I.as<int>(),
                                                 s->alb.as<float>(), s->emi.as<float>(), s->smooth ? 1 : 0,
                                                 s->ekind.as<uint8_t>());
    if (s->L > 0)
        k_light_cdf<<<1, 64, 0, st>>>(s->lights.as<int>(), s->L, s->P.as<float>(), s->I.as<int>(), s->lcdf.as<double>(),
                                      s->scal.as<float>());
    k_tri_prep<<<blocks(T, BS), BS, 0, st>>>(s->P.as<float>(), s->I.as<int>(), T, s->tri.as<float4>());
    if (T > 1) {
        k_fill_int<<<blocks(T - 1, BS), BS, 0, st>>>(s->ids.as<int>(), T - 1, 0);
        k_bvh_refit<<<blocks(T, BS), BS, 0, st>>>(s->P.as<float>(), s->I.as<int>(), T, s->ids_s.as<int>(),
                                                  s->parent.as<int>(), s->bvh.as<BvhNode>(), s->ids.as<int>());
    }
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}

// Edge kinds from the current vertices and albedos (after an albedo update:
// nothing else of the scene depends on the albedos). Kernel launch only.
drStatus refresh_edge_kinds(drScene_t* s, hipStream_t st) {
    if (s->E > 0)
        k_edge_kind<<<blocks(s->E, 256), 256, 0, st>>>(s->edges.as<int4>(), s->E, s->P.as<float>(), s->I.as<int>(),
                                                       s->alb.as<float>(), s->emi.as<float>(), s->smooth ? 1 : 0,
                                                       s->ekind.as<uint8_t>());
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}

// Mixture of the primary edge pdf with the proposal q (weights, FP64 scan,
// normalised CDF with the total at [E]) and the CDF of q alone.
drStatus build_view_mix(drScene_t* s, const float* q, float mix, bool primary, bool secondary, hipStream_t st) {
    const int BS = 256;
    int E = s->E;
    if (E == 0) return DR_SUCCESS;
    DR_ALLOC(s->mixw, sizeof(double) * E);
    size_t tmp = 0;
    DR_CHECK(hipcub::DeviceScan::InclusiveSum(nullptr, tmp, s->mixw.as<double>(), s->mixw.as<double>(), E, st));
    DR_ALLOC(s->scan_tmp, tmp + 256);
    if (primary) {
        DR_ALLOC(s->mcdf, sizeof(double) * (E + 1));
        k_mix_weights<<<blocks(E, BS), BS, 0, st>>>(s->plen.as<double>(), s->pcdf.as<double>() + E, q, (double)mix, E,
                                                    s->mixw.as<double>());
        DR_CHECK(hipcub::DeviceScan::InclusiveSum(s->scan_tmp.p, tmp, s->mixw.as<double>(), s->mcdf.as<double>(), E, st));
        k_store_total<<<1, 1, 0, st>>>(s->mcdf.as<double>(), E, s->mcdf.as<double>() + E);
        k_normalize_cdf<<<blocks(E, BS), BS, 0, st>>>(s->mcdf.as<double>(), E);
    }
    if (secondary) {
        DR_ALLOC(s->qcdf, sizeof(double) * (E + 1));
        k_to_double<<<blocks(E, BS), BS, 0, st>>>(q, E, s->mixw.as<double>());
        DR_CHECK(hipcub::DeviceScan::InclusiveSum(s->scan_tmp.p, tmp, s->mixw.as<double>(), s->qcdf.as<double>(), E, st));
        k_store_total<<<1, 1, 0, st>>>(s->qcdf.as<double>(), E, s->qcdf.as<double>() + E);
        k_normalize_cdf<<<blocks(E, BS), BS, 0, st>>>(s->qcdf.as<double>(), E);
    }
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}

}  // namespace dr
