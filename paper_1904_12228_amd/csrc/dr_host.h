// Host-side scene object and the launch entry points shared by the
// library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/diffrt.h"
#include "dr_args.h"
#include "dr_common.h"

namespace dr {

// Device buffer that grows on demand and is freed with the scene.
struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t n) {
        if (n <= bytes) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, n);
        if (e == hipSuccess) bytes = n;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

struct ViewKey {
    float cam[9], fov, nearc;
    int w, h, win[4];
    int spp, depth;
    uint64_t seed;
    uint32_t view;
    const uint8_t* mask;
    int aov;
    uint64_t version;
    bool operator==(const ViewKey& o) const;
};

}  // namespace dr

struct drScene_t {
    int V = 0, T = 0, E = 0, L = 0;
    bool smooth = false;
    int two_sided = 0;
    float background = 0.0f;
    float diag = 0.0f, tmin = 0.0f, atot = 0.0f;
    float nee_w = 0.0f;              // default strip width of next event estimation for edges
    int bvh_depth = 0;               // internal nodes on the longest root-to-leaf path
    int grad_shards = 256;           // copies of the gradient arrays (power of two; set by drSceneCreate)
    uint64_t version = 0;            // bumps on every vertex update
    // scene data
    dr::Buf P, I, N, alb, emi, tri, bvh, edges, ekind, lights, lcdf, scal, err;
    dr::Buf towned;                  // [T] int4: edges whose first face is the triangle (-1: none)
    // BVH build scratch
    dr::Buf codes, ids, codes_s, ids_s, keys64, parent, counter, sort_tmp;
    // host side of the SAH build: indices (kept from creation), vertex copy,
    // child links, parent links, triangle per leaf position
    bool sah_bvh = true;
    std::vector<int> hI;
    std::vector<float> hP;
    std::vector<int> hchild, hparent, horder;
    // per-view edge data
    dr::Buf pe, plen, pcdf, scan_tmp, ecls, epos, elist, ecode, ecode_s, elist_s, ekeys, eparent, ecounter, etree,
        ebounds, edepth;
    int n1 = 0, n2 = 0;
    int etree_nodes = 0;
    int tree_m[2] = {0, 0}, tree_base[2] = {0, 0};   // leaves and first node of H1 / H2
    // learned-proposal mixture: weights, mixture CDF of primary edges, CDF of
    // the proposal; edge-tree parent links (node << 1 | side)
    dr::Buf mixw, mcdf, qcdf, eleaf, enpar;
    dr::ViewKey tree_key{};
    bool tree_valid = false;
    // checkpoints of the last forward pass
    dr::Buf ck_tri, ck_x, ck_vis;
    dr::ViewKey ck_key{};
    bool ck_valid = false;
    // camera adjoint accumulator (f, r, u, c: 12 floats)
    dr::Buf camacc;
    // split backward: side-path queries, their radiances, per-(vertex, unit) query index, count
    dr::Buf sq, sres, sqidx, scount, svtri, svx;
    bool split_backward = true;
    dr::Buf pq, pcount;              // primary edge samples whose sides hit different triangles
    bool split_primary = true;
    // wavefront forward (DIFFRT_WAVEFRONT_FORWARD=1): per-bounce queues, their
    // counts, unit radiance; off by default (18.3 ms against the single
    // kernel's 15.2 ms at config 3)
    dr::Buf fq, fcount, fL;
    bool wavefront_forward = false;
    hipStream_t last_stream = nullptr;
    int device = 0;
    // measurement
    bool prof_events = false, prof_counters = false;
    struct EvPair { hipEvent_t a, b; int kind; };
    std::vector<EvPair> evs;
    dr::Buf counters;                  // [8] uint64
    int64_t launches[3] = {0, 0, 0};

    dr::SceneView view() const;
};

namespace dr {

// dr_build.hip
drStatus build_scene_static(drScene_t* s, hipStream_t st);   // kinds, lights, triangles, BVH
drStatus build_view_edges(drScene_t* s, const Cam& cam, const ViewKey& key, bool need_tree, hipStream_t st);
drStatus build_view_mix(drScene_t* s, const float* q, float mix, bool primary, bool secondary, hipStream_t st);
drStatus refit_view(drScene_t* s, const Cam& cam, PEdge* pe, double* plen, double* pcdf, ETNode* nodes,
                    const int* list_s, const int* parent, const int m[2], const int base[2], int* counter, int* depth,
                    void* scan_tmp, size_t scan_bytes, hipStream_t st);
size_t refit_scan_bytes(int E);
// Stores (check = 0) or checks (check = 1, raising *stale) every batch view's
// edge classes against its kept hierarchy; cls is [n][E].
drStatus launch_batch_class(drScene_t* s, const BatchView* views, int n, uint8_t* cls, int check, int* stale,
                            hipStream_t st);
drStatus refit_scene(drScene_t* s, const float* vertices, hipStream_t st);
drStatus refresh_edge_kinds(drScene_t* s, hipStream_t st);
Cam make_cam(const drCamera& c);

// dr_render.hip
drStatus launch_forward(drScene_t* s, const Cam& cam, const drRenderOptions& o, float* image, hipStream_t st);
drStatus launch_backward(drScene_t* s, const Cam& cam, const drRenderOptions& o, const float* d_image,
                         float* d_vertices, float* d_albedo, float* d_camera, hipStream_t st);
RenderArgs render_args(drScene_t* s, const Cam& cam, const drRenderOptions& o);
drStatus launch_batch_forward(drScene_t* s, BatchLaunch L, int ctas, int max_pixels, hipStream_t st);
drStatus launch_batch_backward(drScene_t* s, BatchLaunch L, int ctas, int depth, float* shard, float* d_vertices,
                               float* d_albedo, float* d_cameras, hipStream_t st);
drStatus launch_batch_seed(BatchView* views, int n, uint32_t add, hipStream_t st);

}  // namespace dr

// dr_api.hip: argument checks and the per-view cache key
dr::ViewKey make_key(const drScene_t* s, const drCamera& c, const drRenderOptions& o);
bool valid_camera(const drCamera* c);
bool valid_options(const drRenderOptions* o);
