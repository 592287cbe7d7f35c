// C ABI of the gfx950 differentiable path tracer (see include/diffrt.h).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "dr_host.h"

using namespace dr;

#define API_CHECK(x)                                       \
    do {                                                   \
        hipError_t e_ = (x);                               \
        if (e_ != hipSuccess) return DR_ERROR_DEVICE;      \
    } while (0)
#define API_ALLOC(buf, n)                                                   \
    do {                                                                    \
        if ((buf).ensure(n) != hipSuccess) return DR_ERROR_OUT_OF_MEMORY;  \
    } while (0)

SceneView drScene_t::view() const {
    SceneView v;
    v.V = V; v.T = T; v.E = E; v.L = L;
    v.P = P.as<float>();
    v.I = I.as<int>();
    v.N = smooth ? N.as<float>() : nullptr;
    v.alb = alb.as<float>();
    v.emi = emi.as<float>();
    v.tri = tri.as<float4>();
    v.bvh = bvh.as<BvhNode>();
    v.edges = edges.as<int4>();
    v.towned = towned.as<int4>();
    v.ekind = ekind.as<uint8_t>();
    v.lights = lights.as<int>();
    v.lcdf = lcdf.as<double>();
    v.atot = scal.as<float>() + 12;
    v.diag = diag;
    v.tmin = tmin;
    v.two_sided = two_sided;
    v.background = background;
    v.err = err.as<int>();
    v.stk_cap = kStackDepth;
    return v;
}

static void release_all(drScene_t* s) {
    Buf* bufs[] = {&s->P, &s->I, &s->N, &s->alb, &s->emi, &s->tri, &s->bvh, &s->edges, &s->ekind, &s->lights, &s->lcdf,
                   &s->scal, &s->err, &s->codes, &s->ids, &s->codes_s, &s->ids_s, &s->keys64, &s->parent, &s->counter,
                   &s->sort_tmp, &s->pe, &s->plen, &s->pcdf, &s->scan_tmp, &s->ecls, &s->epos, &s->elist, &s->ecode,
                   &s->ecode_s, &s->elist_s, &s->ekeys, &s->eparent, &s->ecounter, &s->etree, &s->ebounds, &s->edepth,
                   &s->ck_tri, &s->ck_x, &s->ck_vis, &s->camacc, &s->mixw, &s->mcdf, &s->qcdf, &s->eleaf,
                   &s->enpar, &s->towned};
    for (Buf* b : bufs) b->release();
    for (Buf* b : {&s->sq, &s->sres, &s->sqidx, &s->scount, &s->svtri, &s->svx, &s->pq, &s->pcount, &s->fq, &s->fcount,
                   &s->fL})
        b->release();
    s->counters.release();
    for (auto& e : s->evs) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    s->evs.clear();
}

bool valid_camera(const drCamera* c) {
    if (!c || c->width <= 0 || c->height <= 0 || !(c->fov_y_deg > 0.0f && c->fov_y_deg < 180.0f) || !(c->near_clip > 0.0f))
        return false;
    bool full = c->window[0] == 0 && c->window[1] == 0 && c->window[2] == 0 && c->window[3] == 0;
    if (!full && (c->window[0] < 0 || c->window[1] < 0 || c->window[2] > c->width || c->window[3] > c->height ||
                  c->window[0] >= c->window[2] || c->window[1] >= c->window[3]))
        return false;
    float d[3] = {c->look_at[0] - c->position[0], c->look_at[1] - c->position[1], c->look_at[2] - c->position[2]};
    return d[0] * d[0] + d[1] * d[1] + d[2] * d[2] > 0.0f;
}

bool valid_options(const drRenderOptions* o) {
    if (!o || o->spp < 1 || o->max_depth < 0 || o->max_depth > kMaxDepth || (o->terms & ~DR_TERM_ALL) != 0) return false;
    if (!(o->edge_mix >= 0.0f && o->edge_mix < 1.0f) ||
        (o->edge_mix_terms & ~(uint32_t)(DR_TERM_PRIMARY | DR_TERM_SECONDARY)) != 0)
        return false;
    if (o->aov < 0 || o->aov > 8 || (o->aov != 0 && (o->edge_mix != 0.0f || o->edge_stats))) return false;
    if (o->edge_t_mode != 0 && o->edge_t_mode != 1) return false;
    if (o->edge_candidates < 0 || o->edge_candidates > kSelectMax) return false;
    if (!(o->edge_nee >= 0.0f && o->edge_nee < 1.0f) || !(o->edge_nee_width >= 0.0f) || !std::isfinite(o->edge_nee_width))
        return false;
    // the multi-sample selection and the strip strategy run in their own
    // sampling kernels, which the proposal-mixture / harvest kernels are not
    bool mixture = (o->edge_pdf && o->edge_mix > 0.0f) || o->edge_stats;
    if (o->edge_candidates > 1 && (o->max_depth > 3 || o->aov != 0 || mixture)) return false;
    if (o->edge_nee > 0.0f && (o->aov != 0 || o->edge_t_mode != 0 || o->edge_candidates > 1 || mixture)) return false;
    return true;
}

ViewKey make_key(const drScene_t* s, const drCamera& c, const drRenderOptions& o) {
    ViewKey k{};
    for (int i = 0; i < 3; ++i) {
        k.cam[i] = c.position[i];
        k.cam[3 + i] = c.look_at[i];
        k.cam[6 + i] = c.up[i];
    }
    k.fov = c.fov_y_deg;
    k.nearc = c.near_clip;
    k.w = c.width;
    k.h = c.height;
    for (int i = 0; i < 4; ++i) k.win[i] = c.window[i];
    k.spp = o.spp;
    k.depth = o.max_depth;
    k.seed = o.seed;
    k.view = o.view_id;
    k.mask = o.unit_mask;
    k.aov = o.aov;
    k.version = s->version;
    return k;
}

extern "C" {

const char* drGetErrorString(drStatus s) {
    switch (s) {
        case DR_SUCCESS: return "success";
        case DR_ERROR_INVALID_VALUE: return "invalid value";
        case DR_ERROR_OUT_OF_MEMORY: return "out of device memory";
        case DR_ERROR_DEVICE: return "device error";
        case DR_ERROR_UNSUPPORTED: return "unsupported scene";
        case DR_ERROR_DEGENERATE_GEOMETRY: return "degenerate triangle";
    }
    return "unknown status";
}

drStatus drSceneCreate(drScene* out, const drSceneDesc* d, hipStream_t st) {
    if (!out || !d) return DR_ERROR_INVALID_VALUE;
    *out = nullptr;
    if (d->num_vertices < 3 || d->num_triangles < 1 || !d->vertices || !d->indices || !d->albedo || !d->emission)
        return DR_ERROR_INVALID_VALUE;
    // traversal addresses triangle records and tree nodes by 32-bit byte offsets
    if (d->num_triangles > kMaxTriangles) return DR_ERROR_INVALID_VALUE;
    int V = d->num_vertices, T = d->num_triangles;
    std::vector<int> I(3 * (size_t)T);
    std::vector<float> emi(T);
    API_CHECK(hipMemcpyAsync(I.data(), d->indices, sizeof(int) * I.size(), hipMemcpyDeviceToHost, st));
    API_CHECK(hipMemcpyAsync(emi.data(), d->emission, sizeof(float) * T, hipMemcpyDeviceToHost, st));
    API_CHECK(hipStreamSynchronize(st));
    for (int v : I)
        if (v < 0 || v >= V) return DR_ERROR_INVALID_VALUE;
    for (int t = 0; t < T; ++t)
        if (I[3 * t] == I[3 * t + 1] || I[3 * t + 1] == I[3 * t + 2] || I[3 * t] == I[3 * t + 2]) return DR_ERROR_INVALID_VALUE;
    {
        // zero-area triangles have no normal and are never hit: rejected
        std::vector<float> hv(3 * (size_t)V);
        API_CHECK(hipMemcpyAsync(hv.data(), d->vertices, sizeof(float) * hv.size(), hipMemcpyDeviceToHost, st));
        API_CHECK(hipStreamSynchronize(st));
        for (float x : hv)
            if (!std::isfinite(x)) return DR_ERROR_INVALID_VALUE;
        for (int t = 0; t < T; ++t) {
            const float* a = &hv[3 * (size_t)I[3 * t]];
            const float* b = &hv[3 * (size_t)I[3 * t + 1]];
            const float* c = &hv[3 * (size_t)I[3 * t + 2]];
            float e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
            float n0 = e1[1] * e2[2] - e1[2] * e2[1], n1 = e1[2] * e2[0] - e1[0] * e2[2], n2 = e1[0] * e2[1] - e1[1] * e2[0];
            if (n0 == 0.0f && n1 == 0.0f && n2 == 0.0f) return DR_ERROR_DEGENERATE_GEOMETRY;
        }
    }
    // unique undirected edges, sorted by (min vertex, max vertex), faces in index order
    struct K { int a, b, f; };
    std::vector<K> ks;
    ks.reserve(3 * (size_t)T);
    for (int f = 0; f < T; ++f)
        for (int j = 0; j < 3; ++j) {
            int a = I[3 * f + j], b = I[3 * f + (j + 1) % 3];
            ks.push_back({std::min(a, b), std::max(a, b), f});
        }
    std::sort(ks.begin(), ks.end(), [](const K& x, const K& y) {
        if (x.a != y.a) return x.a < y.a;
        if (x.b != y.b) return x.b < y.b;
        return x.f < y.f;
    });
    std::vector<int4> edges;
    for (size_t i = 0; i < ks.size();) {
        size_t j = i;
        while (j < ks.size() && ks[j].a == ks[i].a && ks[j].b == ks[i].b) ++j;
        if (j - i > 2) return DR_ERROR_UNSUPPORTED;
        edges.push_back(make_int4(ks[i].a, ks[i].b, ks[i].f, j - i == 2 ? ks[i + 1].f : -1));
        i = j;
    }
    // per triangle, the edges it is the first face of (each edge once)
    std::vector<int4> towned((size_t)T, make_int4(-1, -1, -1, -1));
    for (size_t i = 0; i < edges.size(); ++i) {
        int4& o = towned[(size_t)edges[i].z];
        if (o.x < 0) o.x = (int)i;
        else if (o.y < 0) o.y = (int)i;
        else o.z = (int)i;
    }
    std::vector<int> lights;
    for (int t = 0; t < T; ++t)
        if (emi[t] > 0.0f) lights.push_back(t);
    drScene_t* s = new drScene_t();
    s->V = V;
    s->T = T;
    s->E = (int)edges.size();
    s->L = (int)lights.size();
    s->smooth = d->normals != nullptr;
    s->two_sided = d->emission_two_sided ? 1 : 0;
    s->background = d->background;
    if (const char* e = std::getenv("DIFFRT_SPLIT_BACKWARD")) s->split_backward = std::atoi(e) != 0;
    if (const char* e = std::getenv("DIFFRT_SPLIT_PRIMARY")) s->split_primary = std::atoi(e) != 0;
    if (const char* e = std::getenv("DIFFRT_WAVEFRONT_FORWARD")) s->wavefront_forward = std::atoi(e) != 0;
    // triangle BVH topology: binned SAH on the host (default) or Morton-code LBVH on the device
    if (const char* e = std::getenv("DIFFRT_BVH")) s->sah_bvh = std::strcmp(e, "lbvh") != 0;
    s->hI = I;
    // gradient copies: FP32 atomics are performed beyond the L2, where updates
    // of one address serialise; 256 copies spread the hot entries (large
    // triangles hit by many paths), halved while all copies exceed 256 MiB
    {
        long copy_bytes = 4L * (3L * V + T);
        int k = 256;
        while (k > 1 && (long)k * copy_bytes > (256L << 20)) k >>= 1;
        s->grad_shards = k;
    }
    if (const char* e = std::getenv("DIFFRT_GRAD_SHARDS")) {
        int k = std::atoi(e);
        if (k >= 1 && k <= 1024 && (k & (k - 1)) == 0) s->grad_shards = k;
    }
    API_CHECK(hipGetDevice(&s->device));
    auto fail = [&](drStatus e) {
        release_all(s);
        delete s;
        return e;
    };
#define TRY_ALLOC(buf, n) \
    if ((buf).ensure(n) != hipSuccess) return fail(DR_ERROR_OUT_OF_MEMORY)
    TRY_ALLOC(s->P, sizeof(float) * 3 * V);
    TRY_ALLOC(s->I, sizeof(int) * 3 * T);
    if (s->smooth) TRY_ALLOC(s->N, sizeof(float) * 3 * V);
    TRY_ALLOC(s->alb, sizeof(float) * T);
    TRY_ALLOC(s->emi, sizeof(float) * T);
    TRY_ALLOC(s->tri, sizeof(float4) * 3 * T);
    TRY_ALLOC(s->bvh, sizeof(BvhNode) * std::max(T - 1, 1));
    TRY_ALLOC(s->edges, sizeof(int4) * s->E);
    TRY_ALLOC(s->towned, sizeof(int4) * T);
    TRY_ALLOC(s->ekind, std::max(s->E, 1));
    TRY_ALLOC(s->lights, sizeof(int) * std::max(s->L, 1));
    TRY_ALLOC(s->lcdf, sizeof(double) * std::max(s->L, 1));
    TRY_ALLOC(s->scal, sizeof(float) * 16);
    TRY_ALLOC(s->err, sizeof(int));
    TRY_ALLOC(s->codes, sizeof(uint32_t) * T);
    TRY_ALLOC(s->ids, sizeof(int) * T);
    TRY_ALLOC(s->codes_s, sizeof(uint32_t) * T);
    TRY_ALLOC(s->ids_s, sizeof(int) * T);
    TRY_ALLOC(s->keys64, sizeof(uint64_t) * T);
    TRY_ALLOC(s->parent, sizeof(int) * 2 * T);
    TRY_ALLOC(s->counter, sizeof(int2) * T);
#undef TRY_ALLOC
    if (hipMemcpyAsync(s->P.p, d->vertices, sizeof(float) * 3 * V, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(s->I.p, I.data(), sizeof(int) * 3 * T, hipMemcpyHostToDevice, st) != hipSuccess ||
        (s->smooth && hipMemcpyAsync(s->N.p, d->normals, sizeof(float) * 3 * V, hipMemcpyDeviceToDevice, st) != hipSuccess) ||
        hipMemcpyAsync(s->alb.p, d->albedo, sizeof(float) * T, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(s->emi.p, d->emission, sizeof(float) * T, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(s->edges.p, edges.data(), sizeof(int4) * s->E, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(s->towned.p, towned.data(), sizeof(int4) * T, hipMemcpyHostToDevice, st) != hipSuccess ||
        (s->L && hipMemcpyAsync(s->lights.p, lights.data(), sizeof(int) * s->L, hipMemcpyHostToDevice, st) != hipSuccess) ||
        hipMemsetAsync(s->err.p, 0, sizeof(int), st) != hipSuccess)
        return fail(DR_ERROR_DEVICE);
    drStatus r = build_scene_static(s, st);
    if (r != DR_SUCCESS) return fail(r);
    s->last_stream = st;
    *out = s;
    return DR_SUCCESS;
}

drStatus drSceneUpdateVertices(drScene s, const float* vertices, hipStream_t st) {
    if (!s || !vertices) return DR_ERROR_INVALID_VALUE;
    API_CHECK(hipMemcpyAsync(s->P.p, vertices, sizeof(float) * 3 * s->V, hipMemcpyDeviceToDevice, st));
    s->version++;
    s->tree_valid = false;
    s->ck_valid = false;
    s->last_stream = st;
    return build_scene_static(s, st);
}

drStatus drSceneUpdateAlbedo(drScene s, const float* albedo, hipStream_t st) {
    if (!s || !albedo) return DR_ERROR_INVALID_VALUE;
    API_CHECK(hipMemcpyAsync(s->alb.p, albedo, sizeof(float) * s->T, hipMemcpyDeviceToDevice, st));
    // edge kinds depend on the albedos of the two faces (paths read the
    // albedos at every hit; nothing else depends on them)
    s->version++;
    s->tree_valid = false;
    s->ck_valid = false;
    s->last_stream = st;
    return refresh_edge_kinds(s, st);
}

drStatus drSceneGetInfo(drScene s, int32_t* nv, int32_t* nt, int32_t* ne) {
    if (!s) return DR_ERROR_INVALID_VALUE;
    if (nv) *nv = s->V;
    if (nt) *nt = s->T;
    if (ne) *ne = s->E;
    return DR_SUCCESS;
}

static drStatus ensure_checkpoints(drScene s, long M) {
    if (s->ck_tri.ensure(sizeof(int) * 3 * (size_t)M) != hipSuccess ||
        s->ck_x.ensure(sizeof(float) * 9 * (size_t)M) != hipSuccess || s->ck_vis.ensure((size_t)M) != hipSuccess)
        return DR_ERROR_OUT_OF_MEMORY;
    return DR_SUCCESS;
}

drStatus drRender(drScene s, const drCamera* c, const drRenderOptions* o, float* image, hipStream_t st) {
    if (!s || !valid_camera(c) || !valid_options(o) || !image) return DR_ERROR_INVALID_VALUE;
    Cam cam = make_cam(*c);
    long M = (long)(cam.x1 - cam.x0) * (cam.y1 - cam.y0) * o->spp;
    if (M >= (1L << 31)) return DR_ERROR_INVALID_VALUE;
    drStatus r = ensure_checkpoints(s, M);
    if (r != DR_SUCCESS) return r;
    r = launch_forward(s, cam, *o, image, st);
    if (r != DR_SUCCESS) return r;
    s->ck_key = make_key(s, *c, *o);
    s->ck_valid = true;
    s->last_stream = st;
    return DR_SUCCESS;
}

drStatus drRenderBackward(drScene s, const drCamera* c, const drRenderOptions* o, const float* d_image, float* d_vertices,
                          float* d_albedo, float* d_camera, hipStream_t st) {
    if (!s || !valid_camera(c) || !valid_options(o) || !d_image) return DR_ERROR_INVALID_VALUE;
    Cam cam = make_cam(*c);
    long npix = (long)(cam.x1 - cam.x0) * (cam.y1 - cam.y0);
    long M = npix * o->spp;
    if (M >= (1L << 31)) return DR_ERROR_INVALID_VALUE;
    ViewKey key = make_key(s, *c, *o);
    drStatus r;
    if (!(s->ck_valid && s->ck_key == key)) {
        // no matching forward pass: recompute the checkpoints
        r = ensure_checkpoints(s, M);
        if (r != DR_SUCCESS) return r;
        // the forward writes every channel it renders: seven for aov = 8
        Buf img;
        if (img.ensure(sizeof(float) * npix * (o->aov == 8 ? 7 : 1)) != hipSuccess) return DR_ERROR_OUT_OF_MEMORY;
        r = launch_forward(s, cam, *o, img.as<float>(), st);
        (void)hipStreamSynchronize(st);
        img.release();
        if (r != DR_SUCCESS) return r;
        s->ck_key = key;
        s->ck_valid = true;
    }
    uint32_t terms = o->terms ? o->terms : DR_TERM_ALL;
    bool need_tree = o->max_depth >= 1 && (terms & DR_TERM_SECONDARY) && !o->aov;
    ViewKey tkey = key;
    tkey.spp = 0; tkey.seed = 0; tkey.view = 0; tkey.mask = nullptr; tkey.depth = 0; tkey.aov = 0;
    r = build_view_edges(s, cam, tkey, need_tree, st);
    if (r != DR_SUCCESS) return r;
    r = launch_backward(s, cam, *o, d_image, d_vertices, d_albedo, d_camera, st);
    s->last_stream = st;
    return r;
}

drStatus drSetProfiling(drScene s, int32_t events, int32_t counters) {
    if (!s) return DR_ERROR_INVALID_VALUE;
    s->prof_events = events != 0;
    s->prof_counters = counters != 0;
    if (s->prof_counters) {
        API_ALLOC(s->counters, 24 * sizeof(unsigned long long));
        API_CHECK(hipMemset(s->counters.p, 0, 24 * sizeof(unsigned long long)));
    }
    return DR_SUCCESS;
}

drStatus drGetProfile(drScene s, drProfile* out, int32_t reset) {
    if (!s || !out) return DR_ERROR_INVALID_VALUE;
    API_CHECK(hipStreamSynchronize(s->last_stream));
    std::memset(out, 0, sizeof(*out));
    for (auto& e : s->evs) {
        float ms = 0.0f;
        API_CHECK(hipEventElapsedTime(&ms, e.a, e.b));
        if (e.kind == 0) out->forward_ms += ms;
        else if (e.kind == 1) out->primary_ms += ms;
        else out->backward_ms += ms;
    }
    out->bvh_depth = s->bvh_depth;
    out->edge_tree_depth = -1;
    if (s->tree_valid && s->edepth.p) API_CHECK(hipMemcpy(&out->edge_tree_depth, s->edepth.p, sizeof(int), hipMemcpyDeviceToHost));
    out->forward_launches = s->launches[0];
    out->primary_launches = s->launches[1];
    out->backward_launches = s->launches[2];
    if (s->counters.p) {
        unsigned long long c[24];
        API_CHECK(hipMemcpy(c, s->counters.p, sizeof(c), hipMemcpyDeviceToHost));
        for (int k = 0; k < 3; ++k)
            for (int i = 0; i < 5; ++i) out->counts[k][i] = (int64_t)c[8 * k + i];
    }
    if (reset) {
        for (auto& e : s->evs) {
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
        s->evs.clear();
        s->launches[0] = s->launches[1] = s->launches[2] = 0;
        if (s->counters.p) API_CHECK(hipMemset(s->counters.p, 0, 24 * sizeof(unsigned long long)));
    }
    return DR_SUCCESS;
}

drStatus drGetLastDeviceError(drScene s) {
    if (!s) return DR_ERROR_INVALID_VALUE;
    int e = 0;
    API_CHECK(hipStreamSynchronize(s->last_stream));
    API_CHECK(hipMemcpy(&e, s->err.p, sizeof(int), hipMemcpyDeviceToHost));
    if (e) {
        API_CHECK(hipMemset(s->err.p, 0, sizeof(int)));
        return DR_ERROR_DEVICE;
    }
    return DR_SUCCESS;
}

drStatus drSceneDestroy(drScene s) {
    if (!s) return DR_ERROR_INVALID_VALUE;
    (void)hipStreamSynchronize(s->last_stream);
    release_all(s);
    delete s;
    return DR_SUCCESS;
}

}  // extern "C"
