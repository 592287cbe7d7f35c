// Batches of views of one scene (many cameras with their own sizes and sample
// counts): per-view primary edge tables and edge hierarchies built once, one
// kernel launch per pass for all views, and a refit path that refreshes the
// per-view tables from moved vertices with kernel launches only, so a whole
// optimisation step can be captured in a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "dr_host.h"

using namespace dr;

struct drBatch_t {
    drScene_t* s = nullptr;
    int n = 0, depth = 0;
    bool tree = false;
    std::vector<Cam> cams;
    std::vector<int> m0, m1, base0, base1;
    int total_blocks = 0, max_pixels = 0;
    int ctas = 0, chunk = 1, shards = 1;
    size_t scan_bytes = 0;
    Buf ck_tri, ck_x, ck_vis, pe, pcdf, eleaf, elist, eparent, camacc, views, boff, queue, plen, counter, depth_scr,
        scan_tmp, dv_scr;   // dv_scr: gradient copies [shards][3V + T]
    Buf cls, stale;         // [n][E] edge classes the hierarchies were built with; int flag set by refits
    std::vector<Buf> etree, enpar;
    std::vector<ViewKey> keys;
    std::vector<BatchView> hv;   // host copy of the views' arguments

    void release() {
        for (Buf* b : {&ck_tri, &ck_x, &ck_vis, &pe, &pcdf, &eleaf, &elist, &eparent, &camacc, &views, &boff, &queue, &plen,
                       &counter, &depth_scr, &scan_tmp, &dv_scr, &cls, &stale})
            b->release();
        for (auto& b : etree) b.release();
        for (auto& b : enpar) b.release();
    }
};

// Primary edge table, CDF and edge hierarchy of view v from the scene's
// current vertices, copied into the batch's buffers (same device addresses
// on every call); updates the view's host-side arguments. Synchronises.
static drStatus build_batch_view(drBatch_t* b, int v, hipStream_t st) {
    drScene_t* s = b->s;
    int E = s->E;
    const Cam& cam = b->cams[v];
    s->tree_valid = false;
    drStatus r = build_view_edges(s, cam, b->keys[v], b->tree, st);
    if (r != DR_SUCCESS) return r;
    PEdge* pe_v = b->pe.as<PEdge>() + (size_t)v * E;
    double* pcdf_v = b->pcdf.as<double>() + (size_t)v * (E + 1);
    if (hipMemcpyAsync(pe_v, s->pe.p, sizeof(PEdge) * E, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(pcdf_v, s->pcdf.p, sizeof(double) * (E + 1), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return DR_ERROR_DEVICE;
    TreeView tv{};
    tv.cam = cam.c;
    tv.valid = 0;
    int mh[2] = {0, 0}, bh[2] = {0, 0};
    if (b->tree) {
        int nn = s->etree_nodes;
        if (nn > std::max(E, 1)) return DR_ERROR_DEVICE;
        if (hipMemcpyAsync(b->etree[v].p, s->etree.p, sizeof(ETNode) * nn, hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(b->enpar[v].p, s->enpar.p, sizeof(int) * nn, hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(b->eleaf.as<int>() + (size_t)v * E, s->eleaf.p, sizeof(int) * E, hipMemcpyDeviceToDevice,
                           st) != hipSuccess ||
            hipMemcpyAsync(b->elist.as<int>() + (size_t)v * 2 * E, s->elist_s.p, sizeof(int) * 2 * E,
                           hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(b->eparent.as<int>() + (size_t)v * 4 * E, s->eparent.p, sizeof(int) * 4 * E,
                           hipMemcpyDeviceToDevice, st) != hipSuccess)
            return DR_ERROR_DEVICE;
        for (int h = 0; h < 2; ++h) { mh[h] = s->tree_m[h]; bh[h] = s->tree_base[h]; }
        tv.nodes = b->etree[v].as<ETNode>();
        tv.eleaf = b->eleaf.as<int>() + (size_t)v * E;
        tv.enpar = b->enpar[v].as<int>();
        tv.valid = (mh[0] + mh[1]) > 0 ? 1 : 0;
    }
    // the scene's buffers are overwritten by the next view: wait before reuse
    if (hipStreamSynchronize(st) != hipSuccess) return DR_ERROR_DEVICE;
    b->m0[v] = mh[0]; b->m1[v] = mh[1]; b->base0[v] = bh[0]; b->base1[v] = bh[1];
    b->hv[v].tv = tv;
    b->hv[v].pe = pe_v;
    b->hv[v].pcdf = pcdf_v;
    return DR_SUCCESS;
}

#define B_CHECK(x)                                    \
    do {                                              \
        hipError_t e_ = (x);                          \
        if (e_ != hipSuccess) return fail(DR_ERROR_DEVICE); \
    } while (0)
#define B_ALLOC(buf, bytes)                                                  \
    do {                                                                     \
        if ((buf).ensure(std::max<size_t>(bytes, 16)) != hipSuccess) return fail(DR_ERROR_OUT_OF_MEMORY); \
    } while (0)

extern "C" drStatus drBatchCreate(drBatch* out, drScene s, int32_t n, const drCamera* cams, const drRenderOptions* opts,
                                  float* const* images, const float* const* d_images, hipStream_t st) {
    if (!out) return DR_ERROR_INVALID_VALUE;
    *out = nullptr;
    if (!s || n < 1 || !cams || !opts || !images || !d_images) return DR_ERROR_INVALID_VALUE;
    for (int v = 0; v < n; ++v) {
        const drRenderOptions& o = opts[v];
        if (!valid_camera(&cams[v]) || !valid_options(&o) || !images[v] || !d_images[v]) return DR_ERROR_INVALID_VALUE;
        if (o.max_depth != opts[0].max_depth || o.edge_pdf || o.edge_stats || o.edge_mix != 0.0f || o.aov != 0 ||
            o.edge_candidates > 1 || o.edge_nee > 0.0f)
            return DR_ERROR_INVALID_VALUE;
    }
    drBatch_t* b = new drBatch_t();
    auto fail = [&](drStatus e) {
        b->release();
        delete b;
        return e;
    };
    b->s = s;
    b->n = n;
    b->depth = opts[0].max_depth;
    b->tree = b->depth >= 1 && s->E > 0;
    int E = s->E;
    std::vector<int> boff(n + 1, 0);
    std::vector<long> ck_off(n + 1, 0);
    for (int v = 0; v < n; ++v) {
        Cam cam = make_cam(cams[v]);
        long npix = (long)(cam.x1 - cam.x0) * (cam.y1 - cam.y0);
        long M = npix * opts[v].spp;
        if (M >= (1L << 31) || (long)boff[v] + (M + BS - 1) / BS >= (1L << 31)) return fail(DR_ERROR_INVALID_VALUE);
        boff[v + 1] = boff[v] + (int)((M + BS - 1) / BS);
        ck_off[v + 1] = ck_off[v] + M;
        b->max_pixels = std::max<int>(b->max_pixels, (int)npix);
        b->cams.push_back(cam);
    }
    b->total_blocks = boff[n];
    long MT = ck_off[n];
    B_ALLOC(b->ck_tri, sizeof(int) * 3 * (size_t)MT);
    B_ALLOC(b->ck_x, sizeof(float) * 9 * (size_t)MT);
    B_ALLOC(b->ck_vis, (size_t)MT);
    B_ALLOC(b->pe, sizeof(PEdge) * (size_t)n * E);
    B_ALLOC(b->pcdf, sizeof(double) * (size_t)n * (E + 1));
    B_ALLOC(b->eleaf, sizeof(int) * (size_t)n * E);
    B_ALLOC(b->elist, sizeof(int) * (size_t)n * 2 * E);
    B_ALLOC(b->eparent, sizeof(int) * (size_t)n * 4 * E);
    b->shards = s->grad_shards;
    B_ALLOC(b->camacc, sizeof(float) * 12 * (size_t)n * b->shards);
    B_ALLOC(b->views, sizeof(BatchView) * (size_t)n);
    B_ALLOC(b->boff, sizeof(int) * (size_t)(n + 1));
    B_ALLOC(b->queue, sizeof(int));
    B_ALLOC(b->plen, sizeof(double) * (size_t)std::max(E, 1));
    B_ALLOC(b->counter, sizeof(int) * (size_t)std::max(E, 1));
    B_ALLOC(b->depth_scr, sizeof(int));
    b->scan_bytes = refit_scan_bytes(std::max(E, 1));
    B_ALLOC(b->scan_tmp, b->scan_bytes);
    B_ALLOC(b->dv_scr, sizeof(float) * (size_t)b->shards * (3 * (size_t)s->V + s->T));
    b->etree.resize(n);
    b->enpar.resize(n);
    b->hv.resize(n);
    b->m0.assign(n, 0); b->m1.assign(n, 0); b->base0.assign(n, 0); b->base1.assign(n, 0);
    if (b->tree) {
        // room for the largest hierarchy pair any vertex positions can give
        // (at most E nodes), so rebuilds keep every device address
        for (int v = 0; v < n; ++v) {
            B_ALLOC(b->etree[v], sizeof(ETNode) * (size_t)std::max(E, 1));
            B_ALLOC(b->enpar[v], sizeof(int) * (size_t)std::max(E, 1));
        }
    }
    B_ALLOC(b->cls, (size_t)n * std::max(E, 1));
    B_ALLOC(b->stale, sizeof(int));
    for (int v = 0; v < n; ++v) {
        const Cam& cam = b->cams[v];
        ViewKey key = make_key(s, cams[v], opts[v]);
        key.spp = 0; key.seed = 0; key.view = 0; key.mask = nullptr; key.depth = 0;
        b->keys.push_back(key);
        RenderArgs a = render_args(s, cam, opts[v]);
        a.counters = nullptr;
        a.debug_unit = -1;
        a.ck_tri = b->ck_tri.as<int>() + 3 * ck_off[v];
        a.ck_x = b->ck_x.as<float>() + 9 * ck_off[v];
        a.ck_vis = b->ck_vis.as<uint8_t>() + ck_off[v];
        BatchView& bv = b->hv[v];
        bv.k = cam;
        bv.a = a;
        bv.image = images[v];
        bv.d_image = d_images[v];
        bv.camacc = b->camacc.as<float>() + 12 * (size_t)v * b->shards;
        bv.reduce = (BS % opts[v].spp) == 0 ? 1 : 0;
        drStatus r = build_batch_view(b, v, st);
        if (r != DR_SUCCESS) return fail(r);
    }
    s->tree_valid = false;
    B_CHECK(hipMemcpyAsync(b->views.p, b->hv.data(), sizeof(BatchView) * n, hipMemcpyHostToDevice, st));
    B_CHECK(hipMemcpyAsync(b->boff.p, boff.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, st));
    B_CHECK(hipMemsetAsync(b->stale.p, 0, sizeof(int), st));
    drStatus r = launch_batch_class(s, b->views.as<BatchView>(), n, b->cls.as<uint8_t>(), 0, b->stale.as<int>(), st);
    if (r != DR_SUCCESS) return fail(r);
    B_CHECK(hipStreamSynchronize(st));
    *out = b;
    return DR_SUCCESS;
}

static BatchLaunch batch_launch(drBatch_t* b) {
    BatchLaunch L;
    L.views = b->views.as<BatchView>();
    L.boff = b->boff.as<int>();
    L.nviews = b->n;
    L.total = b->total_blocks;
    L.chunk = b->chunk;
    L.queue = b->queue.as<int>();
    L.gshards = b->shards;
    L.gstride = 3L * b->s->V + b->s->T;
    return L;
}

extern "C" drStatus drBatchSetLaunch(drBatch b, int32_t ctas, int32_t chunk) {
    if (!b || ctas < 0 || chunk < 1 || chunk > 64) return DR_ERROR_INVALID_VALUE;
    b->ctas = ctas;
    b->chunk = chunk;
    return DR_SUCCESS;
}

extern "C" drStatus drBatchForward(drBatch b, hipStream_t st) {
    if (!b) return DR_ERROR_INVALID_VALUE;
    drStatus r = launch_batch_forward(b->s, batch_launch(b), b->ctas, b->max_pixels, st);
    b->s->last_stream = st;
    return r;
}

extern "C" drStatus drBatchBackward(drBatch b, float* d_vertices, float* d_albedo, float* d_cameras, hipStream_t st) {
    if (!b) return DR_ERROR_INVALID_VALUE;
    drStatus r = launch_batch_backward(b->s, batch_launch(b), b->ctas, b->depth, b->dv_scr.as<float>(), d_vertices,
                                       d_albedo, d_cameras, st);
    b->s->last_stream = st;
    return r;
}

extern "C" drStatus drBatchAdvanceSeed(drBatch b, hipStream_t st) {
    if (!b) return DR_ERROR_INVALID_VALUE;
    return launch_batch_seed(b->views.as<BatchView>(), b->n, 1u, st);
}

extern "C" drStatus drBatchRefit(drBatch b, hipStream_t st) {
    if (!b) return DR_ERROR_INVALID_VALUE;
    drScene_t* s = b->s;
    int E = s->E;
    if (E == 0) return DR_SUCCESS;
    for (int v = 0; v < b->n; ++v) {
        int m[2] = {b->m0[v], b->m1[v]}, base[2] = {b->base0[v], b->base1[v]};
        drStatus r = refit_view(s, b->cams[v], b->pe.as<PEdge>() + (size_t)v * E, b->plen.as<double>(),
                                b->pcdf.as<double>() + (size_t)v * (E + 1), b->tree ? b->etree[v].as<ETNode>() : nullptr,
                                b->elist.as<int>() + (size_t)v * 2 * E, b->eparent.as<int>() + (size_t)v * 4 * E, m, base,
                                b->counter.as<int>(), b->depth_scr.as<int>(), b->scan_tmp.p, b->scan_bytes, st);
        if (r != DR_SUCCESS) return r;
    }
    if (b->tree)
        return launch_batch_class(s, b->views.as<BatchView>(), b->n, b->cls.as<uint8_t>(), 1, b->stale.as<int>(), st);
    return DR_SUCCESS;
}

extern "C" drStatus drBatchCheckHierarchy(drBatch b, int32_t* rebuilt, hipStream_t st) {
    if (!b || !rebuilt) return DR_ERROR_INVALID_VALUE;
    *rebuilt = 0;
    drScene_t* s = b->s;
    int flag = 0;
    if (hipMemcpyAsync(&flag, b->stale.p, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return DR_ERROR_DEVICE;
    if (!flag || !b->tree) return DR_SUCCESS;
    for (int v = 0; v < b->n; ++v) {
        b->keys[v].version = s->version;
        drStatus r = build_batch_view(b, v, st);
        if (r != DR_SUCCESS) return r;
    }
    s->tree_valid = false;
    if (hipMemcpyAsync(b->views.p, b->hv.data(), sizeof(BatchView) * b->n, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemsetAsync(b->stale.p, 0, sizeof(int), st) != hipSuccess)
        return DR_ERROR_DEVICE;
    drStatus r = launch_batch_class(s, b->views.as<BatchView>(), b->n, b->cls.as<uint8_t>(), 0, b->stale.as<int>(), st);
    if (r != DR_SUCCESS) return r;
    if (hipStreamSynchronize(st) != hipSuccess) return DR_ERROR_DEVICE;
    *rebuilt = 1;
    return DR_SUCCESS;
}

extern "C" drStatus drBatchDestroy(drBatch b) {
    if (!b) return DR_ERROR_INVALID_VALUE;
    if (b->s) (void)hipStreamSynchronize(b->s->last_stream);
    b->release();
    delete b;
    return DR_SUCCESS;
}

extern "C" drStatus drSceneRefit(drScene s, const float* vertices, hipStream_t st) {
    if (!s || !vertices) return DR_ERROR_INVALID_VALUE;
    drStatus r = refit_scene(s, vertices, st);
    s->version++;
    s->tree_valid = false;
    s->ck_valid = false;
    s->last_stream = st;
    return r;
}
