// Backward pass orchestration: gradient shards, the learned-proposal
// mixture tables, primary edge samples, path backward at the kernel depth
// that covers max_depth, shard reduction and the camera adjoint.
#include "dr_kernels.h"
#include "dr_launch.h"

namespace dr {

drStatus launch_backward(drScene_t* s, const Cam& cam, const drRenderOptions& o, const float* d_image, float* d_vertices,
                         float* d_albedo, float* d_camera, hipStream_t st) {
    RenderArgs a = make_args(s, cam, o);
    SceneView sv = s->view();
    bool sm = small_stack(s);
    sv.stk_cap = sm ? kSmallStack : kStackDepth;
    // gradients accumulate into `shards` copies (layout per copy: dV [3V] then
    // dA [T]), camera accumulators into `shards` x 12 floats; the copies are
    // summed into the caller's arrays at the end
    int shards = s->grad_shards;
    long stride = 3L * s->V + s->T;
    size_t need = sizeof(float) * (size_t)shards * (stride + 12);
    if (s->camacc.ensure(need) != hipSuccess) return DR_ERROR_OUT_OF_MEMORY;
    float* camacc = s->camacc.as<float>();
    float* dV = camacc + 12 * (size_t)shards;
    float* dA = dV + 3L * s->V;
    a.gshards = shards;
    a.gstride = stride;
    k_fill<<<nblk((long)shards * (stride + 12), 256), 256, 0, st>>>(camacc, (long)shards * (stride + 12), 0.0f);
    uint32_t terms = a.terms;
    unsigned long long* cbase = a.counters;
    // learned-proposal mixture and harvest: the MIX kernel variants (no work counters)
    bool mixing = o.edge_pdf && o.edge_mix > 0.0f;
    uint32_t mterms = o.edge_mix_terms ? o.edge_mix_terms : (DR_TERM_PRIMARY | DR_TERM_SECONDARY);
    MixArgs mx{};
    mx.q = o.edge_pdf;
    mx.mix = mixing ? o.edge_mix : 0.0f;
    mx.prim = mixing && (mterms & DR_TERM_PRIMARY) ? 1 : 0;
    mx.sec = mixing && (mterms & DR_TERM_SECONDARY) && o.max_depth >= 1 && s->tree_valid ? 1 : 0;
    mx.estats = o.edge_stats;
    mx.plen = s->plen.as<double>();
    bool use_mix = mixing || o.edge_stats;
    if (use_mix || o.aov) cbase = nullptr;
    if (o.edge_stats) k_fill<<<nblk(s->E, 256), 256, 0, st>>>(o.edge_stats, s->E, 0.0f);
    if (mx.prim || mx.sec) {
        drStatus r = build_view_mix(s, o.edge_pdf, o.edge_mix, mx.prim != 0, mx.sec != 0, st);
        if (r != DR_SUCCESS) return r;
        mx.mcdf = s->mcdf.as<double>();
        mx.qcdf = s->qcdf.as<double>();
    }
    if ((terms & DR_TERM_PRIMARY) && s->E > 0) {
        EvScope ev(s, 1, st);
        a.counters = cbase ? cbase + 8 : nullptr;
        dim3 g(nblk(a.M, BS));
        const PEdge* pe = s->pe.as<PEdge>();
        const double* pc = s->pcdf.as<double>();
Variant v{o.aov != 0, use_mix, a.counters != nullptr, sm};
        // production variant: edge samples, then a compact queue of those
        // whose two sides hit different triangles, traced densely
        int3* pq = nullptr;
        int* pcount = nullptr;
        if (s->split_primary && !v.aov && !v.counters) {
            if (s->pq.ensure(sizeof(int3) * (size_t)a.M) != hipSuccess || s->pcount.ensure(sizeof(int) * 64) != hipSuccess)
                return DR_ERROR_OUT_OF_MEMORY;
            pq = s->pq.as<int3>();
            pcount = s->pcount.as<int>();
        }
        // persistent grid of the queue kernel: two rounds of the blocks the
        // device holds at once (a grid between one and two rounds leaves the
        // second round partly empty)
        int paths_grid = std::max(1, std::min(nblk((long)a.M, BS), kQueueBlocks));
        launch_primary_kernel(v, g, sv, cam, a, pe, pc, d_image, dV, camacc, mx, pq, pcount, paths_grid, st);
    }
    if (o.aov) {
        // geometry buffer: interior term at the first hit only
        TreeView tv{};
        tv.valid = false;
        tv.cam = cam.c;
        EvScope ev(s, 2, st);
        a.counters = nullptr;
        dim3 g(nblk(a.M, BS)), b(BS);
        if (sm) k_backward<1, kSmallStack, false, false, true><<<g, b, 0, st>>>(sv, cam, a, tv, d_image, dV, dA, camacc, mx);
        else k_backward<1, kStackDepth, false, false, true><<<g, b, 0, st>>>(sv, cam, a, tv, d_image, dV, dA, camacc, mx);
    } else if (o.max_depth >= 1) {
        TreeView tv;
        tv.nodes = s->etree.as<ETNode>();
        tv.valid = (s->n1 + s->n2) > 0 && (terms & DR_TERM_SECONDARY) && s->tree_valid;
        tv.cam = cam.c;
        tv.eleaf = s->eleaf.as<int>();
        tv.enpar = s->enpar.as<int>();
        EvScope ev(s, 2, st);
        a.counters = cbase ? cbase + 16 : nullptr;
        dim3 g(nblk(a.M, BS));
        // the split kernels serve the mixture up to kernel depth 3, and the
        // multi-sample edge selection (which only they implement)
        // the strip strategy of next event estimation for edges, likewise, at
        // any depth
        if (a.cands > 1 || a.nee > 0.0f) a.counters = nullptr;
        bool split = !a.counters && s->split_backward && (!use_mix || o.max_depth <= 3);
        if (a.cands > 1 && !(split && o.max_depth <= 3)) return DR_ERROR_INVALID_VALUE;
        if (a.nee > 0.0f && !split) return DR_ERROR_INVALID_VALUE;
        SplitArgs sp{};
        // queue capacity: MAXD (the kernels' template depth: 1, 3 or 6) slots per unit
        int maxd = o.max_depth <= 1 ? 1 : (o.max_depth <= 3 ? 3 : 6);
        if (split) {
            size_t cap = (size_t)maxd * (size_t)a.M;
            // traced vertices 3 .. MAXD-1 (path vertex index kk + 1 >= 3, slot kk - 1; slot 0 unused)
            size_t vcap = (size_t)std::max(maxd - 2, 1) * (size_t)a.M;
            if (s->sq.ensure(sizeof(SideQuery) * cap) != hipSuccess || s->sres.ensure(sizeof(float2) * cap) != hipSuccess ||
                s->sqidx.ensure(sizeof(int) * cap) != hipSuccess || s->scount.ensure(sizeof(int) * 6) != hipSuccess ||
                s->svtri.ensure(sizeof(int) * vcap) != hipSuccess || s->svx.ensure(sizeof(float) * 3 * vcap) != hipSuccess)
                return DR_ERROR_OUT_OF_MEMORY;
            sp.vtri = s->svtri.as<int>();
            sp.vx = s->svx.as<float>();
            sp.q = s->sq.as<SideQuery>();
            sp.res = s->sres.as<float2>();
            sp.qidx = s->sqidx.as<int>();
            sp.count = s->scount.as<int>();
            k_fill_count<<<1, 64, 0, st>>>(sp.count, maxd);
        }
        int side_grid = std::max(1, std::min(nblk((long)a.M, BS), kQueueBlocks));
PathLaunch pl{Variant{false, use_mix, a.counters != nullptr, sm}, split, g, side_grid, o.max_depth, sv, cam, a,
                      tv, sp, d_image, dV, dA, camacc, mx};
        if (o.max_depth <= 1) {
            if (sm) launch_paths_stack<1, kSmallStack>(pl, st);
            else launch_paths_stack<1, kStackDepth>(pl, st);
        } else if (o.max_depth <= 3) {
            if (sm) launch_paths_stack<3, kSmallStack>(pl, st);
            else launch_paths_stack<3, kStackDepth>(pl, st);
        } else {
            if (sm) launch_paths_stack<6, kSmallStack>(pl, st);
            else launch_paths_stack<6, kStackDepth>(pl, st);
        }
    }
    if (d_vertices) k_reduce_shards<<<nblk(3L * s->V, kReduceEntries), 256, 0, st>>>(dV, shards, stride, 3L * s->V, d_vertices);
    if (d_albedo) k_reduce_shards<<<nblk(s->T, kReduceEntries), 256, 0, st>>>(dA, shards, stride, s->T, d_albedo);
    if (d_camera)
        k_cam_finalize<<<1, BS, 0, st>>>(cam, camacc, shards, d_camera);
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}

RenderArgs render_args(drScene_t* s, const Cam& cam, const drRenderOptions& o) { return make_args(s, cam, o); }

}  // namespace dr
