// Batches of views: one launch per pass for every view of a batch.
#include "dr_kernels.h"
#include "dr_launch.h"

namespace dr {

static int batch_grid(const BatchLaunch& L, int ctas) {
    int items = (L.total + L.chunk - 1) / L.chunk;
    return ctas > 0 ? std::max(1, std::min(ctas, items)) : std::max(1, items);
}

drStatus launch_batch_forward(drScene_t* s, BatchLaunch L, int ctas, int max_pixels, hipStream_t st) {
    SceneView sv = s->view();
    bool sm = small_stack(s);
    sv.stk_cap = sm ? kSmallStack : kStackDepth;
    dim3 zg(std::max(1, std::min((max_pixels + 255) / 256, 1024)), L.nviews);
    k_batch_zero<<<zg, 256, 0, st>>>(L.views, L.nviews, 1, L.gshards);
    if (L.total == 0) return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
    if (!(ctas > 0)) L.queue = nullptr;
    else k_fill_i32<<<1, 1, 0, st>>>(L.queue, 0);
    int grid = batch_grid(L, ctas);
    if (sm) k_forward_batch<kSmallStack><<<grid, BS, 0, st>>>(sv, L);
    else k_forward_batch<kStackDepth><<<grid, BS, 0, st>>>(sv, L);
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}

drStatus launch_batch_backward(drScene_t* s, BatchLaunch L, int ctas, int depth, float* shard, float* d_vertices,
                               float* d_albedo, float* d_cameras, hipStream_t st) {
    SceneView sv = s->view();
    bool sm = small_stack(s);
    sv.stk_cap = sm ? kSmallStack : kStackDepth;
    // `shard`: gshards copies of [dV (3V) | dA (T)], gstride = 3V + T floats apart
    float* dV = shard;
    float* dA = shard + 3L * s->V;
    k_fill<<<nblk((long)L.gshards * L.gstride, 256), 256, 0, st>>>(shard, (long)L.gshards * L.gstride, 0.0f);
    k_batch_zero<<<dim3(1, L.nviews), 64, 0, st>>>(L.views, L.nviews, 0, L.gshards);
    if (L.total > 0) {
        if (!(ctas > 0)) L.queue = nullptr;
        int grid = batch_grid(L, ctas);
        if (s->E > 0) {
            if (L.queue) k_fill_i32<<<1, 1, 0, st>>>(L.queue, 0);
            if (sm) k_primary_batch<kSmallStack><<<grid, BS, 0, st>>>(sv, L, dV);
            else k_primary_batch<kStackDepth><<<grid, BS, 0, st>>>(sv, L, dV);
        }
        if (depth >= 1) {
            if (L.queue) k_fill_i32<<<1, 1, 0, st>>>(L.queue, 0);
if (depth <= 1) launch_batch_paths<1>(sm, grid, sv, L, dV, dA, st);
            else if (depth <= 3) launch_batch_paths<3>(sm, grid, sv, L, dV, dA, st);
            else launch_batch_paths<6>(sm, grid, sv, L, dV, dA, st);
        }
    }
    if (d_vertices) k_reduce_shards<<<nblk(3L * s->V, kReduceEntries), 256, 0, st>>>(dV, L.gshards, L.gstride, 3L * s->V, d_vertices);
    if (d_albedo) k_reduce_shards<<<nblk(s->T, kReduceEntries), 256, 0, st>>>(dA, L.gshards, L.gstride, s->T, d_albedo);
    if (d_cameras) k_cam_finalize_batch<<<(L.nviews + 63) / 64, 64, 0, st>>>(L.views, L.nviews, L.gshards, d_cameras);
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}

drStatus launch_batch_seed(BatchView* views, int n, uint32_t add, hipStream_t st) {
    k_batch_seed<<<(n + 63) / 64, 64, 0, st>>>(views, n, add);
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}

}  // namespace dr
