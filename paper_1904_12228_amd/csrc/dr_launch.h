// Kernel-variant launchers shared between the render translation units: the
// orchestration in dr_render.hip picks a variant, and the unit that compiles
// that variant launches it.
#pragma once
#include <algorithm>
#include "dr_args.h"
#include "dr_host.h"

namespace dr {

// Variant switches of one launch: geometry buffer, learned-proposal mixture,
// work counters, short (kSmallStack-entry) traversal stack.
struct Variant {
    bool aov, mix, counters, small;
};

// Primary edge samples: one lane per unit (k_primary), or, when `pq` is not
// null (production and mixture variants), the split pair k_prim_sample (edge sample,
// first hits, compact queue of the samples whose sides hit different
// triangles: pq [M], *pcount zeroed first) and k_prim_paths (the queued
// samples' camera paths and gradients, paths_grid persistent blocks).
void launch_primary_kernel(const Variant& v, dim3 grid, const SceneView& sv, const Cam& cam, const RenderArgs& a,
                           const PEdge* pe, const double* pcdf, const float* d_image, float* dV, float* camacc,
                           const MixArgs& mx, int3* pq, int* pcount, int paths_grid, hipStream_t st);

// Path backward of the units (secondary edge samples, interior adjoint,
// scatter) for kernel depth maxd (1, 3 or 6): the split sample / side-path /
// adjoint kernels when `split`, the single k_backward otherwise.
struct PathLaunch {
    Variant v;
    bool split;
    dim3 grid;
    int side_grid, depth;
    SceneView sv;
    Cam cam;
    RenderArgs a;
    TreeView tv;
    SplitArgs sp;
    const float* d_image;
    float *dV, *dA, *camacc;
    MixArgs mx;
};
template <int D, int S>
void launch_paths_stack(const PathLaunch& p, hipStream_t st);

// Path backward of every view of a batch (k_backward_batch) at kernel depth D.
template <int D>
void launch_batch_paths(bool small, int grid, const SceneView& sv, const BatchLaunch& L, float* dV, float* dA,
                        hipStream_t st);

}  // namespace dr
