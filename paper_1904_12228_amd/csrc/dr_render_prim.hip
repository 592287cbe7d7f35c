// Primary edge samples: the split pair (k_prim_sample, k_prim_paths) for the
// production and mixture variants, k_primary for every variant.
#include "dr_kernels.h"
#include "dr_launch.h"

namespace dr {

void launch_primary_kernel(const Variant& v, dim3 g, const SceneView& sv, const Cam& cam, const RenderArgs& a,
                           const PEdge* pe, const double* pc, const float* d_image, float* dV, float* camacc,
                           const MixArgs& mx, int3* pq, int* pcount, int paths_grid, hipStream_t st) {
    dim3 b(BS);
    if (pq && !v.aov && !v.counters) {
        k_fill_count<<<1, 64, 0, st>>>(pcount, 1);
#define DR_SPLIT(S, X)                                                                                                \
    k_prim_sample<S, X><<<g, b, 0, st>>>(sv, cam, a, pe, pc, pq, pcount, mx);                                          \
    k_prim_paths<S, X><<<paths_grid, b, 0, st>>>(sv, cam, a, pe, pc, pq, pcount, d_image, dV, camacc, mx)
        if (v.mix) {
            if (v.small) { DR_SPLIT(kSmallStack, true); }
            else { DR_SPLIT(kStackDepth, true); }
        } else {
            if (v.small) { DR_SPLIT(kSmallStack, false); }
            else { DR_SPLIT(kStackDepth, false); }
        }
#undef DR_SPLIT
        return;
    }
#define DR_PRIM(S, C, X, A) k_primary<S, C, X, A><<<g, b, 0, st>>>(sv, cam, a, pe, pc, d_image, dV, camacc, mx)
    if (v.aov) {
        if (v.small) DR_PRIM(kSmallStack, false, false, true);
        else DR_PRIM(kStackDepth, false, false, true);
    } else if (v.mix) {
        if (v.small) DR_PRIM(kSmallStack, false, true, false);
        else DR_PRIM(kStackDepth, false, true, false);
    } else if (v.counters) {
        if (v.small) DR_PRIM(kSmallStack, true, false, false);
        else DR_PRIM(kStackDepth, true, false, false);
    } else {
        if (v.small) DR_PRIM(kSmallStack, false, false, false);
        else DR_PRIM(kStackDepth, false, false, false);
    }
#undef DR_PRIM
}

}  // namespace dr
