// Launch of the path backward at a fixed kernel depth D and traversal stack
// size S; dr_render_d*.hip instantiate it, one or two (D, S) pairs per unit.
#pragma once
#include <algorithm>

#include "dr_kernels.h"
#include "dr_launch.h"

namespace dr {

template <int D, int S>
void launch_paths_stack(const PathLaunch& p, hipStream_t st) {
    dim3 g = p.grid, b(BS);
    if (p.split) {
        // the learned-proposal mixture splits only where every vertex is
        // checkpointed (D <= 3); the caller keeps the fused kernel otherwise
        if (D <= 3) {
            // every vertex checkpointed: one lane per (vertex, unit)
            int nv = std::min(p.depth, D);
            long items = (long)nv * p.a.M;
            dim3 gv((unsigned)((items + BS - 1) / BS));
            if (p.v.mix) k_bwd_sample_v<S, true><<<gv, b, 0, st>>>(p.sv, p.cam, p.a, p.tv, p.sp, nv, p.mx);
            else if (p.a.cands > 1) k_bwd_sample_v<S, false, true><<<gv, b, 0, st>>>(p.sv, p.cam, p.a, p.tv, p.sp, nv, p.mx);
            else if (p.a.nee > 0.0f)
                k_bwd_sample_v<S, false, false, true><<<gv, b, 0, st>>>(p.sv, p.cam, p.a, p.tv, p.sp, nv, p.mx);
            else k_bwd_sample_v<S, false><<<gv, b, 0, st>>>(p.sv, p.cam, p.a, p.tv, p.sp, nv, p.mx);
        } else if (p.a.nee > 0.0f) {
            k_bwd_sample<D, S, true><<<g, b, 0, st>>>(p.sv, p.cam, p.a, p.tv, p.sp);
        } else {
            k_bwd_sample<D, S><<<g, b, 0, st>>>(p.sv, p.cam, p.a, p.tv, p.sp);
        }
        for (int kq = 0; kq < std::min(p.depth, D); ++kq) k_side<S><<<p.side_grid, b, 0, st>>>(p.sv, p.a, p.sp, kq);
        if (p.v.mix && D <= 3)
            k_bwd_adjoint<D, S, true><<<g, b, 0, st>>>(p.sv, p.cam, p.a, p.tv, p.d_image, p.dV, p.dA, p.camacc, p.sp, p.mx);
        else
            k_bwd_adjoint<D, S, false><<<g, b, 0, st>>>(p.sv, p.cam, p.a, p.tv, p.d_image, p.dV, p.dA, p.camacc, p.sp, p.mx);
    } else if (p.v.mix) {
        k_backward<D, S, false, true><<<g, b, 0, st>>>(p.sv, p.cam, p.a, p.tv, p.d_image, p.dV, p.dA, p.camacc, p.mx);
    } else if (p.v.counters) {
        k_backward<D, S, true, false><<<g, b, 0, st>>>(p.sv, p.cam, p.a, p.tv, p.d_image, p.dV, p.dA, p.camacc, p.mx);
    } else {
        k_backward<D, S, false, false><<<g, b, 0, st>>>(p.sv, p.cam, p.a, p.tv, p.d_image, p.dV, p.dA, p.camacc, p.mx);
    }
}


template <int D>
void launch_batch_paths(bool small, int grid, const SceneView& sv, const BatchLaunch& L, float* dV, float* dA,
                        hipStream_t st) {
    if (small) k_backward_batch<D, kSmallStack><<<grid, BS, 0, st>>>(sv, L, dV, dA);
    else k_backward_batch<D, kStackDepth><<<grid, BS, 0, st>>>(sv, L, dV, dA);
}

}  // namespace dr
