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
        if (D <= 3) {
            // every vertex checkpointed: one lane per (vertex, unit)
            int nv = std::min(p.depth, D);
            long items = (long)nv * p.a.M;
            k_bwd_sample_v<S><<<dim3((unsigned)((items + BS - 1) / BS)), b, 0, st>>>(p.sv, p.cam, p.a, p.tv, p.sp, nv);
        } else {
            k_bwd_sample<D, S><<<g, b, 0, st>>>(p.sv, p.cam, p.a, p.tv, p.sp);
        }
        for (int kq = 0; kq < std::min(p.depth, D); ++kq) k_side<S><<<p.side_grid, b, 0, st>>>(p.sv, p.a, p.sp, kq);
        k_bwd_adjoint<D, S><<<g, b, 0, st>>>(p.sv, p.cam, p.a, p.tv, p.d_image, p.dV, p.dA, p.camacc, p.sp);
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
    if (small) k_backward_batch<D, 32><<<grid, BS, 0, st>>>(sv, L, dV, dA);
    else k_backward_batch<D, kStackDepth><<<grid, BS, 0, st>>>(sv, L, dV, dA);
}

}  // namespace dr
