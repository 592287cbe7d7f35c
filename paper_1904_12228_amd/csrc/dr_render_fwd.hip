// Forward pass: camera paths, NEE, checkpoints and the image (k_forward, or,
// with DIFFRT_WAVEFRONT_FORWARD=1, its wavefront form for max_depth 2 and 3),
// or the geometry buffers (k_forward_aov).
#include "dr_kernels.h"

namespace dr {

drStatus launch_forward(drScene_t* s, const Cam& cam, const drRenderOptions& o, float* image, hipStream_t st) {
    RenderArgs a = make_args(s, cam, o);
    SceneView sv = s->view();
    bool sm = small_stack(s);
    sv.stk_cap = sm ? kSmallStack : kStackDepth;
    bool reduce = (BS % o.spp) == 0;
    long npix = (long)a.Ww * (cam.y1 - cam.y0) * (o.aov == 8 ? 7 : 1);
    if (!reduce) k_fill<<<nblk(npix, 256), 256, 0, st>>>(image, npix, 0.0f);
    {
        EvScope ev(s, 0, st);
        dim3 g(nblk(a.M, BS)), b(BS);
        int red = reduce ? 1 : 0;
        if (o.aov) {
            if (sm) k_forward_aov<kSmallStack><<<g, b, 0, st>>>(sv, cam, a, image, red);
            else k_forward_aov<kStackDepth><<<g, b, 0, st>>>(sv, cam, a, image, red);
        } else if (!a.counters && s->wavefront_forward && o.max_depth >= 2 && o.max_depth <= 3 && a.ck_tri && a.ck_x &&
                   a.ck_vis) {
            if (s->fq.ensure(sizeof(int4) * 2 * (size_t)a.M) != hipSuccess ||
                s->fcount.ensure(sizeof(int) * 2) != hipSuccess || s->fL.ensure(sizeof(float) * (size_t)a.M) != hipSuccess)
                return DR_ERROR_OUT_OF_MEMORY;
            FwdQueue fq{s->fq.as<int4>(), s->fcount.as<int>(), s->fL.as<float>()};
            k_fill_count<<<1, 64, 0, st>>>(fq.count, 2);
            // the bounce queues drain on persistent grids (two rounds of the resident blocks)
            dim3 qg(std::max(1, std::min(nblk((long)a.M, BS), kQueueBlocks)));
            if (sm) {
                k_fwd_hit<kSmallStack><<<g, b, 0, st>>>(sv, cam, a, fq);
                k_fwd_bounce<kSmallStack, 1><<<qg, b, 0, st>>>(sv, cam, a, fq);
                if (o.max_depth == 3) k_fwd_bounce<kSmallStack, 2><<<qg, b, 0, st>>>(sv, cam, a, fq);
            } else {
                k_fwd_hit<kStackDepth><<<g, b, 0, st>>>(sv, cam, a, fq);
                k_fwd_bounce<kStackDepth, 1><<<qg, b, 0, st>>>(sv, cam, a, fq);
                if (o.max_depth == 3) k_fwd_bounce<kStackDepth, 2><<<qg, b, 0, st>>>(sv, cam, a, fq);
            }
            k_fwd_image<<<g, b, 0, st>>>(a, fq.L, image, red);
        } else if (a.counters) {
            if (sm) k_forward<kSmallStack, true><<<g, b, 0, st>>>(sv, cam, a, image, red);
            else k_forward<kStackDepth, true><<<g, b, 0, st>>>(sv, cam, a, image, red);
        } else {
            if (sm) k_forward<kSmallStack, false><<<g, b, 0, st>>>(sv, cam, a, image, red);
            else k_forward<kStackDepth, false><<<g, b, 0, st>>>(sv, cam, a, image, red);
        }
    }
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}

}  // namespace dr
