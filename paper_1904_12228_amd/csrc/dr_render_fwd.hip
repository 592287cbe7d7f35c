// Forward pass: camera paths, NEE, checkpoints and the image (k_forward), or
// the geometry buffers (k_forward_aov).
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
