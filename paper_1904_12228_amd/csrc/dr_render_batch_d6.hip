// Batched path backward kernels at kernel depth 6.
#include "dr_paths_impl.h"

namespace dr {
template void launch_batch_paths<6>(bool, int, const SceneView&, const BatchLaunch&, float*, float*, hipStream_t);
}  // namespace dr
