// Path backward kernels at kernel depth 1, both traversal stack sizes.
#include "dr_paths_impl.h"

namespace dr {
template void launch_paths_stack<1, kSmallStack>(const PathLaunch&, hipStream_t);
template void launch_paths_stack<1, kStackDepth>(const PathLaunch&, hipStream_t);
}  // namespace dr
