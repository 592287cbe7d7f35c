// Path backward kernels at kernel depth 6, full-size traversal stack.
#include "dr_paths_impl.h"

namespace dr {
template void launch_paths_stack<6, kStackDepth>(const PathLaunch&, hipStream_t);
}  // namespace dr
