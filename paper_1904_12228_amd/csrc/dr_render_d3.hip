// Path backward kernels at kernel depth 3, 32-entry traversal stack.
#include "dr_paths_impl.h"

namespace dr {
template void launch_paths_stack<3, 32>(const PathLaunch&, hipStream_t);
}  // namespace dr
