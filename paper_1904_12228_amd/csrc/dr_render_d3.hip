// Path backward kernels at kernel depth 3, short traversal stack.
#include "dr_paths_impl.h"

namespace dr {
template void launch_paths_stack<3, kSmallStack>(const PathLaunch&, hipStream_t);
}  // namespace dr
