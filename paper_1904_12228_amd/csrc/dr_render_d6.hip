// Path backward kernels at kernel depth 6, short traversal stack.
#include "dr_paths_impl.h"

namespace dr {
template void launch_paths_stack<6, kSmallStack>(const PathLaunch&, hipStream_t);
}  // namespace dr
