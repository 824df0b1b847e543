// Fused kernel instantiations for 256-thread workgroups.
#include "fused.hpp"

namespace htn {
namespace kern {
template hipError_t launch_fused_blk<256>(const FusedDesc *, const int32_t *, void *const *, int64_t *, void *,
                                          int64_t *, int, int, int, int, int, hipStream_t);
}  // namespace kern
}  // namespace htn
