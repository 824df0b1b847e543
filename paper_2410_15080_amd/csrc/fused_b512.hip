// Fused kernel instantiations for 512-thread workgroups.
#include "fused.hpp"

namespace htn {
namespace kern {
template hipError_t launch_fused_blk<512>(const FusedDesc *, const int32_t *, void *const *, int64_t *, void *,
                                          int64_t *, int, int, int, int, int, hipStream_t);
}  // namespace kern
}  // namespace htn
