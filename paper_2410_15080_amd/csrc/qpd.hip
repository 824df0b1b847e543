// Truncation of QTs after QPD sampling (Sec. 4.3, Fig. 3 (d)): every tensor
// of a batch keeps, along each of its axes, only the listed indices.  One
// launch covers the batch; a block copies 1024 output elements of one item.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace htn {
namespace kern {

namespace {

// Item of the block: the last item whose first block is <= blockIdx.x.
__device__ __forceinline__ int item_of_block(const TruncItem *items, int n) {
    int lo = 0, hi = n - 1;
    const int64_t b = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].block0 <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// dst[o] = src[sum_a map_a[digit_a(o)]]: output digits last-fastest over the
// kept extents; map_a holds kept index x input stride of axis a.
template <typename U>
__global__ __launch_bounds__(kTruncThreads) void k_truncate(const TruncItem *__restrict__ items, int n,
                                                            const int64_t *__restrict__ maps) {
    const TruncItem &it = items[item_of_block(items, n)];
    const U *__restrict__ src = static_cast<const U *>(it.src);
    U *__restrict__ dst = static_cast<U *>(it.dst);
    const int64_t *__restrict__ map = maps + it.map_off;
    const uint32_t base = (uint32_t)(blockIdx.x - it.block0) * (kTruncThreads * kTruncPerThread);
#pragma unroll
    for (int j = 0; j < kTruncPerThread; ++j) {
        const uint32_t o = base + threadIdx.x + j * kTruncThreads;
        if (o >= (uint32_t)it.n_out) break;
        uint32_t rem = o;
        int64_t off = 0;
        for (int a = it.rank - 1; a >= 0; --a) {
            const uint32_t d = (uint32_t)it.odim[a];
            const uint32_t q = rem / d;
            off += map[it.moff[a] + (int)(rem - q * d)];
            rem = q;
        }
        dst[o] = src[off];
    }
}

}  // namespace

hipError_t launch_truncate(const TruncItem *items, int n_items, const int64_t *maps, int64_t n_blocks, int elem_bytes,
                           hipStream_t st) {
    if (n_items <= 0 || n_blocks <= 0) return hipSuccess;
    const dim3 grid((unsigned)n_blocks), block(kTruncThreads);
    if (elem_bytes == 8)
        hipLaunchKernelGGL((k_truncate<uint64_t>), grid, block, 0, st, items, n_items, maps);
    else if (elem_bytes == 4)
        hipLaunchKernelGGL((k_truncate<uint32_t>), grid, block, 0, st, items, n_items, maps);
    else
        hipLaunchKernelGGL((k_truncate<uint16_t>), grid, block, 0, st, items, n_items, maps);
    return hipGetLastError();
}

}  // namespace kern
}  // namespace htn
