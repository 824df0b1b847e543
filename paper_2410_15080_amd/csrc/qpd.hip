// Truncation of QTs after QPD sampling (Sec. 4.3, Fig. 3 (d)): every tensor
// of a batch keeps, along each of its axes, only the listed indices.  One
// launch covers the batch.  Most truncated QTs hold a few hundred elements,
// so a block copies a run of whole small items (up to 1024 elements and 32
// items together) or one 1024-element chunk of a larger item; it first
// stages its item descriptors and gather maps in LDS, so that each element
// costs one dependent global load (its source) instead of a chain of them.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace htn {
namespace kern {

namespace {

// dst[o] = src[sum_a map_a[digit_a(o)]]: output digits last-fastest over the
// kept extents; map_a holds kept index x input stride of axis a.
template <typename U>
__global__ __launch_bounds__(kTruncThreads) void k_truncate(const TruncItem *__restrict__ items,
                                                            const TruncBlock *__restrict__ blocks,
                                                            const int64_t *__restrict__ maps) {
    __shared__ TruncItem s_items[kTruncBlockItems];
    __shared__ int64_t s_map[kTruncMapLds];
    const TruncBlock bk = blocks[blockIdx.x];
    {
        static_assert(sizeof(TruncItem) % 4 == 0, "items copied as 32-bit words");
        const int32_t *gi = reinterpret_cast<const int32_t *>(items + bk.item0);
        int32_t *si = reinterpret_cast<int32_t *>(s_items);
        const int nw = bk.n_items * (int)(sizeof(TruncItem) / 4);
        for (int w = threadIdx.x; w < nw; w += kTruncThreads) si[w] = gi[w];
        for (int w = threadIdx.x; w < bk.map_words; w += kTruncThreads) s_map[w] = maps[bk.map_base + w];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kTruncPerThread; ++j) {
        const int e = threadIdx.x + j * kTruncThreads;
        // the item holding block position e: the last one starting at or
        // before e (items of a block are in ascending start order)
        int lo = 0, hi = bk.n_items - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_items[mid].start <= e)
                lo = mid;
            else
                hi = mid - 1;
        }
        const TruncItem &it = s_items[lo];
        const int64_t o64 = bk.base + (e - it.start);
        if (o64 >= it.n_out) continue;
        uint32_t rem = (uint32_t)o64;
        int64_t off = 0;
        const int64_t *map = bk.map_words > 0 ? s_map + (it.map_off - bk.map_base) : maps + it.map_off;
        for (int a = it.rank - 1; a >= 0; --a) {
            const uint32_t d = (uint32_t)it.odim[a];
            const uint32_t q = rem / d;
            off += map[it.moff[a] + (int)(rem - q * d)];
            rem = q;
        }
        static_cast<U *>(it.dst)[o64] = static_cast<const U *>(it.src)[off];
    }
}

}  // namespace

hipError_t launch_truncate(const TruncItem *items, const TruncBlock *blocks, int64_t n_blocks, const int64_t *maps,
                           int elem_bytes, hipStream_t st) {
    if (n_blocks <= 0) return hipSuccess;
    const dim3 grid((unsigned)n_blocks), block(kTruncThreads);
    if (elem_bytes == 8)
        hipLaunchKernelGGL((k_truncate<uint64_t>), grid, block, 0, st, items, blocks, maps);
    else if (elem_bytes == 4)
        hipLaunchKernelGGL((k_truncate<uint32_t>), grid, block, 0, st, items, blocks, maps);
    else
        hipLaunchKernelGGL((k_truncate<uint16_t>), grid, block, 0, st, items, blocks, maps);
    return hipGetLastError();
}

}  // namespace kern
}  // namespace htn
