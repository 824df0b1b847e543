// Device-side helpers shared by the HIP kernels (element conversions,
// compensated accumulation, wave-level reductions).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace htn {
namespace kern {

typedef uint16_t bf16_t;  // bfloat16 bit pattern

enum { OP_END = 0, OP_LOAD = 1, OP_STEP = 2, OP_SYNC = 3, OP_TSTEP = 4, OP_TCOPY = 5, OP_COPY = 6 };
constexpr int kMaxRankLoad = 16, kMaxScalesLoad = 8;
constexpr int kBlk = 256;

__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40u);  // keep NaN quiet
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (bf16_t)(u >> 16);
}

template <typename ACC, typename T>
struct Ld {
    __device__ __forceinline__ static ACC get(const T *p) { return (ACC)(*p); }
};
template <typename ACC>
struct Ld<ACC, bf16_t> {
    __device__ __forceinline__ static ACC get(const bf16_t *p) { return (ACC)bf2f(*p); }
};

template <typename T, typename ACC>
__device__ __forceinline__ T st_cvt(ACC v) {
    return (T)v;
}
template <>
__device__ __forceinline__ bf16_t st_cvt<bf16_t, float>(float v) {
    return f2bf(v);
}
template <>
__device__ __forceinline__ bf16_t st_cvt<bf16_t, double>(double v) {
    return f2bf((float)v);
}

// Neumaier accumulation (COMP) or plain accumulation.
template <bool COMP, typename ACC>
__device__ __forceinline__ void accum(ACC &s, ACC &c, ACC x) {
    if constexpr (COMP) {
        ACC t = s + x;
        if (fabs(s) >= fabs(x))
            c += (s - t) + x;
        else
            c += (x - t) + s;
        s = t;
    } else {
        s += x;
    }
}

// Combine two partial sums; with COMP the high parts are added by Knuth's
// TwoSum and the rounding error joins the compensation terms.
template <bool COMP, typename ACC>
__device__ __forceinline__ void combine(ACC &s, ACC &c, ACC s2, ACC c2) {
    if constexpr (COMP) {
        ACC t = s + s2;
        ACC bb = t - s;
        ACC e = (s - (t - bb)) + (s2 - bb);
        s = t;
        c = c + c2 + e;
    } else {
        s += s2;
    }
}

template <bool COMP, typename ACC>
__device__ __forceinline__ void lane_reduce(ACC &s, ACC &c, int width) {
    for (int m = width >> 1; m > 0; m >>= 1) {
        ACC s2 = __shfl_xor(s, m);
        ACC c2 = COMP ? __shfl_xor(c, m) : ACC(0);
        combine<COMP>(s, c, s2, c2);
    }
}

}  // namespace kern
}  // namespace htn
