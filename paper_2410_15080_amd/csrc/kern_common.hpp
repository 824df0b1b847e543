// Device-side helpers shared by the HIP kernels (element conversions,
// compensated accumulation, wave-level reductions).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

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

// Value of an input element in the compute type (bf16 bit patterns widen
// to float).
template <typename T, typename TIN>
__device__ __forceinline__ T to_compute(TIN x) {
    if constexpr (std::is_same<TIN, bf16_t>::value)
        return (T)bf2f(x);
    else
        return (T)x;
}

// Input materialisation of fused networks.  A descriptor (in the fused
// image) gives the input's device address, its destination in the network's
// workspace and the digit form of its planned layout: element e of the
// value has mixed-radix digits over the value's labels; its source offset
// and each coefficient tensor's offset are dot products of the digits with
// per-label strides.  Digits are extracted with precomputed magic
// multipliers: floor(e / d) = (e * magic) >> 40, exact for e < 2^24 and
// d < 2^16.
// Descriptor words: [base ptr (2), dst element offset (2), size, rank, ns,
//   scale ptrs (2 each), per label k: (extent, magic (2), source stride,
//   scale strides)]
// One wave materialises one entry (a chunk of kFPrepChunk elements of one
// load); lane = lane index 0..63.  Descriptor words are wave-uniform and
// read-only; Words is their view: the constant address space (scalar
// loads, each digit's words fetched when first needed) or the wave's lanes
// (one vector load up front, no chain of dependent scalar round trips).
// The tensors are read through the global address space.
typedef const int32_t __attribute__((address_space(4))) c_int32;

template <typename T, typename TIN, typename Words, int MR = kMaxRankLoad, int MS = kMaxScalesLoad>
__device__ __forceinline__ void fprep_words(const Words &p, void *ws, int e_first, int lane) {
    typedef const TIN __attribute__((address_space(1))) g_tin;
    auto ptr_at = [&](int w) {
        return (const g_tin *)(uintptr_t)(((uint64_t)(uint32_t)p(w + 1) << 32) | (uint32_t)p(w));
    };
    const int64_t dst_off = (int64_t)(((uint64_t)(uint32_t)p(3) << 32) | (uint32_t)p(2));
    const int size = p(4), rk = p(5), ns = p(6);
    const int per = 7 + 2 * ns;
    const int Wd = 4 + ns;
    const g_tin *src = ptr_at(0);
    T *o = (T *)ws + dst_off;
    const g_tin *sp[MS];
#pragma unroll
    for (int q = 0; q < MS; ++q) sp[q] = q < ns ? ptr_at(7 + 2 * q) : nullptr;
    const int e_end = min(size, e_first + kFPrepChunk);
    // four elements per lane at a time, so their gathers are in flight
    // together; each digit's descriptor words are read once for all four
    for (int e0 = e_first + lane; e0 < e_end; e0 += 4 * 64) {
        int so[4], sc[4][MS];
        uint32_t rem[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            rem[u] = (uint32_t)min(e0 + 64 * u, e_end - 1);
            so[u] = 0;
#pragma unroll
            for (int q = 0; q < MS; ++q) sc[u][q] = 0;
        }
#pragma unroll
        for (int k = MR - 1; k >= 0; --k) {
            if (k < rk) {
                const int pk = per + k * Wd;
                const uint32_t ext = (uint32_t)p(pk);
                const uint64_t magic = ((uint64_t)(uint32_t)p(pk + 2) << 32) | (uint32_t)p(pk + 1);
                const int sstr = p(pk + 3);
                int cs[MS];
#pragma unroll
                for (int q = 0; q < MS; ++q) cs[q] = q < ns ? p(pk + 4 + q) : 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t quo = (uint32_t)(((uint64_t)rem[u] * magic) >> 40);
                    const int dgt = (int)(rem[u] - quo * ext);
                    rem[u] = quo;
                    so[u] += dgt * sstr;
#pragma unroll
                    for (int q = 0; q < MS; ++q) sc[u][q] += dgt * cs[q];
                }
            }
        }
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = to_compute<T>(src[so[u]]);
#pragma unroll
        for (int q = 0; q < MS; ++q)
            if (q < ns) {
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] *= to_compute<T>(sp[q][sc[u][q]]);
            }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (e0 + 64 * u < e_end) o[e0 + 64 * u] = v[u];
    }
}

// Descriptor read in place through the constant address space.
struct ConstWords {
    const c_int32 *p;
    __device__ __forceinline__ int32_t operator()(int i) const { return p[i]; }
};

// Descriptor of at most 64 words held across the wave's lanes (word i in
// lane i), loaded with one vector load; a wave-uniform read is one lane
// read, with no memory round trip.
struct LaneWords {
    int32_t r;
    __device__ __forceinline__ explicit LaneWords(int32_t word) : r(word) {}
    __device__ __forceinline__ LaneWords(const int32_t *desc, int n, int lane) : r(lane < n ? desc[lane] : 0) {}
    __device__ __forceinline__ int32_t operator()(int i) const { return __builtin_amdgcn_readlane(r, i); }
};

// One entry, descriptor read in place through the constant address space.
template <typename T, typename TIN>
__device__ __forceinline__ void fprep_entry(const FPrepEntry &en, int lane) {
    fprep_words<T, TIN>(ConstWords{(const c_int32 *)en.desc}, en.ws, en.e0, lane);
}

}  // namespace kern
}  // namespace htn
