// HIP kernels for h-TN contraction on gfx950 (wave64).
//
//  k_step   one pairwise contraction C[o] = sum_s A[.]*B[.] over arbitrary
//           label layouts.  The operand offsets of output index o and summed
//           index s come from two-level offset tables built by the planner,
//           so one kernel covers every permutation, hyperedge (batch) label,
//           single-operand summed label and outer product.  R lanes
//           cooperate on one output and reduce with cross-lane shuffles.
//  k_prep   applies coefficient tensors folded into an input (entry-wise
//           scaling, Sec. 4.3's fusion of CTs into the QTs they join) and
//           converts to the intermediate type.
//  k_fused  one workgroup contracts an entire network: inputs are loaded
//           once from HBM into LDS (with their coefficient scales), every
//           pairwise step runs LDS-to-LDS, the last step writes the result.
//           One launch serves a batch of networks (one workgroup each).
#include "kernels.hpp"

#include <type_traits>

namespace htn {
namespace kern {

typedef uint16_t bf16_t;  // bfloat16 bit pattern

enum { OP_END = 0, OP_LOAD = 1, OP_STEP = 2, OP_SYNC = 3 };
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

// ------------------------------------------------------------------ k_step

template <typename TA, typename TB, typename TC, typename ACC, bool UNARY, bool COMP>
__global__ __launch_bounds__(kBlk) void k_step(const TA *__restrict__ A, const TB *__restrict__ B, TC *__restrict__ C,
                                              const int2 *__restrict__ tab, StepArgs s) {
    const int64_t gt = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    const int64_t o = gt >> s.log2R;
    const int sub = (int)(gt & (s.R - 1));
    const bool active = o < s.n_out;
    ACC acc = 0, cmp = 0;
    if (active) {
        const int oh = (int)(o / s.n_olo);
        const int ol = (int)(o - (int64_t)oh * s.n_olo);
        const int2 x = tab[s.t_ohi + oh], y = tab[s.t_olo + ol];
        const TA *a0 = A + (x.x + y.x);
        const TB *b0 = B;
        if constexpr (!UNARY) b0 = B + (x.y + y.y);
        const int2 *th = tab + s.t_shi;
        const int2 *tl = tab + s.t_slo;
        if (s.R == 1) {
            for (int sh = 0; sh < s.n_shi; ++sh) {
                const int2 h = th[sh];
                const TA *a1 = a0 + h.x;
                const TB *b1 = b0;
                if constexpr (!UNARY) b1 = b0 + h.y;
                for (int sl = 0; sl < s.n_slo; ++sl) {
                    const int2 l = tl[sl];
                    ACC p = Ld<ACC, TA>::get(a1 + l.x);
                    if constexpr (!UNARY) p *= Ld<ACC, TB>::get(b1 + l.y);
                    accum<COMP>(acc, cmp, p);
                }
            }
        } else {
            const int dq = s.R / s.n_slo, dr = s.R - dq * s.n_slo;
            int sh = sub / s.n_slo;
            int sl = sub - sh * s.n_slo;
            while (sh < s.n_shi) {
                const int2 h = th[sh], l = tl[sl];
                ACC p = Ld<ACC, TA>::get(a0 + h.x + l.x);
                if constexpr (!UNARY) p *= Ld<ACC, TB>::get(b0 + h.y + l.y);
                accum<COMP>(acc, cmp, p);
                sh += dq;
                sl += dr;
                if (sl >= s.n_slo) {
                    sl -= s.n_slo;
                    ++sh;
                }
            }
        }
    }
    lane_reduce<COMP>(acc, cmp, s.R);
    if (active && sub == 0) C[o] = st_cvt<TC>(COMP ? acc + cmp : acc);
}

template <typename TA, typename TB, typename TC, typename ACC, bool U, bool CMP>
static hipError_t go_step(const void *A, const void *B, void *C, const int2 *tab, const StepArgs &s,
                          hipStream_t st) {
    const int64_t threads = s.n_out * (int64_t)s.R;
    const int64_t blocks = (threads + kBlk - 1) / kBlk;
    hipLaunchKernelGGL((k_step<TA, TB, TC, ACC, U, CMP>), dim3((unsigned)blocks), dim3(kBlk), 0, st,
                       (const TA *)A, (const TB *)B, (TC *)C, tab, s);
    return hipGetLastError();
}

template <typename TA, typename TB>
static hipError_t step_out(const void *A, const void *B, void *C, int tc, bool comp, bool unary, const int2 *tab,
                           const StepArgs &s, hipStream_t st) {
    if (tc == 0) {
        if (unary) {
            return comp ? go_step<TA, TA, double, double, true, true>(A, B, C, tab, s, st)
                        : go_step<TA, TA, double, double, true, false>(A, B, C, tab, s, st);
        }
        return comp ? go_step<TA, TB, double, double, false, true>(A, B, C, tab, s, st)
                    : go_step<TA, TB, double, double, false, false>(A, B, C, tab, s, st);
    }
    if (tc == 1 && !comp) {
        if (unary) return go_step<TA, TA, float, float, true, false>(A, B, C, tab, s, st);
        return go_step<TA, TB, float, float, false, false>(A, B, C, tab, s, st);
    }
    if (tc == 2 && !comp && unary) return go_step<TA, TA, bf16_t, float, true, false>(A, B, C, tab, s, st);
    return hipErrorInvalidValue;
}

hipError_t launch_step(const void *A, int ta, const void *B, int tb, void *C, int tc, bool acc_f64, bool comp,
                       const int2 *tab, const StepArgs &s, hipStream_t st) {
    (void)acc_f64;  // the output type fixes the accumulator (FP64 for tc 0)
    const bool unary = (B == nullptr);
    if (unary) tb = ta;
    if (ta == 0 && tb == 0) {
        if (tc != 0) return hipErrorInvalidValue;
        return step_out<double, double>(A, B, C, tc, comp, unary, tab, s, st);
    }
    if (ta == 1 && tb == 1) return step_out<float, float>(A, B, C, tc, comp, unary, tab, s, st);
    if (ta == 2 && tb == 2) return step_out<bf16_t, bf16_t>(A, B, C, tc, comp, unary, tab, s, st);
    if (ta == 2 && tb == 1) return step_out<bf16_t, float>(A, B, C, tc, comp, unary, tab, s, st);
    if (ta == 1 && tb == 2) return step_out<float, bf16_t>(A, B, C, tc, comp, unary, tab, s, st);
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ k_prep

template <typename TIN, typename TI>
__global__ __launch_bounds__(kBlk) void k_prep(const PrepDesc *__restrict__ descs, const int2 *__restrict__ tab) {
    const PrepDesc &q = descs[blockIdx.y];
    const TIN *src = (const TIN *)q.src;
    TI *dst = (TI *)q.dst;
    const int ns = q.ns;
    for (int e = blockIdx.x * kBlk + threadIdx.x; e < q.size; e += gridDim.x * kBlk) {
        TI v = Ld<TI, TIN>::get(src + e);
        for (int k = 0; k < ns; ++k) {
            const int eh = e / q.nlo[k];
            const int el = e - eh * q.nlo[k];
            v *= Ld<TI, TIN>::get((const TIN *)q.sp[k] + tab[q.thi[k] + eh].x + tab[q.tlo[k] + el].x);
        }
        dst[e] = v;
    }
}

hipError_t launch_prep(const PrepDesc *d_desc, int n_desc, int max_size, int tin, int tinter, const int2 *tab,
                       hipStream_t st) {
    if (n_desc <= 0) return hipSuccess;
    int bx = (max_size + kBlk * 4 - 1) / (kBlk * 4);
    bx = bx < 1 ? 1 : (bx > 4096 ? 4096 : bx);
    dim3 grid(bx, n_desc);
    if (tin == 0 && tinter == 0)
        hipLaunchKernelGGL((k_prep<double, double>), grid, dim3(kBlk), 0, st, d_desc, tab);
    else if (tin == 1 && tinter == 1)
        hipLaunchKernelGGL((k_prep<float, float>), grid, dim3(kBlk), 0, st, d_desc, tab);
    else if (tin == 2 && tinter == 1)
        hipLaunchKernelGGL((k_prep<bf16_t, float>), grid, dim3(kBlk), 0, st, d_desc, tab);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ----------------------------------------------------------------- k_fused

// One step inside the fused kernel.  A, B point into LDS; C into LDS or, for
// the final step, global memory.
template <typename T, typename ACC, bool COMP, bool UNARY, typename TOUT>
__device__ __forceinline__ void fstep(const T *A, const T *B, TOUT *C, const int2 *__restrict__ tab,
                                      const int32_t *g, int R, ACC *scratch) {
    const int n_ohi = g[0], n_olo = g[1], n_shi = g[2], n_slo = g[3];
    const int2 *toh = tab + g[4];
    const int2 *tol = tab + g[5];
    const int2 *tsh = tab + g[6];
    const int2 *tsl = tab + g[7];
    const int n_out = n_ohi * n_olo;
    const int tid = threadIdx.x;
    if (R == kBlk) {
        // whole workgroup per output (tiny outputs, long sums)
        const int dq = kBlk / n_slo, dr = kBlk - dq * n_slo;
        for (int o = 0; o < n_out; ++o) {
            const int oh = o / n_olo, ol = o - oh * n_olo;
            const int2 x = toh[oh], y = tol[ol];
            const T *a0 = A + (x.x + y.x);
            const T *b0 = B;
            if constexpr (!UNARY) b0 = B + (x.y + y.y);
            ACC s = 0, c = 0;
            int sh = tid / n_slo, sl = tid - sh * n_slo;
            while (sh < n_shi) {
                const int2 h = tsh[sh], l = tsl[sl];
                ACC p = (ACC)a0[h.x + l.x];
                if constexpr (!UNARY) p *= (ACC)b0[h.y + l.y];
                accum<COMP>(s, c, p);
                sh += dq;
                sl += dr;
                if (sl >= n_slo) {
                    sl -= n_slo;
                    ++sh;
                }
            }
            lane_reduce<COMP>(s, c, 64);
            if ((tid & 63) == 0) {
                scratch[2 * (tid >> 6)] = s;
                scratch[2 * (tid >> 6) + 1] = c;
            }
            __syncthreads();
            if (tid == 0) {
                ACC ts = scratch[0], tc = scratch[1];
                for (int w = 1; w < kBlk / 64; ++w) combine<COMP>(ts, tc, scratch[2 * w], scratch[2 * w + 1]);
                C[o] = st_cvt<TOUT>(COMP ? ts + tc : ts);
            }
            __syncthreads();
        }
        return;
    }
    int log2R = 0;
    while ((1 << log2R) < R) ++log2R;
    const int groups = kBlk >> log2R;
    const int gi = tid >> log2R, sub = tid & (R - 1);
    const int dq = R / n_slo, dr = R - dq * n_slo;
    for (int o0 = 0; o0 < n_out; o0 += groups) {
        const int o = o0 + gi;
        const bool active = o < n_out;
        ACC s = 0, c = 0;
        if (active) {
            const int oh = o / n_olo, ol = o - oh * n_olo;
            const int2 x = toh[oh], y = tol[ol];
            const T *a0 = A + (x.x + y.x);
            const T *b0 = B;
            if constexpr (!UNARY) b0 = B + (x.y + y.y);
            if (R == 1) {
                for (int sh = 0; sh < n_shi; ++sh) {
                    const int2 h = tsh[sh];
                    const T *a1 = a0 + h.x;
                    const T *b1 = b0;
                    if constexpr (!UNARY) b1 = b0 + h.y;
                    for (int sl = 0; sl < n_slo; ++sl) {
                        const int2 l = tsl[sl];
                        ACC p = (ACC)a1[l.x];
                        if constexpr (!UNARY) p *= (ACC)b1[l.y];
                        accum<COMP>(s, c, p);
                    }
                }
            } else {
                int sh = sub / n_slo, sl = sub - sh * n_slo;
                while (sh < n_shi) {
                    const int2 h = tsh[sh], l = tsl[sl];
                    ACC p = (ACC)a0[h.x + l.x];
                    if constexpr (!UNARY) p *= (ACC)b0[h.y + l.y];
                    accum<COMP>(s, c, p);
                    sh += dq;
                    sl += dr;
                    if (sl >= n_slo) {
                        sl -= n_slo;
                        ++sh;
                    }
                }
            }
        }
        lane_reduce<COMP>(s, c, R);
        if (active && sub == 0) C[o] = st_cvt<TOUT>(COMP ? s + c : s);
    }
}

template <typename T, typename TIN, int FM>
__global__ __launch_bounds__(kBlk) void k_fused(const FusedDesc *__restrict__ nets, const int32_t *__restrict__ order,
                                               void *const *__restrict__ outs, int64_t *__restrict__ stamps,
                                               void *out1) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *sm = reinterpret_cast<T *>(smem);
    const int net = order ? order[blockIdx.x] : (int)blockIdx.x;
    const FusedDesc d = nets[net];
    const int64_t t0 = stamps ? (int64_t)wall_clock64() : 0;
    const int32_t *p = d.prog + 3;
    T *scr = (T *)d.scratch;
    for (;;) {
        const int op = p[0];
        if (op == OP_END) break;
        if (op == OP_SYNC) {
            __syncthreads();
            p += 1;
            continue;
        }
        if (op == OP_LOAD) {
            const int base = p[1], dst = p[2], size = p[3], ns = p[4];
            const TIN *src = (const TIN *)d.in[base];
            T *out = dst >= 0 ? sm + dst : scr + (-dst - 2);
            for (int e = threadIdx.x; e < size; e += kBlk) {
                T v = Ld<T, TIN>::get(src + e);
                for (int k = 0; k < ns; ++k) {
                    const int32_t *r = p + 5 + 4 * k;
                    const TIN *sp = (const TIN *)d.in[r[0]];
                    const int eh = e / r[3];
                    const int el = e - eh * r[3];
                    v *= Ld<T, TIN>::get(sp + d.tab[r[1] + eh].x + d.tab[r[2] + el].x);
                }
                out[e] = v;
            }
            p += 5 + 4 * ns;
            continue;
        }
        // OP_STEP: [a, b, c, n_ohi, n_olo, n_shi, n_slo, t_ohi, t_olo, t_shi, t_slo, R, final]
        // Locations: >= 0 LDS offset, <= -2 scratch offset -loc-2, -1 none.
        const int la = p[1], lb = p[2], lc = p[3];
        const bool unary = lb == -1;
        const bool fin = p[13] != 0;
        const int R = p[12];
        const bool all_lds = la >= 0 && (unary || lb >= 0) && (fin || lc >= 0);
        if (all_lds) {
            // every operand in LDS: the compiler sees LDS pointers
            const T *A = sm + la;
            const T *B = unary ? nullptr : sm + lb;
            if (!fin) {
                if (unary)
                    fstep<T, T, false, true, T>(A, B, sm + lc, d.tab, p + 4, R, (T *)smem);
                else
                    fstep<T, T, false, false, T>(A, B, sm + lc, d.tab, p + 4, R, (T *)smem);
            } else {
                typedef typename std::conditional<FM == FM_INTER, T, double>::type TO;
                constexpr bool CMP = (FM == FM_COMP);
                TO *C = (TO *)(out1 ? out1 : outs[net]);
                if (unary)
                    fstep<T, TO, CMP, true, TO>(A, B, C, d.tab, p + 4, R, (TO *)smem);
                else
                    fstep<T, TO, CMP, false, TO>(A, B, C, d.tab, p + 4, R, (TO *)smem);
            }
        } else {
            // some operand spilled: generic (flat) addressing
            const T *A = la >= 0 ? sm + la : scr + (-la - 2);
            const T *B = unary ? nullptr : (lb >= 0 ? sm + lb : scr + (-lb - 2));
            if (!fin) {
                T *C = lc >= 0 ? sm + lc : scr + (-lc - 2);
                if (unary)
                    fstep<T, T, false, true, T>(A, B, C, d.tab, p + 4, R, (T *)smem);
                else
                    fstep<T, T, false, false, T>(A, B, C, d.tab, p + 4, R, (T *)smem);
            } else {
                typedef typename std::conditional<FM == FM_INTER, T, double>::type TO;
                constexpr bool CMP = (FM == FM_COMP);
                TO *C = (TO *)(out1 ? out1 : outs[net]);
                if (unary)
                    fstep<T, TO, CMP, true, TO>(A, B, C, d.tab, p + 4, R, (TO *)smem);
                else
                    fstep<T, TO, CMP, false, TO>(A, B, C, d.tab, p + 4, R, (TO *)smem);
            }
        }
        p += 14;
    }
    if (stamps && threadIdx.x == 0) {
        stamps[2 * net] = t0;
        stamps[2 * net + 1] = (int64_t)wall_clock64();
    }
}

template <typename T, typename TIN, int FM>
static hipError_t go_fused(const FusedDesc *nets, const int32_t *order, void *const *outs, int64_t *stamps,
                           void *out1, int n_blocks, int lds_bytes, hipStream_t st) {
    static int configured = -1;
    if (lds_bytes > configured) {
        hipError_t e = hipFuncSetAttribute((const void *)k_fused<T, TIN, FM>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return e;
        configured = lds_bytes;
    }
    hipLaunchKernelGGL((k_fused<T, TIN, FM>), dim3(n_blocks), dim3(kBlk), lds_bytes, st, nets, order, outs, stamps,
                       out1);
    return hipGetLastError();
}

hipError_t launch_fused(const FusedDesc *nets, const int32_t *order, void *const *outs, int64_t *stamps, void *out1,
                        int n_blocks, int lds_bytes, int compute, int fm, hipStream_t st) {
    if (n_blocks <= 0) return hipSuccess;
    if (compute == 0) {
        if (fm == FM_COMP) return go_fused<double, double, FM_COMP>(nets, order, outs, stamps, out1, n_blocks, lds_bytes, st);
        return go_fused<double, double, FM_INTER>(nets, order, outs, stamps, out1, n_blocks, lds_bytes, st);
    }
    if (compute == 1) {
        if (fm == FM_COMP) return go_fused<float, float, FM_COMP>(nets, order, outs, stamps, out1, n_blocks, lds_bytes, st);
        if (fm == FM_F64) return go_fused<float, float, FM_F64>(nets, order, outs, stamps, out1, n_blocks, lds_bytes, st);
        return go_fused<float, float, FM_INTER>(nets, order, outs, stamps, out1, n_blocks, lds_bytes, st);
    }
    if (compute == 2) {
        if (fm == FM_COMP) return go_fused<float, bf16_t, FM_COMP>(nets, order, outs, stamps, out1, n_blocks, lds_bytes, st);
        if (fm == FM_F64) return go_fused<float, bf16_t, FM_F64>(nets, order, outs, stamps, out1, n_blocks, lds_bytes, st);
        return go_fused<float, bf16_t, FM_INTER>(nets, order, outs, stamps, out1, n_blocks, lds_bytes, st);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- convert

template <typename TS, typename TD>
__global__ __launch_bounds__(kBlk) void k_convert(const TS *__restrict__ s, TD *__restrict__ d, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlk) {
        float f = Ld<float, TS>::get(s + i);
        if constexpr (std::is_same<TD, bf16_t>::value)
            d[i] = f2bf(f);
        else if constexpr (std::is_same<TS, double>::value)
            d[i] = (TD)s[i];
        else
            d[i] = (TD)f;
    }
}

template <typename TS>
static hipError_t convert_from(const void *s, void *d, int td, int64_t n, dim3 g, hipStream_t st) {
    if (td == 0)
        hipLaunchKernelGGL((k_convert<TS, double>), g, dim3(kBlk), 0, st, (const TS *)s, (double *)d, n);
    else if (td == 1)
        hipLaunchKernelGGL((k_convert<TS, float>), g, dim3(kBlk), 0, st, (const TS *)s, (float *)d, n);
    else
        hipLaunchKernelGGL((k_convert<TS, bf16_t>), g, dim3(kBlk), 0, st, (const TS *)s, (bf16_t *)d, n);
    return hipGetLastError();
}

hipError_t launch_convert(const void *src, int ts, void *dst, int td, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t b = (n + kBlk - 1) / kBlk;
    dim3 g((unsigned)(b > 65536 ? 65536 : b));
    if (ts == 0) return convert_from<double>(src, dst, td, n, g, st);
    if (ts == 1) return convert_from<float>(src, dst, td, n, g, st);
    return convert_from<bf16_t>(src, dst, td, n, g, st);
}

}  // namespace kern
}  // namespace htn
