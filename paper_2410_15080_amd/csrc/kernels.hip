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
        int se = e;
        if (q.snlo > 0) {
            const int eh = e / q.snlo;
            se = tab[q.sthi + eh].x + tab[q.stlo + (e - eh * q.snlo)].x;
        }
        TI v = Ld<TI, TIN>::get(src + se);
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
                ACC s1 = 0, s2 = 0, s3 = 0;
                for (int sh = 0; sh < n_shi; ++sh) {
                    const int2 h = tsh[sh];
                    const T *a1 = a0 + h.x;
                    const T *b1 = b0;
                    if constexpr (!UNARY) b1 = b0 + h.y;
                    int sl = 0;
                    if constexpr (!COMP) {
                        // four independent partial sums (ILP)
                        for (; sl + 4 <= n_slo; sl += 4) {
                            const int2 l0 = tsl[sl], l1 = tsl[sl + 1], l2 = tsl[sl + 2], l3 = tsl[sl + 3];
                            ACC p0 = (ACC)a1[l0.x], p1 = (ACC)a1[l1.x], p2 = (ACC)a1[l2.x], p3 = (ACC)a1[l3.x];
                            if constexpr (!UNARY) {
                                p0 *= (ACC)b1[l0.y];
                                p1 *= (ACC)b1[l1.y];
                                p2 *= (ACC)b1[l2.y];
                                p3 *= (ACC)b1[l3.y];
                            }
                            s += p0;
                            s1 += p1;
                            s2 += p2;
                            s3 += p3;
                        }
                    }
                    for (; sl < n_slo; ++sl) {
                        const int2 l = tsl[sl];
                        ACC p = (ACC)a1[l.x];
                        if constexpr (!UNARY) p *= (ACC)b1[l.y];
                        accum<COMP>(s, c, p);
                    }
                }
                s += (s1 + s2) + s3;
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

// Register-tiled step: C[tcm[m] + tcn[n]] = sum_k A[k*M + m] * B[k*N + n].
// Thread (tx, ty) of a GX x (kBlk/GX) grid owns outputs m = m0 + tx + GX*i,
// n = n0 + ty + GY*j (i < TM, j < TN).  Across a wave, A reads are
// consecutive or broadcast, B reads broadcast or consecutive.
template <typename T, typename ACC, int TM, int TN, typename TOUT>
__device__ __forceinline__ void tstep(const T *A, const T *B, TOUT *C, const int *tcm, const int *tcn, int M, int N,
                                      int K, int GX) {
    int lgx = 0;
    while ((1 << lgx) < GX) ++lgx;
    const int GY = kBlk >> lgx;
    const int tx = threadIdx.x & (GX - 1), ty = threadIdx.x >> lgx;
    const int SM = GX * TM, SN = GY * TN;
    for (int m0 = 0; m0 < M; m0 += SM) {
        if (m0 + tx >= M) break;
        for (int n0 = 0; n0 < N; n0 += SN) {
            if (n0 + ty >= N) break;
            int mi[TM], nj[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int m = m0 + tx + GX * i;
                mi[i] = m < M ? m : M - 1;
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int nn = n0 + ty + GY * j;
                nj[j] = nn < N ? nn : N - 1;
            }
            // U independent partial sums over k hide LDS latency (ILP)
            constexpr int U = TM * TN >= 16 ? 1 : (TM * TN >= 8 ? 2 : (TM * TN >= 4 ? 4 : 8));
            ACC acc[U][TM][TN];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) acc[u][i][j] = 0;
            const T *a = A;
            const T *b = B;
            int k = 0;
            for (; k + U <= K; k += U) {
                T av[U][TM], bv[U][TN];
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int i = 0; i < TM; ++i) av[u][i] = a[u * M + mi[i]];
#pragma unroll
                    for (int j = 0; j < TN; ++j) bv[u][j] = b[u * N + nj[j]];
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j) acc[u][i][j] += (ACC)av[u][i] * (ACC)bv[u][j];
                a += U * M;
                b += U * N;
            }
            for (; k < K; ++k) {
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) acc[0][i][j] += (ACC)a[mi[i]] * (ACC)b[nj[j]];
                a += M;
                b += N;
            }
#pragma unroll
            for (int u = 1; u < U; ++u)
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) acc[0][i][j] += acc[u][i][j];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int m = m0 + tx + GX * i;
                if (m < M) {
                    const int cm = tcm[m];
#pragma unroll
                    for (int j = 0; j < TN; ++j) {
                        const int nn = n0 + ty + GY * j;
                        if (nn < N) C[cm + tcn[nn]] = st_cvt<TOUT>(acc[0][i][j]);
                    }
                }
            }
        }
    }
}

template <typename T, typename ACC, typename TOUT>
__device__ __forceinline__ void tstep_sel(const T *A, const T *B, TOUT *C, const int *tcm, const int *tcn, int M,
                                          int N, int K, int TM, int TN, int GX) {
    switch (TM * 8 + TN) {
        case 9: tstep<T, ACC, 1, 1, TOUT>(A, B, C, tcm, tcn, M, N, K, GX); break;
        case 10: tstep<T, ACC, 1, 2, TOUT>(A, B, C, tcm, tcn, M, N, K, GX); break;
        case 12: tstep<T, ACC, 1, 4, TOUT>(A, B, C, tcm, tcn, M, N, K, GX); break;
        case 17: tstep<T, ACC, 2, 1, TOUT>(A, B, C, tcm, tcn, M, N, K, GX); break;
        case 18: tstep<T, ACC, 2, 2, TOUT>(A, B, C, tcm, tcn, M, N, K, GX); break;
        case 20: tstep<T, ACC, 2, 4, TOUT>(A, B, C, tcm, tcn, M, N, K, GX); break;
        case 33: tstep<T, ACC, 4, 1, TOUT>(A, B, C, tcm, tcn, M, N, K, GX); break;
        case 34: tstep<T, ACC, 4, 2, TOUT>(A, B, C, tcm, tcn, M, N, K, GX); break;
        default: tstep<T, ACC, 4, 4, TOUT>(A, B, C, tcm, tcn, M, N, K, GX); break;
    }
}

// OP_TSTEP: [a, b, c, M, N, K, t_cm, t_cn, TM, TN, GX, final]
template <typename T, int FM>
__device__ __forceinline__ void tstep_dispatch(const int32_t *p, T *sm, T *scr, const int *itab, void *out) {
    const int la = p[1], lb = p[2], lc = p[3];
    const int M = p[4], N = p[5], K = p[6];
    const int *tcm = itab + p[7];
    const int *tcn = itab + p[8];
    const int TM = p[9], TN = p[10], GX = p[11];
    const bool fin = p[12] != 0;
    typedef typename std::conditional<FM == FM_INTER, T, double>::type TO;
    if (la >= 0 && lb >= 0 && (fin || lc >= 0)) {
        if (!fin)
            tstep_sel<T, T, T>(sm + la, sm + lb, sm + lc, tcm, tcn, M, N, K, TM, TN, GX);
        else
            tstep_sel<T, TO, TO>(sm + la, sm + lb, (TO *)out, tcm, tcn, M, N, K, TM, TN, GX);
    } else {
        const T *A = la >= 0 ? sm + la : scr + (-la - 2);
        const T *B = lb >= 0 ? sm + lb : scr + (-lb - 2);
        if (!fin)
            tstep_sel<T, T, T>(A, B, lc >= 0 ? sm + lc : scr + (-lc - 2), tcm, tcn, M, N, K, TM, TN, GX);
        else
            tstep_sel<T, TO, TO>(A, B, (TO *)out, tcm, tcn, M, N, K, TM, TN, GX);
    }
}

// Input materialisation for the fused kernel.  A descriptor (in the fused
// image) gives the input's device address, its destination in the network's
// workspace and the digit form of its planned layout: element e of the
// value has mixed-radix digits over the value's labels; its source offset
// and each coefficient tensor's offset are dot products of the digits with
// per-label strides.  Each thread walks e = e0, e0 + stride, ... advancing
// the digits by the digits of the stride with carries (no division in the
// loop).
// Descriptor words: [base ptr (2), dst element offset (2), size, rank, ns,
//   scale ptrs (2 each), per label k: (extent, source stride, scale strides)]
__device__ __forceinline__ const void *word_ptr(const int32_t *w) {
    return (const void *)(uintptr_t)(((uint64_t)(uint32_t)w[1] << 32) | (uint32_t)w[0]);
}

template <typename T, typename TIN>
__global__ __launch_bounds__(kBlk) void k_fprep(const FPrepEntry *__restrict__ entries) {
    const FPrepEntry en = entries[blockIdx.y];
    const int32_t *p = en.desc;
    const int64_t dst_off = (int64_t)(((uint64_t)(uint32_t)p[3] << 32) | (uint32_t)p[2]);
    const int size = p[4], rk = p[5], ns = p[6];
    const int32_t *per = p + 7 + 2 * ns;
    const int W = 2 + ns;
    const TIN *src = (const TIN *)word_ptr(p);
    T *o = (T *)en.ws + dst_off;
    const TIN *sp[kMaxScalesLoad];
#pragma unroll
    for (int q = 0; q < kMaxScalesLoad; ++q) sp[q] = q < ns ? (const TIN *)word_ptr(p + 7 + 2 * q) : nullptr;
    const int e0 = blockIdx.x * kBlk + threadIdx.x;
    const int stride = gridDim.x * kBlk;
    int dig[kMaxRankLoad], inc[kMaxRankLoad];
    int so = 0, sc[kMaxScalesLoad];
#pragma unroll
    for (int q = 0; q < kMaxScalesLoad; ++q) sc[q] = 0;
    {
        int e = e0, c = stride;
#pragma unroll
        for (int k = kMaxRankLoad - 1; k >= 0; --k) {
            if (k < rk) {
                const int dim = per[k * W];
                dig[k] = e % dim;
                e /= dim;
                inc[k] = c % dim;
                c /= dim;
                so += dig[k] * per[k * W + 1];
#pragma unroll
                for (int q = 0; q < kMaxScalesLoad; ++q)
                    if (q < ns) sc[q] += dig[k] * per[k * W + 2 + q];
            }
        }
    }
    for (int e = e0; e < size; e += stride) {
        T v = Ld<T, TIN>::get(src + so);
#pragma unroll
        for (int q = 0; q < kMaxScalesLoad; ++q)
            if (q < ns) v *= Ld<T, TIN>::get(sp[q] + sc[q]);
        o[e] = v;
        int carry = 0;
#pragma unroll
        for (int k = kMaxRankLoad - 1; k >= 0; --k) {
            if (k < rk) {
                const int dim = per[k * W];
                int dd = dig[k] + inc[k] + carry;
                carry = dd >= dim;
                if (carry) dd -= dim;
                const int delta = dd - dig[k];
                so += delta * per[k * W + 1];
#pragma unroll
                for (int q = 0; q < kMaxScalesLoad; ++q)
                    if (q < ns) sc[q] += delta * per[k * W + 2 + q];
                dig[k] = dd;
            }
        }
    }
}

// Contiguous 16-byte-chunk copies of one phase.  The copies that follow a
// step are issued into registers before the step's arithmetic and written
// to LDS after it, so their global latency overlaps the computation.
constexpr int kPrefetch = 4;  // staged chunks per thread
struct CopyOp {
    const uint4 *src;
    uint4 *dst;
    int n;
};

__device__ __forceinline__ CopyOp decode_copy(const int32_t *p, const int32_t *image, const unsigned char *ws,
                                              unsigned char *smem) {
    // [kind, src chunk, chunks, dst chunk]; kind 0: image words, 1: workspace
    CopyOp c;
    c.src = p[1] == 0 ? (const uint4 *)(image) + p[2] : (const uint4 *)ws + p[2];
    c.dst = (uint4 *)smem + p[4];
    c.n = p[3];
    return c;
}

// The fused kernel.  A workgroup copies its network's program into LDS and
// interprets it: COPY moves tables or materialised inputs into LDS,
// STEP / TSTEP contract two values, SYNC ends a phase.
template <typename T, typename TIN, int FM>
__global__ __launch_bounds__(kBlk) void k_fused(const FusedDesc *__restrict__ nets, const int32_t *__restrict__ order,
                                               void *const *__restrict__ outs, int64_t *__restrict__ stamps,
                                               void *out1, int64_t *__restrict__ phase_ticks, int max_phases) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int net = order ? order[blockIdx.x] : (int)blockIdx.x;
    int phase = 0;
    const FusedDesc d = nets[net];
    const int64_t t0 = stamps ? (int64_t)wall_clock64() : 0;
    int32_t *img = reinterpret_cast<int32_t *>(smem);
    {
        const int nw = d.prog[0];
        for (int i = threadIdx.x; i < nw; i += kBlk) img[i] = d.prog[i];
    }
    __syncthreads();
    int32_t *slots = img + img[3];
    const int slot_words = img[4];
    unsigned char *red = smem + img[5];  // reduction scratch (256 bytes)
    const int32_t *gimg = d.prog + img[6];
    T *sm = reinterpret_cast<T *>(smem);
    T *scr = (T *)d.scratch;
    void *out = out1 ? out1 : outs[net];
    const int32_t *p = img + 8;
    for (;;) {
        const int op = p[0];
        if (op == OP_END) break;
        if (op == OP_SYNC) {
            __syncthreads();
            if (phase_ticks && threadIdx.x == 0 && phase < max_phases)
                phase_ticks[(int64_t)net * max_phases + phase] = (int64_t)wall_clock64();
            ++phase;
            p += 1;
            continue;
        }
        if (op == OP_COPY) {
            const CopyOp c = decode_copy(p, gimg, (const unsigned char *)d.scratch, smem);
            for (int i = threadIdx.x; i < c.n; i += kBlk) c.dst[i] = c.src[i];
            p += 5;
            continue;
        }
        const int step_len = op == OP_TSTEP ? 14 : 15;
        // issue the following copies (next phase's tables and operands)
        CopyOp cps[4];
        int starts[5] = {0, 0, 0, 0, 0};
        int nc = 0, tot = 0;
        const int32_t *q = p + step_len;
        while (nc < 4 && q[0] == OP_COPY) {
            cps[nc] = decode_copy(q, gimg, (const unsigned char *)d.scratch, smem);
            starts[nc] = tot;
            tot += cps[nc].n;
            ++nc;
            q += 5;
        }
        starts[nc] = tot;
        uint4 stg[kPrefetch];
#pragma unroll
        for (int j = 0; j < kPrefetch; ++j) {
            const int c = threadIdx.x + j * kBlk;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k < nc && c >= starts[k] && c < starts[k + 1]) stg[j] = cps[k].src[c - starts[k]];
        }
        if (op == OP_TSTEP) {
            tstep_dispatch<T, FM>(p, sm, scr, slots + p[13] * slot_words, out);
        } else {
            // OP_STEP: [a, b, c, n_ohi, n_olo, n_shi, n_slo, t_ohi, t_olo, t_shi, t_slo, R, final, slot]
            const int2 *itab2 = reinterpret_cast<const int2 *>(slots + p[14] * slot_words);
            const int la = p[1], lb = p[2], lc = p[3];
            const bool unary = lb == -1;
            const bool fin = p[13] != 0;
            const int R = p[12];
            typedef typename std::conditional<FM == FM_INTER, T, double>::type TO;
            constexpr bool CMP = (FM == FM_COMP);
            if (la >= 0 && (unary || lb >= 0) && (fin || lc >= 0)) {
                const T *A = sm + la;
                const T *B = unary ? nullptr : sm + lb;
                if (!fin) {
                    if (unary)
                        fstep<T, T, false, true, T>(A, B, sm + lc, itab2, p + 4, R, (T *)red);
                    else
                        fstep<T, T, false, false, T>(A, B, sm + lc, itab2, p + 4, R, (T *)red);
                } else {
                    if (unary)
                        fstep<T, TO, CMP, true, TO>(A, B, (TO *)out, itab2, p + 4, R, (TO *)red);
                    else
                        fstep<T, TO, CMP, false, TO>(A, B, (TO *)out, itab2, p + 4, R, (TO *)red);
                }
            } else {
                const T *A = la >= 0 ? sm + la : scr + (-la - 2);
                const T *B = unary ? nullptr : (lb >= 0 ? sm + lb : scr + (-lb - 2));
                if (!fin) {
                    T *C = lc >= 0 ? sm + lc : scr + (-lc - 2);
                    if (unary)
                        fstep<T, T, false, true, T>(A, B, C, itab2, p + 4, R, (T *)red);
                    else
                        fstep<T, T, false, false, T>(A, B, C, itab2, p + 4, R, (T *)red);
                } else {
                    if (unary)
                        fstep<T, TO, CMP, true, TO>(A, B, (TO *)out, itab2, p + 4, R, (TO *)red);
                    else
                        fstep<T, TO, CMP, false, TO>(A, B, (TO *)out, itab2, p + 4, R, (TO *)red);
                }
            }
        }
        // land the staged chunks, copy any remainder directly
#pragma unroll
        for (int j = 0; j < kPrefetch; ++j) {
            const int c = threadIdx.x + j * kBlk;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k < nc && c >= starts[k] && c < starts[k + 1]) cps[k].dst[c - starts[k]] = stg[j];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nc)
                for (int c = threadIdx.x + kPrefetch * kBlk; c < starts[k + 1]; c += kBlk)
                    if (c >= starts[k]) cps[k].dst[c - starts[k]] = cps[k].src[c - starts[k]];
        p = q;
    }
    if (stamps && threadIdx.x == 0) {
        stamps[2 * net] = t0;
        stamps[2 * net + 1] = (int64_t)wall_clock64();
    }
}

hipError_t launch_fprep(const FPrepEntry *entries, int n_entries, int max_size, int compute, hipStream_t st) {
    if (n_entries <= 0) return hipSuccess;
    int bx = (max_size + kBlk * 4 - 1) / (kBlk * 4);
    bx = bx < 1 ? 1 : (bx > 1024 ? 1024 : bx);
    for (int first = 0; first < n_entries; first += 65535) {
        const int cnt = n_entries - first < 65535 ? n_entries - first : 65535;
        dim3 grid(bx, cnt);
        if (compute == 0)
            hipLaunchKernelGGL((k_fprep<double, double>), grid, dim3(kBlk), 0, st, entries + first);
        else if (compute == 1)
            hipLaunchKernelGGL((k_fprep<float, float>), grid, dim3(kBlk), 0, st, entries + first);
        else
            hipLaunchKernelGGL((k_fprep<float, bf16_t>), grid, dim3(kBlk), 0, st, entries + first);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, typename TIN, int FM>
static hipError_t go_fused(const FusedDesc *nets, const int32_t *order, void *const *outs, int64_t *stamps,
                           void *out1, int64_t *phase_ticks, int max_phases, int n_blocks, int lds_bytes,
                           hipStream_t st) {
    static int configured = -1;
    if (lds_bytes > configured) {
        hipError_t e = hipFuncSetAttribute((const void *)k_fused<T, TIN, FM>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        configured = lds_bytes;
    }
    hipLaunchKernelGGL((k_fused<T, TIN, FM>), dim3(n_blocks), dim3(kBlk), lds_bytes, st, nets, order, outs, stamps,
                       out1, phase_ticks, max_phases);
    return hipGetLastError();
}

hipError_t launch_fused(const FusedDesc *nets, const int32_t *order, void *const *outs, int64_t *stamps, void *out1,
                        int64_t *phase_ticks, int max_phases, int n_blocks, int lds_bytes, int compute, int fm,
                        hipStream_t st) {
    if (n_blocks <= 0) return hipSuccess;
    if (compute == 0) {
        if (fm == FM_COMP) return go_fused<double, double, FM_COMP>(nets, order, outs, stamps, out1, phase_ticks, max_phases, n_blocks, lds_bytes, st);
        return go_fused<double, double, FM_INTER>(nets, order, outs, stamps, out1, phase_ticks, max_phases, n_blocks, lds_bytes, st);
    }
    if (compute == 1) {
        if (fm == FM_COMP) return go_fused<float, float, FM_COMP>(nets, order, outs, stamps, out1, phase_ticks, max_phases, n_blocks, lds_bytes, st);
        if (fm == FM_F64) return go_fused<float, float, FM_F64>(nets, order, outs, stamps, out1, phase_ticks, max_phases, n_blocks, lds_bytes, st);
        return go_fused<float, float, FM_INTER>(nets, order, outs, stamps, out1, phase_ticks, max_phases, n_blocks, lds_bytes, st);
    }
    if (compute == 2) {
        if (fm == FM_COMP) return go_fused<float, bf16_t, FM_COMP>(nets, order, outs, stamps, out1, phase_ticks, max_phases, n_blocks, lds_bytes, st);
        if (fm == FM_F64) return go_fused<float, bf16_t, FM_F64>(nets, order, outs, stamps, out1, phase_ticks, max_phases, n_blocks, lds_bytes, st);
        return go_fused<float, bf16_t, FM_INTER>(nets, order, outs, stamps, out1, phase_ticks, max_phases, n_blocks, lds_bytes, st);
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
