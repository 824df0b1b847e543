// HIP kernels for h-TN contraction on gfx950 (wave64).
//
//  k_step   one pairwise contraction C[o] = sum_s A[.]*B[.] over arbitrary
//           label layouts.  The operand offsets of output index o and summed
//           index s come from two-level offset tables built by the planner,
//           so one kernel covers every permutation, hyperedge (batch) label,
//           single-operand summed label and outer product.  R lanes
//           cooperate on one output and reduce with cross-lane shuffles.
//  k_prep   applies coefficient tensors folded into an input (entry-wise
//           scaling: a coefficient vector on a cut index is a diagonal
//           scaling of a QT carrying that index, absorbed at load time) and
//           converts to the intermediate type.
//  k_fprep  materialises the inputs of fused networks (layout change and
//           coefficient scaling) into their workspaces.
//  The fused whole-network kernel lives in fused.hpp / fused_b*.hip.
#include <algorithm>
#include <climits>
#include <type_traits>

#include "kern_common.hpp"
#include "step_dev.hpp"

namespace htn {
namespace kern {
// ------------------------------------------------------------------ k_step

template <typename TA, typename TB, typename TC, typename ACC, bool UNARY, bool COMP>
__global__ __launch_bounds__(kBlk) void k_step(const TA *__restrict__ A, const TB *__restrict__ B, TC *__restrict__ C,
                                              const int2 *__restrict__ tab, StepArgs s) {
    step_block<TA, TB, TC, ACC, UNARY, COMP>(A, B, C, tab, s, blockIdx.x);
}

// Second pass of a split sum: one wave per output.
template <typename TC, bool COMP>
__global__ __launch_bounds__(64) void k_split_finish(const double *__restrict__ part, TC *__restrict__ C,
                                                    int split) {
    split_finish_one<TC, COMP>(part, C, split, blockIdx.x, threadIdx.x);
}

template <typename TA, typename TB, typename TC, typename ACC, bool U, bool CMP>
static hipError_t go_step(const void *A, const void *B, void *C, const int2 *tab, const StepArgs &s,
                          hipStream_t st) {
    const int64_t threads = s.n_out * (int64_t)s.R * (s.split > 1 ? s.split : 1);
    const int64_t blocks = (threads + kBlk - 1) / kBlk;
    hipLaunchKernelGGL((k_step<TA, TB, TC, ACC, U, CMP>), dim3((unsigned)blocks), dim3(kBlk), 0, st,
                       (const TA *)A, (const TB *)B, (TC *)C, tab, s);
    if (s.split > 1)
        hipLaunchKernelGGL((k_split_finish<TC, CMP>), dim3((unsigned)s.n_out), dim3(64), 0, st, s.part, (TC *)C,
                           s.split);
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
    if (tc == 2 && !comp) {
        if (unary) return go_step<TA, TA, bf16_t, float, true, false>(A, B, C, tab, s, st);
        return go_step<TA, TB, bf16_t, float, false, false>(A, B, C, tab, s, st);
    }
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
__global__ __launch_bounds__(kBlk) void k_prep(const PrepDesc *__restrict__ descs, const int2 *__restrict__ tab,
                                                unsigned char *__restrict__ ws) {
    const PrepDesc &q = descs[blockIdx.y];
    TI *dst = (TI *)(ws + q.dst_off);
    for (int e = blockIdx.x * kBlk + threadIdx.x; e < q.size; e += gridDim.x * kBlk)
        dst[e] = prep_value<TIN, TI>(q, tab, e);
}

hipError_t launch_prep(const PrepDesc *d_desc, int n_desc, int max_size, int tin, int tinter, const int2 *tab,
                       void *ws, hipStream_t st) {
    if (n_desc <= 0) return hipSuccess;
    int bx = (max_size + kBlk * 4 - 1) / (kBlk * 4);
    bx = bx < 1 ? 1 : (bx > 4096 ? 4096 : bx);
    dim3 grid(bx, n_desc);
    if (tin == 0 && tinter == 0)
        hipLaunchKernelGGL((k_prep<double, double>), grid, dim3(kBlk), 0, st, d_desc, tab, (unsigned char *)ws);
    else if (tin == 1 && tinter == 1)
        hipLaunchKernelGGL((k_prep<float, float>), grid, dim3(kBlk), 0, st, d_desc, tab, (unsigned char *)ws);
    else if (tin == 2 && tinter == 1)
        hipLaunchKernelGGL((k_prep<bf16_t, float>), grid, dim3(kBlk), 0, st, d_desc, tab, (unsigned char *)ws);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Input materialisation for the fused kernel, as its own launch (one wave
// per entry); used for networks whose inputs are too large to materialise
// inside their fused workgroup.
// The digit loop is unrolled to a bound on the rank and the number of
// scales; small bounds for the common small loads keep the code a wave
// runs through short (the fully unrolled general form is several times
// larger and its instruction fetches, not its arithmetic, set the time).
template <typename T, typename TIN>
__global__ __launch_bounds__(64) void k_fprep(const FPrepEntry *__restrict__ entries, int64_t *stamp) {
    const int lane = threadIdx.x;
    if (stamp && blockIdx.x == 0 && lane == 0) *stamp = (int64_t)wall_clock64();
    const FPrepEntry en = entries[blockIdx.x];
    if (en.n_words > 64) {
        fprep_entry<T, TIN>(en, lane);
        return;
    }
    const LaneWords p(en.desc, en.n_words, lane);
    const int rk = p(5), ns = p(6);
    if (rk <= 4 && ns <= 4)
        fprep_words<T, TIN, LaneWords, 4, 4>(p, en.ws, en.e0, lane);
    else if (rk <= 8 && ns <= 8)
        fprep_words<T, TIN, LaneWords, 8, 8>(p, en.ws, en.e0, lane);
    else
        fprep_words<T, TIN, LaneWords>(p, en.ws, en.e0, lane);
}

// Entries of rank <= 4 with at most 4 scales only (form 0): the short
// unrolled form alone (descriptors of at most 47 words).
template <typename T, typename TIN>
__global__ __launch_bounds__(64) void k_fprep_small(const FPrepEntry *__restrict__ entries, int64_t *stamp) {
    const int lane = threadIdx.x;
    if (stamp && blockIdx.x == 0 && lane == 0) *stamp = (int64_t)wall_clock64();
    const FPrepEntry en = entries[blockIdx.x];
    const LaneWords p(en.desc, en.n_words, lane);
    fprep_words<T, TIN, LaneWords, 4, 4>(p, en.ws, en.e0, lane);
}

// Entries of rank <= 6 with at most 6 scales (form 1); descriptors of more
// than 64 words (up to 79) are read through the constant address space.
template <typename T, typename TIN>
__global__ __launch_bounds__(64) void k_fprep_mid(const FPrepEntry *__restrict__ entries, int64_t *stamp) {
    const int lane = threadIdx.x;
    if (stamp && blockIdx.x == 0 && lane == 0) *stamp = (int64_t)wall_clock64();
    const FPrepEntry en = entries[blockIdx.x];
    if (en.n_words > 64) {
        fprep_words<T, TIN, ConstWords, 6, 6>(ConstWords{(const c_int32 *)en.desc}, en.ws, en.e0, lane);
        return;
    }
    const LaneWords p(en.desc, en.n_words, lane);
    const int rk = p(5), ns = p(6);
    if (rk <= 4 && ns <= 4)
        fprep_words<T, TIN, LaneWords, 4, 4>(p, en.ws, en.e0, lane);
    else
        fprep_words<T, TIN, LaneWords, 6, 6>(p, en.ws, en.e0, lane);
}

// Device clock read into *dst (one thread).
__global__ void k_stamp(int64_t *dst) {
    if (threadIdx.x == 0) *dst = (int64_t)wall_clock64();
}

// ------------------------------------------------------------------ k_fold

// A tile is worked through in dependent passes (load, one per fold,
// store): 1024 threads per workgroup shorten each pass (narrower tiles with
// more workgroups per CU measured slower).
constexpr int kFoldBlk = 1024;
// matrices of at most this many entries are staged in LDS for their fold
constexpr int kFoldStagedM = 256;

// One workgroup per tf outer indices; LDS holds two [d_max][tf + 1]
// buffers (the +1 keeps the destination-order reads off one bank) and the
// outer offsets of its tf indices.  Every per-element index comes from the
// descriptor's tables: no integer division in the element loops.
// Several independent chains may share a launch (FoldBatch): each takes
// its own range of workgroups, so their tiles run side by side.  The
// source of the first chain has type TS0, that of the second TS1.
template <typename TS0, typename TS1, typename TM, typename TI, typename TO>
__global__ __launch_bounds__(kFoldBlk) void k_fold(const FoldBatch fb) {
    extern __shared__ __align__(16) unsigned char fold_lds[];
    static_assert(kFoldBatch == 2, "the chain of a workgroup is picked from two");
    const int c = (fb.n > 1 && (int)blockIdx.x >= fb.blk0[1]) ? 1 : 0;
    const FoldDesc &fd = c ? fb.fd[1] : fb.fd[0];
    const void *const srcv = c ? fb.src[1] : fb.src[0];
    TO *__restrict__ dst = (TO *)(c ? fb.dst[1] : fb.dst[0]);
    const int blk = (int)blockIdx.x - fb.blk0[c];
    const int tf = fd.tf, ld = tf + 1, lg = fd.lg_tf;
    __shared__ int64_t o_src[64], o_dst[64];
    TI *bin = (TI *)fold_lds;
    TI *bout = bin + (int64_t)fd.d_max * ld;
    // XCD-aware tile order: workgroups are dealt to the eight XCDs in turn,
    // so the workgroups of one XCD take a contiguous range of tiles and
    // neighbouring tiles (which share source cache lines) share its L2
    const int64_t n_tiles = (fd.n_outer_total + tf - 1) / tf;
    const int64_t per_xcd = (n_tiles + 7) / 8;
    const int64_t tile = (int64_t)(blk % 8) * per_xcd + blk / 8;
    if (tile >= n_tiles) return;  // whole workgroup: before any barrier
    const int64_t f0 = tile * tf;
    if (threadIdx.x < tf) {
        int64_t f = f0 + threadIdx.x, os = 0, od = 0;
        if (f < fd.n_outer_total) {
            for (int j = fd.n_outer - 1; j >= 0; --j) {
                const int64_t q = f / fd.o_ext[j], d = f - q * fd.o_ext[j];
                os += d * fd.o_src[j];
                od += d * fd.o_dst[j];
                f = q;
            }
        } else {
            os = od = -1;
        }
        o_src[threadIdx.x] = os;
        o_dst[threadIdx.x] = od;
    }
    __syncthreads();
    const int32_t *tsrc = fd.tab + fd.t_src;
    int D = 1;
    for (int j = 0; j < fd.n_ax; ++j) D *= fd.ext0[j];
    // stage the source: outer index fastest across threads (coalesced along
    // the source's fastest outer axis); kFoldLoads loads in flight per
    // thread (each a table read, then the source read it addresses)
    constexpr int kFoldLoads = 8;
    auto stage = [&](auto tag) {
        typedef decltype(tag) TS;
        const TS *__restrict__ src = (const TS *)srcv;
        for (int e0 = threadIdx.x; e0 < (D << lg); e0 += kFoldBlk * kFoldLoads) {
            TI v[kFoldLoads];
            int dl[kFoldLoads];
#pragma unroll
            for (int u = 0; u < kFoldLoads; ++u) {
                const int e = e0 + u * kFoldBlk;
                dl[u] = -1;
                if (e < (D << lg)) {
                    const int a = e >> lg, fl = e & (tf - 1);
                    const int64_t os = o_src[fl];
                    dl[u] = a * ld + fl;
                    v[u] = os >= 0 ? Ld<TI, TS>::get(src + os + tsrc[a]) : TI(0);
                }
            }
#pragma unroll
            for (int u = 0; u < kFoldLoads; ++u)
                if (dl[u] >= 0) bin[dl[u]] = v[u];
        }
    };
    if (c == 0)  // workgroup-uniform
        stage(TS0{});
    else
        stage(TS1{});
    __syncthreads();
    __shared__ TI m_s[kFoldStagedM];
    for (int st = 0; st < fd.n_stage; ++st) {
        const int din = fd.d_in_ax[st], inner = fd.inner[st], dout = fd.d_out[st];
        const int Dn = D / din * dout;
        const int32_t *tb = fd.tab + fd.t_base[st], *tm = fd.tab + fd.t_mid[st];
        const TM *M = (const TM *)fd.m[st];
        const int mi = fd.m_in[st], mo = fd.m_out[st];
        // a small matrix is staged in LDS as [old digit][new digit], so the
        // sums read no global memory; the terms are added in the same order
        const bool staged = din * dout <= kFoldStagedM;  // workgroup-uniform
        if (staged) {
            for (int q = threadIdx.x; q < din * dout; q += kFoldBlk) {
                const int k = q / dout, o = q - k * dout;
                m_s[q] = Ld<TI, TM>::get(M + (int64_t)k * mi + (int64_t)o * mo);
            }
            __syncthreads();
        }
#pragma unroll 4
        for (int e = threadIdx.x; e < (Dn << lg); e += kFoldBlk) {
            const int a = e >> lg, fl = e & (tf - 1);
            const TI *x = bin + tb[a] * ld + fl;
            const int mid = tm[a];
            TI acc = 0;
            if (staged) {
                const TI *ms = m_s + mid;
#pragma unroll 4
                for (int k = 0; k < din; ++k) acc += x[k * inner * ld] * ms[k * dout];
            } else {
                const TM *m = M + mid * mo;
                for (int k = 0; k < din; ++k) acc += x[k * inner * ld] * Ld<TI, TM>::get(m + k * mi);
            }
            bout[a * ld + fl] = acc;
        }
        __syncthreads();
        TI *t = bin;
        bin = bout;
        bout = t;
        D = Dn;
    }
    // write: in-tile index fastest across threads (contiguous in the
    // destination's fastest in-tile axes)
    const int32_t *tdst = fd.tab + fd.t_dst;
    for (int e = threadIdx.x; e < D * tf; e += kFoldBlk) {
        const int fl = e / D, a = e - fl * D;
        if (o_dst[fl] >= 0) dst[o_dst[fl] + tdst[a]] = st_cvt<TO>(bin[a * ld + fl]);
    }
}

template <typename TS0, typename TS1, typename TM, typename TI, typename TO>
static hipError_t go_fold(const FoldBatch &fb, int lds_bytes, hipStream_t st) {
    static int configured = -1;
    if (lds_bytes > configured) {
        hipError_t e = hipFuncSetAttribute((const void *)k_fold<TS0, TS1, TM, TI, TO>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        configured = lds_bytes;
    }
    hipLaunchKernelGGL((k_fold<TS0, TS1, TM, TI, TO>), dim3((unsigned)fb.blk0[fb.n]), dim3(kFoldBlk), lds_bytes,
                       st, fb);
    return hipGetLastError();
}

// BF16 arithmetic paths: each chain's source is FP32 or BF16
template <typename TO>
static hipError_t go_fold_bf(const FoldBatch &fb, int lds, int ts0, int ts1, hipStream_t st) {
    if (ts0 == 2 && ts1 == 2) return go_fold<bf16_t, bf16_t, bf16_t, float, TO>(fb, lds, st);
    if (ts0 == 2 && ts1 == 1) return go_fold<bf16_t, float, bf16_t, float, TO>(fb, lds, st);
    if (ts0 == 1 && ts1 == 2) return go_fold<float, bf16_t, bf16_t, float, TO>(fb, lds, st);
    if (ts0 == 1 && ts1 == 1) return go_fold<float, float, bf16_t, float, TO>(fb, lds, st);
    return hipErrorInvalidValue;
}

// tm, ti, to: matrix, arithmetic and destination types (0 double, 1 float,
// 2 bf16); every job's source type is jobs[j].ts
static hipError_t go_folds(const FoldJob *jobs, int n, int tm, int ti, int to, hipStream_t st) {
    static_assert(sizeof(FoldBatch) <= 2048, "fold launch arguments");
    for (int j0 = 0; j0 < n; j0 += kFoldBatch) {
        FoldBatch fb;
        fb.n = std::min(kFoldBatch, n - j0);
        fb.blk0[0] = 0;
        int lds = 0;
        for (int c = 0; c < fb.n; ++c) {
            const FoldDesc &fd = *jobs[j0 + c].fd;
            fb.fd[c] = fd;
            fb.src[c] = jobs[j0 + c].src;
            fb.dst[c] = jobs[j0 + c].dst;
            const int64_t blocks = 8 * (((fd.n_outer_total + fd.tf - 1) / fd.tf + 7) / 8);
            if (fb.blk0[c] + blocks > INT32_MAX) return hipErrorInvalidValue;
            fb.blk0[c + 1] = fb.blk0[c] + (int32_t)blocks;
            lds = std::max(lds, fd.lds_bytes);
        }
        for (int c = fb.n; c < kFoldBatch; ++c) fb.blk0[c + 1] = fb.blk0[c];
        const int ts0 = jobs[j0].ts, ts1 = fb.n > 1 ? jobs[j0 + 1].ts : ts0;
        hipError_t e = hipErrorInvalidValue;
        if (tm == 0 && ti == 0 && to == 0 && ts0 == 0 && ts1 == 0)
            e = go_fold<double, double, double, double, double>(fb, lds, st);
        else if (tm == 1 && ti == 1 && to == 1 && ts0 == 1 && ts1 == 1)
            e = go_fold<float, float, float, float, float>(fb, lds, st);
        else if (tm == 2 && ti == 1 && to == 2)
            e = go_fold_bf<bf16_t>(fb, lds, ts0, ts1, st);
        else if (tm == 2 && ti == 1 && to == 1)
            e = go_fold_bf<float>(fb, lds, ts0, ts1, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_folds(const FoldJob *jobs, int n, int tm, int ti, int to, hipStream_t st) {
    if (n < 1 || !jobs) return hipErrorInvalidValue;
    for (int j = 0; j < n; ++j) {
        const FoldDesc *fd = jobs[j].fd;
        if (!fd || fd->n_outer_total <= 0 || fd->tf < 1 || fd->tf > 64 || (1 << fd->lg_tf) != fd->tf || !fd->tab)
            return hipErrorInvalidValue;
    }
    return go_folds(jobs, n, tm, ti, to, st);
}

// ------------------------------------------------------------- k_slice_sum

// out[e] = sum over slices k (in order) of parts[k * n + e], accumulated in
// FP64 (Neumaier-compensated when COMP), stored in the output type.
template <typename T, bool COMP>
__global__ __launch_bounds__(kBlk) void k_slice_sum(const T *__restrict__ parts, int n_slices, int64_t n,
                                                    T *__restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * kBlk + threadIdx.x; e < n; e += (int64_t)gridDim.x * kBlk) {
        double s = 0.0, c = 0.0;
        for (int k = 0; k < n_slices; ++k) accum<COMP>(s, c, (double)parts[(int64_t)k * n + e]);
        out[e] = (T)(COMP ? s + c : s);
    }
}

hipError_t launch_slice_sum(const void *parts, int n_slices, int64_t n, void *out, int tout, bool comp,
                            hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + kBlk - 1) / kBlk, 8192);
    const dim3 grid((unsigned)blocks), block(kBlk);
    if (tout == 0 && comp)
        hipLaunchKernelGGL((k_slice_sum<double, true>), grid, block, 0, st, (const double *)parts, n_slices, n,
                           (double *)out);
    else if (tout == 0)
        hipLaunchKernelGGL((k_slice_sum<double, false>), grid, block, 0, st, (const double *)parts, n_slices, n,
                           (double *)out);
    else if (tout == 1)
        hipLaunchKernelGGL((k_slice_sum<float, false>), grid, block, 0, st, (const float *)parts, n_slices, n,
                           (float *)out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_stamp(int64_t *dst, hipStream_t st) {
    hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, st, dst);
    return hipGetLastError();
}

template <typename T, typename TIN>
static void go_fprep(const FPrepEntry *entries, int n_entries, int form, int64_t *stamp, hipStream_t st) {
    const dim3 grid(n_entries);
    if (form == 0)
        hipLaunchKernelGGL((k_fprep_small<T, TIN>), grid, dim3(64), 0, st, entries, stamp);
    else if (form == 1)
        hipLaunchKernelGGL((k_fprep_mid<T, TIN>), grid, dim3(64), 0, st, entries, stamp);
    else
        hipLaunchKernelGGL((k_fprep<T, TIN>), grid, dim3(64), 0, st, entries, stamp);
}

hipError_t launch_fprep(const FPrepEntry *entries, int n_entries, int form, int max_size, int compute,
                        int64_t *stamp, hipStream_t st) {
    (void)max_size;
    if (n_entries <= 0) return hipSuccess;
    if (form < 0 || form > 2 || compute < 0 || compute > 2) return hipErrorInvalidValue;
    if (compute == 0)
        go_fprep<double, double>(entries, n_entries, form, stamp, st);
    else if (compute == 1)
        go_fprep<float, float>(entries, n_entries, form, stamp, st);
    else
        go_fprep<float, bf16_t>(entries, n_entries, form, stamp, st);
    return hipGetLastError();
}

hipError_t launch_fused(const FusedDesc *nets, const int32_t *order, void *const *outs, int64_t *stamps, void *out1,
                        int64_t *phase_ticks, int max_phases, int n_blocks, int lds_bytes, int compute, int fm,
                        int threads, hipStream_t st) {
    if (n_blocks <= 0) return hipSuccess;
    if (threads == 64)
        return launch_fused_blk<64>(nets, order, outs, stamps, out1, phase_ticks, max_phases, n_blocks, lds_bytes,
                                    compute, fm, st);
    if (threads == 256)
        return launch_fused_blk<256>(nets, order, outs, stamps, out1, phase_ticks, max_phases, n_blocks, lds_bytes,
                                     compute, fm, st);
    if (threads == 512)
        return launch_fused_blk<512>(nets, order, outs, stamps, out1, phase_ticks, max_phases, n_blocks, lds_bytes,
                                     compute, fm, st);
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

