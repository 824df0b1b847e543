// Persistent work queue for the networks of a batch that are too large for
// one workgroup (Sec. 6.1 contracts a network step by step; here the steps
// of many networks become one stream of tasks).
//
// Every input materialisation, every block of a table-driven step, every
// second pass of a split sum, every output tile of a matrix-core product
// and every block of a split-K sum is a task.  Each network belongs to one
// XCD: its tasks form part of that XCD's sub-queue, listed in dependency
// order (a task's producers come earlier), and only workgroups running on
// that XCD (read from the hardware XCC id) take them, in list order, from
// the sub-queue's atomic counter.  A task first waits until the counters
// of the items it reads show all their tasks done, then runs, and is
// counted done once every wave's stores have completed.  Producer and
// consumer thus always share one L2 (the XCD's), which is coherent for its
// CUs: a task needs no L2 write-back or invalidation, only an L1
// invalidation before reading what other CUs wrote.
//
// Since tasks are taken in list order, the earliest unfinished task of a
// sub-queue never waits on an unfinished task, so every sub-queue drains.
// Every wait is bounded as well: a bound that would only trip on an
// inconsistent queue sets an error flag and the task goes on, so the
// launch always ends.  The last workgroup to leave checks that every
// sub-queue was drained and restores the counters, so the next launch (or
// graph replay) starts clean without a memset.
//
// The task bodies are the per-step kernels' own (step_dev.hpp,
// mfma_dev.hpp), so a network gives the same result bit for bit through
// the queue as through per-step launches.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kern_common.hpp"
#include "kernels.hpp"
#include "mfma_dev.hpp"
#include "step_dev.hpp"

namespace htn {
namespace kern {

namespace {

constexpr int kQThreads = 256;
// Longest wait for one dependency, in ticks of the 100 MHz device clock
// (0.5 s: far beyond any legitimate wait).  Once a task has given up, the
// error flag makes every later task of the launch skip its waits, so an
// inconsistent queue still ends promptly.
constexpr int64_t kQWaitTicks = 50000000;

__device__ __forceinline__ int q_load_relaxed(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Hardware id of the XCD the calling wave runs on (HW_REG_XCC_ID).
__device__ __forceinline__ int q_xcc_id() {
    return (int)(__builtin_amdgcn_s_getreg((15 << 11) | (0 << 6) | 20) & 15u);
}

template <typename TA, typename TB, typename TC, typename ACC, bool U, bool CMP>
__device__ void q_blocks(const QItem &it, void *C, int64_t b0, int64_t b1) {
    for (int64_t blk = b0; blk < b1; ++blk)
        step_block<TA, TB, TC, ACC, U, CMP>((const TA *)it.A, (const TB *)it.B, (TC *)C, it.tab, it.s, blk);
}

// Result type and accumulation as the per-step launcher picks them.
template <typename TA, typename TB>
__device__ void q_step_tc(const QItem &it, void *C, int64_t b0, int64_t b1) {
    if (it.tc == 0) {
        if (it.unary) {
            if (it.comp)
                q_blocks<TA, TA, double, double, true, true>(it, C, b0, b1);
            else
                q_blocks<TA, TA, double, double, true, false>(it, C, b0, b1);
        } else {
            if (it.comp)
                q_blocks<TA, TB, double, double, false, true>(it, C, b0, b1);
            else
                q_blocks<TA, TB, double, double, false, false>(it, C, b0, b1);
        }
    } else if (it.tc == 1) {
        if (it.unary)
            q_blocks<TA, TA, float, float, true, false>(it, C, b0, b1);
        else
            q_blocks<TA, TB, float, float, false, false>(it, C, b0, b1);
    } else {
        if (it.unary)
            q_blocks<TA, TA, bf16_t, float, true, false>(it, C, b0, b1);
        else
            q_blocks<TA, TB, bf16_t, float, false, false>(it, C, b0, b1);
    }
}

__device__ void q_step(const QItem &it, void *C, int64_t b0, int64_t b1) {
    const int ta = it.ta, tb = it.unary ? it.ta : it.tb;
    if (ta == 0)
        q_step_tc<double, double>(it, C, b0, b1);
    else if (ta == 1 && tb == 1)
        q_step_tc<float, float>(it, C, b0, b1);
    else if (ta == 2 && tb == 2)
        q_step_tc<bf16_t, bf16_t>(it, C, b0, b1);
    else if (ta == 2)
        q_step_tc<bf16_t, float>(it, C, b0, b1);
    else
        q_step_tc<float, bf16_t>(it, C, b0, b1);
}

// Units of 4 outputs, one wave per output.
template <typename TC, bool COMP>
__device__ void q_finish_t(const QItem &it, void *C, int64_t u0, int64_t u1) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t o = 4 * u0 + wave; o < min(4 * u1, it.s.n_out); o += 4)
        split_finish_one<TC, COMP>(it.s.part, (TC *)C, it.s.split, o, lane);
}

__device__ void q_finish(const QItem &it, void *C, int64_t u0, int64_t u1) {
    if (it.tc == 0) {
        if (it.comp)
            q_finish_t<double, true>(it, C, u0, u1);
        else
            q_finish_t<double, false>(it, C, u0, u1);
    } else if (it.tc == 1) {
        q_finish_t<float, false>(it, C, u0, u1);
    } else {
        q_finish_t<bf16_t, false>(it, C, u0, u1);
    }
}

// Units of 256 elements.
template <typename TIN, typename TI>
__device__ void q_load_t(const QItem &it, void *C, int64_t u0, int64_t u1) {
    const PrepDesc &q = *it.prep;
    TI *dst = (TI *)C;
    const int64_t e1 = min(u1 * kQThreads, (int64_t)q.size);
    for (int64_t e = u0 * kQThreads + threadIdx.x; e < e1; e += kQThreads)
        dst[e] = prep_value<TIN, TI>(q, it.tab, (int)e);
}

__device__ void q_load(const QItem &it, void *C, int64_t u0, int64_t u1) {
    if (it.ta == 0)
        q_load_t<double, double>(it, C, u0, u1);
    else if (it.ta == 1)
        q_load_t<float, float>(it, C, u0, u1);
    else
        q_load_t<bf16_t, float>(it, C, u0, u1);
}

// Units of 256 elements: C[i] = the split-K partial products summed in
// range order.
template <typename TOUT>
__device__ void q_ksum_t(const QItem &it, void *C, int64_t u0, int64_t u1) {
    const TOUT *part = (const TOUT *)it.A;
    const int64_t e1 = min(u1 * kQThreads, it.total);
    for (int64_t i = u0 * kQThreads + threadIdx.x; i < e1; i += kQThreads) {
        TOUT a = part[i];
        for (int kz = 1; kz < it.ksplit; ++kz) a += part[(int64_t)kz * it.total + i];
        ((TOUT *)C)[i] = a;
    }
}

// GEMM items of one (input, output) dtype pair per queue kernel (GK 1..5:
// f64->f64, f32->f64, f32->f32, bf16->f64, bf16->f32; 0: none), so that
// each variant's registers are those of one tile shape.  Tiles of 64 x 128
// with one LDS buffer (about 26 KB): small enough for a queue workgroup to
// share a CU with a fused-kernel workgroup (up to 96 KB), so the queue
// runs beside the fused launch instead of after it.
constexpr int kQTileWI = 2;
template <int GK>
__device__ void q_gemm(const QItem &it, void *C, int64_t u0, int64_t u1, unsigned char *lds) {
    for (int64_t t = u0; t < u1; ++t) {
#define HTN_TILE(T, TOUT, C64)                                                                                  \
    gemm_tile<T, TOUT, C64, kQTileWI, 1>((const T *)it.A, (const T *)it.B, (TOUT *)C, it.M, it.N, it.K, it.kchunk,      \
                                it.ksplit, it.kper, it.batch, it.tiles_m, it.tiles_n, (int)t, lds)
        if constexpr (GK == 1) HTN_TILE(double, double, false);
        if constexpr (GK == 2) HTN_TILE(float, double, true);
        if constexpr (GK == 3) HTN_TILE(float, float, false);
        if constexpr (GK == 4) HTN_TILE(bf16_t, double, true);
        if constexpr (GK == 5) HTN_TILE(bf16_t, float, false);
#undef HTN_TILE
        __syncthreads();  // the tile's LDS is free before the next one is staged
    }
}

template <int GK>
__global__ __launch_bounds__(kQThreads) __attribute__((amdgpu_waves_per_eu(GK ? 2 : 1))) void k_queue(
    const QItem *__restrict__ items, const QTask *__restrict__ tasks, const int32_t *__restrict__ qinfo, int n_sub,
    const int32_t *__restrict__ init, int32_t *__restrict__ counters, int n_items, int32_t *__restrict__ ctrl,
    void *const *__restrict__ outs, int64_t *__restrict__ stamps, int64_t *__restrict__ run_start) {
    extern __shared__ __align__(16) unsigned char q_lds[];
    __shared__ int task_s, last_s;
    const int sub = qinfo[q_xcc_id()];  // uniform: every wave of a workgroup runs on one XCD
    if (sub >= 0) {
        const int q_beg = qinfo[QC_MAX_SUB + sub], q_len = qinfo[QC_MAX_SUB + sub + 1] - q_beg;
        // Thread 0 counts the previous task done and takes the next task in
        // one block at the top of the loop, so that every path back to the
        // loop head runs through the same barriers: were the two thread-0
        // blocks apart, the compiler could thread the lanes that skip them
        // straight back to the head and repeat a task on them.
        int prev = -1;  // the previous task's item (uniform)
        for (;;) {
            if (threadIdx.x == 0) {
                if (prev >= 0) {
                    const int left =
                        __hip_atomic_fetch_add(counters + prev, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const QItem &pi = items[prev];
                    if (stamps && (pi.flags & QF_LAST) && left == 1)
                        stamps[2 * pi.net + 1] = (int64_t)wall_clock64();
                }
                task_s = atomicAdd(ctrl + QC_NEXT + sub, 1);
            }
            __syncthreads();
            // uniform, and known to be: the loop exit must not look divergent
            const int t = __builtin_amdgcn_readfirstlane(task_s);
            if (t >= q_len) break;
            const QTask tk = tasks[q_beg + t];
            const QItem &it = items[tk.item];
            if (threadIdx.x == 0) {
                if (sub == 0 && t == 0 && run_start) *run_start = (int64_t)wall_clock64();
                for (int d = 0; d < 2; ++d) {
                    const int dep = d == 0 ? it.dep0 : it.dep1;
                    if (dep < 0 || q_load_relaxed(ctrl + QC_ERR)) continue;
                    const int64_t t0 = (int64_t)wall_clock64();
                    while (q_load_relaxed(counters + dep) > 0) {
                        if ((int64_t)wall_clock64() - t0 > kQWaitTicks) {
                            atomicExch(ctrl + QC_ERR, 1);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                // the producers ran on this XCD and their stores are in its
                // L2: drop this CU's L1 lines before the workgroup reads
                asm volatile("buffer_inv sc0" ::: "memory");
                if (stamps && (it.flags & QF_FIRST) && tk.task == 0) stamps[2 * it.net] = (int64_t)wall_clock64();
            }
            __syncthreads();  // also: every thread has read task_s before thread 0 writes it again
            void *C = (it.flags & QF_OUT) ? outs[it.net] : it.C;
            const int64_t u0 = (int64_t)tk.task * it.units_per_task;
            const int64_t u1 = min(it.n_units, u0 + it.units_per_task);
            switch (it.kind) {
                case QI_LOAD:
                    q_load(it, C, u0, u1);
                    break;
                case QI_STEP:
                    q_step(it, C, u0, u1);
                    break;
                case QI_FINISH:
                    q_finish(it, C, u0, u1);
                    break;
                case QI_GEMM:
                    if constexpr (GK != 0) q_gemm<GK>(it, C, u0, u1, q_lds);
                    break;
                default:
                    if (it.tc == 0)
                        q_ksum_t<double>(it, C, u0, u1);
                    else
                        q_ksum_t<float>(it, C, u0, u1);
                    break;
            }
            // every wave waits until its stores have reached the L2 (a
            // workgroup-scope fence does not wait: the waves share one CU);
            // thread 0 then counts the task done at the top of the loop
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            prev = __builtin_amdgcn_readfirstlane(tk.item);
        }
    }
    // The last workgroup out checks that every sub-queue was drained and
    // restores the counters for the next launch: by then every other
    // workgroup has stopped touching them.  (The last task's count was made
    // at the top of the final pass of the loop.)
    if (threadIdx.x == 0)
        last_s = __hip_atomic_fetch_add(ctrl + QC_EXITED, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
                 (int)gridDim.x - 1;
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(last_s)) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        for (int i = threadIdx.x; i < n_items; i += kQThreads) counters[i] = init[i];
        if (threadIdx.x == 0) {
            for (int k = 0; k < n_sub; ++k) {
                if (q_load_relaxed(ctrl + QC_NEXT + k) < qinfo[QC_MAX_SUB + k + 1] - qinfo[QC_MAX_SUB + k])
                    atomicExch(ctrl + QC_ERR, 2);
                ctrl[QC_NEXT + k] = 0;
            }
            ctrl[QC_EXITED] = 0;
        }
    }
}

// One wave per workgroup records the XCD it runs on.
__global__ void k_xcc_probe(uint32_t *mask) {
    if (threadIdx.x == 0) atomicOr(mask, 1u << q_xcc_id());
}

template <int GK>
hipError_t go_queue(const QItem *items, const QTask *tasks, const int32_t *qinfo, int n_sub, const int32_t *init,
                    int32_t *counters, int n_items, int32_t *ctrl, void *const *outs, int64_t *stamps,
                    int64_t *run_start, int lds_bytes, int n_blocks, hipStream_t st) {
    static int configured = -1;
    if (lds_bytes > configured) {
        hipError_t e =
            hipFuncSetAttribute((const void *)k_queue<GK>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        configured = lds_bytes;
    }
    hipLaunchKernelGGL((k_queue<GK>), dim3((unsigned)n_blocks), dim3(kQThreads), lds_bytes, st, items, tasks, qinfo,
                       n_sub, init, counters, n_items, ctrl, outs, stamps, run_start);
    return hipGetLastError();
}

template <int GK>
int blocks_per_cu(int lds_bytes) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_queue<GK>, kQThreads, lds_bytes) != hipSuccess || n < 1) {
        (void)hipGetLastError();
        return 1;
    }
    return n;
}

}  // namespace

int queue_gemm_kind(int tin, int tout) {
    if (tin == 0) return tout == 0 ? 1 : -1;
    if (tin == 1) return tout == 0 ? 2 : (tout == 1 ? 3 : -1);
    if (tin == 2) return tout == 0 ? 4 : (tout == 1 ? 5 : -1);
    return -1;
}

int queue_gemm_lds(int gk) {
    switch (gk) {
        case 1: return gemm_lds_bytes<double, kQTileWI, 1>();
        case 2: case 3: return gemm_lds_bytes<float, kQTileWI, 1>();
        case 4: case 5: return gemm_lds_bytes<bf16_t, kQTileWI, 1>();
        default: return 0;
    }
}

int queue_tile_rows() { return 32 * kQTileWI; }

int queue_blocks_per_cu(int gk, int lds_bytes) {
    switch (gk) {
        case 0: return blocks_per_cu<0>(lds_bytes);
        case 1: return blocks_per_cu<1>(lds_bytes);
        case 2: return blocks_per_cu<2>(lds_bytes);
        case 3: return blocks_per_cu<3>(lds_bytes);
        case 4: return blocks_per_cu<4>(lds_bytes);
        case 5: return blocks_per_cu<5>(lds_bytes);
        default: return 1;
    }
}

hipError_t launch_queue(const QItem *items, const QTask *tasks, const int32_t *qinfo, int n_sub, const int32_t *init,
                        int32_t *counters, int n_items, int32_t *ctrl, void *const *outs, int64_t *stamps,
                        int64_t *run_start, int gk, int lds_bytes, int n_blocks, hipStream_t st) {
    if (n_sub < 1 || n_sub > QC_MAX_SUB || n_blocks <= 0) return hipErrorInvalidValue;
#define HTN_GO(G) go_queue<G>(items, tasks, qinfo, n_sub, init, counters, n_items, ctrl, outs, stamps, run_start, lds_bytes, n_blocks, st)
    switch (gk) {
        case 0: return HTN_GO(0);
        case 1: return HTN_GO(1);
        case 2: return HTN_GO(2);
        case 3: return HTN_GO(3);
        case 4: return HTN_GO(4);
        case 5: return HTN_GO(5);
        default: return hipErrorInvalidValue;
    }
#undef HTN_GO
}

uint32_t queue_xcc_mask(uint32_t *d_word) {
    if (hipMemset(d_word, 0, sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    uint32_t h = 0;
    hipLaunchKernelGGL(k_xcc_probe, dim3(4096), dim3(64), 0, 0, d_word);
    if (hipGetLastError() != hipSuccess || hipMemcpy(&h, d_word, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return h;
}

}  // namespace kern
}  // namespace htn
