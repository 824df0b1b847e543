// C ABI of the h-TN library: handles, device state, executors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <limits>
#include <mutex>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "htn.h"
#include "htn_core.hpp"
#include "kernels.hpp"
#include "mfma_dev.hpp"

using namespace htn;

static thread_local std::string g_err;

static htn_status fail(htn_status s, const std::string &m) {
    g_err = m;
    return s;
}

// On failure the thread's sticky HIP error is cleared so that it is not
// reported again by an unrelated later call.
#define HIP_TRY(x)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) {                                                           \
            (void)hipGetLastError();                                                      \
            throw Error{HTN_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)};    \
        }                                                                                 \
    } while (0)

#define API_GUARD_BEGIN try {
#define API_GUARD_END                                                  \
    }                                                                  \
    catch (const Error &e) {                                           \
        return fail(e.st, e.msg);                                      \
    }                                                                  \
    catch (const std::bad_alloc &) {                                   \
        return fail(HTN_E_OOM, "host allocation failed");              \
    }                                                                  \
    catch (...) {                                                      \
        return fail(HTN_E_ARG, "unexpected internal error");           \
    }

namespace htn {
struct DeviceState {
    int device = -1;
    std::vector<void *> in;  // per tensor, compute input dtype
    std::vector<char> own;
    void **d_inptrs = nullptr;
    int32_t *d_prog = nullptr;
    int2 *d_tab = nullptr;
    void *d_ws = nullptr;
    int64_t ws_cap = 0;
    // materialisations of the loads that need a copy: first those the
    // per-step executor runs (n_prep_steps; the rest are fold-chain sources
    // it reads in place), then the others; prep_index[k]: the entry of the
    // k-th such load in plan order (the work queue runs them all)
    kern::PrepDesc *d_prep = nullptr;
    int n_prep = 0, n_prep_steps = 0, prep_max = 0;
    std::vector<int> prep_index;
    kern::FusedDesc *d_fdesc = nullptr;
    kern::FPrepEntry *d_fprep = nullptr;  // input materialisation of the fused path
    std::vector<kern::FPrepEntry> fprep;
    int fprep_form = 0;  // the longest load form among them (kern::fprep_form)
    int fprep_max = 0;
    bool fprep_in_kernel = false;  // the fused workgroup materialises its inputs
    int plan_uploaded = -1;
    int64_t uploads = 0;  // input and plan uploads so far (a batch holds the addresses of one)
    std::vector<kern::FoldDesc> folds;  // per fold chain of the plan (per-step executor)
    int32_t *d_fold_tab = nullptr;      // their index tables
    struct SliceRun *slices = nullptr;  // a sliced net's slice networks (built at first use)
};
}  // namespace htn

static void free_slices(htn::DeviceState &D);
static void run_sliced(htn::Net &n, void *out, hipStream_t st);

// A network contracted on its own (htn_contract, fused) whose inputs total
// at most this many elements materialises them inside its workgroup, which
// saves a launch.  Batches materialise every network's inputs in one wide
// launch instead: spread over thousands of waves it finishes sooner than
// per-workgroup prologues.
static constexpr int64_t kInKernelPrepMax = 65536;

static kern::FusedDesc fused_desc(const DeviceState &D, bool in_kernel_prep, bool lds_only) {
    const bool k = in_kernel_prep && D.fprep_in_kernel;
    return kern::FusedDesc{D.d_prog, D.d_tab, (const void *const *)D.d_inptrs, D.d_ws, k ? D.d_fprep : nullptr,
                           k ? (int32_t)D.fprep.size() : 0, lds_only ? 1 : 0};
}

struct htn_net : public Net {};

struct htn_batch {
    struct Group {
        int compute = 0, fm = 0, lds = 0, threads = 256;
        std::vector<int> idx;  // net indices, heaviest first
        int32_t *d_order = nullptr;
        kern::FPrepEntry *d_fprep = nullptr;  // input materialisation of every net
        int n_fprep = 0, fprep_form = 0, fprep_max = 0;
    };
    std::vector<htn_net *> nets;
    std::vector<int> versions;
    std::vector<Group> groups;
    std::vector<int> step_nets;
    std::vector<int64_t> uploads;  // each net's DeviceState::uploads at creation
    // Work queue of the step-by-step nets (in_queue[k]: step_nets[k] is in
    // it); it runs on its own side stream when the batch has a fused launch.
    struct Queue {
        kern::QItem *d_items = nullptr;
        kern::QTask *d_tasks = nullptr;
        int32_t *d_counters = nullptr, *d_init = nullptr, *d_ctrl = nullptr, *d_qinfo = nullptr;
        void *d_ws = nullptr;
        int n_items = 0, n_tasks = 0, n_nets = 0, gk = 0, lds = 0, n_blocks = 0, n_sub = 0;
        hipStream_t stream = nullptr;
        hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    } q;
    std::vector<char> in_queue;
    kern::FusedDesc *d_desc = nullptr;
    void **d_outs = nullptr;
    int64_t *d_stamps = nullptr;
    std::vector<void *> outs_uploaded;
    bool use_graph = false;
    bool force_capture_failure = false;  // host-forced: the capture fails (tests the fallback)
    bool graph_failed = false;           // a capture failed: runs stay eager
    std::string graph_error;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t graph_stream = nullptr;
    std::vector<void *> graph_outs;
    int64_t *d_phase = nullptr;  // per-phase clock of fused nets (optional)
    int max_phases = 0;
    // Nets run step by step go on side streams, forked from and joined back
    // to the caller's stream, so they overlap each other and the fused
    // launch; side_of[k] is the side stream of step_nets[k].
    std::vector<hipStream_t> sides;
    std::vector<hipEvent_t> ev_join;
    hipEvent_t ev_fork = nullptr;
    std::vector<int> side_of;
    // Optional HIP events around the prep and fused launches of eager runs
    // (htn_batch_set_event_timing): three per run.
    bool event_timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
};

// Side streams of a batch (nets run step by step in parallel).
static constexpr int kSideStreams = 3;
// A net eligible for the fused launch still runs step by step in a batch
// when it would hold one workgroup far longer than the batch's average
// share: above max(kStragglerFloor, kStragglerFactor * mean mults per
// resident workgroup slot).
static constexpr double kStragglerFloor = 1048576.0;
static constexpr double kStragglerFactor = 4.0;
// Resident fused workgroups per CU for a net's launch shape: the fused
// kernel keeps at most two waves per SIMD (eight per CU), and a CU's
// kLdsPerCu bytes of LDS bound the workgroups by their dynamic LDS.
static constexpr int kLdsPerCu = 160 * 1024;
static int fused_slots_per_cu(int threads, int64_t lds_bytes) {
    const int by_waves = std::max(1, 8 / std::max(1, threads / 64));
    const int by_lds = lds_bytes > 0 ? (int)std::max<int64_t>(1, kLdsPerCu / lds_bytes) : by_waves;
    return std::min(by_waves, by_lds);
}
static bool queue_by_default(const Net &n);
static std::vector<int> device_xccs(int dev);

// ------------------------------------------------------------- helpers

// Device memory of the library: hipMalloc/hipFree, or the caller's
// allocator (htn_set_allocator).  Each block remembers the free routine of
// the allocator that made it, so changing the allocator later is safe.
namespace {
struct AllocHook {
    htn_alloc_fn alloc = nullptr;
    htn_free_fn free = nullptr;
    void *ctx = nullptr;
};
std::mutex g_alloc_mu;
AllocHook g_hook;
std::unordered_map<void *, AllocHook> g_hooked;  // blocks made by a caller allocator
}  // namespace

static void dfree(void *p) {
    if (!p) return;
    AllocHook h;
    {
        std::lock_guard<std::mutex> lock(g_alloc_mu);
        auto it = g_hooked.find(p);
        if (it != g_hooked.end()) {
            h = it->second;
            g_hooked.erase(it);
        }
    }
    if (h.free)
        h.free(p, h.ctx);
    else
        (void)hipFree(p);
}

static void *dalloc_bytes(size_t bytes) {
    if (bytes == 0) bytes = 1;
    AllocHook h;
    {
        std::lock_guard<std::mutex> lock(g_alloc_mu);
        h = g_hook;
    }
    if (h.alloc) {
        void *p = h.alloc(bytes, h.ctx);
        if (!p) throw Error{HTN_E_OOM, "the caller's allocator returned NULL for " + std::to_string(bytes) + " bytes"};
        std::lock_guard<std::mutex> lock(g_alloc_mu);
        g_hooked[p] = h;
        return p;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{HTN_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e)};
    }
    return p;
}

template <typename T>
static T *dalloc(size_t count) {
    return (T *)dalloc_bytes(count * sizeof(T));
}

static float bf16_bits_to_f32(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

static uint16_t f32_to_bf16_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Host conversion of n elements from dtype `from` to dtype `to`.
// BF16 results are rounded from FP32 (an FP64 source is first rounded to
// FP32), both steps to nearest-even.
static void host_convert(const void *src, htn_dtype from, void *dst, htn_dtype to, int64_t n) {
    if (from == to) {
        std::memcpy(dst, src, (size_t)n * dtype_size(from));
        return;
    }
    for (int64_t i = 0; i < n; ++i) {
        double v;
        if (from == HTN_F64)
            v = ((const double *)src)[i];
        else if (from == HTN_F32)
            v = ((const float *)src)[i];
        else
            v = bf16_bits_to_f32(((const uint16_t *)src)[i]);
        if (to == HTN_F64)
            ((double *)dst)[i] = v;
        else if (to == HTN_F32)
            ((float *)dst)[i] = (float)v;
        else
            ((uint16_t *)dst)[i] = f32_to_bf16_bits((float)v);
    }
}

static void release_inputs(Net &n) {
    if (!n.dev) return;
    for (size_t i = 0; i < n.dev->in.size(); ++i)
        if (n.dev->own[i]) dfree(n.dev->in[i]);
    n.dev->in.clear();
    n.dev->own.clear();
}

static void release_device(Net &n) {
    if (!n.dev) return;
    free_slices(*n.dev);
    release_inputs(n);
    DeviceState &D = *n.dev;
    dfree(D.d_inptrs);
    dfree(D.d_prog);
    dfree(D.d_tab);
    dfree(D.d_ws);
    dfree(D.d_prep);
    dfree(D.d_fdesc);
    dfree(D.d_fprep);
    dfree(D.d_fold_tab);
    delete n.dev;
    n.dev = nullptr;
}

static void set_data(Net &n, const void *const *data, int on_device) {
    if (!data) throw Error{HTN_E_ARG, "data is NULL"};
    for (int i = 0; i < n.n_t; ++i)
        if (!data[i]) throw Error{HTN_E_ARG, "data[" + std::to_string(i) + "] is NULL"};
    n.data_on_device = on_device != 0;
    n.user_ptrs.assign(n.n_t, nullptr);
    n.host.assign(n.n_t, {});
    const htn_dtype tin = input_dtype(n.compute);
    for (int i = 0; i < n.n_t; ++i) {
        if (n.data_on_device) {
            n.user_ptrs[i] = data[i];
        } else {
            n.host[i].resize((size_t)n.sizes[i] * dtype_size(tin));
            host_convert(data[i], n.storage, n.host[i].data(), tin, n.sizes[i]);
        }
    }
    n.data_dirty = true;
}

static void upload_inputs(Net &n) {
    DeviceState &D = *n.dev;
    const htn_dtype tin = input_dtype(n.compute);
    free_slices(D);  // slice networks read the inputs' device copies
    release_inputs(n);
    D.in.assign(n.n_t, nullptr);
    D.own.assign(n.n_t, 0);
    for (int i = 0; i < n.n_t; ++i) {
        const size_t bytes = (size_t)n.sizes[i] * dtype_size(tin);
        if (n.data_on_device && n.storage == tin) {
            D.in[i] = const_cast<void *>(n.user_ptrs[i]);
            continue;
        }
        D.in[i] = dalloc<unsigned char>(bytes);
        D.own[i] = 1;
        if (n.data_on_device) {
            HIP_TRY(kern::launch_convert(n.user_ptrs[i], n.storage, D.in[i], tin, n.sizes[i], 0));
        } else {
            HIP_TRY(hipMemcpy(D.in[i], n.host[i].data(), bytes, hipMemcpyHostToDevice));
            std::vector<unsigned char>().swap(n.host[i]);
        }
    }
    HIP_TRY(hipDeviceSynchronize());
    dfree(D.d_inptrs);
    D.d_inptrs = dalloc<void *>(n.n_t);
    HIP_TRY(hipMemcpy(D.d_inptrs, D.in.data(), sizeof(void *) * n.n_t, hipMemcpyHostToDevice));
    n.data_dirty = false;
    D.plan_uploaded = -1;  // prep descriptors hold input pointers
    ++D.uploads;
}

static void upload_plan(Net &n) {
    DeviceState &D = *n.dev;
    Plan &P = n.plan;
    // the fused program carries the device addresses of its inputs
    std::vector<int32_t> prog = P.program;
    for (auto &ps : P.ptr_slots) {
        const uint64_t a = (uint64_t)(uintptr_t)D.in[ps.second];
        prog[ps.first] = (int32_t)(uint32_t)(a & 0xffffffffu);
        prog[ps.first + 1] = (int32_t)(uint32_t)(a >> 32);
    }
    dfree(D.d_prog);
    D.d_prog = dalloc<int32_t>(prog.size());
    HIP_TRY(hipMemcpy(D.d_prog, prog.data(), prog.size() * 4, hipMemcpyHostToDevice));
    dfree(D.d_tab);
    D.d_tab = dalloc<int2>(P.tables.size() / 2);
    HIP_TRY(hipMemcpy(D.d_tab, P.tables.data(), P.tables.size() * 4, hipMemcpyHostToDevice));
    const int64_t ws_need = std::max<int64_t>(P.ws_bytes, P.fused_scratch_bytes);
    if (ws_need > D.ws_cap) {
        dfree(D.d_ws);
        D.d_ws = nullptr;
        D.d_ws = dalloc<unsigned char>((size_t)ws_need);
        D.ws_cap = ws_need;
    }
    std::vector<kern::PrepDesc> prep;
    int pmax = 0;
    D.prep_index.clear();
    std::vector<int> order;  // needs_copy loads: per-step ones first
    for (int pass = 0; pass < 2; ++pass)
        for (size_t k = 0; k < P.loads.size(); ++k) {
            const LoadPlan &lp = P.loads[k];
            if (lp.needs_copy() && (P.ws_off[lp.value] >= 0) == (pass == 0)) order.push_back((int)k);
        }
    {
        std::vector<int> slot(P.loads.size(), -1);
        for (size_t i = 0; i < order.size(); ++i) slot[order[i]] = (int)i;
        for (size_t k = 0; k < P.loads.size(); ++k)
            if (P.loads[k].needs_copy()) D.prep_index.push_back(slot[k]);
    }
    D.n_prep_steps = 0;
    for (int k : order) {
        const LoadPlan &lp = P.loads[k];
        kern::PrepDesc q;
        std::memset(&q, 0, sizeof(q));
        q.src = D.in[lp.base];
        q.dst_off = P.ws_off[lp.value];  // -1: not run by the per-step executor
        if (q.dst_off >= 0) ++D.n_prep_steps;
        q.size = (int32_t)lp.size;
        q.ns = (int32_t)lp.scales.size();
        for (int k = 0; k < q.ns; ++k) {
            q.sp[k] = D.in[lp.scales[k].tensor];
            q.thi[k] = (int32_t)lp.scales[k].t_hi;
            q.tlo[k] = (int32_t)lp.scales[k].t_lo;
            q.nlo[k] = (int32_t)lp.scales[k].n_lo;
        }
        q.sthi = (int32_t)lp.src_thi;
        q.stlo = (int32_t)lp.src_tlo;
        q.snlo = (int32_t)lp.src_nlo;
        pmax = std::max<int>(pmax, q.size);
        prep.push_back(q);
    }
    dfree(D.d_prep);
    D.d_prep = nullptr;
    D.n_prep = (int)prep.size();
    D.prep_max = pmax;
    if (!prep.empty()) {
        D.d_prep = dalloc<kern::PrepDesc>(prep.size());
        HIP_TRY(hipMemcpy(D.d_prep, prep.data(), prep.size() * sizeof(kern::PrepDesc), hipMemcpyHostToDevice));
    }
    D.folds.clear();
    dfree(D.d_fold_tab);
    D.d_fold_tab = nullptr;
    std::vector<int32_t> ftab;
    for (const auto &ch : P.chains) {
        const FoldLayout F = fold_layout(n, P, ch);
        if (!F.ok) throw Error{HTN_E_STATE, "fold chain without a layout"};
        kern::FoldDesc fd;
        std::memset(&fd, 0, sizeof(fd));
        // index tables: offsets of every in-tile index at the source and
        // the destination, and per stage each output's first input term
        // and new digit (digits over the in-tile axes, last fastest)
        auto offsets = [&](const std::vector<int> &ext, const std::vector<int64_t> &str) {
            int64_t size = 1;
            for (int e : ext) size *= e;
            for (int64_t a = 0; a < size; ++a) {
                int64_t r = a, off = 0;
                for (int j = (int)ext.size() - 1; j >= 0; --j) {
                    off += (r % ext[j]) * str[j];
                    r /= ext[j];
                }
                if (off > INT32_MAX) throw Error{HTN_E_UNSUPPORTED, "fold chain offset beyond 32 bits"};
                ftab.push_back((int32_t)off);
            }
            return (int32_t)size;
        };
        fd.t_src = (int32_t)ftab.size();
        offsets(F.ext0, F.s_src);
        fd.t_dst = (int32_t)ftab.size();
        fd.d_final = offsets(F.ext1, F.s_dst);
        std::vector<int> ext = F.ext0;
        for (size_t st = 0; st < F.fold_ax.size(); ++st) {
            const int ax = F.fold_ax[st], din = ext[ax], dout = F.fold_ext[st];
            int64_t inner = 1, size = 1;
            for (size_t j = ax + 1; j < ext.size(); ++j) inner *= ext[j];
            for (int e : ext) size *= e;
            const int64_t Dn = size / din * dout;
            fd.d_in_ax[st] = din;
            fd.d_out[st] = dout;
            fd.inner[st] = (int32_t)inner;
            fd.t_base[st] = (int32_t)ftab.size();
            for (int64_t a = 0; a < Dn; ++a) {
                const int64_t hi = a / (dout * inner), rem = a % (dout * inner);
                ftab.push_back((int32_t)(hi * din * inner + rem % inner));
            }
            fd.t_mid[st] = (int32_t)ftab.size();
            for (int64_t a = 0; a < Dn; ++a) ftab.push_back((int32_t)((a % (dout * inner)) / inner));
            ext[ax] = dout;
        }
        fd.lg_tf = 0;
        while ((1 << fd.lg_tf) < F.tf) ++fd.lg_tf;
        fd.n_ax = (int32_t)F.ext0.size();
        fd.n_outer = (int32_t)F.o_ext.size();
        fd.n_stage = (int32_t)F.fold_ax.size();
        fd.tf = F.tf;
        fd.d_max = F.d_max;
        fd.lds_bytes = (int32_t)F.lds_bytes;
        for (int j = 0; j < fd.n_ax; ++j) {
            fd.ext0[j] = F.ext0[j];
            fd.ext1[j] = F.ext1[j];
            fd.s_src[j] = F.s_src[j];
            fd.s_dst[j] = F.s_dst[j];
        }
        for (int j = 0; j < fd.n_stage; ++j) {
            fd.fold_ax[j] = F.fold_ax[j];
            fd.fold_ext[j] = F.fold_ext[j];
            fd.m_in[j] = (int32_t)F.m_in[j];
            fd.m_out[j] = (int32_t)F.m_out[j];
            fd.m[j] = D.in[F.m_tensor[j]];
        }
        for (int j = 0; j < fd.n_outer; ++j) {
            fd.o_ext[j] = F.o_ext[j];
            fd.o_src[j] = F.o_src[j];
            fd.o_dst[j] = F.o_dst[j];
        }
        fd.n_outer_total = F.n_outer;
        D.folds.push_back(fd);
    }
    if (!ftab.empty()) {
        D.d_fold_tab = dalloc<int32_t>(ftab.size());
        HIP_TRY(hipMemcpy(D.d_fold_tab, ftab.data(), ftab.size() * 4, hipMemcpyHostToDevice));
        for (auto &fd : D.folds) fd.tab = D.d_fold_tab;
    }
    D.fprep.clear();
    D.fprep_max = 0;
    D.fprep_form = 0;
    for (const LoadPlan &lp : P.loads) {
        if (lp.desc_word < 0 || lp.desc_word + 7 > (int64_t)P.program.size()) continue;  // no fused image
        const int32_t rk = P.program[lp.desc_word + 5], ns = P.program[lp.desc_word + 6];
        const int32_t words = 7 + 2 * ns + rk * (4 + ns);
        if (words > kern::kFPrepDescMax) throw Error{HTN_E_UNSUPPORTED, "load descriptor too long"};
        for (int64_t e0 = 0; e0 < lp.size; e0 += kern::kFPrepChunk)
            D.fprep.push_back(kern::FPrepEntry{D.d_prog + lp.desc_word, D.d_ws, (int32_t)e0, words});
        D.fprep_max = std::max<int>(D.fprep_max, (int)lp.size);
        D.fprep_form = std::max(D.fprep_form, kern::fprep_form(rk, ns));
    }
    dfree(D.d_fprep);
    D.d_fprep = nullptr;
    if (!D.fprep.empty()) {
        D.d_fprep = dalloc<kern::FPrepEntry>(D.fprep.size());
        HIP_TRY(hipMemcpy(D.d_fprep, D.fprep.data(), D.fprep.size() * sizeof(kern::FPrepEntry),
                          hipMemcpyHostToDevice));
    }
    int64_t in_elems = 0;
    for (const LoadPlan &lp : P.loads) in_elems += lp.size;
    D.fprep_in_kernel = !D.fprep.empty() && in_elems <= kInKernelPrepMax;
    kern::FusedDesc fd = fused_desc(D, true, P.fused_lds_only);
    dfree(D.d_fdesc);
    D.d_fdesc = dalloc<kern::FusedDesc>(1);
    HIP_TRY(hipMemcpy(D.d_fdesc, &fd, sizeof(fd), hipMemcpyHostToDevice));
    D.plan_uploaded = n.plan_version;
    ++D.uploads;
}

static void ensure_device(Net &n) {
    if (!n.dev) {
        n.dev = new DeviceState;
        HIP_TRY(hipGetDevice(&n.dev->device));
    } else {
        int cur = -1;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != n.dev->device) throw Error{HTN_E_STATE, "net was first used on another device"};
    }
    if (n.data_dirty) upload_inputs(n);
    // a sliced net runs its slice networks, never its own plan
    if (n.n_slices == 1 && n.dev->plan_uploaded != n.plan_version) upload_plan(n);
}

static int final_mode(const Net &n) {
    if (n.final_sum == HTN_SUM_COMPENSATED) return kern::FM_COMP;
    if (n.final_sum == HTN_SUM_FP64) return kern::FM_F64;
    return kern::FM_INTER;
}

static bool use_fused_in_batch(const Net &n) {
    if (n.exec == HTN_EXEC_STEPS) return false;
    if (n.exec == HTN_EXEC_FUSED) return n.plan.fused_possible;
    return n.plan.fused_batch_ok;
}

static bool use_fused(const Net &n) {
    if (n.exec == HTN_EXEC_STEPS) return false;
    if (n.exec == HTN_EXEC_FUSED) {
        if (!n.plan.fused_possible)
            throw Error{HTN_E_UNSUPPORTED, "fused kernel: program and table slots exceed the LDS budget"};
        return true;  // values that do not fit LDS spill to global scratch
    }
    return n.plan.fused_ok;
}

static void run_fused_single(Net &n, void *out, hipStream_t st) {
    if (!n.dev->fprep_in_kernel)
        HIP_TRY(kern::launch_fprep(n.dev->d_fprep, (int)n.dev->fprep.size(), n.dev->fprep_form, n.dev->fprep_max,
                                   (int)n.compute, nullptr, st));
    HIP_TRY(kern::launch_fused(n.dev->d_fdesc, nullptr, nullptr, nullptr, out, nullptr, 0, 1,
                               (int)n.plan.fused_lds_bytes, (int)n.compute, final_mode(n), n.fused_threads, st));
}

static kern::StepArgs pack_args(const StepPlan::Pack &pk) {
    kern::StepArgs a;
    a.n_ohi = (int32_t)pk.n_ohi;
    a.n_olo = (int32_t)pk.n_olo;
    a.n_shi = 1;
    a.n_slo = 1;
    a.t_ohi = (int32_t)pk.t_ohi;
    a.t_olo = (int32_t)pk.t_olo;
    a.t_shi = (int32_t)pk.t_one;
    a.t_slo = (int32_t)pk.t_one;
    a.R = 1;
    a.log2R = 0;
    a.n_out = pk.n;
    return a;
}

// Matrix-core step: pack both operands K-contiguous, then one GEMM launch.
static void run_mfma_step(Net &n, const StepPlan &s, const void *A, int ta, const void *B, int tb, void *C, int tc,
                          unsigned char *ws, hipStream_t st) {
    DeviceState &D = *n.dev;
    const int tp = n.compute == HTN_BF16 ? 2 : (int)inter_dtype(n.compute);
    // an operand its producer already wrote in packed order is used in place
    const void *pa = A, *pb = B;
    if (!(s.pack_a.identity && ta == tp)) {
        void *w = ws + s.ws_pa;
        if (s.ws_pa < 0) throw Error{HTN_E_STATE, "packed operand without workspace"};
        HIP_TRY(kern::launch_step(A, ta, nullptr, ta, w, tp, false, false, D.d_tab, pack_args(s.pack_a), st));
        pa = w;
    }
    if (!(s.pack_b.identity && tb == tp)) {
        void *w = ws + s.ws_pb;
        if (s.ws_pb < 0) throw Error{HTN_E_STATE, "packed operand without workspace"};
        HIP_TRY(kern::launch_step(B, tb, nullptr, tb, w, tp, false, false, D.d_tab, pack_args(s.pack_b), st));
        pb = w;
    }
    void *kpart = s.ksplit > 1 ? ws + s.ws_kpart : nullptr;
    HIP_TRY(kern::launch_gemm(pa, pb, C, tp, tc, (int)s.gm, (int)s.gn, (int)s.gk, (int)s.gb, 64, s.ksplit, kpart, st));
}

// ticks (optional): the device clock after each of the first max_ticks
// kernel steps.  ws: the workspace (the net's own when NULL; at least
// plan.ws_bytes bytes).
static void run_steps(Net &n, void *out, hipStream_t st, int64_t *ticks = nullptr, int max_ticks = 0,
                      void *ws_base = nullptr) {
    DeviceState &D = *n.dev;
    const Plan &P = n.plan;
    unsigned char *ws = (unsigned char *)(ws_base ? ws_base : D.d_ws);
    const int tin = (int)input_dtype(n.compute), tint = (int)inter_dtype(n.compute);
    if (D.n_prep_steps)
        HIP_TRY(kern::launch_prep(D.d_prep, D.n_prep_steps, D.prep_max, tin, tint, D.d_tab, ws, st));
    int q = -1;
    for (int k : P.kernel_steps) {
        if (ticks && q >= 0 && q < max_ticks) HIP_TRY(kern::launch_stamp(ticks + q, st));
        ++q;
        const StepPlan &s = P.steps[k];
        if (s.chain >= 0 && s.chain_pos > 0) continue;  // ran with its chain's first step
        auto operand = [&](int id, const void *&ptr, int &t) {
            if (id < 0) {
                ptr = nullptr;
                t = tint;
            } else if (P.ws_off[id] >= 0) {
                ptr = ws + P.ws_off[id];
                const int pr = P.values[id].producer;
                t = (!P.values[id].input && pr >= 0 && P.steps[pr].out_bf16) ? (int)HTN_BF16 : tint;
            } else {
                ptr = D.in[P.values[id].base];
                t = tin;
            }
        };
        const void *A, *B;
        int ta, tb;
        operand(s.a, A, ta);
        operand(s.b, B, tb);
        void *C;
        int tc;
        bool comp = false;
        if (s.final_step) {
            C = out;
            tc = n.final_sum == HTN_SUM_PLAIN ? tint : 0;
            comp = n.final_sum == HTN_SUM_COMPENSATED;
        } else {
            C = ws + P.ws_off[s.c];
            tc = s.out_bf16 ? (int)HTN_BF16 : tint;
        }
        if (s.chain >= 0) {
            // whole fold chains (source X in, each chain's last result out):
            // the chains of the group this step leads, side by side
            if (P.chain_lead[s.chain] != s.chain) continue;  // launched with its group
            std::vector<kern::FoldJob> jobs;
            std::vector<int> types;  // result dtype per job
            for (int c = 0; c < (int)P.chains.size(); ++c) {
                if (P.chain_lead[c] != s.chain) continue;
                const StepPlan &h = P.steps[P.chains[c][0]];
                const StepPlan &last = P.steps[P.chains[c].back()];
                const int x = P.values[h.a].size >= P.values[h.b].size ? h.a : h.b;
                const void *X;
                int tx;
                operand(x, X, tx);
                jobs.push_back({X, tx, ws + P.ws_off[last.c], &D.folds[c]});
                types.push_back(last.out_bf16 ? (int)HTN_BF16 : tint);
            }
            // one launch per run of equal result types
            for (size_t j0 = 0; j0 < jobs.size();) {
                size_t j1 = j0 + 1;
                while (j1 < jobs.size() && types[j1] == types[j0]) ++j1;
                HIP_TRY(kern::launch_folds(jobs.data() + j0, (int)(j1 - j0), tin, tint, types[j0], st));
                j0 = j1;
            }
            continue;
        }
        if (s.mfma) {
            run_mfma_step(n, s, A, ta, B, tb, C, tc, ws, st);
            continue;
        }
        kern::StepArgs a;
        a.n_ohi = (int32_t)s.n_ohi;
        a.n_olo = (int32_t)s.n_olo;
        a.n_shi = (int32_t)s.n_shi;
        a.n_slo = (int32_t)s.n_slo;
        a.t_ohi = (int32_t)s.t_ohi;
        a.t_olo = (int32_t)s.t_olo;
        a.t_shi = (int32_t)s.t_shi;
        a.t_slo = (int32_t)s.t_slo;
        a.R = s.r_global;
        a.log2R = 0;
        while ((1 << a.log2R) < a.R) ++a.log2R;
        a.n_out = s.n_out;
        if (s.split_global > 1) {
            a.split = s.split_global;
            a.chunk = (s.n_sum + s.split_global - 1) / s.split_global;
            a.part = (double *)(ws + s.ws_part);
        }
        HIP_TRY(kern::launch_step(A, ta, B, tb, C, tc, tc == 0, comp, D.d_tab, a, st));
    }
    if (ticks && q >= 0 && q < max_ticks) HIP_TRY(kern::launch_stamp(ticks + q, st));
}

static void contract_one(Net &n, void *out, hipStream_t st) {
    if (n.n_slices > 1)
        run_sliced(n, out, st);
    else if (use_fused(n))
        run_fused_single(n, out, st);
    else
        run_steps(n, out, st);
}

static void replan(Net &n) {
    auto old_path = n.path;
    try {
        plan_net(n);
    } catch (...) {
        n.path = old_path;
        throw;
    }
}

// ------------------------------------------------------------------ ABI

extern "C" {

htn_status htn_create(htn_net_t *out, int32_t n_tensors, const int32_t *ranks, const int32_t *labels,
                      int32_t n_labels, const int64_t *label_dims, const void *const *data, int32_t data_on_device,
                      int32_t n_out, const int32_t *out_labels, htn_dtype storage, htn_dtype compute,
                      htn_final_sum final_sum) {
    API_GUARD_BEGIN
    if (!out) return fail(HTN_E_ARG, "out is NULL");
    *out = nullptr;
    if (n_tensors < 1) return fail(HTN_E_ARG, "n_tensors < 1");
    if (!ranks || !labels || !label_dims) return fail(HTN_E_ARG, "ranks/labels/label_dims is NULL");
    if (n_labels < 1) return fail(HTN_E_ARG, "n_labels < 1");
    if (n_out < 0 || (n_out > 0 && !out_labels)) return fail(HTN_E_ARG, "bad output labels");
    if (storage < HTN_F64 || storage > HTN_BF16 || compute < HTN_F64 || compute > HTN_BF16)
        return fail(HTN_E_ARG, "bad dtype");
    if (final_sum < HTN_SUM_PLAIN || final_sum > HTN_SUM_COMPENSATED) return fail(HTN_E_ARG, "bad final_sum");
    htn_net *n = new htn_net;
    try {
        n->n_t = n_tensors;
        n->dims.assign(label_dims, label_dims + n_labels);
        n->labels.resize(n_tensors);
        int off = 0;
        for (int i = 0; i < n_tensors; ++i) {
            if (ranks[i] < 0) throw Error{HTN_E_SHAPE, "negative rank"};
            n->labels[i].assign(labels + off, labels + off + ranks[i]);
            off += ranks[i];
        }
        n->out_labels.assign(out_labels, out_labels + n_out);
        n->storage = storage;
        n->compute = compute;
        n->final_sum = final_sum;
        validate_structure(*n);
        n->sizes.resize(n_tensors);
        for (int i = 0; i < n_tensors; ++i) {
            int64_t s = 1;
            for (int l : n->labels[i]) s *= n->dims[l];
            n->sizes[i] = s;
        }
        set_data(*n, data, data_on_device);
        n->path = greedy_path(*n);
        n->path_kind = HTN_PATH_GREEDY;
        plan_net(*n);
    } catch (...) {
        delete n;
        throw;
    }
    *out = n;
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_set_path(htn_net_t net, int32_t n_steps, const int32_t *ssa_pairs) {
    API_GUARD_BEGIN
    if (!net) return fail(HTN_E_ARG, "net is NULL");
    auto old = net->path;
    int old_kind = net->path_kind;
    try {
        if (n_steps >= 0) {
            if (n_steps > 0 && !ssa_pairs) return fail(HTN_E_ARG, "ssa_pairs is NULL");
            std::vector<std::pair<int, int>> p(n_steps);
            for (int t = 0; t < n_steps; ++t) p[t] = {ssa_pairs[2 * t], ssa_pairs[2 * t + 1]};
            check_path(*net, p);
            net->path = p;
            net->path_kind = 0;
        } else if (n_steps == HTN_PATH_GREEDY) {
            net->path = greedy_path(*net);
            net->path_kind = n_steps;
        } else if (n_steps == HTN_PATH_SAMPLED) {
            net->path = sampled_path(*net, net->path_samples, net->path_seed);
            net->path_kind = n_steps;
        } else if (n_steps == HTN_PATH_LEARNED) {
            net->path = learned_path(*net);
            net->path_kind = n_steps;
        } else {
            return fail(HTN_E_ARG, "unknown path selector");
        }
        plan_net(*net);
    } catch (...) {
        net->path = old;
        net->path_kind = old_kind;
        throw;
    }
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_get_path(htn_net_t net, int32_t *n_steps, int32_t *ssa_pairs, int32_t capacity, double *mults) {
    API_GUARD_BEGIN
    if (!net || !n_steps) return fail(HTN_E_ARG, "NULL argument");
    *n_steps = (int32_t)net->path.size();
    if (mults) *mults = net->plan.mults;
    if (ssa_pairs)
        for (int t = 0; t < (int)net->path.size() && t < capacity; ++t) {
            ssa_pairs[2 * t] = net->path[t].first;
            ssa_pairs[2 * t + 1] = net->path[t].second;
        }
    if (mults) *mults = net->plan.mults;
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_set_option(htn_net_t net, htn_option opt, int64_t value) {
    API_GUARD_BEGIN
    if (!net) return fail(HTN_E_ARG, "net is NULL");
    switch (opt) {
        case HTN_OPT_EXEC:
            if (value < HTN_EXEC_AUTO || value > HTN_EXEC_FUSED) return fail(HTN_E_ARG, "bad exec mode");
            net->exec = (htn_exec_mode)value;
            return HTN_OK;
        case HTN_OPT_MAX_INTERMEDIATE: {
            if (value < 1 || value > 2147483647)
                return fail(HTN_E_ARG, "cap outside [1, 2^31-1] (offsets are 32-bit)");
            int64_t old = net->max_intermediate;
            net->max_intermediate = value;
            try {
                replan(*net);
            } catch (...) {
                net->max_intermediate = old;
                throw;
            }
            return HTN_OK;
        }
        case HTN_OPT_FUSED_LDS_BYTES: {
            if (value < 1024 || value > 163840) return fail(HTN_E_ARG, "LDS budget outside [1024, 163840]");
            net->fused_lds_budget = value;
            replan(*net);
            return HTN_OK;
        }
        case HTN_OPT_MFMA:
            net->allow_mfma = value ? 1 : 0;
            replan(*net);
            return HTN_OK;
        case HTN_OPT_PATH_SAMPLES:
            if (value < 0 || value > 100000) return fail(HTN_E_ARG, "path samples outside [0, 100000]");
            net->path_samples = (int)value;
            return HTN_OK;
        case HTN_OPT_PATH_SEED:
            net->path_seed = (uint64_t)value;
            return HTN_OK;
        case HTN_OPT_SLICE: {
            if (value != 0 && value != 1) return fail(HTN_E_ARG, "slicing is 0 (off) or 1 (on)");
            const int old = net->slice_mode;
            net->slice_mode = (int)value;
            try {
                replan(*net);
            } catch (...) {
                net->slice_mode = old;
                replan(*net);
                throw;
            }
            return HTN_OK;
        }
        case HTN_OPT_QUEUE:
            if (value < 0 || value > 2) return fail(HTN_E_ARG, "queue mode is 0 (auto), 1 (always) or 2 (never)");
            net->queue_mode = (int)value;
            return HTN_OK;
        case HTN_OPT_FUSED_THREADS: {
            if (value != 64 && value != 256 && value != 512)
                return fail(HTN_E_ARG, "fused threads must be 64, 256 or 512");
            const int old = net->fused_threads;
            net->fused_threads = (int)value;
            try {
                replan(*net);
            } catch (...) {
                net->fused_threads = old;
                throw;
            }
            return HTN_OK;
        }
    }
    return fail(HTN_E_ARG, "unknown option");
    API_GUARD_END
}

htn_status htn_get_info(htn_net_t net, htn_info *info) {
    API_GUARD_BEGIN
    if (!net || !info) return fail(HTN_E_ARG, "NULL argument");
    const Plan &P = net->plan;
    std::memset(info, 0, sizeof(*info));
    int64_t oe = 1;
    for (int l : net->out_labels) oe *= net->dims[l];
    info->out_elements = oe;
    info->out_dtype = (int32_t)out_dtype(*net);
    info->n_steps = (int32_t)net->path.size();
    info->n_kernel_steps = (int32_t)P.kernel_steps.size();
    info->n_absorbed = P.n_absorbed;
    info->fused_ok = P.fused_ok ? 1 : 0;
    info->fused_lds_bytes = (int32_t)P.fused_lds_bytes;
    info->mults = P.mults * (double)net->n_slices;
    info->peak_elements = P.peak;
    info->n_slices = net->n_slices;
    info->workspace_bytes = P.ws_bytes;
    int64_t ib = 0;
    for (int i = 0; i < net->n_t; ++i) ib += net->sizes[i] * dtype_size(input_dtype(net->compute));
    info->input_bytes = ib;
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_get_slicing(htn_net_t net, int32_t *n_labels, int32_t *labels, int32_t capacity, int64_t *n_slices) {
    API_GUARD_BEGIN
    if (!net || !n_labels || capacity < 0) return fail(HTN_E_ARG, "bad arguments");
    *n_labels = (int32_t)net->sliced.size();
    if (labels)
        for (int k = 0; k < (int)net->sliced.size() && k < capacity; ++k) labels[k] = net->sliced[k];
    if (n_slices) *n_slices = net->n_slices;
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_contract(htn_net_t net, void *out_device, void *hip_stream) {
    API_GUARD_BEGIN
    if (!net || !out_device) return fail(HTN_E_ARG, "NULL argument");
    ensure_device(*net);
    contract_one(*net, out_device, (hipStream_t)hip_stream);
    return HTN_OK;
    API_GUARD_END
}

}  // extern "C"

// Workspace of htn_contract_noalloc: one array per device (each device holds
// its own copy from the library's load until the process ends), shared by
// every call on that device.  Host code never uses the array's name as an
// address: the device address comes from hipGetSymbolAddress, resolved once
// per device with that device current.
static __device__ __align__(256) unsigned char scratch[HTN_NOALLOC_SCRATCH_BYTES];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

static void *scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) throw Error{HTN_E_DEVICE, "device ordinal out of range"};
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error{HTN_E_DEVICE, "hipGetSymbolAddress returned NULL"};
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

extern "C" {

htn_status htn_set_allocator(htn_alloc_fn alloc, htn_free_fn free_fn, void *ctx) {
    API_GUARD_BEGIN
    if ((alloc == nullptr) != (free_fn == nullptr)) return fail(HTN_E_ARG, "give both alloc and free, or neither");
    std::lock_guard<std::mutex> lock(g_alloc_mu);
    g_hook.alloc = alloc;
    g_hook.free = free_fn;
    g_hook.ctx = alloc ? ctx : nullptr;
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_contract_noalloc(htn_net_t net, void *out_device, void *hip_stream) {
    API_GUARD_BEGIN
    if (!net || !out_device) return fail(HTN_E_ARG, "NULL argument");
    if (net->n_slices > 1) return fail(HTN_E_UNSUPPORTED, "a sliced net allocates its slice networks");
    if (net->plan.ws_bytes > (int64_t)HTN_NOALLOC_SCRATCH_BYTES)
        return fail(HTN_E_UNSUPPORTED, "the per-step workspace needs " + std::to_string(net->plan.ws_bytes) +
                                           " bytes, above the " + std::to_string((int64_t)HTN_NOALLOC_SCRATCH_BYTES) +
                                           "-byte allocation-free workspace");
    if (!net->dev || net->data_dirty || net->dev->plan_uploaded != net->plan_version)
        return fail(HTN_E_STATE, "device state of the net is not set up: call htn_contract once after the last "
                                 "htn_create, htn_set_path, htn_set_option or htn_update_data");
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != net->dev->device) return fail(HTN_E_STATE, "net was set up on another device");
    run_steps(*net, out_device, (hipStream_t)hip_stream, nullptr, 0, scratch_address(cur));
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_update_data(htn_net_t net, const void *const *data, int32_t data_on_device) {
    API_GUARD_BEGIN
    if (!net) return fail(HTN_E_ARG, "net is NULL");
    set_data(*net, data, data_on_device);
    return HTN_OK;
    API_GUARD_END
}

void htn_destroy(htn_net_t net) {
    if (!net) return;
    try {
        release_device(*net);
    } catch (...) {
    }
    delete net;
}

htn_status htn_plan_json(htn_net_t net, char *buf, int64_t capacity, int64_t *needed) {
    API_GUARD_BEGIN
    if (!net) return fail(HTN_E_ARG, "net is NULL");
    std::string s = plan_json(*net);
    if (needed) *needed = (int64_t)s.size() + 1;
    if (buf && capacity > 0) {
        size_t n = std::min<size_t>((size_t)capacity - 1, s.size());
        std::memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_plan_tables(htn_net_t net, int32_t *buf, int64_t capacity, int64_t *needed) {
    API_GUARD_BEGIN
    if (!net) return fail(HTN_E_ARG, "net is NULL");
    const auto &t = net->plan.tables;
    if (needed) *needed = (int64_t)t.size();
    if (buf && capacity > 0) std::memcpy(buf, t.data(), sizeof(int32_t) * (size_t)std::min<int64_t>(capacity, t.size()));
    return HTN_OK;
    API_GUARD_END
}

// ---------------------------------------------------------------- batch

static void batch_free(htn_batch *b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    for (auto &g : b->groups) {
        dfree(g.d_order);
        dfree(g.d_fprep);
    }
    dfree(b->q.d_items);
    dfree(b->q.d_tasks);
    dfree(b->q.d_counters);
    dfree(b->q.d_init);
    dfree(b->q.d_ctrl);
    dfree(b->q.d_qinfo);
    dfree(b->q.d_ws);
    if (b->q.ev_join) (void)hipEventDestroy(b->q.ev_join);
    if (b->q.ev_fork) (void)hipEventDestroy(b->q.ev_fork);
    if (b->q.stream) (void)hipStreamDestroy(b->q.stream);
    b->q = htn_batch::Queue{};
    dfree(b->d_desc);
    dfree(b->d_outs);
    dfree(b->d_stamps);
    dfree(b->d_phase);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (hipEvent_t e : b->ev_join) (void)hipEventDestroy(e);
    for (hipStream_t q : b->sides) (void)hipStreamDestroy(q);
    b->ev_fork = nullptr;
    b->ev_join.clear();
    b->sides.clear();
    for (hipEvent_t e : b->ev_pool) (void)hipEventDestroy(e);
    b->ev_pool.clear();
    b->ev_used = 0;
}

static hipEvent_t next_event(htn_batch *b) {
    if (b->ev_used == b->ev_pool.size()) {
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreate(&e));
        b->ev_pool.push_back(e);
    }
    return b->ev_pool[b->ev_used++];
}

// ------------------------------------------------------------ work queue

namespace {
// Items of the work queue under construction.  Buffers in the queue's
// workspace are recorded as byte offsets (off: A, B, C, s.part; -1 where
// the field holds a device address already) and patched once the
// workspace is allocated.
struct QBuild {
    std::vector<kern::QItem> items;
    std::vector<std::array<int64_t, 4>> off;
    std::vector<int> level, sub;  // dependency level and sub-queue (XCD) of each item
    int cur_sub = 0;               // sub-queue of the net being added
    int64_t ws = 0;
    int gk = 0;  // GEMM kind of the queue (0: no GEMM items yet)
    int64_t take(int64_t bytes) {
        const int64_t o = ws;
        ws += (std::max<int64_t>(bytes, 1) + 255) / 256 * 256;
        return o;
    }
    int add(kern::QItem it, std::array<int64_t, 4> o) {
        int lvl = 0;
        for (int d : {it.dep0, it.dep1})
            if (d >= 0) lvl = std::max(lvl, level[d] + 1);
        items.push_back(it);
        off.push_back(o);
        level.push_back(lvl);
        sub.push_back(cur_sub);
        return (int)items.size() - 1;
    }
};
}  // namespace

static kern::QItem q_item(int kind, int net, const Net &n) {
    kern::QItem it;
    std::memset(&it, 0, sizeof(it));
    it.kind = kind;
    it.dep0 = it.dep1 = -1;
    it.net = net;
    it.tab = n.dev->d_tab;
    it.units_per_task = 1;
    return it;
}

// Task sizes of the work queue: each task carries about kQTaskWork operand
// reads (or element writes), and one item is cut into at most
// kQMaxItemTasks tasks: a task's fixed cost (taking it, waiting, one
// device-scope acquire and release) is then small against its work.
static constexpr int64_t kQTaskWork = int64_t(1) << 14;
static constexpr int64_t kQMaxItemTasks = 1024;

static int64_t q_units_per_task(int64_t units, int64_t work_per_unit) {
    const int64_t work = units * std::max<int64_t>(1, work_per_unit);
    const int64_t tasks = std::min<int64_t>(kQMaxItemTasks, std::max<int64_t>(1, work / kQTaskWork));
    return std::max<int64_t>(1, (units + tasks - 1) / tasks);
}

// Blocks of a table-driven step per task (operand reads per block: 256
// threads, each summing its share of the summed range).
static int64_t q_step_blocks_per_task(const kern::StepArgs &a, int64_t n_sum, int64_t blocks) {
    const int64_t chunk = a.split > 1 ? a.chunk : n_sum;
    const int64_t per_thread = std::max<int64_t>(1, (chunk + a.R - 1) / a.R);
    return q_units_per_task(blocks, kBlock * per_thread);
}

// Appends the items of net `bi` of the batch; false (nothing appended) if
// it has no kernel step or a matrix-core step of another GEMM kind than the
// queue's.
static bool queue_net(QBuild &Q, Net &n, int bi) {
    const Plan &P = n.plan;
    DeviceState &D = *n.dev;
    if (P.kernel_steps.empty()) return false;
    const int tin = (int)input_dtype(n.compute), tint = (int)inter_dtype(n.compute);
    const int64_t es = dtype_size(inter_dtype(n.compute));
    const int tp = n.compute == HTN_BF16 ? 2 : tint;  // packed GEMM operand type
    const int64_t pes = dtype_size((htn_dtype)tp);
    auto result_type = [&](const StepPlan &s) {
        return s.final_step ? (n.final_sum == HTN_SUM_PLAIN ? tint : 0) : (s.out_bf16 ? 2 : tint);
    };
    int gk = Q.gk;
    for (int k : P.kernel_steps) {
        const StepPlan &s = P.steps[k];
        if (!s.mfma) continue;
        const int g = kern::queue_gemm_kind(tp, result_type(s));
        if (g < 0 || (gk != 0 && g != gk)) return false;
        gk = g;
    }
    Q.gk = gk;
    const size_t first = Q.items.size();
    std::vector<int> prod(P.values.size(), -1);      // item that completes each value
    std::vector<int64_t> voff(P.values.size(), -1);  // its workspace offset
    // input materialisations, in the order of the net's prep descriptors
    int j = 0;
    for (const LoadPlan &lp : P.loads) {
        if (!lp.needs_copy()) continue;
        kern::QItem it = q_item(kern::QI_LOAD, bi, n);
        it.ta = tin;
        it.tc = tint;
        it.prep = D.d_prep + D.prep_index[j++];
        it.n_units = (lp.size + 255) / 256;
        it.units_per_task = (int32_t)q_units_per_task(it.n_units, 256 * (1 + (int64_t)lp.scales.size()));
        voff[lp.value] = Q.take(lp.size * es);
        prod[lp.value] = Q.add(it, {-1, -1, voff[lp.value], -1});
    }
    if (j != D.n_prep) throw Error{HTN_E_STATE, "queue: prep descriptors out of step with the plan"};
    // operand id -> (device address or workspace offset, dtype, producer)
    struct Opd {
        const void *ptr = nullptr;
        int64_t off = -1;
        int t = 0, dep = -1;
    };
    auto operand = [&](int id) {
        Opd o;
        if (id < 0) return o;
        const Value &v = P.values[id];
        o.dep = prod[id];
        if (v.input && voff[id] < 0) {
            o.ptr = D.in[v.base];
            o.t = tin;
        } else {
            if (voff[id] < 0) throw Error{HTN_E_STATE, "queue: operand without a buffer"};
            o.off = voff[id];
            o.t = (!v.input && v.producer >= 0 && P.steps[v.producer].out_bf16) ? 2 : tint;
        }
        return o;
    };
    auto set_ab = [](kern::QItem &it, std::array<int64_t, 4> &o, const Opd &a, const Opd &b) {
        it.A = a.ptr;
        o[0] = a.off;
        it.B = b.ptr;
        o[1] = b.off;
        it.dep0 = a.dep;
        it.dep1 = b.dep;
    };
    int last = -1;
    for (int k : P.kernel_steps) {
        const StepPlan &s = P.steps[k];
        const Opd A = operand(s.a), B = operand(s.b);
        const int tc = result_type(s);
        const bool comp = s.final_step && n.final_sum == HTN_SUM_COMPENSATED;
        int64_t coff = -1;
        if (!s.final_step) coff = voff[s.c] = Q.take(P.values[s.c].size * es);
        const int out_flags = s.final_step ? (kern::QF_OUT | kern::QF_LAST) : 0;
        if (s.mfma) {
            auto pack = [&](const Opd &x, const StepPlan::Pack &pk) {
                if (pk.identity && x.t == tp) return x;
                kern::QItem it = q_item(kern::QI_STEP, bi, n);
                std::array<int64_t, 4> o{-1, -1, -1, -1};
                set_ab(it, o, x, Opd{});
                it.ta = x.t;
                it.tb = x.t;
                it.tc = tp;
                it.unary = 1;
                it.s = pack_args(pk);
                it.n_units = (pk.n + kBlock - 1) / kBlock;
                it.units_per_task = (int32_t)q_step_blocks_per_task(it.s, 1, it.n_units);
                Opd r;
                r.off = o[2] = Q.take(pk.n * pes);
                r.t = tp;
                r.dep = Q.add(it, o);
                return r;
            };
            const Opd pa = pack(A, s.pack_a), pb = pack(B, s.pack_b);
            int ks = s.ksplit, kper = 0;
            kern::gemm_ksplit((int)s.gk, ks, kper);
            const int rows = kern::queue_tile_rows();
            kern::QItem it = q_item(kern::QI_GEMM, bi, n);
            std::array<int64_t, 4> o{-1, -1, -1, -1};
            set_ab(it, o, pa, pb);
            it.ta = tp;
            it.tb = tp;
            it.tc = tc;
            it.M = (int)s.gm;
            it.N = (int)s.gn;
            it.K = (int)s.gk;
            it.batch = (int)s.gb;
            it.kchunk = 64;
            it.ksplit = ks;
            it.kper = kper;
            it.tiles_m = (int)((s.gm + rows - 1) / rows);
            it.tiles_n = (int)((s.gn + 127) / 128);
            it.n_units = (int64_t)it.tiles_m * it.tiles_n * it.batch * ks;
            const int64_t total = s.gb * s.gm * s.gn;
            if (ks > 1) {
                o[2] = Q.take(ks * total * (tc == 0 ? 8 : 4));
                const int64_t part_off = o[2];
                const int g = Q.add(it, o);
                kern::QItem ksum = q_item(kern::QI_KSUM, bi, n);
                ksum.tc = tc;
                ksum.ksplit = ks;
                ksum.total = total;
                ksum.dep0 = g;
                ksum.flags = out_flags;
                ksum.n_units = (total + 255) / 256;
                ksum.units_per_task = (int32_t)q_units_per_task(ksum.n_units, 256 * (int64_t)ks);
                last = Q.add(ksum, {part_off, -1, coff, -1});
            } else {
                it.flags = out_flags;
                o[2] = coff;
                last = Q.add(it, o);
            }
        } else {
            kern::QItem it = q_item(kern::QI_STEP, bi, n);
            std::array<int64_t, 4> o{-1, -1, -1, -1};
            set_ab(it, o, A, B);
            it.ta = A.t;
            it.tb = s.b < 0 ? A.t : B.t;
            it.tc = tc;
            it.comp = comp ? 1 : 0;
            it.unary = s.b < 0 ? 1 : 0;
            kern::StepArgs &a = it.s;
            a.n_ohi = (int32_t)s.n_ohi;
            a.n_olo = (int32_t)s.n_olo;
            a.n_shi = (int32_t)s.n_shi;
            a.n_slo = (int32_t)s.n_slo;
            a.t_ohi = (int32_t)s.t_ohi;
            a.t_olo = (int32_t)s.t_olo;
            a.t_shi = (int32_t)s.t_shi;
            a.t_slo = (int32_t)s.t_slo;
            a.R = s.r_global;
            a.log2R = 0;
            while ((1 << a.log2R) < a.R) ++a.log2R;
            a.n_out = s.n_out;
            a.split = 1;
            a.chunk = 0;
            a.part = nullptr;
            if (s.split_global > 1) {
                a.split = s.split_global;
                a.chunk = (s.n_sum + s.split_global - 1) / s.split_global;
                o[3] = Q.take(s.n_out * s.split_global * 16);
            }
            it.n_units = (s.n_out * a.R * a.split + kBlock - 1) / kBlock;
            it.units_per_task = (int32_t)q_step_blocks_per_task(a, s.n_sum, it.n_units);
            if (a.split > 1) {
                const int g = Q.add(it, o);
                kern::QItem fin = q_item(kern::QI_FINISH, bi, n);
                fin.tc = tc;
                fin.comp = it.comp;
                fin.s = a;
                fin.dep0 = g;
                fin.flags = out_flags;
                fin.n_units = (s.n_out + 3) / 4;
                fin.units_per_task = (int32_t)q_units_per_task(fin.n_units, 4 * (int64_t)a.split);
                last = Q.add(fin, {-1, -1, coff, o[3]});
            } else {
                it.flags = out_flags;
                o[2] = coff;
                last = Q.add(it, o);
            }
        }
        if (!s.final_step) prod[s.c] = last;
    }
    if (last < 0 || !(Q.items[last].flags & kern::QF_OUT)) {
        Q.items.resize(first);
        Q.off.resize(first);
        Q.level.resize(first);
        Q.sub.resize(first);
        throw Error{HTN_E_STATE, "queue: the last kernel step does not write the output"};
    }
    return true;
}

// A net run step by step joins the work queue by default when its kernel
// steps are small (mean below kQueueMeanStepMults multiplications): a
// launch per step would then cost about as much as the step.  Nets of few
// large steps keep one launch per step, which spreads each step over the
// whole device (the queue keeps a net on one XCD).
static constexpr double kQueueMeanStepMults = 524288.0;
static bool queue_by_default(const Net &n) {
    const size_t k = n.plan.kernel_steps.size();
    return k > 0 && n.plan.mults / (double)k < kQueueMeanStepMults;
}

// Hardware ids of the device's XCDs (a probe launch at first use per
// device; {0} if the probe finds none).
static std::vector<int> device_xccs(int dev) {
    static std::mutex mu;
    static std::unordered_map<int, std::vector<int>> known;
    std::lock_guard<std::mutex> lk(mu);
    auto it = known.find(dev);
    if (it != known.end()) return it->second;
    uint32_t *d = dalloc<uint32_t>(1);
    const uint32_t mask = kern::queue_xcc_mask(d);
    dfree(d);
    std::vector<int> ids;
    for (int x = 0; x < kern::QC_MAX_SUB; ++x)
        if (mask & (1u << x)) ids.push_back(x);
    if (ids.empty()) ids.push_back(0);
    known[dev] = ids;
    return ids;
}

// Orders the items by sub-queue, then dependency level (a task's producers
// all come earlier in its sub-queue), cuts them into tasks, allocates the
// workspace and uploads.
static void queue_upload(htn_batch *b, QBuild &Q, const std::vector<int> &sub_xcc) {
    htn_batch::Queue &q = b->q;
    const int ni = (int)Q.items.size();
    const int n_sub = (int)sub_xcc.size();
    std::vector<int> order(ni), pos(ni);
    for (int i = 0; i < ni; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return Q.sub[x] != Q.sub[y] ? Q.sub[x] < Q.sub[y] : Q.level[x] < Q.level[y];
    });
    for (int i = 0; i < ni; ++i) pos[order[i]] = i;
    std::vector<int32_t> qinfo(kern::kQInfoWords, -1);
    for (int k = 0; k < n_sub; ++k) qinfo[sub_xcc[k]] = k;
    for (int k = 0; k <= n_sub; ++k) qinfo[kern::QC_MAX_SUB + k] = 0;
    q.d_ws = Q.ws > 0 ? dalloc_bytes((size_t)Q.ws) : nullptr;
    unsigned char *ws = (unsigned char *)q.d_ws;
    std::vector<kern::QItem> items(ni);
    std::vector<int32_t> init(ni);
    std::vector<kern::QTask> tasks;
    std::vector<char> seen(b->nets.size(), 0);
    for (int i = 0; i < ni; ++i) {
        kern::QItem it = Q.items[order[i]];
        const auto &o = Q.off[order[i]];
        if (o[0] >= 0) it.A = ws + o[0];
        if (o[1] >= 0) it.B = ws + o[1];
        if (o[2] >= 0) it.C = ws + o[2];
        if (o[3] >= 0) it.s.part = (double *)(ws + o[3]);
        if (it.dep0 >= 0) it.dep0 = pos[it.dep0];
        if (it.dep1 >= 0) it.dep1 = pos[it.dep1];
        if (it.dep0 >= i || it.dep1 >= i) throw Error{HTN_E_STATE, "queue: dependency listed after its consumer"};
        if (!seen[it.net]) {
            it.flags |= kern::QF_FIRST;
            seen[it.net] = 1;
        }
        const int64_t nt = (it.n_units + it.units_per_task - 1) / it.units_per_task;
        if (nt < 1 || nt > (int64_t(1) << 30) || (int64_t)tasks.size() + nt > (int64_t(1) << 30))
            throw Error{HTN_E_UNSUPPORTED, "queue: too many tasks"};
        it.n_tasks = (int32_t)nt;
        init[i] = (int32_t)nt;
        for (int64_t t = 0; t < nt; ++t) tasks.push_back(kern::QTask{i, (int32_t)t});
        items[i] = it;
        if (it.dep0 >= 0 && Q.sub[order[it.dep0]] != Q.sub[order[i]]) throw Error{HTN_E_STATE, "queue: dependency across sub-queues"};
        if (it.dep1 >= 0 && Q.sub[order[it.dep1]] != Q.sub[order[i]]) throw Error{HTN_E_STATE, "queue: dependency across sub-queues"};
        qinfo[kern::QC_MAX_SUB + Q.sub[order[i]] + 1] = (int32_t)tasks.size();
    }
    for (int k = 1; k <= n_sub; ++k)  // sub-queues without items
        qinfo[kern::QC_MAX_SUB + k] = std::max(qinfo[kern::QC_MAX_SUB + k], qinfo[kern::QC_MAX_SUB + k - 1]);
    q.n_sub = n_sub;
    q.d_qinfo = dalloc<int32_t>(kern::kQInfoWords);
    HIP_TRY(hipMemcpy(q.d_qinfo, qinfo.data(), kern::kQInfoWords * 4, hipMemcpyHostToDevice));
    q.n_items = ni;
    q.n_tasks = (int)tasks.size();
    q.gk = Q.gk;
    q.lds = kern::queue_gemm_lds(Q.gk);
    q.d_items = dalloc<kern::QItem>(ni);
    HIP_TRY(hipMemcpy(q.d_items, items.data(), ni * sizeof(kern::QItem), hipMemcpyHostToDevice));
    q.d_tasks = dalloc<kern::QTask>(tasks.size());
    HIP_TRY(hipMemcpy(q.d_tasks, tasks.data(), tasks.size() * sizeof(kern::QTask), hipMemcpyHostToDevice));
    q.d_init = dalloc<int32_t>(ni);
    HIP_TRY(hipMemcpy(q.d_init, init.data(), ni * 4, hipMemcpyHostToDevice));
    q.d_counters = dalloc<int32_t>(ni);
    HIP_TRY(hipMemcpy(q.d_counters, init.data(), ni * 4, hipMemcpyHostToDevice));
    std::vector<int32_t> ctrl(kern::QC_WORDS, 0);
    q.d_ctrl = dalloc<int32_t>(kern::QC_WORDS);
    HIP_TRY(hipMemcpy(q.d_ctrl, ctrl.data(), kern::QC_WORDS * 4, hipMemcpyHostToDevice));
    int dev = 0, cus = 256;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // every XCD must get workgroups: the whole resident capacity (workgroups
    // are spread over the XCDs; those without a task leave at once)
    q.n_blocks = std::max(kern::queue_blocks_per_cu(q.gk, q.lds) * cus, 2 * kern::QC_MAX_SUB);
}

htn_status htn_batch_create(htn_batch_t *out, int32_t n, const htn_net_t *nets) {
    API_GUARD_BEGIN
    if (!out || n < 1 || !nets) return fail(HTN_E_ARG, "bad batch arguments");
    *out = nullptr;
    htn_batch *b = new htn_batch;
    try {
        b->nets.assign(nets, nets + n);
        std::vector<kern::FusedDesc> desc(n);
        for (int i = 0; i < n; ++i)
            if (!nets[i]) throw Error{HTN_E_ARG, "nets[" + std::to_string(i) + "] is NULL"};
        // straggler threshold from the work of the fused-eligible nets and
        // the resident workgroup slots of their launch shape
        double fused_total = 0.0;
        int slots_per_cu = 8;
        for (int i = 0; i < n; ++i)
            if (use_fused_in_batch(*nets[i])) {
                fused_total += nets[i]->plan.mults;
                slots_per_cu = std::min(slots_per_cu,
                                        fused_slots_per_cu(nets[i]->fused_threads, nets[i]->plan.fused_lds_bytes));
            }
        int dev = 0, cus = 256;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        double straggler = std::max(kStragglerFloor, kStragglerFactor * fused_total / ((double)slots_per_cu * cus));
        {
            // the work queue gives each net one XCD: fused-eligible nets
            // that would go to it beyond one per XCD (they would wait behind
            // another net there) stay in the fused launch, the lightest first
            std::vector<double> over;
            for (int i = 0; i < n; ++i) {
                const Net &net = *nets[i];
                if (net.queue_mode == 0 && use_fused_in_batch(net) && net.plan.mults > straggler &&
                    queue_by_default(net))
                    over.push_back(net.plan.mults);
            }
            const size_t n_xcd = over.empty() ? 0 : device_xccs(dev).size();
            if (over.size() > n_xcd) {
                std::sort(over.begin(), over.end(), std::greater<double>());
                straggler = std::max(straggler, over[n_xcd]);
            }
        }
        for (int i = 0; i < n; ++i) {
            Net &net = *nets[i];
            if (net.n_slices > 1)
                throw Error{HTN_E_UNSUPPORTED, "net " + std::to_string(i) + " is sliced: contract it with htn_contract"};
            ensure_device(net);
            b->versions.push_back(net.plan_version);
            b->uploads.push_back(net.dev->uploads);
            desc[i] = fused_desc(*net.dev, false, net.plan.fused_lds_only);
            if (net.queue_mode == 1 || !use_fused_in_batch(net) || net.plan.mults > straggler) {
                b->step_nets.push_back(i);
                continue;
            }
            int c = (int)net.compute, fm = final_mode(net);
            if (c == HTN_F64 && fm == kern::FM_F64) fm = kern::FM_INTER;
            const int th = net.fused_threads;
            auto it = std::find_if(b->groups.begin(), b->groups.end(), [&](const htn_batch::Group &g) {
                return g.compute == c && g.fm == fm && g.threads == th;
            });
            if (it == b->groups.end()) {
                b->groups.push_back({});
                it = b->groups.end() - 1;
                it->compute = c;
                it->fm = fm;
                it->threads = th;
            }
            it->idx.push_back(i);
            it->lds = std::max<int>(it->lds, (int)net.plan.fused_lds_bytes);
        }
        for (auto &g : b->groups) {
            std::stable_sort(g.idx.begin(), g.idx.end(),
                             [&](int x, int y) { return nets[x]->plan.mults > nets[y]->plan.mults; });
            g.d_order = dalloc<int32_t>(g.idx.size());
            HIP_TRY(hipMemcpy(g.d_order, g.idx.data(), g.idx.size() * 4, hipMemcpyHostToDevice));
            std::vector<kern::FPrepEntry> fp;
            for (int i : g.idx) {
                const DeviceState &D = *nets[i]->dev;
                fp.insert(fp.end(), D.fprep.begin(), D.fprep.end());
                g.fprep_max = std::max(g.fprep_max, D.fprep_max);
                g.fprep_form = std::max(g.fprep_form, D.fprep_form);
            }
            g.n_fprep = (int)fp.size();
            if (!fp.empty()) {
                g.d_fprep = dalloc<kern::FPrepEntry>(fp.size());
                HIP_TRY(hipMemcpy(g.d_fprep, fp.data(), fp.size() * sizeof(kern::FPrepEntry), hipMemcpyHostToDevice));
            }
        }
        b->d_desc = dalloc<kern::FusedDesc>(n);
        HIP_TRY(hipMemcpy(b->d_desc, desc.data(), n * sizeof(kern::FusedDesc), hipMemcpyHostToDevice));
        b->d_outs = dalloc<void *>(n);
        b->d_stamps = dalloc<int64_t>(2 * (size_t)n + 1);  // [2n]: start of the run
        if (!b->step_nets.empty()) {
            // heaviest first, each to the least loaded side stream
            std::stable_sort(b->step_nets.begin(), b->step_nets.end(),
                             [&](int x, int y) { return nets[x]->plan.mults > nets[y]->plan.mults; });
            const int ns = std::min<int>(kSideStreams, (int)b->step_nets.size());
            std::vector<double> load(ns, 0.0);
            for (int i : b->step_nets) {
                const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                b->side_of.push_back(q);
                load[q] += nets[i]->plan.mults;
            }
            // the work queue takes every step-by-step net it can, each net
            // on the least loaded XCD (heaviest first)
            QBuild Q;
            const std::vector<int> xccs = device_xccs(dev);
            std::vector<double> xload(xccs.size(), 0.0);
            b->in_queue.assign(b->step_nets.size(), 0);
            for (size_t k = 0; k < b->step_nets.size(); ++k) {
                Net &net = *nets[b->step_nets[k]];
                if (net.queue_mode == 2 || (net.queue_mode == 0 && !queue_by_default(net))) continue;
                Q.cur_sub = (int)(std::min_element(xload.begin(), xload.end()) - xload.begin());
                if (queue_net(Q, net, b->step_nets[k])) {
                    b->in_queue[k] = 1;
                    ++b->q.n_nets;
                    xload[Q.cur_sub] += net.plan.mults;
                }
            }
            if (!Q.items.empty()) {
                queue_upload(b, Q, xccs);
                if (!b->groups.empty()) {
                    HIP_TRY(hipStreamCreateWithFlags(&b->q.stream, hipStreamNonBlocking));
                    HIP_TRY(hipEventCreateWithFlags(&b->q.ev_fork, hipEventDisableTiming));
                    HIP_TRY(hipEventCreateWithFlags(&b->q.ev_join, hipEventDisableTiming));
                }
            }
            HIP_TRY(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
            for (int q = 0; q < ns; ++q) {
                hipStream_t sq = nullptr;
                HIP_TRY(hipStreamCreateWithFlags(&sq, hipStreamNonBlocking));
                b->sides.push_back(sq);
                hipEvent_t e = nullptr;
                HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
                b->ev_join.push_back(e);
            }
        }
    } catch (...) {
        batch_free(b);
        delete b;
        throw;
    }
    *out = b;
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_batch_set_graph(htn_batch_t b, int32_t use_graph) {
    API_GUARD_BEGIN
    if (!b) return fail(HTN_E_ARG, "batch is NULL");
    if (use_graph < 0 || use_graph > HTN_GRAPH_FORCE_FAILURE) return fail(HTN_E_ARG, "bad graph mode");
    b->use_graph = use_graph != 0;
    b->force_capture_failure = use_graph == HTN_GRAPH_FORCE_FAILURE;
    b->graph_failed = false;
    b->graph_error.clear();
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_batch_graph_state(htn_batch_t b, int32_t *state) {
    API_GUARD_BEGIN
    if (!b || !state) return fail(HTN_E_ARG, "NULL argument");
    if (b->graph_failed) {
        *state = 2;
        g_err = b->graph_error;
    } else {
        *state = b->gexec ? 1 : 0;
    }
    return HTN_OK;
    API_GUARD_END
}

// Launch sequence of a batch run: a clock read marks the start; input
// materialisation and the fused launch go on the caller's stream; nets run
// step by step (the large ones) are spread over the side streams, forked
// after the fused launch is queued; the caller's stream finally waits for
// every side stream.  Every net's start and completion clock lands in
// d_stamps.
static void batch_enqueue(htn_batch *b, void *const *outs, hipStream_t st, bool events) {
    const size_t n = b->nets.size();
    // the run's start clock: written by the first materialisation launch,
    // or by a launch of its own when there is none
    int64_t *run_start = b->d_stamps + 2 * n;
    const bool prep_stamps = !b->groups.empty() && b->groups[0].n_fprep > 0;
    // the queue (not while per-step phase clocks are asked for); alone, it
    // stamps the run's start itself
    const bool use_queue = b->q.n_tasks > 0 && !b->d_phase;
    const bool queue_alone = use_queue && b->groups.empty();
    if (!prep_stamps && !queue_alone) HIP_TRY(kern::launch_stamp(run_start, st));
    if (events) HIP_TRY(hipEventRecord(next_event(b), st));
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        const auto &g = b->groups[gi];
        HIP_TRY(kern::launch_fprep(g.d_fprep, g.n_fprep, g.fprep_form, g.fprep_max, g.compute,
                                   gi == 0 && prep_stamps ? run_start : nullptr, st));
    }
    if (events) HIP_TRY(hipEventRecord(next_event(b), st));
    if (!b->sides.empty()) {
        HIP_TRY(hipEventRecord(b->ev_fork, st));
        for (hipStream_t q : b->sides) HIP_TRY(hipStreamWaitEvent(q, b->ev_fork, 0));
    }
    if (use_queue && !queue_alone) {
        HIP_TRY(hipEventRecord(b->q.ev_fork, st));
        HIP_TRY(hipStreamWaitEvent(b->q.stream, b->q.ev_fork, 0));
    }
    for (auto &g : b->groups)
        HIP_TRY(kern::launch_fused(b->d_desc, g.d_order, b->d_outs, b->d_stamps, nullptr, b->d_phase, b->max_phases,
                                   (int)g.idx.size(), g.lds, g.compute, g.fm, g.threads, st));
    if (events) HIP_TRY(hipEventRecord(next_event(b), st));
    // the queue goes after the fused launch: launched first, its resident
    // workgroups would hold every CU while the fused nets wait
    if (use_queue) {
        const htn_batch::Queue &q = b->q;
        HIP_TRY(kern::launch_queue(q.d_items, q.d_tasks, q.d_qinfo, q.n_sub, q.d_init, q.d_counters, q.n_items,
                                   q.d_ctrl, b->d_outs, b->d_stamps, queue_alone ? run_start : nullptr, q.gk, q.lds,
                                   q.n_blocks, queue_alone ? st : q.stream));
    }
    if (use_queue && !queue_alone) {
        HIP_TRY(hipEventRecord(b->q.ev_join, b->q.stream));
        HIP_TRY(hipStreamWaitEvent(st, b->q.ev_join, 0));
    }
    for (size_t k = 0; k < b->step_nets.size(); ++k) {
        if (use_queue && b->in_queue[k]) continue;
        const int i = b->step_nets[k];
        hipStream_t ss = b->sides[b->side_of[k]];
        HIP_TRY(kern::launch_stamp(b->d_stamps + 2 * (size_t)i, ss));
        run_steps(*b->nets[i], outs[i], ss, b->d_phase ? b->d_phase + (size_t)i * b->max_phases : nullptr,
                  b->max_phases);
        HIP_TRY(kern::launch_stamp(b->d_stamps + 2 * (size_t)i + 1, ss));
    }
    for (size_t q = 0; q < b->sides.size(); ++q) {
        HIP_TRY(hipEventRecord(b->ev_join[q], b->sides[q]));
        HIP_TRY(hipStreamWaitEvent(st, b->ev_join[q], 0));
    }
}

// Records the batch's launches on st into a HIP graph and instantiates it.
// Any failure (the stream cannot be captured, a launch refused inside the
// capture, instantiation) leaves st out of capture mode, frees what was
// built and marks the batch to run eagerly from then on.
static void capture_batch(htn_batch *b, void *const *outs, hipStream_t st) {
    auto give_up = [&](const std::string &why) {
        b->graph_failed = true;
        b->graph_error = "graph capture failed, running eagerly: " + why;
        if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->gexec = nullptr;
        b->graph = nullptr;
        (void)hipGetLastError();
    };
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return give_up(std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    std::string why;
    try {
        batch_enqueue(b, outs, st, false);
        if (b->force_capture_failure) why = "capture failure forced by the caller";
    } catch (const Error &err) {
        why = err.msg;
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(st, &g);
    if (why.empty() && e != hipSuccess) why = std::string("hipStreamEndCapture: ") + hipGetErrorString(e);
    b->graph = g;
    if (!why.empty()) return give_up(why);
    e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return give_up(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
}

htn_status htn_batch_run(htn_batch_t b, void *const *outs, void *hip_stream) {
    API_GUARD_BEGIN
    if (!b || !outs) return fail(HTN_E_ARG, "NULL argument");
    const int n = (int)b->nets.size();
    for (int i = 0; i < n; ++i) {
        if (!outs[i]) return fail(HTN_E_ARG, "outs[" + std::to_string(i) + "] is NULL");
        if (b->nets[i]->plan_version != b->versions[i] || b->nets[i]->data_dirty ||
            b->nets[i]->dev->uploads != b->uploads[i])
            return fail(HTN_E_STATE, "net " + std::to_string(i) + " changed after htn_batch_create");
    }
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<void *> ov(outs, outs + n);
    if (ov != b->outs_uploaded) {
        HIP_TRY(hipStreamSynchronize(st));
        HIP_TRY(hipMemcpy(b->d_outs, ov.data(), n * sizeof(void *), hipMemcpyHostToDevice));
        b->outs_uploaded = ov;
    }
    if (b->use_graph && st != nullptr && !b->graph_failed) {
        if (b->gexec && (b->graph_outs != ov || b->graph_stream != st)) {
            (void)hipGraphExecDestroy(b->gexec);
            (void)hipGraphDestroy(b->graph);
            b->gexec = nullptr;
            b->graph = nullptr;
        }
        if (!b->gexec) {
            batch_enqueue(b, outs, st, false);  // first run eagerly (also sets kernel attributes)
            capture_batch(b, outs, st);          // on failure: later runs stay eager
            if (!b->graph_failed) {
                b->graph_outs = ov;
                b->graph_stream = st;
            }
            return HTN_OK;
        }
        HIP_TRY(hipGraphLaunch(b->gexec, st));
        return HTN_OK;
    }
    batch_enqueue(b, outs, st, b->event_timing);
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_batch_set_event_timing(htn_batch_t b, int32_t on) {
    API_GUARD_BEGIN
    if (!b) return fail(HTN_E_ARG, "batch is NULL");
    b->event_timing = on != 0;
    b->ev_used = 0;
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_batch_launch_ms(htn_batch_t b, float *prep_ms, float *fused_ms, int32_t *runs) {
    API_GUARD_BEGIN
    if (!b) return fail(HTN_E_ARG, "batch is NULL");
    const size_t k = b->ev_used / 3;
    double sp = 0.0, sf = 0.0;
    for (size_t r = 0; r < k; ++r) {
        float a = 0.0f, c = 0.0f;
        HIP_TRY(hipEventSynchronize(b->ev_pool[3 * r + 2]));
        HIP_TRY(hipEventElapsedTime(&a, b->ev_pool[3 * r], b->ev_pool[3 * r + 1]));
        HIP_TRY(hipEventElapsedTime(&c, b->ev_pool[3 * r + 1], b->ev_pool[3 * r + 2]));
        sp += a;
        sf += c;
    }
    if (prep_ms) *prep_ms = k ? (float)(sp / k) : 0.0f;
    if (fused_ms) *fused_ms = k ? (float)(sf / k) : 0.0f;
    if (runs) *runs = (int32_t)k;
    b->ev_used = 0;
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_batch_timestamps(htn_batch_t b, int64_t *ticks) {
    API_GUARD_BEGIN
    if (!b || !ticks) return fail(HTN_E_ARG, "NULL argument");
    const int n = (int)b->nets.size();
    std::vector<int64_t> st(2 * (size_t)n + 1);
    HIP_TRY(hipMemcpy(st.data(), b->d_stamps, st.size() * 8, hipMemcpyDeviceToHost));
    const int64_t t0 = st[2 * (size_t)n];
    for (size_t k = 0; k < 2 * (size_t)n; ++k) ticks[k] = st[k] - t0;
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_batch_set_phase_timing(htn_batch_t b, int32_t max_phases) {
    API_GUARD_BEGIN
    if (!b || max_phases < 0) return fail(HTN_E_ARG, "bad arguments");
    if (b->gexec) return fail(HTN_E_STATE, "phase timing must be set before the graph is captured");
    dfree(b->d_phase);
    b->d_phase = nullptr;
    b->max_phases = max_phases;
    if (max_phases > 0) {
        const size_t n = (size_t)max_phases * b->nets.size();
        b->d_phase = dalloc<int64_t>(n);
        std::vector<int64_t> neg(n, -1);
        HIP_TRY(hipMemcpy(b->d_phase, neg.data(), n * 8, hipMemcpyHostToDevice));
    }
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_batch_phase_times(htn_batch_t b, int64_t *ticks) {
    API_GUARD_BEGIN
    if (!b || !ticks) return fail(HTN_E_ARG, "NULL argument");
    if (!b->d_phase) return fail(HTN_E_STATE, "phase timing is off");
    const int n = (int)b->nets.size();
    const size_t cnt = (size_t)b->max_phases * n;
    std::vector<int64_t> ph(cnt), st(2 * (size_t)n + 1);
    HIP_TRY(hipMemcpy(ph.data(), b->d_phase, cnt * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(st.data(), b->d_stamps, st.size() * 8, hipMemcpyDeviceToHost));
    const int64_t t0 = st[2 * (size_t)n];
    for (size_t k = 0; k < cnt; ++k) ticks[k] = ph[k] >= 0 ? ph[k] - t0 : -1;
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_batch_step_times(htn_batch_t b, float *times, int32_t capacity) {
    API_GUARD_BEGIN
    if (!b || !times || capacity < 0) return fail(HTN_E_ARG, "bad arguments");
    if (!b->d_phase) return fail(HTN_E_STATE, "phase timing is off");
    const int n = (int)b->nets.size();
    const int mp = b->max_phases;
    std::vector<int64_t> ph((size_t)mp * n), st(2 * (size_t)n);
    HIP_TRY(hipMemcpy(ph.data(), b->d_phase, ph.size() * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(st.data(), b->d_stamps, st.size() * 8, hipMemcpyDeviceToHost));
    const float nan = std::numeric_limits<float>::quiet_NaN();
    for (size_t k = 0; k < (size_t)n * capacity; ++k) times[k] = nan;
    for (auto &g : b->groups)
        for (int i : g.idx) {
            const Plan &P = b->nets[i]->plan;
            const int64_t *t = ph.data() + (size_t)i * mp;
            std::vector<int> heaviest;  // per phase: position of its step with the most multiplications
            for (int q = 0; q < (int)P.kernel_steps.size(); ++q) {
                const int f = P.steps[P.kernel_steps[q]].f_phase;
                if (f < 0) continue;
                if ((int)heaviest.size() <= f) heaviest.resize(f + 1, -1);
                if (heaviest[f] < 0 || P.steps[P.kernel_steps[q]].mults > P.steps[P.kernel_steps[heaviest[f]]].mults)
                    heaviest[f] = q;
            }
            for (int q = 0; q < (int)P.kernel_steps.size() && q < capacity; ++q) {
                const int f = P.steps[P.kernel_steps[q]].f_phase;
                if (f < 0 || f >= mp || t[f] < 0 || heaviest[f] != q) continue;
                const int64_t begin = f == 0 ? st[2 * (size_t)i] : t[f - 1];
                if (begin < 0) continue;
                times[(size_t)i * capacity + q] = (float)(t[f] - begin) * 0.01f;  // 100 MHz ticks -> us
            }
        }
    // nets run step by step: the clock after each kernel step (only nets
    // that run step by step in any batch: a net moved off the fused kernel
    // for its size in this batch is described by fused-executor features)
    for (int i : b->step_nets) {
        if (use_fused_in_batch(*b->nets[i])) continue;
        const Plan &P = b->nets[i]->plan;
        const int64_t *t = ph.data() + (size_t)i * mp;
        for (int q = 0; q < (int)P.kernel_steps.size() && q < capacity && q < mp; ++q) {
            const int64_t begin = q == 0 ? st[2 * (size_t)i] : t[q - 1];
            if (t[q] < 0 || begin < 0 || t[q] < begin) continue;
            times[(size_t)i * capacity + q] = (float)(t[q] - begin) * 0.01f;
        }
    }
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_batch_queue_info(htn_batch_t b, int32_t *n_nets, int32_t *n_tasks, int32_t *error) {
    API_GUARD_BEGIN
    if (!b) return fail(HTN_E_ARG, "batch is NULL");
    if (n_nets) *n_nets = b->q.n_nets;
    if (n_tasks) *n_tasks = b->q.n_tasks;
    if (error) {
        *error = 0;
        if (b->q.d_ctrl) {
            HIP_TRY(hipDeviceSynchronize());
            int32_t e = 0;
            HIP_TRY(hipMemcpy(&e, b->q.d_ctrl + kern::QC_ERR, 4, hipMemcpyDeviceToHost));
            *error = e;
            if (e) {
                const int32_t zero = 0;
                HIP_TRY(hipMemcpy(b->q.d_ctrl + kern::QC_ERR, &zero, 4, hipMemcpyHostToDevice));
            }
        }
    }
    return HTN_OK;
    API_GUARD_END
}

void htn_batch_destroy(htn_batch_t b) {
    if (!b) return;
    batch_free(b);
    delete b;
}

htn_status htn_contract_batch(int32_t n, const htn_net_t *nets, void *const *outs, void *hip_stream) {
    htn_batch_t b = nullptr;
    htn_status s = htn_batch_create(&b, n, nets);
    if (s != HTN_OK) return s;
    s = htn_batch_run(b, outs, hip_stream);
    if (s == HTN_OK) {
        // The batch's device buffers are read by the launch: wait before
        // releasing them.
        hipError_t e = hipStreamSynchronize((hipStream_t)hip_stream);
        if (e != hipSuccess) s = fail(HTN_E_DEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    }
    htn_batch_destroy(b);
    return s;
}

htn_status htn_autotune(int32_t n, const htn_net_t *nets, void *const *outs, void *hip_stream,
                        int32_t *best_threads, int32_t *best_lds_bytes, float *best_ms) {
    API_GUARD_BEGIN
    if (n < 1 || !nets || !outs) return fail(HTN_E_ARG, "bad arguments");
    for (int i = 0; i < n; ++i)
        if (!nets[i] || !outs[i]) return fail(HTN_E_ARG, "NULL net or output");
    static const int cand[][2] = {{64, 32768},   {64, 49152},   {64, 65536},   {256, 32768},
                                  {256, 49152},  {256, 65536},  {256, 98304},  {256, 163840},
                                  {512, 65536},  {512, 98304},  {512, 163840}};
    const hipStream_t st = (hipStream_t)hip_stream;
    std::vector<int> old_threads(n);
    std::vector<int64_t> old_lds(n);
    for (int i = 0; i < n; ++i) {
        old_threads[i] = nets[i]->fused_threads;
        old_lds[i] = nets[i]->fused_lds_budget;
    }
    auto apply = [&](int threads, int64_t lds) {
        for (int i = 0; i < n; ++i) {
            nets[i]->fused_threads = threads;
            nets[i]->fused_lds_budget = lds;
            replan(*nets[i]);
        }
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = -1.0f;
    int bt = old_threads[0];
    int64_t bl = old_lds[0];
    try {
        for (const auto &c : cand) {
            htn_batch_t b = nullptr;
            try {
                apply(c[0], c[1]);
                if (htn_batch_create(&b, n, nets) != HTN_OK) continue;
                // two runs to warm up (first-use uploads, kernel attributes)
                bool ok = htn_batch_run(b, outs, st) == HTN_OK && htn_batch_run(b, outs, st) == HTN_OK;
                std::vector<float> ms;
                for (int r = 0; ok && r < 5; ++r) {
                    HIP_TRY(hipEventRecord(e0, st));
                    ok = htn_batch_run(b, outs, st) == HTN_OK;
                    HIP_TRY(hipEventRecord(e1, st));
                    HIP_TRY(hipEventSynchronize(e1));
                    float t = 0.0f;
                    HIP_TRY(hipEventElapsedTime(&t, e0, e1));
                    ms.push_back(t);
                }
                HIP_TRY(hipStreamSynchronize(st));
                htn_batch_destroy(b);
                b = nullptr;
                if (!ok) continue;  // e.g. an LDS budget the device refuses
                std::sort(ms.begin(), ms.end());
                const float med = ms[ms.size() / 2];
                if (best < 0.0f || med < best) {
                    best = med;
                    bt = c[0];
                    bl = c[1];
                }
            } catch (const Error &) {
                if (b) htn_batch_destroy(b);
                (void)hipStreamSynchronize(st);
            }
        }
        if (best < 0.0f) throw Error{HTN_E_UNSUPPORTED, "no candidate configuration ran"};
        apply(bt, bl);
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        for (int i = 0; i < n; ++i) {
            nets[i]->fused_threads = old_threads[i];
            nets[i]->fused_lds_budget = old_lds[i];
            try {
                replan(*nets[i]);
            } catch (...) {
            }
        }
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best_threads) *best_threads = bt;
    if (best_lds_bytes) *best_lds_bytes = (int32_t)bl;
    if (best_ms) *best_ms = best;
    return HTN_OK;
    API_GUARD_END
}

// ------------------------------------------------------------ cost model

}  // extern "C"

struct htn_model {
    int device = -1;
    float *d_p = nullptr, *d_m = nullptr, *d_v = nullptr, *d_g = nullptr;
    int64_t step = 0;  // Adam steps taken
    int64_t cap = 0;   // samples the work arrays hold
    float *d_x = nullptr, *d_t = nullptr, *d_y = nullptr, *d_z1 = nullptr, *d_z2 = nullptr, *d_d1 = nullptr,
          *d_d2 = nullptr, *d_dy = nullptr, *d_loss = nullptr;
    int32_t *d_idx = nullptr;
    int64_t idx_cap = 0, loss_cap = 0;
    std::mutex predict_mu;  // model_predict shares d_x / d_y between threads
};

namespace {

// Runs a block with the model's device current.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        HIP_TRY(hipGetDevice(&prev));
        if (prev != dev) HIP_TRY(hipSetDevice(dev));
    }
    ~DeviceScope() {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

void model_free_work(htn_model *m) {
    for (float *p : {m->d_x, m->d_t, m->d_y, m->d_z1, m->d_z2, m->d_d1, m->d_d2, m->d_dy}) dfree(p);
    m->d_x = m->d_t = m->d_y = m->d_z1 = m->d_z2 = m->d_d1 = m->d_d2 = m->d_dy = nullptr;
    m->cap = 0;
}

void model_reserve(htn_model *m, int64_t n) {
    if (n <= m->cap) return;
    model_free_work(m);
    const int64_t F = HTN_MODEL_FEATURES, H = HTN_MODEL_HIDDEN;
    m->d_x = dalloc<float>(n * F);
    m->d_t = dalloc<float>(n);
    m->d_y = dalloc<float>(n);
    m->d_z1 = dalloc<float>(n * H);
    m->d_z2 = dalloc<float>(n * H);
    m->d_d1 = dalloc<float>(n * H);
    m->d_d2 = dalloc<float>(n * H);
    m->d_dy = dalloc<float>(n);
    m->cap = n;
}

uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

double uniform01(uint64_t &s) { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

}  // namespace

namespace htn {
std::vector<float> model_predict(htn_model *m, const std::vector<float> &x) {
    const int64_t n = (int64_t)(x.size() / HTN_MODEL_FEATURES);
    std::vector<float> y(n);
    if (n == 0) return y;
    std::lock_guard<std::mutex> lock(m->predict_mu);
    DeviceScope ds(m->device);
    model_reserve(m, n);
    HIP_TRY(hipMemcpy(m->d_x, x.data(), x.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(kern::launch_mlp_forward(m->d_p, m->d_x, nullptr, (int)n, m->d_y, nullptr, nullptr, nullptr));
    HIP_TRY(hipMemcpy(y.data(), m->d_y, n * 4, hipMemcpyDeviceToHost));
    return y;
}
}  // namespace htn

extern "C" {

int64_t htn_model_param_count(void) { return kern::model_param_count(); }

htn_status htn_model_create(htn_model_t *out, uint64_t seed) {
    API_GUARD_BEGIN
    if (!out) return fail(HTN_E_ARG, "out is NULL");
    *out = nullptr;
    const int64_t np = kern::model_param_count();
    const int F = HTN_MODEL_FEATURES, H = HTN_MODEL_HIDDEN;
    std::vector<float> p(np, 0.0f);
    uint64_t s = seed;
    auto fill = [&](int64_t off, int64_t count, int fan_in) {
        const double a = std::sqrt(6.0 / fan_in);
        for (int64_t k = 0; k < count; ++k) p[off + k] = (float)((2.0 * uniform01(s) - 1.0) * a);
    };
    fill(0, (int64_t)H * F, F);                          // W1
    fill((int64_t)H * F + H, (int64_t)H * H, H);         // W2
    fill((int64_t)H * F + H + H * H + H, H, H);          // w3
    auto *m = new htn_model();
    try {
        HIP_TRY(hipGetDevice(&m->device));
        m->d_p = dalloc<float>(np);
        m->d_m = dalloc<float>(np);
        m->d_v = dalloc<float>(np);
        m->d_g = dalloc<float>(np);
        HIP_TRY(hipMemcpy(m->d_p, p.data(), np * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemset(m->d_m, 0, np * 4));
        HIP_TRY(hipMemset(m->d_v, 0, np * 4));
    } catch (...) {
        htn_model_destroy(m);
        throw;
    }
    *out = m;
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_model_set_params(htn_model_t m, const float *params) {
    API_GUARD_BEGIN
    if (!m || !params) return fail(HTN_E_ARG, "NULL argument");
    DeviceScope ds(m->device);
    const int64_t np = kern::model_param_count();
    HIP_TRY(hipMemcpy(m->d_p, params, np * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(m->d_m, 0, np * 4));
    HIP_TRY(hipMemset(m->d_v, 0, np * 4));
    m->step = 0;
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_model_get_params(htn_model_t m, float *params) {
    API_GUARD_BEGIN
    if (!m || !params) return fail(HTN_E_ARG, "NULL argument");
    DeviceScope ds(m->device);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(params, m->d_p, kern::model_param_count() * 4, hipMemcpyDeviceToHost));
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_model_forward(htn_model_t m, int32_t n, const float *x, float *y, void *hip_stream) {
    API_GUARD_BEGIN
    if (!m || n < 0 || (n > 0 && (!x || !y))) return fail(HTN_E_ARG, "bad arguments");
    DeviceScope ds(m->device);
    HIP_TRY(kern::launch_mlp_forward(m->d_p, x, nullptr, n, y, nullptr, nullptr, (hipStream_t)hip_stream));
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_model_gradients(htn_model_t m, int32_t n, const float *x, const float *t, float *grad, float *loss,
                               void *hip_stream) {
    API_GUARD_BEGIN
    if (!m || n <= 0 || !x || !t || !grad) return fail(HTN_E_ARG, "bad arguments");
    DeviceScope ds(m->device);
    model_reserve(m, n);
    const hipStream_t st = (hipStream_t)hip_stream;
    HIP_TRY(kern::launch_mlp_forward(m->d_p, x, nullptr, n, m->d_y, m->d_z1, m->d_z2, st));
    HIP_TRY(kern::launch_mlp_backward(m->d_p, x, t, nullptr, n, m->d_y, m->d_z1, m->d_z2, m->d_d1, m->d_d2, m->d_dy,
                                      grad, loss, st));
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_model_adam_step(htn_model_t m, const float *grad, float lr, void *hip_stream) {
    API_GUARD_BEGIN
    if (!m || !grad) return fail(HTN_E_ARG, "NULL argument");
    DeviceScope ds(m->device);
    HIP_TRY(kern::launch_adam(m->d_p, m->d_m, m->d_v, grad, lr, ++m->step, (hipStream_t)hip_stream));
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_model_train(htn_model_t m, int32_t n, const float *x, const float *t, int32_t epochs, int32_t batch,
                           float lr, uint64_t seed, float *epoch_loss, void *hip_stream) {
    API_GUARD_BEGIN
    if (!m || n <= 0 || !x || !t || epochs < 0 || batch <= 0) return fail(HTN_E_ARG, "bad arguments");
    DeviceScope ds(m->device);
    const hipStream_t st = (hipStream_t)hip_stream;
    const int32_t nb_max = std::min(batch, n);
    const int64_t n_mb = (n + nb_max - 1) / nb_max;
    model_reserve(m, nb_max);
    if (m->idx_cap < n) {
        dfree(m->d_idx);
        m->d_idx = nullptr;
        m->d_idx = dalloc<int32_t>(n);
        m->idx_cap = n;
    }
    if (m->loss_cap < n_mb) {
        dfree(m->d_loss);
        m->d_loss = nullptr;
        m->d_loss = dalloc<float>(n_mb);
        m->loss_cap = n_mb;
    }
    std::vector<int32_t> perm(n);
    std::vector<float> losses(n_mb);
    for (int e = 0; e < epochs; ++e) {
        // Fisher-Yates permutation from splitmix64(seed, epoch)
        uint64_t s = seed * 0x9e3779b97f4a7c15ull + (uint64_t)e;
        for (int32_t i = 0; i < n; ++i) perm[i] = i;
        for (int32_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[(int32_t)(splitmix64(s) % (uint64_t)(i + 1))]);
        HIP_TRY(hipMemcpyAsync(m->d_idx, perm.data(), (size_t)n * 4, hipMemcpyHostToDevice, st));
        for (int64_t k = 0; k < n_mb; ++k) {
            const int32_t b0 = (int32_t)(k * nb_max), nb = std::min<int32_t>(nb_max, n - b0);
            HIP_TRY(kern::launch_mlp_forward(m->d_p, x, m->d_idx + b0, nb, m->d_y, m->d_z1, m->d_z2, st));
            HIP_TRY(kern::launch_mlp_backward(m->d_p, x, t, m->d_idx + b0, nb, m->d_y, m->d_z1, m->d_z2, m->d_d1,
                                              m->d_d2, m->d_dy, m->d_g, m->d_loss + k, st));
            HIP_TRY(kern::launch_adam(m->d_p, m->d_m, m->d_v, m->d_g, lr, ++m->step, st));
        }
        // the permutation buffer is reused next epoch: wait for this one
        HIP_TRY(hipStreamSynchronize(st));
        if (epoch_loss) {
            HIP_TRY(hipMemcpy(losses.data(), m->d_loss, n_mb * 4, hipMemcpyDeviceToHost));
            double a = 0.0;
            for (float v : losses) a += v;
            epoch_loss[e] = (float)(a / (double)n_mb);
        }
    }
    return HTN_OK;
    API_GUARD_END
}

void htn_model_destroy(htn_model_t m) {
    if (!m) return;
    model_free_work(m);
    for (float *p : {m->d_p, m->d_m, m->d_v, m->d_g, m->d_loss}) dfree(p);
    dfree(m->d_idx);
    delete m;
}

htn_status htn_set_model(htn_net_t net, htn_model_t model) {
    API_GUARD_BEGIN
    if (!net) return fail(HTN_E_ARG, "net is NULL");
    net->model = model;
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_step_features(htn_net_t net, float *features, int32_t capacity, int32_t *n_steps) {
    API_GUARD_BEGIN
    if (!net || !n_steps || capacity < 0 || (capacity > 0 && !features)) return fail(HTN_E_ARG, "bad arguments");
    std::vector<float> rows;
    step_features(*net, rows);
    const int32_t k = (int32_t)(rows.size() / HTN_MODEL_FEATURES);
    *n_steps = k;
    std::copy(rows.begin(), rows.begin() + (size_t)std::min(k, capacity) * HTN_MODEL_FEATURES, features);
    return HTN_OK;
    API_GUARD_END
}

const char *htn_status_string(htn_status s) {
    switch (s) {
        case HTN_OK: return "HTN_OK";
        case HTN_E_ARG: return "HTN_E_ARG";
        case HTN_E_LABEL: return "HTN_E_LABEL";
        case HTN_E_SHAPE: return "HTN_E_SHAPE";
        case HTN_E_PATH: return "HTN_E_PATH";
        case HTN_E_OOM: return "HTN_E_OOM";
        case HTN_E_DEVICE: return "HTN_E_DEVICE";
        case HTN_E_UNSUPPORTED: return "HTN_E_UNSUPPORTED";
        case HTN_E_STATE: return "HTN_E_STATE";
    }
    return "unknown status";
}

const char *htn_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// QPD sampling and truncation (Sec. 4.3)
// ---------------------------------------------------------------------------

struct htn_trunc {
    int n = 0;
    int elem_bytes = 8;
    int64_t n_blocks = 0;
    kern::TruncItem *d_items = nullptr;
    kern::TruncBlock *d_blocks = nullptr;
    int64_t *d_maps = nullptr;
    ~htn_trunc() {
        dfree(d_items);
        dfree(d_blocks);
        dfree(d_maps);
    }
};

extern "C" {

htn_status htn_qpd_sample(int32_t n, const double *coeffs, int64_t s_qpd, const double *uniforms, int64_t *counts,
                          double *weights) {
    API_GUARD_BEGIN
    if (n < 1 || s_qpd < 1 || !coeffs || !uniforms || !counts || !weights) return fail(HTN_E_ARG, "bad arguments");
    double gamma = 0.0;
    int last = -1;
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(coeffs[i])) return fail(HTN_E_ARG, "non-finite coefficient");
        gamma += std::fabs(coeffs[i]);
        if (coeffs[i] != 0.0) last = i;
    }
    if (last < 0) return fail(HTN_E_ARG, "all coefficients are 0");
    std::vector<double> cdf((size_t)n);
    double acc = 0.0;
    for (int i = 0; i < n; ++i) {
        acc += std::fabs(coeffs[i]);
        cdf[(size_t)i] = acc / gamma;
    }
    std::vector<int64_t> c((size_t)n, 0);
    for (int64_t j = 0; j < s_qpd; ++j) {
        const double u = uniforms[j];
        if (!(u >= 0.0 && u < 1.0)) return fail(HTN_E_ARG, "uniform outside [0, 1)");
        // first i with u < F_i
        const int i = (int)(std::upper_bound(cdf.begin(), cdf.end(), u) - cdf.begin());
        ++c[(size_t)std::min(i, last)];
    }
    for (int i = 0; i < n; ++i) {
        counts[i] = c[(size_t)i];
        const double sg = coeffs[i] > 0.0 ? 1.0 : (coeffs[i] < 0.0 ? -1.0 : 0.0);
        weights[i] = (double)c[(size_t)i] * gamma * sg / (double)s_qpd;
    }
    return HTN_OK;
    API_GUARD_END
}

}  // extern "C"

// One gather item: dst[o] = src[sum over output axes a of offs[a][digit_a(o)]]
// with output digits row-major over the output axes.
struct GatherSpec {
    const void *src = nullptr;
    void *dst = nullptr;
    std::vector<std::vector<int64_t>> offs;  // per output axis: input offset of each index
};

// Packs the items into gather blocks and uploads their descriptors (the
// launch layout of k_truncate: runs of small items per block, 1024-element
// chunks of larger ones).
static htn_trunc *build_gather(const std::vector<GatherSpec> &items, htn_dtype dtype) {
    const int n = (int)items.size();
    std::vector<kern::TruncItem> h((size_t)n);
    std::vector<int64_t> maps;
    std::vector<kern::TruncBlock> blocks;
    constexpr int64_t per_block = kern::kTruncBlockElems;
    int32_t open_fill = per_block;  // elements in the open packed block (none open)
    for (int i = 0; i < n; ++i) {
        const GatherSpec &g = items[(size_t)i];
        kern::TruncItem &k = h[(size_t)i];
        k = kern::TruncItem{};
        k.src = g.src;
        k.dst = g.dst;
        k.rank = (int32_t)g.offs.size();
        k.map_off = (int64_t)maps.size();
        int64_t n_out = 1;
        for (size_t a = 0; a < g.offs.size(); ++a) {
            k.odim[a] = (int32_t)g.offs[a].size();
            k.moff[a] = (int32_t)(maps.size() - (size_t)k.map_off);
            maps.insert(maps.end(), g.offs[a].begin(), g.offs[a].end());
            n_out *= (int64_t)g.offs[a].size();
        }
        if (n_out >= (int64_t(1) << 31))
            throw Error{HTN_E_UNSUPPORTED, "item " + std::to_string(i) + " has 2^31 or more elements"};
        k.n_out = n_out;
        const int64_t mw = (int64_t)maps.size() - k.map_off;  // this item's map entries
        if (n_out > per_block || mw > kern::kTruncMapLds) {
            // a larger item (or one whose maps alone fill the LDS share):
            // 1024-element chunks, one block each
            k.start = 0;
            const int32_t words = mw <= kern::kTruncMapLds ? (int32_t)mw : 0;
            for (int64_t b = 0; b < n_out; b += per_block)
                blocks.push_back(kern::TruncBlock{i, 1, b, k.map_off, words, 0});
            open_fill = per_block;
        } else {
            // small items share a block while their elements, count and
            // maps fit
            if (open_fill + n_out > per_block || blocks.empty() || blocks.back().n_items == kern::kTruncBlockItems ||
                blocks.back().map_words + mw > kern::kTruncMapLds) {
                blocks.push_back(kern::TruncBlock{i, 0, 0, k.map_off, 0, 0});
                open_fill = 0;
            }
            k.start = open_fill;
            ++blocks.back().n_items;
            blocks.back().map_words += (int32_t)mw;
            open_fill += (int32_t)n_out;
        }
        if ((int64_t)blocks.size() >= (int64_t(1) << 31)) throw Error{HTN_E_UNSUPPORTED, "batch too large"};
    }
    htn_trunc *t = new htn_trunc();
    t->n = n;
    t->elem_bytes = dtype_size(dtype);
    t->n_blocks = (int64_t)blocks.size();
    try {
        t->d_items = dalloc<kern::TruncItem>(h.size());
        t->d_blocks = dalloc<kern::TruncBlock>(blocks.size());
        HIP_TRY(hipMemcpy(t->d_blocks, blocks.data(), blocks.size() * sizeof(kern::TruncBlock), hipMemcpyHostToDevice));
        t->d_maps = dalloc<int64_t>(maps.size());
        HIP_TRY(hipMemcpy(t->d_items, h.data(), h.size() * sizeof(kern::TruncItem), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(t->d_maps, maps.data(), maps.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    } catch (...) {
        delete t;
        throw;
    }
    return t;
}

// Row-major strides of an item's input axes; throws on bad extents.
static std::vector<int64_t> gather_strides(int i, int rank, const int64_t *dims) {
    std::vector<int64_t> strides((size_t)rank);
    int64_t stride = 1;
    for (int a = rank - 1; a >= 0; --a) {
        if (dims[a] < 1 || dims[a] > std::numeric_limits<int32_t>::max())
            throw Error{HTN_E_ARG, "item " + std::to_string(i) + ": bad extent"};
        strides[(size_t)a] = stride;
        if (stride > (int64_t(1) << 40) / dims[a]) throw Error{HTN_E_UNSUPPORTED, "item too large"};
        stride *= dims[a];
    }
    return strides;
}

extern "C" {

htn_status htn_truncate_create(htn_trunc_t *out, int32_t n, const htn_truncation *items, htn_dtype dtype) {
    API_GUARD_BEGIN
    if (!out) return fail(HTN_E_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || !items) return fail(HTN_E_ARG, "bad item list");
    if (dtype != HTN_F64 && dtype != HTN_F32 && dtype != HTN_BF16) return fail(HTN_E_ARG, "bad dtype");
    std::vector<GatherSpec> specs((size_t)n);
    for (int i = 0; i < n; ++i) {
        const htn_truncation &t = items[i];
        if (!t.src || !t.dst) return fail(HTN_E_ARG, "item " + std::to_string(i) + ": NULL buffer");
        if (t.rank < 1 || t.rank > HTN_TRUNC_MAX_RANK) return fail(HTN_E_ARG, "item " + std::to_string(i) + ": bad rank");
        const auto strides = gather_strides(i, t.rank, t.dims);
        GatherSpec &g = specs[(size_t)i];
        g.src = t.src;
        g.dst = t.dst;
        g.offs.resize((size_t)t.rank);
        for (int a = 0; a < t.rank; ++a) {
            const int64_t d = t.kept[a] ? t.n_kept[a] : t.dims[a];
            if (d < 1 || d > t.dims[a]) return fail(HTN_E_ARG, "item " + std::to_string(i) + ": bad n_kept");
            for (int64_t x = 0; x < d; ++x) {
                const int64_t idx = t.kept[a] ? t.kept[a][x] : x;
                if (idx < 0 || idx >= t.dims[a])
                    return fail(HTN_E_ARG, "item " + std::to_string(i) + ": kept index out of range");
                g.offs[(size_t)a].push_back(idx * strides[(size_t)a]);
            }
        }
    }
    *out = build_gather(specs, dtype);
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_gather_create(htn_trunc_t *out, int32_t n, const htn_gather *items, htn_dtype dtype) {
    API_GUARD_BEGIN
    if (!out) return fail(HTN_E_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || !items) return fail(HTN_E_ARG, "bad item list");
    if (dtype != HTN_F64 && dtype != HTN_F32 && dtype != HTN_BF16) return fail(HTN_E_ARG, "bad dtype");
    std::vector<GatherSpec> specs((size_t)n);
    for (int i = 0; i < n; ++i) {
        const htn_gather &t = items[i];
        const std::string it = "item " + std::to_string(i) + ": ";
        if (!t.src || !t.dst) return fail(HTN_E_ARG, it + "NULL buffer");
        if (t.rank < 1 || t.rank > HTN_TRUNC_MAX_RANK) return fail(HTN_E_ARG, it + "bad rank");
        if (t.out_rank < 1 || t.out_rank > t.rank) return fail(HTN_E_ARG, it + "bad out_rank");
        const auto strides = gather_strides(i, t.rank, t.dims);
        std::vector<char> seen((size_t)t.rank, 0);
        int used = 0;
        GatherSpec &g = specs[(size_t)i];
        g.src = t.src;
        g.dst = t.dst;
        g.offs.resize((size_t)t.out_rank);
        for (int o = 0; o < t.out_rank; ++o) {
            const int na = t.n_axes[o];
            if (na < 1 || used + na > t.rank) return fail(HTN_E_ARG, it + "bad n_axes");
            int64_t ext = 1;
            std::vector<int> ax((size_t)na);
            for (int k = 0; k < na; ++k) {
                const int a = t.axes[used + k];
                if (a < 0 || a >= t.rank || seen[(size_t)a]) return fail(HTN_E_ARG, it + "axes is not a permutation");
                seen[(size_t)a] = 1;
                ax[(size_t)k] = a;
                ext *= t.dims[a];
                if (ext >= (int64_t(1) << 31)) return fail(HTN_E_UNSUPPORTED, it + "fused axis too long");
            }
            used += na;
            const int64_t d = t.kept[o] ? t.n_kept[o] : ext;
            if (d < 1 || d > ext) return fail(HTN_E_ARG, it + "bad n_kept");
            for (int64_t x = 0; x < d; ++x) {
                int64_t f = t.kept[o] ? t.kept[o][x] : x;
                if (f < 0 || f >= ext) return fail(HTN_E_ARG, it + "kept index out of range");
                // the fused index, row-major over the axes (first slowest)
                int64_t off = 0;
                for (int k = na - 1; k >= 0; --k) {
                    const int64_t e = t.dims[ax[(size_t)k]];
                    off += (f % e) * strides[(size_t)ax[(size_t)k]];
                    f /= e;
                }
                g.offs[(size_t)o].push_back(off);
            }
        }
        if (used != t.rank) return fail(HTN_E_ARG, it + "axes must list every input axis once");
    }
    *out = build_gather(specs, dtype);
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_qpd_fuse(int32_t n, const int32_t *dims, const double *const *coeffs, double *fused) {
    API_GUARD_BEGIN
    if (n < 1 || !dims || !coeffs || !fused) return fail(HTN_E_ARG, "bad arguments");
    int64_t total = 1;
    for (int k = 0; k < n; ++k) {
        if (dims[k] < 1 || !coeffs[k]) return fail(HTN_E_ARG, "bad coefficient tensor " + std::to_string(k));
        total *= dims[k];
        if (total >= (int64_t(1) << 31)) return fail(HTN_E_UNSUPPORTED, "fused tensor too long");
    }
    // the tensor product, one factor at a time: index row-major over the
    // tensors in the order given (the first slowest)
    fused[0] = 1.0;
    int64_t len = 1;
    for (int k = 0; k < n; ++k) {
        const int64_t d = dims[k];
        for (int64_t f = len - 1; f >= 0; --f) {
            const double v = fused[f];
            for (int64_t x = d - 1; x >= 0; --x) fused[f * d + x] = v * coeffs[k][x];
        }
        len *= d;
    }
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_truncate_run(htn_trunc_t t, void *hip_stream) {
    API_GUARD_BEGIN
    if (!t) return fail(HTN_E_ARG, "handle is NULL");
    HIP_TRY(kern::launch_truncate(t->d_items, t->d_blocks, t->n_blocks, t->d_maps, t->elem_bytes,
                                  (hipStream_t)hip_stream));
    return HTN_OK;
    API_GUARD_END
}

void htn_truncate_destroy(htn_trunc_t t) { delete t; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Sliced networks: every slice (the network with its sliced labels fixed) is
// a network of its own; one gather launch cuts every input's slices out of
// its device copy, the slices run as one batch, and a last launch sums their
// results in FP64.
// ---------------------------------------------------------------------------

namespace htn {
struct SliceRun {
    int version = -1;           // plan version it was built for
    htn_trunc *gather = nullptr;
    void *buf = nullptr;        // slice inputs: [slice][sliced input][elements]
    void *parts = nullptr;      // slice results: [slice][output elements]
    std::vector<htn_net *> subs;
    htn_batch *batch = nullptr;
    std::vector<void *> outs;
};
}  // namespace htn

static void free_slices(DeviceState &D) {
    SliceRun *r = D.slices;
    if (!r) return;
    D.slices = nullptr;
    if (r->batch) htn_batch_destroy(r->batch);
    for (htn_net *m : r->subs) htn_destroy(m);
    delete r->gather;
    dfree(r->buf);
    dfree(r->parts);
    delete r;
}

static void build_slices(Net &n) {
    DeviceState &D = *n.dev;
    const htn_dtype tin = input_dtype(n.compute);
    const int es = dtype_size(tin);
    const std::vector<int64_t> sd = sliced_dims(n);
    const int64_t S = n.n_slices;
    std::vector<char> is_sliced(n.dims.size(), 0);
    for (int l : n.sliced) is_sliced[l] = 1;
    // per slice: each input that carries a sliced label gets its own copy
    std::vector<int64_t> soff(n.n_t, -1), ssize(n.n_t, 1);
    int64_t per = 0;
    for (int i = 0; i < n.n_t; ++i) {
        bool carries = false;
        for (int l : n.labels[i]) {
            ssize[i] *= sd[l];
            carries = carries || is_sliced[l];
        }
        if (carries) {
            soff[i] = per;
            per += (ssize[i] * es + 255) / 256 * 256;
        }
    }
    auto *r = new SliceRun();
    D.slices = r;  // freed by free_slices on any failure below
    if (per > 0) r->buf = dalloc_bytes((size_t)(S * per));
    std::vector<GatherSpec> specs;
    std::vector<int64_t> val(n.dims.size(), 0);
    for (int64_t s = 0; s < S; ++s) {
        int64_t rem = s;  // the slice's label values, row-major over n.sliced (first slowest)
        for (int k = (int)n.sliced.size() - 1; k >= 0; --k) {
            val[n.sliced[k]] = rem % n.dims[n.sliced[k]];
            rem /= n.dims[n.sliced[k]];
        }
        for (int i = 0; i < n.n_t; ++i) {
            if (soff[i] < 0) continue;
            GatherSpec g;
            g.src = D.in[i];
            g.dst = (unsigned char *)r->buf + s * per + soff[i];
            const auto &ls = n.labels[i];
            int64_t stride = 1;
            g.offs.resize(ls.size());
            for (int a = (int)ls.size() - 1; a >= 0; --a) {
                const int l = ls[a];
                if (is_sliced[l])
                    g.offs[a].push_back(val[l] * stride);
                else
                    for (int64_t x = 0; x < n.dims[l]; ++x) g.offs[a].push_back(x * stride);
                stride *= n.dims[l];
            }
            specs.push_back(std::move(g));
        }
    }
    if (!specs.empty()) r->gather = build_gather(specs, tin);
    int64_t out_elems = 1;
    for (int l : n.out_labels) out_elems *= n.dims[l];
    const int oes = dtype_size(out_dtype(n));
    r->parts = dalloc_bytes((size_t)(S * out_elems * oes));
    for (int64_t s = 0; s < S; ++s) {
        auto *m = new htn_net;
        r->subs.push_back(m);
        Net &t = *m;
        t = structure_copy(n);
        t.dims = sd;
        for (int i = 0; i < t.n_t; ++i) t.sizes[i] = ssize[i];
        t.slice_mode = 0;
        t.storage = tin;
        t.data_on_device = true;
        t.user_ptrs.resize(t.n_t);
        t.host.assign(t.n_t, {});
        for (int i = 0; i < t.n_t; ++i)
            t.user_ptrs[i] = soff[i] >= 0 ? (const void *)((unsigned char *)r->buf + s * per + soff[i]) : D.in[i];
        t.data_dirty = true;
        t.path = n.path;
        t.path_kind = 0;
        build_plan(t);
        r->outs.push_back((unsigned char *)r->parts + s * out_elems * oes);
    }
    htn_batch_t b = nullptr;
    if (htn_batch_create(&b, (int32_t)S, (const htn_net_t *)r->subs.data()) != HTN_OK)
        throw Error{HTN_E_DEVICE, std::string("slice batch: ") + htn_last_error()};
    r->batch = b;
    r->version = n.plan_version;
}

static void run_sliced(Net &n, void *out, hipStream_t st) {
    DeviceState &D = *n.dev;
    if (D.slices && D.slices->version != n.plan_version) free_slices(D);
    if (!D.slices) {
        try {
            build_slices(n);
        } catch (...) {
            free_slices(D);
            throw;
        }
    }
    SliceRun &r = *D.slices;
    if (r.gather)
        HIP_TRY(kern::launch_truncate(r.gather->d_items, r.gather->d_blocks, r.gather->n_blocks, r.gather->d_maps,
                                      r.gather->elem_bytes, st));
    if (htn_batch_run(r.batch, r.outs.data(), st) != HTN_OK)
        throw Error{HTN_E_DEVICE, std::string("slice batch: ") + htn_last_error()};
    int64_t out_elems = 1;
    for (int l : n.out_labels) out_elems *= n.dims[l];
    HIP_TRY(kern::launch_slice_sum(r.parts, (int)n.n_slices, out_elems, out, out_dtype(n) == HTN_F64 ? 0 : 1,
                                   n.final_sum == HTN_SUM_COMPENSATED, st));
}

// ---------------------------------------------------------------------------
// QT evaluator (Sec. 6.2)
// ---------------------------------------------------------------------------

struct htn_qteval {
    int n_inst = 0;
    int64_t n_outputs = 0, n_entries = 0;
    kern::SvInst *d_insts = nullptr;
    kern::SvOp *d_ops = nullptr;
    double2 *d_state = nullptr;
    double *d_outs = nullptr;
    int64_t *d_start = nullptr, *d_term = nullptr;
    double *d_coef = nullptr;
    ~htn_qteval() {
        dfree(d_insts);
        dfree(d_ops);
        dfree(d_state);
        dfree(d_outs);
        dfree(d_start);
        dfree(d_term);
        dfree(d_coef);
    }
};

extern "C" {

htn_status htn_qt_eval_create(htn_qteval_t *out, int32_t n_instances, const htn_sv_instance *instances,
                              int64_t n_entries, const int64_t *entry_start, const int64_t *term_output,
                              const double *term_coef) {
    API_GUARD_BEGIN
    if (!out) return fail(HTN_E_ARG, "out is NULL");
    *out = nullptr;
    if (n_instances < 1 || !instances) return fail(HTN_E_ARG, "bad instance list");
    if (n_entries < 0 || (n_entries > 0 && !entry_start)) return fail(HTN_E_ARG, "bad entry list");
    std::vector<kern::SvInst> hi((size_t)n_instances);
    std::vector<kern::SvOp> hops;
    int64_t n_out = 0, n_state = 0;
    for (int i = 0; i < n_instances; ++i) {
        const htn_sv_instance &x = instances[i];
        const std::string it = "instance " + std::to_string(i) + ": ";
        if (x.n_qubits < 1 || x.n_qubits > HTN_SV_MAX_QUBITS) return fail(HTN_E_ARG, it + "bad qubit count");
        if (!x.init || !x.observable || (x.n_ops > 0 && !x.ops) || x.n_ops < 0) return fail(HTN_E_ARG, it + "NULL data");
        if (x.n_kept < 0 || x.n_kept > x.n_qubits || (x.n_kept > 0 && !x.kept)) return fail(HTN_E_ARG, it + "bad kept list");
        kern::SvInst &k = hi[(size_t)i];
        std::memset(&k, 0, sizeof(k));
        const int n = x.n_qubits;
        k.n = n;
        k.n_ops = x.n_ops;
        k.n_kept = x.n_kept;
        k.op_off = (int64_t)hops.size();
        k.out_off = n_out;
        for (int q = 0; q < n; ++q) {
            for (int c = 0; c < 4; ++c) k.init[q][c] = x.init[4 * q + c];
            const int64_t bit = int64_t(1) << (n - 1 - q);
            switch (x.observable[q]) {
                case 'I': break;
                case 'X': k.xmask |= bit; break;
                case 'Y': k.xmask |= bit; k.zymask |= bit; ++k.n_y; break;
                case 'Z': k.zymask |= bit; break;
                default: return fail(HTN_E_ARG, it + "observable must be I, X, Y or Z per qubit");
            }
        }
        for (int j = 0; j < x.n_kept; ++j) {
            const int q = x.kept[j];
            if (q < 0 || q >= n || x.observable[q] != 'I') return fail(HTN_E_ARG, it + "kept qubit out of range or not I");
            for (int j2 = 0; j2 < j; ++j2)
                if (x.kept[j2] == q) return fail(HTN_E_ARG, it + "kept qubit repeated");
            k.kept[j] = q;
        }
        for (int j = 0; j < x.n_ops; ++j) {
            const htn_sv_op &o = x.ops[j];
            const bool two = o.kind == HTN_SV_CZ || o.kind == HTN_SV_CX || o.kind == HTN_SV_RZZ;
            if (o.kind < HTN_SV_U1 || o.kind > HTN_SV_PROJ) return fail(HTN_E_ARG, it + "bad op kind");
            if (o.q0 < 0 || o.q0 >= n) return fail(HTN_E_ARG, it + "op qubit out of range");
            if (two && (o.q1 < 0 || o.q1 >= n || o.q1 == o.q0)) return fail(HTN_E_ARG, it + "bad second qubit");
            if (o.kind == HTN_SV_PROJ && o.q1 != 0 && o.q1 != 1) return fail(HTN_E_ARG, it + "projection bit not 0/1");
            kern::SvOp d;
            d.kind = o.kind;
            d.q0 = o.q0;
            d.q1 = o.q1;
            d.pad = 0;
            for (int c = 0; c < 8; ++c) d.m[c] = o.m[c];
            hops.push_back(d);
        }
        n_out += int64_t(1) << x.n_kept;
        if (n > kern::kSvLdsQubits) {
            k.state_off = n_state;
            n_state += int64_t(1) << n;
        } else {
            k.state_off = -1;
        }
    }
    if (n_entries > 0) {
        if (entry_start[0] != 0) return fail(HTN_E_ARG, "entry_start[0] must be 0");
        for (int64_t e = 0; e < n_entries; ++e)
            if (entry_start[e + 1] < entry_start[e]) return fail(HTN_E_ARG, "entry_start must not decrease");
        const int64_t n_terms = entry_start[n_entries];
        if (n_terms > 0 && (!term_output || !term_coef)) return fail(HTN_E_ARG, "NULL terms");
        for (int64_t t = 0; t < n_terms; ++t)
            if (term_output[t] < 0 || term_output[t] >= n_out) return fail(HTN_E_ARG, "term output out of range");
    }
    auto *q = new htn_qteval();
    try {
        q->n_inst = n_instances;
        q->n_outputs = n_out;
        q->n_entries = n_entries;
        q->d_insts = dalloc<kern::SvInst>(hi.size());
        HIP_TRY(hipMemcpy(q->d_insts, hi.data(), hi.size() * sizeof(kern::SvInst), hipMemcpyHostToDevice));
        q->d_ops = dalloc<kern::SvOp>(std::max<size_t>(1, hops.size()));
        if (!hops.empty())
            HIP_TRY(hipMemcpy(q->d_ops, hops.data(), hops.size() * sizeof(kern::SvOp), hipMemcpyHostToDevice));
        if (n_state > 0) q->d_state = dalloc<double2>((size_t)n_state);
        q->d_outs = dalloc<double>((size_t)n_out);
        if (n_entries > 0) {
            const int64_t n_terms = entry_start[n_entries];
            q->d_start = dalloc<int64_t>((size_t)n_entries + 1);
            HIP_TRY(hipMemcpy(q->d_start, entry_start, ((size_t)n_entries + 1) * 8, hipMemcpyHostToDevice));
            q->d_term = dalloc<int64_t>(std::max<int64_t>(1, n_terms));
            q->d_coef = dalloc<double>(std::max<int64_t>(1, n_terms));
            if (n_terms > 0) {
                HIP_TRY(hipMemcpy(q->d_term, term_output, (size_t)n_terms * 8, hipMemcpyHostToDevice));
                HIP_TRY(hipMemcpy(q->d_coef, term_coef, (size_t)n_terms * 8, hipMemcpyHostToDevice));
            }
        }
    } catch (...) {
        delete q;
        throw;
    }
    *out = q;
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_qt_eval_run(htn_qteval_t q, double *entries, double *outputs, void *hip_stream) {
    API_GUARD_BEGIN
    if (!q) return fail(HTN_E_ARG, "handle is NULL");
    if (q->n_entries > 0 && !entries) return fail(HTN_E_ARG, "entries is NULL");
    const hipStream_t st = (hipStream_t)hip_stream;
    double *outs = outputs ? outputs : q->d_outs;
    HIP_TRY(kern::launch_sv_eval(q->d_insts, q->n_inst, q->d_ops, q->d_state, outs, st));
    HIP_TRY(kern::launch_qt_assemble(q->d_start, q->d_term, q->d_coef, q->n_entries, outs, entries, st));
    return HTN_OK;
    API_GUARD_END
}

htn_status htn_qt_eval_info(htn_qteval_t q, int64_t *n_outputs, int64_t *n_entries) {
    API_GUARD_BEGIN
    if (!q) return fail(HTN_E_ARG, "handle is NULL");
    if (n_outputs) *n_outputs = q->n_outputs;
    if (n_entries) *n_entries = q->n_entries;
    return HTN_OK;
    API_GUARD_END
}

void htn_qt_eval_destroy(htn_qteval_t q) { delete q; }

}  // extern "C"
