// Internal data structures of the h-TN library: network description,
// contraction plan, device state.  Host-only C++ (no HIP types here, so the
// planner can be reasoned about and exercised without a GPU).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "htn.h"

namespace htn {

// Threads per workgroup of the fused and per-step kernels.
constexpr int kBlock = 256;
// Largest number of coefficient tensors folded into one operand load.
constexpr int kMaxScales = 8;

// Largest extent product kept in the low half of a two-level offset table.
constexpr int64_t kTabLoMax = 1024;

// One pairwise step of the path (or a planner-added unary final step).
struct StepPlan {
    int a = -1, b = -1;  // operand SSA ids; b < 0: unary step
    int c = -1;          // result SSA id
    std::vector<int> a_labels, b_labels;  // operand labels (physical order)
    std::vector<int> c_labels;            // result labels (physical order)
    std::vector<int> sum_labels;          // labels summed in this step
    double mults = 0.0;                   // paper's cost of the step
    bool absorbed = false;   // folded into the larger operand's load
    bool final_step = false; // writes the net's output
    bool out_bf16 = false;   // writes its result as BF16 (a packed matrix-core operand)
    bool synthetic = false;  // added by the planner, not part of the path
    // Kernel geometry (kernel steps only).  Output index o = o_hi*n_olo+o_lo,
    // summed index s = s_hi*n_slo+s_lo.  Each table entry is an (A offset,
    // B offset) pair; the operand offset of (o, s) is the sum of the four
    // table entries it selects.
    int64_t n_out = 1, n_sum = 1;
    int64_t n_ohi = 1, n_olo = 1, n_shi = 1, n_slo = 1;
    int64_t t_ohi = 0, t_olo = 0, t_shi = 0, t_slo = 0;  // offsets in pairs
    int r_fused = 1;   // lanes per output in the fused kernel (kBlock = block mode)
    int r_global = 1;  // lanes per output in the per-step kernel
    // per-step kernel: lane groups per output, each summing one chunk of
    // the summed range (split sums of few outputs with long sums), and the
    // workspace byte offset of their (sum, compensation) partials
    int split_global = 1;
    int64_t ws_part = -1;
    // matrix-core steps: K ranges computed in parallel and their partial
    // products' workspace byte offset
    int ksplit = 1;
    int64_t ws_kpart = -1;
    // Matrix-core steps (mfma = 1): C[b][m][n] = sum_k A[b][m][k] B[b][n][k]
    // after packing A to [batch][M][K] and B to [batch][N][K] (same K order).
    int mfma = 0;
    std::vector<int> g_batch, g_m, g_n, g_k;  // label groups
    int64_t gb = 1, gm = 1, gn = 1, gk = 1;   // group extents
    struct Pack {
        int64_t n = 0, n_ohi = 1, n_olo = 1, t_ohi = 0, t_olo = 0, t_one = 0;
        bool identity = false;  // the operand is already packed (no pack launch)
    } pack_a, pack_b;
    int64_t ws_pa = -1, ws_pb = -1;  // workspace byte offsets of the packed operands
    // Register-tiled steps (tile = 1, fused kernel): a plain GEMM view
    // C[m][n] = sum_k A[k][m] B[k][n] with A laid out [K][M] and B [K][N]
    // (same K order), so the inner loop has unit strides; C is written
    // through offset tables t_cm[m] + t_cn[n] into its consumer's layout.
    int tile = 0;
    std::vector<int> t_gm, t_gn, t_gk;  // tiled view's groups (ascending labels)
    int64_t tM = 1, tN = 1, tK = 1;
    int64_t t_cm = 0, t_cn = 0;  // table offsets (pairs, .x used; per-step executor replay)
    // C offset of m (and of n) from mixed-radix digits: per label of the
    // group (last fastest) its extent, magic multiplier (2 words) and C
    // stride; floor(x / d) = (x * magic) >> 40.
    std::vector<int32_t> c_digits_m, c_digits_n;
    int TM = 1, TN = 1, GX = 16;  // per-thread tile and thread-grid width
    // Fused kernel: the waves [f_w0, f_w0 + f_nw) of the workgroup run the
    // step; steps of one phase are independent and run side by side.
    int f_w0 = 0, f_nw = 1;
    // Fused-program facts (features of the learned cost model).
    // Fold chains (per-step executor): a large tensor contracted with small
    // matrices one mode at a time; the chain's steps run as one launch at
    // its first step (chain: index in Plan::chains, chain_pos: position)
    int chain = -1, chain_pos = -1;
    int f_phase = -1;           // phase of the fused kernel that runs the step
    int f_spill = 0;            // bit 0: A, bit 1: B, bit 2: C outside LDS
    int64_t f_copy_chunks = 0;  // 16-byte chunks copied while the step runs
};

// An SSA value: an input tensor (possibly with coefficient tensors folded
// in) or the result of a kernel step.
struct Value {
    std::vector<int> labels;  // physical order
    int64_t size = 1;
    bool input = false;
    int base = -1;            // original tensor id when `input`
    std::vector<int> scales;  // original tensor ids folded into it
    int producer = -1;        // step index when not `input`
};

// A scale table: entry e of the target multiplies by
// scale_tensor[hi[e / n_lo] + lo[e % n_lo]].
struct ScaleRef {
    int tensor = -1;
    int64_t t_hi = 0, t_lo = 0;  // offsets (in pairs; the .x half is used)
    int64_t n_lo = 1;
};

// Materialisation of an input with folded coefficients (per-step executor)
// or its load into LDS (fused executor).
struct LoadPlan {
    int value = -1;   // SSA id
    // digit form of the load (fused kernel): value labels in layout order
    // with extents, the base tensor's stride and each scale's stride per
    // label (0 when the scale does not carry it)
    int base = -1;    // original tensor id
    int64_t size = 0;
    std::vector<ScaleRef> scales;
    // Layout change: entry e of the value reads the base tensor at
    // src_hi[e / src_nlo] + src_lo[e % src_nlo] (src_nlo = 0: same layout).
    int64_t src_thi = 0, src_tlo = 0, src_nlo = 0;
    int64_t desc_word = -1;  // word offset of its digit-form descriptor in the fused image
    bool needs_copy() const { return !scales.empty() || src_nlo > 0; }
};

struct Plan {
    std::vector<StepPlan> steps;     // path steps + optional synthetic final
    std::vector<Value> values;       // indexed by SSA id
    std::vector<int> kernel_steps;   // indices into steps, execution order
    // fused kernel: groups of independent kernel steps (positions in
    // kernel_steps) that run side by side in one phase, in phase order
    std::vector<std::vector<int>> fused_phases;
    std::vector<LoadPlan> loads;     // inputs needing scaling (by first use)
    // fold chains: step indices in chain order (see StepPlan::chain)
    std::vector<std::vector<int>> chains;
    // per chain, the chain at whose first step it is launched: itself, or
    // an earlier chain of its group (chains whose first steps follow one
    // another in the step order, with only steps of the group's chains in
    // between, and whose large tensor is a network input: independent of
    // each other, so one launch runs them side by side)
    std::vector<int> chain_lead;
    // per chain, whether its large tensor is read in place (FoldLayout::x_raw)
    std::vector<char> chain_x_raw;
    std::vector<int32_t> tables;     // flat (x, y) pairs
    int final_value = -1;
    double mults = 0.0;
    double peak = 0.0;
    int n_absorbed = 0;
    // per-step executor workspace (bytes), offsets per SSA id (-1: input)
    int64_t ws_bytes = 0;
    std::vector<int64_t> ws_off;
    // fused executor: program words, LDS need and spill scratch.  Values
    // that do not fit the LDS budget live in a per-network global scratch
    // (fused_scratch_bytes); fused_pure means nothing spilled.
    bool fused_ok = false;        // AUTO picks the fused kernel
    bool fused_batch_ok = false;  // batches run the net in the fused launch
    bool fused_possible = false;  // program and table slots fit the LDS budget
    bool fused_pure = false;
    bool fused_lds_only = false;  // every operand and result of every step in LDS
    int64_t fused_lds_bytes = 0;
    int64_t fused_scratch_bytes = 0;
    std::vector<int32_t> program;
    // word positions of device-pointer slots in `program`: (position, tensor);
    // the executor writes the tensor's device address there at upload
    std::vector<std::pair<int64_t, int>> ptr_slots;
    std::vector<std::pair<int64_t, int>> fused_in_ptr_slots;
    int64_t fused_input_bytes = 0;  // front of the workspace: materialised inputs
};

struct DeviceState;  // defined in the executor

struct Net {
    // structure
    int n_t = 0;
    std::vector<std::vector<int>> labels;
    std::vector<int64_t> dims;
    std::vector<int> out_labels;
    std::vector<int64_t> sizes;
    htn_dtype storage = HTN_F64, compute = HTN_F64;
    htn_final_sum final_sum = HTN_SUM_PLAIN;
    // options
    htn_exec_mode exec = HTN_EXEC_AUTO;
    int64_t max_intermediate = (int64_t(1) << 31) - 1;
    int64_t fused_lds_budget = 65536;
    int fused_threads = 256;  // threads per network in the fused kernel (64, 256 or 512)
    double fused_max_mults = 67108864.0;        // AUTO runs larger spilled nets step by step
    double batch_fused_max_mults = 33554432.0;  // batch limit for nets with matrix-core steps
    int allow_mfma = 1;
    int slice_mode = 0;         // 1: slice summed labels until the path fits max_intermediate
    int queue_mode = 0;         // batches: 0 step-by-step nets in the work queue, 1 always, 2 never
    int path_samples = 32;      // sampled-greedy candidates
    uint64_t path_seed = 0;
    // data
    bool data_on_device = false;
    std::vector<const void *> user_ptrs;          // borrowed device pointers
    std::vector<std::vector<unsigned char>> host;  // host copies (compute input dtype)
    bool data_dirty = true;
    // path and plan
    std::vector<std::pair<int, int>> path;
    int path_kind = HTN_PATH_GREEDY;
    Plan plan;
    int plan_version = 0;
    // slicing: labels fixed per slice (row-major over this list, first
    // slowest) and the number of slices; plan then describes one slice
    std::vector<int> sliced;
    int64_t n_slices = 1;
    DeviceState *dev = nullptr;
    struct htn_model *model = nullptr;  // cost model of HTN_PATH_LEARNED (borrowed)
};

// Element sizes.
inline int dtype_size(htn_dtype t) { return t == HTN_F64 ? 8 : (t == HTN_F32 ? 4 : 2); }
// Type of inputs as stored on the device for a compute type.
inline htn_dtype input_dtype(htn_dtype compute) { return compute; }
// Type of intermediates for a compute type.
inline htn_dtype inter_dtype(htn_dtype compute) { return compute == HTN_F64 ? HTN_F64 : HTN_F32; }
inline htn_dtype out_dtype(const Net &n) {
    return n.final_sum == HTN_SUM_PLAIN ? inter_dtype(n.compute) : HTN_F64;
}

// Host layout of a fold chain (see Plan::chains): in-tile axes (first
// slowest; every folded axis, plus carried axes while the tile stays
// small), outer axes (first slowest), one stage per chain step.
struct FoldLayout {
    bool ok = false;
    int x = -1, y = -1;                 // source value (X) and result value
    // X is a network input with no folded scales: read in place from its
    // original tensor (no materialised copy)
    bool x_raw = false;
    std::vector<int> ext0, ext1;        // in-tile extents at X / at the result
    std::vector<int64_t> s_src, s_dst;  // in-tile strides in X / in the result
    std::vector<int> fold_ax, fold_ext; // per stage: in-tile axis, its new extent
    std::vector<int> m_tensor;          // per stage: the matrix's original tensor id
    std::vector<int64_t> m_in, m_out;   // per stage: matrix strides of the old / new index
    std::vector<int> o_ext;             // outer extents
    std::vector<int64_t> o_src, o_dst;  // outer strides
    int64_t n_outer = 1;
    int d_max = 1, tf = 1;
    int64_t lds_bytes = 0;
};
FoldLayout fold_layout(const Net &n, const Plan &P, const std::vector<int> &chain);

// planner.cpp
struct Error {
    htn_status st;
    std::string msg;
};
void validate_structure(const Net &n);                       // throws Error
std::vector<std::pair<int, int>> greedy_path(const Net &n);  // throws Error
std::vector<std::pair<int, int>> sampled_path(const Net &n, int n_samples, uint64_t seed);
std::vector<std::vector<std::pair<int, int>>> candidate_paths(const Net &n, int n_samples, uint64_t seed);
// A copy of a net's structure and options without its data, path or plan.
Net structure_copy(const Net &n);
// cost_model.cpp
constexpr int kFeatures = HTN_MODEL_FEATURES;
// Appends one row of kFeatures floats per kernel step of n.plan.
void step_features(const Net &n, std::vector<float> &rows);
std::vector<std::pair<int, int>> learned_path(const Net &n);  // throws Error
// api.hip: the model's predictions for rows of x (runs on the current device).
std::vector<float> model_predict(struct htn_model *m, const std::vector<float> &x);
void check_path(const Net &n, const std::vector<std::pair<int, int>> &p);  // throws Error
void build_plan(Net &n);                                     // throws Error
// build_plan, slicing summed labels first when slice_mode is on and the
// path's largest intermediate exceeds max_intermediate (throws Error)
void plan_net(Net &n);
// Extents of a sliced network: every sliced label has extent 1.
std::vector<int64_t> sliced_dims(const Net &n);
// Largest intermediate (elements) of the net's path under the given extents.
double path_peak(const Net &n, const std::vector<int64_t> &dims);
std::string plan_json(const Net &n);

}  // namespace htn
