// Host-side launchers of the HIP kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace htn {
namespace kern {

// dtype codes follow htn_dtype: 0 f64, 1 f32, 2 bf16.

// Final-step accumulation modes.
enum FinalMode { FM_INTER = 0, FM_F64 = 1, FM_COMP = 2 };

// Geometry of one pairwise step (see StepPlan).
struct StepArgs {
    int32_t n_ohi, n_olo, n_shi, n_slo;
    int32_t t_ohi, t_olo, t_shi, t_slo;
    int32_t R;       // lanes per output, power of two <= 64
    int32_t log2R;
    int64_t n_out;
    // Split sums: with split > 1, `split` groups of R lanes per output each
    // sum `chunk` consecutive summed terms into part[2 * (o * split + j)]
    // (sum, compensation); a second launch combines them in order.
    int32_t split = 1;
    int64_t chunk = 0;
    double *part = nullptr;
};

// Generic contraction C[o] = sum_s A[offA(o,s)] * B[offB(o,s)] (B == NULL:
// unary).  ta/tb: operand dtypes; acc_f64: accumulate in FP64; comp:
// Neumaier compensation (needs acc_f64); tc: output dtype (0 or 1).
hipError_t launch_step(const void *A, int ta, const void *B, int tb, void *C, int tc, bool acc_f64, bool comp,
                       const int2 *tab, const StepArgs &s, hipStream_t st);

// Scaled-input materialisation (one launch for all inputs of a net).
constexpr int kMaxScalesDev = 16;
struct PrepDesc {
    const void *src;   // input in its device dtype
    int64_t dst_off;   // byte offset of its intermediate-dtype copy in the workspace
    int32_t size;
    int32_t ns;
    const void *sp[kMaxScalesDev];
    int32_t thi[kMaxScalesDev], tlo[kMaxScalesDev], nlo[kMaxScalesDev];
    int32_t sthi, stlo, snlo;  // source gather table (snlo = 0: same layout)
};
// ws: the workspace the copies are written to (base of dst_off).
hipError_t launch_prep(const PrepDesc *d_desc, int n_desc, int max_size, int tin, int tinter, const int2 *tab,
                       void *ws, hipStream_t st);

// Fused whole-network kernel.
struct FPrepEntry;
struct FusedDesc {
    const int32_t *prog;
    const int2 *tab;
    const void *const *in;  // device array of input pointers
    void *scratch;          // workspace: materialised inputs, then spill space
    // inputs the workgroup materialises itself before its program
    // (n_fprep = 0: already done by a separate launch)
    const FPrepEntry *fprep;
    int32_t n_fprep;
    int32_t lds_only;  // every operand and result of every step in LDS
};
// nets[order[b]] is run by workgroup b; outs[net] receives its result.
// stamps (optional): [2*net] start, [2*net+1] end, 100 MHz ticks.
// out1 (optional): output of a single-network launch, used instead of outs.
// phase_ticks (optional): [net * max_phases + k] receives the clock at the
// end of the network's k-th phase (after its barrier).
// threads: 64, 256 or 512.
hipError_t launch_fused(const FusedDesc *nets, const int32_t *order, void *const *outs, int64_t *stamps, void *out1,
                        int64_t *phase_ticks, int max_phases, int n_blocks, int lds_bytes, int compute, int fm,
                        int threads, hipStream_t st);
// One workgroup size (instantiated in fused_b<BLK>.hip).
template <int BLK>
hipError_t launch_fused_blk(const FusedDesc *nets, const int32_t *order, void *const *outs, int64_t *stamps,
                            void *out1, int64_t *phase_ticks, int max_phases, int n_blocks, int lds_bytes, int compute,
                            int fm, hipStream_t st);

// Matrix-core GEMM C[b][m][n] = sum_k A[b][m][k] B[b][n][k] on packed,
// K-contiguous operands (mfma.hip).  tin: 0 f64, 1 f32, 2 bf16; tout: 0 f64,
// 1 f32.  FP32-accumulating inputs with tout == 0 add every `kchunk` K
// elements into FP64 accumulators.
// ksplit > 1 splits K into ksplit ranges (multiples of 64) whose partial
// products go to `part` ([ksplit][batch][M][N] of the output type) and are
// then summed in order into C.
hipError_t launch_gemm(const void *A, const void *B, void *C, int tin, int tout, int M, int N, int K, int batch,
                       int kchunk, int ksplit, void *part, hipStream_t st);

// Materialisation of fused-kernel inputs: each entry names a digit-form load
// descriptor (in a fused image) and the network's workspace.  grid.y =
// entries; max_size bounds the elements of any entry.
struct FPrepEntry {
    const int32_t *desc;
    void *ws;
    int32_t e0;       // first element of this entry's chunk of the load
    int32_t n_words;  // descriptor length: 7 + 2 ns + rank (4 + ns)
};
// Longest descriptor: 7 + 2 * 8 + 16 * (4 + 8) words.
constexpr int kFPrepDescMax = 215;
// Elements per FPrepEntry chunk (one wave each).
constexpr int kFPrepChunk = 4096;
// stamp (may be null): the device clock at the start of the first workgroup
// form: the longest load form among the entries (fprep_form): 0 when every
// entry has rank <= 4 and at most 4 CT scales, 1 when rank <= 6 and at most
// 6 scales, 2 otherwise.  Each form has a kernel of its own, unrolled to its
// bounds only: the shorter forms need fewer registers (50, 69, 88), so
// more waves stay resident per SIMD (8, 7, 5).
hipError_t launch_fprep(const FPrepEntry *entries, int n_entries, int form, int max_size, int compute,
                        int64_t *stamp, hipStream_t st);
// The form (as above) of one load: rank and number of CT scales.
inline int fprep_form(int rank, int n_scales) {
    if (rank <= 4 && n_scales <= 4) return 0;
    if (rank <= 6 && n_scales <= 6) return 1;
    return 2;
}

// QT evaluator (qteval.hip): statevector instances, one workgroup each.
constexpr int kSvMaxQubits = 24;
constexpr int kSvLdsQubits = 12;  // states of at most this many qubits live in LDS
enum SvKind { SV_U1 = 0, SV_CZ = 1, SV_CX = 2, SV_RZZ = 3, SV_PROJ = 4 };
struct SvOp {
    int32_t kind, q0, q1, pad;  // PROJ: q1 = the bit kept
    double m[8];                // U1: u00, u01, u10, u11 as (re, im); RZZ: m[0] = theta
};
struct SvInst {
    int32_t n, n_ops, n_kept, n_y;  // n_y: qubits measured in Y
    int64_t op_off;                 // first op
    int64_t out_off;                // first output (2^n_kept of them)
    int64_t state_off;              // offset (amplitudes) in the global state buffer; -1: LDS
    int64_t xmask, zymask;          // amplitude-index bits of X|Y qubits and of Z|Y qubits
    int32_t kept[kSvMaxQubits];
    double init[kSvMaxQubits][4];   // (re0, im0, re1, im1) per qubit
};
hipError_t launch_sv_eval(const SvInst *insts, int n_insts, const SvOp *ops, double2 *gstate, double *outs,
                          hipStream_t st);
hipError_t launch_qt_assemble(const int64_t *start, const int64_t *term_out, const double *coef, int64_t n_entries,
                              const double *outs, double *entries, hipStream_t st);

// Persistent work queue (queue.hip).  Items are the units of a network's
// per-step plan: an input materialisation (LOAD), a table-driven step or an
// operand pack (STEP; with split sums its partials), the second pass of a
// split sum (FINISH), a matrix-core product (GEMM) and the sum of its split-K
// partial products (KSUM).  An item is cut into tasks of units_per_task
// units (LOAD and KSUM: 256 elements; STEP: one 256-thread block of the
// per-step kernel's grid; FINISH: 4 outputs; GEMM: one output tile).
enum QItemKind { QI_LOAD = 0, QI_STEP = 1, QI_FINISH = 2, QI_GEMM = 3, QI_KSUM = 4 };
enum QItemFlags { QF_FIRST = 1, QF_LAST = 2, QF_OUT = 4 };
struct QItem {
    int32_t kind;
    int32_t ta, tb, tc;     // dtype codes: operands and result (GEMM: ta packed inputs)
    int32_t comp, unary;    // Neumaier-compensated FP64 result; single-operand step
    int32_t dep0, dep1;     // items whose tasks must all be done first (-1: none)
    int32_t net;            // batch index of the network
    int32_t flags;          // QF_FIRST: the network's first item (start stamp); QF_LAST:
                            // completes it (end stamp); QF_OUT: C is outs[net]
    int32_t units_per_task;
    int32_t n_tasks;
    int64_t n_units;
    const void *A, *B;      // operands (LOAD: unused; KSUM: partial products in A)
    void *C;                // result
    const int2 *tab;        // the network's offset tables
    const PrepDesc *prep;   // LOAD: the materialisation descriptor (dst_off unused)
    StepArgs s;             // STEP and FINISH geometry
    int32_t M, N, K, batch, kchunk, ksplit, kper, tiles_m, tiles_n;  // GEMM; KSUM: ksplit
    int64_t total;          // KSUM: elements of one partial product
};
struct QTask {
    int32_t item, task;
};
// Control words of a queue: error flag, exited workgroups, then the next
// task of each sub-queue.  ctrl[QC_ERR]: 1 a task gave up waiting for a
// dependency, 2 a sub-queue was left with tasks nobody took.
enum { QC_ERR = 0, QC_EXITED = 1, QC_NEXT = 2, QC_MAX_SUB = 16, QC_WORDS = QC_NEXT + QC_MAX_SUB };
// qinfo: [xcc] sub-queue of the workgroups on XCD xcc (-1: none), for
// xcc < QC_MAX_SUB; then QC_MAX_SUB + 1 task offsets (sub-queue k holds
// tasks [qinfo[QC_MAX_SUB + k], qinfo[QC_MAX_SUB + k + 1])).
constexpr int kQInfoWords = 2 * QC_MAX_SUB + 1;
// Bit x set: some workgroup of a wide probe launch (4096 workgroups) ran on
// XCD x (hardware XCC id, x < QC_MAX_SUB).  d_word: one device word of
// scratch.  0 on failure.
uint32_t queue_xcc_mask(uint32_t *d_word);
// GEMM kind of a queue kernel for packed inputs of dtype tin and results of
// dtype tout (1..5; -1: no such product), its dynamic LDS bytes, and the
// resident workgroups per compute unit of the queue kernel of kind gk
// (0: no GEMM items).
int queue_gemm_kind(int tin, int tout);
int queue_gemm_lds(int gk);
int queue_tile_rows();  // output rows of a queue GEMM tile (columns: 128)
int queue_blocks_per_cu(int gk, int lds_bytes);
// Runs the queue in one launch of n_blocks workgroups; each takes tasks from
// the sub-queue of the XCD it runs on.  counters[i] must hold
// items[i].n_tasks and the ctrl words after QC_ERR zero at launch; the
// last workgroup to finish restores them, so the next launch starts clean.
// stamps (optional): [2 net] start, [2 net + 1] end of each network, device
// clock; run_start (optional): clock at the start of the launch.  gk: the
// GEMM kind of every GEMM item (0 if there are none).
hipError_t launch_queue(const QItem *items, const QTask *tasks, const int32_t *qinfo, int n_sub, const int32_t *init,
                        int32_t *counters, int n_items, int32_t *ctrl, void *const *outs, int64_t *stamps,
                        int64_t *run_start, int gk, int lds_bytes, int n_blocks, hipStream_t st);

// Fold chain: a value X contracted with small matrices one mode at a time.
// X's labels split into in-tile axes (every folded axis, plus carried axes
// while the tile stays small; first slowest) and outer axes (first
// slowest).  A workgroup takes tf consecutive outer indices, stages X's
// in-tile sub-tensor for each in LDS, applies the folds in order (stage i
// contracts in-tile axis fold_ax[i] with matrix m[i]: row = the axis's
// current index, column = its new index, strides m_in / m_out), and writes
// the result in the destination's layout.
constexpr int kFoldAxes = 8, kFoldOuter = 4, kFoldStages = 8;
struct FoldDesc {
    int32_t n_ax, n_outer, n_stage, tf, d_max, lds_bytes;
    int32_t lg_tf;                 // tf = 2^lg_tf
    // index tables (built on the host): tab + t_src: source offset of each
    // in-tile index; tab + t_dst: destination offset of each final in-tile
    // index; tab + t_base[i], tab + t_mid[i]: for stage i and each output
    // index, the tile index of its first input term and its new digit
    const int32_t *tab;
    int32_t t_src, t_dst, d_final;
    int32_t t_base[kFoldStages], t_mid[kFoldStages], d_in_ax[kFoldStages], inner[kFoldStages], d_out[kFoldStages];
    int32_t ext0[kFoldAxes], ext1[kFoldAxes];  // in-tile extents at the source / destination
    int64_t s_src[kFoldAxes], s_dst[kFoldAxes];
    int32_t fold_ax[kFoldStages], fold_ext[kFoldStages];  // axis and its new extent, per stage
    int32_t m_in[kFoldStages], m_out[kFoldStages];
    const void *m[kFoldStages];
    int32_t o_ext[kFoldOuter];
    int64_t o_src[kFoldOuter], o_dst[kFoldOuter];
    int64_t n_outer_total;
};
// Chains of one launch: the workgroups of chain c are [blk0[c], blk0[c+1])
// (multiples of 8, so every chain keeps the XCD-aware tile order).
constexpr int kFoldBatch = 2;
struct FoldBatch {
    FoldDesc fd[kFoldBatch];
    const void *src[kFoldBatch];
    void *dst[kFoldBatch];
    int32_t blk0[kFoldBatch + 1];
    int32_t n;
};
struct FoldJob {
    const void *src;
    int ts;  // source dtype
    void *dst;
    const FoldDesc *fd;
};
// n independent chains, side by side in as few launches as possible
// (kFoldBatch per launch).  tm: matrix dtype, ti: arithmetic (0 double,
// 1 float), to: destination dtype of every chain.
hipError_t launch_folds(const FoldJob *jobs, int n, int tm, int ti, int to, hipStream_t st);

// Sum of the slices of a sliced network: out[e] = sum_k parts[k * n + e]
// in FP64 (compensated when comp), k in order; tout 0 f64, 1 f32.
hipError_t launch_slice_sum(const void *parts, int n_slices, int64_t n, void *out, int tout, bool comp,
                            hipStream_t st);

// Writes the device's constant 100 MHz clock to *dst when the launch runs.
hipError_t launch_stamp(int64_t *dst, hipStream_t st);

// Element-wise dtype conversion on the device.
hipError_t launch_convert(const void *src, int ts, void *dst, int td, int64_t n, hipStream_t st);

// Truncation gather (qpd.hip).  Item i copies its n_out (< 2^31) output
// elements; axis a of the item reads maps[map_off + moff[a] + d] (kept
// index d of the axis times its input stride).  A block covers either a
// run of whole items (n_items >= 1, at most 1024 elements together, item
// k's elements at block positions [start_k, start_k + n_out_k)) or one
// 1024-element chunk of a larger item (n_items == 1, elements from base).
constexpr int kTruncMaxRank = 16;
constexpr int kTruncThreads = 256;
constexpr int kTruncPerThread = 4;
constexpr int kTruncBlockElems = kTruncThreads * kTruncPerThread;
struct TruncItem {
    const void *src;
    void *dst;
    int64_t n_out;
    int64_t map_off;
    int32_t rank;
    int32_t start;
    int32_t odim[kTruncMaxRank];
    int32_t moff[kTruncMaxRank];
};
// A block stages its items (at most kTruncBlockItems) and, when they fit in
// kTruncMapLds entries (map_words > 0), their maps
// [map_base, map_base + map_words) in LDS.
constexpr int kTruncBlockItems = 32;
constexpr int kTruncMapLds = 1024;
struct TruncBlock {
    int32_t item0;
    int32_t n_items;
    int64_t base;
    int64_t map_base;
    int32_t map_words;
    int32_t pad;
};
hipError_t launch_truncate(const TruncItem *items, const TruncBlock *blocks, int64_t n_blocks, const int64_t *maps,
                           int elem_bytes, hipStream_t st);

// Cost-model MLP (mlp.hip).  Samples are rows of x ([.][HTN_MODEL_FEATURES]);
// idx (optional) maps batch position s to its row.  z1, z2, d1, d2 are
// [n][HTN_MODEL_HIDDEN] work arrays; forward keeps pre-activations in
// z1/z2 when they are non-null.  backward writes d(loss)/d(params) to grad
// and, when loss is non-null, the batch's mean squared error.
int64_t model_param_count();
hipError_t launch_mlp_forward(const float *prm, const float *x, const int32_t *idx, int n, float *y, float *z1,
                              float *z2, hipStream_t st);
hipError_t launch_mlp_backward(const float *prm, const float *x, const float *t, const int32_t *idx, int n,
                               const float *y, const float *z1, const float *z2, float *d1, float *d2, float *dy,
                               float *grad, float *loss, hipStream_t st);
// One Adam step (b1 0.9, b2 0.999, eps 1e-8); step counts from 1.
hipError_t launch_adam(float *p, float *m, float *v, const float *g, float lr, int64_t step, hipStream_t st);

}  // namespace kern
}  // namespace htn
