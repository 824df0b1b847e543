/*
 * htn.h — contraction of hybrid tensor networks (h-TNs) on AMD Instinct
 * MI355X (gfx950).
 *
 * What is computed.  Circuit knitting reconstructs an expectation value as
 * the sum, over every combination of QPD terms of every cut, of the
 * coefficient product times the product of the subcircuit results
 * (Sec. 2.1, Eq. knitting).  Writing the subcircuit results as quantum
 * tensors (QTs) and the QPD coefficients as classical tensors (CTs) joined
 * by shared indices turns that sum into the contraction of one tensor
 * network (Sec. 4.1, hybrid circuit contraction); contracting it pairwise
 * along a good order gives the same value at a far lower cost (Sec. 4.2).
 * With open output labels the same contraction yields a marginal
 * distribution.  This library performs that contraction (the runtime's
 * Step 4, Sec. 6.1) with hand-written HIP kernels.
 *
 * Index semantics (Sec. 2.2, tensor networks with hyper-indices).  Every
 * tensor mode carries an integer label in [0, n_labels).  A label carried
 * by several tensors is ONE index, summed exactly once (a hyperedge: a CT
 * and the two QTs it joins).  A label that is not an output label is summed;
 * it is summed in the first pairwise step after which no remaining tensor
 * carries it.  All tensors are dense, row-major, last mode fastest.
 *
 * Cost unit.  A pairwise step costs one multiplication per element of the
 * joint index space of its two operands (the product of the extents of the
 * union of their labels), the paper's postprocessing FLOP count
 * (Sec. 2.1, Sec. 4.2).  GFLOP/s figures count 2 flops per multiplication.
 *
 * Conventions for every function below:
 *   - Every call returns an htn_status; HTN_OK is 0.  On failure no state
 *     changes and htn_last_error() returns a message for the calling thread.
 *   - Structural errors (labels, shapes, paths) are detected on the host
 *     before anything is enqueued.  Faults raised by device work surface as
 *     HTN_E_DEVICE at a later call or at stream synchronisation.
 *   - NaN and Inf inputs propagate into the result; they are not errors.
 *   - A net is not thread-safe; distinct nets are independent.
 *   - hip_stream arguments are hipStream_t values passed as void*; NULL
 *     means the default stream of the current device.
 */
#ifndef HTN_H
#define HTN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct htn_net *htn_net_t;
typedef struct htn_batch *htn_batch_t;

typedef enum {
    HTN_OK = 0,
    HTN_E_ARG = 1,         /* NULL pointer, bad count, bad enum value      */
    HTN_E_LABEL = 2,       /* label out of range, repeated in one tensor,
                              output label carried by no tensor          */
    HTN_E_SHAPE = 3,       /* non-positive extent, size overflow         */
    HTN_E_PATH = 4,        /* SSA path malformed or not a full contraction */
    HTN_E_OOM = 5,         /* host/device allocation failed, or a peak
                              intermediate above the configured cap      */
    HTN_E_DEVICE = 6,      /* HIP runtime error                          */
    HTN_E_UNSUPPORTED = 7, /* valid request the library does not support  */
    HTN_E_STATE = 8        /* call out of order (e.g. no device data)    */
} htn_status;

/* Element types.  HTN_F64/HTN_F32 are IEEE binary64/binary32; HTN_BF16 is
 * bfloat16 (the upper 16 bits of a binary32), rounded to nearest-even.    */
typedef enum { HTN_F64 = 0, HTN_F32 = 1, HTN_BF16 = 2 } htn_dtype;

/* How the final contraction step accumulates.
 *   HTN_SUM_PLAIN        in the compute accumulator (FP64 for HTN_F64,
 *                        FP32 otherwise); output dtype = intermediate dtype
 *                        (FP64 for HTN_F64, FP32 for HTN_F32/HTN_BF16).
 *   HTN_SUM_FP64         products and sums of the last step in FP64;
 *                        output FP64.
 *   HTN_SUM_COMPENSATED  as HTN_SUM_FP64 with Neumaier-compensated sums and
 *                        TwoSum combination of partial sums; output FP64.
 * The final signed sum over QPD terms (weights +-1/2, gamma = 3 per CZ cut)
 * is where cancellation concentrates, so it may run in FP64 even when
 * every earlier step ran in FP32 or BF16.                                  */
typedef enum { HTN_SUM_PLAIN = 0, HTN_SUM_FP64 = 1, HTN_SUM_COMPENSATED = 2 } htn_final_sum;

/* Execution strategy for htn_contract.
 *   HTN_EXEC_AUTO   fused when the whole network fits on chip, else steps.
 *   HTN_EXEC_STEPS  one kernel launch per pairwise step (plus one launch
 *                   that applies absorbed coefficient vectors), every
 *                   intermediate in device memory.
 *   HTN_EXEC_FUSED  one workgroup contracts the whole network with every
 *                   operand in LDS; HTN_E_UNSUPPORTED if it does not fit.  */
typedef enum { HTN_EXEC_AUTO = 0, HTN_EXEC_STEPS = 1, HTN_EXEC_FUSED = 2 } htn_exec_mode;

/* Path selectors for htn_set_path's n_steps argument. */
#define HTN_PATH_GREEDY (-1)
#define HTN_PATH_LEARNED (-2)
#define HTN_PATH_SAMPLED (-3)

/* ---------------------------------------------------------------------
 * htn_create — build a net from tensors and labels.
 *
 *   out           receives the handle (set to NULL on failure).
 *   n_tensors     >= 1.
 *   ranks         [n_tensors], each >= 1.
 *   labels        concatenation of ranks[i] labels per tensor, each in
 *                 [0, n_labels), no label twice in one tensor.
 *   n_labels      number of label ids; label_dims[n_labels] extents >= 1.
 *   data          [n_tensors] pointers to row-major tensors of dtype
 *                 `storage`.  data_on_device = 0: host memory, copied into
 *                 net-owned device memory at the first contraction (the
 *                 caller may free it when htn_create returns).
 *                 data_on_device = 1: device memory on the current device,
 *                 borrowed — it must stay valid and unchanged in layout for
 *                 the life of the net; when `storage` differs from the
 *                 compute element type a converted device copy is made.
 *   n_out, out_labels  ordered output labels (n_out = 0: scalar).  Each
 *                 must be carried by at least one tensor.
 *   storage       dtype of `data` (HTN_F64, HTN_F32 or HTN_BF16).
 *   compute       HTN_F64: FP64 inputs, intermediates, accumulation.
 *                 HTN_F32: FP32 inputs, intermediates, accumulation.
 *                 HTN_BF16: BF16 inputs (round-to-nearest-even from
 *                 `storage`), FP32 intermediates and accumulation; operands
 *                 of matrix-core steps enter as BF16.
 *   final_sum     see htn_final_sum.
 * The default path is FLOP-greedy (as after htn_set_path(net, -1, NULL)).
 * ------------------------------------------------------------------- */
htn_status htn_create(htn_net_t *out, int32_t n_tensors, const int32_t *ranks,
                      const int32_t *labels, int32_t n_labels, const int64_t *label_dims,
                      const void *const *data, int32_t data_on_device, int32_t n_out,
                      const int32_t *out_labels, htn_dtype storage, htn_dtype compute,
                      htn_final_sum final_sum);

/* ---------------------------------------------------------------------
 * htn_set_path — choose the pairwise contraction order (Sec. 4.2: the cost
 * depends heavily on the order; Sec. 6.1 Step 3).
 *
 *   n_steps >= 0  explicit SSA path: ssa_pairs[2*t], ssa_pairs[2*t+1] are
 *                 the ids contracted by step t; inputs are ids
 *                 0..n_tensors-1 and step t creates id n_tensors+t.  Every
 *                 id is consumed exactly once and the last step's result
 *                 is the network's value, so n_steps == n_tensors - 1.
 *                 Pairs without a shared label are outer products.
 *   HTN_PATH_GREEDY   FLOP-greedy: repeatedly contract the pair, among
 *                 pairs sharing a label, with the fewest multiplications;
 *                 ties go to the smaller result, then to the lower ids;
 *                 disconnected parts are joined last, smallest first.
 *   HTN_PATH_SAMPLED  the cheapest (by multiplications) of the FLOP-greedy
 *                 path and HTN_OPT_PATH_SAMPLES Boltzmann-sampled greedy
 *                 paths: at each step a sharing pair is drawn with weight
 *                 exp(-(log2 cost - log2 min cost) / T), T cycling through
 *                 0.25, 0.5, 1, 2; deterministic for a given
 *                 HTN_OPT_PATH_SEED.  Never costlier than FLOP-greedy.
 *   HTN_PATH_LEARNED  among the candidates (FLOP-greedy plus the sampled
 *                 paths) within twice the fewest multiplications, the one
 *                 with the lowest total time predicted by the net's cost
 *                 model (htn_set_model); FLOP-greedy when the net has no
 *                 model, and on ties.  Runs the model on the current device
 *                 and waits for it.
 * Errors: HTN_E_PATH for a malformed path; HTN_E_OOM if an intermediate
 * exceeds the size cap (htn_set_option HTN_OPT_MAX_INTERMEDIATE).
 * ------------------------------------------------------------------- */
htn_status htn_set_path(htn_net_t net, int32_t n_steps, const int32_t *ssa_pairs);

/* htn_get_path — the current path.  *n_steps receives its length; if
 * ssa_pairs is non-NULL, min(capacity, n_steps) pairs are written.  If
 * mults is non-NULL it receives the path's multiplication count.        */
htn_status htn_get_path(htn_net_t net, int32_t *n_steps, int32_t *ssa_pairs, int32_t capacity,
                        double *mults);

/* Options (htn_set_option). */
typedef enum {
    HTN_OPT_EXEC = 0,              /* htn_exec_mode                            */
    HTN_OPT_MAX_INTERMEDIATE = 1,  /* cap on intermediate elements (default 2^31-1) */
    HTN_OPT_FUSED_LDS_BYTES = 2,   /* LDS budget of the fused kernel (default 65536) */
    HTN_OPT_MFMA = 3,              /* 1: allow matrix cores (default): GEMM steps of the per-step
                                      executor, 16x16-block tiled steps of the fused kernel;
                                      0: VALU only */
    HTN_OPT_PATH_SAMPLES = 4,      /* sampled candidates of HTN_PATH_SAMPLED/LEARNED (default 32) */
    HTN_OPT_PATH_SEED = 5,         /* seed of the path sampler (default 0) */
    HTN_OPT_FUSED_THREADS = 6,     /* threads per network in the fused kernel: 64, 256 (default) or 512 */
    HTN_OPT_SLICE = 7,             /* 0 (default): a path whose largest intermediate exceeds
                                      HTN_OPT_MAX_INTERMEDIATE is HTN_E_OOM.  1: slicing (see below) */
    HTN_OPT_QUEUE = 8              /* batches: 0 (default) a net run step by step goes to the batch's
                                      work queue if its kernel steps are small (mean below 2^19
                                      multiplications), else one launch per step; 1 the net always
                                      goes to the queue (even one the fused kernel could take);
                                      2 never (one launch per step, on side streams) */
} htn_option;

/* Slicing under the intermediate cap (HTN_OPT_SLICE = 1).  Contraction
 * orders are chosen by cost (Sec. 4.2; Sec. 6.1 Step 3 uses hyper-optimised
 * search, which slices); when the largest intermediate of the net's path
 * (every step's result) exceeds HTN_OPT_MAX_INTERMEDIATE, summed labels are
 * fixed one at a time -- each time the one that leaves the smallest largest
 * intermediate (fewer slices, then the lower label id, on ties) -- until the
 * path fits; at most 65536 slices, else HTN_E_OOM.  A slice is the network
 * with those labels fixed to one value each; htn_contract cuts every
 * input's slices out of its device copy (one gather launch), contracts the
 * slices as one batch (same path, each slice a network of its own) and
 * sums their results in FP64 (compensated under HTN_SUM_COMPENSATED) in
 * slice order.  htn_info.mults counts every slice, htn_info.peak_elements
 * is one slice's largest intermediate, htn_info.n_slices the slice count.
 * A sliced net cannot join a batch (htn_batch_create: HTN_E_UNSUPPORTED) or
 * htn_contract_noalloc.  htn_get_slicing lists the sliced labels (in slice
 * order: the first slowest).                                              */

htn_status htn_set_option(htn_net_t net, htn_option opt, int64_t value);

/* Summary of a planned net. */
typedef struct {
    int64_t out_elements;   /* elements of the result                        */
    int32_t out_dtype;      /* htn_dtype of the result                       */
    int32_t n_steps;        /* path length                                   */
    int32_t n_kernel_steps; /* steps executed as kernels (not absorbed)      */
    int32_t n_absorbed;     /* coefficient tensors folded into operand loads */
    int32_t fused_ok;       /* 1 if the whole net fits the fused kernel      */
    int32_t fused_lds_bytes;/* LDS the fused kernel needs                    */
    double mults;           /* multiplications along the path                */
    double peak_elements;   /* largest intermediate                          */
    int64_t workspace_bytes;/* device workspace of the per-step executor     */
    int64_t input_bytes;    /* bytes of the inputs in compute storage        */
    int64_t n_slices;       /* slices contracted (1: not sliced)             */
} htn_info;

htn_status htn_get_info(htn_net_t net, htn_info *info);

/* htn_get_slicing — the sliced labels of the current plan: *n_labels
 * receives their count, labels (if non-NULL) the first min(capacity,
 * *n_labels) of them, *n_slices (if non-NULL) the number of slices.     */
htn_status htn_get_slicing(htn_net_t net, int32_t *n_labels, int32_t *labels, int32_t capacity, int64_t *n_slices);

/* ---------------------------------------------------------------------
 * htn_contract — contract the net into out_device (caller-owned device
 * memory of info.out_elements elements of info.out_dtype, laid out
 * row-major over out_labels).  Asynchronous on hip_stream.  The first call
 * uploads host data and allocates the net's workspace (synchronously).
 * ------------------------------------------------------------------- */
htn_status htn_contract(htn_net_t net, void *out_device, void *hip_stream);

/* htn_contract_batch — contract n independent nets, outs[i] receiving net
 * i's result, with as few launches as possible: every net that fits the
 * fused kernel runs in one launch (one workgroup per net, heaviest first).
 * The others, and fused-capable nets whose work exceeds
 * max(2^20, 4 x the batch's fused work per resident workgroup slot) (they
 * would hold one workgroup long after the rest finish), run step by step
 * on up to three side streams forked from and joined back to hip_stream,
 * overlapping the fused launch.  Equivalent to htn_batch_create +
 * htn_batch_run + htn_batch_destroy.                                      */
htn_status htn_contract_batch(int32_t n, const htn_net_t *nets, void *const *outs, void *hip_stream);

/* Reusable batch: plans the combined launch once.  The nets must outlive
 * the batch and keep their paths.  htn_batch_run may capture its launches
 * in a HIP graph (htn_batch_set_graph) and replay it on later calls with
 * the same outs.
 * htn_batch_set_graph: use_graph 0 runs eagerly; 1 makes the next run on a
 * non-NULL stream run eagerly once and capture a graph, replayed by later
 * runs with the same outs and stream.  If the capture fails (the stream
 * cannot be captured, a launch is refused while capturing, the graph does
 * not instantiate), the stream is taken out of capture mode, the partial
 * graph is freed and every later run is eager; the run that tried still
 * computed its results.  HTN_GRAPH_FORCE_FAILURE behaves as 1 but fails the
 * capture on purpose after recording, so callers can test that path.
 * htn_batch_graph_state: *state = 0 (eager: graphs off or not yet
 * captured), 1 (a captured graph is replayed) or 2 (a capture failed: eager
 * from then on; htn_last_error() then describes the failure).             */
#define HTN_GRAPH_FORCE_FAILURE 2
htn_status htn_batch_create(htn_batch_t *out, int32_t n, const htn_net_t *nets);
htn_status htn_batch_set_graph(htn_batch_t batch, int32_t use_graph);
htn_status htn_batch_graph_state(htn_batch_t batch, int32_t *state);
htn_status htn_batch_run(htn_batch_t batch, void *const *outs, void *hip_stream);
/* Per-net start and completion times of the last run: ticks[2*i] and
 * ticks[2*i+1], in ticks of the device's constant 100 MHz clock counted
 * from the start of the run (a clock read enqueued ahead of the run's
 * kernels).  Fused nets are stamped by their workgroup, nets run step by
 * step by clock reads around their kernels.  ticks holds 2*n values.
 * Synchronise the stream of the run first.                                */
htn_status htn_batch_timestamps(htn_batch_t batch, int64_t *ticks);
/* Per-phase timing.  A fused network runs as a sequence of phases
 * separated by workgroup barriers (phase 0 loads the operands of the first
 * steps; each later phase runs the kernel steps whose operands are ready,
 * side by side on their own waves, and loads the operands of the next).
 * With max_phases > 0 every run records, for each fused net and each of its
 * first max_phases phases, the clock at the end of the phase; for a net run
 * step by step, the clock after each of its first max_phases kernel steps
 * (a clock read enqueued after the step's launches).
 * htn_batch_phase_times writes n * max_phases values ([net][phase or
 * step], 100 MHz ticks counted from the start of the run; -1 for entries
 * not recorded).  Set before a graph is captured.                         */
htn_status htn_batch_set_phase_timing(htn_batch_t batch, int32_t max_phases);
htn_status htn_batch_phase_times(htn_batch_t batch, int64_t *ticks);
/* Launch timing with HIP events.  With htn_batch_set_event_timing(batch, 1)
 * every eager htn_batch_run (not graph replays) records events on its
 * stream around the input-materialisation launch and around the fused
 * launch.  htn_batch_launch_ms waits for them and returns the mean
 * durations (milliseconds) over the runs since timing was switched on or
 * last read, and their count; then starts a new tally.  Any argument but
 * the batch may be NULL.                                                  */
htn_status htn_batch_set_event_timing(htn_batch_t batch, int32_t on);
/* Work queue of a batch (Sec. 6.1 Step 4 contracts a network step by step;
 * a batch runs the steps of all its step-by-step networks in one launch).
 * Networks too large for one fused workgroup (HTN_OPT_QUEUE, above) have
 * their input materialisations and every block of every step cut into
 * tasks, listed in dependency order; each network is assigned to one XCD
 * (heaviest first, to the least loaded), and the resident workgroups of
 * one persistent launch take the tasks of their own XCD in list order, each
 * waiting (bounded) until the steps it reads are complete.  Each network's intermediates get
 * their own device buffer for the batch's lifetime (no reuse between
 * steps), allocated at htn_batch_create.  A network whose matrix-core
 * steps use another input/output type pair than the first such network's,
 * and every step-by-step network while phase timing is on, runs with one
 * launch per step instead.  Runs of one batch must not overlap.
 * htn_batch_queue_info (waits for the device): *n_nets networks and
 * *n_tasks tasks in the queue; *error = 1 if a task of any run since the
 * last call gave up waiting, 2 if some XCD's tasks were left untaken
 * (neither happens for a consistent queue; the flag is then cleared).
 * Any pointer may be NULL.                                     */
htn_status htn_batch_queue_info(htn_batch_t batch, int32_t *n_nets, int32_t *n_tasks, int32_t *error);
htn_status htn_batch_launch_ms(htn_batch_t batch, float *prep_ms, float *fused_ms, int32_t *runs);
void htn_batch_destroy(htn_batch_t batch);

/* ---------------------------------------------------------------------
 * Learned cost model (HTN_PATH_LEARNED).
 *
 * The paper chooses contraction orders with a hyper-optimised search over
 * a FLOP objective (Sec. 4.2; Sec. 6.1, Step 3).  FLOPs are a poor proxy
 * for time on a GPU when networks are small: a step's duration depends on
 * its kernel class, shape and where its operands live.  The model here
 * predicts the natural log of a kernel step's duration in microseconds
 * from HTN_MODEL_FEATURES features of the step (htn_step_features) with a
 * multilayer perceptron
 *     h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = w3 . h2 + b3,
 * HTN_MODEL_HIDDEN units per hidden layer, FP32 weights and arithmetic, all
 * on the GPU (forward, backward and Adam kernels).
 *
 * Parameter layout (htn_model_param_count() floats, in this order):
 *     W1 [HIDDEN][FEATURES] (row = hidden unit), b1 [HIDDEN],
 *     W2 [HIDDEN][HIDDEN], b2 [HIDDEN], w3 [HIDDEN], b3 [1].
 * Training minimises the mean squared error (1/n) sum (y_s - t_s)^2 of the
 * predictions y_s against targets t_s (log microseconds) with Adam
 * (b1 = 0.9, b2 = 0.999, eps = 1e-8).
 *
 * Step features (row of HTN_MODEL_FEATURES floats; "lg" = log2(v) / 8):
 *   0 lg(1 + multiplications)  1 lg(outputs)  2 lg(summed terms per output)
 *   3 lg(size of operand A)    4 lg(size of operand B; 1 if unary)
 *   5-7 lg(M), lg(N), lg(K) of a register-tiled step (0 otherwise)
 *   8 lg(outputs per thread of a VALU-tiled step)   9 lg(lanes per output)
 *   10 tiled step  11 one lane per output  12 several lanes per output
 *   13 whole workgroup per output  14 matrix cores (GEMM step or
 *   matrix-core tiled step)  15 unary step
 *   16 final step  17-19 operand A / operand B / result outside LDS
 *   20 lg(1 + 16-byte chunks the fused kernel copies during the step)
 *   21 fused executor  22 FP64 compute  23 element bytes / 8
 *   24 lg(threads running the step)  25 steps sharing its phase / 8
 * A candidate's predicted time sums, over the fused kernel's phases, the
 * largest exp(y) among the phase's steps (they run side by side), and over
 * the per-step executor's steps their exp(y).
 * ------------------------------------------------------------------- */
#define HTN_MODEL_FEATURES 26
#define HTN_MODEL_HIDDEN 64
typedef struct htn_model *htn_model_t;

int64_t htn_model_param_count(void);
/* htn_model_create — a model on the current device with weights drawn
 * uniformly from +-sqrt(6 / fan_in) (seeded splitmix64), zero biases and
 * zero Adam state.                                                        */
htn_status htn_model_create(htn_model_t *out, uint64_t seed);
/* Host copies of the parameters (htn_model_param_count() floats).  Setting
 * parameters clears the Adam state.                                       */
htn_status htn_model_set_params(htn_model_t model, const float *params);
htn_status htn_model_get_params(htn_model_t model, float *params);
/* htn_model_forward — y[s] for the n rows of x; x [n][FEATURES] and y [n]
 * are device arrays.  Asynchronous on hip_stream.                         */
htn_status htn_model_forward(htn_model_t model, int32_t n, const float *x, float *y, void *hip_stream);
/* htn_model_gradients — on device arrays: grad (param_count floats)
 * receives the gradient of the mean squared error of the n rows of x
 * against t [n], loss (1 float, may be NULL) the error itself.  No update
 * is made.  Asynchronous on hip_stream.                                   */
htn_status htn_model_gradients(htn_model_t model, int32_t n, const float *x, const float *t, float *grad,
                               float *loss, void *hip_stream);
/* htn_model_adam_step — one Adam update of the parameters with gradient
 * grad (device, param_count floats) and learning rate lr.               */
htn_status htn_model_adam_step(htn_model_t model, const float *grad, float lr, void *hip_stream);
/* htn_model_train — minibatch Adam on the n samples (device x [n][FEATURES],
 * t [n]) for `epochs` passes, each pass over a permutation of the samples
 * drawn from splitmix64(seed) in minibatches of `batch`.  epoch_loss
 * (host, `epochs` floats, may be NULL) receives each pass's mean minibatch
 * loss.  Synchronous.                                                     */
htn_status htn_model_train(htn_model_t model, int32_t n, const float *x, const float *t, int32_t epochs,
                           int32_t batch, float lr, uint64_t seed, float *epoch_loss, void *hip_stream);
void htn_model_destroy(htn_model_t model);

/* htn_set_model — the model HTN_PATH_LEARNED uses for this net (NULL: none).
 * The model is borrowed and must be alive at every later htn_set_path
 * call with HTN_PATH_LEARNED.                                             */
htn_status htn_set_model(htn_net_t net, htn_model_t model);

/* htn_step_features — features of the current plan's kernel steps, in
 * execution order, as rows of HTN_MODEL_FEATURES floats (host array).
 * *n_steps receives the number of kernel steps; min(capacity, n_steps)
 * rows are written.                                                       */
htn_status htn_step_features(htn_net_t net, float *features, int32_t capacity, int32_t *n_steps);

/* htn_batch_step_times — timing collector.  After a run with phase timing
 * on (htn_batch_set_phase_timing), the duration in microseconds of each
 * kernel step of each net: times[i * capacity + q] for net i and kernel
 * step q < capacity, NaN where the step was not recorded (steps beyond
 * max_phases).  A fused step's duration is that of its phase (its
 * arithmetic and the copies issued for the next phase); when independent
 * steps share a phase the duration is recorded for the one with the most
 * multiplications (the phase waits for the slowest) and NaN for the
 * others.  A step of a net that runs step by step in every batch (its
 * executor option, or a plan the fused kernel cannot take) lasts from the
 * previous step's clock read (the net's start stamp for the first step, so
 * it includes the net's input materialisation) to its own: its launches
 * and any gap between them.  Nets moved to the per-step executor only for
 * their size in this batch are not recorded (NaN): their step features
 * describe the fused executor.                                           */
htn_status htn_batch_step_times(htn_batch_t batch, float *times, int32_t capacity);

/* htn_autotune — pick the fused kernel's workgroup size and LDS budget for
 * a set of nets by measurement.  Each candidate (threads, LDS bytes) in
 *   (64, 32K) (64, 48K) (64, 64K) (256, 32K) (256, 48K) (256, 64K)
 *   (256, 96K) (256, 160K) (512, 64K) (512, 96K) (512, 160K)
 * is applied to every net (HTN_OPT_FUSED_THREADS / HTN_OPT_FUSED_LDS_BYTES,
 * which replans them on their current paths), the nets are run as one
 * batch (htn_batch_create/run) twice to warm up and five times timed with
 * HIP events on hip_stream, and the candidate with the lowest median time
 * is applied and left in place.  outs as for htn_contract_batch.
 * best_threads, best_lds_bytes and best_ms (median milliseconds) receive
 * the choice (each may be NULL).  Synchronous.  A candidate that fails to
 * plan or launch is skipped; if none runs the nets keep their previous
 * settings and HTN_E_UNSUPPORTED is returned.                             */
htn_status htn_autotune(int32_t n, const htn_net_t *nets, void *const *outs, void *hip_stream,
                        int32_t *best_threads, int32_t *best_lds_bytes, float *best_ms);

/* ---------------------------------------------------------------------
 * htn_set_allocator — device memory allocator of the library (process
 * wide): every device buffer it allocates from then on (net workspaces,
 * input copies, step tables and descriptors, batch and model buffers)
 * comes from alloc(bytes, ctx), which must return memory of at least
 * `bytes` bytes on the current device, aligned to 256 bytes, or NULL
 * (reported as HTN_E_OOM by the call that needed it).  A buffer is
 * released with the free routine of the allocator that made it, so the
 * allocator may be changed at any time; free(ptr, ctx) is called when the
 * library no longer uses ptr (after the caller has synchronised the
 * streams of work that used it, e.g. before htn_destroy).  This lets the
 * caller route the library's memory through its own pool (e.g. PyTorch's
 * caching allocator).  Both NULL: back to hipMalloc / hipFree.
 * Errors: HTN_E_ARG if exactly one of alloc and free_fn is NULL.
 * ------------------------------------------------------------------- */
typedef void *(*htn_alloc_fn)(size_t bytes, void *ctx);
typedef void (*htn_free_fn)(void *ptr, void *ctx);
htn_status htn_set_allocator(htn_alloc_fn alloc, htn_free_fn free_fn, void *ctx);

/* ---------------------------------------------------------------------
 * htn_contract_noalloc — htn_contract for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid hipMalloc.  It calls no hipMalloc, hipFree or other
 * allocating routine.
 *
 * It runs the per-step executor (as with HTN_EXEC_STEPS: one launch that
 * applies absorbed coefficient tensors, then one kernel sequence per
 * pairwise step) and writes the result to out_device (caller-owned device
 * memory, as for htn_contract), asynchronously on hip_stream.  The
 * executor's workspace (materialised inputs, intermediates, split-sum and
 * split-K partials) lives in a library-wide device array of
 * HTN_NOALLOC_SCRATCH_BYTES bytes.  Each device holds its own copy from
 * the library's load until the process ends.  The array is shared by every
 * call on that device and keeps the last call's contents.  Calls that
 * overlap on one device, on any streams, therefore race: serialise them.
 * No kernel of the executor needs the workspace cleared first.
 *
 * Preconditions: the net's device state (input copies, step tables, load
 * descriptors) has been set up on the current device by an htn_contract
 * call after the net's last htn_create, htn_set_path, htn_set_option or
 * htn_update_data.
 * Errors (all reported before anything is enqueued):
 *   HTN_E_ARG          NULL net or out_device.
 *   HTN_E_UNSUPPORTED  the net's per-step workspace (htn_info.workspace_bytes)
 *                      exceeds HTN_NOALLOC_SCRATCH_BYTES.
 *   HTN_E_STATE        the device state is missing or stale, or it lives on
 *                      another device.
 *   HTN_E_DEVICE       a HIP error while resolving the array's address
 *                      (first call on a device) or enqueueing.
 * ------------------------------------------------------------------- */
#define HTN_NOALLOC_SCRATCH_BYTES (64 * 1024 * 1024)
htn_status htn_contract_noalloc(htn_net_t net, void *out_device, void *hip_stream);

/* htn_update_data — replace the tensor values (same structure and path).
 * Same data / data_on_device semantics as htn_create.                     */
htn_status htn_update_data(htn_net_t net, const void *const *data, int32_t data_on_device);

void htn_destroy(htn_net_t net);

const char *htn_status_string(htn_status s);
const char *htn_last_error(void);

/* htn_plan_json — a JSON description of the current plan (steps, labels,
 * kernel classes, sizes) for tests and tools.  Writes at most `capacity`
 * bytes including the terminating NUL; *needed receives the full length
 * plus one.                                                               */
htn_status htn_plan_json(htn_net_t net, char *buf, int64_t capacity, int64_t *needed);

/* htn_plan_tables — the plan's offset-table arena (int32 pairs as laid out
 * on the device), for tools that check a plan on the host.  Same buffer
 * convention as htn_plan_json: writes min(capacity, size) int32 values;
 * *needed receives the arena length in int32 values.  Offsets named in
 * htn_plan_json ("t_*" fields) index pairs of this arena.                  */
htn_status htn_plan_tables(htn_net_t net, int32_t *buf, int64_t capacity, int64_t *needed);

/* ---------------------------------------------------------------------
 * QPD sampling and h-TN simplification (Sec. 4.3, Fig. 3 (d); Step 1 of
 * Sec. 6.1).  Each sampled coefficient tensor c (rank 1, length n) is drawn
 * s_qpd times on its own, index i with probability |c_i| / gamma,
 * gamma = sum |c_i|; indices drawn zero times are dropped from the CT and
 * from every QT carrying its label.  Wire-cut tensors are not sampled (all
 * their terms weigh the same): the caller leaves them out.
 *
 * htn_qpd_sample (host) — one CT's draws and estimator weights.
 *   coeffs[n]     the CT's coefficients (host, FP64, finite, not all 0).
 *   s_qpd >= 1    number of draws.
 *   uniforms[s_qpd]  host uniforms in [0, 1), one per draw (the caller's
 *                 random numbers): draw j goes to the first index i with
 *                 uniforms[j] < F_i, F_i = (|c_0| + ... + |c_i|) / gamma
 *                 accumulated left to right in FP64; a draw that rounding
 *                 puts past F_{n-1} goes to the last non-zero index.
 *   counts[n]     out: n_i, the draws of index i (they sum to s_qpd).
 *   weights[n]    out: the unbiased QPD estimator weight of index i,
 *                 n_i * gamma * sign(c_i) / s_qpd (0 where n_i = 0); its
 *                 expectation over the draws is c_i.
 * Errors: HTN_E_ARG for NULL pointers, n < 1, s_qpd < 1, a non-finite
 * coefficient, all coefficients 0 or a uniform outside [0, 1).
 * ------------------------------------------------------------------- */
htn_status htn_qpd_sample(int32_t n, const double *coeffs, int64_t s_qpd, const double *uniforms,
                          int64_t *counts, double *weights);

/* htn_truncation — one tensor to truncate (all pointers are the caller's).
 *   src           device, row-major (last axis fastest), extents dims[].
 *   dst           device, row-major, extent n_kept[a] on axis a (dims[a]
 *                 where kept[a] is NULL); must not overlap src.
 *   rank          1..HTN_TRUNC_MAX_RANK.
 *   kept[a]       host list of the n_kept[a] indices (each in [0, dims[a]),
 *                 in the order they take in dst) that axis a keeps; NULL
 *                 keeps the whole axis (n_kept[a] ignored).              */
#define HTN_TRUNC_MAX_RANK 16
typedef struct {
    const void *src;
    void *dst;
    int32_t rank;
    int64_t dims[HTN_TRUNC_MAX_RANK];
    const int32_t *kept[HTN_TRUNC_MAX_RANK];
    int32_t n_kept[HTN_TRUNC_MAX_RANK];
} htn_truncation;
typedef struct htn_trunc *htn_trunc_t;

/* htn_truncate_create — validate n >= 1 items of element type `dtype` and
 * upload their gather descriptors to the current device (synchronous).
 * The src/dst buffers are borrowed: they must stay allocated for the life
 * of the handle.  Errors: HTN_E_ARG (NULL pointers, bad rank or dtype,
 * n_kept < 1, an index out of range), HTN_E_UNSUPPORTED (an item with
 * 2^31 or more elements), HTN_E_OOM, HTN_E_DEVICE.
 * htn_truncate_run — enqueue the batch's gather (one kernel launch) on
 * hip_stream (NULL: the default stream); dst[o] = src[the element whose
 * index on each axis a is kept[a][o_a]].  Bit-exact copies.
 * htn_truncate_destroy — free the descriptors (NULL is ignored).         */
htn_status htn_truncate_create(htn_trunc_t *out, int32_t n, const htn_truncation *items, htn_dtype dtype);
htn_status htn_truncate_run(htn_trunc_t t, void *hip_stream);
void htn_truncate_destroy(htn_trunc_t t);

/* ---------------------------------------------------------------------
 * Fusion of the CTs between the same QTs before sampling (Sec. 4.3;
 * Step 1 of Sec. 6.1): the CTs on parallel cuts between two QTs become one
 * CT, their tensor product, on one fused index, and each QT carrying their
 * indices has those modes merged into that one mode.  The fused network
 * contracts to the same value; its fused CT is then sampled as a whole
 * (htn_qpd_sample), so pairs of terms are drawn jointly.
 *
 * htn_qpd_fuse (host) — fused[f] = coeffs[0][i_0] * ... * coeffs[n-1][i_{n-1}]
 * with f row-major over (i_0, ..., i_{n-1}) (i_0 slowest).
 *   n >= 1 tensors; dims[k] >= 1 their lengths; coeffs[k] host FP64 arrays;
 *   fused: host array of prod(dims) values (caller-owned).
 * Errors: HTN_E_ARG (NULL pointers, n < 1, a length < 1), HTN_E_UNSUPPORTED
 * (2^31 or more fused entries).
 * ------------------------------------------------------------------- */
htn_status htn_qpd_fuse(int32_t n, const int32_t *dims, const double *const *coeffs, double *fused);

/* htn_gather — one tensor to gather with merged (fused) axes and kept
 * indices, the QT side of the fusion and truncation (all pointers the
 * caller's).
 *   src, dst      device; src row-major with extents dims[0..rank-1]; dst
 *                 row-major over the output axes; must not overlap.
 *   rank          input rank, 1..HTN_TRUNC_MAX_RANK.
 *   out_rank      output rank, 1..rank.
 *   n_axes[o]     number of input axes merged into output axis o (>= 1;
 *                 they sum to rank).
 *   axes          the input axes, output axis by output axis (n_axes[0]
 *                 for axis 0, then axis 1's, ...): a permutation of
 *                 0..rank-1.  Output axis o's index is row-major over its
 *                 input axes in the order listed (the first slowest).
 *   kept[o]       host list of the n_kept[o] indices of output axis o that
 *                 dst keeps, in dst order (NULL: all of them).
 * dst[o_0, ..., o_{out_rank-1}] = src[the element whose merged index on
 * each output axis o is kept[o][o_o]].  Bit-exact copies.
 * htn_gather_create — validate n >= 1 items of element type dtype and
 * upload their gather descriptors (synchronous); the handle is run and
 * destroyed with htn_truncate_run / htn_truncate_destroy (one launch for
 * the batch).  Errors: HTN_E_ARG (NULL buffers, bad rank/out_rank/n_axes,
 * axes not a permutation, a kept index out of range), HTN_E_UNSUPPORTED
 * (an item or a merged axis with 2^31 or more elements), HTN_E_OOM,
 * HTN_E_DEVICE.                                                           */
typedef struct {
    const void *src;
    void *dst;
    int32_t rank;
    int64_t dims[HTN_TRUNC_MAX_RANK];
    int32_t out_rank;
    int32_t n_axes[HTN_TRUNC_MAX_RANK];
    int32_t axes[HTN_TRUNC_MAX_RANK];
    const int32_t *kept[HTN_TRUNC_MAX_RANK];
    int32_t n_kept[HTN_TRUNC_MAX_RANK];
} htn_gather;
htn_status htn_gather_create(htn_trunc_t *out, int32_t n, const htn_gather *items, htn_dtype dtype);

/* ---------------------------------------------------------------------
 * QT evaluator (Sec. 6.2; Step 2 of Sec. 6.1): exact statevector
 * simulation of subcircuit instances on the GPU, and the assembly of
 * quantum-tensor entries from their results.  A QT entry is a signed
 * combination of instance results (one instance per QPD term of the cuts
 * it touches; a signed mid-circuit Z measurement is two instances, one per
 * projection, entering with signs +1 and -1; a Pauli operator injected at a
 * cut is the signed sum of two eigenstate preparations).
 *
 * An instance: n_qubits (1..HTN_SV_MAX_QUBITS) in a product state
 * (init[4q..4q+3] = re, im of <0|q>, re, im of <1|q>, host FP64), then
 * n_ops ops in order, then the measurement of a Pauli observable
 * (observable[q] in 'I', 'X', 'Y', 'Z') with the kept qubits kept[0..n_kept)
 * (observable 'I' there) read out in the computational basis:
 *     out[x] = Re <psi| O (x) |x><x|_kept |psi>,  x < 2^n_kept,
 * x row-major over the kept qubits (kept[0] slowest), every other qubit
 * summed.  Ops (htn_sv_op):
 *   HTN_SV_U1    q0: 2x2 unitary m = (re, im) of u00, u01, u10, u11
 *   HTN_SV_CZ    q0, q1 (distinct)
 *   HTN_SV_CX    control q0, target q1
 *   HTN_SV_RZZ   exp(-i m[0]/2 Z_q0 Z_q1)
 *   HTN_SV_PROJ  projection of q0 onto |q1> (q1 = 0 or 1), unnormalised
 * Instance outputs are numbered consecutively (instance 0's first).
 * Assembly: entry e = sum over t in [entry_start[e], entry_start[e+1]) of
 * term_coef[t] * output[term_output[t]], in that order, in FP64.
 * States of up to 12 qubits are simulated in LDS, larger ones (up to 24) in
 * device memory owned by the handle.
 *
 * htn_qt_eval_create — validate and upload (synchronous).  Host arrays are
 *   copied.  Errors: HTN_E_ARG (qubit counts, NULL data, observable
 *   letters, kept qubits out of range, repeated or not 'I', op kinds and
 *   qubits, projection bits, entry_start not starting at 0 or decreasing,
 *   term outputs out of range), HTN_E_OOM, HTN_E_DEVICE.
 * htn_qt_eval_run — enqueue on hip_stream: the instances (one launch, one
 *   workgroup each) and the assembly (one launch) into entries (device,
 *   n_entries FP64 values).  outputs (device, n_outputs FP64 values) may be
 *   NULL; otherwise the raw instance outputs are written there.
 * htn_qt_eval_info — the handle's output and entry counts.
 * ------------------------------------------------------------------- */
#define HTN_SV_MAX_QUBITS 24
typedef enum { HTN_SV_U1 = 0, HTN_SV_CZ = 1, HTN_SV_CX = 2, HTN_SV_RZZ = 3, HTN_SV_PROJ = 4 } htn_sv_kind;
typedef struct {
    int32_t kind;
    int32_t q0, q1;
    int32_t pad;
    double m[8];
} htn_sv_op;
typedef struct {
    int32_t n_qubits;
    const double *init;
    int32_t n_ops;
    const htn_sv_op *ops;
    const char *observable;
    int32_t n_kept;
    const int32_t *kept;
} htn_sv_instance;
typedef struct htn_qteval *htn_qteval_t;
htn_status htn_qt_eval_create(htn_qteval_t *out, int32_t n_instances, const htn_sv_instance *instances,
                              int64_t n_entries, const int64_t *entry_start, const int64_t *term_output,
                              const double *term_coef);
htn_status htn_qt_eval_run(htn_qteval_t q, double *entries, double *outputs, void *hip_stream);
htn_status htn_qt_eval_info(htn_qteval_t q, int64_t *n_outputs, int64_t *n_entries);
void htn_qt_eval_destroy(htn_qteval_t q);

#ifdef __cplusplus
}
#endif

#endif /* HTN_H */
