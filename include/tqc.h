/*
 * tqc.h - reconstruction of cut quantum circuits by tensor-network
 * contraction on one AMD Instinct MI355X (gfx950).
 *
 * The method (TensorQC, arXiv 2502.03445): a circuit on n qubits is cut on
 * K wires into m subcircuits.  Each cut carries a 4-valued Pauli index
 * (I, X, Y, Z); subcircuit j yields a tensor p_j of shape
 * 4^(its cuts) x 2^(its output qubits) (Sec. II-A).  The output distribution
 * is the contraction of those tensors over all cut indices (Eq. (1)),
 * evaluated as an ordered sequence of m-1 pairwise contractions (Sec. III-B,
 * Eq. (3)) with optional slicing of cut indices (Sec. III-E2).
 *
 * Conventions used throughout this interface
 *   - Pauli digit order I=0, X=1, Y=2, Z=3.
 *   - A tensor's rows are digits over its cuts in the order of cut_ids, the
 *     first cut being the slowest digit; its columns are output bits, bit t
 *     of the column index being the measured value of output_qubits[t].
 *   - Raw (measured) tensors: rows are mixed-radix digits over the cuts,
 *     radix 3 where the tensor is the upstream (measured) end of the cut
 *     (0=Z, 1=X, 2=Y basis; I shares the Z rotation), radix 4 where it is
 *     the downstream (prepared) end (0=|0>, 1=|1>, 2=|+>, 3=|i>); columns are
 *     x * 2^u + b, with b bit i the measured value of the i-th upstream cut
 *     in cut_ids order (Sec. II-A, variant count of Eq. (6)).
 *   - Output probability vectors: bit q of the index is the measured value
 *     of qubit q.  With fixed qubits, bit i of the index is the i-th free
 *     qubit in ascending order, and entries are the unnormalised joint
 *     probabilities P(x) with x on the fixed qubits equal to the given values.
 *   - The factor 1/2 per cut of the identity decomposition (left implicit
 *     in Eq. (1)) is applied by the library.
 *
 * Ownership and errors
 *   - Host arrays passed in are copied during the call.
 *   - Device pointers passed in (outputs) remain owned by the caller and must
 *     hold the stated number of bytes on the current HIP device.
 *   - Streams are hipStream_t values passed as void*; NULL is the default
 *     stream.  All device work of a call is enqueued on that stream and may
 *     still be running when the call returns.
 *   - Every call returns a tqc_status; nothing throws or aborts across this
 *     interface.  tqc_last_error() gives a thread-local description of the
 *     last failure.  Device faults surface as TQC_ERR_DEVICE at a later call
 *     or at the caller's stream synchronisation.
 *   - Handles are created and destroyed in pairs; destroy a plan before the
 *     network it was built from.
 */
#ifndef TQC_H
#define TQC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TQC_OK = 0,
  TQC_ERR_INVALID_ARG = 1,     /* null pointer, out-of-range value          */
  TQC_ERR_TOPOLOGY = 2,        /* cut/qubit structure is not a valid network */
  TQC_ERR_SHAPE = 3,           /* data length or buffer size mismatch        */
  TQC_ERR_OUT_OF_MEMORY = 4,   /* device allocation failed                   */
  TQC_ERR_PLAN_INFEASIBLE = 5, /* no slicing fits the memory budget          */
  TQC_ERR_DEVICE = 6,          /* HIP runtime error                          */
  TQC_ERR_UNSUPPORTED = 7,     /* valid request this build does not handle   */
  TQC_ERR_INTERNAL = 8
} tqc_status;

/* Arithmetic form of the pairwise contractions (the Pauli-basis transform and
 * the cross-slice sum are always float64).
 *   FP64   float64 operands, float64 MFMA.
 *   FP32   float32 operands, float32 MFMA accumulation.
 *   BF16X3 operands split a = hi + lo into two bfloat16 values (hi =
 *          RNE(a), lo = RNE(a - hi)); products hi*hi + hi*lo + lo*hi on
 *          bfloat16 MFMA with float32 accumulation.
 *   BF16X6 three-way split a = hi + mid + lo; the six products whose
 *          combined weight is above 2^-24 (hh, hm, mh, hl, mm, lh).
 *   FP16X3 pairwise steps as FP32; the final step's two operands are each
 *          scaled by a power of two that puts their largest |value| in
 *          [2^14, 2^15) and split into two float16 values (hi = RNE(a),
 *          lo = RNE(a - hi), 22 significant bits), products hi*hi + hi*lo +
 *          lo*hi on float16 MFMA with float32 accumulation; the scale is
 *          undone exactly in the output epilogue. */
typedef enum { TQC_FP64 = 0, TQC_FP32 = 1, TQC_BF16X3 = 2, TQC_BF16X6 = 3, TQC_FP16X3 = 4 } tqc_precision;

/* Element type of a device probability vector. */
typedef enum { TQC_F64 = 0, TQC_F32 = 1 } tqc_dtype;

typedef enum { TQC_BASIS_RAW = 0, TQC_BASIS_PAULI = 1 } tqc_basis;

/* One cut edge: the tensor that measures the cut wire (upstream) and the
 * tensor that prepares it (downstream); they must differ (each cut joins
 * exactly two subcircuits, Sec. III-D). */
typedef struct {
  int32_t upstream;
  int32_t downstream;
} tqc_cut;

/* One subcircuit tensor (host memory, float64, row-major).  Rows x columns:
 *   PAULI: 4^num_cuts x 2^num_outputs
 *   RAW:   (3^u * 4^d) x 2^(num_outputs + u)   (u upstream, d downstream) */
typedef struct {
  int32_t num_cuts;
  const int32_t *cut_ids;       /* indices into the network's cut array */
  int32_t num_outputs;
  const int32_t *output_qubits; /* qubit ids, each in exactly one tensor */
  tqc_basis basis;
  const double *data;
} tqc_tensor_desc;

typedef struct tqc_network_s *tqc_network_t;
typedef struct tqc_plan_s *tqc_plan_t;
typedef struct tqc_costmodel_s *tqc_costmodel_t;

/* ------------------------------------------------------------------ network
 * tqc_network_create: validate and copy a network (Sec. II-A notation:
 * n qubits, m subcircuits, cut set E).  Checks: every cut names two distinct
 * tensors and appears in exactly those two tensors' cut lists; every qubit
 * 0..num_qubits-1 is an output of exactly one tensor; data sizes follow the
 * layouts above; values are finite.  Host-only: no device work happens until
 * tqc_network_upload or the first tqc_execute.
 * Errors: INVALID_ARG, TOPOLOGY, SHAPE. */
tqc_status tqc_network_create(int32_t num_qubits, int32_t num_tensors,
                              const tqc_tensor_desc *tensors, int32_t num_cuts,
                              const tqc_cut *cuts, tqc_network_t *out);

/* Copy the tensor data to the current device (synchronous).  Called
 * implicitly by the first tqc_execute.  Errors: OUT_OF_MEMORY, DEVICE. */
tqc_status tqc_network_upload(tqc_network_t net);

void tqc_network_destroy(tqc_network_t net);

/* --------------------------------------------------------------------- plan
 * Contraction order (Sec. III-E1), two-level slicing (Sec. III-E2) and the
 * per-step GEMM mapping.  The planner scores candidate plans with a
 * roofline cost (flops / MFMA peak vs bytes / HBM bandwidth per step, the
 * refinement of Eq. (7)) or with a trained cost model.
 *   TQC_COST_FLOPBYTE  the roofline model: exact dynamic programming over
 *                      subsets (up to 13 tensors), greedy beyond.  Host only.
 *   TQC_COST_MLP       slicing from the roofline planner; the order that the
 *                      trained model (cost_model) predicts fastest among
 *                      num_candidates randomised-greedy orders and the
 *                      roofline order.  Host plus model inference.
 *   TQC_COST_MEASURED  measured time as the judge (Sec. VIII-A observes that
 *                      flops over peak misjudges GPU time): slicing from the
 *                      roofline planner; the roofline plan and the
 *                      num_measured orders ranked best among num_candidates
 *                      sampled ones (by cost_model if given, else by the
 *                      roofline model) are each executed on the current
 *                      device at full size (one warm-up, median of 5 timed
 *                      runs, HIP events on a private stream); unless the
 *                      form is FP64, each result is compared over every
 *                      entry with a float64 run of the roofline plan, and
 *                      candidates above max_rel_error are rejected.  The
 *                      fastest accepted plan is returned, the roofline plan
 *                      when no other is accepted (the fallback).  Needs the
 *                      network's values, device memory for one output, a
 *                      float64 reference and one candidate workspace at a
 *                      time (freed before return); synchronous.  The
 *                      measured-only fields of tqc_plan_stats report it. */
typedef enum { TQC_COST_FLOPBYTE = 0, TQC_COST_MLP = 1, TQC_COST_MEASURED = 2 } tqc_cost_kind;

typedef struct {
  tqc_precision precision;     /* contraction form                          */
  tqc_dtype out_dtype;         /* element type of the output vector         */
  uint64_t mem_budget_bytes;   /* device bytes for inputs + intermediates; 0 = unlimited */
  int32_t num_fixed;           /* fixed-qubit slice of the output           */
  const int32_t *fixed_qubits;
  const int32_t *fixed_values; /* 0 or 1 each                                */
  int32_t num_order_steps;     /* >0: use this contraction sequence          */
  const int32_t *order;        /* 2*num_order_steps SSA ids: step s joins ids
                                  order[2s], order[2s+1] into id m+s          */
  int32_t num_sliced;          /* -1: planner chooses; >=0: slice exactly these */
  const int32_t *sliced_cuts;
  tqc_cost_kind cost_kind;
  tqc_costmodel_t cost_model;  /* required for TQC_COST_MLP                  */
  int32_t num_candidates;      /* randomised-greedy candidates (0 = default) */
  uint64_t seed;
  int32_t tile_policy;         /* 0 fixed default tiles, 1 autotuned table,
                                  2 fixed tiles and the general GEMM for
                                  every step (neither the persistent
                                  final-step kernel nor the long-k kernel) */
  int32_t num_measured;        /* TQC_COST_MEASURED: shortlisted orders timed
                                  besides the roofline plan (0 = 4)          */
  double max_rel_error;        /* TQC_COST_MEASURED: largest accepted
                                  max|P - P_ref| / max|P_ref| (0 = 1e-6)     */
} tqc_plan_options;

void tqc_plan_options_default(tqc_plan_options *opt);

tqc_status tqc_plan_create(tqc_network_t net, const tqc_plan_options *opt, tqc_plan_t *out);
void tqc_plan_destroy(tqc_plan_t plan);

typedef struct {
  int32_t num_steps;
  int32_t num_sliced;
  int32_t k_max_cuts;          /* K_max of Eq. (4): most cuts at any step     */
  int32_t out_qubits;          /* free output qubits (log2 of output entries) */
  uint64_t num_slices;         /* 4^num_sliced                                */
  uint64_t out_entries;
  double flops;                /* 2*M*N*K summed over steps and slices        */
  double mults_per_state;      /* Sec. III-C count: cut dims only             */
  double bytes;                /* algorithmic HBM bytes (operands + outputs)  */
  double predicted_seconds;    /* cost model used by the planner              */
  uint64_t workspace_bytes;    /* device workspace the plan allocates         */
  double plan_seconds;         /* host time spent planning                    */
  int32_t precision;           /* tqc_precision of the plan                   */
  int32_t out_dtype;           /* tqc_dtype of its output                     */
  /* TQC_COST_MEASURED only (0 otherwise): */
  int32_t num_measured;        /* plans timed, the roofline plan included     */
  double measured_seconds;     /* median device time of the chosen plan       */
  double fallback_measured_seconds; /* ... of the roofline plan               */
  double checked_rel_error;    /* its max|P - P_ref| / max|P_ref|; -1 for FP64 */
} tqc_plan_stats;

tqc_status tqc_plan_get_stats(tqc_plan_t plan, tqc_plan_stats *st);

typedef struct {
  int32_t lhs, rhs, result;    /* SSA ids                                    */
  int32_t log2_m, log2_n, log2_k;
  int32_t shared_cuts, open_cuts;
  int32_t slice_dependent;     /* recomputed for every slice                  */
  int32_t tile;                /* kernel tile id                              */
  double flops, bytes;
} tqc_step_info;

tqc_status tqc_plan_get_step(tqc_plan_t plan, int32_t step, tqc_step_info *info);
tqc_status tqc_plan_get_sliced(tqc_plan_t plan, int32_t *cuts_out /* num_sliced */);

/* Plan blobs.  A plan is a property of the network's structure, not of its
 * values (Sec. II-A: the subcircuit tensors change with every run of the
 * subcircuits; Sec. III-E: order and slicing depend only on which tensors
 * share which cuts), so a plan made once can be stored and reused.
 * tqc_plan_serialize writes the plan's decisions (contraction order, sliced
 * cuts in slicing order, fixed qubits and values, precision, output dtype,
 * tile policy, each step's tile, the predicted time) and the network
 * structure it was made for (qubit count, cut ends, each tensor's basis, cut
 * list and output qubits) to buf, host memory: a little-endian byte string
 * ending in a 64-bit FNV-1a hash of the rest.  With buf = NULL it only
 * stores the size in *len; otherwise *len is the capacity on entry and the
 * size written on return.
 * tqc_plan_deserialize rebuilds the plan on `net`, which must have the same
 * structure (values may differ); executing it gives bit-identical results to
 * the original plan on the same network.  Host only.
 * Errors: INVALID_ARG (null, truncated or corrupt blob, bad hash), SHAPE
 * (capacity too small), TOPOLOGY (structure differs). */
tqc_status tqc_plan_serialize(tqc_plan_t plan, void *buf, uint64_t *len);
tqc_status tqc_plan_deserialize(tqc_network_t net, const void *buf, uint64_t len, tqc_plan_t *out);

/* Caller-owned workspace.  tqc_plan_workspace_bytes gives the size of one
 * device region that holds every buffer the plan's execution uses (float64
 * Pauli tensors of raw inputs, transform scratch, split-k partials, packed
 * operands and intermediates of every step, operand scales, the float64
 * accumulator of the slice sum (Sec. III-E2) for float32 output, and the
 * root tile statistics or standalone scan scratch of tqc_execute_summary for
 * any k <= 4096 and any tile choice).  tqc_plan_set_workspace binds such a
 * region (device memory on the network's device, 256-byte aligned, at least
 * that many bytes; e.g. a torch tensor): the library clears it on `stream`
 * and from then on tqc_execute, tqc_execute_profiled, tqc_execute_summary,
 * tqc_execute_slices, tqc_plan_autotune and the multi-job executor allocate
 * no device memory for this plan.  The region stays the caller's: keep it
 * alive while the plan may run, and never let two plans share one region.
 * Buffers the library had allocated for the plan are freed first (hipFree
 * waits for the device).  workspace = NULL returns to library-owned
 * buffers, allocated on the next execute.  Before the first execute the
 * call uploads the network (tqc_network_upload).
 * Errors: INVALID_ARG (misaligned), SHAPE (too small), OUT_OF_MEMORY (the
 * network upload), DEVICE. */
tqc_status tqc_plan_workspace_bytes(tqc_plan_t plan, uint64_t *bytes);
tqc_status tqc_plan_set_workspace(tqc_plan_t plan, void *workspace, uint64_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ execute
 * Run the plan: Pauli-basis transform of raw tensors (float64), packing of
 * the contraction operands (slice and fixed-qubit gathers, cast/split),
 * every pairwise contraction, the float64 sum over slices, and the final
 * conversion to out_dtype.  out must hold out_entries elements of out_dtype.
 * Errors: SHAPE (out_bytes too small), OUT_OF_MEMORY, DEVICE. */
tqc_status tqc_execute(tqc_plan_t plan, void *out, uint64_t out_bytes, void *stream);

/* tqc_execute, then wait for the stream and report device time per phase,
 * measured with HIP events on that stream: phase_ms[0] Pauli-basis
 * transform, [1] operand scaling and packing, [2 + i] pairwise step i
 * (summed over slices; for FP16X3 the final step's phase includes the
 * float16 split of its two operands), [2 + num_steps] float64-to-float32
 * conversion (0 if none).
 * num_phases >= 3 + num_steps.  Synchronous.  Used for the benchmark's
 * per-kernel roofline and as training data of the learned cost model. */
tqc_status tqc_execute_profiled(tqc_plan_t plan, void *out, uint64_t out_bytes, void *stream,
                                double *phase_ms, int32_t num_phases);

/* Run slices [slice_begin, slice_end) only, adding into a float64 output
 * (accumulate=1) or overwriting it (accumulate=0).  Summing disjoint ranges
 * gives the full result; used to resume after a partial run. */
tqc_status tqc_execute_slices(tqc_plan_t plan, double *out, uint64_t out_bytes,
                              uint64_t slice_begin, uint64_t slice_end,
                              int32_t accumulate, void *stream);

/* Pauli-basis tensor of network tensor j after the float64 transform
 * (4^c x 2^o, the layout above) into a device buffer; for checking the
 * transform on its own. */
tqc_status tqc_network_pauli_tensor(tqc_network_t net, int32_t j, double *out,
                                    uint64_t out_bytes, void *stream);

/* ------------------------------------------------------------ output forms
 * Top-k (Eq. (10): the sum of the k largest true probabilities is
 * P_HSS^max): the k largest entries, larger value first, equal values by
 * smaller index.  idx_out/val_out are device arrays of k elements.  1 <= k <=
 * 4096 and k <= len.  Deterministic. */
tqc_status tqc_topk(const void *probs, tqc_dtype dtype, uint64_t len, int32_t k,
                    uint64_t *idx_out, double *val_out, void *stream);

/* Marginal over the kept qubits: out[y] = sum of probs[x] over x whose bit
 * keep[i] equals bit i of y; float64 sums in a fixed order (deterministic).
 * num_keep = 0 gives the total (1 for a physical circuit).  out is a device
 * array of 2^num_keep doubles; num_keep <= 24. */
tqc_status tqc_marginal(const void *probs, tqc_dtype dtype, int32_t num_qubits,
                        int32_t num_keep, const int32_t *keep, double *out, void *stream);

/* The scratch of tqc_topk and tqc_marginal above is library-owned: one
 * device buffer per (device, stream), reused by calls on that stream and
 * grown by synchronizing the stream; calls on different streams never share
 * memory.  The _ws forms below take the scratch from the caller instead and
 * allocate nothing: workspace is device memory of at least the bytes the
 * matching _workspace_bytes call reports, 256-byte aligned, used only on
 * `stream` until the call's work is done; its contents on entry do not
 * matter.  Results equal the library-scratch forms bit for bit.
 * Errors: as tqc_topk / tqc_marginal, plus SHAPE (workspace too small) and
 * INVALID_ARG (workspace NULL or misaligned). */
tqc_status tqc_topk_workspace_bytes(uint64_t len, int32_t k, uint64_t *bytes);

/* tqc_topk for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results as tqc_topk, bit for bit, with their scratch in
 * a fixed 8 MiB device array that the library holds on each GPU it runs on
 * until the process ends.  The call allocates and frees nothing.  That
 * covers len <= 2^32 for every k <= 4096; a longer vector is rejected with
 * INVALID_ARG before any device work.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (two streams, or two host
 * threads) race and give wrong results; one call after another on a stream,
 * or with the stream synchronized in between, is safe.  The kernels
 * initialize every scratch entry they read, so nothing needs clearing.
 * Errors: as tqc_topk, plus DEVICE (the array's address cannot be found). */
tqc_status tqc_topk_noalloc(const void *probs, tqc_dtype dtype, uint64_t len, int32_t k,
                            uint64_t *idx_out, double *val_out, void *stream);
tqc_status tqc_topk_ws(const void *probs, tqc_dtype dtype, uint64_t len, int32_t k,
                       uint64_t *idx_out, double *val_out, void *workspace, uint64_t ws_bytes,
                       void *stream);
tqc_status tqc_marginal_workspace_bytes(int32_t num_qubits, int32_t num_keep, uint64_t *bytes);
tqc_status tqc_marginal_ws(const void *probs, tqc_dtype dtype, int32_t num_qubits, int32_t num_keep,
                           const int32_t *keep, double *out, void *workspace, uint64_t ws_bytes,
                           void *stream);

/* One reconstruction and its summary: tqc_execute into out, then the k
 * largest entries of out (as tqc_topk: top_idx / top_val, device arrays of k
 * elements; k = 0 skips them) and the float64 total of out (as tqc_marginal
 * with num_keep = 0; *total is a device double).  Eq. (1) for the vector,
 * Eq. (10) for the top entries.  For a single-slice plan of two or more
 * tensors the root contraction also writes, for each output tile it stores,
 * the largest value and the float64 sum; the top-k then gathers only the
 * tiles whose maximum reaches the k-th largest tile maximum, and the total
 * adds the tile sums, so no extra pass reads the 2^n vector.  Other plans run
 * the standalone scans.  Top-k results equal tqc_topk's bit for bit; the
 * total differs from tqc_marginal's only in summation order.  phase_ms (may
 * be NULL): as tqc_execute_profiled, with the top-k and total in the last
 * phase; with it the call is synchronous.  0 <= k <= 4096, k <= out_entries.
 * Errors: INVALID_ARG, SHAPE, OUT_OF_MEMORY, DEVICE. */
tqc_status tqc_execute_summary(tqc_plan_t plan, void *out, uint64_t out_bytes, int32_t k,
                               uint64_t *top_idx, double *top_val, double *total,
                               double *phase_ms, int32_t num_phases, void *stream);

/* ---------------------------------------------------------------- cut search
 * Sec. VI, Alg. 2-3, Table I (host only; the step before tqc_network_create).
 * gate_qubits holds two entries per gate in circuit order: the qubits of a
 * two-qubit gate, or (q, -1) for a single-qubit gate.  The circuit DAG keeps
 * one vertex per two-qubit gate and one edge per wire segment between
 * consecutive two-qubit gates of a qubit.  Partitions grow from single gates
 * by merging the adjacent pair with the smallest Table I cost (ties: smaller
 * first gates) while that cost is at most q_max: for the trial union,
 * w/w_max + s/s_max + k/k_t, where w = qubits (one per maximal run of a
 * wire's two-qubit gates inside it), s = two-qubit gates, k = the largest
 * number of contraction edges (cut edges of the union or of a neighbour)
 * between the union and one of its neighbours; w > w_max or s > s_max is not
 * allowed, k > k_t costs 4^(k - k_t) + 1 instead of k/k_t.  After a merge only
 * the pairs touching the merged partition are costed again (Alg. 2).
 * Output: labels[g] = partition of two-qubit gate g (0.. in order of each
 * partition's first gate), -1 for single-qubit gates; num_parts.  The paper
 * uses k_t = 10, q_max = 1e4.  Errors: INVALID_ARG. */
tqc_status tqc_find_cuts(int32_t num_qubits, int32_t num_gates, const int32_t *gate_qubits, int32_t w_max,
                         int32_t s_max, int32_t k_t, double q_max, int32_t *labels, int32_t *num_parts);

/* ------------------------------------------------- heavy state selection
 * Sec. IV, Alg. 1.  tqc_hss_select computes, for every tensor j and every
 * state i of its output qubits, the L2 norm of column i of its Pauli-basis
 * tensor over all rows (edge permutations), in float64 on the device
 * (deterministic order).  Every tensor starts with its heaviest state (ties:
 * smaller i); the other (j, i) join in descending norm order (ties: smaller
 * j, then smaller i) while the product of the subset sizes is below s_max, so
 * the product can exceed s_max by the last state added (at most twofold).
 * Output (host memory): counts[j] = subset size (num_tensors entries);
 * states = the subsets, tensor by tensor, ascending, at most states_cap
 * entries (sum_j 2^o_j always suffices); norms (optional, NULL to skip) =
 * every column norm, tensor by tensor, at most norms_cap entries.  Waits for
 * `stream`.  Errors: INVALID_ARG, SHAPE (a capacity too small), DEVICE.
 *
 * tqc_network_select_states makes a new network (device-resident, Pauli
 * basis) whose tensor j keeps columns states_j (counts[j] ascending states
 * of its output qubits, concatenated as tqc_hss_select gives them) padded
 * with zero columns to 2^b_j, b_j = ceil(log2 counts[j]); its b_j output
 * qubits come after those of tensors 0..j-1.  Contracting it (any plan,
 * form or slicing) gives P at the retained product states: entry
 * sum_j y_j 2^(b_0 + .. + b_{j-1}) is P of the state whose tensor-j output
 * bits are states_j[y_j]; entries with some y_j >= counts[j] are exactly
 * zero.  The source network is only read; destroy the new one with
 * tqc_network_destroy.  Errors: INVALID_ARG (counts out of range, states
 * not ascending or out of range), OUT_OF_MEMORY, DEVICE. */
tqc_status tqc_hss_select(tqc_network_t net, uint64_t s_max, int32_t *counts, int32_t *states,
                          uint64_t states_cap, double *norms, uint64_t norms_cap, void *stream);
tqc_status tqc_network_select_states(tqc_network_t net, const int32_t *counts, const int32_t *states,
                                     void *stream, tqc_network_t *out);

/* --------------------------------------------------------------- multi-job
 * Many independent reconstructions replayed as one HIP graph (batched
 * execution for serving; the paper runs one reconstruction at a time).
 * tqc_multi_create binds num_jobs unsliced plans to their outputs (device
 * pointers to out_entries values of each plan's out_dtype; out_bytes may be
 * NULL, else each entry is checked), allocates every workspace, and spreads
 * the jobs over num_streams streams (0 = 4, at most 16), largest predicted
 * first, each to the least-loaded stream.  With use_graph = 1 the first
 * tqc_multi_execute captures every job's launches (transform, packs,
 * pairwise steps, final step) between a fork from and a join into `stream`
 * once; each call then replays that graph on `stream`.  With use_graph = 0
 * the same launches are enqueued directly (num_streams = 1 gives the jobs as
 * sequential plain launches).  Results equal tqc_execute's bit for bit.  Jobs
 * must not share a plan; a plan must not be executed elsewhere while the
 * object runs it.  The object keeps pointers to the plans and outputs:
 * destroy it before them.  With timed = 1 a one-thread kernel stores the
 * device clock before and after each job (a few microseconds per job);
 * tqc_multi_job_times then waits for the last execute and gives each job's
 * start and end in ms after that execute began (num_jobs doubles in each
 * array; either may be NULL).  Errors: INVALID_ARG (also job times without
 * timed, or before any execute, and grouped outside 0..2), UNSUPPORTED
 * (sliced plan), SHAPE, OUT_OF_MEMORY, DEVICE (also a failed capture). */
typedef struct tqc_multi_s *tqc_multi_t;
tqc_status tqc_multi_create(int32_t num_jobs, const tqc_plan_t *plans, void *const *outs,
                            const uint64_t *out_bytes, int32_t use_graph, int32_t num_streams,
                            int32_t timed, void *stream, tqc_multi_t *out);
/* As tqc_multi_create, with options.  grouped = 1: the jobs' work runs as a
 * short list of shared launches on `stream` (one graph with use_graph)
 * instead of each job's own launches: the clearing of the operand abs-max
 * accumulators, the Pauli-transform passes of all jobs level by level and
 * their per-entry transforms (which take each leaf's abs-max), the abs-max
 * of leaves given in the Pauli basis, the exponents and the leaf packs in
 * one launch each, then the pairwise steps depth by depth, one launch per
 * kernel variant and depth (a step the plain launcher would split over k,
 * and the float16 split of a final step, run alone), and last every final
 * step that runs on the persistent final-step kernel (float32 output, K <=
 * 256, at least 2^7 rows and columns): one persistent launch per (form, K),
 * each job on a row of the launch grid, jobs with the most tiles first.
 * Each record computes what the job's own tqc_execute computes (the same
 * maxima give the same exponents, whether a pack or the exponent launch
 * turns them into scales), and a workgroup of a shared launch runs as the
 * same workgroup of that launch would, so results equal tqc_execute's bit
 * for bit.  num_streams is unused in this mode.  With timed = 1 every job
 * starts with the first launch and ends with the launch that runs its final
 * step.  grouped = 2 (grouped heads): only the launches before the pairwise
 * steps are shared, per wave (transform passes, per-entry transforms,
 * scales, leaf packs of the wave's jobs), the waves one after another on one
 * extra stream; each job's pairwise steps and final step are its own
 * launches, as tqc_execute makes them, on one of num_streams worker streams
 * (each wave's jobs, largest first, to the least-loaded stream), after its
 * wave's shared launches; job times as without grouping.  tqc_multi_info:
 * launches per execute (-1 unless grouped; with grouped heads the shared
 * launches only), final steps in shared persistent launches, and those
 * launches. */
typedef struct {
  int32_t use_graph;      /* as tqc_multi_create                          */
  int32_t num_streams;    /* as tqc_multi_create (0 = 4, at most 16)       */
  int32_t timed;          /* as tqc_multi_create                          */
  int32_t grouped;        /* 1: every kind of work in shared launches;
                             2: the launches before the pairwise steps  */
  int32_t waves;          /* grouped: the jobs split into this many waves
                             of about equal predicted cost (0 = 1), each a
                             launch list on its own stream; wave w + 1's
                             launches start when wave w's launches before
                             its final steps are done (grouped = 2: when
                             wave w's shared launches are done)          */
} tqc_multi_options;
tqc_status tqc_multi_create_ex(int32_t num_jobs, const tqc_plan_t *plans, void *const *outs,
                               const uint64_t *out_bytes, const tqc_multi_options *opt, void *stream,
                               tqc_multi_t *out);
tqc_status tqc_multi_info(tqc_multi_t multi, int32_t *launches, int32_t *shared_root_jobs,
                          int32_t *shared_root_launches);
tqc_status tqc_multi_execute(tqc_multi_t multi, void *stream);
tqc_status tqc_multi_job_times(tqc_multi_t multi, double *start_ms, double *end_ms);
void tqc_multi_destroy(tqc_multi_t multi);

/* -------------------------------------------------------------------- batch
 * tqc_batch_execute is switched off (returns UNSUPPORTED): GPU runs of the
 * persistent launch below did not finish, and the cause has not been
 * identified.  tqc_batch_execute_sequential (plain per-job launches) works;
 * tqc_multi_* above is the working batched path.
 * Design of the persistent path: many independent reconstructions in a few
 * launches, captured once into a HIP graph and replayed: three short launches over all jobs (Pauli
 * transform, operand abs-max, power-of-two exponents), then persistent
 * launches whose workgroups claim pack chunks and GEMM tiles of all jobs
 * from a shared queue.  Default: one persistent launch per depth of the
 * contraction trees (level-synchronous, items never wait).  With
 * dependency_waits = 1: a single persistent launch in which each item waits
 * on its producers' completion counters (bounded by spin_limit).  Jobs are unsliced plans of one precision; outputs are
 * bound at creation (device pointers, out_entries of each plan's out_dtype).
 * The batch keeps pointers to the plans: destroy it before them. */
typedef struct tqc_batch_s *tqc_batch_t;

typedef struct {
  int32_t use_graph;           /* 1: capture reset + launch in a HIP graph   */
  int32_t grid;                /* workgroups; 0 = occupancy x compute units  */
  int32_t dependency_waits;    /* 0: one launch per tree level; 1: one launch */
  uint64_t spin_limit;         /* bound of each dependency wait; 0 = default.
                                  On overrun the item sets the batch error
                                  flag and skips its work (the launch still
                                  completes); tqc_batch_job_times reports it. */
} tqc_batch_options;

/* Host emulation of the batch launch for these plans (no device work, no
 * GPU needed): the plans' device pointers are replaced by synthetic
 * addresses for the duration of the call (each buffer its own region), the
 * work tables are built exactly as tqc_batch_create builds them, and every
 * loop bound and address of the pre-pass kernels (Pauli transform, leaf
 * abs-max, exponents) and of every item of the persistent part (unit
 * lookup, pack chunks, GEMM tiles: operand rows, k step, output addresses,
 * staged compact index) is walked, as are the level and dependency order of
 * the units.  out_bytes may be NULL (each job's exact output size).  Returns
 * OK when every access stays inside the buffer it is made through, else
 * INTERNAL with the first violation in tqc_last_error() and in report
 * (optional, report_cap bytes, NUL-terminated).  The plans must not run
 * meanwhile.  Cost: every transform term, pack entry and output entry once;
 * meant for checking small batches. */
tqc_status tqc_batch_validate(int32_t num_jobs, const tqc_plan_t *plans, const uint64_t *out_bytes,
                              char *report, uint64_t report_cap);

tqc_status tqc_batch_create(int32_t num_jobs, const tqc_plan_t *plans, void *const *outs,
                            const uint64_t *out_bytes, const tqc_batch_options *opt,
                            void *stream, tqc_batch_t *out);
tqc_status tqc_batch_execute(tqc_batch_t batch, void *stream);

/* The same jobs as one ordinary tqc_execute each, in order, on `stream`
 * (the baseline).  Synchronous; job_ms[2j], job_ms[2j+1] = start and end of
 * job j in ms since the first job started (HIP events). */
tqc_status tqc_batch_execute_sequential(tqc_batch_t batch, void *stream, double *job_ms);

/* After tqc_batch_execute: waits for the stream, then gives each job's first
 * and last item times (device wall clock, ms since the earliest start) and
 * the error flag (nonzero if a dependency wait overran). */
tqc_status tqc_batch_job_times(tqc_batch_t batch, double *start_ms, double *end_ms,
                               uint32_t *error);
tqc_status tqc_batch_info(tqc_batch_t batch, uint64_t *items, int32_t *units, int32_t *grid);
void tqc_batch_destroy(tqc_batch_t batch);

/* ----------------------------------------------------------------- autotune
 * Time every tile shape for each step of an (unsliced) plan with HIP events,
 * keep the fastest in the plan and in a process-wide table keyed by
 * (precision, log2 M, log2 N, log2 K); plans created with tile_policy = 1
 * take their tiles from that table.  Save / load keep it across processes. */
tqc_status tqc_plan_autotune(tqc_plan_t plan, void *out, uint64_t out_bytes, int32_t reps,
                             void *stream);
tqc_status tqc_autotune_save(const char *path);
tqc_status tqc_autotune_load(const char *path);

/* --------------------------------------------------------------- cost model
 * A small MLP (16 features -> 64 -> 64 -> 1, ReLU, float32) predicting the
 * natural log of one contraction launch's device time; trained on timings
 * of the plain contractor (tqc_execute_profiled) with the library's own
 * forward / backward / Adam kernels, and used by tqc_plan_create with
 * cost_kind = TQC_COST_MLP to rank num_candidates contraction orders (the
 * roofline planner's choice, its greedy variant and randomised-greedy
 * samples) for the roofline planner's slicing.  The flop/byte model stays
 * the fallback (TQC_COST_FLOPBYTE).  Feature rows come from
 * tqc_plan_step_features (raw; the model normalises with statistics taken
 * from its training data).  Parameter vector order: W1 (16x64, row-major),
 * b1, W2 (64x64), b2, w3, b3.  Host arrays throughout. */
typedef struct {
  int32_t epochs;              /* default 200                                 */
  int32_t batch;               /* default 256                                 */
  float lr;                    /* Adam step size, default 3e-3                */
  uint64_t seed;               /* shuffling                                   */
} tqc_train_options;

tqc_status tqc_costmodel_create(uint64_t seed, tqc_costmodel_t *out);
void tqc_costmodel_destroy(tqc_costmodel_t m);
int32_t tqc_costmodel_num_params(void);
int32_t tqc_costmodel_num_features(void);
tqc_status tqc_costmodel_get_params(tqc_costmodel_t m, float *out, int32_t n);
tqc_status tqc_costmodel_set_params(tqc_costmodel_t m, const float *in, int32_t n);
/* raw network (no normalisation): y[i] = f(x[i, :]) */
tqc_status tqc_costmodel_forward(tqc_costmodel_t m, const float *x, int64_t n, float *y, void *stream);
/* raw gradient of mean_i (f(x_i) - t_i)^2 with respect to the parameters */
tqc_status tqc_costmodel_gradients(tqc_costmodel_t m, const float *x, const float *t, int64_t n,
                                   float *grad, void *stream);
/* fit on (raw features, measured seconds); loss_per_epoch (may be NULL)
 * receives the normalised training MSE after each epoch */
tqc_status tqc_costmodel_train(tqc_costmodel_t m, const float *feats, const float *seconds, int64_t n,
                               const tqc_train_options *opt, float *loss_per_epoch, void *stream);
tqc_status tqc_costmodel_predict(tqc_costmodel_t m, const float *feats, int64_t n, double *seconds,
                                 void *stream);
tqc_status tqc_costmodel_save(tqc_costmodel_t m, const char *path);
tqc_status tqc_costmodel_load(const char *path, tqc_costmodel_t *out);
/* raw feature rows (num_steps x 16) of a plan's launches */
tqc_status tqc_plan_step_features(tqc_plan_t plan, float *out, int32_t max_steps);

/* --------------------------------------------------------------------- misc */
const char *tqc_status_string(tqc_status s);
const char *tqc_last_error(void);
int32_t tqc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TQC_H */
