/*
 * pws.h -- C ABI of the MI355X pilot-wave exact sampler.
 *
 * The engine implements the gate-by-gate ("pilot-wave") Markov chain of the
 * paper (Section 2, Algorithm 1) and its noisy extension (Section 3,
 * Appendix A, Algorithm 2).  For every gate that is not monomial, each chain
 * needs the amplitudes amp(C_t, y) = <y|U_t...U_1|0^n> of all candidates y
 * that agree with its classical state outside the gate's non-diagonal
 * qubits S (the block of BlockDecompose).  Those amplitudes are contractions
 * of the prefix circuit's tensor network (the amplitude oracle of Section 2);
 * this library plans them on the host and runs them, batched over chains, in
 * HIP kernels on gfx950, followed by the FP64-normalised transition draw.
 *
 * Conventions
 *  - Qubit k of a bitstring is bit (k % 64) of 64-bit word (k / 64); a
 *    bitstring occupies `words` = ceil(n_qubits / 64) consecutive words.
 *  - A two-qubit gate on (q0, q1) uses local index 2*b(q0) + b(q1); matrices
 *    are row-major [out][in], complex128 as (re, im) pairs.
 *  - Gate angle = coeff * theta[param] + offset (param < 0: offset only).
 *    Rotations are R_P(t) = exp(-i t P / 2) (appendix on QAOA).
 *  - Op order: every noise site is executed right after the gate named by
 *    `after_gate`; sites sharing a gate keep their list order.  The op index
 *    (position in that merged order) keys the random draw made there.
 *  - Random stream: u = (w0 >> 11) * 2^-53 with (w0..w3) =
 *    Philox4x64-10(counter = (op_index, chain, 0, 0), key = (seed, 0)).
 *    A draw picks the smallest candidate v (ascending local index) with
 *    u * P < C_v, C_v the inclusive prefix sum of p_v = |amp_v|^2 (FP64) and
 *    P the total; P = 0 keeps the state (zero-mass block, Section 2).
 *
 * Ownership: every input struct and array is borrowed for the duration of the
 * call and deep-copied into the plan.  Output buffers are owned by the
 * caller; a `pws_bits` with on_device = 1 points to device memory.
 * Streams: all device work is enqueued on the stream given to
 * pws_set_stream (default: the null stream); calls whose outputs are host
 * memory synchronise that stream before returning.
 * Errors: every call returns a pws_status; no exception or abort crosses the
 * ABI.  pws_last_error() gives a thread-local message for the last non-OK
 * status.  On error the outputs are undefined; the plan stays usable unless
 * the status is PWS_ERR_DEVICE.
 * Threading: one plan serves one stream at a time.
 */
#ifndef PWS_H_
#define PWS_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PWS_OK = 0,
  PWS_ERR_ARG = 1,          /* invalid argument or size                          */
  PWS_ERR_UNSUPPORTED = 2,  /* gate on > 2 qubits, non-LSM noise, unknown kind    */
  PWS_ERR_NOMEM = 3,        /* slicing cannot meet the memory budget / alloc fail */
  PWS_ERR_PLAN = 4,         /* planner failure (e.g. width beyond the limit)     */
  PWS_ERR_DEVICE = 5,       /* HIP runtime error, extension not usable            */
  PWS_ERR_NUMERIC = 6       /* zero-mass block or zero amplitude where forbidden  */
} pws_status;

typedef enum {
  PWS_PREC_FP64 = 0,   /* contraction in FP64 (validation mode)                  */
  PWS_PREC_FP32 = 1,   /* contraction in FP32 with per-chain log2 exponents      */
  PWS_PREC_BF16X3 = 2  /* FP32 storage; the noiseless sweep steps' dense runs
                          multiply bf16 hi/lo splits of both operands (three
                          products, FP32 accumulation); other work in FP32  */
} pws_precision;

/* Gate kinds: same spelling as the instance files. */
enum {
  PWS_GATE_H = 0, PWS_GATE_X = 1, PWS_GATE_RX = 2, PWS_GATE_RZ = 3, PWS_GATE_RZZ = 4,
  PWS_GATE_CNOT = 5, PWS_GATE_CZ = 6, PWS_GATE_U1 = 7, PWS_GATE_U2 = 8,
  PWS_GATE_CRX = 9, PWS_GATE_FSIM = 10
};
/* Noise kinds (local-submonomial channels, Appendix A). */
enum { PWS_NOISE_DEPOL1 = 0, PWS_NOISE_DEPOL2 = 1, PWS_NOISE_AMPDAMP = 2,
       PWS_NOISE_PHASEDAMP = 3, PWS_NOISE_PAULI1 = 4 };

/* One gate (Appendix A: a gate is a pair (A, q)).  q1 = -1 for one-qubit gates.
 * FSIM uses (param, coeff, offset) for theta and (param2, coeff2, offset2) for
 * phi, with matrix entry [3][3] = exp(+i phi) (Figure 1(c)).
 * `matrix` (U1: 4, U2: 16 complex entries as 8/32 doubles) is read only for U1/U2. */
typedef struct {
  int32_t kind, q0, q1, param;
  double coeff, offset;
  int32_t param2, _pad;
  double coeff2, offset2;
  const double *matrix;
} pws_gate;

typedef struct {
  int32_t n_qubits, n_gates, n_params, _pad;
  const pws_gate *gates;
  const double *theta;          /* n_params angles */
} pws_circuit;

/* Noise site applied right after gate `after_gate` (Eq. (2)-(4)).
 * DEPOL1/DEPOL2: p = total error probability (identity keeps 1 - p, each of the
 * 3 / 15 non-identity Pauli products p/3 / p/15); AMPDAMP: p[0] = gamma;
 * PHASEDAMP: p[0] = lambda; PAULI1: p = (px, py, pz).  q1 = -1 for 1-qubit sites. */
typedef struct {
  int32_t after_gate, kind, q0, q1;
  double p[3];
} pws_noise_site;

/* readout (nullable): per-qubit probability that the measured bit is
 * flipped (a classical error on the sampled bitstring s XOR x, applied
 * after the last operation; Section 4, the simulated chip's readout error).
 * Qubit q's flip draws u = (w0 >> 11) 2^-53 from Philox4x64-10(counter =
 * (n_ops + q, chain, 0, 0), key = (seed, 0)), n_ops the number of gates and
 * noise sites, and flips when u < readout[q]. */
typedef struct {
  int32_t n_sites, _pad;
  const pws_noise_site *sites;
  const double *readout;        /* n_qubits probabilities, or NULL */
} pws_noise;                    /* NULL = ideal circuit */

/* Optional contraction order of the full-circuit amplitude network (every
 * output leg fixed; Section 2: a schedule for any prefix subcircuit follows
 * from the full circuit's): n_pairs = L - 1 pairs (i, j) in SSA form over
 * its L leaves -- ids 0..L-1 are the leaves, pair k produces id L + k, every
 * id is used once.  The leaves and their legs are those pws_plan_export
 * reports for step -1 ("network": "legs", with the tree in use as "pairs").
 * The tree contracts the amplitude network of pws_amplitudes; sampling steps
 * keep the internal planner.  NULL / n_pairs = 0: internal planner.
 * PWS_ERR_ARG when the pairs are not such a tree. */
typedef struct {
  int32_t n_pairs, _pad;
  const int32_t *ssa_pairs;     /* 2 * n_pairs ids */
} pws_tree;

/* A plan option (key, value); the keys below, all optional. */
typedef struct {
  int32_t key, value;
} pws_option;
enum {
  PWS_OPT_GRID = 1,             /* node form: most workgroups of a wave-form launch            */
  PWS_OPT_SWEEP_WIDTH = 2,      /* steps whose running tensor fits 2^value elements use the
                                   sweep form (0: every step as a tree of nodes)              */
  PWS_OPT_GRAPH = 3,            /* 0: launch sampling passes one by one instead of replaying a
                                   captured graph                                             */
  PWS_OPT_LDS_BLOCK = 4,        /* LDS node form: threads per workgroup                       */
  PWS_OPT_LDS_BYTES = 5,        /* LDS a workgroup may use                                    */
  PWS_OPT_WAVES_PER_CU = 6,     /* sweep form: most resident chains (waves) per compute unit  */
  PWS_OPT_COOP4_WIDTH = 7,      /* sweep form: tensors of 2^value elements and more take four
                                   waves per chain                                            */
  PWS_OPT_COOP8_WIDTH = 8,      /* ... and eight                                              */
  PWS_OPT_RANGE_WIDTH = 9,      /* sweep form: consecutive steps up to 2^value elements share a
                                   launch (0: one launch per step)                            */
  PWS_OPT_CPW8 = 10,            /* sweep form: chains per wave for tensors up to 2^8 elements  */
  PWS_OPT_CPW10 = 11,           /* ... for 2^9 and 2^10 elements                              */
  PWS_OPT_WINDOW = 12,          /* sweep form: op-matrix entries per chain in LDS (0: the whole
                                   table)                                                     */
  PWS_OPT_FUSE = 13,            /* 0: keep diagonal ops apart instead of folding them        */
  PWS_OPT_KEEP = 14,            /* 0: no running tensor kept from one step to the next       */
  PWS_OPT_FRESH = 15,           /* 0: contract one-qubit gates on untouched qubits too       */
  PWS_OPT_MERGE = 16,           /* two-sided steps: 0 never, 1 when cheaper, 2 always         */
  PWS_OPT_LDS_FORM = 17,        /* 1: node-form networks sliced to fit the LDS               */
  PWS_OPT_DENSE_RANGE = 18,     /* dense runs: most steps per launch (0: no limit)           */
  PWS_OPT_DENSE_CPW2_WIDTH = 19 /* dense runs: tensors up to 2^value elements put two chains
                                   in a wave when the chains outnumber the resident waves     */
};

/* Memory bound, precision, slicing and options.  hbm_budget_bytes bounds the
 * device working set (arenas of all in-flight chains, kept tensors); legs are
 * sliced until one chain's network fits.  sliced_edges: n_sliced legs
 * (segment ids, as pws_plan_export reports them) that every node-form
 * network contracting them slices first (their values summed over
 * launches).  max_chains bounds chains per launch (0 = all).  NULL =
 * defaults (200 GiB, FP32, no options). */
typedef struct {
  uint64_t hbm_budget_bytes;
  int32_t n_sliced;
  int32_t flags;                /* PWS_PLAN_HOST_ONLY, PWS_PLAN_DENSE            */
  const int32_t *sliced_edges;
  int64_t max_chains;
  pws_precision precision;
  int32_t planner;              /* 0 = best of all, 1 = greedy, 2 = sweep       */
  int32_t n_options, _pad;
  const pws_option *options;
} pws_slices;

/* Plan on the host only (no device tables are uploaded); such a plan serves
 * pws_plan_stats / pws_step_* inspection and pws_plan_export, and every call
 * that needs the device returns PWS_ERR_DEVICE. */
#define PWS_PLAN_HOST_ONLY 1
/* FP32 plans: the noiseless sweep steps run as dense runs (consecutive ops on
 * at most four tensor positions multiplied on the host, in complex double,
 * into one 16 x 16 complex matrix per value of the chain bits they read)
 * applied with FP32 matrix-core products.  BF16x3 plans always run them,
 * with bf16 hi/lo split products accumulated in FP32. */
#define PWS_PLAN_DENSE 2

/* Bitstrings: n rows of `words` uint64.  on_device: data is a device pointer. */
typedef struct {
  int64_t n;
  int32_t words, on_device;
  uint64_t *data;
} pws_bits;

typedef struct pws_plan_impl *pws_plan_t;

/* Plan a circuit (Section 2 Algorithm 1, Appendix A Algorithm 2):
 * classifies every gate (monomial / diagonal / non-monomial with its block
 * table), lowers the noise sites to Kraus factor tables, builds every
 * non-monomial step's tensor network (legs of diagonal gates identified,
 * Appendix A), plans a contraction order per step, slices to the budget,
 * uploads gate tables and programs.  Errors: PWS_ERR_ARG (bad qubit index,
 * angle index, sizes), PWS_ERR_UNSUPPORTED (kind, > 2 qubits), PWS_ERR_PLAN,
 * PWS_ERR_NOMEM, PWS_ERR_DEVICE. */
pws_status pws_plan(const pws_circuit *circuit, const pws_noise *noise,
                    const pws_tree *tree, const pws_slices *slices, pws_plan_t *out);

/* amp(C, y) = <y|C|0^n> of the whole noiseless circuit for every bitstring
 * (Section 2, the amplitude oracle).  out_re_im: 2*n doubles (mantissa),
 * out_log2 (nullable): n int32 exponents, amp = mantissa * 2^exp; with
 * out_log2 == NULL the mantissa is scaled to the full value (may underflow).
 * Host or device outputs per `out_on_device` of the bits struct. */
pws_status pws_amplitudes(pws_plan_t plan, const pws_bits *bitstrings,
                          double *out_re_im, int32_t *out_log2);

/* Run n_chains independent chains of Algorithm 1 (ideal plan) or Algorithm 2
 * (noisy plan) with the given seed; writes the n_chains sampled bitstrings
 * (s XOR x for noisy plans).  out->n must be >= n_chains and out->words equal
 * ceil(n_qubits/64).  Errors: PWS_ERR_ARG, PWS_ERR_NUMERIC (zero-mass block),
 * PWS_ERR_DEVICE. */
pws_status pws_sample(pws_plan_t plan, int64_t n_chains, uint64_t seed, pws_bits *out);

/* For callers that cannot allocate device memory (code that runs between
 * graph captures, serving loops, harnesses that forbid hipMalloc): the
 * sampling pass of pws_sample with the same results bit for bit, run with
 * its workspace (chain states, kept running tensors, error flag) in a static
 * device array of 64 MiB that every device holds from the library's load
 * until the process ends; the call allocates nothing and captures no graph.
 * out must be on the device (on_device = 1).  All calls on one device share
 * that array: calls that overlap on one device (several streams or threads)
 * race and give undefined results.  Returns after the pass has finished.
 * Errors: PWS_ERR_ARG, PWS_ERR_NOMEM (the workspace for n_chains exceeds the
 * static array; the message states both sizes), PWS_ERR_NUMERIC,
 * PWS_ERR_DEVICE. */
pws_status pws_sample_noalloc(pws_plan_t plan, int64_t n_chains, uint64_t seed, pws_bits *out);

/* Sample several planned circuits, of any sizes, in one replay: a hipGraph
 * holds every plan's sampling pass (the same launches pws_sample makes) as a
 * branch of its own, forked from and joined into the first plan's stream, so
 * that instances too small to fill the device run side by side.  Plan i runs
 * n_chains[i] chains with seeds[i] into outs[i]; each result equals that of
 * pws_sample(plans[i], n_chains[i], seeds[i], &outs[i]) bit for bit (chains
 * of different plans are independent Markov chains, Section 2).  The graph is
 * kept in plans[0] and replayed while the plans, their programs, chain counts,
 * workspaces and output buffers stay the same; it is captured again
 * otherwise.  Arguments: arrays of n_plans entries (host memory); outs must be
 * on the device (on_device = 1) and, like the plans, distinct; every plan on
 * one device, none with max_chains below its chain count.  Returns after the
 * replay has finished.  pws_last_timing(plans[0]) then reports the replay's
 * time and launch count.  Errors: PWS_ERR_ARG, PWS_ERR_NUMERIC (a zero-mass
 * block in some plan), PWS_ERR_DEVICE. */
pws_status pws_sample_batch(int32_t n_plans, const pws_plan_t *plans, const int64_t *n_chains,
                            const uint64_t *seeds, pws_bits *outs);

/* Per-sample gradient d log|amp(C, x_i)|^2 / d theta_j of the noiseless circuit
 * by an adjoint (reverse-mode) contraction through each sample's tree.
 * dtheta: n * n_params doubles (row-major), host or device per samples->on_device.
 * Samples are processed as many at a time as hbm_budget_bytes allows (each
 * keeps its whole forward network); PWS_ERR_NOMEM when not even one fits, or
 * when the device allocation fails.  PWS_ERR_NUMERIC if some amp(C, x_i) is
 * exactly zero. */
pws_status pws_grad(pws_plan_t plan, const pws_bits *samples, double *dtheta);

/* ---- auxiliaries ---------------------------------------------------------- */

/* Enqueue all later work on this hipStream_t (NULL = null stream). */
pws_status pws_set_stream(pws_plan_t plan, void *hip_stream);

/* Device bytes pws_sample would need for n_chains (workspace + state). */
pws_status pws_workspace_bytes(pws_plan_t plan, int64_t n_chains, uint64_t *bytes);

/* Give the plan caller-owned device memory for its workspace (>= the size
 * pws_workspace_bytes reports); NULL/0 returns to library allocation. */
pws_status pws_bind_workspace(pws_plan_t plan, void *device_ptr, uint64_t bytes);

/* Plan ledger: algorithmic complex flops and bytes per sample summed over all
 * steps (unsliced tree), log2 of the largest per-chain intermediate, slices. */
pws_status pws_plan_stats(pws_plan_t plan, double *flops_per_sample,
                          double *bytes_per_sample, int32_t *log2_width, int64_t *n_slices);

/* Number of contraction steps (non-monomial gates) and the op index of step k. */
pws_status pws_step_count(pws_plan_t plan, int32_t *n_steps);
pws_status pws_step_info(pws_plan_t plan, int32_t step, int32_t *op_index,
                         int32_t *gate_index, int32_t *n_candidates);

/* Candidate amplitudes of one step for given chain states (before the step's
 * draw): for every state s_i, the 2^|S| amplitudes amp(C_t, y_v) with y_v = s_i
 * outside S, in ascending candidate order (mantissa pairs + one exponent per
 * state).  Ideal plans only.  out_re_im: n * 2^|S| * 2 doubles. */
pws_status pws_step_amplitudes(pws_plan_t plan, int32_t step, const pws_bits *states,
                               double *out_re_im, int32_t *out_log2);

/* Like pws_sample but also records the candidate chosen at every step:
 * trace is n_chains * n_steps bytes, n_steps as pws_step_count reports it
 * (step-major: trace[k * n_chains + c]; 254 where a chain's step had a single
 * candidate or no mass and kept its state, 255 where the draw failed). */
pws_status pws_sample_trace(pws_plan_t plan, int64_t n_chains, uint64_t seed,
                            pws_bits *out, uint8_t *trace);

/* The sampling pass of pws_sample run through step `step` only: out gets
 * every chain's state after that step's draw, out_re_im (n_chains * 2^|S| *
 * 2 doubles) and out_log2 (n_chains int32) the candidate amplitudes that
 * draw used, amp = mantissa * 2^exp, with the step's fixed-leg factor
 * included (so they equal amp(C_t, y_v) at the chain's state before the
 * draw; zeros where the chain's step had a single candidate).  It measures
 * the amplitudes a pass of this precision draws from, at states the pass
 * itself reaches.  Device outputs only (out->on_device = 1; the amplitude
 * arrays device pointers).  Errors: PWS_ERR_ARG (step out of range, or a
 * step drawn from its gate alone: a one-qubit gate on an untouched qubit),
 * PWS_ERR_UNSUPPORTED (max_chains below n_chains), PWS_ERR_NUMERIC,
 * PWS_ERR_DEVICE. */
pws_status pws_sample_probe(pws_plan_t plan, int64_t n_chains, uint64_t seed, int32_t step, pws_bits *out,
                            double *out_re_im, int32_t *out_log2);

/* Pick the fastest execution form for batches of n_chains by timing full
 * sampling passes: per-wave device arenas at several launch widths, and the
 * LDS-resident form (one workgroup per chain, each step sliced to fit on chip)
 * at several workgroup sizes.  The choice is kept in the plan and, when
 * cache_path is not NULL, in a text cache keyed by a hash of the circuit,
 * precision and batch size (a cached entry is reused without timing).
 * The forms differ only for steps contracted as a tree of nodes.  When every
 * step runs in the sweep form, the call tunes the sweep launches instead:
 * chains per wave of narrow launches, steps per range launch, the width from
 * which four waves share a chain, the widest step joined to a range and (op
 * by op plans) the op-matrix window, one knob at a time over a few values,
 * each timed over whole passes (cache key suffix ":sweep").  Every choice
 * gives the same samples.  *chosen (nullable) receives a short description
 * (the values kept and the times measured).  Errors as pws_sample. */
pws_status pws_autotune(pws_plan_t plan, int64_t n_chains, uint64_t seed, const char *cache_path,
                        char *chosen, int64_t chosen_len);

/* Ledger of the sweep-form steps (steps contracted by absorbing leaves one at
 * a time into a running tensor held on chip): how many steps use that form,
 * their real flops per sample (8 per complex multiply-add of every op),
 * the bytes of running-tensor elements the ops read and write per sample
 * (on-chip traffic, element size of the plan's precision), and the widest
 * running tensor (log2 elements).  Any pointer may be NULL. */
pws_status pws_plan_sweep_stats(pws_plan_t plan, int32_t *n_sweep_steps, double *flops_per_sample,
                                double *tensor_bytes_per_sample, int32_t *max_width);

/* Time the last pws_sample's contraction launches (HIP events on the plan's
 * stream): total milliseconds and number of step launches. */
pws_status pws_last_timing(pws_plan_t plan, double *ms_total, int32_t *n_launches);

/* Replace the angle vector theta (n_params doubles, host memory) of a
 * planned circuit without planning again: the gate matrices, their angle
 * derivatives and every tabulated leaf are recomputed on the host and written
 * over the plan's device tables in place, so the contraction orders, slicing,
 * workspaces and captured sampling graphs stay valid.  Blocks until work
 * already queued on the plan's stream has finished.  Errors: PWS_ERR_ARG
 * (n_params differs from the circuit's, theta NULL), PWS_ERR_PLAN (at the new
 * angles a gate's structure changes -- for instance a rotation by zero becomes
 * diagonal -- so the plan no longer matches the circuit and must be made
 * again; the plan keeps its old angles), PWS_ERR_DEVICE. */
pws_status pws_set_theta(pws_plan_t plan, const double *theta, int32_t n_params);

/* JSON description of one step's plan (tensors, factor sources, contraction
 * pairs, gate tables) for host-side inspection; returns required length in
 * *len when buf is NULL or too small. step = -1: the full-circuit network. */
pws_status pws_plan_export(pws_plan_t plan, int32_t step, char *buf, int64_t *len);

const char *pws_last_error(void);
void pws_destroy(pws_plan_t plan);

#ifdef __cplusplus
}
#endif
#endif /* PWS_H_ */
