// Host-side plan structures: lowered circuit, per-step tensor networks,
// contraction trees and the emitted device programs.
#pragma once
#include <complex>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "program.hpp"
#include "pws.h"

namespace pws {

using cd = std::complex<double>;

struct GateIR {
  int kind = 0, nq = 1, q[2] = {0, -1};
  int param = -1, param2 = -1;
  double coeff = 1, coeff2 = 1;
  cd mat[16];        // [out * d + in]
  cd dmat[16];       // coeff * d mat / d angle  (param >= 0, single-angle gates)
  bool diag_on[2] = {false, false};
  bool diagonal = false, monomial = false;
  int sigma[4] = {0, 1, 2, 3};
  int nS = 0, sq[2] = {0, 0};
  int cand_mask[4] = {0, 0, 0, 0};
  int in_seg[2] = {-1, -1}, out_seg[2] = {-1, -1};
};

struct NoiseIR {
  int kind = 0, nq = 1, q[2] = {0, -1}, after_gate = 0;
  int nbranch = 0;
  std::vector<NoiseBranch> tab;  // nbranch * nq entries, branch-major
  int seg[2] = {-1, -1};
};

struct OpIR { int type, idx; };

// A tensor of the step network while it is being built: free legs (global
// segment ids, sorted) and the factors multiplied into it.
struct LeafBuild {
  std::vector<int> legs;
  std::vector<FactorDesc> factors;   // SRC_FREE payload = global leg id
  bool chain = false;
};

struct StepNet {
  int op = -1, gate = -1;
  std::vector<LeafBuild> leaves;
  std::vector<FactorDesc> scalars;   // factors with every leg fixed (common to all candidates)
  std::vector<int> open_legs;   // candidate order: S qubit j = 0 first (MSB of v)
  std::vector<int> zero_q;
};

struct Pair { int a, b; };

struct TreeCost {
  double flops = 0;     // complex multiply-adds per chain (per slice)
  double bytes = 0;     // complex elements moved (A + B + out) per chain: algorithmic
  double kbytes = 0;    // elements the node kernels actually move (re-reads included)
  double peak = 0;      // peak live elements
  int max_bits = 0;     // log2 of the largest tensor
};

struct PlanOptions {
  int planner = 0;               // 0 best, 1 greedy, 2 sweep
  int greedy_trials = 8;
  uint64_t arena_limit_elems = 1ull << 26;   // per chain, after slicing
  int forbid_slicing = 0;
  double traffic_weight = 10.0;  // cost of one element moved, in complex multiply-adds
  int lds_mode = 0;              // arenas live in LDS: arena_limit_elems is the LDS capacity
  double node_overhead = 512.0;  // per-node synchronisation, in complex multiply-adds
  int sweep_max_width = 0;       // > 0: steps whose sweep fits this many positions use the sweep form
  int sweep_lds_bytes = 160 * 1024;  // LDS one sweep-form workgroup may use
  int sweep_fuse = 1;            // fold diagonal sweep ops into neighbouring ops
  int sweep_cache = 1;           // restore a step's leading leaves from the previous step's tensor
  int sweep_cache_min = 4;       // shortest restored prefix worth a store and a load (leaves)
  int sweep_merge = 1;           // two-sided steps: contract with an anchor step's kept tensor
                                 // (1: when they touch fewer elements than one-sided steps, 2: always)
  int sweep_merge_min = 8;       // fewest anchor leaves worth a snapshot
  int sweep_snap_max = 128;      // snapshots per anchor step (cache slots)
  int sweep_anchor_horizon = 512;   // later steps an anchor's snapshots are planned for
  int precision = 1;             // PWS_PREC_* of the plan (element size of on-chip tensors)
  int fresh_steps = 1;           // sampling draws one-qubit gates on untouched qubits from the gate alone
  std::vector<int> forced_slices;   // legs (segment ids) every node-form network slices first
};

struct CircuitIR {
  int n = 0;
  int n_params = 0;
  std::vector<double> theta;
  std::vector<GateIR> gates;
  std::vector<NoiseIR> noise;
  std::vector<OpIR> ops;
  std::vector<int> seg_qubit;    // segment id -> qubit
  std::vector<int> seg_base;     // qubit -> first segment id
  int n_segs = 0;
  bool noisy = false;
  std::vector<double> readout;   // per-qubit readout flip probability (empty: none)
  std::vector<int> gate_op;      // gate index -> op index
  std::vector<int> first_noise_op_on_q;  // op index of first noise site touching q (INT_MAX if none)
  std::vector<std::vector<int>> qorders; // low-cutwidth qubit orders for sweep trees
  std::vector<pws_gate> specs;           // gate specifications (angles recomputed by set_theta)
  std::vector<std::vector<double>> spec_mats;
};

// Device programs of one plan, concatenated over steps.
struct Programs {
  std::vector<StepDesc> steps;
  std::vector<LeafDesc> leaves;
  std::vector<FactorDesc> factors;
  std::vector<NodeDesc> nodes;
  std::vector<int32_t> ktab;
  std::vector<int32_t> zero_q;
  std::vector<double> ltab;       // tabulated leaves (complex pairs)
  std::vector<int32_t> lvar;      // variant-bit codes
  std::vector<int32_t> lelem;     // per step: (leaf, element) pairs, flattened
  std::vector<SweepOp> sweeps;   // sweep-form ops of all steps
  std::vector<int32_t> mtab;     // sweep-form matrix-entry codes
  std::vector<MEntry> ment;      // the same entries, constants folded (flatten_mtab)
  std::vector<SnapDesc> snaps;   // anchor steps' kept tensors
  std::vector<int32_t> mmap;     // two-sided steps' leg position pairs
  int32_t n_slots = 1;           // cache slots per chain (slot 0: the next step's prefix)
  std::vector<int> merge_step, merge_op;   // per step: the anchor step and op of its snapshot (-1)
  int32_t max_snap_w = -1;       // widest snapshot (log2 elements)
  std::vector<double> mterm;     // chain-dependent term tables (complex pairs)
  std::vector<int32_t> mflat;    // flat factor records of PWS_MENTRY_FLAT entries
  std::vector<DenseRun> druns;   // dense-run form of the sweep steps (build_dense)
  std::vector<uint32_t> dtab;    // their F tables (512 words per variant)
  int32_t n_dense_steps = 0;
  bool dense_bf16 = false;       // dtab holds bf16 hi/lo pairs (else FP32 values)
  int32_t max_sweep_width = 0, max_leaf_area = 0, n_sweep_steps = 0;
  double sweep_flops_per_sample = 0;   // complex multiply-adds of the sweep-form steps
  double sweep_elems_per_sample = 0;   // running-tensor elements read + written by the sweep ops
  int32_t max_arena = 0, max_exp = 0, max_slice_bits = 0;
  double flops_per_sample = 0, bytes_per_sample = 0;   // unsliced algorithmic ledger
  double flops_executed = 0;                           // with slicing
  int log2_width = 0;
  int64_t n_slices_total = 0;
  // gradient extras (full-circuit program only)
  std::vector<NodeDesc> bnodes;                 // backward nodes
  std::vector<int32_t> grad_terms;              // (leaf, factor index in leaf, param, adj_off, adj_exp) x5
  std::vector<int32_t> leaf_adj_off;            // per leaf: arena offset of its adjoint
  std::vector<int32_t> leaf_adj_exp;
  int32_t adj_root_off = -1;                    // arena offset of the root's adjoint (seed 1)
};

// Circuit lowering (Algorithm 1 op classification, Kraus tables of
// Algorithm 2, segment numbering); returns "" or an error message.
std::string lower(const pws_circuit *c, const pws_noise *noise, CircuitIR &ir);
// New angles: gate tables recomputed; fails if a gate's structure changes.
std::string set_theta(CircuitIR &ir, const double *theta);
// Recompute the stored leaf tables of a program after new angles.
void retabulate(const CircuitIR &ir, Programs &prog);
// Fold the chain-independent factors of every sweep-form matrix entry into
// one constant and tabulate the chain-dependent ones (ment, mterm).  The
// layout depends only on the codes, so new angles rewrite values in place.
void flatten_mtab(Programs &prog);

// network of the prefix ending at gate `gate_limit` (inclusive) with the
// given open qubits; `op` is the step's op index.
StepNet build_step_net(const CircuitIR &ir, int gate_limit, const std::vector<int> &open_qubits,
                       int op, bool full_projection);
void fuse_leaves(StepNet &net, bool split_scalars = true);
void compute_qubit_orders(CircuitIR &ir);

std::vector<Pair> plan_tree(const CircuitIR &ir, const std::vector<std::vector<int>> &legs,
                            const std::vector<int> &open_legs, const PlanOptions &opt,
                            TreeCost *cost);
double kernel_traffic(const std::vector<int> &a, const std::vector<int> &b, const std::vector<int> &o);
TreeCost eval_tree(const std::vector<std::vector<int>> &legs, const std::vector<int> &open_legs,
                   const std::vector<Pair> &pairs);

// Emit one step (or the full-circuit network) into `prog`; returns "" or an error.
std::string emit_step(const CircuitIR &ir, StepNet &net, const std::vector<Pair> &pairs,
                      const PlanOptions &opt, int op_begin, Programs &prog, bool with_backward);

// Sweep form of one step (leaves absorbed one at a time into an on-chip
// running tensor); "" on success, else the reason it does not apply.
std::string emit_sweep(const CircuitIR &ir, StepNet &net, const PlanOptions &opt, int op_begin,
                       Programs &prog);
// The same in two stages: the absorption order (taking over the leading
// leaves of the previous sweep step when their tensor can be restored from
// it: dirty_q / dirty_seg mark the chain bits and noise records changed since
// that step), then the emission (store_n set by the next step's planning).
struct AnchorState;
struct SweepPlan {
  StepNet net;
  int op_begin = 0;
  std::vector<std::vector<int>> legs;
  std::vector<char> is_open;      // open legs of the sweep (the step's, and a merge's boundary)
  std::vector<std::string> sig;   // per leaf: content key
  std::vector<int> order;         // absorption order (the swept leaves)
  int W = 0;                      // positions of the running tensor
  int load_n = 0;                 // leading leaves restored from the previous step's tensor
  int store_n = 0;                // leading leaves after which the tensor is kept for the next step
  double run_cost = 0;            // elements the ops a sampling pass runs touch
  // two-sided steps: the leaves not swept here are an anchor step's kept
  // tensor (a snapshot), contracted with the swept tensor over `bound` at the end
  std::vector<char> swept;        // per leaf (empty: all)
  std::vector<int> bound;         // legs shared with the snapshot
  std::shared_ptr<AnchorState> merge_from;
  int merge_snap = -1;
  // anchor steps: the running tensor is kept at several points for later steps
  std::shared_ptr<AnchorState> anchor;
};
// A step whose sweep keeps running tensors at several points (snapshots) for
// later steps, which contract their own sweep of the other leaves with one.
struct AnchorState {
  SweepPlan plan;                 // the anchor's plan (order, legs, contents)
  int step_index = -1;            // set at emission
  std::vector<char> dirty_q, dirty_seg;   // chain bits / noise records changed since it ran
  struct Snap {
    int j = 0;                    // leaves of the anchor's order absorbed
    int slot = 0;                 // cache slot (1, 2, ...)
    int op = -1, w = 0;           // set at emission: op index it is stored before, positions
    std::vector<int> leg_pos;     // set at emission: position of each live leg (-1 elsewhere)
  };
  std::vector<Snap> snaps;
};
// Leg lists, open flags and leaf contents of a step's network (no order yet).
std::string sweep_setup(const CircuitIR &ir, const StepNet &net, int op_begin, SweepPlan &out);
std::string plan_sweep(const CircuitIR &ir, const StepNet &net, const PlanOptions &opt, int op_begin,
                       const SweepPlan *prev, const std::vector<char> &dirty_q, const std::vector<char> &dirty_seg,
                       SweepPlan &out, const std::vector<char> *swept = nullptr,
                       const std::vector<int> *bound = nullptr);
// Longest prefix of src's order that this step holds unchanged (same contents,
// none reading a chain bit or noise record marked dirty), among `usable`
// leaves, at which both leave the same legs live; valid[k]: the first k
// leaves form such a cut.  Leaves touching a leg in `forbid` end the prefix.
struct PrefixMatch {
  std::vector<int> mapped;        // this step's leaf for src->order[k]
  std::vector<char> valid;        // size mapped.size() + 1
};
PrefixMatch match_prefix(const SweepPlan &src, const SweepPlan &cur, const std::vector<char> &usable,
                         const std::vector<char> &dirty_q, const std::vector<char> &dirty_seg,
                         const std::vector<char> &forbid_leg);
// Anchor plan: the order (either direction of each qubit order) whose leading
// leaves stay clean longest, by each leaf's first dirty step (leaf_dirty);
// snapshots at the points later steps can use.  "" on success.
std::string plan_anchor(const CircuitIR &ir, const StepNet &net, const PlanOptions &opt, int op_begin,
                        const std::vector<int> &leaf_dirty, int this_step, SweepPlan &out, double *benefit);
std::string emit_sweep_plan(const CircuitIR &ir, SweepPlan &sp, const PlanOptions &opt, Programs &prog);
// Dense-run form of every noiseless sweep step (see DenseRun), tables as
// FP32 complex values or, with split_bf16, as bf16 hi/lo pairs: every op of
// each step when all tables take at most `full_bytes`, otherwise the ops a
// sampling pass runs (from its restore point on); steps whose tables would
// take the total past `max_bytes` keep no dense form.  Recomputes the
// tables from the current matrix entries (call again after retabulate: the
// layout depends only on the plan's structure).
void build_dense(Programs &prog, bool split_bf16, uint64_t full_bytes, uint64_t max_bytes);
std::string export_json(const CircuitIR &ir, const Programs &prog, int step);

}  // namespace pws
