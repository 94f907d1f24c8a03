// C ABI of the pilot-wave sampler: plan construction, device uploads and
// the launch sequences of pws_sample / pws_amplitudes / pws_grad.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "device.hpp"
#include "host.hpp"
#include "pws.h"

using namespace pws;

namespace {

thread_local std::string g_last_error;

pws_status fail(pws_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(PWS_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));  \
  } while (0)

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  ~DevBuf() { if (p) (void)hipFree(p); }
  hipError_t ensure(size_t b) {
    if (b <= bytes && p) return hipSuccess;
    if (p) { (void)hipFree(p); p = nullptr; bytes = 0; }
    hipError_t e = hipMalloc(&p, std::max<size_t>(b, 256));
    if (e == hipSuccess) bytes = std::max<size_t>(b, 256);
    return e;
  }
};

template <typename T>
hipError_t upload(std::vector<std::unique_ptr<DevBuf>> &bufs, const std::vector<T> &v, const T **out) {
  auto b = std::make_unique<DevBuf>();
  hipError_t e = b->ensure(std::max<size_t>(v.size() * sizeof(T), 16));
  if (e != hipSuccess) return e;
  if (!v.empty()) {
    e = hipMemcpy(b->p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
  }
  *out = reinterpret_cast<const T *>(b->p);
  bufs.push_back(std::move(b));
  return hipSuccess;
}

}  // namespace

struct pws_plan_impl {
  CircuitIR ir;
  PlanOptions opt;
  int precision = PWS_PREC_FP32;  // element type of stored tensors (FP32 for BF16x3 plans)
  int requested_precision = PWS_PREC_FP32;
  int dense = 0;                  // sweep steps as dense runs: 1 FP32 matrix cores, 2 bf16 hi/lo split
  int dense_range_steps = 0;      // dense runs: most steps per range launch (0: no limit; a
                                  // plan's consecutive narrow steps then form one launch, the
                                  // fastest for batches, whose branches overlap)
  int dense_cpw2_width = 10;      // dense runs: tensors this narrow put two chains in a wave
  int64_t batch_chains = 0;       // pws_sample_batch: chains of every plan replayed together (0: alone)
  std::vector<std::unique_ptr<DevBuf>> dbufs;   // dense-run tables (P->prog)
  uint64_t budget = 200ull << 30;
  int64_t max_chains = 0;
  int device = 0;
  bool host_only = false;
  hipStream_t stream = nullptr;
  Programs prog;                 // sampling steps + epilogue (active form)
  Programs prog_alt;             // the other form, once planned by the autotuner
  DevProg dp_alt{};
  std::vector<std::unique_ptr<DevBuf>> altbufs;
  int have_alt = 0;
  Programs prog_solo;            // steps that run on their own (no kept tensors), for
  DevProg dp_solo{};             // single-step amplitude calls of plans with two-sided steps
  std::vector<std::unique_ptr<DevBuf>> solobufs;
  bool have_solo = false;
  uint64_t plan_hash = 0;
  Programs full_amp, full_grad;  // whole-circuit networks (lazy)
  bool have_amp = false, have_grad = false;
  std::vector<std::unique_ptr<DevBuf>> tables;   // gate / noise / op tables
  std::vector<std::unique_ptr<DevBuf>> pbufs, abufs, gbufs;
  DevProg dp{}, dp_amp{}, dp_grad{};
  // workspaces
  DevBuf ws_state, ws_arena, ws_err, ws_io, ws_io2;
  void *bound = nullptr;
  uint64_t bound_bytes = 0;
  int grid_max = 1024;
  int cus = 256;
  int lds_mode = 0;              // arenas in LDS (one workgroup per chain)
  int amp_lds = 0;               // the whole-circuit amplitude program's form
  uint64_t budget_limit = 1ull << 26;  // per-chain arena limit in device memory (elements)
  int lds_capacity = 160 * 1024; // bytes per workgroup
  int lds_per_cu = 160 * 1024;   // bytes per compute unit
  int sweep_waves_per_cu = 32;   // sweep form: resident chains per compute unit (upper bound)
  int sweep_coop_width = 12;     // sweep form: tensors this wide are shared by four waves
  int sweep_coop8_width = 15;    // ... and this wide by eight
  int sweep_range_w = 8;         // sweep form: steps this narrow share launches (0: one launch per step;
                                 // 10 for noiseless FP32 plans)
  int sweep_cpw8 = 2;            // sweep form: chains per wave for tensors of up to 2^8 elements
  int sweep_cpw8_few = 0;        // ... where at most 16 waves per CU are launched (0: as above;
                                 // 1 for noisy plans)
  int sweep_cpw10 = 1;           // ... and of 2^9 or 2^10 elements (2 for noiseless FP32 plans)
  int sweep_mt_cap = 128;        // sweep form: op-matrix entries per chain in LDS (a window of the
                                 // step's table; 0: the whole table)
  int block = 256;               // threads per workgroup in the LDS form
  double last_ms = 0;
  int last_launches = 0;
  // persistent form: the whole sampling pass captured once and replayed
  bool use_graph = true;
  hipStream_t own_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  int64_t g_K = -1;
  const void *g_state = nullptr, *g_arena = nullptr, *g_out = nullptr;
  hipStream_t g_stream = nullptr;
  int g_launches = 0;            // kernel launches inside the captured graph
  DevBuf seed_buf;
  // pws_sample_batch with this plan first: the captured graph of every plan's
  // pass (one branch per plan), the branch streams and fork / join events
  uint64_t uid = 0;              // distinct for every plan made in this process
  hipGraphExec_t bexec = nullptr;
  std::vector<uint64_t> b_key;
  std::vector<hipStream_t> b_streams;
  std::vector<hipEvent_t> b_events;
  int b_launches = 0;
  ~pws_plan_impl() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (bexec) (void)hipGraphExecDestroy(bexec);
    for (hipStream_t b : b_streams) (void)hipStreamDestroy(b);
    for (hipEvent_t e : b_events) (void)hipEventDestroy(e);
    if (own_stream) (void)hipStreamDestroy(own_stream);
  }
  const GateDev *d_gates = nullptr;
  const double *d_gmat = nullptr, *d_gdmat = nullptr;
  const NoiseDev *d_noise = nullptr;
  const NoiseBranch *d_ntab = nullptr;
  const double *d_ncum = nullptr;
  const OpDesc *d_ops = nullptr;
  const double *d_readout = nullptr;
  // the full-circuit amplitude network: the caller's contraction tree (SSA
  // pairs over its leaves, empty: the internal planner) and the tree used
  std::vector<Pair> user_tree;
  std::vector<std::vector<int>> full_legs;
  std::vector<Pair> full_pairs;
};

namespace {

size_t elem_bytes(int precision) { return precision == PWS_PREC_FP64 ? 16 : 8; }

// Branch sums of one noise site for every value of its true bits: the
// weights Pr(i | t) = prod_j |column t_j of M_ij|^2 (Eq. (4)) added in branch
// order, each product and sum a separate IEEE operation (no fused
// multiply-add), so that a draw against them decides exactly as summing the
// weights on the fly; then the last branch with a nonzero weight.
void branch_sums(const NoiseIR &N, std::vector<double> &out) {
#pragma clang fp contract(off)
  for (int t = 0; t < (1 << N.nq); ++t) {
    const int t0 = t & 1, t1 = (t >> 1) & 1;
    double C = 0.0;
    int last = -1;
    for (int i = 0; i < N.nbranch; ++i) {
      double v = N.tab[(size_t)i * N.nq].colnorm[t0];
      if (N.nq > 1) v = v * N.tab[(size_t)i * N.nq + 1].colnorm[t1];
      C = C + v;
      if (v > 0.0) last = i;
      out.push_back(C);
    }
    out.push_back((double)last);
  }
}

pws_status upload_tables(pws_plan_impl *P) {
  const CircuitIR &ir = P->ir;
  std::vector<GateDev> gd(ir.gates.size());
  std::vector<double> gm(ir.gates.size() * 32, 0.0), gdm(ir.gates.size() * 32, 0.0);
  for (size_t g = 0; g < ir.gates.size(); ++g) {
    const GateIR &G = ir.gates[g];
    GateDev &d = gd[g];
    d.nq = G.nq;
    d.q0 = G.q[0];
    d.q1 = G.q[1];
    d.monomial = G.monomial;
    d.diagonal = G.diagonal;
    for (int i = 0; i < 4; ++i) { d.sigma[i] = G.sigma[i]; d.cand_mask[i] = G.cand_mask[i]; }
    d.sq[0] = G.sq[0];
    d.sq[1] = G.sq[1];
    d.nS = G.nS;
    const int dd = 1 << G.nq;
    for (int e = 0; e < dd * dd; ++e) {
      gm[g * 32 + 2 * e] = G.mat[e].real();
      gm[g * 32 + 2 * e + 1] = G.mat[e].imag();
      gdm[g * 32 + 2 * e] = G.dmat[e].real();
      gdm[g * 32 + 2 * e + 1] = G.dmat[e].imag();
    }
  }
  std::vector<NoiseDev> nd(ir.noise.size());
  std::vector<NoiseBranch> nt;
  std::vector<double> ncum;
  for (size_t i = 0; i < ir.noise.size(); ++i) {
    const NoiseIR &N = ir.noise[i];
    nd[i].nq = N.nq;
    nd[i].q0 = N.q[0];
    nd[i].q1 = N.q[1];
    nd[i].nbranch = N.nbranch;
    nd[i].seg[0] = N.seg[0];
    nd[i].seg[1] = N.seg[1];
    nd[i].tab_off = (int)nt.size();
    nt.insert(nt.end(), N.tab.begin(), N.tab.end());
    nd[i].cum_off = (int)ncum.size();
    branch_sums(N, ncum);
  }
  std::vector<OpDesc> ops(ir.ops.size());
  for (size_t i = 0; i < ir.ops.size(); ++i) ops[i] = {ir.ops[i].type, ir.ops[i].idx};
  HIP_TRY(upload(P->tables, gd, &P->d_gates));
  HIP_TRY(upload(P->tables, gm, &P->d_gmat));
  HIP_TRY(upload(P->tables, gdm, &P->d_gdmat));
  HIP_TRY(upload(P->tables, nd, &P->d_noise));
  HIP_TRY(upload(P->tables, nt, &P->d_ntab));
  HIP_TRY(upload(P->tables, ncum, &P->d_ncum));
  HIP_TRY(upload(P->tables, ops, &P->d_ops));
  if (!ir.readout.empty()) HIP_TRY(upload(P->tables, ir.readout, &P->d_readout));
  return PWS_OK;
}

// Kernel records of the sweep ops for 64, 256, 512, 16 and 32 threads per chain.
void sweep_op_records(const std::vector<SweepOp> &ops, std::vector<SweepOpDev> &out) {
  const int lognth[5] = {6, 8, 9, 4, 5};
  out.assign(5 * ops.size(), SweepOpDev{});
  for (int v = 0; v < 5; ++v)
    for (size_t i = 0; i < ops.size(); ++i) {
      const SweepOp &so = ops[i];
      SweepOpDev &d = out[(size_t)v * ops.size() + i];
      const int ln = lognth[v];
      d.moff = so.moff;
      d.outer_mask = so.outer_mask;
      d.info = (so.np & 0xff) | ((so.diag & 0xff) << 8) | ((so.renorm & 0xff) << 16);
      d.pos = 0;
      for (int j = 0; j < PWS_SWEEP_MAXNP; ++j) d.pos |= (so.pos[j] & 0xff) << (8 * j);
      // thread bits go to the lowest ln positions of the outer mask
      int lo = 0, m = so.outer_mask, nb = 0;
      int shift[32], tmask[32], nterm = 0;
      for (int b = 0; b < ln && m; ++b, ++nb) {
        const int bit = m & -m;
        const int p = __builtin_ctz(bit);
        lo |= bit;
        m &= m - 1;
        const int sh = p - b;
        if (nterm == 0 || shift[nterm - 1] != sh) {
          shift[nterm] = sh;
          tmask[nterm] = 0;
          ++nterm;
        }
        tmask[nterm - 1] |= bit;
      }
      const int log_rounds = so.n_outer > ln ? so.n_outer - ln : 0;
      const int log_tg = so.n_outer < ln ? so.n_outer : ln;
      d.hi = ((so.outer_mask & ~lo) & 0xffff) | (log_rounds << 16) | (log_tg << 24);
      if (nterm > PWS_SWDEV_TERMS) {
        d.shifts = 1 << 23;
      } else {
        d.shifts = nterm << 20;
        d.mask01 = d.mask23 = 0;
        for (int j = 0; j < nterm; ++j) {
          d.shifts |= (shift[j] & 31) << (5 * j);
          if (j < 2) d.mask01 |= (tmask[j] & 0xffff) << (16 * j);
          else d.mask23 |= (tmask[j] & 0xffff) << (16 * (j - 2));
        }
      }
    }
}

// The plan's step records with their hot blocks filled in: the per-step
// fields and the gate's classification (and, for fresh steps, the gate's
// first column, which a change of parameters rewrites).
std::vector<StepDesc> hot_steps(const pws_plan_impl *P, const Programs &pr) {
  const CircuitIR &ir = P->ir;
  std::vector<StepDesc> steps = pr.steps;
  for (StepDesc &sd : steps) {
    StepHot &h = sd.hot;
    h = StepHot{};
    h.gate = sd.gate;
    h.op = sd.op;
    h.op_begin = sd.op_begin;
    h.nS = sd.nS;
    h.flags = (sd.fresh ? 1 : 0) | (sd.replay ? 2 : 0);
    if (sd.gate >= 0) {
      const GateIR &G = ir.gates[sd.gate];
      h.g_nq = G.nq;
      h.g_q0 = G.q[0];
      h.g_q1 = G.q[1];
      h.g_nS = G.nS;
      h.g_sq = G.sq[0] | (G.sq[1] << 8);
      for (int t = 0; t < 4; ++t) h.g_cand |= (G.cand_mask[t] & 0xff) << (8 * t);
    }
    h.sw_begin = sd.sw_begin;
    h.sw_count = sd.sw_count;
    h.sw_width = sd.sw_width;
    h.m_begin = sd.m_begin;
    h.m_count = sd.m_count;
    h.leaf_begin = sd.leaf_begin;
    h.load_op = sd.load_op;
    h.store_op = sd.store_op;
    h.load_w = sd.load_w;
    h.store_w = sd.store_w;
    h.snap_begin = sd.snap_begin;
    h.snap_count = sd.snap_count;
    h.merge_slot = sd.merge_slot;
    h.dn_begin = sd.dn_begin;
    h.dn_count = sd.dn_count;
    h.dn_load = sd.dn_load;
    h.dn_w = sd.dn_w;
    for (int v = 0; v < 4; ++v) h.root_index[v] = sd.root_index[v];
    h.merge_nb = sd.merge_slot >= 0 ? sd.merge_nb : 0;
    h.merge_map = sd.merge_map;
    h.merge_pack = -1;
    if (sd.merge_slot >= 0 && sd.merge_nb <= 4) {
      int pk = 0;
      bool fits = true;
      for (int k = 0; k < sd.merge_nb; ++k) {
        const int here = pr.mmap[sd.merge_map + 2 * k], kept = pr.mmap[sd.merge_map + 2 * k + 1];
        if (here > 15 || kept > 15) fits = false;
        pk |= (here | (kept << 4)) << (8 * k);
      }
      if (fits) h.merge_pack = pk;
    }
    if (sd.fresh && sd.gate >= 0) {
      const GateIR &G = ir.gates[sd.gate];
      const int dd = 1 << G.nq;
      for (int v = 0; v < 2 && v < dd; ++v) {
        h.fresh_amp[2 * v] = G.mat[v * dd].real();
        h.fresh_amp[2 * v + 1] = G.mat[v * dd].imag();
      }
    }
  }
  return steps;
}

pws_status upload_prog(pws_plan_impl *P, const Programs &pr, std::vector<std::unique_ptr<DevBuf>> &bufs,
                       DevProg &dp) {
  const CircuitIR &ir = P->ir;
  dp = DevProg{};
  {
    const std::vector<StepDesc> steps = hot_steps(P, pr);
    HIP_TRY(upload(bufs, steps, &dp.steps));
  }
  HIP_TRY(upload(bufs, pr.leaves, &dp.leaves));
  HIP_TRY(upload(bufs, pr.factors, &dp.factors));
  HIP_TRY(upload(bufs, pr.nodes, &dp.nodes));
  HIP_TRY(upload(bufs, pr.ktab, &dp.ktab));
  HIP_TRY(upload(bufs, pr.zero_q, &dp.zero_q));
  HIP_TRY(upload(bufs, pr.bnodes, &dp.bnodes));
  HIP_TRY(upload(bufs, pr.grad_terms, &dp.grad_terms));
  HIP_TRY(upload(bufs, pr.ltab, &dp.ltab));
  HIP_TRY(upload(bufs, pr.lvar, &dp.lvar));
  HIP_TRY(upload(bufs, pr.lelem, &dp.lelem));
  HIP_TRY(upload(bufs, pr.sweeps, &dp.sweeps));
  {
    std::vector<SweepOpDev> recs;
    sweep_op_records(pr.sweeps, recs);
    HIP_TRY(upload(bufs, recs, &dp.swdev));
    dp.n_sweep_ops = (int32_t)pr.sweeps.size();
  }
  HIP_TRY(upload(bufs, pr.mtab, &dp.mtab));
  HIP_TRY(upload(bufs, pr.ment, &dp.ment));
  HIP_TRY(upload(bufs, pr.snaps, &dp.snaps));
  HIP_TRY(upload(bufs, pr.mmap, &dp.mmap));
  HIP_TRY(upload(bufs, pr.mterm, &dp.mterm));
  HIP_TRY(upload(bufs, pr.mflat, &dp.mflat));
  HIP_TRY(upload(bufs, pr.druns, &dp.druns));
  HIP_TRY(upload(bufs, pr.dtab, &dp.dtab));
  dp.ops = P->d_ops;
  dp.readout = P->d_readout;
  dp.gates = P->d_gates;
  dp.noise = P->d_noise;
  dp.ntab = P->d_ntab;
  dp.ncum = P->d_ncum;
  dp.gmat = P->d_gmat;
  dp.gdmat = P->d_gdmat;
  dp.n_qubits = ir.n;
  dp.words = (ir.n + 63) / 64;
  dp.n_gates = (int)ir.gates.size();
  dp.n_segs = ir.n_segs;
  dp.n_ops = (int)ir.ops.size();
  dp.noisy = ir.noisy ? 1 : 0;
  dp.n_params = ir.n_params;
  dp.n_bnodes = (int)pr.bnodes.size();
  dp.n_grad_terms = (int)pr.grad_terms.size() / 5;
  dp.adj_root_off = pr.adj_root_off;
  return PWS_OK;
}

pws_status build_full(pws_plan_impl *P, bool backward) {
  Programs &pr = backward ? P->full_grad : P->full_amp;
  const CircuitIR &ir = P->ir;
  if (ir.gates.empty()) return fail(PWS_ERR_ARG, "empty circuit");
  StepNet net0 = build_step_net(ir, (int)ir.gates.size() - 1, {}, -1, true);
  fuse_leaves(net0, !backward);   // the adjoint keeps fixed-leg factors (their derivatives count)
  std::vector<std::vector<int>> legs;
  for (auto &l : net0.leaves) legs.push_back(l.legs);
  const bool given = !backward && !P->user_tree.empty();
  if (given && P->user_tree.size() + 1 != legs.size())
    return fail(PWS_ERR_ARG, "contraction tree does not span the amplitude network's leaves");
  // amplitudes follow the sampling form; the adjoint keeps every forward
  // tensor and runs with per-wave arenas in device memory
  PlanOptions o = P->opt;
  bool lds = !backward && P->lds_mode;
  std::string err;
  for (int pass = 0; pass < 2; ++pass) {
    if (!lds) {
      o.lds_mode = 0;
      o.arena_limit_elems = P->budget_limit;
    }
    pr = Programs();
    StepNet net = net0;
    std::vector<Pair> pairs = given ? P->user_tree : plan_tree(ir, legs, net.open_legs, o, nullptr);
    err = emit_step(ir, net, pairs, o, 0, pr, backward);
    if (!backward) {
      P->full_legs = legs;
      P->full_pairs = pairs;
    }
    if (err.empty() && lds &&
        lds_bytes_arena(P->precision, pr.max_arena, pr.max_exp) + 512 > P->lds_capacity)
      err = "arena exceeds LDS";
    if (err.empty()) break;
    if (!lds) break;
    lds = false;
  }
  if (!err.empty()) return fail(PWS_ERR_PLAN, err);
  if (!backward) P->amp_lds = lds ? 1 : 0;
  auto &bufs = backward ? P->gbufs : P->abufs;
  bufs.clear();
  pws_status st = upload_prog(P, pr, bufs, backward ? P->dp_grad : P->dp_amp);
  if (st != PWS_OK) return st;
  (backward ? P->have_grad : P->have_amp) = true;
  return PWS_OK;
}

struct Workspace {
  ChainState st{};
  void *arena = nullptr;
  int32_t *err = nullptr;
  void *cache = nullptr;        // sweep form: kept tensors, cache_stride elements per chain
  int64_t cache_stride = 0;
  int32_t *cache_exp = nullptr; // two ints per chain and slot
  int cache_slots = 1;          // slots per chain
  void *mscratch = nullptr;     // sweep form: op-matrix tables in device memory
  int64_t ms_stride = 0;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Layout of the chain state + arena for K chains and a grid of G workgroups.
// Extra device memory of sweep-form steps: the running tensor each chain keeps
// for the next step (with its exponent pair), and op-matrix tables that do
// not fit in LDS next to the tensor (per workgroup).
struct SweepNeeds {
  int cache_w = -1;          // widest kept tensor (log2 elements), -1: none
  int n_slots = 1;           // kept tensors per chain (the next step's prefix, snapshots)
  int64_t ms_elems = 0;      // matrix entries per workgroup in device memory
  int ms_grid = 0;           // workgroups of such launches
};

size_t workspace_layout(const pws_plan_impl *P, int64_t K, int G, int64_t arena_elems, const SweepNeeds &sn,
                        size_t *offs) {
  const int W = (P->ir.n + 63) / 64;
  const size_t eb = elem_bytes(P->precision);
  size_t o = 0;
  offs[0] = o; o = align256(o + (size_t)K * W * 8);                         // s
  offs[1] = o; o = align256(o + (P->ir.noisy ? (size_t)K * W * 8 : 0));     // x
  offs[2] = o; o = align256(o + (P->ir.noisy ? (size_t)K * P->ir.gates.size() : 0));  // gframe
  offs[3] = o; o = align256(o + (P->ir.noisy ? (size_t)K * P->ir.n_segs * 32 : 0));   // segfac
  offs[4] = o; o = align256(o + 64);                                                    // err
  offs[5] = o; o = align256(o + (size_t)G * kWavesPerBlock * arena_elems * eb);         // arena / wave
  offs[6] = o; o = align256(o + (sn.cache_w >= 0 ? ((size_t)K * sn.n_slots << sn.cache_w) * eb : 0));  // kept tensors
  offs[7] = o; o = align256(o + (sn.cache_w >= 0 ? (size_t)K * sn.n_slots * 8 : 0));                    // exponents
  offs[8] = o; o = align256(o + (size_t)sn.ms_grid * sn.ms_elems * eb);                     // matrix tables
  return o;
}

// The workspace's pointers inside device memory at `base` (laid out by
// workspace_layout).
void place_workspace(char *base, const size_t *offs, const SweepNeeds &sn, Workspace &w) {
  w.st.s = (uint64_t *)(base + offs[0]);
  w.st.x = (uint64_t *)(base + offs[1]);
  w.st.gframe = (uint8_t *)(base + offs[2]);
  w.st.segfac = (double *)(base + offs[3]);
  w.err = (int32_t *)(base + offs[4]);
  w.arena = base + offs[5];
  w.cache = sn.cache_w >= 0 ? base + offs[6] : nullptr;
  w.cache_stride = sn.cache_w >= 0 ? (int64_t)1 << sn.cache_w : 0;
  w.cache_exp = sn.cache_w >= 0 ? (int32_t *)(base + offs[7]) : nullptr;
  w.cache_slots = sn.n_slots;
  w.mscratch = sn.ms_elems > 0 ? base + offs[8] : nullptr;
  w.ms_stride = sn.ms_elems;
}

pws_status get_workspace(pws_plan_impl *P, int64_t K, int G, int64_t arena_elems, Workspace &w,
                         const SweepNeeds &sn = SweepNeeds()) {
  size_t offs[9];
  const size_t need = workspace_layout(P, K, G, arena_elems, sn, offs);
  char *base;
  if (P->bound) {
    if (P->bound_bytes < need) return fail(PWS_ERR_NOMEM, "bound workspace too small");
    base = (char *)P->bound;
  } else {
    if (need > P->budget)
      return fail(PWS_ERR_NOMEM, "workspace of " + std::to_string(need) + " bytes exceeds the memory budget of " +
                                     std::to_string(P->budget) + " bytes");
    const hipError_t e = P->ws_state.ensure(need);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
      (void)hipGetLastError();   // the failed allocation leaves the device usable
      return fail(PWS_ERR_NOMEM, "device allocation of " + std::to_string(need) + " bytes failed");
    }
    if (e != hipSuccess) return fail(PWS_ERR_DEVICE, std::string("workspace allocation: ") + hipGetErrorString(e));
    base = (char *)P->ws_state.p;
  }
  place_workspace(base, offs, sn, w);
  return PWS_OK;
}

// One wave per chain in flight; workgroups of kWavesPerBlock waves.
// Launch shape of a step program: LDS form (one workgroup per chain, as many
// workgroups per CU as LDS allows) or wave form (per-wave device arenas).
void launch_shape(const pws_plan_impl *P, const Programs &pr, bool lds, int64_t K, StepLaunch &L,
                  int64_t *ws_arena_elems, int *grid);
// Matrix entries a sweep-form launch needs: from the restore point on when a
// sampling pass restores the previous step's tensor, all of them otherwise.
int64_t sweep_m_entries(const Programs &pr, const StepDesc &sd, int mode, bool restore_ok = true) {
  if (mode == MODE_SAMPLE && sd.load_op >= 0 && restore_ok) {
    const int64_t m0 = sd.load_op < sd.sw_count ? pr.sweeps[(size_t)sd.sw_begin + sd.load_op].moff : sd.m_count;
    return sd.m_count - m0;
  }
  return sd.m_count;
}

// Launch shape of a sweep-form step: one workgroup per chain slot, as many per
// CU as LDS allows; four waves per chain for wide tensors.  When the step's op
// matrices do not fit in LDS next to the tensor they go to device memory
// (w.mscratch, one table per workgroup, at most 4 workgroups per CU).
// Op-matrix entries one chain's LDS slot holds: the step's whole table, or
// a window of sweep_mt_cap entries (at least the widest op's matrix) that the
// kernel rebuilds as the ops move past it.  A small window leaves the LDS to
// more resident chains: on the 6x8 grid the tables are larger than the
// running tensors for widths 9 to 11, and a 128-entry window runs the
// sampling pass a quarter faster than whole tables.
int64_t mt_window(const pws_plan_impl *P, int64_t me, int max_np) {
  if (P->sweep_mt_cap <= 0) return me;
  return std::min<int64_t>(me, std::max<int64_t>(P->sweep_mt_cap, max_np > 2 ? 256 : 16));
}

// Chains per wave for a one-wave sweep step of the given width.
int sweep_cpw(const pws_plan_impl *P, int width, int64_t K) {
  int c = width <= 8 ? P->sweep_cpw8 : width <= 10 ? P->sweep_cpw10 : 1;
  if (width <= 8 && P->sweep_cpw8_few > 0 && K <= (int64_t)P->cus * 16) c = P->sweep_cpw8_few;
  return c >= 4 ? 4 : c >= 2 ? 2 : 1;
}

// The dense-run form serves a step's launch when the plan has one for the
// step and the launch starts where its runs start: op 0, or the restore
// point of a sampling pass that restores.
int dense_mode(const pws_plan_impl *P, const Programs &pr, const StepDesc &sd, int mode, bool restore_ok) {
  if (!P->dense || &pr != &P->prog) return 0;
  // a sampling pass draws a fresh qubit's step from the gate alone (no runs)
  if (sd.fresh && mode == MODE_SAMPLE) return P->dense;
  if (sd.dn_count == 0) return 0;
  if (sd.dn_op0 == 0 || (mode == MODE_SAMPLE && restore_ok && sd.load_op == sd.dn_op0)) return P->dense;
  return 0;
}

void sweep_shape(const pws_plan_impl *P, const Programs &pr, int step, int64_t K, int mode, const Workspace *w,
                 StepLaunch &L) {
  const StepDesc &sd = pr.steps[step];
  L.sweep = 0;
  L.dense = 0;
  L.u_off = -1;
  L.mt_global = nullptr;
  L.mt_stride = 0;
  L.step_end = step + 1;
  L.range_w = sd.sw_width;
  if (!sd.sweep) return;
  L.dense = dense_mode(P, pr, sd, mode, w && w->cache);
  if (L.dense) {
    // no op matrices are built: the LDS slot holds the head and the tensor;
    // when one chain per wave would leave chains waiting for a wave, narrow
    // tensors put two chains in a wave (each run then serves both, one after
    // the other, with all 64 lanes)
    const int wpc = sd.dn_w >= P->sweep_coop8_width ? 8 : sd.dn_w >= P->sweep_coop_width ? 4 : 1;
    const int64_t resident = std::max(K, P->batch_chains);   // chains competing for the device's waves
    const int cpw = wpc == 1 && sd.dn_w <= P->dense_cpw2_width && resident > (int64_t)P->cus * P->sweep_waves_per_cu ? 2 : 1;
    L.sweep = 1 + (wpc == 4 ? 2 : wpc == 8 ? 4 : 0) + (cpw == 2 ? 16 : 0);
    L.range_w = sd.dn_w;
    L.mt_cap = 0;
    L.slot_bytes = sweep_slot_bytes(P->precision, sd.dn_w, 0);
    L.lds_bytes = lds_bytes_sweep(P->precision, sd.dn_w, 0, cpw);
    // (one-wave chains also hold a static 2 KB table buffer per chain)
    const int wg_lds = L.lds_bytes + (wpc == 1 ? cpw * kDenseTabBytes : 0);
    const int per_cu = std::max(1, std::min(P->sweep_waves_per_cu / wpc, P->lds_per_cu / wg_lds));
    L.grid = (int)std::max<int64_t>(1, std::min<int64_t>((K + cpw - 1) / cpw, (int64_t)P->cus * per_cu));
    L.block = 64 * wpc;
    L.cache = w ? w->cache : nullptr;
    L.cache_stride = w ? w->cache_stride : 0;
    L.cache_exp = w ? w->cache_exp : nullptr;
    L.cache_slots = w ? w->cache_slots : 1;
    return;
  }
  const int wpc = sd.sw_width >= P->sweep_coop8_width ? 8 : sd.sw_width >= P->sweep_coop_width ? 4 : 1;
  L.sweep = 1 + (sd.sw_max_np > 2 ? 1 : 0) + (wpc == 4 ? 2 : wpc == 8 ? 4 : 0);
  const int64_t me = mt_window(P, sweep_m_entries(pr, sd, mode, w && w->cache), sd.sw_max_np);
  L.mt_cap = (int)me;
  // several chains per wave for narrow tensors with ops of at most two positions
  int cpw = 1;
  if (wpc == 1 && sd.sw_max_np <= 2) cpw = sweep_cpw(P, sd.sw_width, K);
  L.slot_bytes = sweep_slot_bytes(P->precision, sd.sw_width, (int)me);
  L.lds_bytes = lds_bytes_sweep(P->precision, sd.sw_width, (int)me, cpw);
  if (L.lds_bytes > P->lds_capacity && cpw > 1) {
    cpw = 1;
    L.lds_bytes = lds_bytes_sweep(P->precision, sd.sw_width, (int)me, 1);
  }
  int cap = P->sweep_waves_per_cu / wpc;
  if (L.lds_bytes > P->lds_capacity) {
    L.slot_bytes = sweep_slot_bytes(P->precision, sd.sw_width, 0);
    L.lds_bytes = lds_bytes_sweep(P->precision, sd.sw_width, 0, 1);
    L.mt_global = w ? w->mscratch : nullptr;
    L.mt_stride = w ? w->ms_stride : 0;
    L.sweep += 8;
    cap = std::min(cap, 4);
  }
  if (cpw == 2) L.sweep += 16;
  if (cpw == 4) L.sweep += 32;
  const int per_cu = std::max(1, std::min(cap, P->lds_per_cu / L.lds_bytes));
  const int64_t groups = (K + cpw - 1) / cpw;
  L.grid = (int)std::max<int64_t>(1, std::min<int64_t>(groups, (int64_t)P->cus * per_cu));
  L.block = 64 * wpc;
  L.cache = w ? w->cache : nullptr;
  L.cache_stride = w ? w->cache_stride : 0;
  L.cache_exp = w ? w->cache_exp : nullptr;
  L.cache_slots = w ? w->cache_slots : 1;
}

// Consecutive narrow sweep-form steps (one wave per chain, ops of at most two
// positions) share one launch: each chain runs them in turn with its state in
// LDS.  Returns one past the last step joined to the range starting at k and
// sets the launch's LDS layout and shape for the whole range.
int sweep_range(const pws_plan_impl *P, const Programs &pr, int k, int n_steps, int64_t K, int mode,
                const Workspace *w, StepLaunch &L) {
  const StepDesc &s0 = pr.steps[k];
  if (L.dense) {
    // consecutive dense steps one wave wide share the launch; chains run
    // them in turn with their state in LDS (grid-strided over the chains)
    if (P->sweep_range_w <= 0 || (L.sweep & ~16) != 1) return k + 1;
    const int cpw = L.sweep & 16 ? 2 : 1;
    const bool restore_ok = w && w->cache;
    int wmax = s0.dn_w;
    if (wmax > P->sweep_range_w) return k + 1;
    int k1 = k + 1;
    while (k1 < n_steps && (P->dense_range_steps <= 0 || k1 - k < P->dense_range_steps)) {
      const StepDesc &sd = pr.steps[k1];
      if (!sd.sweep || dense_mode(P, pr, sd, mode, restore_ok) != L.dense) break;
      if (sd.dn_w > P->sweep_range_w || sd.dn_w >= P->sweep_coop_width) break;
      if (cpw == 2 && sd.dn_w > P->dense_cpw2_width) break;
      wmax = std::max(wmax, (int)sd.dn_w);
      ++k1;
    }
    L.step_end = k1;
    L.range_w = wmax;
    L.slot_bytes = sweep_slot_bytes(P->precision, wmax, 0);
    L.u_off = lds_bytes_sweep(P->precision, wmax, 0, cpw);   // the draw uniforms follow
    L.lds_bytes = L.u_off + kRangeUniformBytes;
    const int per_cu =
        std::max(1, std::min(P->sweep_waves_per_cu, P->lds_per_cu / (L.lds_bytes + cpw * kDenseTabBytes)));
    L.grid = (int)std::max<int64_t>(1, std::min<int64_t>((K + cpw - 1) / cpw, (int64_t)P->cus * per_cu));
    return k1;
  }
  if (!s0.sweep || P->sweep_range_w <= 0 || (L.sweep & ~48) != 1 || L.mt_global) return k + 1;
  const bool restore_ok = w && w->cache;
  int wmax = s0.sw_width;
  int k1 = k + 1;
  // chains per wave: as chosen for the widest step the range may reach
  const int cpw = sweep_cpw(P, P->sweep_range_w, K);
  // every chain of the launch resident at once (a range's chains run their
  // steps one after another, so a second round would double its time)
  const int64_t groups = (K + cpw - 1) / cpw;
  const int64_t want_per_cu = std::max<int64_t>(1, (groups + P->cus - 1) / P->cus);
  if (want_per_cu > P->sweep_waves_per_cu) return k + 1;
  const int budget = (int)(P->lds_per_cu / want_per_cu);
  int64_t mmax = mt_window(P, sweep_m_entries(pr, s0, mode, restore_ok), s0.sw_max_np);
  if (lds_bytes_sweep(P->precision, wmax, (int)mmax, cpw) + kRangeUniformBytes > budget) return k + 1;
  while (k1 < n_steps) {
    const StepDesc &sd = pr.steps[k1];
    if (!sd.sweep || sd.sw_max_np > 2 || sd.sw_width > P->sweep_range_w || sd.sw_width >= P->sweep_coop_width) break;
    const int w2 = std::max(wmax, sd.sw_width);
    const int64_t m2 = std::max(mmax, mt_window(P, sweep_m_entries(pr, sd, mode, restore_ok), sd.sw_max_np));
    if (lds_bytes_sweep(P->precision, w2, (int)m2, cpw) + kRangeUniformBytes > budget) break;
    wmax = w2;
    mmax = m2;
    ++k1;
  }
  if (k1 == k + 1) return k1;
  if (s0.sw_width > P->sweep_range_w) return k + 1;
  L.step_end = k1;
  L.range_w = wmax;
  L.sweep = 1 + (cpw == 2 ? 16 : cpw == 4 ? 32 : 0);
  L.slot_bytes = sweep_slot_bytes(P->precision, wmax, (int)mmax);
  L.u_off = lds_bytes_sweep(P->precision, wmax, (int)mmax, cpw);   // the draw uniforms follow
  L.lds_bytes = L.u_off + kRangeUniformBytes;
  L.mt_cap = (int)mmax;
  const int per_cu = std::max(1, std::min(P->sweep_waves_per_cu, P->lds_per_cu / L.lds_bytes));
  L.grid = (int)std::max<int64_t>(1, std::min<int64_t>(groups, (int64_t)P->cus * per_cu));
  return k1;
}

// Device memory the sweep-form launches of a program need.
SweepNeeds sweep_needs(const pws_plan_impl *P, const Programs &pr, int64_t K, int mode, int step_only) {
  SweepNeeds sn;
  for (int k = 0; k < (int)pr.steps.size(); ++k) {
    if (step_only >= 0 && k != step_only) continue;
    const StepDesc &sd = pr.steps[k];
    if (!sd.sweep) continue;
    if (mode == MODE_SAMPLE && sd.store_op >= 0) sn.cache_w = std::max(sn.cache_w, sd.store_w);
    if (mode == MODE_SAMPLE && sd.snap_count > 0) {
      for (int i = 0; i < sd.snap_count; ++i) sn.cache_w = std::max(sn.cache_w, pr.snaps[sd.snap_begin + i].w);
      sn.n_slots = std::max(sn.n_slots, pr.n_slots);
    }
    const int64_t me = sweep_m_entries(pr, sd, mode);
    if (lds_bytes_sweep(P->precision, sd.sw_width, (int)mt_window(P, me, sd.sw_max_np)) > P->lds_capacity) {
      sn.ms_elems = std::max(sn.ms_elems, me);
      sn.ms_grid = (int)std::max<int64_t>(sn.ms_grid, std::min<int64_t>(K, (int64_t)P->cus * 4));
    }
  }
  return sn;
}

int choose_grid(const pws_plan_impl *P, int64_t K) {
  const int64_t wgs = (K + kWavesPerBlock - 1) / kWavesPerBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(wgs, P->grid_max));
}

void launch_shape(const pws_plan_impl *P, const Programs &pr, bool lds, int64_t K, StepLaunch &L,
                  int64_t *ws_arena_elems, int *grid) {
  if (lds) {
    L.lds_arena = 1;
    L.arena_stride = std::max(pr.max_arena, 2);
    L.n_exp = std::max(pr.max_exp, 1);
    L.lds_bytes = lds_bytes_arena(P->precision, (int)L.arena_stride, L.n_exp);
    const int per_cu = std::max(1, P->lds_capacity / (L.lds_bytes + 512));
    L.grid = (int)std::max<int64_t>(1, std::min<int64_t>(K, (int64_t)P->cus * per_cu));
    L.block = P->block;
    *ws_arena_elems = 0;
  } else {
    L.lds_arena = 0;
    L.arena_stride = std::max(pr.max_arena, 2);
    L.lds_bytes = lds_bytes_for(std::max(pr.max_exp, 1));
    L.grid = choose_grid(P, K);
    L.block = 256;
    *ws_arena_elems = L.arena_stride;
  }
  *grid = L.grid;
}

pws_status check_bits(const pws_plan_impl *P, const pws_bits *b, int64_t need) {
  if (P->host_only) return fail(PWS_ERR_DEVICE, "host-only plan: no device tables");
  if (!b || !b->data) return fail(PWS_ERR_ARG, "bits struct or data is NULL");
  if (b->words != (P->ir.n + 63) / 64) return fail(PWS_ERR_ARG, "bits.words must be ceil(n_qubits/64)");
  if (b->n < need) return fail(PWS_ERR_ARG, "bits.n too small");
  return PWS_OK;
}

pws_status read_err(pws_plan_impl *P, int32_t *derr) {
  int32_t h = 0;
  HIP_TRY(hipMemcpyAsync(&h, derr, 4, hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  if (h & 1) return fail(PWS_ERR_NUMERIC, "zero-mass block reached (all candidate amplitudes zero)");
  if (h & 2) return fail(PWS_ERR_NUMERIC, "noise site with zero total branch probability");
  if (h & 4) return fail(PWS_ERR_NUMERIC, "zero amplitude for a gradient sample");
  return PWS_OK;
}

// One sampling pass of K chains (global ids base..base+K-1) on stream s:
// state init, the step launches, finalize into dst.  The seed is read from
// seed_ptr (device) when it is set.
pws_status enqueue_pass(pws_plan_impl *P, const StepLaunch &L0, const Workspace &w, int64_t K, int64_t base,
                        uint64_t seed, const uint64_t *seed_ptr, uint64_t *dst, hipStream_t s, int *launched) {
  const int n_steps = (int)P->prog.steps.size();
  *launched = 0;
  HIP_TRY(launch_init_state(P->dp, w.st, K, s));
  for (int k = 0; k < n_steps;) {
    StepLaunch L = L0;
    L.step = k;
    L.n_chains = K;
    L.chain_offset = base;
    L.seed = seed;
    L.seed_ptr = seed_ptr;
    L.arena = w.arena;
    L.mode = MODE_SAMPLE;
    L.trace = nullptr;
    L.trace_row = k;
    L.err = w.err;
    sweep_shape(P, P->prog, k, K, MODE_SAMPLE, &w, L);
    const int k1 = sweep_range(P, P->prog, k, n_steps, K, MODE_SAMPLE, &w, L);
    HIP_TRY(launch_step(P->precision, P->dp, w.st, L, s));
    ++*launched;
    k = k1;
  }
  HIP_TRY(launch_finalize(P->dp, w.st, K, dst, s, seed, seed_ptr, base, true));
  return PWS_OK;
}

pws_status err_flags(int32_t h) {
  if (h & 1) return fail(PWS_ERR_NUMERIC, "zero-mass block reached (all candidate amplitudes zero)");
  if (h & 2) return fail(PWS_ERR_NUMERIC, "noise site with zero total branch probability");
  return PWS_OK;
}

pws_status run_sample(pws_plan_t P, int64_t n_chains, uint64_t seed, pws_bits *out) {
  if (!P) return fail(PWS_ERR_ARG, "plan is NULL");
  if (n_chains < 0) return fail(PWS_ERR_ARG, "n_chains < 0");
  pws_status st = check_bits(P, out, n_chains);
  if (st != PWS_OK) return st;
  if (n_chains == 0) return PWS_OK;
  HIP_TRY(hipSetDevice(P->device));
  const int W = (P->ir.n + 63) / 64;
  const int64_t chunk = P->max_chains > 0 ? std::min<int64_t>(P->max_chains, n_chains) : n_chains;
  // a null stream means the legacy default stream; captures need a real one,
  // so the plan owns a (blocking, default-priority) stream for that case
  if (!P->stream && !P->own_stream) HIP_TRY(hipStreamCreate(&P->own_stream));
  hipStream_t s = P->stream ? P->stream : P->own_stream;
  const bool graph = P->use_graph && chunk == n_chains;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  double total_ms = 0;
  int launches = 0;
  for (int64_t base = 0; base < n_chains; base += chunk) {
    const int64_t K = std::min(chunk, n_chains - base);
    StepLaunch L0{};
    int64_t ws_arena = 0;
    int G = 0;
    launch_shape(P, P->prog, P->lds_mode, K, L0, &ws_arena, &G);
    Workspace w;
    st = get_workspace(P, K, G, ws_arena, w, sweep_needs(P, P->prog, K, MODE_SAMPLE, -1));
    if (st != PWS_OK) return st;
    uint64_t *dst;
    if (out->on_device) {
      dst = out->data + base * W;
    } else {
      HIP_TRY(P->ws_io.ensure((size_t)K * W * 8));
      dst = (uint64_t *)P->ws_io.p;
    }
    int launched = 0;
    auto enqueue = [&](const uint64_t *seed_ptr) -> pws_status {
      return enqueue_pass(P, L0, w, K, base, seed, seed_ptr, dst, s, &launched);
    };
    HIP_TRY(hipMemsetAsync(w.err, 0, 4, s));
    if (graph) {
      HIP_TRY(P->seed_buf.ensure(8));
      HIP_TRY(hipMemcpyAsync(P->seed_buf.p, &seed, 8, hipMemcpyHostToDevice, s));
      const bool same = P->gexec && P->g_K == K && P->g_state == (const void *)w.st.s &&
                        P->g_arena == w.arena && P->g_out == (const void *)dst && P->g_stream == s;
      if (!same) {
        if (P->gexec) { (void)hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
        hipGraph_t g;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        pws_status cs = enqueue((const uint64_t *)P->seed_buf.p);
        hipError_t ee = hipStreamEndCapture(s, &g);
        if (cs != PWS_OK) return cs;
        if (ee != hipSuccess) return fail(PWS_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(ee));
        hipError_t ie = hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return fail(PWS_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
        P->g_K = K; P->g_state = w.st.s; P->g_arena = w.arena; P->g_out = dst; P->g_stream = s;
        P->g_launches = launched;
      }
      launched = P->g_launches;
      HIP_TRY(hipEventRecord(e0, s));
      HIP_TRY(hipGraphLaunch(P->gexec, s));
      HIP_TRY(hipEventRecord(e1, s));
    } else {
      HIP_TRY(hipEventRecord(e0, s));
      st = enqueue(nullptr);
      if (st != PWS_OK) return st;
      HIP_TRY(hipEventRecord(e1, s));
    }
    launches += launched;
    if (!out->on_device)
      HIP_TRY(hipMemcpyAsync(out->data + base * W, dst, (size_t)K * W * 8, hipMemcpyDeviceToHost, s));
    {
      int32_t h = 0;
      HIP_TRY(hipMemcpyAsync(&h, w.err, 4, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      st = err_flags(h);
      if (st != PWS_OK) return st;
    }
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    total_ms += ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P->last_ms = total_ms;
  P->last_launches = launches;
  return PWS_OK;
}

// One step per non-monomial gate (Algorithm 1), trailing ops in an epilogue.
// Consecutive sweep-form steps are planned one ahead: a step is emitted once
// the next one has decided how many of its leading leaves it restores from it.
std::string plan_steps_once(const CircuitIR &ir, const PlanOptions &opt, Programs &prog) {
  int op_begin = 0;
  SweepPlan pending;
  bool have_pending = false;
  auto flush = [&]() -> std::string {
    if (!have_pending) return "";
    have_pending = false;
    return emit_sweep_plan(ir, pending, opt, prog);
  };
  // the steps (non-monomial gates) in order
  std::vector<int> step_ops;
  for (size_t op = 0; op < ir.ops.size(); ++op)
    if (ir.ops[op].type == 0 && !ir.gates[ir.ops[op].idx].monomial) step_ops.push_back((int)op);
  // first step after step t at which each chain bit / noise record differs
  // from its value at step t (its qubit sampled, flipped or opened)
  auto first_dirty = [&](int t, std::vector<int> &fq, std::vector<int> &fs) {
    fq.assign(ir.n, INT_MAX);
    fs.assign(ir.n_segs, INT_MAX);
    const int t_end = std::min((int)step_ops.size(), t + 1 + opt.sweep_anchor_horizon);
    for (int u = t; u < t_end; ++u) {
      const GateIR &G = ir.gates[ir.ops[step_ops[u]].idx];
      for (int k = 0; k < G.nS; ++k) {
        const int q = G.q[G.sq[k]];
        fq[q] = std::min(fq[q], u == t ? t + 1 : u);
      }
      const int o_end = u + 1 < (int)step_ops.size() ? step_ops[u + 1] : (int)ir.ops.size();
      for (int o = step_ops[u] + 1; o < o_end; ++o) {
        const OpIR &x = ir.ops[o];
        if (x.type == 0) {
          const GateIR &XG = ir.gates[x.idx];
          if (XG.monomial && !XG.diagonal)
            for (int j = 0; j < XG.nq; ++j) fq[XG.q[j]] = std::min(fq[XG.q[j]], u + 1);
        } else {
          const NoiseIR &N = ir.noise[x.idx];
          for (int j = 0; j < N.nq; ++j) {
            fq[N.q[j]] = std::min(fq[N.q[j]], u + 1);
            fs[N.seg[j]] = std::min(fs[N.seg[j]], u + 1);
          }
        }
      }
    }
  };
  auto leaf_first_dirty = [&](const StepNet &net, const std::vector<int> &fq, const std::vector<int> &fs) {
    std::vector<int> out(net.leaves.size(), INT_MAX);
    for (size_t i = 0; i < net.leaves.size(); ++i)
      for (const FactorDesc &f : net.leaves[i].factors) {
        if (f.kind == FAC_SEGFAC && f.id < (int)fs.size()) out[i] = std::min(out[i], fs[f.id]);
        for (int j = 0; j < f.nq; ++j)
          for (int32_t src : {f.src_out[j], f.src_in[j]})
            if (src_type(src) == SRC_CHAIN) out[i] = std::min(out[i], fq[src_payload(src)]);
      }
    return out;
  };
  std::shared_ptr<AnchorState> anchor;
  for (int t = 0; t < (int)step_ops.size(); ++t) {
    const int op = step_ops[t];
    const int g = ir.ops[op].idx;
    const GateIR &G = ir.gates[g];
    std::vector<int> S;
    for (int k = 0; k < G.nS; ++k) S.push_back(G.q[G.sq[k]]);
    StepNet net = build_step_net(ir, g, S, (int)op, false);
    fuse_leaves(net);
    if (opt.sweep_max_width > 0) {
      // chain bits and noise records that change between the pending step and this one
      std::vector<char> dirty_q(ir.n, 0), dirty_seg(ir.n_segs, 0);
      if (have_pending) {
        const GateIR &PG = ir.gates[pending.net.gate];
        for (int k = 0; k < PG.nS; ++k) dirty_q[PG.q[PG.sq[k]]] = 1;
        for (int o = pending.net.op + 1; o < (int)op; ++o) {
          const OpIR &x = ir.ops[o];
          if (x.type == 0) {
            const GateIR &XG = ir.gates[x.idx];
            if (XG.monomial && !XG.diagonal)
              for (int j = 0; j < XG.nq; ++j) dirty_q[XG.q[j]] = 1;
          } else {
            const NoiseIR &N = ir.noise[x.idx];
            for (int j = 0; j < N.nq; ++j) {
              dirty_q[N.q[j]] = 1;
              dirty_seg[N.seg[j]] = 1;
            }
          }
        }
      }
      if (anchor) {
        for (int q = 0; q < ir.n; ++q) anchor->dirty_q[q] |= dirty_q[q];
        for (int sg = 0; sg < ir.n_segs; ++sg) anchor->dirty_seg[sg] |= dirty_seg[sg];
      }
      const SweepPlan *prev = have_pending ? &pending : nullptr;
      // one-sided plan: the leading leaves restored from the previous step
      SweepPlan sp;
      std::string perr = plan_sweep(ir, net, opt, op_begin, prev, dirty_q, dirty_seg, sp);
      const int L = (int)net.leaves.size();
      double cost = perr.empty() ? sp.run_cost : 1e300;
      // two-sided plan: the current anchor's snapshot contracted with a sweep of
      // the other leaves
      if (anchor && opt.sweep_merge && opt.sweep_cache) {
        SweepPlan probe;
        if (sweep_setup(ir, net, op_begin, probe).empty()) {
          std::vector<char> usable(L, 1), forbid(ir.n_segs, 0);
          for (int l : net.open_legs) forbid[l] = 1;
          PrefixMatch pm = match_prefix(anchor->plan, probe, usable, anchor->dirty_q, anchor->dirty_seg, forbid);
          int best_s = -1;
          for (int si = 0; si < (int)anchor->snaps.size(); ++si) {
            const int j = anchor->snaps[si].j;
            if (j <= (int)pm.mapped.size() && pm.valid[j] && j >= opt.sweep_merge_min &&
                (best_s < 0 || j > anchor->snaps[best_s].j))
              best_s = si;
          }
          if (best_s >= 0) {
            const int j = anchor->snaps[best_s].j;
            std::vector<char> swept(L, 1);
            for (int k2 = 0; k2 < j; ++k2) swept[pm.mapped[k2]] = 0;
            // legs of the snapshot's leaves with holders among the swept ones
            std::vector<int> hold(ir.n_segs, 0), in_r(ir.n_segs, 0);
            for (int i = 0; i < L; ++i)
              for (int l : net.leaves[i].legs) {
                ++hold[l];
                if (!swept[i]) ++in_r[l];
              }
            std::vector<int> bound;
            for (int l = 0; l < ir.n_segs; ++l)
              if (in_r[l] > 0 && in_r[l] < hold[l]) bound.push_back(l);
            SweepPlan mp;
            if (plan_sweep(ir, net, opt, op_begin, prev, dirty_q, dirty_seg, mp, &swept, &bound).empty()) {
              // the contraction reads both tensors once per candidate
              const double mcost = mp.run_cost + std::ldexp(1.0 + (1 << net.open_legs.size()), (int)bound.size());
              if (mcost < cost) {
                mp.merge_from = anchor;
                mp.merge_snap = best_s;
                sp = std::move(mp);
                perr.clear();
                cost = mcost;
              }
            }
          }
        }
      }
      // a new anchor where neither restores much: its snapshots serve the next steps
      if (opt.sweep_merge && opt.sweep_cache && !sp.merge_from && (perr.empty() ? sp.load_n * 4 < L : true)) {
        std::vector<int> fq, fs;
        first_dirty(t, fq, fs);
        const std::vector<int> ld = leaf_first_dirty(net, fq, fs);
        SweepPlan ap;
        double benefit = 0;
        // worth it when later steps skip more than twice what the anchor runs
        // beyond the one-sided plan
        if (plan_anchor(ir, net, opt, op_begin, ld, t, ap, &benefit).empty() && !ap.anchor->snaps.empty() &&
            benefit >= 2.0 * std::max(ap.run_cost - (perr.empty() ? sp.run_cost : 0.0), ap.run_cost * 0.25)) {
          sp = std::move(ap);
          perr.clear();
          anchor = sp.anchor;
          anchor->plan = sp;
          anchor->plan.anchor = nullptr;
          anchor->dirty_q.assign(ir.n, 0);
          anchor->dirty_seg.assign(ir.n_segs, 0);
        }
      }
      if (perr.empty()) {
        if (have_pending) {
          pending.store_n = sp.load_n;
          std::string err = flush();
          if (!err.empty()) return err;
        }
        pending = std::move(sp);
        have_pending = true;
        op_begin = (int)op + 1;
        continue;
      }
    }
    std::string err = flush();
    if (!err.empty()) return err;
    anchor = nullptr;
    std::vector<std::vector<int>> legs;
    for (auto &l : net.leaves) legs.push_back(l.legs);
    std::vector<Pair> pairs = plan_tree(ir, legs, net.open_legs, opt, nullptr);
    err = emit_step(ir, net, pairs, opt, op_begin, prog, false);
    if (!err.empty()) return err;
    op_begin = (int)op + 1;
  }
  {
    std::string err = flush();
    if (!err.empty()) return err;
  }
  StepDesc sd{};
  sd.op = -1;
  sd.gate = -1;
  sd.op_begin = op_begin;
  sd.leaf_begin = (int)prog.leaves.size();
  sd.node_begin = (int)prog.nodes.size();
  sd.root_exp = -1;
  sd.zero_q_begin = (int)prog.zero_q.size();
  prog.steps.push_back(sd);
  // prologues replay the ops between steps only where one of them acts on the chain
  for (StepDesc &st : prog.steps) {
    const int op_end = st.op >= 0 ? st.op : (int)ir.ops.size();
    st.replay = 0;
    for (int o = st.op_begin; o < op_end; ++o) {
      const OpIR &x = ir.ops[o];
      if (x.type != 0 || ir.noisy) st.replay = 1;
      else if (ir.gates[x.idx].monomial && !ir.gates[x.idx].diagonal) st.replay = 1;
    }
  }
  // one-qubit gates on qubits no earlier gate touched
  std::vector<char> touched(ir.n, 0);
  size_t next = 0;
  for (StepDesc &st : prog.steps) {
    st.fresh = 0;
    if (st.gate < 0) continue;
    for (; next < (size_t)st.gate; ++next)
      for (int j = 0; j < ir.gates[next].nq; ++j) touched[ir.gates[next].q[j]] = 1;
    const GateIR &G = ir.gates[st.gate];
    if (opt.fresh_steps && G.nq == 1 && !touched[G.q[0]] && st.store_op < 0 && st.snap_count == 0) st.fresh = 1;
  }
  flatten_mtab(prog);
  return "";
}

// Steps of a plan.  Two-sided steps (an anchor step's kept tensors contracted
// with a sweep of the other leaves) pay off on some layouts and not on
// others: when the plan has any, the one-sided plan is made as well and the
// one whose sampling pass touches fewer tensor elements is kept.
std::string plan_steps(const CircuitIR &ir, const PlanOptions &opt, Programs &prog) {
  std::string err = plan_steps_once(ir, opt, prog);
  if (!err.empty() || !opt.sweep_merge) return err;
  bool any = false;
  for (const StepDesc &sd : prog.steps) any |= sd.sweep && (sd.merge_slot >= 0 || sd.snap_count > 0);
  if (!any) return "";
  PlanOptions o = opt;
  o.sweep_merge = 0;
  Programs one;
  if (!plan_steps_once(ir, o, one).empty()) return "";
  bool merges = false;
  for (const StepDesc &sd : prog.steps) merges |= sd.sweep && sd.merge_slot >= 0;
  if (opt.sweep_merge == 1 && (!merges || one.sweep_elems_per_sample <= prog.sweep_elems_per_sample))
    prog = std::move(one);
  return "";
}

}  // namespace

extern "C" {

const char *pws_last_error(void) { return g_last_error.c_str(); }

pws_status pws_plan(const pws_circuit *circuit, const pws_noise *noise, const pws_tree *tree,
                    const pws_slices *slices, pws_plan_t *out) {
  if (!out) return fail(PWS_ERR_ARG, "out is NULL");
  *out = nullptr;
  std::unique_ptr<pws_plan_impl> P(new pws_plan_impl());
  static std::atomic<uint64_t> next_uid{1};
  P->uid = next_uid++;
  // plan options: (key, value) pairs of pws_slices
  std::map<int, int> opts;
  if (slices && slices->n_options > 0) {
    if (!slices->options) return fail(PWS_ERR_ARG, "plan options without a list");
    for (int i = 0; i < slices->n_options; ++i) {
      const int k = slices->options[i].key;
      if (k < PWS_OPT_GRID || k > PWS_OPT_DENSE_CPW2_WIDTH) return fail(PWS_ERR_ARG, "unknown plan option " + std::to_string(k));
      opts[k] = slices->options[i].value;
    }
  }
  auto has_opt = [&](int k) { return opts.count(k) > 0; };
  auto opt_val = [&](int k) { return opts.at(k); };
  std::string err = lower(circuit, noise, P->ir);
  if (!err.empty()) {
    const bool unsup = err.find("unsupported") != std::string::npos || err.find("unknown") != std::string::npos;
    return fail(unsup ? PWS_ERR_UNSUPPORTED : PWS_ERR_ARG, err);
  }
  if (P->ir.n > 64 * 16) return fail(PWS_ERR_UNSUPPORTED, "more than 1024 qubits");
  {
    uint64_t hsh = 1469598103934665603ull;
    auto mix = [&](const void *d, size_t n) {
      const unsigned char *b = (const unsigned char *)d;
      for (size_t i = 0; i < n; ++i) { hsh ^= b[i]; hsh *= 1099511628211ull; }
    };
    mix(&circuit->n_qubits, 4);
    for (int i = 0; i < circuit->n_gates; ++i) {
      const pws_gate &g = circuit->gates[i];
      mix(&g.kind, 16); mix(&g.coeff, 16); mix(&g.param2, 4); mix(&g.coeff2, 16);
    }
    mix(circuit->theta, sizeof(double) * circuit->n_params);
    if (noise) for (int i = 0; i < noise->n_sites; ++i) mix(&noise->sites[i], sizeof(pws_noise_site));
    if (noise && noise->readout) mix(noise->readout, sizeof(double) * circuit->n_qubits);
    P->plan_hash = hsh;
  }
  if (tree && tree->n_pairs > 0) {
    if (!tree->ssa_pairs) return fail(PWS_ERR_ARG, "contraction tree without pairs");
    for (int i = 0; i < tree->n_pairs; ++i) P->user_tree.push_back({tree->ssa_pairs[2 * i], tree->ssa_pairs[2 * i + 1]});
  }
  if (slices) {
    if (slices->precision < PWS_PREC_FP64 || slices->precision > PWS_PREC_BF16X3)
      return fail(PWS_ERR_ARG, "unknown precision");
    P->requested_precision = slices->precision;
    if (slices->precision == PWS_PREC_BF16X3) {
      P->precision = PWS_PREC_FP32;
      P->dense = 2;
    } else {
      P->precision = slices->precision;
      if ((slices->flags & PWS_PLAN_DENSE) && slices->precision == PWS_PREC_FP32) P->dense = 1;
    }
    P->plan_hash ^= (uint64_t)slices->precision * 0x9E3779B97F4A7C15ull;
    if (slices->hbm_budget_bytes) P->budget = slices->hbm_budget_bytes;
    P->max_chains = slices->max_chains;
    P->opt.planner = slices->planner;
    P->host_only = (slices->flags & PWS_PLAN_HOST_ONLY) != 0;
    if (slices->n_sliced < 0 || (slices->n_sliced > 0 && !slices->sliced_edges))
      return fail(PWS_ERR_ARG, "bad sliced legs");
    for (int i = 0; i < slices->n_sliced; ++i) P->opt.forced_slices.push_back(slices->sliced_edges[i]);
  }
  if (has_opt(PWS_OPT_GRID)) P->grid_max = std::max(1, opt_val(PWS_OPT_GRID));
  if (!P->host_only) {
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) P->device = dev;
    int cus = 0;
    if (!has_opt(PWS_OPT_GRID) &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device) == hipSuccess && cus > 0)
      P->grid_max = cus * 4;   // 16 waves (chains) per CU
  }
  P->opt.arena_limit_elems =
      std::max<uint64_t>(64, P->budget / ((uint64_t)P->grid_max * kWavesPerBlock * elem_bytes(P->precision)) / 2);
  compute_qubit_orders(P->ir);
  for (int l : P->opt.forced_slices)
    if (l < 0 || l >= P->ir.n_segs) return fail(PWS_ERR_ARG, "sliced leg out of range (a segment id)");
  if (!P->user_tree.empty()) {
    // an SSA sequence over the full-circuit amplitude network: every id a
    // leaf or an earlier result, each used once, one root at the end
    StepNet net = build_step_net(P->ir, (int)P->ir.gates.size() - 1, {}, -1, true);
    fuse_leaves(net);
    const int L = (int)net.leaves.size();
    if ((int)P->user_tree.size() != L - 1)
      return fail(PWS_ERR_ARG, "contraction tree needs " + std::to_string(L - 1) + " pairs over the " +
                                   std::to_string(L) + " leaves of the amplitude network (pws_plan_export, step -1)");
    std::vector<char> used(2 * L, 0);
    for (int i = 0; i < (int)P->user_tree.size(); ++i) {
      const Pair &pr = P->user_tree[i];
      if (pr.a < 0 || pr.b < 0 || pr.a >= L + i || pr.b >= L + i || pr.a == pr.b || used[pr.a] || used[pr.b])
        return fail(PWS_ERR_ARG, "contraction tree pair " + std::to_string(i) + " is not in SSA form");
      used[pr.a] = used[pr.b] = 1;
    }
  }
  // sweep form: running tensors up to 2^13 (FP32) / 2^12 (FP64) elements, 64 KB of LDS
  P->opt.sweep_max_width = P->precision == PWS_PREC_FP64 ? 12 : 13;
  if (has_opt(PWS_OPT_SWEEP_WIDTH)) P->opt.sweep_max_width = std::max(0, std::min(PWS_SWEEP_MAXW, opt_val(PWS_OPT_SWEEP_WIDTH)));
  if (!P->host_only) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, P->device) == hipSuccess && v > 0)
      P->lds_capacity = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, P->device) == hipSuccess && v > 0)
      P->cus = v;
  }
  if (has_opt(PWS_OPT_GRAPH)) P->use_graph = opt_val(PWS_OPT_GRAPH) != 0;
  // Noiseless FP32 plans: steps of up to 2^10 elements join the narrow
  // launches at two chains per wave.  Noisy plans keep them at one chain per
  // wave (each chain's matrix window holds entries that read its noise
  // record, and building it on half as many lanes costs more than the shared
  // wave saves), and so do FP64 plans (twice the LDS per chain, fewer
  // resident waves).
  if (!P->ir.noisy && P->precision == PWS_PREC_FP32) {
    P->sweep_range_w = 10;
    P->sweep_cpw10 = 2;
  }
  // Noisy plans run narrow tensors at one chain per wave when every chain's
  // wave is resident at once: the matrix windows they build per chain take
  // most of those launches, and more lanes per chain build them sooner.
  if (P->ir.noisy) P->sweep_cpw8_few = 1;
  if (has_opt(PWS_OPT_LDS_BLOCK)) P->block = std::max(64, std::min(1024, opt_val(PWS_OPT_LDS_BLOCK)));
  if (has_opt(PWS_OPT_LDS_BYTES)) P->lds_capacity = std::max(4096, std::min(P->lds_capacity, opt_val(PWS_OPT_LDS_BYTES)));
  if (has_opt(PWS_OPT_WAVES_PER_CU)) P->sweep_waves_per_cu = std::max(1, std::min(64, opt_val(PWS_OPT_WAVES_PER_CU)));
  if (has_opt(PWS_OPT_COOP4_WIDTH)) P->sweep_coop_width = std::max(0, std::min(64, opt_val(PWS_OPT_COOP4_WIDTH)));
  if (has_opt(PWS_OPT_COOP8_WIDTH)) P->sweep_coop8_width = std::max(0, std::min(64, opt_val(PWS_OPT_COOP8_WIDTH)));
  if (has_opt(PWS_OPT_RANGE_WIDTH)) P->sweep_range_w = std::max(0, std::min(PWS_SWEEP_MAXW, opt_val(PWS_OPT_RANGE_WIDTH)));
  if (has_opt(PWS_OPT_CPW8)) {
    P->sweep_cpw8 = opt_val(PWS_OPT_CPW8);
    P->sweep_cpw8_few = 0;
  }
  if (has_opt(PWS_OPT_CPW10)) P->sweep_cpw10 = opt_val(PWS_OPT_CPW10);
  if (has_opt(PWS_OPT_WINDOW)) P->sweep_mt_cap = std::max(0, opt_val(PWS_OPT_WINDOW));
  P->lds_per_cu = P->lds_capacity;
  P->opt.sweep_lds_bytes = P->lds_capacity;
  if (has_opt(PWS_OPT_FUSE)) P->opt.sweep_fuse = opt_val(PWS_OPT_FUSE) != 0;
  if (has_opt(PWS_OPT_KEEP)) P->opt.sweep_cache = opt_val(PWS_OPT_KEEP) != 0;
  if (has_opt(PWS_OPT_FRESH)) P->opt.fresh_steps = opt_val(PWS_OPT_FRESH) != 0;
  if (has_opt(PWS_OPT_MERGE)) P->opt.sweep_merge = std::max(0, std::min(2, opt_val(PWS_OPT_MERGE)));
  if (has_opt(PWS_OPT_DENSE_RANGE)) P->dense_range_steps = std::max(0, opt_val(PWS_OPT_DENSE_RANGE));
  if (has_opt(PWS_OPT_DENSE_CPW2_WIDTH)) P->dense_cpw2_width = opt_val(PWS_OPT_DENSE_CPW2_WIDTH);
  P->opt.precision = P->precision;
  // LDS form first: slice every step until its arena fits on chip; fall back
  // to per-wave arenas in device memory when that multiplies the work too much.
  const uint64_t budget_limit = P->opt.arena_limit_elems;
  P->budget_limit = budget_limit;
  std::string perr;
  bool lds_ok = false;
  const int eb = (int)elem_bytes(P->precision);
  // the LDS form is chosen when asked for (PWS_FORM=lds) or by pws_autotune
  if (has_opt(PWS_OPT_LDS_FORM) && opt_val(PWS_OPT_LDS_FORM) != 0) {
    int reserve = 4096;
    for (int attempt = 0; attempt < 4 && !lds_ok; ++attempt) {
      PlanOptions o = P->opt;
      o.lds_mode = 1;
      o.arena_limit_elems = (uint64_t)std::max(64, (P->lds_capacity - 512 - reserve) / eb);
      Programs pr;
      perr = plan_steps(P->ir, o, pr);
      if (!perr.empty()) break;
      const int need = lds_bytes_arena(P->precision, pr.max_arena, pr.max_exp) + 512;
      if (need > P->lds_capacity) { reserve += need - P->lds_capacity + 1024; continue; }
      if (pr.flops_executed > 16.0 * pr.flops_per_sample) break;   // slicing blew the work up
      P->prog = std::move(pr);
      P->opt = o;
      lds_ok = true;
    }
  }
  P->lds_mode = lds_ok ? 1 : 0;
  if (!lds_ok) {
    P->opt.lds_mode = 0;
    P->opt.arena_limit_elems = budget_limit;
    P->prog = Programs();
    perr = plan_steps(P->ir, P->opt, P->prog);
    if (!perr.empty())
      return fail(perr.find("memory") != std::string::npos ? PWS_ERR_NOMEM : PWS_ERR_PLAN, perr);
  }
  // dense runs for the noiseless sweep steps (every op when the tables stay
  // within 256 MiB, else the ops sampling passes run; at most 4 GiB)
  if (P->dense) build_dense(P->prog, P->dense == 2, 256ull << 20, 4ull << 30);
  if (!P->host_only) {
    HIP_TRY(hipSetDevice(P->device));
    // the static workspace's address on this device, looked up once per
    // device (a failure here only disables pws_sample_noalloc, which reports it)
    {
      void *sp = nullptr;
      size_t sb = 0;
      (void)scratch_region(P->device, &sp, &sb);
    }
    pws_status st = upload_tables(P.get());
    if (st != PWS_OK) return st;
    st = upload_prog(P.get(), P->prog, P->pbufs, P->dp);
    if (st != PWS_OK) return st;
  }
  *out = P.release();
  return PWS_OK;
}

void pws_destroy(pws_plan_t plan) { delete plan; }

pws_status pws_set_stream(pws_plan_t P, void *hip_stream) {
  if (!P) return fail(PWS_ERR_ARG, "plan is NULL");
  P->stream = (hipStream_t)hip_stream;
  return PWS_OK;
}

pws_status pws_workspace_bytes(pws_plan_t P, int64_t n_chains, uint64_t *bytes) {
  if (!P || !bytes || n_chains < 0) return fail(PWS_ERR_ARG, "bad argument");
  const int64_t K = P->max_chains > 0 ? std::min<int64_t>(P->max_chains, n_chains) : n_chains;
  size_t offs[9];
  StepLaunch L{};
  int64_t ws_arena = 0;
  int G = 0;
  const int64_t K1 = std::max<int64_t>(K, 1);
  launch_shape(P, P->prog, P->lds_mode, K1, L, &ws_arena, &G);
  *bytes = workspace_layout(P, K1, G, ws_arena, sweep_needs(P, P->prog, K1, MODE_SAMPLE, -1), offs);
  return PWS_OK;
}

pws_status pws_bind_workspace(pws_plan_t P, void *device_ptr, uint64_t bytes) {
  if (!P) return fail(PWS_ERR_ARG, "plan is NULL");
  P->bound = bytes ? device_ptr : nullptr;
  P->bound_bytes = device_ptr ? bytes : 0;
  return PWS_OK;
}

pws_status pws_plan_stats(pws_plan_t P, double *flops_per_sample, double *bytes_per_sample,
                          int32_t *log2_width, int64_t *n_slices) {
  if (!P) return fail(PWS_ERR_ARG, "plan is NULL");
  // complex multiply-add = 8 real flops; complex64 element = 8 bytes
  if (flops_per_sample) *flops_per_sample = 8.0 * P->prog.flops_per_sample;
  if (bytes_per_sample) *bytes_per_sample = 8.0 * P->prog.bytes_per_sample;
  if (log2_width) *log2_width = P->prog.log2_width;
  if (n_slices) *n_slices = P->prog.n_slices_total;
  return PWS_OK;
}

pws_status pws_plan_sweep_stats(pws_plan_t P, int32_t *n_sweep_steps, double *flops_per_sample,
                                 double *tensor_bytes_per_sample, int32_t *max_width) {
  if (!P) return fail(PWS_ERR_ARG, "plan is NULL");
  if (n_sweep_steps) *n_sweep_steps = P->prog.n_sweep_steps;
  if (flops_per_sample) *flops_per_sample = 8.0 * P->prog.sweep_flops_per_sample;
  if (tensor_bytes_per_sample)
    *tensor_bytes_per_sample = P->prog.sweep_elems_per_sample * (double)elem_bytes(P->precision);
  if (max_width) *max_width = P->prog.max_sweep_width;
  return PWS_OK;
}

pws_status pws_step_count(pws_plan_t P, int32_t *n_steps) {
  if (!P || !n_steps) return fail(PWS_ERR_ARG, "bad argument");
  *n_steps = (int32_t)P->prog.steps.size() - 1;
  return PWS_OK;
}

pws_status pws_step_info(pws_plan_t P, int32_t step, int32_t *op_index, int32_t *gate_index,
                         int32_t *n_candidates) {
  if (!P || step < 0 || step >= (int32_t)P->prog.steps.size() - 1) return fail(PWS_ERR_ARG, "bad step");
  const StepDesc &sd = P->prog.steps[step];
  if (op_index) *op_index = sd.op;
  if (gate_index) *gate_index = sd.gate;
  if (n_candidates) *n_candidates = 1 << sd.nS;
  return PWS_OK;
}

pws_status pws_sample(pws_plan_t P, int64_t n_chains, uint64_t seed, pws_bits *out) {
  return run_sample(P, n_chains, seed, out);
}

pws_status pws_sample_noalloc(pws_plan_t P, int64_t n_chains, uint64_t seed, pws_bits *out) {
  if (!P) return fail(PWS_ERR_ARG, "plan is NULL");
  if (n_chains < 0) return fail(PWS_ERR_ARG, "n_chains < 0");
  pws_status st = check_bits(P, out, n_chains);
  if (st != PWS_OK) return st;
  if (!out->on_device) return fail(PWS_ERR_ARG, "pws_sample_noalloc writes device outputs only (on_device = 1)");
  if (n_chains == 0) return PWS_OK;
  HIP_TRY(hipSetDevice(P->device));
  void *region = nullptr;
  size_t cap = 0;
  HIP_TRY(scratch_region(P->device, &region, &cap));
  const int64_t K = n_chains;
  StepLaunch L0{};
  int64_t ws_arena = 0;
  int G = 0;
  launch_shape(P, P->prog, P->lds_mode, K, L0, &ws_arena, &G);
  const SweepNeeds sn = sweep_needs(P, P->prog, K, MODE_SAMPLE, -1);
  size_t offs[9];
  const size_t need = workspace_layout(P, K, G, ws_arena, sn, offs);
  if (need > cap)
    return fail(PWS_ERR_NOMEM, "pws_sample_noalloc: " + std::to_string(n_chains) + " chains need " +
                                   std::to_string(need) + " bytes of workspace; the static workspace holds " +
                                   std::to_string(cap));
  Workspace w;
  place_workspace((char *)region, offs, sn, w);
  hipStream_t s = P->stream;
  HIP_TRY(launch_clear_flags(w.err, 1, s));
  int launched = 0;
  st = enqueue_pass(P, L0, w, K, 0, seed, nullptr, out->data, s, &launched);
  if (st != PWS_OK) return st;
  int32_t h = 0;
  HIP_TRY(hipMemcpyAsync(&h, w.err, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return err_flags(h);
}

pws_status pws_sample_batch(int32_t n_plans, const pws_plan_t *plans, const int64_t *n_chains,
                            const uint64_t *seeds, pws_bits *outs) {
  if (n_plans <= 0 || !plans || !n_chains || !seeds || !outs) return fail(PWS_ERR_ARG, "bad argument");
  for (int i = 0; i < n_plans; ++i) {
    pws_plan_impl *P = plans[i];
    if (!P) return fail(PWS_ERR_ARG, "plan is NULL");
    if (n_chains[i] < 0) return fail(PWS_ERR_ARG, "n_chains < 0");
    pws_status st = check_bits(P, &outs[i], n_chains[i]);
    if (st != PWS_OK) return st;
    if (n_chains[i] > 0 && !outs[i].on_device) return fail(PWS_ERR_ARG, "batch outputs must be on the device");
    if (P->max_chains > 0 && P->max_chains < n_chains[i])
      return fail(PWS_ERR_ARG, "a batched plan may not split its chains (max_chains)");
    if (P->device != plans[0]->device) return fail(PWS_ERR_ARG, "batched plans must share one device");
    for (int j = 0; j < i; ++j)
      if (plans[j] == P) return fail(PWS_ERR_ARG, "a plan appears twice in the batch");
  }
  pws_plan_impl *P0 = plans[0];
  HIP_TRY(hipSetDevice(P0->device));
  if (!P0->stream && !P0->own_stream) HIP_TRY(hipStreamCreate(&P0->own_stream));
  hipStream_t s = P0->stream ? P0->stream : P0->own_stream;
  // workspaces, launch shapes and the graph key (plan identity, programs,
  // chain count, state, arena and output addresses of every branch)
  struct Branch {
    pws_plan_impl *P;
    int64_t K;
    StepLaunch L0;
    Workspace w;
    uint64_t *dst;
  };
  std::vector<Branch> br;
  std::vector<uint64_t> key{(uint64_t)(uintptr_t)s};
  int64_t total = 0;
  for (int i = 0; i < n_plans; ++i) total += n_chains[i];
  for (int i = 0; i < n_plans; ++i) {
    if (n_chains[i] == 0) continue;
    Branch b{plans[i], n_chains[i], StepLaunch{}, Workspace{}, outs[i].data};
    int64_t ws_arena = 0;
    int G = 0;
    launch_shape(b.P, b.P->prog, b.P->lds_mode, b.K, b.L0, &ws_arena, &G);
    pws_status st = get_workspace(b.P, b.K, G, ws_arena, b.w, sweep_needs(b.P, b.P->prog, b.K, MODE_SAMPLE, -1));
    if (st != PWS_OK) return st;
    HIP_TRY(b.P->seed_buf.ensure(8));
    for (uint64_t v : {b.P->uid, (uint64_t)(uintptr_t)b.P->dp.steps, (uint64_t)b.K, (uint64_t)(uintptr_t)b.w.st.s,
                       (uint64_t)(uintptr_t)b.w.arena, (uint64_t)(uintptr_t)b.dst})
      key.push_back(v);
    br.push_back(b);
  }
  if (br.empty()) return PWS_OK;
  // seeds and error flags are written before the replay (outside the graph)
  for (int i = 0, j = 0; i < n_plans; ++i) {
    if (n_chains[i] == 0) continue;
    HIP_TRY(hipMemcpyAsync(br[j].P->seed_buf.p, &seeds[i], 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(br[j].w.err, 0, 4, s));
    ++j;
  }
  if (!P0->bexec || P0->b_key != key) {
    if (P0->bexec) { (void)hipGraphExecDestroy(P0->bexec); P0->bexec = nullptr; }
    while (P0->b_streams.size() < br.size()) {
      hipStream_t x;
      HIP_TRY(hipStreamCreate(&x));
      P0->b_streams.push_back(x);
    }
    while (P0->b_events.size() < br.size() + 1) {
      hipEvent_t e;
      HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      P0->b_events.push_back(e);
    }
    // fork from s into one stream per plan, join back into s
    hipGraph_t g;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    pws_status cs = PWS_OK;
    int launched = 0;
    hipError_t ce = hipEventRecord(P0->b_events[0], s);
    for (size_t j = 0; j < br.size() && cs == PWS_OK && ce == hipSuccess; ++j) {
      hipStream_t bs = P0->b_streams[j];
      ce = hipStreamWaitEvent(bs, P0->b_events[0], 0);
      if (ce != hipSuccess) break;
      int n = 0;
      // the launch shapes see every chain of the batch competing for waves
      br[j].P->batch_chains = total;
      cs = enqueue_pass(br[j].P, br[j].L0, br[j].w, br[j].K, 0, 0, (const uint64_t *)br[j].P->seed_buf.p,
                        br[j].dst, bs, &n);
      br[j].P->batch_chains = 0;
      launched += n;
      if (cs != PWS_OK) break;
      ce = hipEventRecord(P0->b_events[j + 1], bs);
      if (ce == hipSuccess) ce = hipStreamWaitEvent(s, P0->b_events[j + 1], 0);
    }
    hipError_t ee = hipStreamEndCapture(s, &g);
    if (cs != PWS_OK) return cs;
    if (ce != hipSuccess) return fail(PWS_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
    if (ee != hipSuccess) return fail(PWS_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(ee));
    hipError_t ie = hipGraphInstantiate(&P0->bexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return fail(PWS_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
    P0->b_key = key;
    P0->b_launches = launched;
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, s));
  HIP_TRY(hipGraphLaunch(P0->bexec, s));
  HIP_TRY(hipEventRecord(e1, s));
  std::vector<int32_t> h(br.size(), 0);
  for (size_t j = 0; j < br.size(); ++j)
    HIP_TRY(hipMemcpyAsync(&h[j], br[j].w.err, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P0->last_ms = ms;
  P0->last_launches = P0->b_launches;
  for (size_t j = 0; j < br.size(); ++j) {
    pws_status st = err_flags(h[j]);
    if (st != PWS_OK) return st;
  }
  return PWS_OK;
}

pws_status pws_sample_trace(pws_plan_t P, int64_t n_chains, uint64_t seed, pws_bits *out, uint8_t *trace) {
  if (!P) return fail(PWS_ERR_ARG, "plan is NULL");
  if (!trace) return fail(PWS_ERR_ARG, "trace is NULL");
  if (P->max_chains > 0 && P->max_chains < n_chains)
    return fail(PWS_ERR_UNSUPPORTED, "trace needs all chains in one launch (max_chains)");
  if (n_chains <= 0) return pws_sample(P, n_chains, seed, out);
  pws_status st = check_bits(P, out, n_chains);
  if (st != PWS_OK) return st;
  HIP_TRY(hipSetDevice(P->device));
  const int W = (P->ir.n + 63) / 64;
  const int n_steps = (int)P->prog.steps.size();
  const int64_t K = n_chains;
  StepLaunch L0{};
  int64_t ws_arena = 0;
  int G = 0;
  launch_shape(P, P->prog, P->lds_mode, K, L0, &ws_arena, &G);
  Workspace w;
  st = get_workspace(P, K, G, ws_arena, w, sweep_needs(P, P->prog, K, MODE_SAMPLE, -1));
  if (st != PWS_OK) return st;
  HIP_TRY(P->ws_io2.ensure((size_t)K * std::max(n_steps - 1, 1)));
  HIP_TRY(hipMemsetAsync(w.err, 0, 4, P->stream));
  HIP_TRY(launch_init_state(P->dp, w.st, K, P->stream));
  for (int k = 0; k < n_steps;) {
    StepLaunch L = L0;
    L.step = k;
    L.n_chains = K;
    L.chain_offset = 0;
    L.seed = seed;
    L.arena = w.arena;
    L.mode = MODE_SAMPLE;
    L.trace = k < n_steps - 1 ? (uint8_t *)P->ws_io2.p : nullptr;
    L.trace_row = k;
    L.err = w.err;
    sweep_shape(P, P->prog, k, K, MODE_SAMPLE, &w, L);
    const int k1 = sweep_range(P, P->prog, k, n_steps, K, MODE_SAMPLE, &w, L);
    HIP_TRY(launch_step(P->precision, P->dp, w.st, L, P->stream));
    k = k1;
  }
  HIP_TRY(P->ws_io.ensure((size_t)K * W * 8));
  uint64_t *dst = out->on_device ? out->data : (uint64_t *)P->ws_io.p;
  HIP_TRY(launch_finalize(P->dp, w.st, K, dst, P->stream, seed, nullptr, 0, true));
  if (!out->on_device)
    HIP_TRY(hipMemcpyAsync(out->data, dst, (size_t)K * W * 8, hipMemcpyDeviceToHost, P->stream));
  if (n_steps > 1)
    HIP_TRY(hipMemcpyAsync(trace, P->ws_io2.p, (size_t)K * (n_steps - 1), hipMemcpyDeviceToHost, P->stream));
  return read_err(P, w.err);
}

pws_status pws_sample_probe(pws_plan_t P, int64_t n_chains, uint64_t seed, int32_t step, pws_bits *out,
                            double *out_re_im, int32_t *out_log2) {
  if (!P) return fail(PWS_ERR_ARG, "plan is NULL");
  if (!out_re_im || !out_log2) return fail(PWS_ERR_ARG, "probe outputs are NULL");
  const int n_steps = (int)P->prog.steps.size();
  if (step < 0 || step >= n_steps || P->prog.steps[step].gate < 0) return fail(PWS_ERR_ARG, "step out of range");
  if (P->prog.steps[step].fresh)
    return fail(PWS_ERR_ARG, "the step's gate acts on an untouched qubit: sampling passes draw it from the gate alone");
  if (P->max_chains > 0 && P->max_chains < n_chains)
    return fail(PWS_ERR_UNSUPPORTED, "a probe needs all chains in one launch (max_chains)");
  if (n_chains < 0) return fail(PWS_ERR_ARG, "n_chains < 0");
  pws_status st = check_bits(P, out, n_chains);
  if (st != PWS_OK) return st;
  if (!out->on_device) return fail(PWS_ERR_ARG, "probe outputs must be on the device (on_device = 1)");
  if (n_chains == 0) return PWS_OK;
  HIP_TRY(hipSetDevice(P->device));
  const int64_t K = n_chains;
  StepLaunch L0{};
  int64_t ws_arena = 0;
  int G = 0;
  launch_shape(P, P->prog, P->lds_mode, K, L0, &ws_arena, &G);
  Workspace w;
  st = get_workspace(P, K, G, ws_arena, w, sweep_needs(P, P->prog, K, MODE_SAMPLE, -1));
  if (st != PWS_OK) return st;
  HIP_TRY(hipMemsetAsync(w.err, 0, 4, P->stream));
  HIP_TRY(launch_init_state(P->dp, w.st, K, P->stream));
  for (int k = 0; k <= step;) {
    StepLaunch L = L0;
    L.step = k;
    L.n_chains = K;
    L.chain_offset = 0;
    L.seed = seed;
    L.arena = w.arena;
    L.mode = MODE_SAMPLE;
    L.trace = nullptr;
    L.trace_row = k;
    L.err = w.err;
    sweep_shape(P, P->prog, k, K, MODE_SAMPLE, &w, L);
    int k1 = sweep_range(P, P->prog, k, n_steps, K, MODE_SAMPLE, &w, L);
    if (k1 > step + 1) {
      k1 = step + 1;
      L.step_end = k1;
    }
    if (k <= step && step < k1) {
      L.out_amp = out_re_im;
      L.out_log2 = out_log2;
      L.probe_step = step;
    }
    HIP_TRY(launch_step(P->precision, P->dp, w.st, L, P->stream));
    k = k1;
  }
  HIP_TRY(launch_finalize(P->dp, w.st, K, out->data, P->stream, seed, nullptr, 0, false));
  return read_err(P, w.err);
}

static pws_status run_amps(pws_plan_t P, const DevProg &dp, const Programs &pr, bool lds, int step,
                           const pws_bits *bits, double *out_re_im, int32_t *out_log2, bool scale_out) {
  const int64_t K = bits->n;
  const int W = (P->ir.n + 63) / 64;
  const int nS = pr.steps[step].nS;
  const int m = 1 << nS;
  if (K == 0) return PWS_OK;
  HIP_TRY(hipSetDevice(P->device));
  StepLaunch L{};
  int64_t ws_arena = 0;
  int G = 0;
  launch_shape(P, pr, lds, K, L, &ws_arena, &G);
  Workspace w;
  pws_status st = get_workspace(P, K, G, ws_arena, w, sweep_needs(P, pr, K, MODE_AMPS, step));
  if (st != PWS_OK) return st;
  HIP_TRY(hipMemsetAsync(w.err, 0, 4, P->stream));
  HIP_TRY(launch_init_state(dp, w.st, K, P->stream));
  HIP_TRY(hipMemcpyAsync(w.st.s, bits->data, (size_t)K * W * 8,
                         bits->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, P->stream));
  const size_t amp_bytes = (size_t)K * m * 16, log_bytes = (size_t)K * 4;
  HIP_TRY(P->ws_io.ensure(amp_bytes + log_bytes + 256));
  double *d_amp = (double *)P->ws_io.p;
  int32_t *d_log = (int32_t *)((char *)P->ws_io.p + align256(amp_bytes));
  L.step = step;
  L.n_chains = K;
  L.arena = w.arena;
  L.mode = MODE_AMPS;
  L.out_amp = d_amp;
  L.out_log2 = d_log;
  L.err = w.err;
  sweep_shape(P, pr, step, K, MODE_AMPS, &w, L);
  HIP_TRY(launch_step(P->precision, dp, w.st, L, P->stream));
  std::vector<double> ha((size_t)K * m * 2);
  std::vector<int32_t> hl(K);
  HIP_TRY(hipMemcpyAsync(ha.data(), d_amp, amp_bytes, hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipMemcpyAsync(hl.data(), d_log, log_bytes, hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  if (!out_log2 && scale_out) {
    for (int64_t c = 0; c < K; ++c)
      for (int v = 0; v < 2 * m; ++v) ha[c * 2 * m + v] = std::ldexp(ha[c * 2 * m + v], hl[c]);
  }
  if (bits->on_device) {
    HIP_TRY(hipMemcpy(out_re_im, ha.data(), amp_bytes, hipMemcpyHostToDevice));
    if (out_log2) HIP_TRY(hipMemcpy(out_log2, hl.data(), log_bytes, hipMemcpyHostToDevice));
  } else {
    std::memcpy(out_re_im, ha.data(), amp_bytes);
    if (out_log2) std::memcpy(out_log2, hl.data(), log_bytes);
  }
  return PWS_OK;
}

pws_status pws_amplitudes(pws_plan_t P, const pws_bits *bitstrings, double *out_re_im, int32_t *out_log2) {
  if (!P) return fail(PWS_ERR_ARG, "plan is NULL");
  pws_status st = check_bits(P, bitstrings, 0);
  if (st != PWS_OK) return st;
  if (!out_re_im) return fail(PWS_ERR_ARG, "out_re_im is NULL");
  if (!P->have_amp) {
    HIP_TRY(hipSetDevice(P->device));
    st = build_full(P, false);
    if (st != PWS_OK) return st;
  }
  return run_amps(P, P->dp_amp, P->full_amp, P->amp_lds, 0, bitstrings, out_re_im, out_log2, true);
}

pws_status pws_step_amplitudes(pws_plan_t P, int32_t step, const pws_bits *states, double *out_re_im,
                               int32_t *out_log2) {
  if (!P) return fail(PWS_ERR_ARG, "plan is NULL");
  if (step < 0 || step >= (int32_t)P->prog.steps.size() - 1) return fail(PWS_ERR_ARG, "bad step");
  if (P->ir.noisy) return fail(PWS_ERR_UNSUPPORTED, "step amplitudes of noisy plans depend on the chain's noise record");
  pws_status st = check_bits(P, states, 0);
  if (st != PWS_OK) return st;
  if (!out_re_im) return fail(PWS_ERR_ARG, "out_re_im is NULL");
  // a two-sided step needs an earlier step's kept tensor: single steps run
  // from a plan of steps that stand alone
  bool two_sided = false;
  for (const StepDesc &sd : P->prog.steps) two_sided |= sd.sweep && (sd.merge_slot >= 0 || sd.snap_count > 0);
  if (!two_sided) return run_amps(P, P->dp, P->prog, P->lds_mode, step, states, out_re_im, out_log2, true);
  if (!P->have_solo) {
    PlanOptions o = P->opt;
    o.sweep_cache = 0;
    o.sweep_merge = 0;
    Programs pr;
    std::string err = plan_steps_once(P->ir, o, pr);
    if (!err.empty()) return fail(PWS_ERR_PLAN, err);
    if (pr.steps.size() != P->prog.steps.size()) return fail(PWS_ERR_PLAN, "standalone steps differ");
    P->prog_solo = std::move(pr);
    pws_status ust = upload_prog(P, P->prog_solo, P->solobufs, P->dp_solo);
    if (ust != PWS_OK) return ust;
    P->have_solo = true;
  }
  return run_amps(P, P->dp_solo, P->prog_solo, P->lds_mode, step, states, out_re_im, out_log2, true);
}

pws_status pws_grad(pws_plan_t P, const pws_bits *samples, double *dtheta) {
  if (!P) return fail(PWS_ERR_ARG, "plan is NULL");
  pws_status st = check_bits(P, samples, 0);
  if (st != PWS_OK) return st;
  if (!dtheta) return fail(PWS_ERR_ARG, "dtheta is NULL");
  if (P->ir.n_params == 0) return PWS_OK;
  const int64_t K = samples->n;
  if (K == 0) return PWS_OK;
  HIP_TRY(hipSetDevice(P->device));
  if (!P->have_grad) {
    st = build_full(P, true);
    if (st != PWS_OK) return st;
  }
  const int W = (P->ir.n + 63) / 64;
  // waves in flight, each with one sample's adjoint network in its arena
  // (every forward tensor is kept): as many as the memory budget allows
  // (the kernel strides over the samples)
  const int64_t arena = std::max(P->full_grad.max_arena, 2);
  const double per_group = (double)kWavesPerBlock * (double)arena * (double)elem_bytes(P->precision);
  const double fixed = (double)K * W * 8 + 4096;
  if (fixed + per_group > (double)P->budget)
    return fail(PWS_ERR_NOMEM, "one sample's adjoint network needs " + std::to_string((int64_t)per_group / kWavesPerBlock) +
                                   " bytes of workspace; the memory budget is " + std::to_string(P->budget) + " bytes");
  const int G = (int)std::max<int64_t>(1, std::min<int64_t>(choose_grid(P, K), (int64_t)(((double)P->budget - fixed) / per_group)));
  Workspace w;
  st = get_workspace(P, K, G, arena, w);
  if (st != PWS_OK) return st;
  HIP_TRY(hipMemsetAsync(w.err, 0, 4, P->stream));
  HIP_TRY(launch_init_state(P->dp_grad, w.st, K, P->stream));
  HIP_TRY(hipMemcpyAsync(w.st.s, samples->data, (size_t)K * W * 8,
                         samples->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, P->stream));
  const size_t out_bytes = (size_t)K * P->ir.n_params * 8;
  double *d_out = dtheta;
  if (!samples->on_device) {
    HIP_TRY(P->ws_io.ensure(out_bytes));
    d_out = (double *)P->ws_io.p;
  }
  GradLaunch L{};
  L.n_chains = K;
  L.arena = w.arena;
  L.arena_stride = std::max(P->full_grad.max_arena, 2);
  L.grid = G;
  L.block = 256;
  L.dtheta = d_out;
  L.err = w.err;
  L.lds_bytes = lds_bytes_for(std::max(P->full_grad.max_exp, 1));
  HIP_TRY(launch_grad(P->precision, P->dp_grad, w.st, L, P->stream));
  if (!samples->on_device)
    HIP_TRY(hipMemcpyAsync(dtheta, d_out, out_bytes, hipMemcpyDeviceToHost, P->stream));
  return read_err(P, w.err);
}

static void swap_forms(pws_plan_t P) {
  std::swap(P->prog, P->prog_alt);
  std::swap(P->dp, P->dp_alt);
  std::swap(P->pbufs, P->altbufs);
  P->lds_mode = P->lds_mode ? 0 : 1;
  if (P->gexec) { (void)hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
}

// Sweep-form launch shapes, tuned by timing whole sampling passes: one knob
// at a time over a few values each (the others at their best so far), in
// the order the knobs matter: chains per wave of the narrow launches, steps
// per range launch, the width from which four waves share a chain, the
// widest step in a range, and (op-by-op plans) the op-matrix window.  Every
// value gives the same samples; only the time differs.
namespace {
struct SweepKnob {
  const char *name;
  int *field;
  std::vector<int> values;
};

pws_status autotune_sweep(pws_plan_impl *P, int64_t n_chains, uint64_t seed, const char *cache_path,
                          const char *key, char *chosen, int64_t chosen_len) {
  std::vector<SweepKnob> knobs;
  if (P->dense) {
    knobs.push_back({"cpw2", &P->dense_cpw2_width, {0, 8, 10}});
    knobs.push_back({"range", &P->dense_range_steps, {0, 32, 64, 128}});
  } else {
    knobs.push_back({"cpw8", &P->sweep_cpw8, {1, 2, 4}});
    knobs.push_back({"cpw10", &P->sweep_cpw10, {1, 2}});
  }
  knobs.push_back({"coop4", &P->sweep_coop_width, {11, 12, 13}});
  knobs.push_back({"rangew", &P->sweep_range_w, {8, 10}});
  if (!P->dense) knobs.push_back({"window", &P->sweep_mt_cap, {64, 128, 160}});
  const std::string skey = std::string(key) + ":sweep";
  auto describe = [&](const char *tail) {
    if (!chosen || chosen_len <= 0) return;
    std::string s = "sweep";
    for (const SweepKnob &k : knobs) s += std::string(" ") + k.name + "=" + std::to_string(*k.field);
    s += tail;
    snprintf(chosen, (size_t)chosen_len, "%s", s.c_str());
  };
  auto reset_graph = [&]() {
    if (P->gexec) { (void)hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
  };
  // cached decision: "key:sweep v0 v1 ... ms" with one value per knob
  if (cache_path) {
    FILE *f = fopen(cache_path, "r");
    if (f) {
      char line[512];
      std::vector<int> found;
      while (fgets(line, sizeof line, f)) {
        std::istringstream is(line);
        std::string k;
        is >> k;
        if (k != skey) continue;
        std::vector<int> v(knobs.size());
        bool ok = true;
        for (int &x : v) ok = ok && (bool)(is >> x);
        if (ok) found = v;
      }
      fclose(f);
      if (!found.empty()) {
        for (size_t i = 0; i < knobs.size(); ++i) *knobs[i].field = found[i];
        reset_graph();
        describe(" (cached)");
        return PWS_OK;
      }
    }
  }
  std::vector<uint64_t> out((size_t)n_chains * ((P->ir.n + 63) / 64));
  pws_bits b{n_chains, (P->ir.n + 63) / 64, 0, out.data()};
  auto time_now = [&](double *ms) -> pws_status {
    reset_graph();
    pws_status st = run_sample(P, n_chains, seed, &b);   // warm (captures the graph)
    if (st != PWS_OK) return st;
    double best = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
      st = run_sample(P, n_chains, seed + 1 + rep, &b);
      if (st != PWS_OK) return st;
      best = std::min(best, P->last_ms);
    }
    *ms = best;
    return PWS_OK;
  };
  double best_ms;
  pws_status st = time_now(&best_ms);
  if (st != PWS_OK) return st;
  std::string log = " | start " + std::to_string(best_ms).substr(0, 6) + "ms";
  for (SweepKnob &k : knobs) {
    const int keep = *k.field;
    int best_v = keep;
    for (int v : k.values) {
      if (v == keep) continue;
      *k.field = v;
      double ms;
      st = time_now(&ms);
      if (st != PWS_OK) { *k.field = keep; reset_graph(); return st; }
      log += std::string(" ") + k.name + "=" + std::to_string(v) + ":" + std::to_string(ms).substr(0, 6);
      if (ms < best_ms) { best_ms = ms; best_v = v; }
    }
    *k.field = best_v;
  }
  reset_graph();
  if (cache_path) {
    FILE *f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "%s", skey.c_str());
      for (const SweepKnob &k : knobs) fprintf(f, " %d", *k.field);
      fprintf(f, " %.4f\n", best_ms);
      fclose(f);
    }
  }
  describe((" " + std::to_string(best_ms).substr(0, 6) + "ms" + log).c_str());
  return PWS_OK;
}
}  // namespace

pws_status pws_autotune(pws_plan_t P, int64_t n_chains, uint64_t seed, const char *cache_path,
                        char *chosen, int64_t chosen_len) {
  if (!P) return fail(PWS_ERR_ARG, "plan is NULL");
  if (P->host_only) return fail(PWS_ERR_DEVICE, "host-only plan");
  if (n_chains <= 0) return fail(PWS_ERR_ARG, "n_chains must be positive");
  HIP_TRY(hipSetDevice(P->device));
  char key[96];
  snprintf(key, sizeof key, "%016llx:%lld", (unsigned long long)P->plan_hash, (long long)n_chains);
  {
    // the node forms differ only in how node-form steps run; a plan whose
    // steps all run in the sweep form tunes the sweep launches instead
    int node_steps = 0;
    for (const StepDesc &sd : P->prog.steps) node_steps += (!sd.sweep && sd.n_nodes > 0) ? 1 : 0;
    if (node_steps == 0) return autotune_sweep(P, n_chains, seed, cache_path, key, chosen, chosen_len);
  }
  // cached decision?
  int c_form = -1, c_grid = 0, c_block = 0;
  if (cache_path) {
    FILE *f = fopen(cache_path, "r");
    if (f) {
      char k2[96];
      int fo, gr, bl;
      double ms;
      while (fscanf(f, "%95s %d %d %d %lf", k2, &fo, &gr, &bl, &ms) == 5)
        if (std::string(k2) == key) { c_form = fo; c_grid = gr; c_block = bl; }
      fclose(f);
    }
  }
  // plan the LDS form once (if every step can be sliced onto the chip)
  if (!P->have_alt) {
    PlanOptions o = P->opt;
    Programs pr;
    std::string err;
    const int eb = (int)elem_bytes(P->precision);
    bool ok = false;
    int reserve = 4096;
    if (!P->lds_mode) {
      for (int attempt = 0; attempt < 4 && !ok; ++attempt) {
        o.lds_mode = 1;
        o.arena_limit_elems = (uint64_t)std::max(64, (P->lds_capacity - 512 - reserve) / eb);
        pr = Programs();
        err = plan_steps(P->ir, o, pr);
        if (!err.empty()) break;
        const int need = lds_bytes_arena(P->precision, pr.max_arena, pr.max_exp) + 512;
        if (need > P->lds_capacity) { reserve += need - P->lds_capacity + 1024; continue; }
        if (pr.flops_executed > 16.0 * pr.flops_per_sample) break;
        ok = true;
      }
    } else {
      o.lds_mode = 0;
      o.arena_limit_elems = P->budget_limit;
      err = plan_steps(P->ir, o, pr);
      ok = err.empty();
    }
    if (ok) {
      P->prog_alt = std::move(pr);
      pws_status st = upload_prog(P, P->prog_alt, P->altbufs, P->dp_alt);
      if (st != PWS_OK) return st;
      P->have_alt = 1;
    } else {
      P->have_alt = -1;
    }
  }
  std::vector<uint64_t> out((size_t)n_chains * ((P->ir.n + 63) / 64));
  pws_bits b{n_chains, (P->ir.n + 63) / 64, 0, out.data()};
  const int base_grid = P->grid_max;
  struct Cand { int form, grid, block; double ms; };
  std::vector<Cand> cands;
  auto want_form = [&](int form) -> pws_status {
    if (form != P->lds_mode) {
      if (P->have_alt != 1) return fail(PWS_ERR_PLAN, "form not available");
      swap_forms(P);
    }
    return PWS_OK;
  };
  if (c_form >= 0) {
    if (want_form(c_form) == PWS_OK) {
      P->grid_max = c_grid;
      P->block = c_block;
      if (P->gexec) { (void)hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
      if (chosen) snprintf(chosen, (size_t)chosen_len, "%s grid=%d block=%d (cached)",
                           c_form ? "lds" : "wave", c_grid, c_block);
      return PWS_OK;
    }
  }
  for (int form = 0; form < 2; ++form) {
    if (want_form(form) != PWS_OK) continue;
    std::vector<std::pair<int, int>> shapes;
    if (form == 0) {
      for (int mult : {2, 4, 5}) shapes.push_back({P->cus * mult, 256});
    } else {
      for (int blk : {256, 512}) shapes.push_back({base_grid, blk});
    }
    for (auto &sh : shapes) {
      P->grid_max = sh.first;
      P->block = sh.second;
      if (P->gexec) { (void)hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
      pws_status st = run_sample(P, n_chains, seed, &b);   // warm (captures the graph)
      if (st != PWS_OK) return st;
      st = run_sample(P, n_chains, seed + 1, &b);
      if (st != PWS_OK) return st;
      cands.push_back({form, sh.first, sh.second, P->last_ms});
    }
  }
  if (cands.empty()) return fail(PWS_ERR_PLAN, "no execution form could run");
  const Cand *best = &cands[0];
  for (auto &c : cands) if (c.ms < best->ms) best = &c;
  if (want_form(best->form) != PWS_OK) return fail(PWS_ERR_PLAN, "lost the chosen form");
  P->grid_max = best->grid;
  P->block = best->block;
  if (P->gexec) { (void)hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
  if (cache_path) {
    FILE *f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "%s %d %d %d %.4f\n", key, best->form, best->grid, best->block, best->ms);
      fclose(f);
    }
  }
  if (chosen) {
    std::string s;
    for (auto &c : cands) {
      char t[96];
      snprintf(t, sizeof t, "%s%s/%d/%d:%.2fms", s.empty() ? "" : " ", c.form ? "lds" : "wave", c.grid, c.block, c.ms);
      s += t;
    }
    snprintf(chosen, (size_t)chosen_len, "%s grid=%d block=%d | %s", best->form ? "lds" : "wave", best->grid,
             best->block, s.c_str());
  }
  return PWS_OK;
}

pws_status pws_last_timing(pws_plan_t P, double *ms_total, int32_t *n_launches) {
  if (!P) return fail(PWS_ERR_ARG, "plan is NULL");
  if (ms_total) *ms_total = P->last_ms;
  if (n_launches) *n_launches = P->last_launches;
  return PWS_OK;
}

pws_status pws_set_theta(pws_plan_t P, const double *theta, int32_t n_params) {
  if (!P) return fail(PWS_ERR_ARG, "plan is NULL");
  if (n_params != P->ir.n_params || (n_params > 0 && !theta)) return fail(PWS_ERR_ARG, "bad theta");
  CircuitIR next = P->ir;
  const std::string err = set_theta(next, theta);
  if (!err.empty()) return fail(PWS_ERR_PLAN, err);
  if (!P->host_only) {
    // work queued with the old tables finishes before they are overwritten
    HIP_TRY(hipStreamSynchronize(P->stream));
    if (P->own_stream) HIP_TRY(hipStreamSynchronize(P->own_stream));
  }
  P->ir.gates.swap(next.gates);
  P->ir.theta.swap(next.theta);
  retabulate(P->ir, P->prog);
  // the dense runs' tables follow the new matrix entries (same runs, same layout)
  const size_t dtab_words = P->prog.dtab.size();
  if (P->dense) build_dense(P->prog, P->dense == 2, 256ull << 20, 4ull << 30);
  if (P->prog.dtab.size() != dtab_words) return fail(PWS_ERR_PLAN, "dense-run tables changed layout");
  if (P->have_alt) retabulate(P->ir, P->prog_alt);
  if (P->have_solo) retabulate(P->ir, P->prog_solo);
  if (P->have_amp) retabulate(P->ir, P->full_amp);
  if (P->have_grad) retabulate(P->ir, P->full_grad);
  if (P->host_only) return PWS_OK;
  // same device buffers as before, so captured graphs stay valid
  std::vector<double> gm(P->ir.gates.size() * 32, 0.0), gdm(P->ir.gates.size() * 32, 0.0);
  for (size_t g = 0; g < P->ir.gates.size(); ++g) {
    const GateIR &G = P->ir.gates[g];
    const int dd = 1 << G.nq;
    for (int e = 0; e < dd * dd; ++e) {
      gm[g * 32 + 2 * e] = G.mat[e].real();
      gm[g * 32 + 2 * e + 1] = G.mat[e].imag();
      gdm[g * 32 + 2 * e] = G.dmat[e].real();
      gdm[g * 32 + 2 * e + 1] = G.dmat[e].imag();
    }
  }
  if (!gm.empty()) {
    HIP_TRY(hipMemcpy(const_cast<double *>(P->d_gmat), gm.data(), gm.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(const_cast<double *>(P->d_gdmat), gdm.data(), gdm.size() * 8, hipMemcpyHostToDevice));
  }
  const std::pair<const Programs *, const DevProg *> progs[5] = {
      {&P->prog, &P->dp}, {P->have_alt ? &P->prog_alt : nullptr, &P->dp_alt},
      {P->have_solo ? &P->prog_solo : nullptr, &P->dp_solo},
      {P->have_amp ? &P->full_amp : nullptr, &P->dp_amp}, {P->have_grad ? &P->full_grad : nullptr, &P->dp_grad}};
  for (const auto &pd : progs) {
    if (pd.first && !pd.first->ltab.empty())
      HIP_TRY(hipMemcpy(const_cast<double *>(pd.second->ltab), pd.first->ltab.data(), pd.first->ltab.size() * 8,
                        hipMemcpyHostToDevice));
    if (pd.first && !pd.first->ment.empty())
      HIP_TRY(hipMemcpy(const_cast<MEntry *>(pd.second->ment), pd.first->ment.data(),
                        pd.first->ment.size() * sizeof(MEntry), hipMemcpyHostToDevice));
    if (pd.first && !pd.first->mterm.empty())
      HIP_TRY(hipMemcpy(const_cast<double *>(pd.second->mterm), pd.first->mterm.data(), pd.first->mterm.size() * 8,
                        hipMemcpyHostToDevice));
    if (pd.first && !pd.first->dtab.empty())
      HIP_TRY(hipMemcpy(const_cast<uint32_t *>(pd.second->dtab), pd.first->dtab.data(), pd.first->dtab.size() * 4,
                        hipMemcpyHostToDevice));
    if (pd.first && !pd.first->steps.empty()) {
      const std::vector<StepDesc> steps = hot_steps(P, *pd.first);
      HIP_TRY(hipMemcpy(const_cast<StepDesc *>(pd.second->steps), steps.data(), steps.size() * sizeof(StepDesc),
                        hipMemcpyHostToDevice));
    }
  }
  return PWS_OK;
}

pws_status pws_plan_export(pws_plan_t P, int32_t step, char *buf, int64_t *len) {
  if (!P || !len) return fail(PWS_ERR_ARG, "bad argument");
  std::string s;
  if (step == -1) {
    std::vector<std::vector<int>> legs;
    std::vector<Pair> pairs;
    if (!P->have_amp) {
      Programs tmp;
      StepNet net = build_step_net(P->ir, (int)P->ir.gates.size() - 1, {}, -1, true);
      fuse_leaves(net);
      for (auto &l : net.leaves) legs.push_back(l.legs);
      pairs = P->user_tree.empty() ? plan_tree(P->ir, legs, net.open_legs, P->opt, nullptr) : P->user_tree;
      std::string err = emit_step(P->ir, net, pairs, P->opt, 0, tmp, false);
      if (!err.empty()) return fail(PWS_ERR_PLAN, err);
      s = export_json(P->ir, tmp, 0);
    } else {
      s = export_json(P->ir, P->full_amp, 0);
      legs = P->full_legs;
      pairs = P->full_pairs;
    }
    // the network itself: each leaf's legs (segment ids) and the SSA pairs
    std::string net = ",\"network\":{\"legs\":[";
    for (size_t i = 0; i < legs.size(); ++i) {
      net += i ? ",[" : "[";
      for (size_t j = 0; j < legs[i].size(); ++j) net += (j ? "," : "") + std::to_string(legs[i][j]);
      net += "]";
    }
    net += "],\"pairs\":[";
    for (size_t i = 0; i < pairs.size(); ++i)
      net += (i ? ",[" : "[") + std::to_string(pairs[i].a) + "," + std::to_string(pairs[i].b) + "]";
    net += "]}";
    s.insert(s.size() - 1, net);
  } else {
    if (step < 0 || step >= (int32_t)P->prog.steps.size()) return fail(PWS_ERR_ARG, "bad step");
    s = export_json(P->ir, P->prog, step);
  }
  const int64_t need = (int64_t)s.size() + 1;
  if (!buf || *len < need) {
    *len = need;
    return buf ? fail(PWS_ERR_ARG, "buffer too small") : PWS_OK;
  }
  std::memcpy(buf, s.c_str(), need);
  *len = need;
  return PWS_OK;
}

}  // extern "C"
