// Dense-run form of the sweep steps.
//
// A sweep step absorbs the leaves of its prefix network one at a time into a
// running tensor (Section 2: the amplitude of each candidate is a contraction
// of the prefix circuit's network); each absorption is an op that multiplies
// the groups of elements over the op's (at most four) positions by a small
// matrix whose entries are products of chain-independent constants and of
// table lookups indexed by a few of the chain's classical bits (the output
// projections onto the chain's state).  A run of consecutive ops whose
// positions together fit in four is one linear map on the 16-dimensional
// space of those positions, identity on every other position: its matrix F is
// the product of the ops' matrices, which this file forms on the host in
// complex double for every value of the chain bits the run's entries read.
// The kernels then apply one F per run as 16 x 16 complex matrix products on
// the matrix cores instead of the run's ops one by one.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <cstdint>
#include <vector>

#include "host.hpp"

namespace pws {

namespace {

using cplx = std::complex<double>;

struct RunBuild {
  int op0 = 0, op1 = 0;           // sweep ops [op0, op1) of the step
  int pmask = 0;                  // positions the ops touch
  std::vector<int> qubits;        // chain bits the entries read
  bool renorm = false;
};

// Chain qubits one matrix entry reads (its two term lookups).
void entry_qubits(const MEntry &me, std::vector<int> &qs) {
  for (const auto &tp : {std::make_pair(me.t0, me.p0), std::make_pair(me.t1, me.p1)}) {
    if (tp.first < 0) continue;
    const int nv = (tp.second >> 24) & 3;
    for (int k = 0; k < nv; ++k) {
      const int q = (tp.second >> (12 * k)) & 0xfff;
      if (std::find(qs.begin(), qs.end(), q) == qs.end()) qs.push_back(q);
    }
  }
}

int op_entries(const SweepOp &so) {
  const int n = 1 << so.np;
  return so.diag == 1 ? n : n * n;
}

bool plain_entry(const MEntry &me) { return me.t0 != PWS_MENTRY_CODES && me.t0 != PWS_MENTRY_FLAT; }

// An entry given by its codes (a product of leaf elements, each summed over
// the leaf's internal legs) can be formed on the host when every leaf it
// reads is tabulated with chain bits as its only variant bits and carries no
// per-chain noise record.  Appends the chain qubits it reads; false when it
// cannot be formed.
bool codes_qubits(const Programs &prog, const StepDesc &sd, const int32_t *codes, std::vector<int> &qs) {
  for (int t = 0; t < PWS_MTERMS; ++t) {
    const int32_t code = codes[t];
    if (code < 0) return true;   // structural zero
    if (code & PWS_MCODE_ONE) continue;
    const LeafDesc &ld = prog.leaves[sd.leaf_begin + (code & 0xffff)];
    if (ld.tab_off < 0 || ld.r_count > 0) return false;
    for (int k = 0; k < ld.nvar; ++k) {
      const int32_t vc = prog.lvar[ld.var_begin + k];
      if ((vc >> 24) != VAR_CHAIN) return false;
      const int q = vc & 0xffffff;
      if (std::find(qs.begin(), qs.end(), q) == qs.end()) qs.push_back(q);
    }
  }
  return true;
}

// Value of entry `i` of the step for the chain bits `bit(q)`: the folded
// form (constant times term lookups) or the product of its codes.
template <typename BitOf>
cplx entry_value(const Programs &prog, const StepDesc &sd, int i, BitOf bit) {
  const MEntry &me = prog.ment[sd.m_begin / PWS_MTERMS + i];
  if (plain_entry(me)) {
    cplx v(me.re, me.im);
    for (const auto &tp : {std::make_pair(me.t0, me.p0), std::make_pair(me.t1, me.p1)}) {
      if (tp.first < 0) continue;
      const int nv = (tp.second >> 24) & 3;
      int idx = 0;
      for (int k = 0; k < nv; ++k) idx |= bit((tp.second >> (12 * k)) & 0xfff) << k;
      const size_t at = 2 * ((size_t)tp.first + idx);
      v *= cplx(prog.mterm[at], prog.mterm[at + 1]);
    }
    return v;
  }
  const int32_t *codes = &prog.mtab[(size_t)sd.m_begin + (size_t)i * PWS_MTERMS];
  cplx v(1.0, 0.0);
  for (int t = 0; t < PWS_MTERMS; ++t) {
    const int32_t code = codes[t];
    if (code < 0) return 0.0;
    if (code & PWS_MCODE_ONE) continue;
    const LeafDesc &ld = prog.leaves[sd.leaf_begin + (code & 0xffff)];
    int var = 0;
    for (int k = 0; k < ld.nvar; ++k) var |= bit(prog.lvar[ld.var_begin + k] & 0xffffff) << k;
    const int e0 = (code >> 16) & 15, im = (code >> 20) & 15;
    cplx acc(0.0, 0.0);
    for (int sub = im;; sub = (sub - 1) & im) {
      const size_t at = 2 * ((size_t)ld.tab_off + ((size_t)var << ld.nfree) + (size_t)(e0 | sub));
      acc += cplx(prog.ltab[at], prog.ltab[at + 1]);
      if (sub == 0) break;
    }
    v *= acc;
  }
  return v;
}

// Chain qubits entry `i` reads; false when the host cannot form it.
bool entry_qubits(const Programs &prog, const StepDesc &sd, int i, std::vector<int> &qs) {
  const MEntry &me = prog.ment[sd.m_begin / PWS_MTERMS + i];
  if (plain_entry(me)) {
    entry_qubits(me, qs);
    return true;
  }
  return codes_qubits(prog, sd, &prog.mtab[(size_t)sd.m_begin + (size_t)i * PWS_MTERMS], qs);
}

// Runs of one step: consecutive ops joined while their positions fit in four
// and their entries read at most PWS_DENSE_JOINBITS chain bits; runs end
// where a tensor is kept (the next step's prefix, snapshots) and, when they
// start at op 0, where a sampling pass restores.  False when the step has no
// dense form.
bool partition_step(const Programs &prog, const StepDesc &sd, int op0, std::vector<RunBuild> &runs) {
  runs.clear();
  const SweepOp *ops = prog.sweeps.data() + sd.sw_begin;
  std::vector<std::vector<int>> op_qs(sd.sw_count);
  for (int k = op0; k < sd.sw_count; ++k)
    for (int e = 0; e < op_entries(ops[k]); ++e)
      if (!entry_qubits(prog, sd, ops[k].moff + e, op_qs[k])) return false;
  std::vector<char> cut(sd.sw_count + 1, 0);
  if (sd.store_op >= 0 && sd.store_op <= sd.sw_count) cut[sd.store_op] = 1;
  for (int i = 0; i < sd.snap_count; ++i) {
    const int o = prog.snaps[sd.snap_begin + i].op;
    if (o >= 0 && o <= sd.sw_count) cut[o] = 1;
  }
  if (sd.load_op > 0 && sd.load_op <= sd.sw_count) cut[sd.load_op] = 1;
  for (int k = op0; k < sd.sw_count; ++k) {
    const SweepOp &so = ops[k];
    int pm = 0;
    for (int j = 0; j < so.np; ++j) pm |= 1 << so.pos[j];
    const std::vector<int> &qs = op_qs[k];
    bool join = !runs.empty() && !cut[k];
    if (join) {
      RunBuild &r = runs.back();
      const int pm2 = r.pmask | pm;
      std::vector<int> q2 = r.qubits;
      for (int q : qs)
        if (std::find(q2.begin(), q2.end(), q) == q2.end()) q2.push_back(q);
      // the other live positions must be the same for every op of a run
      const int outer_r = ops[r.op0].outer_mask & ~pm2;
      join = __builtin_popcount(pm2) <= 4 && (int)q2.size() <= PWS_DENSE_JOINBITS &&
             (so.outer_mask & ~pm2) == outer_r;
      if (join) {
        r.pmask = pm2;
        r.qubits = q2;
        r.op1 = k + 1;
        r.renorm |= so.renorm != 0;
      }
    }
    if (!join) {
      if ((int)qs.size() > PWS_DENSE_VARBITS) return false;
      RunBuild r;
      r.op0 = k;
      r.op1 = k + 1;
      r.pmask = pm;
      r.qubits = qs;
      r.renorm = so.renorm != 0;
      runs.push_back(r);
    }
  }
  return true;
}

uint64_t table_bytes(const std::vector<RunBuild> &runs) {
  uint64_t b = 0;
  for (const RunBuild &r : runs) b += (uint64_t)(1u << r.qubits.size()) * 512 * 4;
  return b;
}

// Nearest bf16 value of x (round to nearest, ties to even), for normal
// magnitudes; bf16 keeps 8 significant bits.
double round_bf16(double x) {
  if (x == 0.0 || !std::isfinite(x)) return x;
  int e;
  std::frexp(x, &e);                       // |x| in [2^(e-1), 2^e)
  const double scale = std::ldexp(1.0, 8 - e);
  return std::nearbyint(x * scale) / scale;   // default rounding mode: ties to even
}

// The bf16 encoding of a value that is exactly representable in bf16.
uint32_t bf16_bits(double v) {
  const float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u >> 16;
}

// The run's record and its F tables (every variant) appended to prog.
void emit_run(Programs &prog, const StepDesc &sd, const RunBuild &r, int W, bool split_bf16) {
  const SweepOp *ops = prog.sweeps.data() + sd.sw_begin;
  // rows: the ops' positions, padded to four with other live positions
  // (fewer columns) and then with free ones (whose 1-half holds zeros)
  int outer = ops[r.op0].outer_mask & ~r.pmask;
  int pm = r.pmask;
  for (int b = 0; b < W && __builtin_popcount(pm) < 4; ++b)
    if ((outer >> b) & 1) { pm |= 1 << b; outer &= ~(1 << b); }
  for (int b = 0; b < W && __builtin_popcount(pm) < 4; ++b)
    if (!((pm >> b) & 1)) pm |= 1 << b;
  int pos[4], np = 0;
  for (int b = 0; b < W; ++b)
    if ((pm >> b) & 1) pos[np++] = b;
  DenseRun dr{};
  dr.foff = (int32_t)(prog.dtab.size() / 512);
  // rows and the lowest four columns as nibbles (positions stay below 16:
  // dense steps are at most 2^12 elements wide)
  int cols = 0, hi = outer;
  for (int t = 0; t < 4 && hi; ++t) {
    const int b = __builtin_ctz(hi);
    cols |= b << (4 * t);
    hi &= hi - 1;
  }
  dr.pos = pos[0] | (pos[1] << 4) | (pos[2] << 8) | (pos[3] << 12) | (cols << 16);
  dr.outer_mask = hi;
  const int nq = (int)r.qubits.size();
  dr.info = __builtin_popcount(outer) | (nq << 8) | ((r.renorm ? 1 : 0) << 16);
  for (int b = 0; b < nq; ++b) {
    int32_t &wq = b < 3 ? dr.q012 : b < 6 ? dr.q345 : dr.q67;
    wq |= r.qubits[b] << (10 * (b % 3));
  }
  dr.op = r.op0;
  // each op as (row-bit indices, its matrix entries' indices)
  for (int vi = 0; vi < (1 << nq); ++vi) {
    auto bit = [&](int q) {
      for (int b = 0; b < nq; ++b)
        if (r.qubits[b] == q) return (vi >> b) & 1;
      return 0;
    };
    cplx F[16][16];
    for (int u = 0; u < 16; ++u)
      for (int w = 0; w < 16; ++w) F[u][w] = u == w ? 1.0 : 0.0;
    for (int k = r.op0; k < r.op1; ++k) {
      const SweepOp &so = ops[k];
      const int n = 1 << so.np;
      int rb[PWS_SWEEP_MAXNP], obits = 0;
      for (int j = 0; j < so.np; ++j) {
        rb[j] = (int)(std::find(pos, pos + 4, (int)so.pos[j]) - pos);
        obits |= 1 << rb[j];
      }
      int spread[16], local[16];
      for (int x = 0; x < n; ++x) {
        int u = 0;
        for (int j = 0; j < so.np; ++j) u |= ((x >> j) & 1) << rb[j];
        spread[x] = u;
      }
      for (int u = 0; u < 16; ++u) {
        int x = 0;
        for (int j = 0; j < so.np; ++j) x |= ((u >> rb[j]) & 1) << j;
        local[u] = x;
      }
      // the op's matrix M[o][i] for these chain bits
      cplx M[256];
      for (int o = 0; o < n; ++o)
        for (int i = 0; i < n; ++i) {
          cplx m = 0.0;
          if (so.diag == 1) {
            if (o == i) m = entry_value(prog, sd, so.moff + o, bit);
          } else if (!(so.diag == 2 && ((o ^ i) & 2))) {   // block-diagonal: structural zeros
            m = entry_value(prog, sd, so.moff + o * n + i, bit);
          }
          M[o * n + i] = m;
        }
      cplx G[16][16];
      for (int u = 0; u < 16; ++u) {
        const int o = local[u], rest = u & ~obits;
        for (int w = 0; w < 16; ++w) G[u][w] = 0.0;
        for (int i = 0; i < n; ++i) {
          const cplx m = M[o * n + i];
          if (m == 0.0) continue;
          const cplx *Fr = F[rest | spread[i]];
          for (int w = 0; w < 16; ++w) G[u][w] += m * Fr[w];
        }
      }
      for (int u = 0; u < 16; ++u)
        for (int w = 0; w < 16; ++w) F[u][w] = G[u][w];
    }
    // Tables are laid out so that each matrix-core operand register set is
    // one contiguous read.  FP32: entry (u, w) as the words fl32(re),
    // fl32(im) at 2 (16 w + u) (column-major).  bf16: x = hi + lo with
    // hi = rn_bf16(x) and lo = rn_bf16(x - hi) (x the double value); the
    // operand of lane l (row u = l % 16, columns w = 4 (l / 16) + q, q < 4) is
    // the four pairs (Re F[u][w], -Im F[u][w]), the first in the low half:
    // part p (0: hi, 1: lo) of pair q at word 256 p + 4 l + q.
    const size_t at = prog.dtab.size();
    prog.dtab.resize(at + 512);
    for (int u = 0; u < 16; ++u)
      for (int w = 0; w < 16; ++w) {
        if (split_bf16) {
          const double x[2] = {F[u][w].real(), -F[u][w].imag()};
          const int word = 4 * (16 * (w / 4) + u) + w % 4;
          for (int c = 0; c < 2; ++c) {
            const double h = round_bf16(x[c]);
            const uint32_t bh = bf16_bits(h), bl = bf16_bits(round_bf16(x[c] - h));
            prog.dtab[at + word] |= bh << (16 * c);
            prog.dtab[at + 256 + word] |= bl << (16 * c);
          }
        } else {
          const double x[2] = {F[u][w].real(), F[u][w].imag()};
          for (int c = 0; c < 2; ++c) {
            const float f = (float)x[c];
            uint32_t word;
            std::memcpy(&word, &f, 4);
            prog.dtab[at + 2 * (16 * w + u) + c] = word;
          }
        }
      }
  }
  prog.druns.push_back(dr);
}

// Renormalisation of dense runs.  A run's matrix is a product of unitary
// gate blocks and projections on chain bits, so a run moves the tensor's
// largest magnitude by a few binary orders (at most about 3 on the measured
// workloads), far inside FP32's range: a run renormalises once
// kDenseRenormRuns runs have passed without one along the path its tensor
// took, which for a restoring pass starts at the previous keeping step's
// count at its kept point (a step kept without runs counts as due).  The
// sweep ops' own flags (every few ops and at the step's end) stay for the
// op-by-op form.
void flag_dense_renorm(Programs &prog) {
  constexpr int kDenseRenormRuns = 8;
  int carry = kDenseRenormRuns;
  for (StepDesc &sd : prog.steps) {
    if (sd.dn_count == 0) {
      if (sd.store_op >= 0) carry = kDenseRenormRuns;
      continue;
    }
    // amplitude calls run every run from a fresh tensor, sampling passes
    // from the restore point on (the larger count where the two meet)
    int cnt_amp = 0, cnt = sd.load_op >= 0 ? carry : 0, carry_next = -1;
    for (int r = 0; r < sd.dn_count; ++r) {
      DenseRun &dr = prog.druns[sd.dn_begin + r];
      int &c = r < sd.dn_load ? cnt_amp : cnt;
      if (r == sd.dn_load) cnt = std::max(cnt, cnt_amp);
      if (r >= sd.dn_load && dr.op == sd.store_op) carry_next = cnt;   // kept before this run
      const bool due = ++c >= kDenseRenormRuns;
      if (due) c = 0;
      dr.info = (dr.info & ~(1 << 16)) | ((due ? 1 : 0) << 16);
    }
    if (sd.store_op >= 0) carry = carry_next >= 0 ? carry_next : std::max(cnt, cnt_amp);
  }
}

}  // namespace

void build_dense(Programs &prog, bool split_bf16, uint64_t full_bytes, uint64_t max_bytes) {
  const int n_steps = (int)prog.steps.size();
  std::vector<std::vector<RunBuild>> runs(n_steps);
  std::vector<char> ok(n_steps, 0);
  std::vector<int> op0(n_steps, 0);
  // every op when the tables stay within full_bytes, else the ops a
  // sampling pass runs (from the restore point on)
  for (int cover_all = 1; cover_all >= 0; --cover_all) {
    uint64_t total = 0;
    for (int k = 0; k < n_steps; ++k) {
      const StepDesc &sd = prog.steps[k];
      ok[k] = 0;
      // (run records hold positions as nibbles)
      if (!sd.sweep || sd.fresh || sd.sw_count == 0 || sd.sw_width > 15) continue;
      op0[k] = cover_all ? 0 : std::max(sd.load_op, 0);
      if (op0[k] >= sd.sw_count) continue;
      ok[k] = partition_step(prog, sd, op0[k], runs[k]);
      if (ok[k]) total += table_bytes(runs[k]);
    }
    if (!cover_all || total <= full_bytes) break;
  }
  prog.druns.clear();
  prog.dtab.clear();
  prog.n_dense_steps = 0;
  prog.dense_bf16 = split_bf16;
  for (int k = 0; k < n_steps; ++k) {
    StepDesc &sd = prog.steps[k];
    sd.dn_begin = (int32_t)prog.druns.size();
    sd.dn_count = 0;
    sd.dn_op0 = 0;
    sd.dn_w = 0;
    sd.dn_load = 0;
    if (sd.sweep && sd.fresh) sd.dn_w = std::max(sd.sw_width, 4);
    if (!ok[k]) continue;
    if ((uint64_t)prog.dtab.size() * 4 + table_bytes(runs[k]) > max_bytes) continue;
    const int W = std::max(sd.sw_width, 4);
    for (const RunBuild &r : runs[k]) emit_run(prog, sd, r, W, split_bf16);
    sd.dn_count = (int32_t)(prog.druns.size() - sd.dn_begin);
    sd.dn_op0 = op0[k];
    sd.dn_w = W;
    // a restoring pass skips the runs before the restore point (all of
    // them when the kept tensor is the step's whole network)
    for (int r = 0; r < sd.dn_count; ++r)
      if (prog.druns[sd.dn_begin + r].op < std::max(sd.load_op, op0[k])) sd.dn_load = r + 1;
    ++prog.n_dense_steps;
  }
  flag_dense_renorm(prog);
}

}  // namespace pws
