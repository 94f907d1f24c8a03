// Circuit lowering: gate matrices, the monomial / diagonal / block
// classification of Algorithm 1 (UpdateState, BlockDecompose), qubit
// segments (legs of gates that are diagonal on a qubit are identified,
// Appendix A) and the Kraus factor tables of Algorithm 2 / Eq. (4).
#include <algorithm>
#include <climits>
#include <cmath>
#include <string>

#include "host.hpp"

// Kraus column norms feed draws that must match the oracle bit for bit:
// keep every product and sum separately rounded.
#pragma STDC FP_CONTRACT OFF

namespace pws {

namespace {

const cd I1(0.0, 1.0);

void set_rot1(cd *m, double t, int pauli) {  // exp(-i t P / 2), P in {X=1, Z=3}
  const double c = std::cos(t / 2), s = std::sin(t / 2);
  if (pauli == 1) {
    m[0] = cd(c, 0); m[1] = cd(0, -s); m[2] = cd(0, -s); m[3] = cd(c, 0);
  } else {
    m[0] = cd(c, -s); m[1] = 0; m[2] = 0; m[3] = cd(c, s);
  }
}

void matmul(const cd *a, const cd *b, cd *out, int d) {
  cd t[16];
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      cd acc = 0;
      for (int k = 0; k < d; ++k) acc += a[i * d + k] * b[k * d + j];
      t[i * d + j] = acc;
    }
  for (int i = 0; i < d * d; ++i) out[i] = t[i];
}

double angle(const pws_gate &g, const double *theta, bool second) {
  const int p = second ? g.param2 : g.param;
  const double co = second ? g.coeff2 : g.coeff, of = second ? g.offset2 : g.offset;
  double a = of;
  if (p >= 0) a += co * theta[p];
  return a;
}

int bit_of(int local, int j, int nq) { return (local >> (nq - 1 - j)) & 1; }

}  // namespace

// Matrices (and the derivative of a single-angle rotation) of one gate at the
// given angles, and its classification: monomial / diagonal / diagonal on each
// qubit, the permutation of a monomial gate, and the candidate masks of
// BlockDecompose (Algorithm 1).
std::string fill_gate(const pws_gate &g, const double *theta, GateIR &G) {
  const int d = 1 << G.nq;
  for (int i = 0; i < 16; ++i) { G.mat[i] = 0; G.dmat[i] = 0; }
  const double t = angle(g, theta, false);
  switch (g.kind) {
    case PWS_GATE_H: {
      const double r = 1.0 / std::sqrt(2.0);
      G.mat[0] = r; G.mat[1] = r; G.mat[2] = r; G.mat[3] = -r;
      break;
    }
    case PWS_GATE_X: G.mat[1] = 1; G.mat[2] = 1; break;
    case PWS_GATE_RX: set_rot1(G.mat, t, 1); break;
    case PWS_GATE_RZ: set_rot1(G.mat, t, 3); break;
    case PWS_GATE_RZZ: {
      const double cc = std::cos(t / 2), s = std::sin(t / 2);
      for (int l = 0; l < 4; ++l) {
        const int par = bit_of(l, 0, 2) ^ bit_of(l, 1, 2);
        G.mat[l * 4 + l] = par ? cd(cc, s) : cd(cc, -s);
      }
      break;
    }
    case PWS_GATE_CNOT:
      for (int b0 = 0; b0 < 2; ++b0)
        for (int b1 = 0; b1 < 2; ++b1) G.mat[(2 * b0 + (b1 ^ b0)) * 4 + 2 * b0 + b1] = 1;
      break;
    case PWS_GATE_CZ:
      G.mat[0] = 1; G.mat[5] = 1; G.mat[10] = 1; G.mat[15] = -1;
      break;
    case PWS_GATE_CRX: {
      cd r[4];
      set_rot1(r, t, 1);
      G.mat[0] = 1; G.mat[5] = 1;
      G.mat[10] = r[0]; G.mat[11] = r[1]; G.mat[14] = r[2]; G.mat[15] = r[3];
      break;
    }
    case PWS_GATE_FSIM: {
      const double ph = angle(g, theta, true);
      G.mat[0] = 1;
      G.mat[5] = std::cos(t); G.mat[10] = std::cos(t);
      G.mat[6] = cd(0, -std::sin(t)); G.mat[9] = cd(0, -std::sin(t));
      G.mat[15] = std::exp(I1 * ph);
      break;
    }
    case PWS_GATE_U1:
    case PWS_GATE_U2:
      if (!g.matrix) return "U1/U2 gate without matrix";
      for (int i = 0; i < d * d; ++i) G.mat[i] = cd(g.matrix[2 * i], g.matrix[2 * i + 1]);
      break;
  }
  // derivative of the single-angle rotations, times d(angle)/d(theta) = coeff
  if (g.param >= 0) {
    cd P[16] = {};
    bool has = true;
    if (g.kind == PWS_GATE_RX) { P[1] = 1; P[2] = 1; }
    else if (g.kind == PWS_GATE_RZ) { P[0] = 1; P[3] = -1; }
    else if (g.kind == PWS_GATE_RZZ) { P[0] = 1; P[5] = -1; P[10] = -1; P[15] = 1; }
    else if (g.kind == PWS_GATE_CRX) { P[11] = 1; P[14] = 1; }
    else has = false;
    if (has) {
      matmul(P, G.mat, G.dmat, d);
      for (int i = 0; i < d * d; ++i) G.dmat[i] *= cd(0, -0.5) * g.coeff;
    }
  }
  // classification (Algorithm 1: monomial test, BlockDecompose)
  G.diagonal = true;
  for (int o = 0; o < d; ++o)
    for (int i = 0; i < d; ++i)
      if (o != i && G.mat[o * d + i] != cd(0)) G.diagonal = false;
  G.monomial = true;
  for (int i = 0; i < d; ++i) {
    int cnt_col = 0, cnt_row = 0;
    for (int o = 0; o < d; ++o) {
      if (G.mat[o * d + i] != cd(0)) { ++cnt_col; G.sigma[i] = o; }
      if (G.mat[i * d + o] != cd(0)) ++cnt_row;
    }
    if (cnt_col != 1 || cnt_row != 1) G.monomial = false;
  }
  G.nS = 0;
  for (int j = 0; j < G.nq; ++j) {
    bool dj = true;
    for (int o = 0; o < d; ++o)
      for (int i = 0; i < d; ++i)
        if (bit_of(o, j, G.nq) != bit_of(i, j, G.nq) && G.mat[o * d + i] != cd(0)) dj = false;
    G.diag_on[j] = dj;
    if (!dj) G.sq[G.nS++] = j;
  }
  // candidate masks: block of each local value, restricted to the S bits
  for (int l = 0; l < d; ++l) {
    int comp[4] = {0, 0, 0, 0};
    comp[l] = 1;
    bool grown = true;
    while (grown) {
      grown = false;
      for (int x = 0; x < d; ++x)
        if (comp[x])
          for (int y = 0; y < d; ++y)
            if (!comp[y] && (G.mat[x * d + y] != cd(0) || G.mat[y * d + x] != cd(0))) {
              comp[y] = 1;
              grown = true;
            }
    }
    int mask = 0;
    for (int v = 0; v < (1 << G.nS); ++v) {
      int loc = l;
      for (int k = 0; k < G.nS; ++k) {
        const int j = G.sq[k];
        const int bit = (v >> (G.nS - 1 - k)) & 1;
        const int pos = G.nq - 1 - j;
        loc = (loc & ~(1 << pos)) | (bit << pos);
      }
      if (comp[loc]) mask |= 1 << v;
    }
    G.cand_mask[l] = mask;
  }
  return "";
}

std::string lower(const pws_circuit *c, const pws_noise *noise, CircuitIR &ir) {
  if (!c) return "circuit is NULL";
  if (c->n_qubits <= 0) return "n_qubits must be positive";
  if (c->n_gates < 0 || (c->n_gates > 0 && !c->gates)) return "bad gate list";
  if (c->n_params < 0 || (c->n_params > 0 && !c->theta)) return "bad theta";
  ir = CircuitIR();
  ir.n = c->n_qubits;
  ir.n_params = c->n_params;
  ir.theta.assign(c->theta, c->theta + c->n_params);
  ir.specs.clear();
  ir.spec_mats.clear();
  const int n = ir.n;
  ir.gates.resize(c->n_gates);
  for (int gi = 0; gi < c->n_gates; ++gi) {
    const pws_gate &g = c->gates[gi];
    GateIR &G = ir.gates[gi];
    G.kind = g.kind;
    const bool two = (g.kind == PWS_GATE_RZZ || g.kind == PWS_GATE_CNOT || g.kind == PWS_GATE_CZ ||
                      g.kind == PWS_GATE_U2 || g.kind == PWS_GATE_CRX || g.kind == PWS_GATE_FSIM);
    if (g.kind < 0 || g.kind > PWS_GATE_FSIM) return "unknown gate kind at gate " + std::to_string(gi);
    G.nq = two ? 2 : 1;
    G.q[0] = g.q0;
    G.q[1] = two ? g.q1 : -1;
    for (int j = 0; j < G.nq; ++j)
      if (G.q[j] < 0 || G.q[j] >= n) return "qubit out of range at gate " + std::to_string(gi);
    if (two && G.q[0] == G.q[1]) return "repeated qubit at gate " + std::to_string(gi);
    if (g.param >= c->n_params || g.param2 >= c->n_params)
      return "parameter index out of range at gate " + std::to_string(gi);
    G.param = g.param;
    G.param2 = g.param2;
    G.coeff = g.coeff;
    G.coeff2 = g.coeff2;
    const std::string ferr = fill_gate(g, c->theta, G);
    if (!ferr.empty()) return ferr + " at gate " + std::to_string(gi);
    ir.specs.push_back(g);
    if (g.matrix) ir.spec_mats.emplace_back(g.matrix, g.matrix + 2 * (1 << G.nq) * (1 << G.nq));
    else ir.spec_mats.emplace_back();
  }
  // segments: a qubit's segment ends at every gate that is not diagonal on it
  std::vector<int> cnt(n, 1);
  for (auto &G : ir.gates)
    for (int j = 0; j < G.nq; ++j)
      if (!G.diag_on[j]) cnt[G.q[j]]++;
  ir.seg_base.assign(n, 0);
  int tot = 0;
  for (int q = 0; q < n; ++q) { ir.seg_base[q] = tot; tot += cnt[q]; }
  ir.n_segs = tot;
  ir.seg_qubit.assign(tot, 0);
  for (int q = 0; q < n; ++q)
    for (int k = 0; k < cnt[q]; ++k) ir.seg_qubit[ir.seg_base[q] + k] = q;
  std::vector<int> cur(n);
  for (int q = 0; q < n; ++q) cur[q] = ir.seg_base[q];
  // current segment of every qubit after each gate (needed for noise sites)
  std::vector<std::vector<int>> cur_after_gate_site;  // filled lazily below
  // noise sites
  const int ns = noise ? noise->n_sites : 0;
  if (ns < 0 || (ns > 0 && !noise->sites)) return "bad noise list";
  ir.noisy = ns > 0;
  ir.readout.clear();
  if (noise && noise->readout) {
    bool any = false;
    for (int q = 0; q < n; ++q) {
      const double r = noise->readout[q];
      if (!(r >= 0.0 && r <= 1.0)) return "readout probability out of [0,1]";
      any |= r > 0.0;
    }
    if (any) ir.readout.assign(noise->readout, noise->readout + n);
  }
  std::vector<std::vector<int>> sites_after(c->n_gates);
  for (int si = 0; si < ns; ++si) {
    const pws_noise_site &s = noise->sites[si];
    if (s.after_gate < 0 || s.after_gate >= c->n_gates) return "noise after_gate out of range";
    sites_after[s.after_gate].push_back(si);
  }
  ir.noise.resize(ns);
  ir.gate_op.assign(c->n_gates, 0);
  ir.first_noise_op_on_q.assign(n, INT_MAX);
  for (int gi = 0; gi < c->n_gates; ++gi) {
    GateIR &G = ir.gates[gi];
    for (int j = 0; j < G.nq; ++j) {
      const int q = G.q[j];
      G.in_seg[j] = cur[q];
      if (!G.diag_on[j]) cur[q] += 1;
      G.out_seg[j] = cur[q];
    }
    ir.gate_op[gi] = (int)ir.ops.size();
    ir.ops.push_back({0, gi});
    for (int si : sites_after[gi]) {
      const pws_noise_site &s = noise->sites[si];
      NoiseIR &N = ir.noise[si];
      N.kind = s.kind;
      N.after_gate = s.after_gate;
      const bool two = s.kind == PWS_NOISE_DEPOL2;
      if (s.kind < 0 || s.kind > PWS_NOISE_PAULI1) return "unsupported noise kind (not local-submonomial)";
      N.nq = two ? 2 : 1;
      N.q[0] = s.q0;
      N.q[1] = two ? s.q1 : -1;
      for (int j = 0; j < N.nq; ++j) {
        if (N.q[j] < 0 || N.q[j] >= n) return "noise qubit out of range";
        N.seg[j] = cur[N.q[j]];
        ir.first_noise_op_on_q[N.q[j]] = std::min(ir.first_noise_op_on_q[N.q[j]], (int)ir.ops.size());
      }
      if (two && N.q[0] == N.q[1]) return "repeated noise qubit";
      // Kraus factors (each E_i a tensor product of 2x2 factors)
      const cd pauli[4][4] = {{1, 0, 0, 1}, {0, 1, 1, 0}, {0, cd(0, -1), cd(0, 1), 0}, {1, 0, 0, -1}};
      std::vector<std::vector<std::vector<cd>>> fl;   // branch -> factor -> 4 entries
      auto scaled = [&](int a, double sw) {
        std::vector<cd> m(4);
        for (int e = 0; e < 4; ++e) m[e] = pauli[a][e] * sw;
        return m;
      };
      auto plain = [&](int a) { return std::vector<cd>(pauli[a], pauli[a] + 4); };
      if (s.kind == PWS_NOISE_DEPOL1 || s.kind == PWS_NOISE_PAULI1) {
        double w[4];
        if (s.kind == PWS_NOISE_DEPOL1) {
          w[0] = 1.0 - s.p[0]; w[1] = w[2] = w[3] = s.p[0] / 3.0;
        } else {
          w[0] = 1.0 - s.p[0] - s.p[1] - s.p[2]; w[1] = s.p[0]; w[2] = s.p[1]; w[3] = s.p[2];
        }
        for (int a = 0; a < 4; ++a) {
          if (w[a] < 0) return "negative noise probability";
          fl.push_back({scaled(a, std::sqrt(w[a]))});
        }
      } else if (s.kind == PWS_NOISE_DEPOL2) {
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b) {
            const double w = (a == 0 && b == 0) ? 1.0 - s.p[0] : s.p[0] / 15.0;
            if (w < 0) return "negative noise probability";
            fl.push_back({scaled(a, std::sqrt(w)), plain(b)});
          }
      } else if (s.kind == PWS_NOISE_AMPDAMP) {
        const double gm = s.p[0];
        if (gm < 0 || gm > 1) return "amplitude damping rate out of [0,1]";
        fl.push_back({{1, 0, 0, std::sqrt(1.0 - gm)}});
        fl.push_back({{0, std::sqrt(gm), 0, 0}});
      } else {  // PHASEDAMP
        const double lam = s.p[0];
        if (lam < 0 || lam > 1) return "phase damping rate out of [0,1]";
        fl.push_back({{1, 0, 0, std::sqrt(1.0 - lam)}});
        fl.push_back({{0, 0, 0, std::sqrt(lam)}});
      }
      N.nbranch = (int)fl.size();
      for (auto &br : fl)
        for (int j = 0; j < N.nq; ++j) {
          const auto &M = br[j];
          NoiseBranch nb{};
          for (int t = 0; t < 2; ++t) {
            const cd a = M[0 * 2 + t], b = M[1 * 2 + t];
            nb.colnorm[t] = (a.real() * a.real() + a.imag() * a.imag()) +
                            (b.real() * b.real() + b.imag() * b.imag());
          }
          nb.anti = (M[0] == cd(0) && M[3] == cd(0)) ? 1 : 0;
          cd d0 = nb.anti ? M[1] : M[0];   // diagonal of M sigma_X = (M01, M10)
          cd d1 = nb.anti ? M[2] : M[3];
          nb.d0re = d0.real(); nb.d0im = d0.imag();
          nb.d1re = d1.real(); nb.d1im = d1.imag();
          N.tab.push_back(nb);
        }
      ir.ops.push_back({1, si});
    }
  }
  return "";
}

std::string set_theta(CircuitIR &ir, const double *theta) {
  std::vector<GateIR> next = ir.gates;
  for (size_t gi = 0; gi < ir.gates.size(); ++gi) {
    pws_gate g = ir.specs[gi];
    g.matrix = ir.spec_mats[gi].empty() ? nullptr : ir.spec_mats[gi].data();
    GateIR &G = next[gi];
    const std::string err = fill_gate(g, theta, G);
    if (!err.empty()) return err;
    const GateIR &O = ir.gates[gi];
    bool same = G.diagonal == O.diagonal && G.monomial == O.monomial && G.nS == O.nS;
    for (int j = 0; j < 2; ++j) same = same && G.diag_on[j] == O.diag_on[j] && G.sq[j] == O.sq[j];
    for (int i = 0; i < 4; ++i) same = same && G.cand_mask[i] == O.cand_mask[i] && G.sigma[i] == O.sigma[i];
    if (!same) return "gate " + std::to_string(gi) + " changes its structure at these angles: plan again";
  }
  ir.gates.swap(next);
  ir.theta.assign(theta, theta + ir.n_params);
  return "";
}

}  // namespace pws
