// Per-step tensor networks, leaf fusion, contraction-tree planning, index
// slicing and emission of the device programs.
//
// Network of a prefix C_t (Section 2, amp(C_t, i) as a tensor-network
// contraction): every gate is a tensor over the segments it touches; a gate
// that is diagonal on a qubit keeps the qubit on one segment, so its in and
// out legs are one hyperedge (Appendix A).  The first segment of each qubit is
// fixed to |0>, the last one to the chain's bit s[q] (projection), except for
// the step gate's non-diagonal qubits S, whose last segments stay open (the
// 2^|S| candidates of the block).  One-leg and lower-rank tensors are fused
// into a neighbour that holds all their legs (step (i) in Appendix A), so the
// noisy network (extra one-qubit diagonal factors, Proposition 2) has the same
// shape as the ideal one.
//
// The tree of pairwise contractions is chosen per step: the best (fewest
// multiply-adds, then smallest peak) of a greedy pair search (with randomised
// restarts) and linear sweeps along low-cutwidth qubit orders.  When one
// chain's working set exceeds the arena limit, legs are sliced (fixed to each
// value in turn and the root accumulated).
#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <complex>
#include <cstdio>
#include <functional>
#include <map>
#include <numeric>
#include <queue>
#include <random>
#include <set>
#include <sstream>

#include "device.hpp"
#include "host.hpp"

namespace pws {

// ------------------------------------------------------------------ network

StepNet build_step_net(const CircuitIR &ir, int gate_limit, const std::vector<int> &open_qubits,
                       int op, bool full_projection) {
  StepNet net;
  net.op = op;
  net.gate = full_projection ? -1 : gate_limit;
  const int n = ir.n;
  std::vector<int> last(n);
  for (int q = 0; q < n; ++q) last[q] = ir.seg_base[q];
  for (int g = 0; g <= gate_limit; ++g) {
    const GateIR &G = ir.gates[g];
    for (int j = 0; j < G.nq; ++j) last[G.q[j]] = G.out_seg[j];
  }
  std::vector<char> is_open(n, 0);
  for (int q : open_qubits) is_open[q] = 1;
  for (int q : open_qubits) net.open_legs.push_back(last[q]);
  for (int q = 0; q < n; ++q)
    if (!is_open[q] && last[q] == ir.seg_base[q]) net.zero_q.push_back(q);

  auto src_of = [&](int leg) -> int32_t {
    const int q = ir.seg_qubit[leg];
    if (leg == ir.seg_base[q]) return src_make(SRC_CONST, 0);
    if (leg == last[q] && !is_open[q]) return src_make(SRC_CHAIN, q);
    return src_make(SRC_FREE, leg);
  };
  auto add_factor = [&](FactorDesc f) {
    LeafBuild lb;
    for (int j = 0; j < f.nq; ++j) {
      for (int32_t s : {f.src_out[j], f.src_in[j]}) {
        if (src_type(s) == SRC_FREE) lb.legs.push_back(src_payload(s));
        if (src_type(s) == SRC_CHAIN) lb.chain = true;
      }
    }
    if (f.frame || f.kind == FAC_SEGFAC) lb.chain = true;
    std::sort(lb.legs.begin(), lb.legs.end());
    lb.legs.erase(std::unique(lb.legs.begin(), lb.legs.end()), lb.legs.end());
    lb.factors.push_back(f);
    net.leaves.push_back(lb);
  };
  for (int g = 0; g <= gate_limit; ++g) {
    const GateIR &G = ir.gates[g];
    FactorDesc f{};
    f.kind = FAC_GATE;
    f.id = g;
    f.nq = G.nq;
    f.frame = 0;
    if (ir.noisy && !full_projection)
      for (int j = 0; j < G.nq; ++j)
        if (ir.first_noise_op_on_q[G.q[j]] < ir.gate_op[g]) f.frame = 1;
    for (int j = 0; j < 2; ++j) { f.src_out[j] = src_make(SRC_CONST, 0); f.src_in[j] = src_make(SRC_CONST, 0); }
    for (int j = 0; j < G.nq; ++j) {
      f.src_in[j] = src_of(G.in_seg[j]);
      f.src_out[j] = src_of(G.out_seg[j]);
    }
    add_factor(f);
  }
  if (ir.noisy && !full_projection) {
    std::set<int> segs;
    for (size_t si = 0; si < ir.noise.size(); ++si) {
      const NoiseIR &N = ir.noise[si];
      // sites executed before this step's gate
      if (ir.gate_op[N.after_gate] >= ir.gate_op[gate_limit]) continue;
      for (int j = 0; j < N.nq; ++j) segs.insert(N.seg[j]);
    }
    for (int sg : segs) {
      FactorDesc f{};
      f.kind = FAC_SEGFAC;
      f.id = sg;
      f.nq = 1;
      f.src_out[0] = f.src_in[0] = src_of(sg);
      f.src_out[1] = f.src_in[1] = src_make(SRC_CONST, 0);
      add_factor(f);
    }
  }
  return net;
}

void fuse_leaves(StepNet &net, bool split_scalars) {
  if (split_scalars) {
    // tensors with every leg fixed are a per-chain scalar shared by all
    // candidates: keep them out of the network (a long product of them would
    // leave the single-precision range on large circuits)
    std::vector<LeafBuild> keep;
    for (auto &l : net.leaves) {
      if (l.legs.empty()) net.scalars.insert(net.scalars.end(), l.factors.begin(), l.factors.end());
      else keep.push_back(l);
    }
    if (keep.empty()) keep.push_back(LeafBuild());
    net.leaves.swap(keep);
  }
  const int L = (int)net.leaves.size();
  std::vector<int> order(L);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return net.leaves[a].legs.size() < net.leaves[b].legs.size();
  });
  std::map<int, std::vector<int>> by_leg;
  for (int i = 0; i < L; ++i)
    for (int l : net.leaves[i].legs) by_leg[l].push_back(i);
  std::vector<int> parent(L, -1);
  int first_nonempty = -1;
  for (int i = 0; i < L; ++i)
    if (!net.leaves[i].legs.empty()) { first_nonempty = i; break; }
  for (int t : order) {
    const auto &lt = net.leaves[t].legs;
    int best = -1;
    if (lt.empty()) {
      best = (first_nonempty >= 0 && first_nonempty != t) ? first_nonempty : -1;
    } else {
      for (int h : by_leg[lt[0]]) {
        if (h == t) continue;
        const auto &lh = net.leaves[h].legs;
        if (lh.size() < lt.size() || (lh.size() == lt.size() && h > t)) continue;
        if (!std::includes(lh.begin(), lh.end(), lt.begin(), lt.end())) continue;
        if (best < 0 || lh.size() < net.leaves[best].legs.size() ||
            (lh.size() == net.leaves[best].legs.size() && h < best))
          best = h;
      }
    }
    parent[t] = best;
  }
  auto root = [&](int i) { while (parent[i] >= 0) i = parent[i]; return i; };
  std::vector<int> gid(L, -1);
  std::vector<LeafBuild> out;
  for (int i = 0; i < L; ++i) {
    if (parent[i] >= 0) continue;
    gid[i] = (int)out.size();
    out.push_back(net.leaves[i]);
  }
  for (int i = 0; i < L; ++i) {
    if (parent[i] < 0) continue;
    LeafBuild &h = out[gid[root(i)]];
    for (auto &f : net.leaves[i].factors) h.factors.push_back(f);
    h.chain = h.chain || net.leaves[i].chain;
  }
  if (out.size() == 1) {  // a lone tensor still needs its dangling legs summed
    LeafBuild unit;
    out.push_back(unit);
  }
  net.leaves.swap(out);
}

// ------------------------------------------------------------------ tree evaluation

namespace {

struct Holders {
  std::vector<int> count;   // per leg: number of alive tensors holding it
  std::vector<char> open;
};

std::vector<int> contract_legs(const std::vector<int> &a, const std::vector<int> &b, Holders &h) {
  std::vector<int> u;
  std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(u));
  std::vector<int> out;
  for (int l : u) {
    int c = h.count[l];
    if (std::binary_search(a.begin(), a.end(), l)) --c;
    if (std::binary_search(b.begin(), b.end(), l)) --c;
    if (c > 0 || h.open[l]) out.push_back(l);
  }
  return out;
}

void apply_contraction(const std::vector<int> &a, const std::vector<int> &b,
                       const std::vector<int> &out, Holders &h) {
  for (int l : a) h.count[l]--;
  for (int l : b) h.count[l]--;
  for (int l : out) h.count[l]++;
}

int max_leg(const std::vector<std::vector<int>> &legs, const std::vector<int> &open) {
  int m = 0;
  for (auto &v : legs)
    for (int l : v) m = std::max(m, l + 1);
  for (int l : open) m = std::max(m, l + 1);
  return m;
}

Holders make_holders(const std::vector<std::vector<int>> &legs, const std::vector<int> &open) {
  Holders h;
  const int m = max_leg(legs, open);
  h.count.assign(m, 0);
  h.open.assign(m, 0);
  for (auto &v : legs)
    for (int l : v) h.count[l]++;
  for (int l : open) h.open[l] = 1;
  return h;
}

inline double p2(size_t k) { return std::ldexp(1.0, (int)k); }

}  // namespace

// Elements a node kernel moves for out = contract(a, b) (see the node forms
// in program.hpp).  Blocked form: the larger operand once, the other once per
// 64 lanes of its own-only output legs, the output once.  Generic form: both
// operands gathered once per output element and contracted value.
double kernel_traffic(const std::vector<int> &a0, const std::vector<int> &b0, const std::vector<int> &o) {
  const bool sw = b0.size() > a0.size();
  const std::vector<int> &a = sw ? b0 : a0, &b = sw ? a0 : b0;
  int nM = 0, nN = 0;
  for (int l : o) {
    const bool ina = std::binary_search(a.begin(), a.end(), l), inb = std::binary_search(b.begin(), b.end(), l);
    if (ina && !inb) nM++;
    if (!ina) nN++;
  }
  std::vector<int> u;
  std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(u));
  const int nK = (int)u.size() - (int)o.size();
  if (nK <= PWS_BLOCK_KBITS && nN <= PWS_BLOCK_NBITS)
    return p2(a.size()) + p2(b.size()) * std::max(1.0, std::ldexp(1.0, nM - 6)) + p2(o.size());
  return 2.0 * p2(o.size() + nK) + p2(o.size());
}

TreeCost eval_tree(const std::vector<std::vector<int>> &legs, const std::vector<int> &open_legs,
                   const std::vector<Pair> &pairs) {
  TreeCost c;
  Holders h = make_holders(legs, open_legs);
  std::vector<std::vector<int>> T = legs;
  double live = 0;
  for (auto &v : legs) {
    live += p2(v.size());
    c.max_bits = std::max(c.max_bits, (int)v.size());
  }
  c.peak = live;
  for (const Pair &p : pairs) {
    std::vector<int> out = contract_legs(T[p.a], T[p.b], h);
    apply_contraction(T[p.a], T[p.b], out, h);
    std::vector<int> u;
    std::set_union(T[p.a].begin(), T[p.a].end(), T[p.b].begin(), T[p.b].end(), std::back_inserter(u));
    c.flops += p2(u.size());
    c.bytes += p2(T[p.a].size()) + p2(T[p.b].size()) + p2(out.size());
    c.kbytes += kernel_traffic(T[p.a], T[p.b], out);
    live += p2(out.size());
    c.peak = std::max(c.peak, live);
    live -= p2(T[p.a].size()) + p2(T[p.b].size());
    c.max_bits = std::max(c.max_bits, (int)out.size());
    T.push_back(out);
  }
  return c;
}

// ------------------------------------------------------------------ planners

namespace {

std::vector<Pair> greedy_tree(const std::vector<std::vector<int>> &legs, const std::vector<int> &open,
                              uint64_t seed, double noise) {
  const int L = (int)legs.size();
  Holders h = make_holders(legs, open);
  std::vector<std::vector<int>> T = legs;
  std::vector<char> alive(L, 1);
  std::vector<std::vector<int>> holders(h.count.size());
  for (int i = 0; i < L; ++i)
    for (int l : legs[i]) holders[l].push_back(i);
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  struct Cand { double score; uint64_t tie; int a, b; };
  auto cmp = [](const Cand &x, const Cand &y) {
    if (x.score != y.score) return x.score > y.score;
    return x.tie > y.tie;
  };
  std::priority_queue<Cand, std::vector<Cand>, decltype(cmp)> pq(cmp);
  auto push = [&](int a, int b) {
    if (a > b) std::swap(a, b);
    std::vector<int> out = contract_legs(T[a], T[b], h);
    double s = p2(out.size()) - p2(T[a].size()) - p2(T[b].size());
    if (noise > 0) s -= noise * std::log(-std::log(U(rng) + 1e-300)) * std::max(p2(T[a].size()), p2(T[b].size()));
    pq.push({s, (uint64_t)a * 1000003ull + (uint64_t)b, a, b});
  };
  {
    std::set<std::pair<int, int>> seen;
    for (size_t l = 0; l < holders.size(); ++l)
      for (size_t i = 0; i < holders[l].size(); ++i)
        for (size_t j = i + 1; j < holders[l].size(); ++j) {
          int a = holders[l][i], b = holders[l][j];
          if (a > b) std::swap(a, b);
          if (seen.insert({a, b}).second) push(a, b);
        }
  }
  std::vector<Pair> pairs;
  while (!pq.empty()) {
    Cand c = pq.top();
    pq.pop();
    if (!alive[c.a] || !alive[c.b]) continue;
    std::vector<int> out = contract_legs(T[c.a], T[c.b], h);
    apply_contraction(T[c.a], T[c.b], out, h);
    alive[c.a] = alive[c.b] = 0;
    for (int l : T[c.a]) {
      auto &v = holders[l];
      v.erase(std::remove(v.begin(), v.end(), c.a), v.end());
    }
    for (int l : T[c.b]) {
      auto &v = holders[l];
      v.erase(std::remove(v.begin(), v.end(), c.b), v.end());
    }
    const int id = (int)T.size();
    T.push_back(out);
    alive.push_back(1);
    pairs.push_back({c.a, c.b});
    std::set<int> nb;
    for (int l : out)
      for (int o : holders[l]) nb.insert(o);
    for (int l : out) holders[l].push_back(id);
    for (int o : nb) push(o, id);
  }
  // disconnected pieces: outer products, smallest first
  while (true) {
    std::vector<int> rest;
    for (int i = 0; i < (int)T.size(); ++i)
      if (alive[i]) rest.push_back(i);
    if (rest.size() <= 1) break;
    std::sort(rest.begin(), rest.end(), [&](int a, int b) {
      return T[a].size() < T[b].size() || (T[a].size() == T[b].size() && a < b);
    });
    int a = rest[0], b = rest[1];
    std::vector<int> out = contract_legs(T[a], T[b], h);
    apply_contraction(T[a], T[b], out, h);
    alive[a] = alive[b] = 0;
    T.push_back(out);
    alive.push_back(1);
    pairs.push_back({a, b});
  }
  return pairs;
}

// Linear order of qubits with a small cut: grow a visited set, always taking
// the frontier vertex that leaves the fewest visited vertices with
// unvisited neighbours.
std::vector<int> min_boundary_order(const std::vector<std::vector<int>> &adj, int start) {
  const int n = (int)adj.size();
  std::vector<char> vis(n, 0);
  std::vector<int> unvis_nb(n);
  for (int v = 0; v < n; ++v) unvis_nb[v] = (int)adj[v].size();
  std::vector<int> order;
  int boundary = 0;
  auto visit = [&](int v) {
    vis[v] = 1;
    order.push_back(v);
    if (unvis_nb[v] > 0) boundary++;
    for (int u : adj[v]) {
      unvis_nb[u]--;
      if (vis[u] && unvis_nb[u] == 0) boundary--;
    }
  };
  visit(start);
  while ((int)order.size() < n) {
    int best = -1, bb = 1 << 30, bv = -1;
    for (int v = 0; v < n; ++v) {
      if (vis[v]) continue;
      bool front = false;
      int nvis = 0;
      for (int u : adj[v])
        if (vis[u]) { front = true; nvis++; }
      if (!front) continue;
      int nb = boundary + (unvis_nb[v] > 0 ? 1 : 0);
      for (int u : adj[v])
        if (vis[u] && unvis_nb[u] == 1) nb--;
      if (nb < bb || (nb == bb && nvis > bv)) { best = v; bb = nb; bv = nvis; }
    }
    if (best < 0)
      for (int v = 0; v < n; ++v)
        if (!vis[v]) { best = v; break; }
    visit(best);
  }
  return order;
}

int cutwidth(const std::vector<std::vector<int>> &adj, const std::vector<int> &order) {
  const int n = (int)adj.size();
  std::vector<int> pos(n);
  for (int i = 0; i < n; ++i) pos[order[i]] = i;
  int best = 0;
  std::vector<int> diff(n + 1, 0);
  for (int v = 0; v < n; ++v)
    for (int u : adj[v])
      if (pos[u] > pos[v]) { diff[pos[v]]++; diff[pos[u]]--; }
  int cur = 0;
  for (int i = 0; i < n; ++i) { cur += diff[i]; best = std::max(best, cur); }
  return best;
}

std::vector<Pair> sweep_tree(const CircuitIR &ir, const std::vector<std::vector<int>> &legs,
                             const std::vector<int> &qorder) {
  const int L = (int)legs.size();
  std::vector<int> pos(ir.n);
  for (int i = 0; i < ir.n; ++i) pos[qorder[i]] = i;
  std::vector<std::tuple<int, int, int>> key;
  for (int i = 0; i < L; ++i) {
    int mx = -1, mn = 1 << 30;
    for (int l : legs[i]) {
      const int p = pos[ir.seg_qubit[l]];
      mx = std::max(mx, p);
      mn = std::min(mn, p);
    }
    key.emplace_back(mx, mn, i);
  }
  std::sort(key.begin(), key.end());
  std::vector<Pair> pairs;
  int acc = std::get<2>(key[0]);
  int next = L;
  for (int i = 1; i < L; ++i) {
    pairs.push_back({acc, std::get<2>(key[i])});
    acc = next++;
  }
  return pairs;
}

}  // namespace

void compute_qubit_orders(CircuitIR &ir) {
  std::vector<std::vector<int>> adj(ir.n);
  for (auto &G : ir.gates)
    if (G.nq == 2) {
      adj[G.q[0]].push_back(G.q[1]);
      adj[G.q[1]].push_back(G.q[0]);
    }
  for (auto &a : adj) {
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
  std::vector<std::pair<int, std::vector<int>>> cands;
  std::vector<int> ident(ir.n);
  std::iota(ident.begin(), ident.end(), 0);
  cands.push_back({cutwidth(adj, ident), ident});
  // start from low-degree vertices (corners) and a few others
  std::vector<int> starts;
  int mindeg = 1 << 30;
  for (int v = 0; v < ir.n; ++v) mindeg = std::min(mindeg, (int)adj[v].size());
  for (int v = 0; v < ir.n && starts.size() < 8; ++v)
    if ((int)adj[v].size() == mindeg) starts.push_back(v);
  starts.push_back(0);
  starts.push_back(ir.n - 1);
  starts.push_back(ir.n / 2);
  std::sort(starts.begin(), starts.end());
  starts.erase(std::unique(starts.begin(), starts.end()), starts.end());
  if (ir.n <= 600)
    for (int s : starts) {
      auto o = min_boundary_order(adj, s);
      cands.push_back({cutwidth(adj, o), o});
    }
  std::stable_sort(cands.begin(), cands.end(),
                   [](const auto &a, const auto &b) { return a.first < b.first; });
  ir.qorders.clear();
  for (size_t i = 0; i < cands.size() && i < 3; ++i) ir.qorders.push_back(cands[i].second);
}

std::vector<Pair> plan_tree(const CircuitIR &ir, const std::vector<std::vector<int>> &legs,
                            const std::vector<int> &open_legs, const PlanOptions &opt,
                            TreeCost *cost) {
  std::vector<Pair> best;
  TreeCost bc;
  bool have = false;
  auto consider = [&](std::vector<Pair> p) {
    TreeCost c = eval_tree(legs, open_legs, p);
    // modelled time: multiply-adds plus element traffic (an arena element moved
    // costs about as much as `traffic_weight` complex multiply-adds)
    auto cost = [&](const TreeCost &x, size_t nn) {
      if (opt.lds_mode) {
        // everything stays on chip: multiply-adds and per-node synchronisation,
        // times the slices needed to fit the arena
        const double s = std::max(0.0, std::ceil(std::log2(x.peak / (double)opt.arena_limit_elems)));
        return std::ldexp(x.flops + opt.node_overhead * (double)nn, (int)s);
      }
      return x.flops + opt.traffic_weight * x.kbytes;
    };
    const double tc = cost(c, p.size());
    const double tb = cost(bc, best.size());
    if (!have || tc < tb * (1 - 1e-12) || (tc <= tb * (1 + 1e-12) && c.peak < bc.peak)) {
      best.swap(p);
      bc = c;
      have = true;
    }
  };
  const int L = (int)legs.size();
  if (L == 1) {
    if (cost) *cost = eval_tree(legs, open_legs, {});
    return {};
  }
  if (opt.planner == 0 || opt.planner == 1) {
    consider(greedy_tree(legs, open_legs, 1, 0.0));
    int trials = opt.greedy_trials;
    if (L > 600) trials = std::min(trials, 2);
    for (int t = 1; t < trials; ++t) consider(greedy_tree(legs, open_legs, 1000 + t, 0.5));
  }
  if (opt.planner == 0 || opt.planner == 2) {
    for (auto &o : ir.qorders) consider(sweep_tree(ir, legs, o));
  }
  if (cost) *cost = bc;
  return best;
}

// ------------------------------------------------------------------ emission

namespace {

struct Arena {
  std::vector<std::pair<int, int>> free_;   // (offset, size), sorted by offset
  int top = 0;
  int peak = 0;                              // high-water mark: the arena size
  int alloc(int size) {
    size = (size + 1) & ~1;
    for (size_t i = 0; i < free_.size(); ++i)
      if (free_[i].second >= size) {
        const int off = free_[i].first;
        free_[i].first += size;
        free_[i].second -= size;
        if (free_[i].second == 0) free_.erase(free_.begin() + i);
        return off;
      }
    const int off = top;
    top += size;
    peak = std::max(peak, top);
    return off;
  }
  void release(int off, int size) {
    size = (size + 1) & ~1;
    free_.push_back({off, size});
    std::sort(free_.begin(), free_.end());
    std::vector<std::pair<int, int>> m;
    for (auto &f : free_) {
      if (!m.empty() && m.back().first + m.back().second == f.first) m.back().second += f.second;
      else m.push_back(f);
    }
    if (!m.empty() && m.back().first + m.back().second == top) {
      top = m.back().first;
      m.pop_back();
    }
    free_.swap(m);
  }
};

struct SlotPool {
  std::vector<int> free_;
  int top = 0;
  int alloc() {
    if (!free_.empty()) { int s = free_.back(); free_.pop_back(); return s; }
    return top++;
  }
  void release(int s) { if (s >= 0) free_.push_back(s); }
};

// Node descriptor for out = contract(a, b).  a and b are given in their
// storage order (position = bit of the flat index); o is the set of output
// legs.  Generic form: lanes over all output legs, stored in sorted order.
// Blocked form (few contracted legs K): lanes over the output legs held by a;
// with `free_order` the output is laid out as [legs of a only (M), legs of
// both (batch), legs of b only (N)], so consecutive lanes store consecutive
// elements and, once M spans the 64 lanes, every lane of a wave reads the same
// element of b.  The chosen storage order of the output is returned.
// Matrix-core form (kind = NODE_MFMA, FP32 plans, at least four legs of a
// only (M) and four of b only (N)): 16 x 16 output tiles, rows from four M
// legs and columns from four N legs, K taken four values at a time; the
// tiles run over the other output legs (the modes).  With `free_order` the
// output is laid out as [the four tile N legs, M, batch, other N legs].
std::string make_node(const std::vector<int> &a, const std::vector<int> &b, const std::vector<int> &o,
                      NodeDesc &nd, std::vector<int32_t> &ktab, std::vector<int> *out_order,
                      bool free_order, bool mfma_ok) {
  std::map<int, int> pa, pb, po;
  for (size_t i = 0; i < a.size(); ++i) pa[a[i]] = (int)i;
  for (size_t i = 0; i < b.size(); ++i) pb[b[i]] = (int)i;
  std::vector<int> u, k, as(a), bs(b);
  std::sort(as.begin(), as.end());
  std::sort(bs.begin(), bs.end());
  std::set_union(as.begin(), as.end(), bs.begin(), bs.end(), std::back_inserter(u));
  std::set_difference(u.begin(), u.end(), o.begin(), o.end(), std::back_inserter(k));
  if ((int)k.size() > PWS_MAX_KBITS) return "contracted legs exceed kernel limit";
  nd.out_bits = (int)o.size();
  nd.k_bits = (int)k.size();
  std::vector<int> M, Bt, N;
  for (int l : o) {
    if (!pa.count(l)) N.push_back(l);
    else if (pb.count(l)) Bt.push_back(l);
    else M.push_back(l);
  }
  const bool mfma = mfma_ok && M.size() >= 4 && N.size() >= 4;
  const bool blocked = !mfma && (int)N.size() <= PWS_BLOCK_NBITS && (int)k.size() <= PWS_BLOCK_KBITS;
  nd.kind = mfma ? NODE_MFMA : blocked ? NODE_BLOCKED : NODE_GENERIC;
  // matrix-core tiles: the four M legs nearest the start of a (rows) and the
  // four N legs nearest the start of b (columns)
  std::vector<int> tm, tn, Mr, Nr;
  if (mfma) {
    std::vector<int> ms(M), ns(N);
    std::sort(ms.begin(), ms.end(), [&](int x, int y) { return pa[x] < pa[y]; });
    std::sort(ns.begin(), ns.end(), [&](int x, int y) { return pb[x] < pb[y]; });
    tm.assign(ms.begin(), ms.begin() + 4);
    tn.assign(ns.begin(), ns.begin() + 4);
    Mr.assign(ms.begin() + 4, ms.end());
    Nr.assign(ns.begin() + 4, ns.end());
  }
  std::vector<int> order;
  if (mfma && free_order) {
    order = tn;
    order.insert(order.end(), M.begin(), M.end());
    order.insert(order.end(), Bt.begin(), Bt.end());
    order.insert(order.end(), Nr.begin(), Nr.end());
  } else if (blocked && free_order) {
    order = M;
    order.insert(order.end(), Bt.begin(), Bt.end());
    order.insert(order.end(), N.begin(), N.end());
  } else {
    order = o;
  }
  for (size_t i = 0; i < order.size(); ++i) po[order[i]] = (int)i;
  std::vector<int> lane_legs;
  if (mfma) {
    lane_legs = Mr;   // the tiles' legs
    lane_legs.insert(lane_legs.end(), Bt.begin(), Bt.end());
    lane_legs.insert(lane_legs.end(), Nr.begin(), Nr.end());
  } else if (blocked) {
    for (int l : order)
      if (pa.count(l)) lane_legs.push_back(l);
  } else {
    lane_legs = order;
  }
  nd.p_bits = (int)lane_legs.size();
  nd.n_bits = blocked ? (int)N.size() : 0;
  nd.nmodes = 0;
  int cur_w = 0;
  int64_t bA = 0, bB = 0, bO = 0;
  for (size_t i = 0; i < lane_legs.size(); ++i) {
    const int l = lane_legs[i];
    const int64_t sA = pa.count(l) ? (1ll << pa[l]) : 0;
    const int64_t sB = pb.count(l) ? (1ll << pb[l]) : 0;
    const int64_t sO = 1ll << po[l];
    const bool extend = nd.nmodes > 0 && sA == (bA << cur_w) && sB == (bB << cur_w) && sO == (bO << cur_w);
    if (extend) {
      cur_w++;
      nd.mode_width[nd.nmodes - 1] = cur_w;
    } else {
      if (nd.nmodes == PWS_MAX_MODES) return "too many index modes";
      bA = sA; bB = sB; bO = sO;
      cur_w = 1;
      nd.mode_width[nd.nmodes] = 1;
      nd.strideA[nd.nmodes] = (int32_t)sA;
      nd.strideB[nd.nmodes] = (int32_t)sB;
      nd.strideO[nd.nmodes] = (int32_t)sO;
      nd.nmodes++;
    }
  }
  nd.ktab_off = (int32_t)ktab.size();
  for (int kv = 0; kv < (1 << k.size()); ++kv) {
    int32_t oa = 0, ob = 0;
    for (size_t j = 0; j < k.size(); ++j)
      if ((kv >> j) & 1) {
        if (pa.count(k[j])) oa += 1 << pa[k[j]];
        if (pb.count(k[j])) ob += 1 << pb[k[j]];
      }
    ktab.push_back(oa);
    ktab.push_back(ob);
  }
  nd.ntab_off = (int32_t)ktab.size();
  if (mfma) {
    // tile offsets: rows in a and the output, then columns in b and the output
    for (int part = 0; part < 4; ++part)
      for (int v = 0; v < 16; ++v) {
        int32_t off = 0;
        for (int j = 0; j < 4; ++j) {
          if (!((v >> j) & 1)) continue;
          if (part == 0) off += 1 << pa[tm[j]];
          if (part == 1) off += 1 << po[tm[j]];
          if (part == 2) off += 1 << pb[tn[j]];
          if (part == 3) off += 1 << po[tn[j]];
        }
        ktab.push_back(off);
      }
  }
  if (blocked) {
    for (int nv = 0; nv < (1 << N.size()); ++nv) {
      int32_t ob = 0, oo = 0;
      for (size_t j = 0; j < N.size(); ++j)
        if ((nv >> j) & 1) {
          ob += 1 << pb[N[j]];
          oo += 1 << po[N[j]];
        }
      ktab.push_back(ob);
      ktab.push_back(oo);
    }
  }
  if (out_order) *out_order = order;
  return "";
}

// Peak arena size (elements) of a tree under the emission allocator: leaves
// first, then per node the output is allocated before its inputs are freed.
int arena_peak(const std::vector<std::vector<int>> &legs, const std::vector<int> &open,
               const std::vector<Pair> &pairs) {
  Arena arena;
  std::vector<std::vector<int>> T = legs;
  std::vector<int> off;
  for (auto &l : legs) off.push_back(arena.alloc(1 << l.size()));
  Holders h = make_holders(legs, open);
  for (const Pair &p : pairs) {
    std::vector<int> out = contract_legs(T[p.a], T[p.b], h);
    apply_contraction(T[p.a], T[p.b], out, h);
    off.push_back(arena.alloc(1 << out.size()));
    arena.release(off[p.a], 1 << T[p.a].size());
    arena.release(off[p.b], 1 << T[p.b].size());
    T.push_back(out);
  }
  return arena.peak;
}

}  // namespace

// Store a leaf for every value of its chain-dependent bits (projected qubits,
// slice bits, recorded frame bits of conjugated gates); noise factors stay
// per chain (residual factors).
void tabulate_leaf(const CircuitIR &ir, Programs &prog, LeafDesc &ld, bool in_place = false);

void retabulate(const CircuitIR &ir, Programs &prog) {
  for (LeafDesc &ld : prog.leaves)
    if (ld.tab_off >= 0) tabulate_leaf(ir, prog, ld, true);
  flatten_mtab(prog);
}

// An entry whose factors are single leaf-table elements (no internal legs)
// times noise records becomes PWS_MENTRY_FLAT: each factor's table offset,
// variant-bit codes and noise records written out, so the kernels read no
// leaf or factor descriptor.  Other entries keep their codes.
static void flatten_entry(Programs &prog, const StepDesc &sd, const int32_t *codes, MEntry &me) {
  std::vector<int32_t> rec;
  int nf = 0;
  for (int t = 0; t < PWS_MTERMS; ++t) {
    const int32_t code = codes[t];
    if (code < 0) {   // a structural zero
      me = MEntry{0.0, 0.0, -1, 0, -1, 0};
      return;
    }
    if (code & PWS_MCODE_ONE) continue;
    const LeafDesc &ld = prog.leaves[sd.leaf_begin + (code & 0xffff)];
    const int el = (code >> 16) & 15, im = (code >> 20) & 15;
    if (ld.tab_off < 0 || im != 0 || ld.nvar > 4 || ld.r_count > 2) return;
    int32_t r[8] = {ld.tab_off + el, ld.nfree | (ld.nvar << 8) | (ld.r_count << 16), 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < ld.nvar; ++k) {
      const int32_t vc = prog.lvar[ld.var_begin + k];
      if ((vc >> 24) == VAR_SLICE) return;
      r[2 + k] = vc;
    }
    for (int fi = 0; fi < ld.r_count; ++fi) {
      const FactorDesc &f = prog.factors[ld.r_begin + fi];
      if (f.kind != FAC_SEGFAC || f.id >= (1 << 16)) return;
      const int32_t s = f.src_out[0], pl = src_payload(s);
      if (src_type(s) == SRC_FREE) r[6 + fi] = f.id | (((el >> pl) & 1) << 28);
      else if (src_type(s) == SRC_CONST) r[6 + fi] = f.id | ((pl & 1) << 28);
      else if (src_type(s) == SRC_CHAIN && pl < (1 << 12)) r[6 + fi] = f.id | (2 << 28) | (pl << 16);
      else return;
    }
    rec.insert(rec.end(), r, r + 8);
    ++nf;
  }
  if (nf == 0) return;
  me = MEntry{1.0, 0.0, PWS_MENTRY_FLAT, (int32_t)(prog.mflat.size() / 8), -1, nf};
  prog.mflat.insert(prog.mflat.end(), rec.begin(), rec.end());
}

void flatten_mtab(Programs &prog) {
  const size_t n_entries = prog.mtab.size() / PWS_MTERMS;
  prog.ment.assign(n_entries, MEntry{1.0, 0.0, -1, 0, -1, 0});
  prog.mterm.clear();
  prog.mflat.clear();
  std::map<std::array<int32_t, 3>, int32_t> term_of;   // (leaf, element, internal mask) -> table offset
  for (const StepDesc &sd : prog.steps) {
    if (!sd.sweep || sd.m_count == 0) continue;
    const size_t e0 = (size_t)sd.m_begin / PWS_MTERMS;
    for (int i = 0; i < sd.m_count; ++i) {
      MEntry &me = prog.ment[e0 + i];
      const int32_t *codes = &prog.mtab[(size_t)sd.m_begin + (size_t)i * PWS_MTERMS];
      std::complex<double> val(1.0, 0.0);
      int32_t terms[2][2];
      int nterm = 0;
      bool general = false, zero = false;
      for (int t = 0; t < PWS_MTERMS && !general && !zero; ++t) {
        const int32_t code = codes[t];
        if (code < 0) { zero = true; break; }
        if (code & PWS_MCODE_ONE) continue;
        const int leaf = sd.leaf_begin + (code & 0xffff);
        const LeafDesc &ld = prog.leaves[leaf];
        const int el = (code >> 16) & 15, im = (code >> 20) & 15;
        if (ld.tab_off < 0 || ld.r_count > 0 || ld.nvar > 2) { general = true; break; }
        for (int k = 0; k < ld.nvar; ++k) {
          const int32_t vc = prog.lvar[ld.var_begin + k];
          if ((vc >> 24) != VAR_CHAIN || (vc & 0xffffff) >= 4096) general = true;
        }
        if (general) break;
        // the factor summed over its internal legs, for every variant
        auto factor = [&](int var) {
          std::complex<double> acc(0.0, 0.0);
          for (int sub = im;; sub = (sub - 1) & im) {
            const size_t at = 2 * ((size_t)ld.tab_off + ((size_t)var << ld.nfree) + (size_t)(el | sub));
            acc += std::complex<double>(prog.ltab[at], prog.ltab[at + 1]);
            if (sub == 0) break;
          }
          return acc;
        };
        if (ld.nvar == 0) {
          val *= factor(0);
          continue;
        }
        if (nterm == 2) { general = true; break; }
        const std::array<int32_t, 3> key{leaf, el, im};
        auto it = term_of.find(key);
        int32_t off;
        if (it != term_of.end()) {
          off = it->second;
        } else {
          off = (int32_t)(prog.mterm.size() / 2);
          for (int var = 0; var < (1 << ld.nvar); ++var) {
            const std::complex<double> f = factor(var);
            prog.mterm.push_back(f.real());
            prog.mterm.push_back(f.imag());
          }
          term_of[key] = off;
        }
        int32_t p = ld.nvar << 24;
        for (int k = 0; k < ld.nvar; ++k) p |= (prog.lvar[ld.var_begin + k] & 0xfff) << (12 * k);
        terms[nterm][0] = off;
        terms[nterm][1] = p;
        ++nterm;
      }
      if (general) {
        me = MEntry{1.0, 0.0, PWS_MENTRY_CODES, 0, -1, 0};
        flatten_entry(prog, sd, codes, me);
        continue;
      }
      if (zero) val = 0.0;
      me.re = val.real();
      me.im = val.imag();
      if (!zero && nterm > 0) { me.t0 = terms[0][0]; me.p0 = terms[0][1]; }
      if (!zero && nterm > 1) { me.t1 = terms[1][0]; me.p1 = terms[1][1]; }
    }
  }
}

void tabulate_leaf(const CircuitIR &ir, Programs &prog, LeafDesc &ld, bool in_place) {
  std::vector<int32_t> vb;
  int ngate = 0;
  auto add = [&](int32_t code) {
    if (std::find(vb.begin(), vb.end(), code) == vb.end()) vb.push_back(code);
  };
  for (int fi = 0; fi < ld.f_count; ++fi) {
    const FactorDesc &f = prog.factors[ld.f_begin + fi];
    if (f.kind == FAC_SEGFAC) continue;
    ++ngate;
    for (int j = 0; j < f.nq; ++j)
      for (int32_t s : {f.src_out[j], f.src_in[j]}) {
        if (src_type(s) == SRC_CHAIN) add((VAR_CHAIN << 24) | src_payload(s));
        if (src_type(s) == SRC_SLICE) add((VAR_SLICE << 24) | src_payload(s));
      }
    if (f.frame)
      for (int j = 0; j < f.nq; ++j) add((VAR_FRAME << 24) | (f.id << 2) | (f.nq - 1 - j));
  }
  size_t wpos = 0;
  if (in_place) {
    wpos = 2 * (size_t)ld.tab_off;   // same variant bits, same layout: overwrite the values
  } else {
    ld.r_begin = ld.f_begin + ngate;
    ld.r_count = ld.f_count - ngate;
    ld.tab_off = -1;
    ld.nvar = (int)vb.size();
    ld.var_begin = (int)prog.lvar.size();
    if ((int)vb.size() > PWS_LEAF_VAR_BITS) return;
    prog.lvar.insert(prog.lvar.end(), vb.begin(), vb.end());
    ld.tab_off = (int)(prog.ltab.size() / 2);
  }
  const int ne = 1 << ld.nfree;
  for (int v = 0; v < (1 << vb.size()); ++v) {
    auto vbit = [&](int32_t code) {
      const size_t k = std::find(vb.begin(), vb.end(), code) - vb.begin();
      return (v >> k) & 1;
    };
    for (int e = 0; e < ne; ++e) {
      cd val = 1.0;
      for (int fi = 0; fi < ngate; ++fi) {
        const FactorDesc &f = prog.factors[ld.f_begin + fi];
        auto bit = [&](int32_t s) -> int {
          const int t = src_type(s), pl = src_payload(s);
          if (t == SRC_FREE) return (e >> pl) & 1;
          if (t == SRC_CONST) return pl;
          if (t == SRC_CHAIN) return vbit((VAR_CHAIN << 24) | pl);
          return vbit((VAR_SLICE << 24) | pl);
        };
        int out = 0, in = 0, fr = 0;
        for (int j = 0; j < f.nq; ++j) {
          out = 2 * out + bit(f.src_out[j]);
          in = 2 * in + bit(f.src_in[j]);
          fr = 2 * fr + (f.frame ? vbit((VAR_FRAME << 24) | (f.id << 2) | (f.nq - 1 - j)) : 0);
        }
        out ^= fr;
        in ^= fr;
        const GateIR &G = ir.gates[f.id];
        val *= (f.kind == FAC_GATE_DERIV ? G.dmat : G.mat)[out * (1 << f.nq) + in];
      }
      if (in_place) {
        prog.ltab[wpos++] = val.real();
        prog.ltab[wpos++] = val.imag();
      } else {
        prog.ltab.push_back(val.real());
        prog.ltab.push_back(val.imag());
      }
    }
  }
}

// One leaf of a step: factors with their free legs renumbered to bit
// positions of the leaf's element index (legs in ascending order), sliced
// legs turned into slice bits, the table of its chain variants, and its
// (leaf, element) pairs.
static void emit_leaf(const CircuitIR &ir, const LeafBuild &lb, const std::vector<int> &legs_i,
                      const std::vector<int> &sliced, int out_off, int leaf_begin, Programs &prog) {
  LeafDesc ld{};
  ld.nfree = (int)legs_i.size();
  ld.out_off = out_off;
  ld.f_begin = (int)prog.factors.size();
  ld.f_count = (int)lb.factors.size();
  std::vector<FactorDesc> fs = lb.factors;
  std::stable_partition(fs.begin(), fs.end(), [](const FactorDesc &f) { return f.kind != FAC_SEGFAC; });
  for (FactorDesc f : fs) {
    auto conv = [&](int32_t s) -> int32_t {
      if (src_type(s) != SRC_FREE) return s;
      const int leg = src_payload(s);
      auto it = std::find(sliced.begin(), sliced.end(), leg);
      if (it != sliced.end()) return src_make(SRC_SLICE, (int)(it - sliced.begin()));
      auto jt = std::lower_bound(legs_i.begin(), legs_i.end(), leg);
      return src_make(SRC_FREE, (int)(jt - legs_i.begin()));
    };
    for (int j = 0; j < 2; ++j) { f.src_out[j] = conv(f.src_out[j]); f.src_in[j] = conv(f.src_in[j]); }
    prog.factors.push_back(f);
  }
  tabulate_leaf(ir, prog, ld);
  for (int e = 0; e < (1 << ld.nfree); ++e) {
    prog.lelem.push_back((int32_t)prog.leaves.size() - leaf_begin);   // step-local leaf index
    prog.lelem.push_back(e);
  }
  prog.leaves.push_back(ld);
}

std::string emit_step(const CircuitIR &ir, StepNet &net, const std::vector<Pair> &pairs_in,
                      const PlanOptions &opt, int op_begin, Programs &prog, bool with_backward) {
  const int L = (int)net.leaves.size();
  std::vector<std::vector<int>> legs(L);
  for (int i = 0; i < L; ++i) legs[i] = net.leaves[i].legs;
  const std::vector<Pair> &pairs = pairs_in;
  // matrix-core nodes in FP32 / BF16x3 plans whose arenas live in device memory
  const bool mfma_ok = opt.precision != 0 && !opt.lds_mode;
  TreeCost unsliced = eval_tree(legs, net.open_legs, pairs);
  // ---- slicing: the caller's legs first (those this network contracts),
  // then legs fixed until one chain's working set fits
  std::vector<int> sliced;
  if (!with_backward) {
    for (int fl : opt.forced_slices) {
      if (std::find(net.open_legs.begin(), net.open_legs.end(), fl) != net.open_legs.end()) continue;
      bool present = false;
      for (const auto &v : legs) present |= std::find(v.begin(), v.end(), fl) != v.end();
      if (!present || std::find(sliced.begin(), sliced.end(), fl) != sliced.end()) continue;
      if (sliced.size() >= 20) return "too many sliced legs";
      sliced.push_back(fl);
      for (auto &v : legs) v.erase(std::remove(v.begin(), v.end(), fl), v.end());
    }
  }
  if (!with_backward && !opt.forbid_slicing) {
    while (true) {
      if (arena_peak(legs, net.open_legs, pairs) <= (int64_t)opt.arena_limit_elems) break;
      // score legs by the total size of the tensors that hold them
      Holders h = make_holders(legs, net.open_legs);
      std::vector<std::vector<int>> T = legs;
      std::map<int, double> score;
      for (const Pair &p : pairs) {
        std::vector<int> out = contract_legs(T[p.a], T[p.b], h);
        apply_contraction(T[p.a], T[p.b], out, h);
        for (int l : out) score[l] += p2(out.size());
        T.push_back(out);
      }
      int bl = -1;
      double bs = -1;
      for (auto &kv : score) {
        if (std::find(net.open_legs.begin(), net.open_legs.end(), kv.first) != net.open_legs.end()) continue;
        if (kv.second > bs) { bs = kv.second; bl = kv.first; }
      }
      if (bl < 0 || sliced.size() >= 20) return "cannot slice network to the memory budget";
      sliced.push_back(bl);
      for (auto &v : legs) v.erase(std::remove(v.begin(), v.end(), bl), v.end());
    }
  }
  TreeCost sc = eval_tree(legs, net.open_legs, pairs);
  // ---- all tensor leg lists (with slicing applied)
  std::vector<std::vector<int>> T = legs;
  {
    Holders h = make_holders(legs, net.open_legs);
    for (const Pair &p : pairs) {
      std::vector<int> out = contract_legs(T[p.a], T[p.b], h);
      apply_contraction(T[p.a], T[p.b], out, h);
      T.push_back(out);
    }
  }
  const int root = (int)T.size() - 1;
  {
    std::vector<int> ol = net.open_legs;
    std::sort(ol.begin(), ol.end());
    if (T[root] != ol) return "root legs differ from the open legs";
  }
  StepDesc sd{};
  sd.op = net.op;
  sd.gate = net.gate;
  sd.op_begin = op_begin;
  sd.leaf_begin = (int)prog.leaves.size();
  sd.n_leaves = L;
  sd.node_begin = (int)prog.nodes.size();
  sd.n_nodes = (int)pairs.size();
  sd.nS = (int)net.open_legs.size();
  sd.n_slice_bits = (int)sliced.size();
  sd.zero_q_begin = (int)prog.zero_q.size();
  sd.zero_q_count = (int)net.zero_q.size();
  for (int q : net.zero_q) prog.zero_q.push_back(q);
  sd.scal_begin = (int)prog.factors.size();
  sd.scal_count = (int)net.scalars.size();
  for (const FactorDesc &f : net.scalars) prog.factors.push_back(f);   // sources are CONST / CHAIN only
  Arena arena;
  SlotPool slots;
  std::vector<int> off(T.size(), -1), slot(T.size(), -1);
  std::vector<std::vector<int>> ord(T.size());   // storage order of every tensor
  for (int i = 0; i < L; ++i) ord[i] = legs[i];
  std::vector<int> drift(T.size(), 0);             // leaves since the last renormalisation
  for (int i = 0; i < L; ++i) drift[i] = 1;
  // leaves
  sd.elem_begin = (int)prog.lelem.size() / 2;
  for (int i = 0; i < L; ++i) {
    off[i] = arena.alloc(1 << (int)legs[i].size());
    emit_leaf(ir, net.leaves[i], legs[i], sliced, off[i], sd.leaf_begin, prog);
  }
  sd.n_elems = (int)prog.lelem.size() / 2 - sd.elem_begin;
  // nodes
  for (size_t pi = 0; pi < pairs.size(); ++pi) {
    const Pair &p = pairs[pi];
    const int id = L + (int)pi;
    NodeDesc nd{};
    const bool sw = T[p.b].size() > T[p.a].size();   // lanes run over the larger operand
    const int ia = sw ? p.b : p.a, ib = sw ? p.a : p.b;
    std::string err = make_node(ord[ia], ord[ib], T[id], nd, prog.ktab, &ord[id], !with_backward, mfma_ok);
    if (!err.empty()) return err;
    nd.a_off = off[ia];
    nd.b_off = off[ib];
    nd.exp_a = slot[ia];
    nd.exp_b = slot[ib];
    // exact power-of-two renormalisation: on large tensors, at the root, and
    // after every 16 leaves absorbed since the last renormalised subtree
    drift[id] = drift[p.a] + drift[p.b];
    nd.renorm = (T[id].size() >= 8 || drift[id] >= 16 || (int)pi + 1 == (int)pairs.size()) ? 1 : 0;
    if (nd.renorm || with_backward) drift[id] = 0;
    if (with_backward) nd.renorm = 1;
    off[id] = arena.alloc(1 << T[id].size());
    slot[id] = slots.alloc();
    nd.out_off = off[id];
    nd.exp_out = slot[id];
    if (!with_backward) {
      arena.release(off[p.a], 1 << T[p.a].size());
      arena.release(off[p.b], 1 << T[p.b].size());
      slots.release(slot[p.a]);
      slots.release(slot[p.b]);
    }
    prog.nodes.push_back(nd);
  }
  sd.root_off = off[root];
  sd.root_exp = slot[root];
  for (int v = 0; v < (1 << sd.nS); ++v) {
    int idx = 0;
    for (int k = 0; k < sd.nS; ++k) {
      const int bit = (v >> (sd.nS - 1 - k)) & 1;
      const int pos = (int)(std::find(ord[root].begin(), ord[root].end(), net.open_legs[k]) - ord[root].begin());
      idx |= bit << pos;
    }
    sd.root_index[v] = idx;
  }
  // ---- backward program (adjoint contraction for gradients)
  if (with_backward) {
    prog.bnodes.clear();
    prog.grad_terms.clear();
    prog.leaf_adj_off.assign(L, -1);
    prog.leaf_adj_exp.assign(L, -1);
    std::vector<int> aoff(T.size(), -1), aslot(T.size(), -1);
    // adjoint of the root (a scalar 1 written by the kernel)
    aoff[root] = arena.alloc(1 << T[root].size());
    aslot[root] = -1;
    prog.adj_root_off = aoff[root];
    for (int pi = (int)pairs.size() - 1; pi >= 0; --pi) {
      const Pair &p = pairs[pi];
      const int id = L + pi;
      for (int side = 0; side < 2; ++side) {
        const int tgt = side == 0 ? p.a : p.b;
        const int oth = side == 0 ? p.b : p.a;
        NodeDesc nd{};
        nd.renorm = 1;
        const bool sw = T[oth].size() > T[id].size();
        // adjoints are stored in sorted order (the leaf gradient terms read them so)
        std::string err = sw ? make_node(ord[oth], T[id], T[tgt], nd, prog.ktab, nullptr, false, mfma_ok)
                             : make_node(T[id], ord[oth], T[tgt], nd, prog.ktab, nullptr, false, mfma_ok);
        if (!err.empty()) return err;
        nd.a_off = sw ? off[oth] : aoff[id];
        nd.exp_a = sw ? slot[oth] : aslot[id];
        nd.b_off = sw ? aoff[id] : off[oth];
        nd.exp_b = sw ? aslot[id] : slot[oth];
        aoff[tgt] = arena.alloc(1 << T[tgt].size());
        aslot[tgt] = slots.alloc();
        nd.out_off = aoff[tgt];
        nd.exp_out = aslot[tgt];
        prog.bnodes.push_back(nd);
      }
    }
    for (int i = 0; i < L; ++i) {
      prog.leaf_adj_off[i] = aoff[i];
      prog.leaf_adj_exp[i] = aslot[i];
      const auto &fs = net.leaves[i].factors;
      for (size_t fi = 0; fi < fs.size(); ++fi) {
        if (fs[fi].kind != FAC_GATE) continue;
        const GateIR &G = ir.gates[fs[fi].id];
        if (G.param < 0) continue;
        bool has = false;
        for (int e = 0; e < 16; ++e) has = has || G.dmat[e] != cd(0);
        if (!has) continue;
        prog.grad_terms.push_back(i);
        prog.grad_terms.push_back((int)fi);
        prog.grad_terms.push_back(G.param);
        prog.grad_terms.push_back(aoff[i]);
        prog.grad_terms.push_back(aslot[i]);
      }
    }
  }
  sd.arena_elems = arena.peak;
  sd.n_exp_slots = std::max(slots.top, 1);
  prog.max_arena = std::max(prog.max_arena, sd.arena_elems);
  prog.max_exp = std::max(prog.max_exp, sd.n_exp_slots);
  prog.max_slice_bits = std::max(prog.max_slice_bits, sd.n_slice_bits);
  prog.flops_per_sample += unsliced.flops;
  prog.bytes_per_sample += unsliced.bytes;
  prog.flops_executed += sc.flops * std::ldexp(1.0, (int)sliced.size());
  prog.log2_width = std::max(prog.log2_width, unsliced.max_bits);
  prog.n_slices_total += 1ll << sliced.size();
  prog.steps.push_back(sd);
  return "";
}


// ------------------------------------------------------------------ sweep form

namespace {

struct SweepOrder {
  std::vector<int> order;   // leaf absorption order
  int width = 1 << 30;      // peak positions of the running tensor
  double cost = 0;          // elements touched, summed over the ops
  std::vector<double> step_cost;   // elements touched by each op
};

// Greedy absorption order: among the leaves sharing a leg with the running
// tensor, absorb the one that leaves it narrowest (ties: smallest key, i.e.
// earliest along the qubit order); with no such leaf, start at the smallest
// key.  A leg stays live while some unabsorbed leaf holds it or it is open.
SweepOrder sweep_order(const std::vector<std::vector<int>> &legs, const std::vector<char> &is_open,
                       const std::vector<int64_t> &key, int n_legs, const std::vector<int> &prefix) {
  const int L = (int)legs.size();
  std::vector<int> remaining(n_legs, 0);
  std::vector<std::vector<int>> holders(n_legs);
  for (int i = 0; i < L; ++i)
    for (int l : legs[i]) { ++remaining[l]; holders[l].push_back(i); }
  std::vector<char> live(n_legs, 0), done(L, 0), in_cand(L, 0);
  std::vector<int> cand, by_key(L);
  std::iota(by_key.begin(), by_key.end(), 0);
  std::stable_sort(by_key.begin(), by_key.end(), [&](int a, int b) { return key[a] < key[b]; });
  size_t next = 0;
  int width = 0;
  SweepOrder so;
  so.width = 0;
  for (int step = 0; step < L; ++step) {
    int best = -1, best_after = 1 << 30;
    int64_t best_key = 0;
    size_t w = 0;
    if (step < (int)prefix.size()) best = prefix[step];   // leaves taken over from the previous step
    for (size_t ci = 0; ci < cand.size() && step >= (int)prefix.size(); ++ci) {
      const int i = cand[ci];
      if (done[i]) { in_cand[i] = 0; continue; }
      cand[w++] = i;
      int after = width;
      for (int l : legs[i]) {
        if (live[l]) { if (remaining[l] == 1 && !is_open[l]) --after; }
        else if (remaining[l] > 1 || is_open[l]) ++after;
      }
      if (best < 0 || after < best_after || (after == best_after && key[i] < best_key)) {
        best = i; best_after = after; best_key = key[i];
      }
    }
    if (step >= (int)prefix.size()) cand.resize(w);
    if (best < 0) {
      while (done[by_key[next]]) ++next;
      best = by_key[next];
    }
    const int before = width;
    for (int l : legs[best]) {
      --remaining[l];
      if (live[l]) {
        if (remaining[l] == 0 && !is_open[l]) { live[l] = 0; --width; }
      } else if (remaining[l] > 0 || is_open[l]) {
        live[l] = 1;
        ++width;
        for (int h : holders[l])
          if (!done[h] && !in_cand[h] && h != best) { in_cand[h] = 1; cand.push_back(h); }
      }
    }
    done[best] = 1;
    so.order.push_back(best);
    so.width = std::max(so.width, std::max(before, width));
    so.cost += std::ldexp(1.0, std::max(before, width));
    so.step_cost.push_back(std::ldexp(1.0, std::max(before, width)));
  }
  return so;
}

}  // namespace

// Content key of a leaf: its factors with their sources (free legs by leg id).
static std::string leaf_signature(const LeafBuild &lb) {
  std::vector<std::string> fs;
  for (const FactorDesc &f : lb.factors) {
    char buf[160];
    snprintf(buf, sizeof buf, "%d,%d,%d,%d,%d,%d,%d,%d;", f.kind, f.id, f.nq, f.frame, f.src_out[0], f.src_out[1],
             f.src_in[0], f.src_in[1]);
    fs.push_back(buf);
  }
  std::sort(fs.begin(), fs.end());
  std::string k;
  for (auto &x : fs) k += x;
  return k;
}

PrefixMatch match_prefix(const SweepPlan &src, const SweepPlan &cur, const std::vector<char> &usable,
                         const std::vector<char> &dirty_q, const std::vector<char> &dirty_seg,
                         const std::vector<char> &forbid_leg) {
  PrefixMatch pm;
  pm.valid.push_back(1);
  const StepNet &net = cur.net;
  const int L = (int)net.leaves.size();
  const int n_legs = (int)cur.is_open.size();
  std::multimap<std::string, int> by_sig;
  for (int i = 0; i < L; ++i)
    if (usable[i]) by_sig.emplace(cur.sig[i], i);
  auto clean = [&](int i) {
    for (const FactorDesc &f : net.leaves[i].factors) {
      if (f.kind == FAC_SEGFAC && f.id < (int)dirty_seg.size() && dirty_seg[f.id]) return false;
      for (int j = 0; j < f.nq; ++j)
        for (int32_t s : {f.src_out[j], f.src_in[j]})
          if (src_type(s) == SRC_CHAIN && dirty_q[src_payload(s)]) return false;
    }
    for (int l : cur.legs[i])
      if (forbid_leg[l]) return false;
    return true;
  };
  // a leg is live after a prefix when some but not all of its holders (in the
  // step's swept leaves) are absorbed, or it is open and touched
  std::vector<int> hold_p(n_legs, 0), hold_c(n_legs, 0), cnt(n_legs, 0);
  for (int i : src.order)
    for (int l : src.legs[i]) ++hold_p[l];
  for (int i = 0; i < L; ++i)
    if (usable[i])
      for (int l : cur.legs[i]) ++hold_c[l];
  auto live = [&](int l, const std::vector<int> &hold, const std::vector<char> &open) {
    return cnt[l] > 0 && (cnt[l] < hold[l] || open[l]);
  };
  int diff = 0;
  for (size_t k = 0; k < src.order.size(); ++k) {
    const int ip = src.order[k];
    auto range = by_sig.equal_range(src.sig[ip]);
    if (range.first == range.second) break;
    const int i = range.first->second;
    by_sig.erase(range.first);
    if (!clean(i)) break;
    pm.mapped.push_back(i);
    for (int l : cur.legs[i]) {
      const bool bp = live(l, hold_p, src.is_open), bc = live(l, hold_c, cur.is_open);
      diff -= bp != bc;
      ++cnt[l];
      const bool ap = live(l, hold_p, src.is_open), ac = live(l, hold_c, cur.is_open);
      diff += ap != ac;
    }
    pm.valid.push_back(diff == 0 ? 1 : 0);
  }
  return pm;
}

std::string sweep_setup(const CircuitIR &ir, const StepNet &net_in, int op_begin, SweepPlan &sp) {
  sp = SweepPlan();
  sp.net = net_in;
  sp.op_begin = op_begin;
  const StepNet &net = sp.net;
  const int L = (int)net.leaves.size();
  if (L == 0) return "empty network";
  if (L > 32767) return "too many leaves for a sweep";
  sp.legs.resize(L);
  for (int i = 0; i < L; ++i) {
    sp.legs[i] = net.leaves[i].legs;
    if ((int)sp.legs[i].size() > PWS_SWEEP_MAXNP) return "leaf with more legs than a sweep op takes";
  }
  sp.is_open.assign(ir.n_segs, 0);
  for (int l : net.open_legs) sp.is_open[l] = 1;
  sp.sig.resize(L);
  for (int i = 0; i < L; ++i) sp.sig[i] = leaf_signature(net.leaves[i]);
  return "";
}

namespace {

// Orders of the swept leaves by each qubit order (and its reverse), with the
// given leaves first.
std::vector<SweepOrder> candidate_orders(const CircuitIR &ir, const SweepPlan &sp, const std::vector<int> &prefix,
                                         bool both_directions) {
  const int L = (int)sp.legs.size();
  std::vector<int> idx;   // swept leaves
  std::vector<int> sub_of(L, -1);
  for (int i = 0; i < L; ++i)
    if (sp.swept.empty() || sp.swept[i]) { sub_of[i] = (int)idx.size(); idx.push_back(i); }
  std::vector<std::vector<int>> legs;
  for (int i : idx) legs.push_back(sp.legs[i]);
  std::vector<int> pre;
  for (int i : prefix) pre.push_back(sub_of[i]);
  std::vector<std::vector<int>> qorders = ir.qorders;
  {
    std::vector<int> id(ir.n);
    std::iota(id.begin(), id.end(), 0);
    qorders.push_back(id);
  }
  std::vector<SweepOrder> out;
  for (const auto &qo : qorders)
    for (int dir = 0; dir < (both_directions ? 2 : 1); ++dir) {
      std::vector<int> rank(ir.n, 0);
      for (int k = 0; k < (int)qo.size(); ++k) rank[qo[k]] = dir ? (int)qo.size() - 1 - k : k;
      std::vector<int64_t> key(legs.size(), 0);
      for (size_t i = 0; i < legs.size(); ++i) {
        int mx = -1, mn = ir.n;
        for (int l : legs[i]) {
          const int r = rank[ir.seg_qubit[l]];
          mx = std::max(mx, r);
          mn = std::min(mn, r);
        }
        key[i] = legs[i].empty() ? -1 : (int64_t)mx * (ir.n + 1) + mn;
      }
      SweepOrder so = sweep_order(legs, sp.is_open, key, ir.n_segs, pre);
      for (int &o : so.order) o = idx[o];
      out.push_back(so);
    }
  return out;
}

}  // namespace

std::string plan_sweep(const CircuitIR &ir, const StepNet &net_in, const PlanOptions &opt, int op_begin,
                       const SweepPlan *prev, const std::vector<char> &dirty_q, const std::vector<char> &dirty_seg,
                       SweepPlan &sp, const std::vector<char> *swept, const std::vector<int> *bound) {
  std::string err = sweep_setup(ir, net_in, op_begin, sp);
  if (!err.empty()) return err;
  const int L = (int)sp.legs.size();
  if (swept) sp.swept = *swept;
  if (bound) {
    sp.bound = *bound;
    for (int l : sp.bound) sp.is_open[l] = 1;
  }
  // ---- prefix restored from the previous step: its leading leaves that this
  // step holds unchanged (same factors, none reading a chain bit or noise
  // record changed since), up to the longest point where both steps leave the
  // same legs live (then the running tensors there are equal)
  std::vector<int> prefix;
  if (prev && opt.sweep_cache) {
    std::vector<char> usable(L, 1), forbid(ir.n_segs, 0);
    if (!sp.swept.empty()) usable = sp.swept;
    PrefixMatch pm = match_prefix(*prev, sp, usable, dirty_q, dirty_seg, forbid);
    int best_j = 0;
    for (size_t j = 0; j < pm.valid.size(); ++j)
      if (pm.valid[j]) best_j = (int)j;
    // the previous step keeps its tensor after these leaves; it may itself have
    // restored a longer prefix, and never materialises the tensor before that
    if (best_j < prev->load_n) best_j = 0;
    if (best_j >= opt.sweep_cache_min) prefix.assign(pm.mapped.begin(), pm.mapped.begin() + best_j);
  }
  sp.load_n = (int)prefix.size();
  SweepOrder best;
  for (SweepOrder &so : candidate_orders(ir, sp, prefix, false))
    if (so.width < best.width || (so.width == best.width && so.cost < best.cost)) best = so;
  sp.order = best.order;
  sp.W = std::max(best.width, 0);
  sp.run_cost = 0;
  for (size_t k = (size_t)sp.load_n; k < best.step_cost.size(); ++k) sp.run_cost += best.step_cost[k];
  if (sp.W > opt.sweep_max_width || sp.W > PWS_SWEEP_MAXW) return "sweep wider than the on-chip tensor";
  if (lds_bytes_sweep(opt.precision, sp.W, 0) > opt.sweep_lds_bytes) return "sweep tensor exceeds the LDS";
  return "";
}

std::string plan_anchor(const CircuitIR &ir, const StepNet &net_in, const PlanOptions &opt, int op_begin,
                        const std::vector<int> &leaf_dirty, int this_step, SweepPlan &sp, double *benefit) {
  std::string err = sweep_setup(ir, net_in, op_begin, sp);
  if (!err.empty()) return err;
  *benefit = 0;
  SweepOrder best;
  double best_b = -1;
  std::vector<int> best_pts;
  for (SweepOrder &so : candidate_orders(ir, sp, {}, true)) {
    if (so.width > opt.sweep_max_width || so.width > PWS_SWEEP_MAXW) continue;
    // the first k leaves serve every later step before the first of them
    // turns dirty: snapshot points where that step moves earlier
    const int n = (int)so.order.size();
    std::vector<int> pm(n + 1, INT_MAX);
    std::vector<double> pc(n + 1, 0.0);   // elements touched by the first k ops
    for (int k = 0; k < n; ++k) {
      pm[k + 1] = std::min(pm[k], leaf_dirty[so.order[k]]);
      pc[k + 1] = pc[k] + so.step_cost[k];
    }
    std::vector<int> pts;
    double b = 0;
    for (int k = opt.sweep_merge_min; k < n; ++k) {
      const bool last = pm[k + 1] < pm[k];
      if (!last || pm[k] <= this_step + 1) continue;
      // steps max(this_step+1, pm[k+1]) .. min(pm[k], horizon) - 1 can use it
      const int until = std::min(pm[k], this_step + 1 + opt.sweep_anchor_horizon);
      const int from = std::max(this_step + 1, pm[k + 1]);
      if (until > from) {
        pts.push_back(k);
        b += pc[k] * (until - from);
      }
    }
    if ((int)pts.size() > opt.sweep_snap_max) {   // evenly spread, the widest kept
      std::vector<int> keep;
      const double stride = (double)pts.size() / opt.sweep_snap_max;
      for (int s = 0; s < opt.sweep_snap_max; ++s)
        keep.push_back(pts[(size_t)std::min<double>(pts.size() - 1, std::floor((s + 1) * stride) - 1)]);
      pts = keep;
    }
    if (b > best_b || (b == best_b && (so.width < best.width || (so.width == best.width && so.cost < best.cost)))) {
      best_b = b;
      best = so;
      best_pts = pts;
    }
  }
  if (best_b < 0) return "no anchor order fits the on-chip tensor";
  sp.order = best.order;
  sp.W = std::max(best.width, 0);
  sp.run_cost = best.cost;
  if (lds_bytes_sweep(opt.precision, sp.W, 0) > opt.sweep_lds_bytes) return "sweep tensor exceeds the LDS";
  *benefit = best_b;
  sp.anchor = std::make_shared<AnchorState>();
  for (size_t s = 0; s < best_pts.size(); ++s) {
    AnchorState::Snap sn;
    sn.j = best_pts[s];
    sn.slot = (int)s + 1;
    sp.anchor->snaps.push_back(sn);
  }
  return "";
}

std::string emit_sweep(const CircuitIR &ir, StepNet &net, const PlanOptions &opt, int op_begin,
                       Programs &prog) {
  SweepPlan sp;
  std::vector<char> none_q(ir.n, 0), none_s(ir.n_segs, 0);
  std::string err = plan_sweep(ir, net, opt, op_begin, nullptr, none_q, none_s, sp, nullptr, nullptr);
  if (!err.empty()) return err;
  return emit_sweep_plan(ir, sp, opt, prog);
}

std::string emit_sweep_plan(const CircuitIR &ir, SweepPlan &sp, const PlanOptions &opt, Programs &prog) {
  const StepNet &net = sp.net;
  const int op_begin = sp.op_begin;
  const int L = (int)net.leaves.size();
  const int n_legs = ir.n_segs;
  const std::vector<std::vector<int>> &legs = sp.legs;
  const std::vector<char> &is_open = sp.is_open;
  struct {
    std::vector<int> order;
  } best;
  best.order = sp.order;
  const int W = sp.W;


  // undo the appends of this step if a later check fails
  const size_t n_zq = prog.zero_q.size(), n_fac = prog.factors.size(), n_le = prog.lelem.size(),
               n_lv = prog.leaves.size(), n_lt = prog.ltab.size(), n_var = prog.lvar.size(),
               n_sw = prog.sweeps.size(), n_mt = prog.mtab.size(), n_sn = prog.snaps.size(),
               n_mm = prog.mmap.size();
  const int n_slots0 = prog.n_slots, max_snap_w0 = prog.max_snap_w;
  auto undo = [&](const char *why) {
    prog.snaps.resize(n_sn);
    prog.mmap.resize(n_mm);
    prog.n_slots = n_slots0;
    prog.max_snap_w = max_snap_w0;
    prog.zero_q.resize(n_zq);
    prog.factors.resize(n_fac);
    prog.lelem.resize(n_le);
    prog.leaves.resize(n_lv);
    prog.ltab.resize(n_lt);
    prog.lvar.resize(n_var);
    prog.sweeps.resize(n_sw);
    prog.mtab.resize(n_mt);
    return std::string(why);
  };
  StepDesc sd{};
  sd.op = net.op;
  sd.gate = net.gate;
  sd.op_begin = op_begin;
  sd.leaf_begin = (int)prog.leaves.size();
  sd.n_leaves = L;
  sd.node_begin = (int)prog.nodes.size();
  sd.n_nodes = 0;
  sd.nS = (int)net.open_legs.size();
  sd.n_slice_bits = 0;
  sd.zero_q_begin = (int)prog.zero_q.size();
  sd.zero_q_count = (int)net.zero_q.size();
  for (int q : net.zero_q) prog.zero_q.push_back(q);
  sd.scal_begin = (int)prog.factors.size();
  sd.scal_count = (int)net.scalars.size();
  for (const FactorDesc &f : net.scalars) prog.factors.push_back(f);
  sd.elem_begin = (int)prog.lelem.size() / 2;
  int area = 0;
  for (int i = 0; i < L; ++i) {
    emit_leaf(ir, net.leaves[i], legs[i], {}, area, sd.leaf_begin, prog);
    area += 1 << (int)legs[i].size();
  }
  sd.n_elems = (int)prog.lelem.size() / 2 - sd.elem_begin;
  sd.sweep = 1;
  const int m_begin = (int)prog.mtab.size();
  sd.m_begin = m_begin;
  sd.sw_begin = (int)prog.sweeps.size();
  sd.sw_width = W;
  sd.root_off = 0;
  sd.root_exp = -1;
  sd.arena_elems = 0;
  sd.n_exp_slots = 1;

  // ---- one op per absorbed leaf: positions, roles and the leaf's legs
  struct Term {
    int leaf = -1, nleg = 0;
    int code[PWS_SWEEP_MAXNP] = {0, 0, 0, 0};   // group bit | 8 output side | 16 internal
  };
  struct HOp {
    int np = 0, pos[PWS_SWEEP_MAXNP] = {0, 0, 0, 0}, role[PWS_SWEEP_MAXNP] = {0, 0, 0, 0};
    int outer_mask = 0, leaf = -1;
    bool dead = false;
    std::vector<Term> terms;
    int gbit(int pp) const {
      for (int j = 0; j < np; ++j)
        if (pos[j] == pp) return j;
      return -1;
    }
    bool diag() const {
      for (int j = 0; j < np; ++j)
        if (role[j] != SW_KEEP) return false;
      return true;
    }
  };
  std::vector<HOp> hops;
  std::vector<int> width_after(best.order.size() + 1, 0);   // highest live position + 1 after k leaves
  std::vector<int> final_pos;                                // position of each leg after the last op
  {
    std::vector<int> remaining(n_legs, 0), pos_of(n_legs, -1);
    for (int i : best.order)
      for (int l : legs[i]) ++remaining[l];
    std::vector<int> occupant(PWS_SWEEP_MAXW, -1);   // leg at each position
    std::vector<AnchorState::Snap> *snaps = sp.anchor ? &sp.anchor->snaps : nullptr;
    for (size_t oi = 0; oi < best.order.size(); ++oi) {
      const int i = best.order[oi];
      std::vector<int> sum_pos, keep_pos, new_legs;
      std::vector<int> leg_pos(legs[i].size(), -1);
      std::vector<char> internal(legs[i].size(), 0);
      for (size_t k = 0; k < legs[i].size(); ++k) {
        const int l = legs[i][k];
        if (pos_of[l] >= 0) {
          leg_pos[k] = pos_of[l];
          if (remaining[l] == 1 && !is_open[l]) sum_pos.push_back(pos_of[l]);
          else keep_pos.push_back(pos_of[l]);
        } else if (remaining[l] > 1 || is_open[l]) {
          new_legs.push_back((int)k);
        } else {
          internal[k] = 1;
        }
      }
      // created legs take the positions of contracted ones first, then the lowest free
      std::vector<int> replace_pos;
      std::vector<char> taken(W, 0);
      for (int pp : sum_pos) taken[pp] = 1;
      for (int pp : keep_pos) taken[pp] = 1;
      size_t reuse = 0;
      for (int k : new_legs) {
        int pp = -1;
        if (reuse < sum_pos.size()) {
          pp = sum_pos[reuse++];
          replace_pos.push_back(pp);
        } else {
          for (int q = 0; q < W; ++q)
            if (occupant[q] < 0 && !taken[q]) { pp = q; break; }
          if (pp < 0) return undo("sweep position allocation failed");
          taken[pp] = 1;
        }
        leg_pos[k] = pp;
      }
      HOp h;
      h.leaf = i;
      for (int q = 0; q < W; ++q)
        if (taken[q]) {
          if (h.np == PWS_SWEEP_MAXNP) return undo("sweep op with too many positions");
          h.pos[h.np++] = q;
        }
      for (int j = 0; j < h.np; ++j) {
        const int pp = h.pos[j];
        const bool is_sum = std::find(sum_pos.begin(), sum_pos.end(), pp) != sum_pos.end();
        const bool is_rep = std::find(replace_pos.begin(), replace_pos.end(), pp) != replace_pos.end();
        const bool is_keep = std::find(keep_pos.begin(), keep_pos.end(), pp) != keep_pos.end();
        h.role[j] = is_rep ? SW_REPLACE : is_sum ? SW_SUM : is_keep ? SW_KEEP : SW_NEW;
      }
      Term t;
      t.leaf = i;
      t.nleg = (int)legs[i].size();
      for (size_t k = 0; k < legs[i].size(); ++k) {
        if (internal[k]) { t.code[k] = 16; continue; }
        const bool created = pos_of[legs[i][k]] < 0;
        t.code[k] = h.gbit(leg_pos[k]) | (created ? 8 : 0);
      }
      h.terms.push_back(t);
      for (int q = 0; q < W; ++q)
        if (occupant[q] >= 0 && !taken[q]) h.outer_mask |= 1 << q;
      for (size_t k = 0; k < legs[i].size(); ++k) --remaining[legs[i][k]];
      for (int pp : sum_pos) { pos_of[occupant[pp]] = -1; occupant[pp] = -1; }
      for (int k : new_legs) { pos_of[legs[i][k]] = leg_pos[k]; occupant[leg_pos[k]] = legs[i][k]; }
      hops.push_back(h);
      int top = 0;
      for (int q = 0; q < W; ++q)
        if (occupant[q] >= 0) top = q + 1;
      width_after[oi + 1] = top;
      if (snaps)
        for (auto &sn : *snaps)
          if (sn.j == (int)oi + 1) {
            sn.leg_pos = pos_of;
            sn.w = top;
          }
    }
    for (int v = 0; v < (1 << sd.nS); ++v) {
      int idx = 0;
      for (int k = 0; k < sd.nS; ++k) {
        const int bit = (v >> (sd.nS - 1 - k)) & 1;
        const int pp = pos_of[net.open_legs[k]];
        if (pp < 0) return undo("open leg without a position");
        idx |= bit << pp;
      }
      sd.root_index[v] = idx;
    }
    for (int q = 0; q < W; ++q)
      if (occupant[q] >= 0 && !is_open[occupant[q]]) return undo("closed leg left in the sweep tensor");
    final_pos = pos_of;
  }
  // ---- fusion: a diagonal op (every leg kept) commutes with the ops that do
  // not touch its positions, so it is folded into the nearest op that does,
  // as one more factor of that op's matrix (on its output side when the op
  // comes first, its input side otherwise); positions it adds to that op are
  // kept legs.  An op stays within two positions and four factors.
  // ops on either side of a cache point stay apart (the restored and the
  // stored tensors are the ones after exactly load_n / store_n leaves)
  std::vector<int> cuts;
  if (sp.load_n > 0) cuts.push_back(sp.load_n);
  if (sp.store_n > 0) cuts.push_back(sp.store_n);
  if (sp.anchor)
    for (const auto &sn : sp.anchor->snaps) cuts.push_back(sn.j);
  std::sort(cuts.begin(), cuts.end());
  auto segment = [&](int h) { return (int)(std::upper_bound(cuts.begin(), cuts.end(), h) - cuts.begin()); };
  if (opt.sweep_fuse) {
    const int H = (int)hops.size();
    for (int i = 0; i < H; ++i) {
      HOp &d = hops[i];
      if (!d.diag() || d.np == 0 || d.terms.size() != 1) continue;
      auto touches = [&](const HOp &x) {
        for (int j = 0; j < d.np; ++j)
          if (x.gbit(d.pos[j]) >= 0) return true;
        return false;
      };
      int cand[2] = {-1, -1};
      for (int j = i - 1; j >= 0; --j)
        if (!hops[j].dead && touches(hops[j])) { cand[0] = j; break; }
      for (int j = i + 1; j < H; ++j)
        if (!hops[j].dead && touches(hops[j])) { cand[1] = j; break; }
      for (int side = 0; side < 2; ++side)
        if (cand[side] >= 0 && segment(cand[side]) != segment(i)) cand[side] = -1;
      for (int side = 0; side < 2 && !d.dead; ++side) {
        if (cand[side] < 0) continue;
        HOp &x = hops[cand[side]];
        if (x.terms.size() >= 4) continue;
        int extra = 0;
        for (int j = 0; j < d.np; ++j)
          if (x.gbit(d.pos[j]) < 0) ++extra;
        if (x.np + extra > 2) continue;
        for (int j = 0; j < d.np; ++j)
          if (x.gbit(d.pos[j]) < 0) {
            x.pos[x.np] = d.pos[j];
            x.role[x.np] = SW_KEEP;
            x.outer_mask &= ~(1 << d.pos[j]);
            ++x.np;
          }
        Term t = d.terms[0];
        for (int k = 0; k < t.nleg; ++k) {
          if (t.code[k] & 16) continue;
          const int pp = d.pos[t.code[k] & 7];
          t.code[k] = x.gbit(pp) | (side == 0 ? 8 : 0);   // after x: its output bits
        }
        x.terms.push_back(t);
        d.dead = true;
      }
    }
  }
  // ---- emit: group bits ordered so that a two-position op with one kept
  // leg has it at bit 1 (block-diagonal form), masks, matrix entry codes
  int since_renorm = 0;
  double macs = 0, elems = 0;
  int n_live_ops = 0;
  for (const HOp &h : hops) n_live_ops += !h.dead;
  int emitted = 0;
  sd.load_op = -1;
  sd.store_op = -1;
  for (size_t hi = 0; hi < hops.size(); ++hi) {
    if (sp.load_n > 0 && (int)hi == sp.load_n) sd.load_op = emitted;
    if (sp.store_n > 0 && (int)hi == sp.store_n) sd.store_op = emitted;
    if (sp.anchor)
      for (auto &sn : sp.anchor->snaps)
        if (sn.j == (int)hi) sn.op = emitted;
    HOp h = hops[hi];
    if (h.dead) continue;
    if (h.np == 2 && !h.diag() && h.role[0] == SW_KEEP && h.role[1] != SW_KEEP) {
      std::swap(h.pos[0], h.pos[1]);
      std::swap(h.role[0], h.role[1]);
      for (Term &t : h.terms)
        for (int k = 0; k < t.nleg; ++k)
          if (!(t.code[k] & 16)) t.code[k] = ((t.code[k] & 7) ^ 1) | (t.code[k] & 8);
    }
    SweepOp so{};
    so.leaf = (int16_t)h.leaf;
    so.np = (int8_t)h.np;
    const bool diag = h.diag();
    so.diag = diag ? 1 : (h.np == 2 && h.role[1] == SW_KEEP && h.role[0] != SW_KEEP) ? 2 : 0;
    for (int j = 0; j < h.np; ++j) {
      so.pos[j] = (int8_t)h.pos[j];
      so.role[j] = (int8_t)h.role[j];
    }
    so.nleg = (int8_t)h.terms[0].nleg;
    for (int k = 0; k < h.terms[0].nleg; ++k) so.leg[k] = (int8_t)h.terms[0].code[k];
    const int ng = 1 << so.np;
    so.in_mask = so.out_mask = 0;
    for (int g = 0; g < ng; ++g) {
      bool in_ok = true, out_ok = true;
      for (int j = 0; j < so.np; ++j) {
        if (so.role[j] == SW_NEW && ((g >> j) & 1)) in_ok = false;
        if (so.role[j] == SW_SUM && ((g >> j) & 1)) out_ok = false;
      }
      if (in_ok) so.in_mask = (int16_t)(so.in_mask | (1 << g));
      if (out_ok) so.out_mask = (int16_t)(so.out_mask | (1 << g));
    }
    // matrix entries (row o, column in): the product of the op's factors
    so.moff = (int32_t)((prog.mtab.size() - (size_t)m_begin) / PWS_MTERMS);
    int valid = 0;
    for (int o = 0; o < ng; ++o)
      for (int in = 0; in < ng; ++in) {
        if (diag && o != in) continue;
        bool ok = ((so.out_mask >> o) & 1) && ((so.in_mask >> in) & 1);
        for (int j = 0; j < so.np; ++j)
          if (so.role[j] == SW_KEEP && ((o >> j) & 1) != ((in >> j) & 1)) ok = false;
        valid += ok;
        for (int ti = 0; ti < PWS_MTERMS; ++ti) {
          if (!ok) { prog.mtab.push_back(ti == 0 ? PWS_MCODE_ZERO : PWS_MCODE_ONE); continue; }
          if (ti >= (int)h.terms.size()) { prog.mtab.push_back(PWS_MCODE_ONE); continue; }
          const Term &t = h.terms[ti];
          int e0 = 0, imask = 0;
          for (int k = 0; k < t.nleg; ++k) {
            const int code = t.code[k];
            if (code & 16) { imask |= 1 << k; continue; }
            e0 |= ((((code & 8) ? o : in) >> (code & 7)) & 1) << k;
          }
          prog.mtab.push_back((int32_t)t.leaf | (e0 << 16) | (imask << 20));
        }
      }
    int n_outer = 0;
    for (int q = 0; q < W; ++q)
      if ((h.outer_mask >> q) & 1) ++n_outer;
    so.n_outer = (int8_t)n_outer;
    so.outer_mask = h.outer_mask;
    // ledger: what a sampling pass runs (ops before the restore point are skipped)
    if (sp.load_n == 0 || (int)hi >= sp.load_n) {
      macs += std::ldexp((double)valid, n_outer);
      elems += std::ldexp((double)(__builtin_popcount(so.in_mask & 0xffff) + __builtin_popcount(so.out_mask & 0xffff)),
                          n_outer);
    }
    ++since_renorm;
    const bool last = ++emitted == n_live_ops;
    so.renorm = (since_renorm >= 8 || last) ? 1 : 0;
    if (so.renorm) since_renorm = 0;
    sd.sw_max_np = std::max(sd.sw_max_np, (int)so.np);
    prog.sweeps.push_back(so);
  }
  if (sp.load_n > 0 && sp.load_n == (int)hops.size()) sd.load_op = emitted;
  if (sp.store_n > 0 && sp.store_n == (int)hops.size()) sd.store_op = emitted;
  // snapshots kept for later steps
  sd.snap_begin = (int)prog.snaps.size();
  sd.snap_count = 0;
  if (sp.anchor) {
    for (auto &sn : sp.anchor->snaps) {
      if (sn.j == (int)hops.size()) sn.op = emitted;
      if (sn.op < 0 || sn.leg_pos.empty()) return undo("snapshot point outside the sweep");
      prog.snaps.push_back(SnapDesc{sn.op, sn.slot, sn.w});
      prog.n_slots = std::max(prog.n_slots, sn.slot + 1);
      prog.max_snap_w = std::max(prog.max_snap_w, sn.w);
      ++sd.snap_count;
    }
    sp.anchor->step_index = (int)prog.steps.size();
  }
  // two-sided: contraction with the snapshot over the shared legs
  sd.merge_slot = -1;
  sd.merge_nb = 0;
  sd.merge_map = (int)prog.mmap.size();
  int merge_src_step = -1, merge_src_op = -1;
  if (sp.merge_from) {
    const AnchorState::Snap &sn = sp.merge_from->snaps[sp.merge_snap];
    if (sn.leg_pos.empty()) return undo("snapshot not emitted before its use");
    for (int l : sp.bound) {
      const int pt = final_pos[l], pr = sn.leg_pos[l];
      if (pt < 0 || pr < 0) return undo("merge leg without a position");
      prog.mmap.push_back(pt);
      prog.mmap.push_back(pr);
    }
    sd.merge_slot = sn.slot;
    sd.merge_nb = (int)sp.bound.size();
    merge_src_step = sp.merge_from->step_index;
    merge_src_op = sn.op;
    macs += std::ldexp((double)(1 << sd.nS), sd.merge_nb);
    elems += std::ldexp(1.0 + (1 << sd.nS), sd.merge_nb);
  }
  sd.load_w = sp.load_n > 0 ? width_after[sp.load_n] : 0;
  sd.store_w = sp.store_n > 0 ? width_after[sp.store_n] : 0;
  sd.sw_count = (int)prog.sweeps.size() - sd.sw_begin;
  sd.m_count = (int)(prog.mtab.size() - (size_t)m_begin) / PWS_MTERMS;
  sd.leaf_area = sd.m_count;
  prog.max_sweep_width = std::max(prog.max_sweep_width, W);
  prog.max_leaf_area = std::max(prog.max_leaf_area, sd.m_count);
  prog.n_sweep_steps += 1;
  prog.sweep_flops_per_sample += macs;   // complex multiply-adds, like the tree ledger
  prog.sweep_elems_per_sample += elems;
  prog.flops_per_sample += macs;
  prog.flops_executed += macs;
  prog.log2_width = std::max(prog.log2_width, W);
  prog.n_slices_total += 1;
  prog.max_exp = std::max(prog.max_exp, 1);
  prog.merge_step.resize(prog.steps.size(), -1);
  prog.merge_op.resize(prog.steps.size(), -1);
  prog.merge_step.push_back(merge_src_step);
  prog.merge_op.push_back(merge_src_op);
  prog.steps.push_back(sd);
  return "";
}

// ------------------------------------------------------------------ export (inspection)

std::string export_json(const CircuitIR &ir, const Programs &prog, int step) {
  std::ostringstream os;
  os.precision(17);
  const StepDesc &sd = prog.steps[step];
  os << "{\"op\":" << sd.op << ",\"gate\":" << sd.gate << ",\"op_begin\":" << sd.op_begin
     << ",\"nS\":" << sd.nS << ",\"root_off\":" << sd.root_off << ",\"root_exp\":" << sd.root_exp
     << ",\"n_slice_bits\":" << sd.n_slice_bits << ",\"arena_elems\":" << sd.arena_elems
     << ",\"root_index\":[" << sd.root_index[0] << "," << sd.root_index[1] << "," << sd.root_index[2]
     << "," << sd.root_index[3] << "],\"zero_q\":[";
  for (int i = 0; i < sd.zero_q_count; ++i) os << (i ? "," : "") << prog.zero_q[sd.zero_q_begin + i];
  os << "],\"scalars\":[";
  for (int f = 0; f < sd.scal_count; ++f) {
    const FactorDesc &fd = prog.factors[sd.scal_begin + f];
    os << (f ? "," : "") << "[" << fd.kind << "," << fd.id << "," << fd.nq << "," << fd.frame << ","
       << fd.src_out[0] << "," << fd.src_out[1] << "," << fd.src_in[0] << "," << fd.src_in[1] << "]";
  }
  os << "],\"elems\":[";
  for (int i = 0; i < 2 * sd.n_elems; ++i) os << (i ? "," : "") << prog.lelem[2 * (size_t)sd.elem_begin + i];
  os << "],\"leaves\":[";
  for (int i = 0; i < sd.n_leaves; ++i) {
    const LeafDesc &ld = prog.leaves[sd.leaf_begin + i];
    os << (i ? "," : "") << "{\"off\":" << ld.out_off << ",\"nfree\":" << ld.nfree << ",\"tab_off\":" << ld.tab_off
       << ",\"r_count\":" << ld.r_count << ",\"var\":[";
    for (int v = 0; v < (ld.tab_off >= 0 ? ld.nvar : 0); ++v) os << (v ? "," : "") << prog.lvar[ld.var_begin + v];
    os << "],\"tab\":[";
    if (ld.tab_off >= 0)
      for (int v = 0; v < (2 << ld.nvar) << ld.nfree; ++v) os << (v ? "," : "") << prog.ltab[2 * (size_t)ld.tab_off + v];
    os << "],\"factors\":[";
    for (int f = 0; f < ld.f_count; ++f) {
      const FactorDesc &fd = prog.factors[ld.f_begin + f];
      os << (f ? "," : "") << "[" << fd.kind << "," << fd.id << "," << fd.nq << "," << fd.frame << ","
         << fd.src_out[0] << "," << fd.src_out[1] << "," << fd.src_in[0] << "," << fd.src_in[1] << "]";
    }
    os << "]}";
  }
  os << "],\"nodes\":[";
  for (int i = 0; i < sd.n_nodes; ++i) {
    const NodeDesc &nd = prog.nodes[sd.node_begin + i];
    os << (i ? "," : "") << "{\"kind\":" << nd.kind << ",\"p_bits\":" << nd.p_bits << ",\"n_bits\":" << nd.n_bits
       << ",\"out\":" << nd.out_off << ",\"a\":" << nd.a_off << ",\"b\":" << nd.b_off
       << ",\"out_bits\":" << nd.out_bits << ",\"k_bits\":" << nd.k_bits << ",\"exp\":[" << nd.exp_a << ","
       << nd.exp_b << "," << nd.exp_out << "],\"modes\":[";
    for (int m = 0; m < nd.nmodes; ++m)
      os << (m ? "," : "") << "[" << nd.mode_width[m] << "," << nd.strideA[m] << "," << nd.strideB[m] << ","
         << nd.strideO[m] << "]";
    os << "],\"ktab\":[";
    for (int k = 0; k < (2 << nd.k_bits); ++k) os << (k ? "," : "") << prog.ktab[nd.ktab_off + k];
    os << "],\"ntab\":[";
    for (int k = 0; k < (nd.kind == NODE_BLOCKED ? (2 << nd.n_bits) : nd.kind == NODE_MFMA ? 64 : 0); ++k)
      os << (k ? "," : "") << prog.ktab[nd.ntab_off + k];
    os << "]}";
  }
  os << "],\"fresh\":" << sd.fresh << ",\"sweep\":" << sd.sweep << ",\"sw_width\":" << sd.sw_width << ",\"leaf_area\":" << sd.leaf_area
     << ",\"load_op\":" << (sd.sweep ? sd.load_op : -1) << ",\"store_op\":" << (sd.sweep ? sd.store_op : -1)
     << ",\"load_w\":" << sd.load_w << ",\"store_w\":" << sd.store_w << ",\"snaps\":[";
  for (int i = 0; i < (sd.sweep ? sd.snap_count : 0); ++i) {
    const SnapDesc &sn = prog.snaps[sd.snap_begin + i];
    os << (i ? "," : "") << "[" << sn.op << "," << sn.slot << "," << sn.w << "]";
  }
  os << "],\"merge\":";
  if (sd.sweep && sd.merge_slot >= 0) {
    const int ms = step < (int)prog.merge_step.size() ? prog.merge_step[step] : -1;
    const int mo = step < (int)prog.merge_op.size() ? prog.merge_op[step] : -1;
    os << "{\"slot\":" << sd.merge_slot << ",\"step\":" << ms << ",\"op\":" << mo << ",\"pairs\":[";
    for (int k = 0; k < sd.merge_nb; ++k)
      os << (k ? "," : "") << "[" << prog.mmap[sd.merge_map + 2 * k] << "," << prog.mmap[sd.merge_map + 2 * k + 1] << "]";
    os << "]}";
  } else {
    os << "null";
  }
  os << ",\"dense\":";
  if (sd.sweep && sd.dn_count > 0) {
    os << "{\"bf16\":" << (prog.dense_bf16 ? 1 : 0) << ",\"op0\":" << sd.dn_op0 << ",\"w\":" << sd.dn_w << ",\"load\":" << sd.dn_load << ",\"runs\":[";
    for (int r = 0; r < sd.dn_count; ++r) {
      const DenseRun &dr = prog.druns[sd.dn_begin + r];
      const int nq = (dr.info >> 8) & 0xff;
      const int n_outer = dr.info & 0xff;
      int outer = dr.outer_mask;
      for (int t = 0; t < std::min(n_outer, 4); ++t) outer |= 1 << ((dr.pos >> (16 + 4 * t)) & 15);
      os << (r ? "," : "") << "{\"op\":" << dr.op << ",\"pos\":[" << (dr.pos & 15) << "," << ((dr.pos >> 4) & 15)
         << "," << ((dr.pos >> 8) & 15) << "," << ((dr.pos >> 12) & 15) << "],\"outer_mask\":" << outer
         << ",\"n_outer\":" << n_outer << ",\"renorm\":" << ((dr.info >> 16) & 1) << ",\"qubits\":[";
      for (int b = 0; b < nq; ++b)
        os << (b ? "," : "") << dense_qubit(dr.q012, dr.q345, dr.q67, b);
      os << "],\"F\":[";
      for (int v = 0; v < (1 << nq); ++v)
        for (int e = 0; e < 512; ++e)
          os << ((v || e) ? "," : "") << prog.dtab[((size_t)dr.foff + v) * 512 + e];
      os << "]}";
    }
    os << "]}";
  } else {
    os << "null";
  }
  os << ",\"sweeps\":[";
  for (int i = 0; i < (sd.sweep ? sd.sw_count : 0); ++i) {
    const SweepOp &so = prog.sweeps[sd.sw_begin + i];
    os << (i ? "," : "") << "{\"leaf\":" << so.leaf << ",\"np\":" << (int)so.np << ",\"diag\":" << (int)so.diag
       << ",\"renorm\":" << (int)so.renorm << ",\"n_outer\":" << (int)so.n_outer << ",\"in_mask\":" << so.in_mask
       << ",\"out_mask\":" << so.out_mask << ",\"outer_mask\":" << so.outer_mask << ",\"mtab\":[";
    {
      const int ng = 1 << so.np, msz = so.diag == 1 ? ng : ng * ng;
      for (int e = 0; e < msz * PWS_MTERMS; ++e)
        os << (e ? "," : "") << prog.mtab[(size_t)sd.m_begin + (size_t)so.moff * PWS_MTERMS + e];
      os << "],\"ment\":[";
      for (int e = 0; e < msz; ++e) {
        const MEntry &me = prog.ment[(size_t)sd.m_begin / PWS_MTERMS + (size_t)so.moff + e];
        // [re, im, from codes, [[bit positions..., term values (re, im) by variant...]...]]
        os << (e ? "," : "") << "[" << me.re << "," << me.im << "," << (me.t0 == PWS_MENTRY_CODES || me.t0 == PWS_MENTRY_FLAT ? 1 : 0) << ",[";
        int nt = 0;
        for (const auto &tp : {std::make_pair(me.t0, me.p0), std::make_pair(me.t1, me.p1)}) {
          if (tp.first < 0) continue;
          const int nv = tp.second >> 24;
          os << (nt++ ? "," : "") << "[[";
          for (int k = 0; k < nv; ++k) os << (k ? "," : "") << ((tp.second >> (12 * k)) & 0xfff);
          os << "]";
          for (int v = 0; v < (1 << nv); ++v)
            os << "," << prog.mterm[2 * ((size_t)tp.first + v)] << "," << prog.mterm[2 * ((size_t)tp.first + v) + 1];
          os << "]";
        }
        os << "]]";
      }
    }
    os << "],\"pos\":[";
    for (int j = 0; j < so.np; ++j) os << (j ? "," : "") << (int)so.pos[j];
    os << "],\"role\":[";
    for (int j = 0; j < so.np; ++j) os << (j ? "," : "") << (int)so.role[j];
    os << "],\"leg\":[";
    for (int k = 0; k < so.nleg; ++k) os << (k ? "," : "") << (int)so.leg[k];
    os << "]}";
  }
  os << "],\"gates\":[";
  for (size_t g = 0; g < ir.gates.size(); ++g) {
    const GateIR &G = ir.gates[g];
    const int d = 1 << G.nq;
    os << (g ? "," : "") << "{\"nq\":" << G.nq << ",\"q\":[" << G.q[0] << "," << G.q[1] << "],\"mat\":[";
    for (int e = 0; e < d * d; ++e) os << (e ? "," : "") << G.mat[e].real() << "," << G.mat[e].imag();
    os << "]}";
  }
  os << "]}";
  return os.str();
}

}  // namespace pws
