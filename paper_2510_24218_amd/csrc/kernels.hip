// Device kernels of the pilot-wave sampler (gfx950).
//
// One launch per contraction step ("persistent" over chains: each workgroup
// loops over chains).  For one chain a workgroup
//   1. replays the ops since the previous step: monomial gates move the
//      classical state (Algorithm 1, s[q] <- sigma(s[q])), diagonal gates do
//      nothing, noise sites draw their Kraus branch from Eq. (4) on the true
//      bit and update the X-frame and the per-segment diagonal factors
//      (Algorithm 2, PropagateX / AddGate);
//   2. materialises the leaves of the step's network (gate entries with the
//      projected legs read from the chain's bits, frame-conjugated gates and
//      noise factors);
//   3. contracts the network node by node in a per-workgroup arena, keeping
//      every intermediate as mantissa * 2^exponent (exact power-of-two
//      renormalisation after each node);
//   4. draws the next state among the block's candidates with FP64
//      probabilities, their prefix sum and a Philox4x64-10 uniform.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"

namespace pws {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxWords = 16;   // up to 1024 qubits

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

// ---------------------------------------------------------------- Philox4x64-10
// Salmon, Moraes, Dror, Shaw (SC'11): published round multipliers and Weyl
// key increments; counter (op, chain, 0, 0), key (seed, 0).
__device__ inline uint64_t philox_w0(uint64_t c0, uint64_t c1, uint64_t k0) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t c2 = 0, c3 = 0, k1 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return c0;
}

__device__ inline double uniform53(uint64_t op, uint64_t chain, uint64_t seed) {
  return (double)(philox_w0(op, chain, seed) >> 11) * 0x1p-53;
}

// Draw rule shared with the oracle: smallest v with u * P < C_v (inclusive
// prefix), P = 0 -> -1, rounding fallback: last v with p_v > 0.  Plain IEEE
// double operations in a fixed order (no fused multiply-add).
__device__ __noinline__ int draw_index(const double *p, int m, double u) {
#pragma clang fp contract(off)
  double P = p[0];
  for (int v = 1; v < m; ++v) P = P + p[v];
  if (!(P > 0.0)) return -1;
  const double target = u * P;
  double C = 0.0;
  for (int v = 0; v < m; ++v) {
    C = C + p[v];
    if (target < C) return v;
  }
  for (int v = m - 1; v >= 0; --v)
    if (p[v] > 0.0) return v;
  return -1;
}

__device__ inline double norm2_exact(double re, double im) {
#pragma clang fp contract(off)
  return re * re + im * im;
}

__device__ inline int getbit(const uint64_t *w, int q) { return (int)((w[q >> 6] >> (q & 63)) & 1ull); }
__device__ inline void setbit(uint64_t *w, int q, int b) {
  const uint64_t m = 1ull << (q & 63);
  w[q >> 6] = b ? (w[q >> 6] | m) : (w[q >> 6] & ~m);
}

struct cplxd { double re, im; };
__device__ inline cplxd cmul(cplxd a, cplxd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// Value of one factor at leaf element e.
__device__ inline cplxd factor_value(const DevProg &p, const ChainState &st, int64_t c,
                                     const FactorDesc &f, int e, int slice, const uint64_t *s_sh,
                                     bool deriv) {
  auto bit = [&](int32_t src) -> int {
    const int t = src_type(src), pl = src_payload(src);
    if (t == SRC_FREE) return (e >> pl) & 1;
    if (t == SRC_CONST) return pl;
    if (t == SRC_CHAIN) return getbit(s_sh, pl);
    return (slice >> pl) & 1;
  };
  if (f.kind == FAC_SEGFAC) {
    const double *sf = st.segfac + ((size_t)c * p.n_segs + f.id) * 4;
    return bit(f.src_out[0]) ? cplxd{sf[2], sf[3]} : cplxd{sf[0], sf[1]};
  }
  int out = 0, in = 0;
  for (int j = 0; j < f.nq; ++j) {
    out = 2 * out + bit(f.src_out[j]);
    in = 2 * in + bit(f.src_in[j]);
  }
  if (f.frame) {
    const int fr = st.gframe[(size_t)c * p.n_gates + f.id];
    out ^= fr;
    in ^= fr;
  }
  const int d = 1 << f.nq;
  const double *m = ((deriv || f.kind == FAC_GATE_DERIV) ? p.gdmat : p.gmat) + (size_t)f.id * 32 + 2 * (out * d + in);
  return {m[0], m[1]};
}

template <typename T>
__device__ inline T block_max(T v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[wave] = (double)v;
  __syncthreads();
  double m = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
  return (T)m;
}

__device__ inline double block_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

// One pairwise contraction of the step tree for the current chain, followed
// by an exact power-of-two renormalisation.  Ends with a barrier.
template <typename T>
__device__ void run_node(const NodeDesc &nd, typename Cplx<T>::type *arena, const int32_t *ktab,
                         int *exps, double *red) {
  using V = typename Cplx<T>::type;
  const int nout = 1 << nd.out_bits;
  const int nk = 1 << nd.k_bits;
  const V *A = arena + nd.a_off;
  const V *B = arena + nd.b_off;
  V *O = arena + nd.out_off;
  const int32_t *kt = ktab + nd.ktab_off;
  T lmax = 0;
  for (int o = threadIdx.x; o < nout; o += blockDim.x) {
    int offA = 0, offB = 0, rem = o;
    for (int m = 0; m < nd.nmodes; ++m) {
      const int w = nd.mode_width[m];
      const int v = rem & ((1 << w) - 1);
      rem >>= w;
      offA += v * nd.strideA[m];
      offB += v * nd.strideB[m];
    }
    T ar = 0, ai = 0;
    for (int k = 0; k < nk; ++k) {
      const V a = A[offA + kt[2 * k]];
      const V b = B[offB + kt[2 * k + 1]];
      ar += a.x * b.x - a.y * b.y;
      ai += a.x * b.y + a.y * b.x;
    }
    V r;
    r.x = ar;
    r.y = ai;
    O[o] = r;
    lmax = fmax(lmax, fmax(fabs(ar), fabs(ai)));
  }
  const T gmax = block_max<T>(lmax, red);
  int e = 0;
  if (gmax > 0) e = ilogb(gmax) + 1;
  if (e != 0) {
    const T sc = ldexp((T)1, -e);
    for (int o = threadIdx.x; o < nout; o += blockDim.x) {
      V r = O[o];
      r.x *= sc;
      r.y *= sc;
      O[o] = r;
    }
  }
  if (threadIdx.x == 0)
    exps[nd.exp_out] = e + (nd.exp_a >= 0 ? exps[nd.exp_a] : 0) + (nd.exp_b >= 0 ? exps[nd.exp_b] : 0);
  __syncthreads();
}

template <typename T>
__device__ void materialise_leaves(const DevProg &p, const ChainState &st, const StepDesc &sd,
                                   int64_t c, int slice, const uint64_t *s_sh,
                                   typename Cplx<T>::type *arena) {
  using V = typename Cplx<T>::type;
  for (int li = threadIdx.x; li < sd.n_leaves; li += blockDim.x) {
    const LeafDesc ld = p.leaves[sd.leaf_begin + li];
    const int ne = 1 << ld.nfree;
    for (int e = 0; e < ne; ++e) {
      cplxd v{1.0, 0.0};
      for (int fi = 0; fi < ld.f_count; ++fi)
        v = cmul(v, factor_value(p, st, c, p.factors[ld.f_begin + fi], e, slice, s_sh, false));
      V r;
      r.x = (T)v.re;
      r.y = (T)v.im;
      arena[ld.out_off + e] = r;
    }
  }
}

// Replay ops [op_begin, op_end) for one chain (thread 0 only).
__device__ bool replay_ops(const DevProg &p, const ChainState &st, int64_t c, uint64_t chain_gid,
                           uint64_t seed, int op_begin, int op_end, uint64_t *s_sh, uint64_t *x_sh) {
  bool ok = true;
  for (int op = op_begin; op < op_end; ++op) {
    const OpDesc od = p.ops[op];
    if (od.type == 0) {
      const GateDev g = p.gates[od.idx];
      const int q[2] = {g.q0, g.q1};
      int f = 0, loc = 0;
      for (int j = 0; j < g.nq; ++j) {
        f = 2 * f + getbit(x_sh, q[j]);
        loc = 2 * loc + getbit(s_sh, q[j]);
      }
      if (p.noisy) st.gframe[(size_t)c * p.n_gates + od.idx] = (uint8_t)f;
      if (g.monomial && !g.diagonal) {
        const int nl = g.sigma[loc ^ f] ^ f;
        for (int j = 0; j < g.nq; ++j) setbit(s_sh, q[j], (nl >> (g.nq - 1 - j)) & 1);
      }
    } else {
      const NoiseDev nd = p.noise[od.idx];
      const int q[2] = {nd.q0, nd.q1};
      int t[2] = {0, 0};
      for (int j = 0; j < nd.nq; ++j) t[j] = getbit(s_sh, q[j]) ^ getbit(x_sh, q[j]);
      double pr[16];
      for (int i = 0; i < nd.nbranch; ++i) {
#pragma clang fp contract(off)
        double v = p.ntab[nd.tab_off + i * nd.nq].colnorm[t[0]];
        for (int j = 1; j < nd.nq; ++j) v = v * p.ntab[nd.tab_off + i * nd.nq + j].colnorm[t[j]];
        pr[i] = v;
      }
      const int br = draw_index(pr, nd.nbranch, uniform53((uint64_t)op, chain_gid, seed));
      if (br < 0) { ok = false; continue; }
      for (int j = 0; j < nd.nq; ++j) {
        const NoiseBranch nb = p.ntab[nd.tab_off + br * nd.nq + j];
        if (nb.anti) setbit(x_sh, q[j], getbit(x_sh, q[j]) ^ 1);
        cplxd d0{nb.d0re, nb.d0im}, d1{nb.d1re, nb.d1im};
        if (getbit(x_sh, q[j])) { cplxd tmp = d0; d0 = d1; d1 = tmp; }
        double *sf = st.segfac + ((size_t)c * p.n_segs + nd.seg[j]) * 4;
        const cplxd a0 = cmul(cplxd{sf[0], sf[1]}, d0), a1 = cmul(cplxd{sf[2], sf[3]}, d1);
        sf[0] = a0.re; sf[1] = a0.im; sf[2] = a1.re; sf[3] = a1.im;
      }
    }
  }
  return ok;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void step_kernel(DevProg p, ChainState st, StepLaunch L) {
  using V = typename Cplx<T>::type;
  extern __shared__ int exps[];
  __shared__ uint64_t s_sh[kMaxWords], x_sh[kMaxWords];
  __shared__ double red[kBlock / 64];
  __shared__ double acc[8];
  __shared__ int ctl[4];   // 0: run contraction, 1: candidate mask, 2: zero root, 3: acc exponent
  const StepDesc sd = p.steps[L.step];
  V *arena = reinterpret_cast<V *>(L.arena) + (int64_t)blockIdx.x * L.arena_stride;
  const int W = p.words;
  for (int64_t c = blockIdx.x; c < L.n_chains; c += gridDim.x) {
    const uint64_t chain_gid = (uint64_t)(L.chain_offset + c);
    if (threadIdx.x < W) {
      s_sh[threadIdx.x] = st.s[(size_t)c * W + threadIdx.x];
      x_sh[threadIdx.x] = p.noisy ? st.x[(size_t)c * W + threadIdx.x] : 0ull;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      bool ok = true;
      if (L.mode == MODE_SAMPLE) {
        const int op_end = sd.op >= 0 ? sd.op : p.n_ops;
        ok = replay_ops(p, st, c, chain_gid, L.seed, sd.op_begin, op_end, s_sh, x_sh);
      }
      int run = sd.n_nodes > 0 ? 1 : 0, mask = (1 << sd.nS) - 1, zero = 0;
      if (sd.gate >= 0) {
        const GateDev g = p.gates[sd.gate];
        const int q[2] = {g.q0, g.q1};
        int f = 0, loc = 0;
        for (int j = 0; j < g.nq; ++j) {
          f = 2 * f + getbit(x_sh, q[j]);
          loc = 2 * loc + getbit(s_sh, q[j]);
        }
        if (p.noisy && L.mode == MODE_SAMPLE) st.gframe[(size_t)c * p.n_gates + sd.gate] = (uint8_t)f;
        if (L.mode == MODE_SAMPLE) {
          int fS = 0;
          for (int k = 0; k < g.nS; ++k) fS = 2 * fS + ((f >> (g.nq - 1 - g.sq[k])) & 1);
          const int raw = g.cand_mask[loc ^ f];
          mask = 0;
          for (int v = 0; v < (1 << g.nS); ++v)
            if ((raw >> (v ^ fS)) & 1) mask |= 1 << v;
          if (__popc(mask) <= 1) run = 0;   // block of size one: s stays
        }
      }
      for (int i = 0; i < sd.zero_q_count; ++i)
        if (getbit(s_sh, p.zero_q[sd.zero_q_begin + i])) zero = 1;
      if (zero) run = 0;
      if (!ok) atomicOr(L.err, 2);
      ctl[0] = run;
      ctl[1] = mask;
      ctl[2] = zero;
    }
    __syncthreads();
    const int run = ctl[0];
    if (run) {
      const int nsl = 1 << sd.n_slice_bits;
      for (int sl = 0; sl < nsl; ++sl) {
        materialise_leaves<T>(p, st, sd, c, sl, s_sh, arena);
        __syncthreads();
        for (int i = 0; i < sd.n_nodes; ++i) run_node<T>(p.nodes[sd.node_begin + i], arena, p.ktab, exps, red);
        if (threadIdx.x == 0) {
          const int er = sd.root_exp >= 0 ? exps[sd.root_exp] : 0;
          const int m = 1 << sd.nS;
          if (sl == 0) {
            ctl[3] = er;
            for (int v = 0; v < m; ++v) {
              const V r = arena[sd.root_off + sd.root_index[v]];
              acc[2 * v] = (double)r.x;
              acc[2 * v + 1] = (double)r.y;
            }
          } else {
            int ea = ctl[3];
            if (er > ea) {
              for (int v = 0; v < 2 * m; ++v) acc[v] = ldexp(acc[v], ea - er);
              ea = er;
              ctl[3] = ea;
            }
            for (int v = 0; v < m; ++v) {
              const V r = arena[sd.root_off + sd.root_index[v]];
              acc[2 * v] += ldexp((double)r.x, er - ea);
              acc[2 * v + 1] += ldexp((double)r.y, er - ea);
            }
          }
        }
        __syncthreads();
      }
    }
    if (threadIdx.x == 0) {
      const int m = 1 << sd.nS;
      if (L.mode == MODE_SAMPLE) {
        if (run && sd.gate >= 0) {
          double pv[4];
          const int mask = ctl[1];
          for (int v = 0; v < m; ++v) pv[v] = ((mask >> v) & 1) ? norm2_exact(acc[2 * v], acc[2 * v + 1]) : 0.0;
          const double u = uniform53((uint64_t)sd.op, chain_gid, L.seed);
          const int vs = draw_index(pv, m, u);
          if (vs < 0) {
            atomicOr(L.err, 1);
          } else {
            const GateDev g = p.gates[sd.gate];
            const int q[2] = {g.q0, g.q1};
            for (int k = 0; k < g.nS; ++k) setbit(s_sh, q[g.sq[k]], (vs >> (g.nS - 1 - k)) & 1);
          }
          if (L.trace) L.trace[(size_t)L.trace_row * L.n_chains + c] = (uint8_t)(vs < 0 ? 255 : vs);
        } else if (L.trace && sd.gate >= 0) {
          L.trace[(size_t)L.trace_row * L.n_chains + c] = 254;
        }
      } else {
        const bool z = !run || ctl[2];
        for (int v = 0; v < m; ++v) {
          L.out_amp[((size_t)c * m + v) * 2] = z ? 0.0 : acc[2 * v];
          L.out_amp[((size_t)c * m + v) * 2 + 1] = z ? 0.0 : acc[2 * v + 1];
        }
        L.out_log2[c] = z ? 0 : ctl[3];
      }
    }
    __syncthreads();
    if (L.mode == MODE_SAMPLE && threadIdx.x < W) {
      st.s[(size_t)c * W + threadIdx.x] = s_sh[threadIdx.x];
      if (p.noisy) st.x[(size_t)c * W + threadIdx.x] = x_sh[threadIdx.x];
    }
    __syncthreads();
  }
}

__global__ void init_state_kernel(DevProg p, ChainState st, int64_t K) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int W = p.words;
  if (i < K * W) {
    st.s[i] = 0ull;
    if (p.noisy) st.x[i] = 0ull;
  }
  if (p.noisy) {
    if (i < K * p.n_gates) st.gframe[i] = 0;
    if (i < K * p.n_segs) {
      double *sf = st.segfac + i * 4;
      sf[0] = 1.0; sf[1] = 0.0; sf[2] = 1.0; sf[3] = 0.0;
    }
  }
}

__global__ void finalize_kernel(DevProg p, ChainState st, int64_t K, uint64_t *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K * p.words) out[i] = p.noisy ? (st.s[i] ^ st.x[i]) : st.s[i];
}

// ---------------------------------------------------------------- gradient
// Forward contraction of the full circuit with every leg projected onto the
// sample, then the reverse pass: the adjoint of each child is the contraction
// of its parent's adjoint with its sibling; each parametrised gate factor adds
// <adjoint of its leaf, d leaf / d theta> to d amp / d theta.
template <typename T>
__global__ __launch_bounds__(kBlock) void grad_kernel(DevProg p, ChainState st, GradLaunch L) {
  using V = typename Cplx<T>::type;
  extern __shared__ int exps[];
  __shared__ uint64_t s_sh[kMaxWords];
  __shared__ double red[kBlock / 64];
  __shared__ double root[3];
  const StepDesc sd = p.steps[0];
  V *arena = reinterpret_cast<V *>(L.arena) + (int64_t)blockIdx.x * L.arena_stride;
  const int W = p.words;
  for (int64_t c = blockIdx.x; c < L.n_chains; c += gridDim.x) {
    if (threadIdx.x < W) s_sh[threadIdx.x] = st.s[(size_t)c * W + threadIdx.x];
    __syncthreads();
    materialise_leaves<T>(p, st, sd, c, 0, s_sh, arena);
    __syncthreads();
    for (int i = 0; i < sd.n_nodes; ++i) run_node<T>(p.nodes[sd.node_begin + i], arena, p.ktab, exps, red);
    if (threadIdx.x == 0) {
      const V r = arena[sd.root_off];
      root[0] = (double)r.x;
      root[1] = (double)r.y;
      root[2] = (double)(sd.root_exp >= 0 ? exps[sd.root_exp] : 0);
      // adjoint of the root: 1 (stored right after the forward tensors by the planner)
      V one;
      one.x = 1;
      one.y = 0;
      arena[p.bnodes[0].a_off] = one;
    }
    __syncthreads();
    for (int i = 0; i < p.n_bnodes; ++i) run_node<T>(p.bnodes[i], arena, p.ktab, exps, red);
    const double mr = root[0], mi = root[1];
    const int er = (int)root[2];
    const double den = mr * mr + mi * mi;
    for (int j = 0; j < p.n_params; ++j) {
      double part_re = 0, part_im = 0;
      for (int t = threadIdx.x; t < p.n_grad_terms; t += blockDim.x) {
        const int32_t *gt = p.grad_terms + 5 * t;
        if (gt[2] != j) continue;
        const LeafDesc ld = p.leaves[sd.leaf_begin + gt[0]];
        const int ea = gt[4] >= 0 ? exps[gt[4]] : 0;
        const int ne = 1 << ld.nfree;
        double sre = 0, sim = 0;
        for (int e = 0; e < ne; ++e) {
          cplxd v{1.0, 0.0};
          for (int fi = 0; fi < ld.f_count; ++fi)
            v = cmul(v, factor_value(p, st, c, p.factors[ld.f_begin + fi], e, 0, s_sh, fi == gt[1]));
          const V a = arena[gt[3] + e];
          sre += (double)a.x * v.re - (double)a.y * v.im;
          sim += (double)a.x * v.im + (double)a.y * v.re;
        }
        part_re += ldexp(sre, ea - er);
        part_im += ldexp(sim, ea - er);
      }
      const double tre = block_sum(part_re, red);
      const double tim = block_sum(part_im, red);
      if (threadIdx.x == 0) {
        // d log|amp|^2 = 2 Re(d amp / amp) = 2 Re(t * conj(m)) / |m|^2
        const double val = den > 0 ? 2.0 * (tre * mr + tim * mi) / den : 0.0;
        L.dtheta[(size_t)c * p.n_params + j] = val;
        if (!(den > 0)) atomicOr(L.err, 4);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0 && L.amp) {
      L.amp[2 * c] = mr;
      L.amp[2 * c + 1] = mi;
      if (L.amp_log2) L.amp_log2[c] = er;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_init_state(const DevProg &p, const ChainState &st, int64_t K, hipStream_t s) {
  int64_t n = K * (int64_t)p.words;
  if (p.noisy) {
    n = std::max<int64_t>(n, K * (int64_t)p.n_gates);
    n = std::max<int64_t>(n, K * (int64_t)p.n_segs);
  }
  const int blocks = (int)((n + 255) / 256);
  hipLaunchKernelGGL(init_state_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, s, p, st, K);
  return hipGetLastError();
}

hipError_t launch_step(int precision, const DevProg &p, const ChainState &st, const StepLaunch &l,
                       hipStream_t s) {
  if (precision == 0)
    hipLaunchKernelGGL(step_kernel<double>, dim3(l.grid), dim3(l.block), l.lds_bytes, s, p, st, l);
  else
    hipLaunchKernelGGL(step_kernel<float>, dim3(l.grid), dim3(l.block), l.lds_bytes, s, p, st, l);
  return hipGetLastError();
}

hipError_t launch_finalize(const DevProg &p, const ChainState &st, int64_t K, uint64_t *out,
                           hipStream_t s) {
  const int64_t n = K * (int64_t)p.words;
  const int blocks = (int)((n + 255) / 256);
  hipLaunchKernelGGL(finalize_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, s, p, st, K, out);
  return hipGetLastError();
}

hipError_t launch_grad(int precision, const DevProg &p, const ChainState &st, const GradLaunch &l,
                       hipStream_t s) {
  if (precision == 0)
    hipLaunchKernelGGL(grad_kernel<double>, dim3(l.grid), dim3(l.block), l.lds_bytes, s, p, st, l);
  else
    hipLaunchKernelGGL(grad_kernel<float>, dim3(l.grid), dim3(l.block), l.lds_bytes, s, p, st, l);
  return hipGetLastError();
}

}  // namespace pws
