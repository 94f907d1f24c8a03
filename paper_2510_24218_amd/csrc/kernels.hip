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
#include <climits>
#include <mutex>

#include "device.hpp"

namespace pws {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxWords = 16;   // up to 1024 qubits

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

// matrix-core operand and accumulator vectors
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

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
// double operations in a fixed order (no fused multiply-add).  Candidate
// blocks have at most four members; the weights stay in registers.
__device__ inline int draw4(double p0, double p1, double p2, double p3, int m, double u) {
#pragma clang fp contract(off)
  double P = p0;
  if (m > 1) P = P + p1;
  if (m > 2) P = P + p2;
  if (m > 3) P = P + p3;
  if (!(P > 0.0)) return -1;
  const double target = u * P;
  double C = 0.0 + p0;
  if (target < C) return 0;
  if (m > 1) { C = C + p1; if (target < C) return 1; }
  if (m > 2) { C = C + p2; if (target < C) return 2; }
  if (m > 3) { C = C + p3; if (target < C) return 3; }
  if (m > 3 && p3 > 0.0) return 3;
  if (m > 2 && p2 > 0.0) return 2;
  if (m > 1 && p1 > 0.0) return 1;
  return p0 > 0.0 ? 0 : -1;
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

// ---------------------------------------------------------------- wave helpers
// One wavefront owns one chain at a time: every tensor of the chain's network
// is read and written only by the 64 lanes of that wave, so node-to-node
// ordering needs no workgroup barrier.  Vector memory operations of a wave
// complete in issue order; the fence keeps the compiler from reordering.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// ilogb of a non-negative value from the high 32 bits of its encoding
// (INT_MIN for zero; a subnormal counts as the smallest normal exponent).
template <typename T>
__device__ inline int hiword_ilogb(unsigned hw) {
  if (hw == 0) return INT_MIN;
  if constexpr (sizeof(T) == 8) return (int)((hw >> 20) & 0x7ff) - 1023;
  else return (int)((hw >> 23) & 0xff) - 127;
}

template <typename T>
__device__ inline T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

template <int CTRL>
__device__ inline unsigned dpp_umax(unsigned u) {
  return max(u, (unsigned)__builtin_amdgcn_update_dpp((int)u, (int)u, CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ inline double dpp_add_f64(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, 0xf, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return x + __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum of x over the NL lanes of a chain (16, 32 or 64 lanes, aligned), of
// which only the first `used` hold non-zero values: within each row of 16
// lanes a butterfly of DPP row permutations (every lane ends with the row's
// sum, the same additions in every lane), then the rows in use.  All lanes
// of the wave take part.
template <int NL>
__device__ inline double chain_sum_f64(double x, int used) {
  x = dpp_add_f64<0xB1>(x);    // lane ^ 1
  x = dpp_add_f64<0x4E>(x);    // lane ^ 2
  x = dpp_add_f64<0x141>(x);   // the other quad of each half row
  x = dpp_add_f64<0x140>(x);   // the other half row
  if constexpr (NL >= 32) {
    if (used > 16) {
      const unsigned long long b = (unsigned long long)__double_as_longlong(x);
      const unsigned lo = (unsigned)__builtin_amdgcn_ds_swizzle((int)b, 0x401f);   // lane ^ 16
      const unsigned hi = (unsigned)__builtin_amdgcn_ds_swizzle((int)(b >> 32), 0x401f);
      x += __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    }
  }
  if constexpr (NL >= 64)
    if (used > 32) x += __shfl_xor(x, 32, 64);
  return x;
}

// Exponent (ilogb) of the largest of the wave's non-negative values, taken
// from the high 32 bits of their encodings (which order non-negative values):
// DPP max within each row of 16 lanes, then the four row results through
// scalar registers.  Returns INT_MIN when every value is zero.
template <typename T>
__device__ inline int wave_max_ilogb(T v) {
  unsigned u;
  if constexpr (sizeof(T) == 8) u = (unsigned)((unsigned long long)__double_as_longlong(v) >> 32);
  else u = __float_as_uint(v);
  u = dpp_umax<0xB1>(u);    // quad_perm [1,0,3,2]
  u = dpp_umax<0x4E>(u);    // quad_perm [2,3,0,1]
  u = dpp_umax<0x141>(u);   // row_half_mirror
  u = dpp_umax<0x140>(u);   // row_mirror
  const unsigned r = max(max((unsigned)__builtin_amdgcn_readlane((int)u, 0), (unsigned)__builtin_amdgcn_readlane((int)u, 16)),
                         max((unsigned)__builtin_amdgcn_readlane((int)u, 32), (unsigned)__builtin_amdgcn_readlane((int)u, 48)));
  return hiword_ilogb<T>(r);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Per-wave scratch in LDS.
struct WaveLds {
  uint64_t *s;      // kMaxWords
  uint64_t *x;      // kMaxWords
  double *acc;      // 8
  int *ctl;         // 4
  int *E;           // accumulated exponent per tensor slot
  int *M;           // max exponent of the stored mantissas per slot
};

__host__ __device__ inline int wave_lds_bytes(int n_exp) {
  return (kMaxWords * 8) * 2 + 8 * 8 + 4 * 4 + ((2 * n_exp * 4 + 15) / 16) * 16;
}

__device__ inline WaveLds wave_lds(unsigned char *base, int wave, int n_exp) {
  unsigned char *p = base + (size_t)wave * wave_lds_bytes(n_exp);
  WaveLds w;
  w.s = (uint64_t *)p;
  w.x = w.s + kMaxWords;
  w.acc = (double *)(w.x + kMaxWords);
  w.ctl = (int *)(w.acc + 8);
  w.E = w.ctl + 4;
  w.M = w.E + n_exp;
  return w;
}

// One pairwise contraction for the wave's chain.  Stored values are
// mantissas: a tensor's value is mantissa * 2^E[slot]; M[slot] is the
// exponent of its largest stored component.  The output mantissa is
// (sum A B) * 2^-(M_A + M_B), so operands stay near unit size whatever the
// network's scale (exact power-of-two scaling, no rounding added).
#ifndef PWS_NODE_ROWS
#define PWS_NODE_ROWS 2
#endif
// Matrix-core node (NODE_MFMA), kept out of line so that its registers do
// not count against the other node forms.  Returns the lane's largest
// written component.
template <typename T>
__device__ __attribute__((noinline)) T node_mfma(const NodeDesc *__restrict__ ndp,
                                                 const typename Cplx<T>::type *A, const typename Cplx<T>::type *B,
                                                 typename Cplx<T>::type *O, const int32_t *kt, const int32_t *nt,
                                                 T sc, int lane) {
  using V = typename Cplx<T>::type;
  const int nmodes = ndp->nmodes;
  const int np = 1 << ndp->p_bits, nk = 1 << ndp->k_bits;
  T lmax = 0;
  // tile offsets (the tile index cut into the node's fields)
  auto tile_offsets = [&](int t, int &offA, int &offB, int &offO) {
    int rem = t;
    offA = offB = offO = 0;
    for (int m = 0; m < nmodes; ++m) {
      const int wd = ndp->mode_width[m];
      const int v = rem & ((1 << wd) - 1);
      rem >>= wd;
      offA += v * ndp->strideA[m];
      offB += v * ndp->strideB[m];
      offO += v * ndp->strideO[m];
    }
  };
  // 16 x 16 output tiles (rows: four legs of A only, columns: four legs of
  // B only).  FP32 matrix cores, 16x16x4 products: lane (r = l % 16,
  // g = l / 16) feeds A[row r][k] and B[k][column r] for k = 4 kc + g; the
  // real and imaginary parts take four products per four contracted values
  // (Re += Re A Re B - Im A Im B, Im += Im A Re B + Re A Im B); the lane
  // then holds rows 4 g .. + 3 of column r.
  const int r = lane & 15, g = lane >> 4;
  const int rowA = nt[r], colB = nt[32 + r], colO = nt[48 + r];
  int rowO[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) rowO[j] = nt[16 + 4 * g + j];
  for (int t = 0; t < np; ++t) {
    int tA, tB, tO;
    tile_offsets(t, tA, tB, tO);
    T cr[4], ci[4];
    if constexpr (sizeof(T) == 4) {
      f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
      for (int kc = 0; kc < nk; kc += 4) {
        const int kk = kc + g;
        V a{0, 0}, b{0, 0};
        if (kk < nk) {
          a = A[tA + rowA + kt[2 * kk]];
          b = B[tB + colB + kt[2 * kk + 1]];
        }
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, c0, 0, 0, 0);
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, b.y, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.x, c1, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.y, c1, 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cr[j] = c0[j];
        ci[j] = c1[j];
      }
    } else {
      // (FP64 plans do not use this form; plain sums keep the path total)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cr[j] = ci[j] = 0;
        const int ra = nt[4 * g + j];
        for (int k = 0; k < nk; ++k) {
          const V a = A[tA + ra + kt[2 * k]], b = B[tB + colB + kt[2 * k + 1]];
          cr[j] += a.x * b.x - a.y * b.y;
          ci[j] += a.x * b.y + a.y * b.x;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      V o;
      o.x = cr[j] * sc;
      o.y = ci[j] * sc;
      O[tO + rowO[j] + colO] = o;
      lmax = fmax(lmax, fmax(fabs(o.x), fabs(o.y)));
    }
  }
  return lmax;
}

template <typename T>
__device__ void run_node_wave(const NodeDesc *__restrict__ ndp, typename Cplx<T>::type *arena,
                              const int32_t *__restrict__ ktab, WaveLds &w, int lane) {
  using V = typename Cplx<T>::type;
  const int kind = ndp->kind;
  const int out_bits = ndp->out_bits, k_bits = ndp->k_bits, nmodes = ndp->nmodes;
  const int p_bits = ndp->p_bits, n_bits = ndp->n_bits;
  const int ea = ndp->exp_a, eb = ndp->exp_b, eo = ndp->exp_out;
  const V *A = arena + ndp->a_off;
  const V *B = arena + ndp->b_off;
  V *O = arena + ndp->out_off;
  const int32_t *kt = ktab + ndp->ktab_off;
  const int32_t *nt = ktab + ndp->ntab_off;
  const int mA = ea >= 0 ? w.M[ea] : 0, mB = eb >= 0 ? w.M[eb] : 0;
  const int EA = ea >= 0 ? w.E[ea] : 0, EB = eb >= 0 ? w.E[eb] : 0;
  const T sc = ldexp((T)1, -(mA + mB));
  const int np = 1 << p_bits;
  const int nk = 1 << k_bits;
  constexpr int kUnroll = 5;   // output fields kept in scalar registers
  int mw[kUnroll], sa[kUnroll], sb[kUnroll], so[kUnroll];
#pragma unroll
  for (int m = 0; m < kUnroll; ++m) {
    mw[m] = m < nmodes ? ndp->mode_width[m] : 0;
    sa[m] = m < nmodes ? ndp->strideA[m] : 0;
    sb[m] = m < nmodes ? ndp->strideB[m] : 0;
    so[m] = m < nmodes ? ndp->strideO[m] : 0;
  }
  T lmax = 0;
  // offsets of output row p (lane part) into A, B and the output
  auto row_offsets = [&](int p, int &offA, int &offB, int &offO) {
    int rem = p;
    offA = offB = offO = 0;
#pragma unroll
    for (int m = 0; m < kUnroll; ++m) {
      if (m < nmodes) {
        const int v = rem & ((1 << mw[m]) - 1);
        rem >>= mw[m];
        offA += v * sa[m];
        offB += v * sb[m];
        offO += v * so[m];
      }
    }
    for (int m = kUnroll; m < nmodes; ++m) {
      const int wd = ndp->mode_width[m];
      const int v = rem & ((1 << wd) - 1);
      rem >>= wd;
      offA += v * ndp->strideA[m];
      offB += v * ndp->strideB[m];
      offO += v * ndp->strideO[m];
    }
  };
  if (kind == NODE_MFMA) {
    lmax = node_mfma<T>(ndp, A, B, O, kt, nt, sc, lane);
  } else if (kind == NODE_BLOCKED && k_bits <= 1 && n_bits <= 1) {
    // short rows (at most two contracted values and two outputs per row):
    // R rows per lane at a time, every load issued before the first product
    constexpr int R = PWS_NODE_ROWS;
    const int nn = 1 << n_bits;
    for (int p0 = lane; p0 < np; p0 += 64 * R) {
      int oA[R], oB[R], oO[R];
      V a[R][2], b[R][2][2];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        oA[r] = oB[r] = oO[r] = 0;
        if (p0 + 64 * r < np) row_offsets(p0 + 64 * r, oA[r], oB[r], oO[r]);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (p0 + 64 * r >= np) continue;
#pragma unroll
        for (int k = 0; k < 2; ++k)
          if (k < nk) a[r][k] = A[oA[r] + kt[2 * k]];
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
          for (int k = 0; k < 2; ++k)
            if (n < nn && k < nk) b[r][n][k] = B[oB[r] + nt[2 * n] + kt[2 * k + 1]];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (p0 + 64 * r >= np) continue;
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          if (n >= nn) continue;
          T ar = 0, ai = 0;
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            if (k < nk) {
              ar += a[r][k].x * b[r][n][k].x - a[r][k].y * b[r][n][k].y;
              ai += a[r][k].x * b[r][n][k].y + a[r][k].y * b[r][n][k].x;
            }
          }
          V o;
          o.x = ar * sc;
          o.y = ai * sc;
          O[oO[r] + nt[2 * n + 1]] = o;
          lmax = fmax(lmax, fmax(fabs(o.x), fabs(o.y)));
        }
      }
    }
  } else if (kind == NODE_BLOCKED) {
    const int nn = 1 << n_bits;
    for (int p = lane; p < np; p += 64) {
      int offA = 0, offB = 0, offO = 0, rem = p;
#pragma unroll
      for (int m = 0; m < kUnroll; ++m) {
        if (m < nmodes) {
          const int v = rem & ((1 << mw[m]) - 1);
          rem >>= mw[m];
          offA += v * sa[m];
          offB += v * sb[m];
          offO += v * so[m];
        }
      }
      for (int m = kUnroll; m < nmodes; ++m) {
        const int wd = ndp->mode_width[m];
        const int v = rem & ((1 << wd) - 1);
        rem >>= wd;
        offA += v * ndp->strideA[m];
        offB += v * ndp->strideB[m];
        offO += v * ndp->strideO[m];
      }
      V arow[1 << PWS_BLOCK_KBITS];
#pragma unroll
      for (int k = 0; k < (1 << PWS_BLOCK_KBITS); ++k)
        if (k < nk) arow[k] = A[offA + kt[2 * k]];
#pragma unroll 2
      for (int n = 0; n < nn; ++n) {
        const int bn = offB + nt[2 * n];
        T ar = 0, ai = 0;
#pragma unroll
        for (int k = 0; k < (1 << PWS_BLOCK_KBITS); ++k) {
          if (k < nk) {
            const V b = B[bn + kt[2 * k + 1]];
            ar += arow[k].x * b.x - arow[k].y * b.y;
            ai += arow[k].x * b.y + arow[k].y * b.x;
          }
        }
        V r;
        r.x = ar * sc;
        r.y = ai * sc;
        O[offO + nt[2 * n + 1]] = r;
        lmax = fmax(lmax, fmax(fabs(r.x), fabs(r.y)));
      }
    }
  } else if (np < 64 && nk >= 64) {
    // few outputs, long contraction: lanes split K, then a wave sum
    for (int p = 0; p < np; ++p) {
      int offA = 0, offB = 0, rem = p;
      for (int m = 0; m < nmodes; ++m) {
        const int wd = ndp->mode_width[m];
        const int v = rem & ((1 << wd) - 1);
        rem >>= wd;
        offA += v * ndp->strideA[m];
        offB += v * ndp->strideB[m];
      }
      double ar = 0, ai = 0;
#pragma unroll 4
      for (int k = lane; k < nk; k += 64) {
        const V a = A[offA + kt[2 * k]];
        const V b = B[offB + kt[2 * k + 1]];
        ar += (double)(a.x * b.x - a.y * b.y);
        ai += (double)(a.x * b.y + a.y * b.x);
      }
      ar = wave_sum(ar);
      ai = wave_sum(ai);
      V r;
      r.x = (T)ar * sc;
      r.y = (T)ai * sc;
      if (lane == 0) O[p] = r;
      lmax = fmax(lmax, fmax(fabs(r.x), fabs(r.y)));
    }
  } else {
    for (int o = lane; o < np; o += 64) {
      int offA = 0, offB = 0, rem = o;
#pragma unroll
      for (int m = 0; m < kUnroll; ++m) {
        if (m < nmodes) {
          const int v = rem & ((1 << mw[m]) - 1);
          rem >>= mw[m];
          offA += v * sa[m];
          offB += v * sb[m];
        }
      }
      for (int m = kUnroll; m < nmodes; ++m) {
        const int wd = ndp->mode_width[m];
        const int v = rem & ((1 << wd) - 1);
        rem >>= wd;
        offA += v * ndp->strideA[m];
        offB += v * ndp->strideB[m];
      }
      T ar = 0, ai = 0;
      // several independent loads in flight per lane
#pragma unroll 8
      for (int k = 0; k < nk; ++k) {
        const V a = A[offA + kt[2 * k]];
        const V b = B[offB + kt[2 * k + 1]];
        ar += a.x * b.x - a.y * b.y;
        ai += a.x * b.y + a.y * b.x;
      }
      V r;
      r.x = ar * sc;
      r.y = ai * sc;
      O[o] = r;
      lmax = fmax(lmax, fmax(fabs(r.x), fabs(r.y)));
    }
  }
  (void)out_bits;
  const T gmax = wave_max<T>(lmax);
  const int mo = gmax > 0 ? ilogb(gmax) + 1 : 0;
  if (lane == 0) {
    w.E[eo] = EA + EB + mA + mB;
    w.M[eo] = mo;
  }
  wave_sync();
}

// Leaves of the step's network for the wave's chain: lane l builds leaves
// l, l + 64, ...
template <typename T>
__device__ void materialise_leaves_wave(const DevProg &p, const ChainState &st, const StepDesc &sd,
                                        int64_t c, int slice, const uint64_t *s_sh,
                                        typename Cplx<T>::type *arena, int lane) {
  using V = typename Cplx<T>::type;
  for (int li = lane; li < sd.n_leaves; li += 64) {
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
  wave_sync();
}

// Leaves of a step for one chain, element-parallel: (leaf, element) pairs are
// spread over the threads.  Tabulated leaves are one lookup (variant index
// from the chain's bits) times the per-chain noise factors.
// Value of element e of one leaf for one chain: a table lookup (variant
// index from the chain's bits) times the per-chain noise factors, or the
// product of the leaf's factors.
__device__ inline cplxd leaf_value(const DevProg &p, const ChainState &st, const LeafDesc &ld, int64_t c,
                                   int e, int slice, const uint64_t *s_sh) {
  cplxd v{1.0, 0.0};
  if (ld.tab_off >= 0) {
    int var = 0;
    for (int k = 0; k < ld.nvar; ++k) {
      const int32_t code = p.lvar[ld.var_begin + k];
      const int t = code >> 24, pl = code & 0xffffff;
      int b;
      if (t == VAR_CHAIN) b = getbit(s_sh, pl);
      else if (t == VAR_SLICE) b = (slice >> pl) & 1;
      else b = (st.gframe[(size_t)c * p.n_gates + (pl >> 2)] >> (pl & 3)) & 1;   // recorded frame bit
      var |= b << k;
    }
    const double *t = p.ltab + 2 * ((size_t)ld.tab_off + ((size_t)var << ld.nfree) + e);
    v = cplxd{t[0], t[1]};
    for (int fi = 0; fi < ld.r_count; ++fi)
      v = cmul(v, factor_value(p, st, c, p.factors[ld.r_begin + fi], e, slice, s_sh, false));
  } else {
    for (int fi = 0; fi < ld.f_count; ++fi)
      v = cmul(v, factor_value(p, st, c, p.factors[ld.f_begin + fi], e, slice, s_sh, false));
  }
  return v;
}

// Leaves of a step for one chain, element-parallel: (leaf, element) pairs are
// spread over the threads.
template <typename T>
__device__ void leaf_elems(const DevProg &p, const ChainState &st, const StepDesc &sd, int64_t c, int slice,
                           const uint64_t *s_sh, typename Cplx<T>::type *arena, int tid, int nth) {
  using V = typename Cplx<T>::type;
  for (int i = tid; i < sd.n_elems; i += nth) {
    const int li = p.lelem[2 * (sd.elem_begin + i)];
    const int e = p.lelem[2 * (sd.elem_begin + i) + 1];
    const LeafDesc &ld = p.leaves[sd.leaf_begin + li];
    const cplxd v = leaf_value(p, st, ld, c, e, slice, s_sh);
    V r;
    r.x = (T)v.re;
    r.y = (T)v.im;
    arena[ld.out_off + e] = r;
  }
}

// Product of a step's fixed-leg factors for one chain in FP64, kept as
// mantissa * 2^exp (folded into the amplitude outputs; draws ignore it).
__device__ inline void apply_scalars(const DevProg &p, const ChainState &st, const StepDesc &sd, int64_t c,
                                     const uint64_t *s_sh, double *acc, int m, int *exp2) {
  cplxd v{1.0, 0.0};
  int e = 0;
  for (int i = 0; i < sd.scal_count; ++i) {
    v = cmul(v, factor_value(p, st, c, p.factors[sd.scal_begin + i], 0, 0, s_sh, false));
    const double mx = fmax(fabs(v.re), fabs(v.im));
    if (mx > 0 && (mx < 0x1p-300 || mx > 0x1p300)) {
      const int k = ilogb(mx);
      v.re = ldexp(v.re, -k);
      v.im = ldexp(v.im, -k);
      e += k;
    }
  }
  for (int u = 0; u < m; ++u) {
    const cplxd r = cmul(cplxd{acc[2 * u], acc[2 * u + 1]}, v);
    acc[2 * u] = r.re;
    acc[2 * u + 1] = r.im;
  }
  *exp2 += e;
}

// Replay ops [op_begin, op_end) for one chain (one lane).
__device__ bool replay_ops(const DevProg &p, const ChainState &st, int64_t c, uint64_t chain_gid,
                           uint64_t seed, int op_begin, int op_end, uint64_t *s_sh, uint64_t *x_sh) {
  bool ok = true;
  for (int op = op_begin; op < op_end; ++op) {
    const OpDesc od = p.ops[op];
    if (od.type == 0) {
      const GateDev &g = p.gates[od.idx];
      if (!p.noisy && (g.diagonal || !g.monomial)) continue;   // nothing to replay
      const int q0 = g.q0, q1 = g.q1;
      int f = 0, loc = 0;
      for (int j = 0; j < g.nq; ++j) {
        f = 2 * f + getbit(x_sh, (j ? q1 : q0));
        loc = 2 * loc + getbit(s_sh, (j ? q1 : q0));
      }
      if (p.noisy) st.gframe[(size_t)c * p.n_gates + od.idx] = (uint8_t)f;
      if (g.monomial && !g.diagonal) {
        const int nl = g.sigma[loc ^ f] ^ f;
        for (int j = 0; j < g.nq; ++j) setbit(s_sh, j ? q1 : q0, (nl >> (g.nq - 1 - j)) & 1);
      }
    } else {
      const NoiseDev nd = p.noise[od.idx];
      const int q0 = nd.q0, q1 = nd.q1;
      const int t0 = getbit(s_sh, q0) ^ getbit(x_sh, q0);
      const int t1 = nd.nq > 1 ? (getbit(s_sh, q1) ^ getbit(x_sh, q1)) : 0;
      // Eq. (4): Pr(i) = prod_j |column t_j of M_ij|^2; same draw rule as the
      // candidates (two passes: total, then inclusive prefix).
      // the prefix sums of the weights come from the host (summed in branch
      // order, no fused multiply-add: the same values as summing here)
      int br = -1;
      {
        const double *cum = p.ncum + nd.cum_off + (t0 | (t1 << 1)) * (nd.nbranch + 1);
        const double P = cum[nd.nbranch - 1];
        if (P > 0.0) {
          const double target = uniform53((uint64_t)op, chain_gid, seed) * P;
          for (int i = 0; i < nd.nbranch && br < 0; ++i)
            if (target < cum[i]) br = i;
          if (br < 0) br = (int)cum[nd.nbranch];   // rounding: the last branch with weight
        }
      }
      if (br < 0) { ok = false; continue; }
      for (int j = 0; j < nd.nq; ++j) {
        const NoiseBranch nb = p.ntab[nd.tab_off + br * nd.nq + j];
        if (nb.anti) setbit(x_sh, (j ? q1 : q0), getbit(x_sh, (j ? q1 : q0)) ^ 1);
        cplxd d0{nb.d0re, nb.d0im}, d1{nb.d1re, nb.d1im};
        if (getbit(x_sh, (j ? q1 : q0))) { cplxd tmp = d0; d0 = d1; d1 = tmp; }
        double *sf = st.segfac + ((size_t)c * p.n_segs + nd.seg[j]) * 4;
        const cplxd a0 = cmul(cplxd{sf[0], sf[1]}, d0), a1 = cmul(cplxd{sf[2], sf[3]}, d1);
        sf[0] = a0.re; sf[1] = a0.im; sf[2] = a1.re; sf[3] = a1.im;
      }
    }
  }
  return ok;
}

// Scalar-load view of read-only device records (the constant address space).
typedef const __attribute__((address_space(4))) int32_t *ConstIntPtr;

// A step's hot fields (the first 128 bytes of its record) by scalar loads.
__device__ inline StepHot fetch_hot(const StepDesc *sdp) {
  const ConstIntPtr q = (ConstIntPtr)(uintptr_t)sdp;
  StepHot h;
  int32_t *d = reinterpret_cast<int32_t *>(&h);
#pragma unroll
  for (int i = 0; i < kHotInts; ++i) d[i] = q[i];
  return h;
}

// Per-chain prologue of a step (lanes of one wave): load the chain's state,
// replay the ops since the previous step, and decide whether the step's
// block has more than one candidate (ctl[0] run, ctl[1] candidate mask,
// ctl[2] forced-zero amplitude).
// h: the step's hot fields (fetch_hot), sd: its record (rarely read fields).
__device__ inline void chain_prologue(const DevProg &p, const ChainState &st, const StepLaunch &L,
                                      const StepDesc &sd, const StepHot &h, int64_t c, uint64_t chain_gid,
                                      uint64_t seed, const WaveLds &w, int lane, int m, bool has_work,
                                      bool load_state = true) {
  const int W = p.words;
  if (load_state && lane < W) {
    w.s[lane] = st.s[(size_t)c * W + lane];
    w.x[lane] = p.noisy ? st.x[(size_t)c * W + lane] : 0ull;
  }
  wave_sync();
  if (lane == 0) {
    bool ok = true;
    if (L.mode == MODE_SAMPLE && (h.flags & 2)) {
      const int op_end = h.op >= 0 ? h.op : p.n_ops;
      ok = replay_ops(p, st, c, chain_gid, seed, h.op_begin, op_end, w.s, w.x);
    }
    int run = has_work ? 1 : 0, mask = m - 1, zero = 0;
    if (h.gate >= 0) {
      const int q0 = h.g_q0, q1 = h.g_q1, gnq = h.g_nq, gnS = h.g_nS;
      int f = 0, loc = 0;
      for (int j = 0; j < gnq; ++j) {
        f = 2 * f + getbit(w.x, (j ? q1 : q0));
        loc = 2 * loc + getbit(w.s, (j ? q1 : q0));
      }
      if (p.noisy && L.mode == MODE_SAMPLE) st.gframe[(size_t)c * p.n_gates + h.gate] = (uint8_t)f;
      if (L.mode == MODE_SAMPLE) {
        int fS = 0;
        for (int k = 0; k < gnS; ++k) fS = 2 * fS + ((f >> (gnq - 1 - ((h.g_sq >> (8 * k)) & 0xff))) & 1);
        const int raw = (h.g_cand >> (8 * (loc ^ f))) & 0xff;
        mask = 0;
        for (int v = 0; v < (1 << gnS); ++v)
          if ((raw >> (v ^ fS)) & 1) mask |= 1 << v;
        if (__popc(mask) <= 1) run = 0;   // block of size one: s stays
      }
    }
    // an untouched qubit set to 1 zeroes the amplitude (amplitude calls; a
    // sampling pass never sets one: only gates on a qubit change its bit)
    if (L.mode != MODE_SAMPLE)
      for (int i = 0; i < sd.zero_q_count; ++i)
        if (getbit(w.s, p.zero_q[sd.zero_q_begin + i])) zero = 1;
    if (zero) run = 0;
    if (!ok) atomicOr(L.err, 2);
    w.ctl[0] = run;
    w.ctl[1] = mask;
    w.ctl[2] = zero;
  }
  wave_sync();
}

// Per-chain epilogue: draw the next state from the candidate amplitudes in
// acc (MODE_SAMPLE) or write them out with their exponent ctl[3]
// (MODE_AMPS), then store the chain's state.
__device__ inline void chain_epilogue(const DevProg &p, const ChainState &st, const StepLaunch &L,
                                      const StepDesc &sd, const StepHot &h, int64_t c, uint64_t chain_gid,
                                      uint64_t seed, const WaveLds &w, int lane, int m, int run,
                                      bool store_state = true, const double *u_pre = nullptr) {
  const int W = p.words;
  if (lane == 0) {
    if (L.mode == MODE_SAMPLE) {
      if (run && h.gate >= 0) {
        const int mask = w.ctl[1];
        auto pw = [&](int v) {
          return (v < m && ((mask >> v) & 1)) ? norm2_exact(w.acc[2 * v], w.acc[2 * v + 1]) : 0.0;
        };
        // the step's uniform (computed ahead by the caller, or here)
        const double u = u_pre ? *u_pre : uniform53((uint64_t)h.op, chain_gid, seed);
        const int vs = draw4(pw(0), pw(1), pw(2), pw(3), m, u);
        if (vs < 0) {
          atomicOr(L.err, 1);
        } else {
          const int q0 = h.g_q0, q1 = h.g_q1, gnS = h.g_nS;
          for (int k = 0; k < gnS; ++k)
            setbit(w.s, (((h.g_sq >> (8 * k)) & 0xff) ? q1 : q0), (vs >> (gnS - 1 - k)) & 1);
        }
        if (L.trace) L.trace[(size_t)L.trace_row * L.n_chains + c] = (uint8_t)(vs < 0 ? 255 : vs);
      } else if (L.trace && h.gate >= 0) {
        L.trace[(size_t)L.trace_row * L.n_chains + c] = 254;
      }
    }
    // amplitude outputs: every chain of an amplitude call, or a sampling
    // pass's probe step (after its draw, which ignores the step's fixed-leg
    // factor; that factor reads no candidate qubit, so the drawn bits do
    // not change it)
    if (L.mode != MODE_SAMPLE || (L.out_amp && L.step == L.probe_step)) {
      const bool z = !run || w.ctl[2];
      if (!z) apply_scalars(p, st, sd, c, w.s, w.acc, m, &w.ctl[3]);
      for (int v = 0; v < m; ++v) {
        L.out_amp[((size_t)c * m + v) * 2] = z ? 0.0 : w.acc[2 * v];
        L.out_amp[((size_t)c * m + v) * 2 + 1] = z ? 0.0 : w.acc[2 * v + 1];
      }
      L.out_log2[c] = z ? 0 : w.ctl[3];
    }
  }
  wave_sync();
  if (store_state && L.mode == MODE_SAMPLE && lane < W) {
    st.s[(size_t)c * W + lane] = w.s[lane];
    if (p.noisy) st.x[(size_t)c * W + lane] = w.x[lane];
  }
  wave_sync();
}

template <typename T>
__global__ __launch_bounds__(kBlock) void step_kernel(DevProg p, ChainState st, StepLaunch L) {
  using V = typename Cplx<T>::type;
  extern __shared__ unsigned char lds_raw[];
  const StepDesc &sd = p.steps[L.step];
  const StepHot hot = fetch_hot(p.steps + L.step);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  const int64_t gw = (int64_t)blockIdx.x * wpb + wave, TW = (int64_t)gridDim.x * wpb;
  WaveLds w = wave_lds(lds_raw, wave, sd.n_exp_slots);
  V *arena = reinterpret_cast<V *>(L.arena) + gw * L.arena_stride;
  const int m = 1 << sd.nS;
  const uint64_t seed = L.seed_ptr ? *L.seed_ptr : L.seed;
  for (int64_t c = gw; c < L.n_chains; c += TW) {
    const uint64_t chain_gid = (uint64_t)(L.chain_offset + c);
    chain_prologue(p, st, L, sd, hot, c, chain_gid, seed, w, lane, m, sd.n_nodes > 0);
    const int run = w.ctl[0];
    if (run) {
      const int nsl = 1 << sd.n_slice_bits;
      for (int sl = 0; sl < nsl; ++sl) {
        leaf_elems<T>(p, st, sd, c, sl, w.s, arena, lane, 64);
        wave_sync();
        for (int i = 0; i < sd.n_nodes; ++i) run_node_wave<T>(p.nodes + sd.node_begin + i, arena, p.ktab, w, lane);
        if (lane == 0) {
          const int er = sd.root_exp >= 0 ? w.E[sd.root_exp] : 0;
          if (sl == 0) {
            w.ctl[3] = er;
            for (int v = 0; v < m; ++v) {
              const V r = arena[sd.root_off + sd.root_index[v]];
              w.acc[2 * v] = (double)r.x;
              w.acc[2 * v + 1] = (double)r.y;
            }
          } else {
            int ea = w.ctl[3];
            if (er > ea) {
              for (int v = 0; v < 2 * m; ++v) w.acc[v] = ldexp(w.acc[v], ea - er);
              ea = er;
              w.ctl[3] = ea;
            }
            for (int v = 0; v < m; ++v) {
              const V r = arena[sd.root_off + sd.root_index[v]];
              w.acc[2 * v] += ldexp((double)r.x, er - ea);
              w.acc[2 * v + 1] += ldexp((double)r.y, er - ea);
            }
          }
        }
        wave_sync();
      }
    }
    chain_epilogue(p, st, L, sd, hot, c, chain_gid, seed, w, lane, m, run);
  }
}

// ---------------------------------------------------------------- sweep form
// One wavefront per chain; the step's running tensor (2^sw_width elements),
// the leaf values and the current op's matrix live in the wave's LDS.  Each
// op updates the tensor in place, group by group (every group is read and
// written by one lane), so consecutive ops only need a wave-level fence.
// An op's descriptor is read once into wave-uniform registers.

__host__ __device__ inline int sweep_lds_head() { return (wave_lds_bytes(1) + 15) / 16 * 16; }

// The eight words of a SweepOp, wave-uniform.
struct SwOp {
  int moff, hi, log_rounds, log_tg, mask01, mask23, np, diag, renorm, pos, outer_mask, shifts;
  __device__ int posj(int j) const { return (pos >> (8 * j)) & 0xff; }
};

// Op records are read through the constant address space: the address is
// uniform, so they arrive in scalar registers by scalar loads.

struct RawOp {
  int w[8];
};

__device__ inline RawOp fetch_op(const SweepOpDev *rec) {
  const ConstIntPtr q = (ConstIntPtr)(uintptr_t)rec;
  RawOp r;
#pragma unroll
  for (int i = 0; i < 8; ++i) r.w[i] = q[i];
  return r;
}

__device__ inline SwOp decode_op(const RawOp &r) {
  SwOp o;
  o.moff = r.w[0];
  o.hi = r.w[1] & 0xffff;
  o.log_rounds = (r.w[1] >> 16) & 0xff;
  o.log_tg = (r.w[1] >> 24) & 0xff;
  o.mask01 = r.w[2];
  o.mask23 = r.w[3];
  o.np = r.w[4] & 0xff;
  o.diag = (r.w[4] >> 8) & 0xff;
  o.renorm = (r.w[4] >> 16) & 0xff;
  o.pos = r.w[5];
  o.outer_mask = r.w[6];
  o.shifts = r.w[7];
  return o;
}

// Apply one op with NP group positions to the workgroup's groups; returns
// the thread's largest written component when `track` (renormalisation).
// Group index g = tid + nth * r: the thread part is deposited into the
// lowest log2(nth) outer positions once, the uniform part r steps through
// the subsets of the remaining outer positions.
// KIND: 0 dense, 1 diagonal, 2 block-diagonal (two positions, bit 1 kept).
// Every free position's 1-half of the tensor holds zeros (the tensor is
// zero-filled before a step and an op's structurally zero rows write zeros
// when it closes a leg), so whole groups are read and written without masks.
// TRACK: return the thread's largest written component (renormalisation).
template <typename T, int NP, int KIND, bool TRACK>
__device__ inline T sweep_apply(const SwOp &so, typename Cplx<T>::type *ten,
                                const typename Cplx<T>::type *Mb, int pend, int tid, int log_nth) {
  using V = typename Cplx<T>::type;
  constexpr int n = 1 << NP;
  constexpr bool DIAG = KIND == 1;
  constexpr bool BLK = KIND == 2;
  static_assert(!BLK || NP == 2, "block-diagonal ops have two positions");
  constexpr bool kRegM = NP <= 2;
  int off[n];
#pragma unroll
  for (int x = 0; x < n; ++x) {
    int o = 0;
#pragma unroll
    for (int j = 0; j < NP; ++j) o |= ((x >> j) & 1) << so.posj(j);
    off[x] = o;
  }
  V Mr[kRegM ? (DIAG ? n : n * n) : 1];
  if constexpr (kRegM) {
#pragma unroll
    for (int k = 0; k < (DIAG ? n : n * n); ++k) {
      if (BLK && (((k / n) ^ (k % n)) & 2)) continue;   // structural zero
      Mr[k] = Mb[k];
    }
    if (pend != 0) {   // uniform: only the op after a renormalisation
      const T scale = ldexp((T)1, -pend);
#pragma unroll
      for (int k = 0; k < (DIAG ? n : n * n); ++k) {
        Mr[k].x *= scale;
        Mr[k].y *= scale;
      }
    }
  }
  // the thread's part of its groups' addresses: the lowest log_nth outer
  // positions take the thread bits (terms worked out on the host)
  int dep_tid = 0;
  const int nterm = (so.shifts >> 20) & 7;
  if (so.shifts & (1 << 23)) {
    int m = so.outer_mask;
    for (int b = 0; b < log_nth && m; ++b) {
      const int bit = m & -m;
      if ((tid >> b) & 1) dep_tid |= bit;
      m &= m - 1;
    }
  } else {
#pragma unroll
    for (int j = 0; j < PWS_SWDEV_TERMS; ++j) {
      if (j >= nterm) break;
      const int mask = ((j < 2 ? so.mask01 : so.mask23) >> (16 * (j & 1))) & 0xffff;
      dep_tid |= (tid << ((so.shifts >> (5 * j)) & 31)) & mask;
    }
  }
  const int hi = so.hi;
  const int tgroups = 1 << so.log_tg;
  const int rounds = 1 << so.log_rounds;
  T mx = 0;
  if (tid >= tgroups) return mx;
  // one group: load, multiply by the op's matrix, store (each accumulator
  // starts from its first product: adding to a zero costs an instruction)
  auto group = [&](int base, V (&in)[n], bool load) {
    if (load) {
#pragma unroll
      for (int i = 0; i < n; ++i) in[i] = ten[base + off[i]];
      return;
    }
#pragma unroll
    for (int o = 0; o < n; ++o) {
      V acc;
      // complex products as chains of fused multiply-adds (two per component)
      if constexpr (DIAG) {
        const V mm = kRegM ? Mr[o] : Mb[o];
        acc.x = fma(-mm.y, in[o].y, mm.x * in[o].x);
        acc.y = fma(mm.y, in[o].x, mm.x * in[o].y);
      } else {
        bool first = true;
#pragma unroll
        for (int i = 0; i < n; ++i) {
          if (BLK && ((o ^ i) & 2)) continue;   // kept bit: block-diagonal
          const V mm = kRegM ? Mr[o * n + i] : Mb[o * n + i];
          if (first) {
            acc.x = mm.x * in[i].x;
            acc.y = mm.x * in[i].y;
            first = false;
          } else {
            acc.x = fma(mm.x, in[i].x, acc.x);
            acc.y = fma(mm.x, in[i].y, acc.y);
          }
          acc.x = fma(-mm.y, in[i].y, acc.x);
          acc.y = fma(mm.y, in[i].x, acc.y);
        }
      }
      if constexpr (!kRegM) {
        if (pend != 0) {
          const T scale = ldexp((T)1, -pend);
          acc.x *= scale;
          acc.y *= scale;
        }
      }
      ten[base + off[o]] = acc;
      if constexpr (TRACK) mx = fmax(mx, fmax(fabs(acc.x), fabs(acc.y)));
    }
  };
  int dep_hi = 0;   // subsets of `hi` in increasing order
  int r = 0;
  // two groups per iteration: the second group's loads overlap the first's work
  // (ops on three or four positions keep one group: their registers)
  for (; NP <= 2 && r + 1 < rounds; r += 2) {
    const int b0 = dep_tid | dep_hi;
    dep_hi = (dep_hi - hi) & hi;
    const int b1 = dep_tid | dep_hi;
    dep_hi = (dep_hi - hi) & hi;
    V in0[n], in1[n];
    group(b0, in0, true);
    group(b1, in1, true);
    group(b0, in0, false);
    group(b1, in1, false);
  }
  for (; r < rounds; ++r) {
    const int b0 = dep_tid | dep_hi;
    dep_hi = (dep_hi - hi) & hi;
    V in0[n];
    group(b0, in0, true);
    group(b0, in0, false);
  }
  return mx;
}

// One op, dispatched on its shape (np, kind) and on whether it renormalises.
template <typename T, int MAXNP, bool TRACK>
__device__ inline T sweep_op(const SwOp &cur, typename Cplx<T>::type *ten, const typename Cplx<T>::type *Mop,
                             int pend, int tid, int log_nth) {
  switch (cur.np) {
    case 0: return sweep_apply<T, 0, 1, TRACK>(cur, ten, Mop, pend, tid, log_nth);
    case 1:
      return cur.diag ? sweep_apply<T, 1, 1, TRACK>(cur, ten, Mop, pend, tid, log_nth)
                      : sweep_apply<T, 1, 0, TRACK>(cur, ten, Mop, pend, tid, log_nth);
    case 2:
      return cur.diag == 1 ? sweep_apply<T, 2, 1, TRACK>(cur, ten, Mop, pend, tid, log_nth)
           : cur.diag == 2 ? sweep_apply<T, 2, 2, TRACK>(cur, ten, Mop, pend, tid, log_nth)
                           : sweep_apply<T, 2, 0, TRACK>(cur, ten, Mop, pend, tid, log_nth);
    default:
      if constexpr (MAXNP > 2) {
        if (cur.np == 3)
          return cur.diag ? sweep_apply<T, 3, 1, TRACK>(cur, ten, Mop, pend, tid, log_nth)
                          : sweep_apply<T, 3, 0, TRACK>(cur, ten, Mop, pend, tid, log_nth);
        return cur.diag ? sweep_apply<T, 4, 1, TRACK>(cur, ten, Mop, pend, tid, log_nth)
                        : sweep_apply<T, 4, 0, TRACK>(cur, ten, Mop, pend, tid, log_nth);
      } else {
        return (T)0;
      }
  }
}

// Sync of the threads that share one chain: a wave-level fence for one
// wave, a workgroup barrier for several.
template <int WPC>
__device__ inline void chain_sync() {
  if constexpr (WPC == 1) wave_sync();
  else __syncthreads();
}

// Largest ilogb over the threads of one chain when several chains share a
// wave (CPW of them, 64 / CPW lanes each): DPP max within rows of 16 lanes,
// then across the two rows of a 32-lane chain.  INT_MIN when all are zero.
template <typename T, int CPW>
__device__ inline int chain_max_ilogb(T v) {
  if constexpr (CPW == 1) {
    return wave_max_ilogb(v);
  } else {
    unsigned u;
    if constexpr (sizeof(T) == 8) u = (unsigned)((unsigned long long)__double_as_longlong(v) >> 32);
    else u = __float_as_uint(v);
    u = dpp_umax<0xB1>(u);
    u = dpp_umax<0x4E>(u);
    u = dpp_umax<0x141>(u);
    u = dpp_umax<0x140>(u);
    if constexpr (CPW == 2) u = max(u, (unsigned)__builtin_amdgcn_ds_swizzle((int)u, 0x401f));   // lane ^ 16
    return hiword_ilogb<T>(u);
  }
}

// ---------------------------------------------------------------- dense runs

// Deposit the low bits of x into the set bits of mask, lowest first.
__device__ inline int deposit(int x, int mask) {
  int r = 0;
  for (int m = mask; m && x; m &= m - 1, x >>= 1)
    if (x & 1) r |= m & -m;
  return r;
}

// Tensor offset of row (or column) v of a run: bit b of v at the position
// in nibble b of nib.
__device__ inline int nib_row(int v, int nib) {
  return (((v >> 0) & 1) << (nib & 15)) | (((v >> 1) & 1) << ((nib >> 4) & 15)) |
         (((v >> 2) & 1) << ((nib >> 8) & 15)) | (((v >> 3) & 1) << ((nib >> 12) & 15));
}

// x = hi + lo with hi, lo bf16 (round to nearest even each; x - hi is exact
// in FP32); |x - hi - lo| <= 2^-16 |x|, so products of such pairs carry about
// 16 bits.  Both parts of a complex value at once: hi and lo as packed bf16
// pairs (real part in the low half), one conversion instruction each.
typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
__device__ inline void split_bf16_pair(float2 x, uint32_t &hi, uint32_t &lo) {
  hi = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2v){x.x, x.y}, bf16x2v));
  const float hr = __uint_as_float(hi << 16), hm = __uint_as_float(hi & 0xffff0000u);
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2v){x.x - hr, x.y - hm}, bf16x2v));
}

// One dense run on one chain: T <- (F (x) I) T over the run's four row
// positions, F = the run's table for the chain's bits, the columns (the
// other live positions) taken 16 at a time.  A 16-column tile is the real
// product of the embedding of F (32 x 32) with the tile's real and imaginary
// parts (32 x 16): two 16 x 16 output tiles (real and imaginary rows), K = 32.
//   DN = 1: FP32 matrix-core products (16x16x4, eight per output tile), K
//           = (real parts of rows 0..15, then their imaginary parts);
//   DN = 2: bf16 hi/lo split of both operands (F's split made on the host
//           from its double value), three products per output tile (lo*hi,
//           hi*lo, hi*hi, accumulated in FP32 in that order), K interleaved
//           as (Re, Im) of row 0, of row 1, ...: lane group g = l / 16 holds
//           K 8 g .. 8 g + 7, i.e. rows 4 g .. 4 g + 3, which are also the
//           output rows it writes, so a lane reads four complex values and
//           writes back the same four cells.  The real output rows take the
//           pairs (Re F, -Im F), the imaginary ones (Im F, Re F): the table
//           holds the former, the latter is a half swap and a sign flip.
// Lane l owns output column l % 16 and rows 4 (l / 16) .. + 3 of each tile;
// the A operand row is l % 16.  Lanes past the run's column count (fewer
// than four outer positions) repeat a column: they read the same values and
// write the same results again.  dense_variant_bits gathers the chains'
// variant bits, dense_read / dense_stage fetch a chain's F (one-wave chains
// stage the next run's tables in LDS while the current run computes),
// dense_apply multiplies,
// scales the outputs by 2^-pe (a pending renormalisation) and, when TRACK,
// returns the lane's largest written component.
template <int DN> struct DenseA;
template <> struct DenseA<2> { u32x4 hi, lo; };    // the pairs (Re F, -Im F) of 4 columns, hi and lo
template <> struct DenseA<1> { float2 e[4]; };     // 4 entries: FP32 (re, im)

// Variant bits of a run for every chain of the wave: lane b of each chain's
// 64 / CPW lanes reads the chain bit of the run's variant qubit b; chain
// ch's bits sit at bit ch * 64 / CPW of the ballot.
template <int CPW>
__device__ inline uint64_t dense_variant_bits(const RawOp &rr, unsigned char *lds_raw, int slot_bytes, int lane) {
  constexpr int kL = 64 / CPW;
  const int nq = (rr.w[3] >> 8) & 0xff;
  const int ch = CPW == 1 ? 0 : lane / kL, b = lane % kL;
  int bit = 0;
  if (b < nq) bit = getbit(wave_lds(lds_raw + ch * slot_bytes, 0, 1).s, dense_qubit(rr.w[4], rr.w[5], rr.w[7], b));
  return __builtin_amdgcn_ballot_w64(bit != 0);
}

// Waits for the wave's vector memory operations (the staged tables' direct
// loads to LDS included) / its LDS and scalar memory operations, as waits
// the compiler's own wait placement sees, and as compiler memory barriers.
__device__ inline void wait_vm0() {
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), expcnt and lgkmcnt unbounded
  asm volatile("" ::: "memory");
}
__device__ inline void wait_lgkm0() {
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0), vmcnt and expcnt unbounded
  asm volatile("" ::: "memory");
}

// The lane's operand registers of F (one variant's table, in device memory
// or staged in LDS; see the table layout in the run builder).
template <int DN>
__device__ inline void dense_read(const uint32_t *F, int lane, DenseA<DN> &A) {
  const int g = lane >> 4, cl = lane & 15;
  if constexpr (DN == 2) {
    // row cl, columns 4 g .. 4 g + 3: the lane's 16 bytes of each part
    const u32x4 *fr = reinterpret_cast<const u32x4 *>(F) + lane;
    A.hi = fr[0];
    A.lo = fr[64];
  } else {
    // row cl, columns g, 4 + g, 8 + g, 12 + g (chunk c: column 4 c + g)
    const float2 *fr = reinterpret_cast<const float2 *>(F) + 16 * g + cl;
#pragma unroll
    for (int i = 0; i < 4; ++i) A.e[i] = fr[64 * i];
  }
}

// The workgroup's LDS table buffers (512 words per chain), an array of
// their own: the compiler then knows that the direct loads into them do not
// touch the chains' tensors, and does not wait for them before tensor writes.
template <int N>
__device__ inline uint32_t *dense_tab_lds() {
  __shared__ __attribute__((aligned(16))) uint32_t buf[N];
  return buf;
}

// Starts copying each chain's variant of run rr's table into the chain's
// LDS table buffer (tabs + 512 ch): two 1 KB direct loads to LDS per chain,
// 16 bytes per lane, with no registers held.  The caller waits for them
// (vmcnt) before reading a buffer, and reads a buffer's previous contents
// into registers (lgkmcnt) before restaging it.
template <int CPW>
__device__ inline void dense_stage(const RawOp &rr, const uint32_t *dtab, unsigned char *lds_raw, int slot_bytes,
                                   uint32_t *tabs, int lane) {
  const uint64_t vb = dense_variant_bits<CPW>(rr, lds_raw, slot_bytes, lane);
  const int vmask = (1 << ((rr.w[3] >> 8) & 0xff)) - 1;
#pragma unroll
  for (int ch = 0; ch < CPW; ++ch) {
    const int vi = (int)(vb >> (ch * (64 / CPW))) & vmask;
    const uint32_t *F = dtab + (size_t)(rr.w[0] + vi) * 512 + lane * 4;
    uint32_t *dst = tabs + ch * 512;
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)F,
                                     (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(F + 256),
                                     (__attribute__((address_space(3))) void *)(dst + 256), 16, 0, 0);
  }
}

template <int DN, int WPC, bool TRACK, bool SCALED>
__device__ inline float dense_apply(const RawOp &rr, const DenseA<DN> &A, float2 *__restrict__ ten, int pe, int lane,
                                    int wave) {
  const int pos = rr.w[1], hi_mask = rr.w[2], info = rr.w[3];
  const int n_outer = info & 0xff;
  const int g = lane >> 4, cl = lane & 15;
  // columns: the lane's (the lowest four outer positions), then the tile's
  // (the remaining ones, a subset walk)
  const int ncl = n_outer < 4 ? 1 << n_outer : 16;
  const int dep_lane = nib_row(cl & (ncl - 1), pos >> 16);
  const int ntiles = n_outer > 4 ? 1 << (n_outer - 4) : 1;
  int woff[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) woff[j] = nib_row(4 * g + j, pos);
  float mx = 0.f;
  auto store = [&](int base, const f32x4 &c0, const f32x4 &c1) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      // (an exact power-of-two scaling, where one is pending)
      const float2 y = SCALED ? float2{ldexpf(c0[j], -pe), ldexpf(c1[j], -pe)} : float2{c0[j], c1[j]};
      ten[base | woff[j]] = y;
      if constexpr (TRACK) mx = fmaxf(mx, fmaxf(fabsf(y.x), fabsf(y.y)));
    }
  };
  if constexpr (DN == 2) {
    // (Im F, Re F) from (Re F, -Im F): swap the halves, flip the new low sign
    u32x4 ih, il;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ih[q] = ((A.hi[q] >> 16) | (A.hi[q] << 16)) ^ 0x8000u;
      il[q] = ((A.lo[q] >> 16) | (A.lo[q] << 16)) ^ 0x8000u;
    }
    const bf16x8 a0h = __builtin_bit_cast(bf16x8, A.hi), a0l = __builtin_bit_cast(bf16x8, A.lo);
    const bf16x8 a1h = __builtin_bit_cast(bf16x8, ih), a1l = __builtin_bit_cast(bf16x8, il);
    int dt = deposit(wave, hi_mask);
    for (int t = wave; t < ntiles; t += WPC) {
      const int base = dep_lane | dt;
      float2 x[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) x[j] = ten[base | woff[j]];
      u32x4 bhw, blw;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        uint32_t h, l;
        split_bf16_pair(x[j], h, l);
        bhw[j] = h;
        blw[j] = l;
      }
      const bf16x8 bh = __builtin_bit_cast(bf16x8, bhw), bl = __builtin_bit_cast(bf16x8, blw);
      f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
      c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0l, bh, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1l, bh, c1, 0, 0, 0);
      c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0h, bl, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1h, bl, c1, 0, 0, 0);
      c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0h, bh, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1h, bh, c1, 0, 0, 0);
      store(base, c0, c1);
#pragma unroll
      for (int s = 0; s < WPC; ++s) dt = (dt - hi_mask) & hi_mask;
    }
  } else {
    const float are[4] = {A.e[0].x, A.e[1].x, A.e[2].x, A.e[3].x};
    const float aim[4] = {A.e[0].y, A.e[1].y, A.e[2].y, A.e[3].y};
    int roff[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) roff[m] = nib_row(4 * m + g, pos);
    int dt = deposit(wave, hi_mask);
    for (int t = wave; t < ntiles; t += WPC) {
      const int base = dep_lane | dt;
      float2 x[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) x[m] = ten[base | roff[m]];
      f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < 4; ++c) {   // K rows 0..15: real parts of the inputs
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(are[c], x[c].x, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(aim[c], x[c].x, c1, 0, 0, 0);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {   // K rows 16..31: imaginary parts
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(-aim[c], x[c].y, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(are[c], x[c].y, c1, 0, 0, 0);
      }
      store(base, c0, c1);
#pragma unroll
      for (int s = 0; s < WPC; ++s) dt = (dt - hi_mask) & hi_mask;
    }
  }
  return mx;
}

// Copies n elements of a chain's LDS tensor to device memory, the chain's
// NTH threads in turn, B reads in flight before their stores.  The
// restrict-qualified operands tell the compiler that the reads do not touch
// the staged tables, so it does not wait for their direct loads first.
// (Measured: B = 4 pays where a wave holds several chains or stages tables;
// one-chain op-by-op launches, as in noisy plans, run faster with B = 1.)
template <int NTH, int B, typename V>
__device__ inline void copy_out(const V *__restrict__ src, V *__restrict__ dst, int n, int ct) {
  int i = ct;
  if constexpr (B > 1) {
    for (; i + (B - 1) * NTH < n; i += B * NTH) {
      V a[B];
#pragma unroll
      for (int u = 0; u < B; ++u) a[u] = src[i + u * NTH];
#pragma unroll
      for (int u = 0; u < B; ++u) dst[i + u * NTH] = a[u];
    }
  }
  for (; i < n; i += NTH) dst[i] = src[i];
}

// Fills a chain's LDS tensor with zeros at [i0, n) (the chain's NTH threads
// in turn from i0 + ct), and copies a kept tensor from device memory into it
// with B loads in flight per thread before their LDS writes.  As in
// copy_out, the restrict-qualified operands tell the compiler that these LDS
// writes do not touch the tables that direct loads may be staging, so it
// does not wait for those first.
template <int NTH, typename V>
__device__ inline void fill_zero(V *__restrict__ dst, int i0, int n) {
  for (int i = i0; i < n; i += NTH) dst[i] = V{0, 0};
}
template <int NTH, int B, typename V>
__device__ inline void copy_in(const V *__restrict__ src, V *__restrict__ dst, int n, int ct) {
  int i = ct;
  for (; i + (B - 1) * NTH < n; i += B * NTH) {
    V a[B];
#pragma unroll
    for (int u = 0; u < B; ++u) a[u] = src[i + u * NTH];
#pragma unroll
    for (int u = 0; u < B; ++u) dst[i + u * NTH] = a[u];
  }
  for (; i < n; i += NTH) dst[i] = src[i];
}
template <typename V>
__device__ inline void set_one(V *__restrict__ dst) { dst[0] = V{1, 0}; }

// MAXNP: the widest op of the step (the 3- and 4-position variants need far
// more registers, so steps without them run a leaner instantiation).
// WPC: waves that share one chain (wide tensors split their groups over
// several waves so that more of them are in flight per compute unit).
// CPW: chains that share one wave (narrow tensors: 64 / CPW lanes per chain,
// so that the work common to a wave, such as reading and decoding each op,
// serves several chains).  Each chain has an LDS slot of L.slot_bytes: its
// head (state bits, controls), its running tensor (2^range_w elements) and
// its op matrices.
// A launch runs the steps [L.step, L.step_end) for each of its chains in
// turn (a range of narrow consecutive steps, or a single step): the chain's
// state stays in LDS between the steps of a range.
// MG: the op matrices are built in device memory (L.mt_global) instead of LDS.
// FP32 kernels with several chains per wave, and four-wave dense-run chains,
// keep to 128 registers (four resident waves per SIMD): these launches are
// bound by latency.
template <typename T, int MAXNP, int WPC, bool MG, int CPW, int DN>
__global__ __launch_bounds__(64 * WPC)
__attribute__((amdgpu_waves_per_eu((CPW > 1 || (DN > 0 && WPC == 4)) && sizeof(T) == 4 ? 4 : 1)))
void step_kernel_sweep(DevProg p, ChainState st, StepLaunch L) {
  static_assert(CPW == 1 || (WPC == 1 && !MG), "several chains per wave: one wave, matrices in LDS");
  static_assert(DN == 0 || ((CPW == 1 || WPC == 1) && !MG && sizeof(T) == 4),
                "dense runs: FP32 tensors, matrices from the tables, several chains only in one-wave launches");
  using V = typename Cplx<T>::type;
  extern __shared__ unsigned char lds_raw[];
  // (one-wave launches know the wave index at compile time)
  const int tid = threadIdx.x, lane = tid & 63, wave = WPC == 1 ? 0 : tid >> 6;
  constexpr int kNth = 64 * WPC / CPW;   // threads per chain
  constexpr int kLogNth = kNth == 16 ? 4 : kNth == 32 ? 5 : kNth == 64 ? 6 : kNth == 256 ? 8 : 9;
  const int slot = CPW == 1 ? 0 : lane >> kLogNth;
  const int ct = CPW == 1 ? tid : lane & (kNth - 1);   // thread index within the chain
  unsigned char *sb = lds_raw + slot * L.slot_bytes;
  WaveLds w = wave_lds(sb, 0, 1);
  V *ten = reinterpret_cast<V *>(sb + sweep_lds_head());
  T *red = reinterpret_cast<T *>(lds_raw + CPW * L.slot_bytes);   // waves' partial results
  // a pointer of one address space per instantiation: LDS tables are read
  // with LDS instructions
  V *Mt = MG ? reinterpret_cast<V *>(L.mt_global) + (int64_t)blockIdx.x * L.mt_stride
             : ten + (1 << L.range_w);
  V *cache = reinterpret_cast<V *>(L.cache);
  const uint64_t seed = L.seed_ptr ? *L.seed_ptr : L.seed;
  // op records for this number of threads per chain
  const SweepOpDev *recs_all =
      p.swdev + (kLogNth == 6 ? 0 : kLogNth == 8 ? 1 : kLogNth == 9 ? 2 : kLogNth == 4 ? 3 : 4) * (size_t)p.n_sweep_ops;
  // range launches: the draws' uniforms kU steps at a time, thread t < kU of
  // each chain (in wave 0) writing the uniform of the batch's step t to the
  // chain's row of the workgroup's uniforms (single steps draw their own)
  constexpr int kU = kNth < 64 ? kNth : 64;
  // (ranges are one-wave launches; the wider instantiations keep without)
  double *u_arr = nullptr;
  if constexpr (WPC == 1)
    if (L.u_off >= 0) u_arr = reinterpret_cast<double *>(lds_raw + L.u_off) + slot * kU;
  // dense runs in one-wave chains: the staged tables' buffers
  [[maybe_unused]] uint32_t *dn_tabs = nullptr;
  if constexpr (DN > 0 && WPC == 1) dn_tabs = dense_tab_lds<CPW * 512>();
  for (int64_t cb = (int64_t)blockIdx.x * CPW; cb < L.n_chains; cb += (int64_t)gridDim.x * CPW) {
    const int64_t c = cb + slot;
    const bool active = c < L.n_chains;   // the last group of chains may be short
    const uint64_t chain_gid = (uint64_t)(L.chain_offset + c);
    for (int step = L.step; step < L.step_end; ++step) {
      const int j_step = step - L.step;
      if (u_arr && L.mode == MODE_SAMPLE && j_step % kU == 0 && wave == 0 && active && step + ct < L.step_end) {
        const int op_t = p.steps[step + ct].op;
        u_arr[ct] = op_t >= 0 ? uniform53((uint64_t)op_t, chain_gid, seed) : 0.0;
      }
      // the step's descriptor, read once per step (the compiler cannot keep
      // device-memory fields across the kernel's own stores)
      // (all of them at once by scalar loads: the compiler cannot keep
      // device-memory fields across the kernel's own stores)
      const StepDesc *sdp = p.steps + step;
      const StepDesc &sd = *sdp;
      const StepHot h = fetch_hot(sdp);
      const int sw_count = h.sw_count;
      const int sw_width = DN > 0 ? h.dn_w : h.sw_width;
      const int m_count = h.m_count;
      const int m_begin = h.m_begin;
      const int leaf_begin = h.leaf_begin;
      const int nS = h.nS;
      const SweepOpDev *recs = recs_all + h.sw_begin;
      const int32_t *mcodes = p.mtab + m_begin;
      const int m = 1 << nS;
      // the previous step's tensor is restored / this step's is kept for the next
      const bool restore = L.mode == MODE_SAMPLE && L.cache && h.load_op >= 0;
      const bool keep = L.mode == MODE_SAMPLE && L.cache && h.store_op >= 0;
      const int load_op = restore ? h.load_op : 0;
      const int store_op = keep ? h.store_op : -1;
      const int load_n = restore ? 1 << h.load_w : 0;
      const int store_n = keep ? 1 << h.store_w : 0;
      // anchor steps keep snapshots for later steps; two-sided steps contract with one
      const bool cached = L.mode == MODE_SAMPLE && L.cache;
      const int snap_count = cached ? h.snap_count : 0;
      const SnapDesc *snaps = p.snaps + h.snap_begin;
      const int merge_slot = cached ? h.merge_slot : -1;
      const int last_snap = snap_count > 0 ? snaps[snap_count - 1].op : -1;
      StepLaunch Ls = L;
      Ls.step = step;
      Ls.trace_row = L.trace_row + (step - L.step);
      if (wave == 0 && active)
        chain_prologue(p, st, Ls, sd, h, c, chain_gid, seed, w, ct, m, sw_count > 0, step == L.step);
      chain_sync<WPC>();
      const int run = active ? w.ctl[0] : 0;
      // the op sequence is common to the chains of a wave: it runs as far as
      // the furthest of them needs (a chain whose step has nothing to draw
      // still builds the kept prefix; extra ops on a chain are harmless)
      const bool run_any = CPW == 1 ? run != 0 : __builtin_amdgcn_ballot_w64(run != 0) != 0;
      if (L.mode == MODE_SAMPLE && (h.flags & 1)) {
        // a one-qubit gate on an untouched qubit: the candidates' amplitudes
        // are column 0 of the gate times a factor common to all of them
        // (the step record holds that column, next to the hot fields)
        if (run && ct == 0) {
          typedef const __attribute__((address_space(4))) double *ConstDblPtr;
          const ConstDblPtr g0 = (ConstDblPtr)(uintptr_t)sdp->hot.fresh_amp;
          w.ctl[3] = 0;
          for (int v = 0; v < m && v < 2; ++v) {
            w.acc[2 * v] = g0[2 * v];
            w.acc[2 * v + 1] = g0[2 * v + 1];
          }
        }
        chain_sync<WPC>();
      } else if (run_any || keep || snap_count > 0) {
        const int op0 = load_op;
        const int op1 = run_any ? sw_count : max(store_op, last_snap);
        const int m0 = DN > 0 ? 0 : op0 < sw_count ? fetch_op(recs + op0).w[0] : m_count;
        const int m1 = DN > 0 ? 0 : op1 < sw_count ? fetch_op(recs + op1).w[0] : m_count;
        RawOp nxt{};   // the next op's record, loaded one op ahead (decoded when used)
        if (DN == 0 && op0 < op1) nxt = fetch_op(recs + op0);
        // the ops' matrices for this chain, entry-parallel: each entry is its
        // folded constant times its chain-dependent terms (or, for entries
        // with noise records, frame or slice bits, a product of leaf
        // elements summed over their internal legs).  Entries [c0, c1) are
        // built at a time (at most cap of them: the LDS slot holds a window
        // of the step's table, rebuilt from an op's first entry when that
        // op's matrix lies beyond it).
        const MEntry *ment = p.ment + m_begin / PWS_MTERMS;
        const int cap = MG || L.mt_cap <= 0 ? INT_MAX : L.mt_cap;
        int c0 = m0, c1 = MG ? m1 : m0;   // LDS windows are built inside the op loop
        // Entries made of leaf-table elements times noise records, from flat
        // records: the n entries of a round advance factor by factor together,
        // so that their record, frame-bit, table and noise-record loads are
        // in flight at the same time.
        auto flat_entries = [&](const int4 *hb, cplxd *fv, auto n_tag) {
          constexpr int n = decltype(n_tag)::value;
          const int4 *mflat = reinterpret_cast<const int4 *>(p.mflat);
          int nf[n], nmax = 0;
#pragma unroll
          for (int u = 0; u < n; ++u) {
            nf[u] = hb[u].x == PWS_MENTRY_FLAT ? hb[u].w : 0;
            fv[u] = cplxd{1.0, 0.0};
            nmax = max(nmax, nf[u]);
          }
          for (int f = 0; f < nmax; ++f) {
            int4 a[n], b[n];
#pragma unroll
            for (int u = 0; u < n; ++u) {
              if (f < nf[u]) {
                a[u] = mflat[2 * (hb[u].y + f)];
                b[u] = mflat[2 * (hb[u].y + f) + 1];
              } else {
                a[u] = int4{0, 0, 0, 0};
                b[u] = int4{0, 0, 0, 0};
              }
            }
            int var[n];
#pragma unroll
            for (int u = 0; u < n; ++u) {
              const int nvar = (a[u].y >> 8) & 0xff;
              const int vc[4] = {a[u].z, a[u].w, b[u].x, b[u].y};
              int bits = 0;
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                if (k < nvar) {
                  const int pl = vc[k] & 0xffffff;
                  const int bit = (vc[k] >> 24) == VAR_CHAIN
                                      ? getbit(w.s, pl)
                                      : (st.gframe[(size_t)c * p.n_gates + (pl >> 2)] >> (pl & 3)) & 1;
                  bits |= bit << k;
                }
              }
              var[u] = bits;
            }
            double2 tv[n], sv[n][2];
#pragma unroll
            for (int u = 0; u < n; ++u) {
              tv[u] = double2{1.0, 0.0};
              if (f < nf[u]) tv[u] = reinterpret_cast<const double2 *>(p.ltab)[a[u].x + (var[u] << (a[u].y & 0xff))];
              const int nres = (a[u].y >> 16) & 0xff;
              const int refs[2] = {b[u].z, b[u].w};
#pragma unroll
              for (int r = 0; r < 2; ++r) {
                sv[u][r] = double2{1.0, 0.0};
                if (r < nres) {
                  const int mode = (refs[r] >> 28) & 3;
                  const int half = mode == 2 ? getbit(w.s, (refs[r] >> 16) & 0xfff) : mode;
                  const double2 *sf =
                      reinterpret_cast<const double2 *>(st.segfac + ((size_t)c * p.n_segs + (refs[r] & 0xffff)) * 4);
                  sv[u][r] = sf[half ? 1 : 0];
                }
              }
            }
#pragma unroll
            for (int u = 0; u < n; ++u) {
              if (f < nf[u]) {
                const int nres = (a[u].y >> 16) & 0xff;
                cplxd v{tv[u].x, tv[u].y};
#pragma unroll
                for (int r = 0; r < 2; ++r)
                  if (r < nres) v = cmul(v, cplxd{sv[u][r].x, sv[u][r].y});
                fv[u] = cmul(fv[u], v);
              }
            }
          }
        };
        // entries evaluated from their codes (frame or slice bits, wider variants)
        auto codes_entry = [&](int i) {
          cplxd val{1.0, 0.0};
#pragma unroll
          for (int t = 0; t < PWS_MTERMS; ++t) {
            const int32_t code = mcodes[PWS_MTERMS * i + t];
            if (code < 0) { val = cplxd{0.0, 0.0}; break; }
            if (code & PWS_MCODE_ONE) continue;
            const LeafDesc &ld = p.leaves[leaf_begin + (code & 0xffff)];
            const int e0 = (code >> 16) & 15, im = (code >> 20) & 15;
            cplxd acc{0.0, 0.0};
            for (int sub = im;; sub = (sub - 1) & im) {
              const cplxd v = leaf_value(p, st, ld, c, e0 | sub, 0, w.s);
              acc.re += v.re;
              acc.im += v.im;
              if (sub == 0) break;
            }
            val = cmul(val, acc);
          }
          return val;
        };
        // Each thread takes kBU entries per round with every header load, and
        // then every term load, issued before the first product.
        constexpr int kBU = 2;
        auto build = [&]() {
          for (int i0 = c0 + ct; active && i0 < c1; i0 += kBU * kNth) {
            double2 cv[kBU];
            int4 hb[kBU];
#pragma unroll
            for (int u = 0; u < kBU; ++u) {
              const int i = i0 + u * kNth;
              if (i < c1) {
                cv[u] = *reinterpret_cast<const double2 *>(ment + i);
                hb[u] = reinterpret_cast<const int4 *>(ment + i)[1];
              } else {
                cv[u] = double2{0.0, 0.0};
                hb[u] = int4{-1, 0, -1, 0};
              }
            }
            auto term = [&](int t, int pc) {
              const int nv = pc >> 24;
              int v = getbit(w.s, pc & 0xfff);
              if (nv > 1) v |= getbit(w.s, (pc >> 12) & 0xfff) << 1;
              return reinterpret_cast<const double2 *>(p.mterm)[t + v];
            };
            double2 ta[kBU], tb[kBU];
#pragma unroll
            for (int u = 0; u < kBU; ++u) {
              const bool plain = hb[u].x != PWS_MENTRY_FLAT && hb[u].x != PWS_MENTRY_CODES;
              ta[u] = plain && hb[u].x >= 0 ? term(hb[u].x, hb[u].y) : double2{1.0, 0.0};
              tb[u] = plain && hb[u].z >= 0 ? term(hb[u].z, hb[u].w) : double2{1.0, 0.0};
            }
            // flat entries advance together kFL at a time (one at a time where
            // several chains share a wave, whose kernels keep to 128 VGPRs)
            constexpr int kFL = CPW == 1 ? kBU : 1;
            cplxd fv[kBU];
#pragma unroll
            for (int u0 = 0; u0 < kBU; u0 += kFL) {
              bool any_flat = false;
#pragma unroll
              for (int u = u0; u < u0 + kFL; ++u) any_flat |= hb[u].x == PWS_MENTRY_FLAT;
              if (any_flat) flat_entries(hb + u0, fv + u0, std::integral_constant<int, kFL>{});
            }
#pragma unroll
            for (int u = 0; u < kBU; ++u) {
              const int i = i0 + u * kNth;
              if (i >= c1) break;
              cplxd val{cv[u].x, cv[u].y};
              if (hb[u].x == PWS_MENTRY_FLAT) {
                val = fv[u];
              } else if (hb[u].x == PWS_MENTRY_CODES) {
                val = codes_entry(i);
              } else {
                if (hb[u].x >= 0) val = cmul(val, cplxd{ta[u].x, ta[u].y});
                if (hb[u].z >= 0) val = cmul(val, cplxd{tb[u].x, tb[u].y});
              }
              Mt[i - c0] = V{(T)val.re, (T)val.im};
            }
          }
        };
        if constexpr (MG) build();
        // dense runs: the first run's record, and its tables staged in LDS
        // (one-wave chains) while the tensor is cleared and restored below
        [[maybe_unused]] int dn_count = 0, dn_r0 = 0;
        [[maybe_unused]] const DenseRun *runs = nullptr;
        [[maybe_unused]] RawOp dn_first{};
        if constexpr (DN > 0) {
          runs = p.druns + h.dn_begin;
          dn_count = h.dn_count;
          dn_r0 = restore ? h.dn_load : 0;
          if (dn_r0 < dn_count) {
            dn_first = fetch_op(reinterpret_cast<const SweepOpDev *>(runs + dn_r0));
            if constexpr (WPC == 1)
              if (dn_first.w[6] < op1) dense_stage<CPW>(dn_first, p.dtab, lds_raw, L.slot_bytes, dn_tabs, lane);
          }
        }
        // slot s of this chain's kept tensors (slot 0: the next step's prefix)
        auto slot_of = [&](int sl) { return cache + ((int64_t)c * L.cache_slots + sl) * L.cache_stride; };
        auto exps_of = [&](int sl) { return L.cache_exp + ((int64_t)c * L.cache_slots + sl) * 2; };
        // two-sided steps with a packed leg map: thread ct < 2^nb takes the
        // shared legs' value b = ct, whose cells are positions m_it here and
        // m_ir in the kept tensor (an earlier step's); dense-run kernels load
        // that cell here, with the restore, the others when they use it
        const int m_nb = merge_slot >= 0 ? h.merge_nb : 0;
        const bool m_fast = DN > 0 && merge_slot >= 0 && h.merge_pack != -1 && (1 << m_nb) <= kNth;
        int m_it = 0, m_ir = 0, m_eR = 0, m_pR = 0;
        V m_r{0, 0};
        auto merge_cells = [&]() {
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            if (kk >= m_nb) break;
            const int bit = (ct >> kk) & 1, pk = h.merge_pack >> (8 * kk);
            m_it |= bit << (pk & 15);
            m_ir |= bit << ((pk >> 4) & 15);
          }
          if (ct < (1 << m_nb)) m_r = slot_of(merge_slot)[m_ir];
          m_eR = exps_of(merge_slot)[0];
          m_pR = exps_of(merge_slot)[1];
        };
        if constexpr (DN > 0)
          if (m_fast && run) merge_cells();
        // the kept prefix's exponents first (their loads then travel with
        // the tensor's), free positions cleared (they hold zeros from the
        // start, see sweep_apply), the prefix restored
        int expo = 0, pend = 0;
        if (restore && active) {
          expo = exps_of(0)[0];
          pend = exps_of(0)[1];
        }
        fill_zero<kNth>(ten, ct + (restore ? load_n : 1), 1 << sw_width);
        // (eight loads per thread: a 2^8-element prefix over two chains' 32
        // lanes each in one round; the other kernels keep their registers)
        constexpr int kRestoreBatch = (DN > 0 && kNth == 32) ? 8 : 4;
        if (restore && active) copy_in<kNth, kRestoreBatch>(slot_of(0), ten, load_n, ct);
        else if (ct == 0) set_one(ten);
        // (dense runs: the restored exponents and the first run's staged
        // tables are in, so nothing in flight reaches the run loop)
        if constexpr (DN > 0) wait_vm0();
        chain_sync<WPC>();
        auto keep_tensor = [&](int sl, int n) {
          if (!active) return;
          copy_out<kNth, (DN > 0 || CPW > 1 ? 4 : 1)>(ten, slot_of(sl), n, ct);
          if (ct == 0) {
            exps_of(sl)[0] = expo;
            exps_of(sl)[1] = pend;
          }
        };
        int si = 0;   // next snapshot
        auto snapshots_at = [&](int k) {
          while (si < snap_count && snaps[si].op == k) {
            keep_tensor(snaps[si].slot, 1 << snaps[si].w);
            ++si;
            chain_sync<WPC>();
          }
        };
        // the next op before which a tensor is kept (one compare per op)
        int ev = INT_MAX;
        auto next_event = [&](int from) {
          ev = store_op >= from ? store_op : INT_MAX;
          if (si < snap_count) ev = min(ev, snaps[si].op);
        };
        next_event(op0);
        if constexpr (DN > 0) {
          // dense runs: one F matrix per run applied to the tensor's 16-row
          // tiles on the matrix cores (runs start at the kept-tensor and
          // snapshot points, so those events fall between runs)
          int r = dn_r0;
          RawOp rn = dn_first;
          for (; r < dn_count; ++r) {
            const RawOp rr = rn;
            const int k = rr.w[6];
            if (k >= op1) break;
            if (r + 1 < dn_count) rn = fetch_op(reinterpret_cast<const SweepOpDev *>(runs + r + 1));
            // the wave's chains one after another, all 64 lanes on each
            // (their tables' loads issued first)
            DenseA<DN> A[CPW];
            if constexpr (WPC == 1) {
              // this run's tables were staged in LDS during the previous run
              // (or the step's set-up); the next run's follow behind them
              wait_vm0();
#pragma unroll
              for (int ch = 0; ch < CPW; ++ch)
                dense_read<DN>(dn_tabs + ch * 512, lane, A[ch]);
              wait_lgkm0();
              if (r + 1 < dn_count && rn.w[6] < op1) dense_stage<CPW>(rn, p.dtab, lds_raw, L.slot_bytes, dn_tabs, lane);
            } else {
              const uint64_t vb = dense_variant_bits<CPW>(rr, lds_raw, L.slot_bytes, lane);
              const int vmask = (1 << ((rr.w[3] >> 8) & 0xff)) - 1;
#pragma unroll
              for (int ch = 0; ch < CPW; ++ch)
                dense_read<DN>(p.dtab + (size_t)(rr.w[0] + ((int)(vb >> (ch * (64 / CPW))) & vmask)) * 512, lane, A[ch]);
            }
            // tensors kept before this run (after the staging above, so that
            // their stores drain while the run computes)
            if (k == ev) {   // the previous run ended with a barrier
              if (k == store_op) {
                keep_tensor(0, store_n);
                chain_sync<WPC>();
              }
              snapshots_at(k);
              next_event(k + 1);
            }
            const int pe = pend;   // each lane: its chain's pending renormalisation
            expo += pend;
            pend = 0;
            const bool track = ((rr.w[3] >> 16) & 1) != 0;
#pragma unroll
            for (int ch = 0; ch < CPW; ++ch) {
              V *tch = reinterpret_cast<V *>(lds_raw + ch * L.slot_bytes + sweep_lds_head());
              const int pe_ch = CPW == 1 ? pe : __builtin_amdgcn_readlane(pe, ch * (64 / CPW));
              const T mx = track      ? (pe_ch != 0 ? dense_apply<DN, WPC, true, true>(rr, A[ch], tch, pe_ch, lane, wave)
                                                     : dense_apply<DN, WPC, true, false>(rr, A[ch], tch, pe_ch, lane, wave))
                           : pe_ch != 0 ? dense_apply<DN, WPC, false, true>(rr, A[ch], tch, pe_ch, lane, wave)
                                        : dense_apply<DN, WPC, false, false>(rr, A[ch], tch, pe_ch, lane, wave);
              if (track) {
                int e = chain_max_ilogb<T, 1>(mx);
                if constexpr (WPC > 1) {
                  int *ired = reinterpret_cast<int *>(red);
                  if (lane == 0) ired[wave] = e;
                  chain_sync<WPC>();
                  e = ired[0];
#pragma unroll
                  for (int q = 1; q < WPC; ++q) e = max(e, ired[q]);
                }
                if (e != INT_MIN && slot == ch) pend = e;
              }
            }
            chain_sync<WPC>();
          }
        } else
        for (int k = op0; k < op1; ++k) {
          if (k == ev) {   // the previous op ended with a barrier
            if (k == store_op) {
              keep_tensor(0, store_n);
              chain_sync<WPC>();
            }
            snapshots_at(k);
            next_event(k + 1);
          }
          const SwOp cur = decode_op(nxt);
          if (k + 1 < op1) nxt = fetch_op(recs + k + 1);
          if (!MG && cur.moff + (cur.diag == 1 ? 1 << cur.np : 1 << (2 * cur.np)) > c1) {
            // the op's matrix lies beyond the window: build the window from
            // there (the previous op, or the set-up, ended with a barrier)
            c0 = cur.moff;
            c1 = min(m1, c0 + cap);
            build();
            chain_sync<WPC>();
          }
          const int pe = pend;   // pending renormalisation, folded into this op
          expo += pend;
          pend = 0;
          const V *Mop = Mt + (cur.moff - c0);
          const bool track = cur.renorm != 0;
          T mx = track ? sweep_op<T, MAXNP, true>(cur, ten, Mop, pe, ct, kLogNth)
                       : sweep_op<T, MAXNP, false>(cur, ten, Mop, pe, ct, kLogNth);
          if (track) {
            int e = chain_max_ilogb<T, CPW>(mx);
            if constexpr (WPC > 1) {
              int *ired = reinterpret_cast<int *>(red);
              if (lane == 0) ired[wave] = e;
              chain_sync<WPC>();
              e = ired[0];
#pragma unroll
              for (int q = 1; q < WPC; ++q) e = max(e, ired[q]);
            }
            if (e != INT_MIN) pend = e;
          }
          chain_sync<WPC>();
        }
        if (op1 == store_op) {
          keep_tensor(0, store_n);
          chain_sync<WPC>();
        }
        snapshots_at(op1);
        if (merge_slot >= 0) {
          // two-sided step: candidate v = sum over the shared legs' values b of
          // this tensor at (b, v) times the kept tensor at b
          const int nb = m_nb;
          double ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
          int eR = m_eR, pR = m_pR;
          if (m_fast) {
            if constexpr (DN == 0)
              if (run) merge_cells();
            eR = m_eR;
            pR = m_pR;
            if (run && ct < (1 << nb)) {
              // (an opaque use, so that the compiler converts the early-loaded
              // cell here rather than next to its load, where the conversion
              // would wait for it and for everything issued before it)
              T rx = m_r.x, ry = m_r.y;
              asm volatile("" : "+v"(rx), "+v"(ry));
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                if (v >= m) break;
                const V t = ten[m_it | h.root_index[v]];
                ar[v] = (double)t.x * rx - (double)t.y * ry;
                ai[v] = (double)t.x * ry + (double)t.y * rx;
              }
            }
          } else if (run) {
            const ConstIntPtr mm = (ConstIntPtr)(uintptr_t)(p.mmap + h.merge_map);
            const V *Rt = slot_of(merge_slot);
            eR = exps_of(merge_slot)[0];
            pR = exps_of(merge_slot)[1];
            for (int b = ct; b < (1 << nb); b += kNth) {
              int it = 0, ir = 0;
              for (int kk = 0; kk < nb; ++kk) {
                const int bit = (b >> kk) & 1;
                it |= bit << mm[2 * kk];
                ir |= bit << mm[2 * kk + 1];
              }
              const V r = Rt[ir];
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                if (v >= m) break;
                const V t = ten[it | h.root_index[v]];
                ar[v] += (double)t.x * r.x - (double)t.y * r.y;
                ai[v] += (double)t.x * r.y + (double)t.y * r.x;
              }
            }
          }
          // sum over the chain's threads: within the wave, then across waves
          constexpr int kLanes = kNth < 64 ? kNth : 64;
          const int used = min(1 << nb, kLanes);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if (v >= m) break;
            ar[v] = chain_sum_f64<kLanes>(ar[v], used);
            ai[v] = chain_sum_f64<kLanes>(ai[v], used);
          }
          if constexpr (WPC > 1) {
            double *dred = reinterpret_cast<double *>(red);
            if (lane == 0)
              for (int v = 0; v < 4; ++v) {
                dred[(wave * 4 + v) * 2] = ar[v];
                dred[(wave * 4 + v) * 2 + 1] = ai[v];
              }
            chain_sync<WPC>();
            for (int v = 0; v < 4; ++v) {
              ar[v] = ai[v] = 0;
              for (int q = 0; q < WPC; ++q) {
                ar[v] += dred[(q * 4 + v) * 2];
                ai[v] += dred[(q * 4 + v) * 2 + 1];
              }
            }
          }
          if (run && ct == 0) {
            w.ctl[3] = expo + pend + eR + pR;
            for (int v = 0; v < m; ++v) {
              w.acc[2 * v] = ldexp(ar[v], -(pend + pR));
              w.acc[2 * v + 1] = ldexp(ai[v], -(pend + pR));
            }
          }
        } else if (run && ct == 0) {
          w.ctl[3] = expo + pend;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if (v >= m) break;
            const V r = ten[h.root_index[v]];
            w.acc[2 * v] = ldexp((double)r.x, -pend);
            w.acc[2 * v + 1] = ldexp((double)r.y, -pend);
          }
        }
        chain_sync<WPC>();
      }
      if (wave == 0 && active)
        chain_epilogue(p, st, Ls, sd, h, c, chain_gid, seed, w, ct, m, run, step + 1 == L.step_end,
                       u_arr && L.mode == MODE_SAMPLE ? u_arr + j_step % kU : nullptr);
      chain_sync<WPC>();
    }
  }
}

// ---------------------------------------------------------------- LDS-resident form
// One workgroup per chain; the chain's whole arena (leaves and intermediates
// of the step's network) lives in LDS, so every node reads and writes on-chip
// memory.  Threads of the workgroup share each node; nodes are separated by
// barriers.  Renormalisation (nodes flagged by the planner) takes the
// workgroup maximum through a 64-bit LDS atomic max on non-negative values.
template <typename T>
__device__ __attribute__((always_inline)) inline void run_node_blk(
    const NodeDesc *__restrict__ ndp, typename Cplx<T>::type *arena, const int32_t *__restrict__ ktab,
    int *E, int *M, unsigned long long *red3, int idx, int tid, int nth) {
  using V = typename Cplx<T>::type;
  const int kind = ndp->kind, k_bits = ndp->k_bits, nmodes = ndp->nmodes;
  const int p_bits = ndp->p_bits, n_bits = ndp->n_bits, renorm = ndp->renorm;
  const int ea = ndp->exp_a, eb = ndp->exp_b, eo = ndp->exp_out;
  const V *A = arena + ndp->a_off;
  const V *B = arena + ndp->b_off;
  V *O = arena + ndp->out_off;
  const int32_t *kt = ktab + ndp->ktab_off;
  const int32_t *nt = ktab + ndp->ntab_off;
  const int mA = ea >= 0 ? M[ea] : 0, mB = eb >= 0 ? M[eb] : 0;
  const int EA = ea >= 0 ? E[ea] : 0, EB = eb >= 0 ? E[eb] : 0;
  const T sc = ldexp((T)1, -(mA + mB));
  const int np = 1 << p_bits;
  const int nk = 1 << k_bits;
  if (tid == 0) red3[(idx + 1) % 3] = 0ull;
  constexpr int kUnroll = 5;
  int mw[kUnroll], sa[kUnroll], sb[kUnroll], so[kUnroll];
#pragma unroll
  for (int m = 0; m < kUnroll; ++m) {
    mw[m] = m < nmodes ? ndp->mode_width[m] : 0;
    sa[m] = m < nmodes ? ndp->strideA[m] : 0;
    sb[m] = m < nmodes ? ndp->strideB[m] : 0;
    so[m] = m < nmodes ? ndp->strideO[m] : 0;
  }
  T lmax = 0;
  if (kind == NODE_BLOCKED) {
    const int nn = 1 << n_bits;
    for (int p = tid; p < np; p += nth) {
      int offA = 0, offB = 0, offO = 0, rem = p;
#pragma unroll
      for (int m = 0; m < kUnroll; ++m) {
        if (m < nmodes) {
          const int v = rem & ((1 << mw[m]) - 1);
          rem >>= mw[m];
          offA += v * sa[m];
          offB += v * sb[m];
          offO += v * so[m];
        }
      }
      for (int m = kUnroll; m < nmodes; ++m) {
        const int wd = ndp->mode_width[m];
        const int v = rem & ((1 << wd) - 1);
        rem >>= wd;
        offA += v * ndp->strideA[m];
        offB += v * ndp->strideB[m];
        offO += v * ndp->strideO[m];
      }
      V arow[1 << PWS_BLOCK_KBITS];
#pragma unroll
      for (int k = 0; k < (1 << PWS_BLOCK_KBITS); ++k)
        if (k < nk) arow[k] = A[offA + kt[2 * k]];
#pragma unroll 2
      for (int n = 0; n < nn; ++n) {
        const int bn = offB + nt[2 * n];
        T ar = 0, ai = 0;
#pragma unroll
        for (int k = 0; k < (1 << PWS_BLOCK_KBITS); ++k) {
          if (k < nk) {
            const V b = B[bn + kt[2 * k + 1]];
            ar += arow[k].x * b.x - arow[k].y * b.y;
            ai += arow[k].x * b.y + arow[k].y * b.x;
          }
        }
        V r;
        r.x = ar * sc;
        r.y = ai * sc;
        O[offO + nt[2 * n + 1]] = r;
        lmax = fmax(lmax, fmax(fabs(r.x), fabs(r.y)));
      }
    }
  } else {
    for (int o = tid; o < np; o += nth) {
      int offA = 0, offB = 0, rem = o;
#pragma unroll
      for (int m = 0; m < kUnroll; ++m) {
        if (m < nmodes) {
          const int v = rem & ((1 << mw[m]) - 1);
          rem >>= mw[m];
          offA += v * sa[m];
          offB += v * sb[m];
        }
      }
      for (int m = kUnroll; m < nmodes; ++m) {
        const int wd = ndp->mode_width[m];
        const int v = rem & ((1 << wd) - 1);
        rem >>= wd;
        offA += v * ndp->strideA[m];
        offB += v * ndp->strideB[m];
      }
      T ar = 0, ai = 0;
      // several independent loads in flight per lane
#pragma unroll 8
      for (int k = 0; k < nk; ++k) {
        const V a = A[offA + kt[2 * k]];
        const V b = B[offB + kt[2 * k + 1]];
        ar += a.x * b.x - a.y * b.y;
        ai += a.x * b.y + a.y * b.x;
      }
      V r;
      r.x = ar * sc;
      r.y = ai * sc;
      O[o] = r;
      lmax = fmax(lmax, fmax(fabs(r.x), fabs(r.y)));
    }
  }
  if (renorm) {
    const double wm = (double)wave_max<T>(lmax);
    if ((tid & 63) == 0) atomicMax(&red3[idx % 3], (unsigned long long)__double_as_longlong(wm));
    __syncthreads();
    const double g = __longlong_as_double((long long)red3[idx % 3]);
    if (tid == 0) {
      E[eo] = EA + EB + mA + mB;
      M[eo] = g > 0 ? ilogb(g) + 1 : 0;
    }
  } else if (tid == 0) {
    E[eo] = EA + EB + mA + mB;
    M[eo] = 0;
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(1024) void step_kernel_lds(DevProg p, ChainState st, StepLaunch L) {
  using V = typename Cplx<T>::type;
  extern __shared__ unsigned char lds_raw[];
  __shared__ uint64_t s_sh[kMaxWords], x_sh[kMaxWords];
  __shared__ double acc[8];
  __shared__ int ctl[4];
  __shared__ unsigned long long red3[3];
  const StepDesc &sd = p.steps[L.step];
  V *arena = reinterpret_cast<V *>(lds_raw);
  int *E = reinterpret_cast<int *>(arena + L.arena_stride);
  int *M = E + L.n_exp;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int W = p.words;
  const int m = 1 << sd.nS;
  const uint64_t seed = L.seed_ptr ? *L.seed_ptr : L.seed;
  for (int64_t c = blockIdx.x; c < L.n_chains; c += gridDim.x) {
    const uint64_t chain_gid = (uint64_t)(L.chain_offset + c);
    if (tid < W) {
      s_sh[tid] = st.s[(size_t)c * W + tid];
      x_sh[tid] = p.noisy ? st.x[(size_t)c * W + tid] : 0ull;
    }
    __syncthreads();
    if (tid == 0) {
      bool ok = true;
      if (L.mode == MODE_SAMPLE) {
        const int op_end = sd.op >= 0 ? sd.op : p.n_ops;
        ok = replay_ops(p, st, c, chain_gid, seed, sd.op_begin, op_end, s_sh, x_sh);
      }
      int run = sd.n_nodes > 0 ? 1 : 0, mask = m - 1, zero = 0;
      if (sd.gate >= 0) {
        const GateDev &g = p.gates[sd.gate];
        const int q0 = g.q0, q1 = g.q1;
        int f = 0, loc = 0;
        for (int j = 0; j < g.nq; ++j) {
          f = 2 * f + getbit(x_sh, j ? q1 : q0);
          loc = 2 * loc + getbit(s_sh, j ? q1 : q0);
        }
        if (p.noisy && L.mode == MODE_SAMPLE) st.gframe[(size_t)c * p.n_gates + sd.gate] = (uint8_t)f;
        if (L.mode == MODE_SAMPLE) {
          int fS = 0;
          for (int k = 0; k < g.nS; ++k) fS = 2 * fS + ((f >> (g.nq - 1 - g.sq[k])) & 1);
          const int raw = g.cand_mask[loc ^ f];
          mask = 0;
          for (int v = 0; v < (1 << g.nS); ++v)
            if ((raw >> (v ^ fS)) & 1) mask |= 1 << v;
          if (__popc(mask) <= 1) run = 0;
        }
      }
      if (L.mode != MODE_SAMPLE)   // (a sampling pass never sets an untouched qubit)
        for (int i = 0; i < sd.zero_q_count; ++i)
          if (getbit(s_sh, p.zero_q[sd.zero_q_begin + i])) zero = 1;
      if (zero) run = 0;
      if (!ok) atomicOr(L.err, 2);
      ctl[0] = run;
      ctl[1] = mask;
      ctl[2] = zero;
      red3[0] = red3[1] = red3[2] = 0ull;
    }
    __syncthreads();
    const int run = ctl[0];
    if (run) {
      const int nsl = 1 << sd.n_slice_bits;
      for (int sl = 0; sl < nsl; ++sl) {
        leaf_elems<T>(p, st, sd, c, sl, s_sh, arena, tid, nth);
        __syncthreads();
        for (int i = 0; i < sd.n_nodes; ++i)
          run_node_blk<T>(p.nodes + sd.node_begin + i, arena, p.ktab, E, M, red3, i, tid, nth);
        if (tid == 0) {
          const int er = sd.root_exp >= 0 ? E[sd.root_exp] : 0;
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
          red3[0] = red3[1] = red3[2] = 0ull;
        }
        __syncthreads();
      }
    }
    if (tid == 0) {
      if (L.mode == MODE_SAMPLE) {
        if (run && sd.gate >= 0) {
          const int mask = ctl[1];
          auto pw = [&](int v) {
            return (v < m && ((mask >> v) & 1)) ? norm2_exact(acc[2 * v], acc[2 * v + 1]) : 0.0;
          };
          const double u = uniform53((uint64_t)sd.op, chain_gid, seed);
          const int vs = draw4(pw(0), pw(1), pw(2), pw(3), m, u);
          if (vs < 0) {
            atomicOr(L.err, 1);
          } else {
            const GateDev &g = p.gates[sd.gate];
            const int q0 = g.q0, q1 = g.q1;
            for (int k = 0; k < g.nS; ++k) setbit(s_sh, g.sq[k] ? q1 : q0, (vs >> (g.nS - 1 - k)) & 1);
          }
          if (L.trace) L.trace[(size_t)L.trace_row * L.n_chains + c] = (uint8_t)(vs < 0 ? 255 : vs);
        } else if (L.trace && sd.gate >= 0) {
          L.trace[(size_t)L.trace_row * L.n_chains + c] = 254;
        }
      } else {
        const bool z = !run || ctl[2];
        if (!z) apply_scalars(p, st, sd, c, s_sh, acc, m, &ctl[3]);
        for (int v = 0; v < m; ++v) {
          L.out_amp[((size_t)c * m + v) * 2] = z ? 0.0 : acc[2 * v];
          L.out_amp[((size_t)c * m + v) * 2 + 1] = z ? 0.0 : acc[2 * v + 1];
        }
        L.out_log2[c] = z ? 0 : ctl[3];
      }
    }
    __syncthreads();
    if (L.mode == MODE_SAMPLE && tid < W) {
      st.s[(size_t)c * W + tid] = s_sh[tid];
      if (p.noisy) st.x[(size_t)c * W + tid] = x_sh[tid];
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

// Output word i (chain i / words): s XOR x, then the readout errors of its
// qubits (Section 4's simulated chip): qubit q flips when its uniform, drawn
// at op index n_ops + q, is below its readout probability.
__global__ void finalize_kernel(DevProg p, ChainState st, int64_t K, uint64_t *out, uint64_t seed,
                                const uint64_t *seed_ptr, int64_t chain_offset, int readout) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K * p.words) return;
  uint64_t v = p.noisy ? (st.s[i] ^ st.x[i]) : st.s[i];
  if (readout && p.readout) {
    const uint64_t sd = seed_ptr ? *seed_ptr : seed;
    const int64_t c = i / p.words;
    const int q0 = (int)(i % p.words) * 64;
    const int q1 = min(q0 + 64, p.n_qubits);
    for (int q = q0; q < q1; ++q) {
      const double r = p.readout[q];
      if (r > 0.0 && uniform53((uint64_t)(p.n_ops + q), (uint64_t)(chain_offset + c), sd) < r)
        v ^= 1ull << (q - q0);
    }
  }
  out[i] = v;
}

// ---------------------------------------------------------------- gradient
// Forward contraction of the full circuit with every leg projected onto the
// sample, then the reverse pass: the adjoint of each child is the contraction
// of its parent's adjoint with its sibling; each parametrised gate factor adds
// <adjoint of its leaf, d leaf / d theta> to d amp / d theta.  One wave per
// sample.
template <typename T>
__global__ __launch_bounds__(kBlock) void grad_kernel(DevProg p, ChainState st, GradLaunch L) {
  using V = typename Cplx<T>::type;
  extern __shared__ unsigned char lds_raw[];
  const StepDesc &sd = p.steps[0];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  const int64_t gw = (int64_t)blockIdx.x * wpb + wave, TW = (int64_t)gridDim.x * wpb;
  WaveLds w = wave_lds(lds_raw, wave, sd.n_exp_slots);
  V *arena = reinterpret_cast<V *>(L.arena) + gw * L.arena_stride;
  const int W = p.words;
  for (int64_t c = gw; c < L.n_chains; c += TW) {
    if (lane < W) w.s[lane] = st.s[(size_t)c * W + lane];
    wave_sync();
    materialise_leaves_wave<T>(p, st, sd, c, 0, w.s, arena, lane);
    for (int i = 0; i < sd.n_nodes; ++i) run_node_wave<T>(p.nodes + sd.node_begin + i, arena, p.ktab, w, lane);
    const V r = arena[sd.root_off];
    const int er = sd.root_exp >= 0 ? w.E[sd.root_exp] : 0;
    const double mr = (double)r.x, mi = (double)r.y;
    if (lane == 0 && p.adj_root_off >= 0) {
      V one;
      one.x = 1;
      one.y = 0;
      arena[p.adj_root_off] = one;   // adjoint of the root
    }
    wave_sync();
    for (int i = 0; i < p.n_bnodes; ++i) run_node_wave<T>(p.bnodes + i, arena, p.ktab, w, lane);
    const double den = mr * mr + mi * mi;
    for (int j = 0; j < p.n_params; ++j) {
      double part_re = 0, part_im = 0;
      for (int t = lane; t < p.n_grad_terms; t += 64) {
        const int32_t *gt = p.grad_terms + 5 * t;
        if (gt[2] != j) continue;
        const LeafDesc ld = p.leaves[sd.leaf_begin + gt[0]];
        const int ea = gt[4] >= 0 ? w.E[gt[4]] : 0;
        const int ne = 1 << ld.nfree;
        double sre = 0, sim = 0;
        for (int e = 0; e < ne; ++e) {
          cplxd v{1.0, 0.0};
          for (int fi = 0; fi < ld.f_count; ++fi)
            v = cmul(v, factor_value(p, st, c, p.factors[ld.f_begin + fi], e, 0, w.s, fi == gt[1]));
          const V a = arena[gt[3] + e];
          sre += (double)a.x * v.re - (double)a.y * v.im;
          sim += (double)a.x * v.im + (double)a.y * v.re;
        }
        part_re += ldexp(sre, ea - er);
        part_im += ldexp(sim, ea - er);
      }
      const double tre = wave_sum(part_re);
      const double tim = wave_sum(part_im);
      if (lane == 0) {
        // d log|amp|^2 = 2 Re(d amp / amp) = 2 Re(t * conj(m)) / |m|^2
        const double val = den > 0 ? 2.0 * (tre * mr + tim * mi) / den : 0.0;
        L.dtheta[(size_t)c * p.n_params + j] = val;
        if (!(den > 0)) atomicOr(L.err, 4);
      }
    }
    if (lane == 0 && L.amp) {
      L.amp[2 * c] = mr;
      L.amp[2 * c + 1] = mi;
      if (L.amp_log2) L.amp_log2[c] = er;
    }
    wave_sync();
  }
}

}  // namespace

// ---------------------------------------------------------------- static workspace
// The workspace of pws_sample_noalloc: device memory that exists from the
// moment the code object is loaded on a device (each device holds its own
// copy until the process ends), so that those calls allocate nothing.  Host
// code never passes the array's name to a kernel (on the host it names a
// stand-in, not device memory): it passes the address looked up per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

__global__ void clear_flags_kernel(int32_t *flags, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flags[i] = 0;
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int lds_bytes_for(int n_exp_slots) { return kWavesPerBlock * wave_lds_bytes(n_exp_slots); }

hipError_t scratch_region(int device, void **ptr, size_t *bytes) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  *bytes = kScratchBytes;
  return hipSuccess;
}

hipError_t launch_clear_flags(int32_t *flags, int n, hipStream_t s) {
  hipLaunchKernelGGL(clear_flags_kernel, dim3((n + 63) / 64), dim3(64), 0, s, flags, n);
  return hipGetLastError();
}

int sweep_slot_bytes(int precision, int width, int m_entries) {
  // head, tensor, the ops' matrices (16-byte aligned)
  return (sweep_lds_head() + ((1 << width) + m_entries) * (precision == 0 ? 16 : 8) + 15) / 16 * 16;
}

int lds_bytes_sweep(int precision, int width, int m_entries, int cpw) {
  // one slot per chain of the workgroup, then the waves' partial results
  // (maxima; candidate sums of up to eight waves of one chain)
  return cpw * sweep_slot_bytes(precision, width, m_entries) + (cpw == 1 ? 512 : 64);
}

int lds_bytes_arena(int precision, int arena_elems, int n_exp) {
  return arena_elems * (precision == 0 ? 16 : 8) + 2 * n_exp * 4;
}

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
  if (l.sweep) {
    auto go = [&](const void *fn, auto kern, int wpc) {
      (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, l.lds_bytes);
      hipLaunchKernelGGL(kern, dim3(l.grid), dim3(64 * wpc), l.lds_bytes, s, p, st, l);
    };
    const int v = l.sweep - 1;   // bit 0: widest op has 3 or 4 positions, bits 1-2: 4 / 8 waves per chain
    // bit 3: the op matrices live in device memory (too large for LDS);
    // bits 4-5: two / four chains per wave
#define PWS_SWEEP_GO(TT, NP, WPC, MG, CPW) \
  go((const void *)step_kernel_sweep<TT, NP, WPC, MG, CPW, 0>, step_kernel_sweep<TT, NP, WPC, MG, CPW, 0>, WPC)
#define PWS_DENSE_GO(DN, WPC, CPW) \
  go((const void *)step_kernel_sweep<float, 2, WPC, false, CPW, DN>, step_kernel_sweep<float, 2, WPC, false, CPW, DN>, WPC)
    if (l.dense) {   // dense runs: one or two chains per wave, or four / eight waves per chain
      if (precision == 0) return hipErrorInvalidValue;
      const int wpc = v & 2 ? 4 : v & 4 ? 8 : 1;
      const bool two = (v & 16) != 0;
      if (l.dense == 1) {
        if (wpc == 1) { if (two) PWS_DENSE_GO(1, 1, 2); else PWS_DENSE_GO(1, 1, 1); }
        else if (wpc == 4) PWS_DENSE_GO(1, 4, 1); else PWS_DENSE_GO(1, 8, 1);
      } else {
        if (wpc == 1) { if (two) PWS_DENSE_GO(2, 1, 2); else PWS_DENSE_GO(2, 1, 1); }
        else if (wpc == 4) PWS_DENSE_GO(2, 4, 1); else PWS_DENSE_GO(2, 8, 1);
      }
      return hipGetLastError();
    }
#define PWS_SWEEP_SWITCH(TT, MG)                        \
  switch (v & 7) {                                      \
    case 0: PWS_SWEEP_GO(TT, 2, 1, MG, 1); break;       \
    case 1: PWS_SWEEP_GO(TT, 4, 1, MG, 1); break;       \
    case 2: PWS_SWEEP_GO(TT, 2, 4, MG, 1); break;       \
    case 3: PWS_SWEEP_GO(TT, 4, 4, MG, 1); break;       \
    case 4: PWS_SWEEP_GO(TT, 2, 8, MG, 1); break;       \
    default: PWS_SWEEP_GO(TT, 4, 8, MG, 1); break;      \
  }
    if (v & 48) {   // several chains per wave: lean instantiation, one wave, matrices in LDS
      if ((v & 15) != 0) return hipErrorInvalidValue;
      if (precision == 0) {
        if (v & 16) PWS_SWEEP_GO(double, 2, 1, false, 2);
        else PWS_SWEEP_GO(double, 2, 1, false, 4);
      } else {
        if (v & 16) PWS_SWEEP_GO(float, 2, 1, false, 2);
        else PWS_SWEEP_GO(float, 2, 1, false, 4);
      }
    } else if (precision == 0) {
      if (v & 8) { PWS_SWEEP_SWITCH(double, true) } else { PWS_SWEEP_SWITCH(double, false) }
    } else {
      if (v & 8) { PWS_SWEEP_SWITCH(float, true) } else { PWS_SWEEP_SWITCH(float, false) }
    }
#undef PWS_SWEEP_SWITCH
#undef PWS_SWEEP_GO
#undef PWS_DENSE_GO
    return hipGetLastError();
  }
  if (l.lds_arena) {
    if (precision == 0) {
      (void)hipFuncSetAttribute((const void *)step_kernel_lds<double>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, l.lds_bytes);
      hipLaunchKernelGGL(step_kernel_lds<double>, dim3(l.grid), dim3(l.block), l.lds_bytes, s, p, st, l);
    } else {
      (void)hipFuncSetAttribute((const void *)step_kernel_lds<float>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, l.lds_bytes);
      hipLaunchKernelGGL(step_kernel_lds<float>, dim3(l.grid), dim3(l.block), l.lds_bytes, s, p, st, l);
    }
    return hipGetLastError();
  }
  if (precision == 0)
    hipLaunchKernelGGL(step_kernel<double>, dim3(l.grid), dim3(l.block), l.lds_bytes, s, p, st, l);
  else
    hipLaunchKernelGGL(step_kernel<float>, dim3(l.grid), dim3(l.block), l.lds_bytes, s, p, st, l);
  return hipGetLastError();
}

hipError_t launch_finalize(const DevProg &p, const ChainState &st, int64_t K, uint64_t *out,
                           hipStream_t s, uint64_t seed, const uint64_t *seed_ptr, int64_t chain_offset,
                           bool readout) {
  const int64_t n = K * (int64_t)p.words;
  const int blocks = (int)((n + 255) / 256);
  hipLaunchKernelGGL(finalize_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, s, p, st, K, out, seed, seed_ptr,
                     chain_offset, readout ? 1 : 0);
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
