// Plain-data description of the per-step work that the device kernels
// execute.  Built by the host planner, uploaded once per plan.
//
// A "step" is one non-monomial gate (Algorithm 1, UpdateState with a block
// of size > 1): its prologue replays the monomial / diagonal gates and noise
// sites since the previous step (Algorithm 2), then the prefix network's
// leaves are materialised per chain, contracted node by node, and the
// candidate amplitudes feed the transition draw.
#pragma once
#include <stdint.h>

#if !defined(__HIPCC__) && !defined(__host__)
#define __host__
#define __device__
#endif

namespace pws {

// Source of one bit of a gate-tensor index (an in or out leg of one qubit).
enum : int32_t {
  SRC_FREE = 0,   // payload = bit position in the leaf's element index
  SRC_CONST = 1,  // payload = 0/1 (input legs are fixed to |0>)
  SRC_CHAIN = 2,  // payload = qubit: the chain's classical bit s[q] (output projection)
  SRC_SLICE = 3   // payload = slice bit index (index slicing)
};
__host__ __device__ inline int32_t src_make(int32_t type, int32_t payload) { return (type << 24) | payload; }
__host__ __device__ inline int32_t src_type(int32_t s) { return (s >> 24) & 0xff; }
__host__ __device__ inline int32_t src_payload(int32_t s) { return s & 0xffffff; }

enum : int32_t { FAC_GATE = 0, FAC_GATE_DERIV = 1, FAC_SEGFAC = 2 };

struct FactorDesc {
  int32_t kind;        // FAC_*
  int32_t id;          // gate index, or segment id for FAC_SEGFAC
  int32_t nq;          // gate qubits (1 or 2); 1 for FAC_SEGFAC
  int32_t frame;       // 1: gate conjugated by the chain's recorded X-frame (PropagateX)
  int32_t src_out[2];  // per gate qubit j (j = 0 is the most significant local bit)
  int32_t src_in[2];
};

// A leaf is the product of its factors.  Its gate factors depend on the
// chain only through a few bits (projected qubits, recorded frame bits, slice
// bits): when there are at most PWS_LEAF_VAR_BITS of them the planner stores
// the leaf for every value of those bits (tab_off into the leaf table, variant
// v laid out as v << nfree | element) and the kernel only looks the entry up
// and multiplies the remaining per-chain noise factors (r_begin, r_count).
#define PWS_LEAF_VAR_BITS 8
enum : int32_t { VAR_CHAIN = 0, VAR_SLICE = 1, VAR_FRAME = 2 };  // variant-bit sources

struct LeafDesc {
  int32_t out_off;     // arena offset in elements
  int32_t nfree;       // free legs: the leaf has 1 << nfree elements
  int32_t f_begin, f_count;   // all factors (gate factors first)
  int32_t tab_off;     // complex entries into the leaf table, -1: evaluate factors
  int32_t nvar, var_begin;    // variant bits: codes (type << 24 | payload), FRAME payload =
                              // gate << 2 | the bit's position in the gate's recorded frame
  int32_t r_begin, r_count;   // residual factors applied after the table lookup
};

#define PWS_MAX_MODES 24
#define PWS_MAX_KBITS 24

// out[o] = sum_k A[offA(o) + kA[k]] * B[offB(o) + kB[k]], where the output
// index o is cut into `nmodes` bit fields (mode 0 lowest); field m has
// mode_width[m] bits and moves A / B by strideA[m] / strideB[m] per unit.
//
// Blocked form (kind = NODE_BLOCKED, used when the contracted legs K are at
// most PWS_BLOCK_KBITS and the B-only output legs N at most PWS_BLOCK_NBITS):
// lanes run over the output legs held by A (p, cut into `nmodes` fields with
// strides into A, B and the output); for each p the K values of A are loaded
// once into registers and reused for every one of the 2^n_bits outputs that
// differ only in N legs (ntab: B and output offsets of each N value).
#define PWS_BLOCK_KBITS 3
#define PWS_BLOCK_NBITS 12
// Matrix-core form (kind = NODE_MFMA): out[tile t, row r, column c] =
// sum_k A[tA(t) + rowA[r] + kA[k]] * B[tB(t) + colB[c] + kB[k]] written at
// tO(t) + rowO[r] + colO[c], for 16 x 16 tiles; the tile index t is cut into
// the `nmodes` fields (p_bits bits in all) and ntab holds rowA, rowO, colB,
// colO (16 ints each).
enum : int32_t { NODE_GENERIC = 0, NODE_BLOCKED = 1, NODE_MFMA = 2 };

struct NodeDesc {
  int32_t kind;
  int32_t out_off, a_off, b_off;
  int32_t out_bits, k_bits, nmodes;
  int32_t exp_a, exp_b, exp_out;   // exponent slots (-1 = exponent 0)
  int32_t ktab_off;                // kA, kB interleaved: 2 << k_bits ints
  int32_t p_bits, n_bits, ntab_off;  // blocked form: lane bits, N bits, (offB, offO) pairs
  int32_t renorm;                    // 1: rescale the output by its largest exponent
  int32_t mode_width[PWS_MAX_MODES];
  int32_t strideA[PWS_MAX_MODES];
  int32_t strideB[PWS_MAX_MODES];
  int32_t strideO[PWS_MAX_MODES];
};

// Sweep form of a step: the network is contracted by absorbing its leaves one
// at a time into a single running tensor that stays in the wave's LDS.  The
// tensor has `sw_width` bit positions; a live leg occupies one position and a
// free position holds no data (only its 0-half is ever read).  Absorbing a
// leaf is an in-place update of groups of 2^np elements that differ only in
// the op's positions: out[o] = sum_i M[o][i] in[i], with M built from the
// leaf's values.  Group bit j sits at position pos[j] with role:
//   KEEP     leg present before and after (M diagonal in that bit),
//   SUM      leg contracted here (input bit summed, output written at 0),
//   NEW      leg created here (input read at 0, output bit = the leg),
//   REPLACE  a contracted leg and a created leg share the position.
// Leaf leg k (bit k of the leaf element index) takes its value from group
// bit (leg[k] & 7) of the output index when leg[k] & 8, of the input index
// otherwise; legs with leg[k] & 16 occur in no other tensor and are summed
// inside M.  Groups are enumerated over the untouched live positions
// (outer_mask): bit t of the group index goes to the t-th lowest position of
// the mask, every other position is 0 in a group's base address.
#define PWS_SWEEP_MAXW 14
#define PWS_SWEEP_MAXNP 4
enum : int32_t { SW_KEEP = 0, SW_SUM = 1, SW_NEW = 2, SW_REPLACE = 3 };

// The matrices of a step's ops are built once per chain into one table
// (moff: an op's first entry; a diagonal op stores its 2^np diagonal
// entries, any other op its 4^np entries, row o, column i).  An entry is the
// product of PWS_MTERMS factors, each described by a code (mtab): bit 31 set
// = structural zero, bit 30 set = 1; else bits 0-15 the step-local leaf,
// bits 16-19 the leaf element with its internal legs at 0, bits 20-23 the
// mask of internal legs (the factor sums the leaf over them).  Several
// factors arise when diagonal ops are folded into a neighbouring op.
#define PWS_MTERMS 4
#define PWS_MCODE_ZERO (int32_t)0x80000000
#define PWS_MCODE_ONE (int32_t)0x40000000

// The same entries in the form the kernels read: the product of the
// chain-independent factors (value re, im, folded on the host) times at most
// two chain-dependent terms.  A term t >= 0 looks its value up in the term
// table at t + v, where v packs the chain bits named by p (bits 24-25: their
// count, bits 0-11 and 12-23: their positions; bit k of v is the k-th bit);
// t = -1: no term.  t0 = PWS_MENTRY_CODES: the entry is evaluated from its
// codes (noise records, frame or slice bits, wider variants).
#define PWS_MENTRY_CODES (-2)
// t0 = PWS_MENTRY_FLAT: the entry is the product of p1 factors described by
// flat records (eight int32 each, record p0 onwards): [0] the factor's first
// leaf-table entry (complex index: table offset plus element), [1] free legs
// | variant bits << 8 | noise records << 16, [2..5] the variant-bit codes
// (chain or frame bits; variant v reads entry [0] + (v << free legs)), [6..7]
// the noise records multiplied into it: segment | 1 << 28 for its 1-half |
// 2 << 28 | qubit << 16 for the half the chain's bit of that qubit selects.
#define PWS_MENTRY_FLAT (-3)
struct MEntry {
  double re, im;
  int32_t t0, p0, t1, p1;
};
static_assert(sizeof(MEntry) == 32, "MEntry is read as two 16-byte words");

// 32 bytes, read by the kernels as eight 32-bit words.
struct SweepOp {
  int32_t moff;               // the op's matrix in the step's table
  int32_t outer_mask;         // untouched live positions: 1 << n_outer groups
  int16_t in_mask, out_mask;  // group inputs read / outputs written (bit = group index)
  int16_t leaf;               // step-local leaf of the op's first factor
  int8_t np;                  // group positions (0..PWS_SWEEP_MAXNP)
  int8_t diag;                // 1: every position KEEP (elementwise product); 2: two positions,
                              // bit 1 KEEP and bit 0 not (block-diagonal matrix)
  int8_t renorm;              // rescale by the tensor's largest power of two afterwards
  int8_t n_outer;
  int8_t nleg;                // legs of that leaf (leg[]: their group bits)
  int8_t _pad;
  int8_t pos[PWS_SWEEP_MAXNP];
  int8_t role[PWS_SWEEP_MAXNP];
  int8_t leg[PWS_SWEEP_MAXNP];
};
static_assert(sizeof(SweepOp) == 32, "sweep op layout");

// What the kernels read of a sweep op, with the thread mapping worked out on
// the host for one workgroup size (2^log_nth threads per chain; one record
// array per size).  Threads take the lowest log_nth positions of outer_mask:
// thread t's part of a group address is the sum over terms j of
// (t << shift_j) & mask_j (positions of equal offset from their thread bit
// form one term), and the remaining positions (hi) are stepped through in
// 2^log_rounds rounds.  More than four such terms: the kernel deposits the
// bits one by one from outer_mask.
#define PWS_SWDEV_TERMS 4
struct SweepOpDev {
  int32_t moff;
  int32_t hi;          // bits 0-15 hi positions, 16-23 log2 rounds, 24-31 log2 threads with a group
  int32_t mask01;      // term masks 0 and 1 (16 bits each)
  int32_t mask23;      // term masks 2 and 3
  int32_t info;        // np | diag << 8 | renorm << 16
  int32_t pos;         // four position bytes
  int32_t outer_mask;  // for the bit-by-bit deposit
  int32_t shifts;      // 5 bits per term; bits 20-22 term count; bit 23: deposit bit by bit
};
static_assert(sizeof(SweepOpDev) == 32, "sweep op record layout");

// Dense-run form of a sweep step (noiseless plans): consecutive ops whose
// positions fit in four are multiplied, on the host in complex double, into
// one 16 x 16 complex matrix F per value of the chain bits their matrix
// entries read (at most PWS_DENSE_VARBITS of them); the kernels apply F to
// the running tensor viewed as 16 rows (the run's positions, bit b of the row
// at pos[b]) by 2^n_outer columns (the other live positions) with
// matrix-core instructions.  F tables: per variant 256 entries (row-major
// [row][col]), two 32-bit words each (re, im): FP32 values for FP32
// products, or for bf16 split products a pair of bf16 values per word, hi =
// rn(x) in the low half and lo = rn(x - hi) in the high half, formed from F
// in double (hi + lo carries x to about 16 bits); variant v of run r at
// foff + v (units of 512 words), v packing the bits of qubits q[0..nq)
// (bit b = s[q[b]]).  Ops
// join a run while its entries read at most PWS_DENSE_JOINBITS chain bits;
// an op that alone reads up to PWS_DENSE_VARBITS forms a run of its own.
#define PWS_DENSE_JOINBITS 4
#define PWS_DENSE_VARBITS 8
struct DenseRun {
  int32_t foff;        // first variant's table (units of 512 words)
  int32_t pos;         // row positions (bit b of the row index at nibble b) | the lowest
                       // min(n_outer, 4) column positions, in the same form, << 16
  int32_t outer_mask;  // live positions outside the run beyond those four columns
  int32_t info;        // n_outer | nq << 8 | renorm << 16
  int32_t q012, q345;  // variant qubits 0-5, ten bits each (qubit b: bits 10 (b % 3) of word b / 3)
  int32_t op;          // first sweep op the run covers (kept tensors and snapshots fall between runs)
  int32_t q67;         // variant qubits 6 and 7
};
__host__ __device__ inline int dense_qubit(int32_t q012, int32_t q345, int32_t q67, int b) {
  const int32_t w = b < 3 ? q012 : b < 6 ? q345 : q67;
  return (w >> (10 * (b % 3))) & 0x3ff;
}
static_assert(sizeof(DenseRun) == 32, "dense run layout");

// The fields that every step of a sampling pass reads, with the step gate's
// classification, copied at upload into the first 128 bytes of the step's
// record so that a wave reads them with two 64-byte scalar loads.
struct StepHot {
  int32_t gate, op, op_begin, nS;
  int32_t flags;                 // bit 0: fresh, bit 1: replay
  int32_t g_nq, g_q0, g_q1;      // step gate: qubits
  int32_t g_nS, g_sq;            // candidate qubits: count, positions sq[0] | sq[1] << 8
  int32_t g_cand;                // candidate masks by local value t of s[q] (byte t)
  int32_t sw_begin, sw_count, sw_width, m_begin, m_count, leaf_begin;
  int32_t load_op, store_op, load_w, store_w;
  int32_t snap_begin, snap_count, merge_slot;
  int32_t dn_begin, dn_count, dn_load, dn_w;
  int32_t root_index[4];
  int32_t merge_nb, merge_map;   // two-sided steps: shared legs and their map
  int32_t merge_pack;            // the map packed (at most four legs at positions
                                 // below 16): byte k = here | kept << 4; -1: none
  int32_t hot_pad;
  // fresh steps (a one-qubit gate on an untouched qubit): column 0 of the
  // gate, (re, im) of candidates 0 and 1; read by scalar loads next to the
  // hot fields (not part of the block the kernels fetch at every step)
  double fresh_amp[4];
};
static_assert(sizeof(StepHot) == 176, "hot step fields");
constexpr int kHotInts = 36;   // the per-step block: the fields before fresh_amp

struct StepDesc {
  StepHot hot;                   // device copy of the fields below (filled at upload)
  int32_t elem_begin, n_elems;   // flat leaf elements: (leaf index, element) pairs
  int32_t scal_begin, scal_count;  // factors with all legs fixed: a per-chain scalar common to
                                   // every candidate (skipped by draws, applied to amplitudes)
  int32_t op;            // op index of the step gate (-1: epilogue only)
  int32_t gate;          // gate index (-1: epilogue)
  int32_t op_begin;      // first op replayed in the prologue
  int32_t leaf_begin, n_leaves;
  int32_t node_begin, n_nodes;
  int32_t root_off, root_exp;
  int32_t nS;                 // open legs: 1 << nS candidates
  int32_t root_index[4];      // root element of candidate v
  int32_t n_slice_bits;
  int32_t zero_q_begin, zero_q_count;  // qubits that must be 0 (untouched)
  int32_t arena_elems;
  int32_t n_exp_slots;
  int32_t sweep;              // 1: sweep form (ops below), 0: node form
  int32_t sw_begin, sw_count; // sweep ops
  int32_t sw_width;           // positions of the running tensor
  int32_t leaf_area;          // sweep form: entries of the op matrix table (LDS)
  int32_t sw_max_np;          // sweep form: positions of the widest op
  int32_t m_begin, m_count;   // sweep form: matrix-entry codes of the step's ops
  // sweep form, consecutive steps: the running tensor after ops [0, store_op)
  // (store_w positions, and its exponent) is kept per chain for the next step,
  // whose ops [0, load_op) rebuild exactly that tensor; a sampling pass
  // restores it and starts at load_op (-1: no such point)
  int32_t load_op, store_op;
  int32_t load_w, store_w;
  int32_t replay;             // 1: some op in [op_begin, op) changes the chain's bits or
                              // records (monomial gates, noise sites, frame records)
  // sweep form, anchor steps: the running tensor is also kept before ops
  // snaps[snap_begin ..+ snap_count) (cache slots 1, 2, ...) for later steps
  int32_t snap_begin, snap_count;
  // sweep form, two-sided steps: the candidate amplitudes are the contraction
  // of the final running tensor with the tensor kept in cache slot
  // merge_slot over merge_nb legs (mmap[merge_map + 2k]: the leg's position
  // here, mmap[merge_map + 2k + 1]: in the kept tensor); -1: none
  int32_t merge_slot = -1, merge_nb, merge_map;
  // 1: the step's gate acts on one qubit that no earlier gate touched, so the
  // prefix state is G|0> on that qubit times the rest and a sampling pass
  // draws from |G[v][0]|^2 without contracting (the common factor cancels in
  // the normalisation); the step keeps no tensor for later steps.
  int32_t fresh = 0;
  // dense-run form: runs [dn_begin, dn_begin + dn_count) cover the sweep ops
  // [dn_op0, sw_count) (dn_op0 = 0, or the restore point when only sampling
  // passes use them); dn_w = positions of the tensor (at least four);
  // dn_count = 0: the step has no dense form (entries that read noise
  // records, frame or slice bits)
  int32_t dn_begin = 0, dn_count = 0, dn_op0 = 0, dn_w = 0;
  int32_t dn_load = 0;        // the run a restoring sampling pass starts at (the first whose op is
                              // at or after load_op; dn_count when no run is left)
};

struct SnapDesc {
  int32_t op;     // kept before this op runs (after the op before it)
  int32_t slot;   // cache slot
  int32_t w;      // positions kept (2^w elements)
};

struct OpDesc {
  int32_t type;   // 0 gate, 1 noise
  int32_t idx;
};

struct GateDev {
  int32_t nq, q0, q1;
  int32_t monomial, diagonal;
  int32_t sigma[4];        // monomial: out local index of in local index
  int32_t sq[2], nS;       // non-diagonal qubit positions j within the gate
  int32_t cand_mask[4];    // by local value of s[q]: bitmask over candidates v
};

struct NoiseDev {
  int32_t nq, q0, q1, nbranch;
  int32_t seg[2];          // segment id of each qubit when the site acts
  int32_t tab_off;         // into the noise table (NoiseBranch entries)
  // into the branch-sum table: for each value t = t0 | t1 << 1 of the true
  // bits the site acts on, nbranch + 1 doubles: the inclusive prefix sums of
  // Pr(i | t) (Eq. (4), summed in branch order; the last one is the total)
  // and the index of the last branch with a nonzero weight
  int32_t cum_off;
};

// One (branch i, factor j) entry of a Kraus list.
struct NoiseBranch {
  double colnorm[2];       // |column t of M_ij|^2, t = 0, 1
  double d0re, d0im, d1re, d1im;  // diagonal of M (or of M sigma_X when anti)
  int32_t anti;            // M has a zero diagonal: flip the frame bit
  int32_t _pad;
};

}  // namespace pws
