// Host-side view of the device program and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "program.hpp"

namespace pws {

// Device pointers of one plan's programs and tables (uploaded once).
struct DevProg {
  const StepDesc *steps;
  const LeafDesc *leaves;
  const FactorDesc *factors;
  const NodeDesc *nodes;
  const int32_t *ktab;
  const int32_t *zero_q;
  const OpDesc *ops;
  const GateDev *gates;
  const NoiseDev *noise;
  const NoiseBranch *ntab;
  const double *ncum;      // branch-sum tables of the noise sites (NoiseDev::cum_off)
  const double *gmat;      // per gate 16 complex entries (32 doubles)
  const double *gdmat;     // derivative matrices, same layout
  const NodeDesc *bnodes;  // backward nodes (gradient program)
  const int32_t *grad_terms;
  const double *ltab;       // tabulated leaves
  const int32_t *lvar;      // variant-bit codes
  const int32_t *lelem;     // (leaf, element) pairs per step
  const SweepOp *sweeps;    // sweep-form ops
  const SweepOpDev *swdev;  // the same ops as kernel records, for 64, 256 and 512 threads per chain
  int32_t n_sweep_ops;      // records per workgroup size
  const int32_t *mtab;      // sweep-form matrix-entry codes
  const MEntry *ment;       // the same entries with their constant factors folded
  const SnapDesc *snaps;    // anchor steps' kept tensors
  const int32_t *mmap;      // two-sided steps' leg position pairs
  const double *mterm;      // chain-dependent term tables
  const int32_t *mflat;     // flat factor records (PWS_MENTRY_FLAT entries)
  const DenseRun *druns;    // dense-run form of sweep steps
  const uint32_t *dtab;     // their F tables
  const double *readout;    // per-qubit readout flip probability (null: none)
  int32_t n_qubits, words, n_gates, n_segs;
  int32_t n_ops, noisy, n_params, n_bnodes;
  int32_t n_grad_terms, adj_root_off;   // gradient program: arena offset of the root adjoint
};

// Per-chain state in device memory.
struct ChainState {
  uint64_t *s;        // [K][words] classical state
  uint64_t *x;        // [K][words] X-frame (noisy plans)
  uint8_t *gframe;    // [K][n_gates] frame bits recorded per gate (noisy plans)
  double *segfac;     // [K][n_segs][4] diagonal noise factors per segment (noisy plans)
};

enum { MODE_SAMPLE = 0, MODE_AMPS = 1 };

struct StepLaunch {
  int step;              // index into steps (sweep form: first step of the launch's range)
  int step_end;          // sweep form: one past the last step of the range
  int range_w;           // sweep form: widest running tensor of the range (LDS layout)
  int64_t n_chains;
  int64_t chain_offset;  // global id of chain 0 (random stream key)
  uint64_t seed;
  const uint64_t *seed_ptr;  // when set, the seed is read from device memory (graph replays)
  void *arena;           // grid * arena_stride elements
  int64_t arena_stride;
  int grid, block;
  int mode;
  double *out_amp;       // MODE_AMPS: [K][1 << nS][2]
  int32_t *out_log2;     // MODE_AMPS: [K]
  uint8_t *trace;        // MODE_SAMPLE (nullable): [n_steps][K]
  int trace_row;
  int32_t *err;          // error flags (device int)
  int lds_bytes;
  int lds_arena;         // 1: one workgroup per chain, arena in LDS (arena_stride elements)
  int n_exp;             // LDS form: exponent slots reserved after the arena
  int sweep;             // > 0: sweep-form step; sweep - 1: bit 0 widest op has 3-4 positions,
                         // bit 1 four / bit 2 eight waves per chain, bit 3 op matrices in device
                         // memory, bit 4 two / bit 5 four chains per wave
  void *cache;           // sweep form: kept running tensors, cache_stride elements per chain
  int64_t cache_stride;
  int32_t *cache_exp;    // sweep form: exponent pair of each kept tensor
  void *mt_global;       // sweep form: op-matrix tables in device memory (null: in LDS)
  int64_t mt_stride;     // elements per workgroup
  int slot_bytes;        // sweep form: LDS bytes per chain (head, tensor, op matrices)
  int cache_slots;       // sweep form: kept tensors per chain (cache_stride elements each)
  int mt_cap;            // sweep form: op-matrix entries the LDS slot holds (a window of the
                         // step's table when smaller than the table)
  int probe_step;        // MODE_SAMPLE with out_amp set: the step whose candidate amplitudes are
                         // written to out_amp / out_log2
  int dense;             // sweep form: 0 op by op on the vector ALUs, 1 dense runs with FP32
                         // matrix-core products, 2 dense runs with bf16 hi/lo split products
  int u_off;             // sweep-form ranges: LDS byte offset of the draw uniforms (64 doubles
                         // per workgroup), -1: each step draws its own
};

constexpr int kRangeUniformBytes = 64 * 8;

constexpr int kWavesPerBlock = 4;   // one chain per wave, 256-thread workgroups
int lds_bytes_for(int n_exp_slots);  // dynamic LDS of a wave-form step / gradient launch
int lds_bytes_arena(int precision, int arena_elems, int n_exp);  // dynamic LDS of the LDS form
int sweep_slot_bytes(int precision, int width, int m_entries);   // LDS of one chain of a sweep-form step
int lds_bytes_sweep(int precision, int width, int m_entries, int cpw = 1);   // dynamic LDS of a workgroup

// Static LDS of a dense-run launch with one wave per chain: the staged table
// of the chain's next run (512 words per chain).
constexpr int kDenseTabBytes = 2048;

// Static workspace of the allocation-free sampling call: kScratchBytes of
// device memory per device, its address looked up once per device (with that
// device current) and kept.  Calls on one device share it.
constexpr size_t kScratchBytes = size_t(64) << 20;
hipError_t scratch_region(int device, void **ptr, size_t *bytes);
hipError_t launch_clear_flags(int32_t *flags, int n, hipStream_t s);

hipError_t launch_init_state(const DevProg &p, const ChainState &st, int64_t K, hipStream_t s);
hipError_t launch_step(int precision, const DevProg &p, const ChainState &st, const StepLaunch &l,
                       hipStream_t s);
// Output bits s XOR x of every chain (global ids chain_offset ..), with the
// readout flips of p.readout drawn when `readout` is set.
hipError_t launch_finalize(const DevProg &p, const ChainState &st, int64_t K, uint64_t *out,
                           hipStream_t s, uint64_t seed, const uint64_t *seed_ptr, int64_t chain_offset,
                           bool readout);

struct GradLaunch {
  int64_t n_chains;
  void *arena;
  int64_t arena_stride;
  int grid, block;
  double *dtheta;    // [K][n_params]
  double *amp;       // [K][2] root mantissa (diagnostics, nullable)
  int32_t *amp_log2; // [K] (nullable)
  int32_t *err;
  int lds_bytes;
};
hipError_t launch_grad(int precision, const DevProg &p, const ChainState &st, const GradLaunch &l,
                       hipStream_t s);

}  // namespace pws
