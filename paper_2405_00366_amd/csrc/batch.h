// Internal declarations of the batched engine (many instances x replicas).
#pragma once

#include "kernels.h"

namespace l0 {

// Device table entry of one instance: its sizes and the device addresses of
// everything it reads and writes, so that instances may live anywhere (the
// pools of a batch plan, a serving arena, a caller's single-instance buffers).
struct BInst {
  int n, m, ld;          // spins, measurement rows, padded row length (multiple of 32)
  int ldj;               // row stride of J (multiple of 32)
  int tile0, ntiles;     // row tiles of this instance in the tile table
  int lda;               // leading dimension of A
  int alt;               // alternation index (used when the launch passes alt < 0)
  uint64_t seed;
  double eta;            // threshold eta of the alternation (used when no global eta is passed)
  const float* A;        // m x lda
  const float* y;        // m
  float* G;              // n x ld Gram rows
  float* Gc;             // n x ld scratch: G restricted to the support's columns
  void* J;               // couplings (FP32, BF16 or FP8 e4m3) in the panel layout, n16 x ld
  float *b, *z, *rs;     // ld: A^T y, Zeeman term R o b, per-row coupling scale
  float* R;              // n amplitudes (in/out)
  uint8_t* sig;          // n chosen support (out)
  float *c, *c2, *e;     // P x ld: amplitudes (double-buffered) and error variables
  uint32_t *xb, *xb2;    // support bits of c and c2 (binarised field), xbits_words(ld, P) each
  float* jw;             // CDP and report scratch: 5 ld + 192 words
  uint8_t* sig_all;      // P x n supports of every replica
  double* hpart;         // P x n per-spin eq. 4 terms
  int* status;           // status word (first field of the instance's stats)
  l0cim_stats* st;       // report of the instance
};

// Panel layout of the couplings: rows in panels of 16 (the row count padded
// to n16 = 16 np, a multiple of 16), columns in chunks of 32 (ld); block
// (p, c) holds J[16 p, 16 p + 16) x [32 c, 32 c + 32) as 512 consecutive
// elements in the order the matrix-core operands are loaded, so that each
// wavefront load reads one contiguous run:
//   4-byte elements: (li, 8 lk + 4 h + u) at ((16 h + li) * 4 + lk) * 4 + u
//   1- and 2-byte:   (li, 8 lk + t)       at (4 li + lk) * 8 + t
// Panels go in groups of kPanelGroup (the last group holds the rest): group
// g holds chunk c of its gs panels side by side, so that a row tile of up to
// kPanelGroup panels (aligned to its size) reads one contiguous run of
// gs blocks per chunk: block (p, c) starts at
//   (kPanelGroup g nch + c gs + p mod kPanelGroup) 512,  g = p / kPanelGroup.
constexpr int kPanelGroup = 8;
__host__ __device__ inline int jpanel_group_size(int p, int np) {
  const int rest = np - (p / kPanelGroup) * kPanelGroup;
  return rest < kPanelGroup ? rest : kPanelGroup;
}
// First element of panel group p / kPanelGroup: a row tile of RB panels
// (RB dividing kPanelGroup) starting at panel p0 finds chunk c of its panel
// p0 + rb at jpanel_group_base(p0, nch) + (c gs + (p0 + rb) mod kPanelGroup) 512.
__host__ __device__ inline size_t jpanel_group_base(int p0, int nch) {
  return size_t(p0 / kPanelGroup) * kPanelGroup * nch * 512;
}
__host__ __device__ inline size_t jpanel_block(int p, int c, int nch, int np) {
  const int g = p / kPanelGroup;
  return (size_t(g) * kPanelGroup * nch + size_t(c) * jpanel_group_size(p, np) + size_t(p % kPanelGroup)) * 512;
}
__host__ __device__ inline size_t jpanel_offset(int r, int j, int ld, int np, int esize) {
  const int li = r & 15, jj = j & 31, lk = jj >> 3, t = jj & 7;
  const size_t blk = jpanel_block(r >> 4, j >> 5, ld >> 5, np);
  if (esize == 4) return blk + size_t(((16 * (t >> 2) + li) * 4 + lk) * 4 + (t & 3));
  return blk + size_t((4 * li + lk) * 8 + t);
}
inline int round_up16(int n) { return (n + 15) / 16 * 16; }
// Support bits: for each 32-column chunk c a block of 16 QB words (QB =
// ceil(P / 16)); bit t of word c * 16 QB + li * QB + qb holds
// H(c_q) of column 32 c + t for replica q = 16 qb + li, so the QB words a
// lane needs for one chunk are adjacent.
inline int xbits_qb(int P) { return P <= 16 ? 1 : (P <= 32 ? 2 : 4); }
inline size_t xbits_words(int ld, int P) { return size_t(ld / 32) * 16 * xbits_qb(P); }
// Tile shapes with RB panels per workgroup and 16 QB replicas.
inline bool step_shape_ok(int qb, int rb) {
  return (qb == 1 && (rb == 1 || rb == 2 || rb == 4 || rb == 8)) ||
         (qb == 2 && (rb == 1 || rb == 2 || rb == 4 || rb == 8)) || (qb == 4 && (rb == 1 || rb == 2 || rb == 4));
}

struct BTile {
  int inst, row0;   // inst < 0: an empty tile (its workgroup exits at once)
};

// XCDs of the device; the dispatcher deals workgroup b to XCD b mod kXcds.
constexpr int kXcds = 8;

struct BStepArgs {
  int P, n_steps, linear_j, field;
  double dt, p_thr, d, t_c, t_w, K, j, beta, tau;
  float* trace;          // optional: (k, c|e, q, r) for k < trace_steps (single instance)
  int trace_steps;
};

// Device tables of one batched launch sequence.
struct BatchDev {
  int count;
  const BInst* insts;
  const BTile* tiles;
  const int64_t* row_prefix;   // count + 1: prefix sums of n16 (rows padded to 16)
  const int64_t* st_prefix;    // count + 1: prefix sums of P * ld
  const double* eta;           // one eta for every instance, or NULL: each instance's own
};

// A step kernel and its workgroup size (fn NULL: no kernel for that shape).
struct StepKernel {
  const void* fn;
  int threads;
};
StepKernel batch_step_kernel(l0cim_dtype jdt, int field, int qb, int rb);
l0cim_status launch_bcouplings(const BatchDev& d, l0cim_dtype jdt, int64_t total_rows, hipStream_t s);
l0cim_status launch_binit(const BatchDev& d, int P, int alt, double std, int64_t total_state, hipStream_t s);
l0cim_status launch_bbits(const BatchDev& d, int QB, int64_t total_words, hipStream_t s);
l0cim_status launch_bselect(const BatchDev& d, int P, hipStream_t s);
// Words of per-instance CDP scratch for padded row length ld.
inline size_t bjac_words(int ld) { return size_t(5) * ld + 192; }
// Row tiles of `rows_per_tile` rows (the same tile table as the step launches).
l0cim_status launch_bjacobi(const BatchDev& d, int ntiles, int rows_per_tile, double dtc, int iters,
                            hipStream_t s);
// lam < 0: each instance's own 0.5 eta^2, alternation count alt + 1 and
// spin-steps n P steps_per_alt (alt + 1); otherwise the given values.
l0cim_status launch_bobjective(const BatchDev& d, double lam, int64_t steps_per_alt, int n_outer, int P,
                               hipStream_t s);
l0cim_status launch_bstats_init(const BatchDev& d, hipStream_t s);
l0cim_status enqueue_bsteps(const BatchDev& d, StepKernel k, const BStepArgs& a, int ntiles, int k0, int k1,
                            hipStream_t s);
l0cim_status launch_bfill(float* p, int64_t count, hipStream_t s);
l0cim_status launch_bset_scalar(double* p, double v, hipStream_t s);

}  // namespace l0
