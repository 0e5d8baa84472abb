// Internal declarations of the batched engine (many instances x replicas).
#pragma once

#include "kernels.h"

namespace l0 {

// Device table entry of one instance (offsets in elements of each pool).
struct BInst {
  int n, m, ld;          // spins, measurement rows, padded row length (multiple of 32)
  int ldj;               // row stride of J (multiple of 32)
  int tile0, ntiles;     // row tiles of this instance in the tile table
  int lda;               // leading dimension of A
  int64_t oG;            // n x ld floats in the G (and compact-G) pools
  int64_t oJ;            // n x ld coupling elements in the J pool
  int64_t oV;            // ld floats in the b, z and row-scale pools
  int64_t oS;            // P x ld floats in the c, c2 and e pools
  int64_t oSig;          // P x n bytes in the all-replica support pool
  int64_t oX;            // n elements of R and sigma in the caller's pools
  int64_t oA, oY;        // A (m x lda) and y (m) in the caller's pools
  uint64_t seed;
  int alt;               // alternation index of this instance (serving form)
  int pad0;
  double eta;            // its threshold eta_alt (serving form)
};

struct BTile {
  int inst, row0;
};

struct BStepArgs {
  int P, n_steps, linear_j, field;
  double dt, p_thr, d, t_c, t_w, K, j, beta, tau;
  float* trace;          // optional: (k, c|e, q, r) for k < trace_steps (single instance)
  int trace_steps;
};

// Device pointers of one batched solve (carved from the workspace).
struct BatchDev {
  int count;
  const BInst* insts;
  const BTile* tiles;
  const int64_t* row_prefix;   // count + 1: prefix sums of n
  const int64_t* st_prefix;    // count + 1: prefix sums of P * ld
  double* eta;
  float *G, *Gc, *b, *z, *rs, *c, *c2, *e;
  void* J;
  uint8_t* sig_all;
  double* hpart;
  float* R;          // caller pool
  uint8_t* sig_out;  // caller pool
  l0cim_stats* stats;
};

const void* batch_step_kernel(l0cim_dtype jdt, int field, int qb, int rb);
l0cim_status launch_bcouplings(const BatchDev& d, l0cim_dtype jdt, int64_t total_rows, hipStream_t s);
l0cim_status launch_binit(const BatchDev& d, int P, int alt, double std, int64_t total_state, hipStream_t s);
l0cim_status launch_bselect(const BatchDev& d, int P, hipStream_t s);
l0cim_status launch_bjacobi(const BatchDev& d, int max_ld, double dtc, int iters, hipStream_t s);
l0cim_status launch_bobjective(const BatchDev& d, const float* A, const float* y, double lam,
                               int64_t steps_per_spin, int n_outer, int P, hipStream_t s);
l0cim_status launch_bstats_init(l0cim_stats* st, int count, hipStream_t s);
l0cim_status launch_bfill(float* p, int64_t count, hipStream_t s);
l0cim_status launch_bset_scalar(double* p, double v, hipStream_t s);

}  // namespace l0
