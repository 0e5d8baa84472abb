// Host-side launchers of the l0cim kernels (internal).
#pragma once

#include "common.h"

namespace l0 {

// ---- Gram / Zeeman prep -------------------------------------------------
l0cim_status launch_gram(l0cim_dtype dt, int m, int n, const void* A, int64_t lda, const void* y,
                         void* G, int64_t ldg, void* b, hipStream_t s);

// ---- couplings, initial state, R_init ------------------------------------
l0cim_status launch_couplings(l0cim_dtype dt, int n, const void* G, int64_t ldg, const void* b,
                              const void* R, l0cim_dtype jdt, void* J, int64_t ldj, float* rscale,
                              void* z, hipStream_t s);
l0cim_status launch_init_state(l0cim_dtype dt, int n, int P, uint64_t seed, int alt, double std,
                               void* c, void* e, hipStream_t s);
// Several MRI-shaped instances of one launch: instance k's arrays sit at k
// times these strides (elements) from the first instance's.  One instance:
// all zero.
struct MriStrides {
  int64_t mask;     // sampling masks (bytes)
  int64_t vec;      // per-spin vectors: R, b, the selected support
  int64_t D;        // diagonals D (elements; read with the launch's incd)
  int64_t state;    // replica arrays c, e, sigma (P * n)
  int64_t H;        // replica energies (P)
  int64_t status;   // status words (ints)
  int64_t it;       // CG iteration counts (ints)
};
l0cim_status launch_mri_mfcim(int size, int levels, int P, const uint8_t* mask, const float* R,
                              const float* D, int64_t incd, const float* b, double gamma, const CimArgs& a, float* c,
                              float* e, uint8_t* sigma, double* H, float* trace, int* status, hipStream_t s,
                              int count = 1, const MriStrides& ms = MriStrides{});
l0cim_status launch_mri_l2_diag(int size, int levels, double gamma, const float* D_in, int64_t incd, float* D_out,
                                hipStream_t s);
l0cim_status launch_mri_lasso(int size, int levels, double gamma, const uint8_t* mask, const float* b, double lam1,
                              int iters, float* R_out, hipStream_t s, int count = 1,
                              const MriStrides& ms = MriStrides{});
l0cim_status launch_mri_jacobi(int size, int levels, double gamma, const uint8_t* mask, const float* D,
                               int64_t incd, const float* b, const uint8_t* sigma, float* R, int iters, double dtc,
                               int* status, hipStream_t s, int count = 1, const MriStrides& ms = MriStrides{});
l0cim_status launch_mri_aty_colnorm(int m, int n, const float* A, int64_t lda, const float* y, float* b, float* D,
                                    hipStream_t s);
l0cim_status launch_mri_r_init(int n, const float* b, const float* D, float* R, int* status, hipStream_t s);
l0cim_status launch_mri_cg(int size, int levels, double gamma, const uint8_t* mask, const float* D, int64_t incd,
                           const float* b, const uint8_t* sigma, float* R, int max_iter, double tol, int* iters_out,
                           int* status, hipStream_t s, int count = 1, const MriStrides& ms = MriStrides{});
l0cim_status launch_r_init(l0cim_dtype dt, int n, const void* G, int64_t ldg, const void* b,
                           const void* R_init, void* R, int* status, hipStream_t s);
// the same, also writing the diagonal G_rr to D_out (n, may be NULL)
l0cim_status launch_r_init_diag(l0cim_dtype dt, int n, const void* G, int64_t ldg, const void* b,
                                const void* R_init, void* R, void* D_out, int* status, hipStream_t s);

// ---- CIM run ---------------------------------------------------------------
size_t mfcim_ws_bytes(l0cim_dtype dt, int n, int P);
// the part of a run's workspace the launches other than the matrix-core form use
size_t mfcim_base_ws_bytes(l0cim_dtype dt, int n, int P);
size_t matrix_ws_offset(int n, int P);
// allow_matrix = false never takes the matrix-core form (whose panel copy of J
// lives past mfcim_base_ws_bytes in the workspace)
l0cim_status launch_mfcim(l0cim_dtype dt, int n, int P, l0cim_dtype jdt, const void* J, int64_t ldj,
                          const float* rscale, const void* z, const CimArgs& a, void* c, void* e,
                          uint8_t* sigma, double* H, void* trace, int* status, void* ws,
                          size_t ws_bytes, hipStream_t s, bool allow_matrix = true);
// argument checks of l0cim_mfcim_run, then the run on workspace ws
l0cim_status mfcim_run_checked(l0cim_dtype dtype, int n, int P, l0cim_dtype j_dtype, const void* J, int64_t ldj,
                               const float* row_scale, const void* z, double eta, const l0cim_cim_params* prm,
                               void* c, void* e, uint8_t* sigma, double* H, void* trace, int trace_steps,
                               int* status, void* ws, size_t ws_bytes, bool allow_matrix, hipStream_t s);
// several single-replica FP32 runs of the same n in one register-resident
// launch: instance i at J + i sJ, per-spin vectors + i sv, run workspace + i
// sws bytes (each at least mfcim_base_ws_bytes(F32, n, 1)), status + i sst,
// H + i sh; UNSUPPORTED when that form does not apply (the caller runs them one
// by one)
l0cim_status launch_mfcim_many(l0cim_dtype jdt, int count, int n, const void* J, int64_t ldj, int64_t sJ,
                               const float* rscale, const float* z, int64_t sv, const CimArgs& a, float* c, float* e,
                               uint8_t* sigma, double* H, int64_t sh, int* status, int64_t sst, void* ws,
                               int64_t sws, hipStream_t s);
size_t matrix_ws_bytes(int n, int P, size_t jsize);
bool matrix_supported(int n, int P, int64_t ldj);
l0cim_status launch_matrix_run(int n, int P, l0cim_dtype jdt, const void* J, int64_t ldj, const float* rscale,
                               const float* z, const CimArgs& a, float* c, float* e, uint8_t* sigma, double* H,
                               float* trace, int* status, void* ws, hipStream_t s, int rb_hint);
l0cim_status launch_select(int n, int P, const double* H, const uint8_t* sigma, uint8_t* out,
                           int32_t* q_out, double* H_out, hipStream_t s);

// ---- CDP ----------------------------------------------------------------
size_t jacobi_ws_bytes(l0cim_dtype dt, int n);
l0cim_status launch_jacobi(l0cim_dtype dt, int n, const void* G, int64_t ldg, const void* b,
                           const uint8_t* sigma, double dtc, int iters, void* R, int* status,
                           void* ws, size_t ws_bytes, hipStream_t s, int64_t spin_limit);
size_t chol_ws_bytes(int n);
l0cim_status launch_chol_refit(l0cim_dtype dt, int n, const void* G, int64_t ldg, const void* b,
                               const uint8_t* sigma, void* R, int* status, void* ws, size_t ws_bytes,
                               hipStream_t s);
// the same refit with G_SS, b_S and the off-support rows formed from A (m x n)
// and y in FP64
size_t chol_a_ws_bytes(int n, int m);
l0cim_status launch_chol_refit_a(l0cim_dtype dt, int m, int n, const void* A, int64_t lda, const void* y,
                                 const uint8_t* sigma, void* R, int* status, void* ws, size_t ws_bytes,
                                 hipStream_t s);

// ---- solve epilogue ------------------------------------------------------
size_t objective_ws_bytes(int m);
l0cim_status launch_objective(l0cim_dtype dt, int m, int n, const void* A, int64_t lda, const void* y,
                              const uint8_t* sigma, const void* R, double lam, l0cim_stats* stats,
                              int64_t spin_steps, int n_outer, void* ws, size_t ws_bytes,
                              hipStream_t s);

}  // namespace l0
