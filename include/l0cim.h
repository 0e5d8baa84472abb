/*
 * l0cim.h -- C ABI of the MI355X (gfx950) MF-CIM solver for L0-regularised
 * compressed sensing (L0RBCS).
 *
 * The method (Gunathilaka et al., "L0-regularized compressed sensing with
 * Mean-field Coherent Ising Machines", arXiv:2405.00366) alternates two
 * minimisations of the L0RBCS objective (eq. 3):
 *   - sigma in {0,1}^N, by integrating the mean-field CIM with chaotic
 *     amplitude control (MFZ-CIM, eq. 12-16) on the Ising form of the
 *     objective (eq. 4), with couplings J = -(A^T A) o R R^T (zero diagonal)
 *     and Zeeman term z = R o A^T y;
 *   - R in R^N, by a classical digital processor (CDP): Jacobi relaxation
 *     (Numerical experiments, parameter paragraph) or an FP64 least-squares
 *     refit on the support;
 * with the pump (eq. 21) and threshold (eq. 22) schedules of Algorithm 1.
 *
 * Conventions for every entry point
 *   - Array pointers are DEVICE memory owned by the caller unless stated
 *     otherwise; parameter structs are HOST memory, read during the call only.
 *   - Matrices are row-major with an explicit leading dimension (in elements).
 *   - `dtype` selects the arithmetic of the call: L0CIM_F32 or L0CIM_F64.
 *     Every floating-point array of the call except J and row_scale has that
 *     type (float* or double* passed as void*).
 *   - Every call enqueues work on `stream` (a hipStream_t passed as void*,
 *     NULL = the null stream) and returns without synchronising.  Outputs are
 *     valid once the caller has synchronised the stream.
 *   - No call allocates or frees device memory.  Scratch comes from the
 *     caller's workspace `ws` of `ws_bytes` bytes (256-byte aligned); the
 *     matching *_workspace_bytes() function returns the exact size needed.
 *     A workspace may be reused by consecutive calls on one stream; calls that
 *     overlap in time must use different workspaces.
 *   - Errors the host can detect (NULL pointer, bad size or leading
 *     dimension, unsupported dtype, workspace too small) return before
 *     anything is enqueued and leave every output untouched.  Launch errors
 *     return L0CIM_ERR_HIP.  l0cim_last_error() gives a thread-local message.
 *   - Numerical failures are found on the device and reported through a
 *     device-resident status word (bits L0CIM_ST_*), OR-ed in by the kernels.
 */
#ifndef L0CIM_H
#define L0CIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define L0CIM_VERSION 100

typedef enum {
  L0CIM_OK = 0,
  L0CIM_ERR_ARG = 1,          /* NULL pointer or out-of-range scalar */
  L0CIM_ERR_SHAPE = 2,        /* bad size or leading dimension */
  L0CIM_ERR_WORKSPACE = 3,    /* ws NULL or ws_bytes too small */
  L0CIM_ERR_HIP = 4,          /* a HIP runtime call failed */
  L0CIM_ERR_UNSUPPORTED = 5   /* dtype / field / method combination not built */
} l0cim_status;

typedef enum {
  L0CIM_F32 = 0,
  L0CIM_F64 = 1,
  L0CIM_BF16 = 2,             /* coupling storage only */
  L0CIM_FP8E4M3 = 3           /* coupling storage only (OCP e4m3, max 448) */
} l0cim_dtype;

typedef enum {
  L0CIM_FIELD_CN = 0,         /* continuous local field, eq. 15 */
  L0CIM_FIELD_BN = 1          /* binarised local field,  eq. 16 */
} l0cim_field;

typedef enum {
  L0CIM_LAUNCH_AUTO = 0,
  L0CIM_LAUNCH_RESIDENT = 1,
  L0CIM_LAUNCH_STREAMED = 2,
  L0CIM_LAUNCH_MATRIX = 3     /* FP32 state: J X on the matrix cores, one launch per step */
} l0cim_launch;

typedef enum {
  L0CIM_CDP_JACOBI = 0,       /* damped Jacobi sweeps over all r */
  L0CIM_CDP_CHOL_F64 = 1,     /* FP64 Cholesky least squares on the support */
  L0CIM_CDP_CG = 2            /* conjugate gradients on the support (MRI form) */
} l0cim_cdp;

/* Device status bits. */
#define L0CIM_ST_NONFINITE  0x01  /* an amplitude or error variable is not finite */
#define L0CIM_ST_BLOWUP     0x02  /* |c| > 1e3 at the end of a run */
#define L0CIM_ST_CHOL_RIDGE 0x04  /* Cholesky pivot <= 1e-12 max diag: ridge added */
#define L0CIM_ST_TINY_DIAG  0x08  /* some G_rr < 1e-12: that R_r held at 0 */
#define L0CIM_ST_TIMEOUT    0x10  /* a bounded device wait gave up (run aborted) */

/* MFZ-CIM dynamics: eq. 12-16 and the pump schedule eq. 21. */
typedef struct {
  double dt;          /* Euler increment (0.02) */
  int32_t n_steps;    /* Euler steps per CIM run (1000 = 20 photon lifetimes) */
  int32_t field;      /* l0cim_field */
  double p_thr;       /* pump threshold (1) */
  double d;           /* pump swing (0.4 random data, 0.6 MRI) */
  double t_c, t_w;    /* sigmoid centre and width (4, 2) */
  double K;           /* feedback strength (1 random data, 0.1 MRI) */
  double j;           /* out-coupling rate (no value printed; default 0.2) */
  double beta;        /* CAC rate (no value printed; default 0.3) */
  double tau;         /* CAC target amplitude (1) */
  double c0_std;      /* std of the initial amplitudes (1e-2: variance 1e-4) */
  int32_t linear_j;   /* 1: linear term (-1 + p - j - c^2) (supporting info) */
  int32_t launch;     /* l0cim_launch: 0 automatic; 1 resident (one persistent launch, J on
                         chip, error if it does not fit); 2 streamed (one launch per step);
                         3 matrix cores (FP32 state, P <= 64) */
  int64_t spin_limit; /* bound on polls of one device wait; 0 = default (2^22) */
} l0cim_cim_params;

/* Alternating minimisation (Algorithm 1), threshold schedule eq. 22, CDP. */
typedef struct {
  double eta_init, eta_end;  /* eta_i = max(eta_init (1 - i/velo), eta_end) */
  int32_t velo;              /* schedule length (51 random data, 11 MRI) */
  int32_t n_outer;           /* number of alternations performed */
  int32_t cdp;               /* l0cim_cdp used inside the loop (JACOBI) */
  int32_t cdp_iters;         /* Jacobi sweeps per alternation (100) */
  double dtc;                /* Jacobi time increment (0.1) */
  int32_t final_refit_f64;   /* 1: FP64 Cholesky refit of R on the final support */
  int32_t replicas;          /* P >= 1 independent CIM trajectories */
  uint64_t seed;             /* key of the initial-amplitude generator */
  int32_t j_dtype;           /* coupling storage: F32 | F64 | BF16 | FP8E4M3 */
  int32_t flags;             /* OR of L0CIM_SOLVE_*: NO_GRAPH launches the batched form's Euler
                                steps one by one instead of replaying a HIP graph */
} l0cim_solve_params;

#define L0CIM_SOLVE_NO_GRAPH 1

/* Per-solve report, written by the device into caller memory. */
typedef struct {
  int32_t status_bits;       /* OR of L0CIM_ST_* over the whole solve */
  int32_t selected_replica;  /* replica kept in the last alternation */
  int32_t support_size;      /* |sigma| returned */
  int32_t n_outer_done;
  double H;                  /* eq. 4 energy of the returned sigma (at the R of the last run) */
  double E;                  /* eq. 3 objective of (sigma, R_out) at the last lambda */
  int64_t spin_steps;        /* N * P * n_steps * n_outer */
} l0cim_stats;

int l0cim_version(void);
const char* l0cim_status_string(l0cim_status s);
const char* l0cim_last_error(void);

/* Paper defaults for random data (Numerical experiments, parameter paragraph). */
void l0cim_cim_params_default(l0cim_cim_params* p);
void l0cim_solve_params_default(l0cim_solve_params* p);

/*
 * l0cim_gram -- G = A^T A (n x n, leading dim ldg) and b = A^T y (n).
 * The couplings and Zeeman term of the Ising form are minus G and
 * sqrt(tau) b (stated after eq. 11 and after eq. 15).
 * A: m x n (lda >= n), y: m.  G is exactly symmetric.
 */
l0cim_status l0cim_gram(l0cim_dtype dtype, int32_t m, int32_t n, const void* A, int64_t lda,
                        const void* y, void* G, int64_t ldg, void* b, void* stream);

/*
 * l0cim_build_couplings -- J_rr' = -G_rr' R_r R_r' (r != r'), J_rr = 0, and
 * z_r = R_r b_r: the R-scaled couplings with which R_r h_r of eq. 15 is
 * (J (c + sqrt(tau))/4)_r + (sqrt(tau)/2) z_r and R_r h^BN_r of eq. 16 is
 * (sqrt(tau)/2)((J sigma)_r + z_r).
 * J is written in j_dtype with leading dim ldj (>= n):
 *   F32 (dtype F32) / F64 (dtype F64): exact elementwise product;
 *   BF16 / FP8E4M3 (dtype F32): row_scale[r] = max_r' |J_rr'| / Q_max
 *   (Q_max = 448 for FP8, 1 for BF16; 1 where the row is all zero) and the
 *   stored value is RNE(J_rr' / row_scale[r]) (FP8 saturating).
 * row_scale (float, n) is required for BF16/FP8 and ignored otherwise.
 */
l0cim_status l0cim_build_couplings(l0cim_dtype dtype, int32_t n, const void* G, int64_t ldg,
                                   const void* b, const void* R, l0cim_dtype j_dtype, void* J,
                                   int64_t ldj, float* row_scale, void* z, void* stream);

/*
 * l0cim_init_r -- the starting amplitudes of Algorithm 1 when the caller has
 * none: R_r = b_r / G_rr, the fixed point of the CDP step (below) for an empty
 * support; r with G_rr < 1e-12 get R_r = 0 and raise status bit TINY_DIAG.
 * G: n x n (ldg >= n), b: n, R: n, all in dtype (F32 or F64).  D_out (n, may
 * be NULL) receives the diagonal G_rr as a contiguous vector (for
 * l0cim_mri_mfcim_run).  status (int32, may be NULL) is OR-ed with L0CIM_ST_*
 * bits.  l0cim_solve applies the same rule where R_init is NULL.
 */
l0cim_status l0cim_init_r(l0cim_dtype dtype, int32_t n, const void* G, int64_t ldg, const void* b,
                          void* R, void* D_out, int32_t* status, void* stream);

/*
 * l0cim_init_state -- initial CIM state for alternation `alt`:
 * c[q][r] = c0_std * N(0,1) and e[q][r] = 1 (the vacuum-noise start stated
 * after eq. 16 and in Algorithm 1).  The normal draw is counter-based:
 * SplitMix64 outputs 2k+1 and 2k+2 of the stream keyed by `seed`, with
 * k = (alt << 40) | (q << 24) | r, as two 53-bit uniforms u1, u2 and
 * Box-Muller sqrt(-2 ln(1-u1)) cos(2 pi u2).  c, e: P x n, row stride n.
 */
l0cim_status l0cim_init_state(l0cim_dtype dtype, int32_t n, int32_t P, uint64_t seed, int32_t alt,
                              double c0_std, void* c, void* e, void* stream);

/*
 * l0cim_mfcim_run -- integrate the MFZ-CIM (eq. 12-14 with the field of
 * eq. 15 or 16 and the pump of eq. 21) for prm->n_steps forward-Euler steps
 * of P independent replicas, all sharing J and z:
 *   p_k  = (p_thr - d) + 2d / (1 + exp(-(k dt - t_c)/t_w))
 *   phi  = R h  (CN: J (c + sqrt tau)/4 + (sqrt tau/2) z;  BN: (sqrt tau/2)(J H(c) + z))
 *   c'   = c + dt [ (-1 + p_k - c^2) c + K j e (phi - eta^2 sqrt(tau)/4) ]
 *   e'   = e + dt [ -beta (c^2 - tau) e ]
 * c, e (P x n, row stride n) hold the initial state on entry and the final
 * state on exit.  sigma (P x n, uint8) receives H(c) = [c > 0] at the end.
 * H (P doubles, may be NULL) receives the eq. 4 energy of each sigma_q:
 * -1/2 s^T J s - z^T s + lambda 1^T s with lambda = eta^2/2.
 * trace (may be NULL): for k < trace_steps, trace[((k*2 + v)*P + q)*n + r] is
 * variable v (0: c, 1: e) of replica q after k+1 steps.
 * J: n x n in j_dtype (F32 or F64 matching dtype; BF16 / FP8 with row_scale,
 * dtype F32).  status (int32, may be NULL) is OR-ed with L0CIM_ST_* bits.
 */
size_t l0cim_mfcim_run_workspace_bytes(l0cim_dtype dtype, int32_t n, int32_t P, l0cim_dtype j_dtype);
l0cim_status l0cim_mfcim_run(l0cim_dtype dtype, int32_t n, int32_t P, l0cim_dtype j_dtype,
                             const void* J, int64_t ldj, const float* row_scale, const void* z,
                             double eta, const l0cim_cim_params* prm, void* c, void* e,
                             uint8_t* sigma, double* H, void* trace, int32_t trace_steps,
                             int32_t* status, void* ws, size_t ws_bytes, void* stream);

/*
 * l0cim_mfcim_run_noalloc -- l0cim_mfcim_run for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments and results without
 * ws / ws_bytes: the run's scratch (exchange words, abort word, per-workgroup
 * energies, the streamed form's copy of c) lives in a library-owned device
 * array of l0cim_noalloc_scratch_bytes() (8 MiB) that each device the library
 * runs on holds until the process ends.  The call allocates and frees
 * nothing.  The matrix-core launch form is never taken (its panel copy of J
 * would not fit): prm->launch = MATRIX returns L0CIM_ERR_UNSUPPORTED and AUTO
 * chooses among the other forms, which for a given problem are the ones
 * l0cim_mfcim_run takes whenever it does not take the matrix cores, with the
 * same bits.  A problem whose scratch exceeds the array returns
 * L0CIM_ERR_WORKSPACE before anything is enqueued; the scratch is 16 P n
 * bytes of exchange words (32 P n with FP64 state), 8 P n of energies and
 * P n state values, each rounded up to 256 bytes, plus 256 (FP32, P = 1:
 * n up to about 290 000).  Every call on one
 * device shares that device's array and leaves its contents behind (the
 * launch sequence itself clears what must start at zero): calls that overlap
 * on one device race, so serialise them (one stream, or events).
 */
size_t l0cim_noalloc_scratch_bytes(void);
l0cim_status l0cim_mfcim_run_noalloc(l0cim_dtype dtype, int32_t n, int32_t P, l0cim_dtype j_dtype,
                                     const void* J, int64_t ldj, const float* row_scale, const void* z,
                                     double eta, const l0cim_cim_params* prm, void* c, void* e,
                                     uint8_t* sigma, double* H, void* trace, int32_t trace_steps,
                                     int32_t* status, void* stream);

/*
 * MRI-shaped form.  A = S C Psi^T: Psi is the orthonormal 2-D Haar analysis
 * over `levels` levels in Mallat layout (coarsest block at the top left), C
 * the orthonormal 2-D DCT-II of the size x size image and S the sampled rows,
 * given as mask[f] (size^2 bytes, row-major frequency index
 * f = k_row * size + k_col, 1 where sampled) -- the sparse-MRI observation
 * model of the paper (wavelet-sparse image, undersampled frequency data).
 * The couplings are applied in factored form instead of a stored J:
 *   (J x)_r = -R_r (G_gamma (R o x))_r + D_r R_r^2 x_r,
 *   G_gamma = A^T A + gamma Psi (D_v^T D_v + D_h^T D_h) Psi^T,
 * J = -G_gamma o R R^T with a zero diagonal (eq. 13, 15, 16; eq. 20 for the
 * L2 term, whose weight gamma is 1e-4 in the paper's MRI runs).  D_v and D_h
 * are the vertical and horizontal second differences with the reflecting
 * boundary (x[-1] = x[0], x[S] = x[S-1]; the paper leaves the boundary rows
 * open); this operator is diagonal in the DCT-II basis, so G_gamma v =
 * Psi C^T diag(mask + gamma (lam_kr^2 + lam_kc^2)) C Psi^T v with
 * lam_k = 4 sin^2(pi k / (2 size)).  gamma = 0 gives A^T A exactly.
 * size must be 128 (L0CIM_ERR_UNSUPPORTED otherwise) and 2^levels <= size;
 * FP32 throughout.  The kernels hold the image in LDS (about 158 KB per
 * workgroup, gfx950's 160 KB; elsewhere the launch fails with L0CIM_ERR_HIP).
 *
 * l0cim_mri_mfcim_run -- the run of l0cim_mfcim_run (same dynamics, state
 * layout, sigma, H, trace and status) with these couplings.  D_r = G_gamma,rr
 * is read as D[r * incd] (incd = ldg + 1 reads the diagonal of a stored G in
 * place, 1 a vector; for gamma > 0 from l0cim_mri_l2_diag), b = A^T y (z =
 * R o b as in l0cim_build_couplings), R: n = size^2 floats; c, e: P x n.  One
 * workgroup per replica; no workspace.
 */
l0cim_status l0cim_mri_mfcim_run(int32_t size, int32_t levels, int32_t P, const uint8_t* mask,
                                 const float* R, const float* D, int64_t incd, const float* b,
                                 double gamma, double eta, const l0cim_cim_params* prm, float* c, float* e,
                                 uint8_t* sigma, double* H, float* trace, int32_t trace_steps,
                                 int32_t* status, void* stream);

/*
 * l0cim_mri_l2_diag -- D_out[r] = D_in[r * incd] + gamma [Psi (D_v^T D_v +
 * D_h^T D_h) Psi^T]_rr: the diagonal of G_gamma from that of A^T A.  The Haar
 * basis image of coefficient r is a product of two unit-norm 1-D Haar
 * functions v(row) h(col), so the added entry is ||D v||^2 + ||D h||^2,
 * evaluated in FP64 per coefficient.  D_out: size^2 floats (may not alias
 * D_in unless incd = 1).
 */
l0cim_status l0cim_mri_l2_diag(int32_t size, int32_t levels, double gamma, const float* D_in, int64_t incd,
                               float* D_out, void* stream);

/*
 * l0cim_mri_lasso -- the LASSO initial R of the paper's MRI runs: FISTA (Beck
 * and Teboulle) on (1/2) r^T G_gamma r - b^T r + lam1 ||r||_1 (eq. 18 with the
 * L0 term replaced by an L1 term, up to a constant) from r = 0, step
 * 1 / (1 + 32 gamma) (an upper bound of ||G_gamma||_2: A A^T = I and
 * ||D||_2 <= 4), `iters` iterations.  b = A^T y; R_out: size^2 floats.  One
 * workgroup.
 */
l0cim_status l0cim_mri_lasso(int32_t size, int32_t levels, double gamma, const uint8_t* mask, const float* b,
                             double lam1, int32_t iters, float* R_out, void* stream);

/*
 * l0cim_mri_update_r -- the CDP step of Algorithm 1 with G_gamma in factored
 * form, on support sigma (size^2 bytes):
 *   L0CIM_CDP_JACOBI: `iters` synchronous sweeps over every r,
 *     R_r <- R_r + dtc [(b_r - sum_{r' != r} G_rr' sigma_r' R_r') / G_rr - R_r];
 *   L0CIM_CDP_CG: conjugate gradients on (G_gamma)_SS R_S = b_S from the
 *     current R_S (the paper's MRI CDP, at most 10^4 iterations there) until
 *     ||residual|| <= cg_tol ||b_S|| or cg_max_iter iterations, dot products in
 *     FP64; then off the support R_r = (b_r - (G_gamma R_S)_r) / D_r, the
 *     Jacobi step's fixed point.  iters_out (device int32, may be NULL)
 *     receives the iteration count.
 * r with D_r < 1e-12 is held at 0 (status bit TINY_DIAG).  D as for
 * l0cim_mri_mfcim_run.  R (size^2) is read and overwritten.  One workgroup.
 */
l0cim_status l0cim_mri_update_r(int32_t size, int32_t levels, double gamma, const uint8_t* mask, const float* D,
                                int64_t incd, const float* b, const uint8_t* sigma, l0cim_cdp cdp, double dtc,
                                int32_t iters, int32_t cg_max_iter, double cg_tol, float* R, int32_t* iters_out,
                                int32_t* status, void* stream);

/*
 * CAC-CIM (Positive-P) form: the stochastic CIM the paper compares the
 * mean-field model against (eq. 5-11), as the sigma-minimiser of Algorithm 1
 * on the same couplings.  Per spin and replica: mean amplitude mu (eq. 5),
 * fluctuation variances n, m (eq. 6, 7), amplitude control e (eq. 9); the
 * field uses the measured amplitudes mu~ = mu + sqrt(g2/(4j)) W (eq. 10):
 *   R_r h_r = 1/2 (J (mu~ + sqrt(tau)))_r + sqrt(tau) z_r     (eq. 11),
 *   inj = j e (R h - sqrt(tau) eta^2 / 4)                    (eq. 8).
 * Forward Euler-Maruyama with time increment dt: one standard normal xi per
 * spin, replica and step, W taken as its step average xi / sqrt(dt) (noise
 * increment of eq. 5: sqrt(j g2)(m + n) xi sqrt(dt)), every right-hand side
 * at step k, pump of eq. 21 at t = k dt.  The normals are counter-based:
 * SplitMix64 keyed by mix64(seed ^ 0x6E6F6973655F7764), outputs 2 ctr + 1
 * and 2 ctr + 2 with ctr = (alt << 52) | (k << 32) | (q << 24) | r, two
 * 53-bit uniforms, Box-Muller in FP64.  A run starts from mu = n = m = 0 and
 * e = 1 (Algorithm 1) and returns sigma = H(mu) of the last step.
 */
typedef struct {
  double dt;                 /* 0.02 */
  int32_t n_steps;           /* Euler steps per run, < 2^20 - 1 */
  double p_thr, d, t_c, t_w; /* pump, eq. 21: 1, 0.4, 4, 2 */
  double K, j, beta;         /* feedback strength (1 for random data), out-coupling rate, CAC rate */
  double tau;                /* target amplitude: 0.21 (noise 0.05) or 0.15 (noise 0.1) */
  double g2;                 /* saturation parameter g^2 (1e-7) */
} l0cim_cac_params;

void l0cim_cac_params_default(l0cim_cac_params* p);

/*
 * l0cim_cac_run -- prm->n_steps steps of the CAC-CIM for P replicas (P <= 256)
 * sharing J (n x n, ldj >= n, zero diagonal) and z (n), both in dtype (F32 or
 * F64), at threshold eta; alternation index alt (0 .. 2047) and seed key the
 * noise.  mu, nvar, mvar, e: P x n outputs (final state); sigma: P x n bytes,
 * H(mu); H (P doubles, may be NULL): the eq. 4 energy of each sigma with
 * lambda = eta^2 / 2; trace (may be NULL): k x 4 x P x n values (mu, n, m, e
 * after step k + 1) for k < trace_steps.  ws: at least
 * l0cim_cac_run_workspace_bytes bytes (two buffers of measured amplitudes,
 * the energy terms and the exchange words of the one-launch form).  Each
 * wavefront owns one row of J.  With P <= 8 and n <= 2048 (F32; 1024 in
 * F64), when the device holds the n / 8 workgroups at once, the whole run is
 * one cooperative launch (rows of J in registers, the measured amplitudes of
 * each step exchanged between workgroups as step-tagged words); otherwise
 * one launch per Euler step.
 */
size_t l0cim_cac_run_workspace_bytes(l0cim_dtype dtype, int32_t n, int32_t P);
l0cim_status l0cim_cac_run(l0cim_dtype dtype, int32_t n, int32_t P, const void* J, int64_t ldj, const void* z,
                           double eta, const l0cim_cac_params* prm, uint64_t seed, int32_t alt, void* mu,
                           void* nvar, void* mvar, void* e, uint8_t* sigma, double* H, void* trace,
                           int32_t trace_steps, int32_t* status, void* ws, size_t ws_bytes, void* stream);

/*
 * l0cim_cac_solve -- Algorithm 1 with the CAC-CIM as the sigma-minimiser:
 * G, b = gram(A, y); R = b / diag(G); per alternation i < n_outer (at most
 * 2048): eta_i (eq. 22), J, z from R, l0cim_cac_run(seed, alt = i), the
 * lowest-energy replica, the Jacobi CDP (dtc, cdp_iters); then the eq. 3
 * objective into stats.  sp supplies the schedule, replicas, seed and CDP
 * constants (j_dtype and final_refit_f64 are not used).  ws: at least
 * l0cim_cac_solve_workspace_bytes bytes.
 */
size_t l0cim_cac_solve_workspace_bytes(l0cim_dtype dtype, int32_t m, int32_t n, int32_t P);
l0cim_status l0cim_cac_solve(l0cim_dtype dtype, int32_t m, int32_t n, const void* A, int64_t lda, const void* y,
                             const l0cim_cac_params* prm, const l0cim_solve_params* sp, void* R_out,
                             uint8_t* sigma_out, l0cim_stats* stats, void* ws, size_t ws_bytes, void* stream);

/* Parameters of the MRI-shaped solve. */
typedef struct {
  int32_t size;              /* image side (128) */
  int32_t levels;            /* Haar levels */
  double gamma;              /* L2 weight of eq. 18 / 20 (0: the plain couplings) */
  int32_t lasso_iters;       /* 0: R_init = b / D; > 0: LASSO start, this many FISTA iterations */
  double lasso_lam1;         /* L1 weight of the LASSO start */
  int32_t cdp;               /* L0CIM_CDP_JACOBI (dtc, cdp_iters of the solve params) or L0CIM_CDP_CG */
  int32_t cg_max_iter;       /* CG iteration cap (10^4 in the paper) */
  double cg_tol;             /* CG stop: ||residual|| <= cg_tol ||b_S|| */
} l0cim_mri_params;

void l0cim_mri_params_default(l0cim_mri_params* p);

/*
 * l0cim_mri_solve -- Algorithm 1 end to end on the MRI-shaped operator:
 *   b = A^T y, D = diag(A^T A) (FP64 sums over the stored A); D += gamma
 *   diag(L2 term) (l0cim_mri_l2_diag) if gamma > 0;
 *   R = LASSO (lasso_iters > 0) or b / D;
 *   for i < n_outer: eta_i (eq. 22), init_state(seed, i), mri_mfcim_run,
 *     select_replica (lambda_i = eta_i^2 / 2), mri_update_r (Jacobi or CG);
 *   optional FP64 refit on the final support (l0cim_refit_f64; gamma = 0
 *   only, L0CIM_ERR_UNSUPPORTED otherwise); stats as l0cim_solve's (E is the
 *   eq. 3 objective, without the L2 term).
 * A: m x size^2 (lda >= size^2) FP32 device memory, used for b, D, the refit
 * and E; sp supplies eta_init/eta_end/velo/n_outer, dtc/cdp_iters (Jacobi),
 * replicas, seed and final_refit_f64.  ws: at least
 * l0cim_mri_solve_workspace_bytes(m, replicas, final_refit_f64) bytes.
 */
size_t l0cim_mri_solve_workspace_bytes(int32_t m, int32_t P, int32_t final_refit_f64);
l0cim_status l0cim_mri_solve(const l0cim_mri_params* mp, int32_t m, const float* A, int64_t lda, const float* y,
                             const uint8_t* mask, const l0cim_cim_params* cim, const l0cim_solve_params* sp,
                             float* R_out, uint8_t* sigma_out, l0cim_stats* stats, void* ws, size_t ws_bytes,
                             void* stream);

/*
 * l0cim_mri_solve_many -- l0cim_mri_solve on `count` independent MRI-shaped
 * instances of one shape (Algorithm 1 for each, in lock step): instance k
 * reads A + k strideA (m x size^2, leading dimension lda; strideA = 0: one A
 * shared by all), y + k stridey (stridey >= m) and mask + k stride_mask
 * (stride_mask = 0: one mask shared, as for the slices of one acquisition),
 * draws its initial amplitudes with seeds[k] (host array; sp->seed is not
 * used), and writes R_out + k size^2, sigma_out + k size^2 and stats[k].
 * The factored CIM runs of all instances are one launch (count x replicas
 * workgroups, one per CU, so that several instances fill the device), and so
 * are the LASSO starts and the CDPs; each instance's result is the one
 * l0cim_mri_solve gives it alone (bitwise).  ws: at least
 * l0cim_mri_solve_many_workspace_bytes(count, m, replicas, final_refit_f64).
 */
size_t l0cim_mri_solve_many_workspace_bytes(int32_t count, int32_t m, int32_t P, int32_t final_refit_f64);
l0cim_status l0cim_mri_solve_many(const l0cim_mri_params* mp, int32_t count, int32_t m, const float* A, int64_t lda,
                                  int64_t strideA, const float* y, int64_t stridey, const uint8_t* mask,
                                  int64_t stride_mask, const uint64_t* seeds, const l0cim_cim_params* cim,
                                  const l0cim_solve_params* sp, float* R_out, uint8_t* sigma_out, l0cim_stats* stats,
                                  void* ws, size_t ws_bytes, void* stream);

/*
 * l0cim_select_replica -- q* = argmin_q H[q] (lowest q on ties, NaN never
 * chosen unless all are NaN) and sigma_out = sigma[q*] (n bytes).
 * q_out (int32, may be NULL) receives q*.
 */
l0cim_status l0cim_select_replica(int32_t n, int32_t P, const double* H, const uint8_t* sigma,
                                  uint8_t* sigma_out, int32_t* q_out, void* stream);

/*
 * l0cim_update_r -- the CDP step of Algorithm 1 on support sigma (n bytes).
 *   L0CIM_CDP_JACOBI: `iters` synchronous sweeps over every r,
 *     R_r <- R_r + dtc [ (b_r - sum_{r' != r} G_rr' sigma_r' R_r') / G_rr - R_r ];
 *   L0CIM_CDP_CHOL_F64: R_S = G_SS^-1 b_S through an FP64 Cholesky factor
 *     (ridge 1e-10 tr(G_SS)/|S| if a pivot is <= 1e-12 max diag, status bit
 *     CHOL_RIDGE), and R_r = (b_r - G_rS R_S) / G_rr off the support.
 * In both, r with G_rr < 1e-12 is held at 0 (status bit TINY_DIAG).
 * R (n) is read as the starting point and overwritten.
 */
size_t l0cim_update_r_workspace_bytes(l0cim_dtype dtype, int32_t n, l0cim_cdp cdp);
l0cim_status l0cim_update_r(l0cim_dtype dtype, int32_t n, const void* G, int64_t ldg, const void* b,
                            const uint8_t* sigma, l0cim_cdp cdp, double dtc, int32_t iters,
                            void* R, int32_t* status, void* ws, size_t ws_bytes, void* stream);

/*
 * l0cim_solve_many -- l0cim_solve on `count` independent instances of the
 * same m x n shape in lockstep: instance k reads A + k strideA (leading
 * dimension lda) and y + k stridey (elements of dtype), draws its initial
 * amplitudes with seeds[k] (host array; sp->seed is not used), and writes
 * R_out + k n, sigma_out + k n and stats[k]; R_init is b / diag(G) for every
 * instance.  Every step is l0cim_solve's, so each instance's result is the
 * one l0cim_solve gives it alone (bitwise).  Where the single-replica FP32
 * run takes its register-resident form, the CIM runs of all instances share
 * one cooperative launch, so their exchange round trips overlap; when the
 * instances do not all fit on the device at once (or another form applies)
 * they run one after another.  ws: at least l0cim_solve_many_workspace_bytes.
 */
size_t l0cim_solve_many_workspace_bytes(l0cim_dtype dtype, int32_t count, int32_t m, int32_t n,
                                        const l0cim_solve_params* sp);
l0cim_status l0cim_solve_many(l0cim_dtype dtype, int32_t count, int32_t m, int32_t n, const void* A, int64_t lda,
                              int64_t strideA, const void* y, int64_t stridey, const uint64_t* seeds,
                              const l0cim_cim_params* cim, const l0cim_solve_params* sp, void* R_out,
                              uint8_t* sigma_out, l0cim_stats* stats, void* ws, size_t ws_bytes, void* stream);

/*
 * l0cim_refit_f64 -- the least-squares refit of R on support sigma (the
 * R-minimisation of eq. 3 with sigma fixed; the final step of Algorithm 1 in
 * the precision form), with every quantity taken from A and y in FP64:
 *   G_SS = A_S^T A_S and b_S = A_S^T y accumulated in FP64 (products of FP32
 *   entries are exact in FP64), R_S = G_SS^-1 b_S through an FP64 Cholesky
 *   factor (ridge 1e-10 tr(G_SS)/|S| if a pivot is <= 1e-12 max diag, status
 *   bit CHOL_RIDGE), and off the support R_r = a_r^T (y - A_S R_S) / a_r^T a_r,
 *   which is (b_r - G_rS R_S) / G_rr; r with a_r^T a_r < 1e-12 is held at 0
 *   (status bit TINY_DIAG).  Unlike l0cim_update_r(CHOL_F64), an FP32 Gram's
 *   rounding does not enter the factor.
 * A: m x n row-major (leading dimension lda >= n), y: m, sigma: n bytes, R:
 * n (overwritten), all device memory of `dtype` (F32 or F64); status (device
 * int32, may be NULL) is OR-ed.  ws: device scratch of at least
 * l0cim_refit_f64_workspace_bytes(m, n) bytes (the padded factor,
 * round_up(n, 64)^2 doubles).  One cooperative launch on `stream`.
 */
size_t l0cim_refit_f64_workspace_bytes(int32_t m, int32_t n);
l0cim_status l0cim_refit_f64(l0cim_dtype dtype, int32_t m, int32_t n, const void* A, int64_t lda, const void* y,
                             const uint8_t* sigma, void* R, int32_t* status, void* ws, size_t ws_bytes,
                             void* stream);

/*
 * l0cim_solve -- Algorithm 1 end to end on one instance:
 *   G, b = gram(A, y);  R = R_init (or b_r / G_rr where R_init is NULL);
 *   for i < n_outer: eta_i (eq. 22); J, z = couplings(G, b, R);
 *     init_state(seed, i); mfcim_run; select_replica (lambda_i = eta_i^2/2);
 *     update_r(JACOBI, dtc, cdp_iters);
 *   optional FP64 Cholesky refit on the final support (l0cim_refit_f64: G_SS
 *   and b_S from A and y in FP64; the same with cdp = CHOL_F64 every
 *   alternation).
 * Outputs R_out (n, dtype), sigma_out (n bytes) and *stats (device memory).
 * A: m x n (lda >= n), y: m, R_init: n or NULL.
 */
size_t l0cim_solve_workspace_bytes(l0cim_dtype dtype, int32_t m, int32_t n,
                                   const l0cim_cim_params* cim, const l0cim_solve_params* sp);
l0cim_status l0cim_solve(l0cim_dtype dtype, int32_t m, int32_t n, const void* A, int64_t lda,
                         const void* y, const void* R_init, const l0cim_cim_params* cim,
                         const l0cim_solve_params* sp, void* R_out, uint8_t* sigma_out,
                         l0cim_stats* stats, void* ws, size_t ws_bytes, void* stream);

/*
 * Batched form: many instances of uneven size, each with P replicas, solved
 * together by Algorithm 1 (FP32 arithmetic; couplings F32, BF16 or FP8E4M3).
 * With several replicas the local field of every instance is the dense
 * product J X (N x N by N x P), done on the matrix cores with the Euler
 * update fused; one launch per Euler step covers every row tile of every
 * instance and the launches of one CIM run are replayed from a HIP graph.
 *
 * Instance k reads A_k at A_pool + a_offset (m x n, leading dim lda) and
 * y_k at y_pool + y_offset, and writes R_k (n floats) at R_pool + x_offset,
 * sigma_k (n bytes) at sigma_pool + x_offset and stats[k].  Its initial
 * amplitudes are keyed by `seed` exactly as l0cim_init_state, so an instance
 * gives the same result whatever else is in the batch.
 *
 * A plan holds host-side tables only; its workspace is the caller's.  The
 * first solve of a new shape class times the candidate tile shapes (it
 * synchronises the stream once) and remembers the fastest for the process.
 * Destroy a plan only after the work enqueued with it has completed.
 */
typedef struct {
  int32_t m, n;          /* measurement rows and spins (n <= 12288) */
  int64_t a_offset;      /* element offset of A_k in A_pool */
  int64_t lda;           /* leading dimension of A_k (>= n) */
  int64_t y_offset;      /* element offset of y_k in y_pool */
  int64_t x_offset;      /* element offset of R_k and byte offset of sigma_k */
  uint64_t seed;         /* key of the instance's initial-amplitude generator */
} l0cim_instance;

typedef struct l0cim_batch_plan_s* l0cim_batch_plan;

l0cim_status l0cim_batch_plan_create(int32_t count, const l0cim_instance* inst, const l0cim_cim_params* cim,
                                     const l0cim_solve_params* sp, l0cim_batch_plan* plan);
size_t l0cim_batch_plan_workspace_bytes(l0cim_batch_plan plan);
l0cim_status l0cim_batch_plan_info(l0cim_batch_plan plan, int32_t* rows_per_tile, int32_t* tiles,
                                   int32_t* tuned);
l0cim_status l0cim_batch_plan_destroy(l0cim_batch_plan plan);
l0cim_status l0cim_solve_batched(l0cim_batch_plan plan, const float* A_pool, const float* y_pool,
                                 float* R_pool, uint8_t* sigma_pool, l0cim_stats* stats, void* ws,
                                 size_t ws_bytes, void* stream);

/*
 * Stepwise batched solve (Algorithm 1 split at its alternation boundaries):
 * l0cim_solve_batched is exactly l0cim_batch_begin, then
 * l0cim_batch_alternations(0, n_outer), then l0cim_batch_finish, with the same
 * arguments.  A caller can enqueue the alternations in chunks (to time them,
 * or to inspect R and sigma between them); the device state between two
 * alternations is R (R_pool) and the workspace, and the next alternation
 * starts from R alone (its initial amplitudes come from the generator).
 *   begin:        uploads the tables, clears the stats, forms G = A^T A and
 *                 b = A^T y and R_init = b / diag(G) for every instance (and
 *                 times the tile shapes on the first solve of a shape class);
 *   alternations: alternations i0 <= i < i1 (0 <= i0 <= i1 <= n_outer) of
 *                 Algorithm 1: eta_i (eq. 22), couplings, initial state, the
 *                 CIM run, the lowest-energy replica (eq. 4) and the Jacobi CDP;
 *                 L0CIM_ERR_ARG for a range outside [0, n_outer] or when no
 *                 begin was enqueued on this workspace;
 *   finish:       the optional FP64 refit and the eq. 3 objective at
 *                 lambda = eta_{n_outer-1}^2 / 2 into the stats.
 * Every call must pass the pools and the workspace of the begin it follows.
 */
l0cim_status l0cim_batch_begin(l0cim_batch_plan plan, const float* A_pool, const float* y_pool, float* R_pool,
                               uint8_t* sigma_pool, l0cim_stats* stats, void* ws, size_t ws_bytes, void* stream);
l0cim_status l0cim_batch_alternations(l0cim_batch_plan plan, int32_t i0, int32_t i1, const float* A_pool,
                                      const float* y_pool, float* R_pool, uint8_t* sigma_pool, l0cim_stats* stats,
                                      void* ws, size_t ws_bytes, void* stream);
l0cim_status l0cim_batch_finish(l0cim_batch_plan plan, const float* A_pool, const float* y_pool, float* R_pool,
                                uint8_t* sigma_pool, l0cim_stats* stats, void* ws, size_t ws_bytes, void* stream);

/*
 * Serving form: continuous batching of solves over one device arena.
 *
 * A server runs Algorithm 1 (the batched form's kernels, one CIM
 * configuration and outer schedule for every request) on requests that
 * arrive over time.  Requests wait in arrival order until a slot is free and
 * their footprint fits in the arena (first fit); each l0cim_server_step then
 * advances every resident request by one alternation in shared launches,
 * each request with its own alternation index, eta_i (eq. 22) and seed, and
 * reports the requests that have completed n_outer alternations.  A
 * request's arithmetic does not depend on the other requests, so its result
 * is bitwise the same alone and in any mix.
 *
 * Memory: the arena (device, 256-byte aligned, caller-owned, untouched by
 * anyone else while the server lives) holds a head of
 * l0cim_server_arena_overhead() bytes and the requests' blocks of
 * l0cim_server_request_bytes() each: G, its support-compacted copy, J, A, y,
 * the per-spin vectors and the P x n state.  No call allocates device memory.
 *
 * submit: A (m x n, leading dim lda) and y (m) are device memory that must
 * stay valid until the request is reported; they are copied into the arena
 * when the request is admitted.  On completion R (n floats), sigma (n bytes)
 * and the stats are copied to R_out, sigma_out and stats_out.  Returns
 * L0CIM_ERR_WORKSPACE for a request larger than the whole arena heap, and
 * L0CIM_ERR_SHAPE for n above max_n.
 *
 * set_step_budget: a cap on the couplings bytes (round_up16(n) *
 * round_up32(n) * coupling size per request) that one Euler step of the
 * resident set streams; 0, the default, sets none.  The head of the queue
 * waits while admitting it would pass the cap, unless nothing is resident, so
 * a request alone always runs and no request overtakes another.  Once one
 * launch already streams enough bytes to keep HBM busy, more co-resident work
 * only lengthens every tick; the cap bounds that slowdown of the largest
 * requests, which set the tail latency.  Takes effect at the next admission.
 *
 * step: admission, one alternation, reports; enqueued on the server's stream
 * and waited for before it returns (the tick boundary is where requests join
 * and leave).  `completed` receives the number of requests reported.
 * After a device error the server refuses further work.
 *
 * completed: copies up to `max` completion records (oldest first) and drops
 * them from the server.  Times are seconds on the server's steady clock
 * (l0cim_server_clock, zero at creation).
 */
typedef struct l0cim_server_s* l0cim_server;

typedef struct {
  int64_t tag;           /* caller's request id */
  int32_t n, m;
  double t_submit;       /* when submit was called */
  double t_admit;        /* start of the tick that admitted it */
  double t_finish;       /* end of the tick that reported it */
} l0cim_completion;

size_t l0cim_server_request_bytes(int32_t m, int32_t n, const l0cim_solve_params* sp);
size_t l0cim_server_arena_overhead(int32_t max_slots, int32_t max_n, const l0cim_solve_params* sp);
l0cim_status l0cim_server_create(const l0cim_cim_params* cim, const l0cim_solve_params* sp, int32_t max_slots,
                                 int32_t max_n, void* arena, size_t arena_bytes, void* stream,
                                 l0cim_server* server);
double l0cim_server_clock(l0cim_server server);
l0cim_status l0cim_server_submit(l0cim_server server, int32_t m, int32_t n, const float* A, int64_t lda,
                                 const float* y, uint64_t seed, int64_t tag, float* R_out,
                                 uint8_t* sigma_out, l0cim_stats* stats_out);
l0cim_status l0cim_server_set_step_budget(l0cim_server server, size_t bytes);
l0cim_status l0cim_server_step(l0cim_server server, int32_t* completed);
int32_t l0cim_server_completed(l0cim_server server, l0cim_completion* out, int32_t max);
l0cim_status l0cim_server_info(l0cim_server server, int32_t* active, int32_t* pending, size_t* bytes_in_use,
                               size_t* heap_bytes, int64_t* ticks);
l0cim_status l0cim_server_destroy(l0cim_server server);

/*
 * The serving scheduler with no device: the same admission (arrival order,
 * a free slot, first fit in the arena heap, the step budget when set and
 * something is resident; the first request that does not fit stops
 * admission), slot reuse and retirement as l0cim_server_*, on request sizes
 * alone (l0cim_server_request_bytes), driven by the caller's clock.  For
 * sizing an arena, choosing slots and a step budget on the host, and testing
 * the scheduling without a GPU.  A tick admits at t_start, advances every
 * resident request by one alternation, and retires at t_end those that have
 * done n_outer.  l0cim_server_sim_resident fills up to `max` entries (tag,
 * slot, heap offset, alternations done) in resident order and returns the
 * resident count; free_blocks is the number of free heap extents.
 */
typedef struct l0cim_server_sim_s* l0cim_server_sim;
l0cim_status l0cim_server_sim_create(const l0cim_solve_params* sp, int32_t max_slots, int32_t max_n,
                                     size_t arena_bytes, l0cim_server_sim* sim);
l0cim_status l0cim_server_sim_submit(l0cim_server_sim sim, int32_t m, int32_t n, int64_t tag, double t_submit);
l0cim_status l0cim_server_sim_set_step_budget(l0cim_server_sim sim, size_t bytes);
l0cim_status l0cim_server_sim_tick(l0cim_server_sim sim, double t_start, double t_end, int32_t* admitted,
                                   int32_t* completed);
int32_t l0cim_server_sim_completed(l0cim_server_sim sim, l0cim_completion* out, int32_t max);
int32_t l0cim_server_sim_resident(l0cim_server_sim sim, int64_t* tags, int32_t* slots, size_t* offsets,
                                  int32_t* alternations, int32_t max);
l0cim_status l0cim_server_sim_info(l0cim_server_sim sim, int32_t* active, int32_t* pending, size_t* bytes_in_use,
                                   size_t* heap_bytes, int32_t* free_blocks);
l0cim_status l0cim_server_sim_destroy(l0cim_server_sim sim);

/*
 * Tile shape of the single-instance matrix-core run (several replicas): rows
 * of J per workgroup, 16 * RB with RB in {1, 2, 4, 8} (RB * ceil(P / 16) <= 16).
 * The first run of a new (n, P, coupling type, field) in a process times the
 * candidates on a few Euler steps (it synchronises the stream once, and is
 * skipped under stream capture) and remembers the fastest.  get returns the
 * remembered shape (0: none yet); set pins one for this process (0 forgets
 * it).  Invalid shapes return L0CIM_ERR_ARG.
 */
l0cim_status l0cim_matrix_tile_get(int32_t n, int32_t P, l0cim_dtype j_dtype, int32_t field, int32_t* rows);
l0cim_status l0cim_matrix_tile_set(int32_t n, int32_t P, l0cim_dtype j_dtype, int32_t field, int32_t rows);

/*
 * Kernel timing for measurement.  Between l0cim_profile_begin() and
 * l0cim_profile_end(), every launch of the CIM-run kernels made by this
 * thread is bracketed by HIP events on its own stream.  profile_end waits for
 * those events and returns the summed kernel time (ms) and launch count.
 */
l0cim_status l0cim_profile_begin(void);
l0cim_status l0cim_profile_end(double* cim_ms, int64_t* cim_launches);

#ifdef __cplusplus
}
#endif
#endif /* L0CIM_H */
