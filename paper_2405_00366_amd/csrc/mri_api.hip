// C entry points of the MRI-shaped form: the CIM run with the couplings in
// factored form (optionally L2-regularised, eq. 20), the diagonal of the
// regularised Gram matrix, the LASSO start, the CDP in factored form (Jacobi
// or conjugate gradients), and Algorithm 1 end to end on this operator.
#include <string.h>

#include "kernels.h"

namespace l0 {
namespace {

constexpr int kSide = 128;

__global__ void mri_stats_init_kernel(l0cim_stats* st) {
  st->status_bits = 0;
  st->selected_replica = 0;
  st->support_size = 0;
  st->n_outer_done = 0;
  st->H = 0.0;
  st->E = 0.0;
  st->spin_steps = 0;
}

l0cim_status check_geometry(int size, int levels, const char* who) {
  if (size != kSide) return set_error(L0CIM_ERR_UNSUPPORTED, "%s: image side %d (128 supported)", who, size);
  if (levels < 0 || levels > 7) return set_error(L0CIM_ERR_SHAPE, "%s: %d Haar levels", who, levels);
  return L0CIM_OK;
}

l0cim_status check_cim_params(const l0cim_cim_params* p, const char* who) {
  if (!p) return set_error(L0CIM_ERR_ARG, "%s: cim params is NULL", who);
  if (p->n_steps < 0 || p->n_steps > (1 << 30)) return set_error(L0CIM_ERR_ARG, "%s: n_steps out of range", who);
  if (p->field != L0CIM_FIELD_CN && p->field != L0CIM_FIELD_BN)
    return set_error(L0CIM_ERR_ARG, "%s: unknown field %d", who, p->field);
  if (!(p->dt > 0.0) || !(p->tau > 0.0) || !(p->t_w > 0.0))
    return set_error(L0CIM_ERR_ARG, "%s: dt, tau and t_w must be positive", who);
  return L0CIM_OK;
}

CimArgs mri_args(int n, int P, const l0cim_cim_params* p, double eta, int trace_steps) {
  CimArgs a{};
  a.n = n;
  a.P = P;
  a.n_steps = p->n_steps;
  a.trace_steps = trace_steps;
  a.field = p->field;
  a.linear_j = p->linear_j;
  a.launch = p->launch;
  a.dt = p->dt;
  a.p_thr = p->p_thr;
  a.d = p->d;
  a.t_c = p->t_c;
  a.t_w = p->t_w;
  a.K = p->K;
  a.j = p->j;
  a.beta = p->beta;
  a.tau = p->tau;
  a.eta = eta;
  a.spin_limit = p->spin_limit > 0 ? p->spin_limit : kDefaultSpinLimit;
  return a;
}

struct MriSolveLayout {
  size_t b, D0, D, c, e, sig, H, its, obj, chol, total;
};

MriSolveLayout mri_solve_layout(int m, int P, bool refit) {
  const int n = kSide * kSide;
  MriSolveLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  L.b = take(size_t(n) * 4);
  L.D0 = take(size_t(n) * 4);
  L.D = take(size_t(n) * 4);
  L.c = take(size_t(P) * n * 4);
  L.e = take(size_t(P) * n * 4);
  L.sig = take(size_t(P) * n);
  L.H = take(size_t(P) * 8);
  L.its = take(sizeof(int));
  L.obj = take(objective_ws_bytes(m));
  L.chol = take(refit ? chol_a_ws_bytes(n, m) : 0);
  L.total = o;
  return L;
}

// The argument checks of Algorithm 1 on the MRI-shaped operator (one
// instance or several of one shape).
l0cim_status check_mri_solve(const l0cim_mri_params* mp, int m, int64_t lda, const l0cim_cim_params* cim,
                             const l0cim_solve_params* sp, const char* who) {
  if (!mp || !sp) return set_error(L0CIM_ERR_ARG, "%s: NULL parameters", who);
  l0cim_status st = check_geometry(mp->size, mp->levels, who);
  if (st != L0CIM_OK) return st;
  st = check_cim_params(cim, who);
  if (st != L0CIM_OK) return st;
  const int n = mp->size * mp->size;
  if (m <= 0 || lda < n) return set_error(L0CIM_ERR_SHAPE, "%s: bad shape", who);
  const int P = sp->replicas;
  if (P <= 0 || P > (1 << 16)) return set_error(L0CIM_ERR_ARG, "%s: replicas out of range", who);
  if (sp->n_outer <= 0 || sp->n_outer >= (1 << 24) || sp->velo <= 0)
    return set_error(L0CIM_ERR_ARG, "%s: n_outer and velo must be positive", who);
  if (!(mp->gamma >= 0.0) || mp->lasso_iters < 0 || !(mp->lasso_lam1 >= 0.0))
    return set_error(L0CIM_ERR_ARG, "%s: gamma, lasso_iters and lasso_lam1 must be >= 0", who);
  if (mp->cdp == L0CIM_CDP_JACOBI) {
    if (sp->cdp_iters < 0) return set_error(L0CIM_ERR_ARG, "%s: cdp_iters < 0", who);
  } else if (mp->cdp == L0CIM_CDP_CG) {
    if (mp->cg_max_iter < 0 || !(mp->cg_tol >= 0.0)) return set_error(L0CIM_ERR_ARG, "%s: bad CG limits", who);
  } else {
    return set_error(L0CIM_ERR_UNSUPPORTED, "%s: cdp %d (Jacobi or CG)", who, mp->cdp);
  }
  if (sp->final_refit_f64 && mp->gamma != 0.0)
    return set_error(L0CIM_ERR_UNSUPPORTED, "%s: the FP64 refit is the unregularised least squares (gamma = 0)", who);
  return L0CIM_OK;
}

// Pools of the many-instance solve: each array holds the `count` instances'
// blocks back to back, so that one launch can address every instance at a
// fixed stride.
struct MriManyLayout {
  size_t b, D0, D, c, e, sig, H, its, obj, chol, total;
  size_t sobj, schol;   // bytes of one instance's objective scratch and of the refit scratch
};

MriManyLayout mri_many_layout(int count, int m, int P, bool refit) {
  const size_t n = size_t(kSide) * kSide;
  MriManyLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  L.sobj = align_up(objective_ws_bytes(m));
  L.schol = refit ? align_up(chol_a_ws_bytes(int(n), m)) : 0;
  L.b = take(count * n * 4);
  L.D0 = take(count * n * 4);
  L.D = take(count * n * 4);
  L.c = take(count * size_t(P) * n * 4);
  L.e = take(count * size_t(P) * n * 4);
  L.sig = take(count * size_t(P) * n);
  L.H = take(count * size_t(P) * 8);
  L.its = take(count * sizeof(int));
  L.obj = take(count * L.sobj);
  L.chol = take(L.schol);   // the refits run one after another on the stream and share it
  L.total = o;
  return L;
}

}  // namespace
}  // namespace l0

using namespace l0;

extern "C" {

void l0cim_mri_params_default(l0cim_mri_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->size = kSide;
  p->levels = 3;
  p->gamma = 0.0;
  p->lasso_iters = 0;
  p->lasso_lam1 = 3e-4;
  p->cdp = L0CIM_CDP_JACOBI;
  p->cg_max_iter = 10000;
  p->cg_tol = 1e-5;
}

l0cim_status l0cim_mri_mfcim_run(int32_t size, int32_t levels, int32_t P, const uint8_t* mask, const float* R,
                                 const float* D, int64_t incd, const float* b, double gamma, double eta,
                                 const l0cim_cim_params* prm, float* c, float* e, uint8_t* sigma, double* H,
                                 float* trace, int32_t trace_steps, int32_t* status, void* stream) {
  l0cim_status st = check_cim_params(prm, "mri_mfcim_run");
  if (st != L0CIM_OK) return st;
  if (!mask || !R || !D || !b || !c || !e || !sigma) return set_error(L0CIM_ERR_ARG, "mri_mfcim_run: NULL pointer");
  if (size <= 0 || P <= 0 || P > (1 << 16) || incd < 1) return set_error(L0CIM_ERR_SHAPE, "mri_mfcim_run: bad shape");
  if (levels < 0 || levels > 30 || (1 << levels) > size)
    return set_error(L0CIM_ERR_SHAPE, "mri_mfcim_run: %d Haar levels", levels);
  if (!(gamma >= 0.0)) return set_error(L0CIM_ERR_ARG, "mri_mfcim_run: gamma must be >= 0");
  if (trace_steps < 0 || (trace_steps > 0 && !trace))
    return set_error(L0CIM_ERR_ARG, "mri_mfcim_run: trace_steps > 0 needs a trace buffer");
  const int n = size * size;
  CimArgs a = mri_args(n, P, prm, eta, trace_steps < prm->n_steps ? trace_steps : prm->n_steps);
  return launch_mri_mfcim(size, levels, P, mask, R, D, incd, b, gamma, a, c, e, sigma, H, trace, status,
                          static_cast<hipStream_t>(stream));
}

l0cim_status l0cim_mri_l2_diag(int32_t size, int32_t levels, double gamma, const float* D_in, int64_t incd,
                               float* D_out, void* stream) {
  l0cim_status st = check_geometry(size, levels, "mri_l2_diag");
  if (st != L0CIM_OK) return st;
  if (!D_in || !D_out) return set_error(L0CIM_ERR_ARG, "mri_l2_diag: NULL pointer");
  if (incd < 1) return set_error(L0CIM_ERR_SHAPE, "mri_l2_diag: incd < 1");
  if (!(gamma >= 0.0)) return set_error(L0CIM_ERR_ARG, "mri_l2_diag: gamma must be >= 0");
  return launch_mri_l2_diag(size, levels, gamma, D_in, incd, D_out, static_cast<hipStream_t>(stream));
}

l0cim_status l0cim_mri_lasso(int32_t size, int32_t levels, double gamma, const uint8_t* mask, const float* b,
                             double lam1, int32_t iters, float* R_out, void* stream) {
  l0cim_status st = check_geometry(size, levels, "mri_lasso");
  if (st != L0CIM_OK) return st;
  if (!mask || !b || !R_out) return set_error(L0CIM_ERR_ARG, "mri_lasso: NULL pointer");
  if (!(gamma >= 0.0) || !(lam1 >= 0.0) || iters < 0)
    return set_error(L0CIM_ERR_ARG, "mri_lasso: gamma, lam1 and iters must be >= 0");
  return launch_mri_lasso(size, levels, gamma, mask, b, lam1, iters, R_out, static_cast<hipStream_t>(stream));
}

l0cim_status l0cim_mri_update_r(int32_t size, int32_t levels, double gamma, const uint8_t* mask, const float* D,
                                int64_t incd, const float* b, const uint8_t* sigma, l0cim_cdp cdp, double dtc,
                                int32_t iters, int32_t cg_max_iter, double cg_tol, float* R, int32_t* iters_out,
                                int32_t* status, void* stream) {
  l0cim_status st = check_geometry(size, levels, "mri_update_r");
  if (st != L0CIM_OK) return st;
  if (!mask || !D || !b || !sigma || !R) return set_error(L0CIM_ERR_ARG, "mri_update_r: NULL pointer");
  if (incd < 1) return set_error(L0CIM_ERR_SHAPE, "mri_update_r: incd < 1");
  if (!(gamma >= 0.0)) return set_error(L0CIM_ERR_ARG, "mri_update_r: gamma must be >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (cdp == L0CIM_CDP_JACOBI) {
    if (iters < 0) return set_error(L0CIM_ERR_ARG, "mri_update_r: iters < 0");
    return launch_mri_jacobi(size, levels, gamma, mask, D, incd, b, sigma, R, iters, dtc, status, s);
  }
  if (cdp == L0CIM_CDP_CG) {
    if (cg_max_iter < 0 || !(cg_tol >= 0.0)) return set_error(L0CIM_ERR_ARG, "mri_update_r: bad CG limits");
    return launch_mri_cg(size, levels, gamma, mask, D, incd, b, sigma, R, cg_max_iter, cg_tol, iters_out, status, s);
  }
  return set_error(L0CIM_ERR_UNSUPPORTED, "mri_update_r: cdp %d (Jacobi or CG)", int(cdp));
}

size_t l0cim_mri_solve_workspace_bytes(int32_t m, int32_t P, int32_t final_refit_f64) {
  if (m <= 0 || P <= 0) return 0;
  return mri_solve_layout(m, P, final_refit_f64 != 0).total;
}

l0cim_status l0cim_mri_solve(const l0cim_mri_params* mp, int32_t m, const float* A, int64_t lda, const float* y,
                             const uint8_t* mask, const l0cim_cim_params* cim, const l0cim_solve_params* sp,
                             float* R_out, uint8_t* sigma_out, l0cim_stats* stats, void* ws, size_t ws_bytes,
                             void* stream) {
  l0cim_status st = check_mri_solve(mp, m, lda, cim, sp, "mri_solve");
  if (st != L0CIM_OK) return st;
  if (!A || !y || !mask || !R_out || !sigma_out || !stats) return set_error(L0CIM_ERR_ARG, "mri_solve: NULL pointer");
  const int n = mp->size * mp->size;
  const int P = sp->replicas;
  const MriSolveLayout L = mri_solve_layout(m, P, sp->final_refit_f64 != 0);
  if (!ws || ws_bytes < L.total) return set_error(L0CIM_ERR_WORKSPACE, "mri_solve: workspace needs %zu bytes", L.total);

  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  float* b = reinterpret_cast<float*>(base + L.b);
  float* D0 = reinterpret_cast<float*>(base + L.D0);
  float* D = mp->gamma != 0.0 ? reinterpret_cast<float*>(base + L.D) : D0;
  float* c = reinterpret_cast<float*>(base + L.c);
  float* e = reinterpret_cast<float*>(base + L.e);
  uint8_t* sig = reinterpret_cast<uint8_t*>(base + L.sig);
  double* H = reinterpret_cast<double*>(base + L.H);
  int* its = reinterpret_cast<int*>(base + L.its);
  int* status = &stats->status_bits;
#define L0_TRY(x)                  \
  do {                             \
    l0cim_status _s = (x);         \
    if (_s != L0CIM_OK) return _s; \
  } while (0)
  hipLaunchKernelGGL(mri_stats_init_kernel, dim3(1), dim3(1), 0, s, stats);
  L0_LAUNCHED("mri_stats_init_kernel");
  L0_TRY(launch_mri_aty_colnorm(m, n, A, lda, y, b, D0, s));
  if (mp->gamma != 0.0) L0_TRY(launch_mri_l2_diag(mp->size, mp->levels, mp->gamma, D0, 1, D, s));
  if (mp->lasso_iters > 0)
    L0_TRY(launch_mri_lasso(mp->size, mp->levels, mp->gamma, mask, b, mp->lasso_lam1, mp->lasso_iters, R_out, s));
  else
    L0_TRY(launch_mri_r_init(n, b, D, R_out, status, s));
  double eta = sp->eta_init;
  for (int i = 0; i < sp->n_outer; ++i) {
    const double v = sp->eta_init * (1.0 - double(i) / double(sp->velo));
    eta = v > sp->eta_end ? v : sp->eta_end;
    L0_TRY(launch_init_state(L0CIM_F32, n, P, sp->seed, i, cim->c0_std, c, e, s));
    const CimArgs a = mri_args(n, P, cim, eta, 0);
    L0_TRY(launch_mri_mfcim(mp->size, mp->levels, P, mask, R_out, D, 1, b, mp->gamma, a, c, e, sig, H, nullptr,
                            status, s));
    L0_TRY(launch_select(n, P, H, sig, sigma_out, &stats->selected_replica, &stats->H, s));
    if (mp->cdp == L0CIM_CDP_CG)
      L0_TRY(launch_mri_cg(mp->size, mp->levels, mp->gamma, mask, D, 1, b, sigma_out, R_out, mp->cg_max_iter,
                           mp->cg_tol, its, status, s));
    else
      L0_TRY(launch_mri_jacobi(mp->size, mp->levels, mp->gamma, mask, D, 1, b, sigma_out, R_out, sp->cdp_iters,
                               sp->dtc, status, s));
  }
  if (sp->final_refit_f64)
    L0_TRY(launch_chol_refit_a(L0CIM_F32, m, n, A, lda, y, sigma_out, R_out, status, base + L.chol,
                               chol_a_ws_bytes(n, m), s));
  const int64_t spin_steps = int64_t(n) * P * cim->n_steps * sp->n_outer;
  L0_TRY(launch_objective(L0CIM_F32, m, n, A, lda, y, sigma_out, R_out, 0.5 * eta * eta, stats, spin_steps,
                          sp->n_outer, base + L.obj, objective_ws_bytes(m), s));
#undef L0_TRY
  return L0CIM_OK;
}

size_t l0cim_mri_solve_many_workspace_bytes(int32_t count, int32_t m, int32_t P, int32_t final_refit_f64) {
  if (count <= 0 || m <= 0 || P <= 0) return 0;
  return mri_many_layout(count, m, P, final_refit_f64 != 0).total;
}

l0cim_status l0cim_mri_solve_many(const l0cim_mri_params* mp, int32_t count, int32_t m, const float* A, int64_t lda,
                                  int64_t strideA, const float* y, int64_t stridey, const uint8_t* mask,
                                  int64_t stride_mask, const uint64_t* seeds, const l0cim_cim_params* cim,
                                  const l0cim_solve_params* sp, float* R_out, uint8_t* sigma_out, l0cim_stats* stats,
                                  void* ws, size_t ws_bytes, void* stream) {
  l0cim_status st = check_mri_solve(mp, m, lda, cim, sp, "mri_solve_many");
  if (st != L0CIM_OK) return st;
  if (!A || !y || !mask || !seeds || !R_out || !sigma_out || !stats)
    return set_error(L0CIM_ERR_ARG, "mri_solve_many: NULL pointer");
  const int n = mp->size * mp->size;
  if (count <= 0 || count > 4096) return set_error(L0CIM_ERR_ARG, "mri_solve_many: count must be 1..4096");
  if (strideA < 0 || (strideA > 0 && strideA < int64_t(m) * lda) || stridey < m ||
      (stride_mask != 0 && stride_mask < n))
    return set_error(L0CIM_ERR_SHAPE, "mri_solve_many: bad stride");
  const int P = sp->replicas;
  const bool refit = sp->final_refit_f64 != 0;
  const MriManyLayout L = mri_many_layout(count, m, P, refit);
  if (!ws || ws_bytes < L.total)
    return set_error(L0CIM_ERR_WORKSPACE, "mri_solve_many: workspace needs %zu bytes", L.total);

  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  float* b = reinterpret_cast<float*>(base + L.b);
  float* D0 = reinterpret_cast<float*>(base + L.D0);
  float* D = mp->gamma != 0.0 ? reinterpret_cast<float*>(base + L.D) : D0;
  float* c = reinterpret_cast<float*>(base + L.c);
  float* e = reinterpret_cast<float*>(base + L.e);
  uint8_t* sig = reinterpret_cast<uint8_t*>(base + L.sig);
  double* H = reinterpret_cast<double*>(base + L.H);
  int* its = reinterpret_cast<int*>(base + L.its);
  const size_t pn = size_t(P) * n;
  auto Ak = [&](int k) { return A + size_t(k) * strideA; };
  auto yk = [&](int k) { return y + size_t(k) * stridey; };
  MriStrides ms;
  ms.mask = stride_mask;
  ms.vec = n;
  ms.D = n;
  ms.state = int64_t(pn);
  ms.H = P;
  ms.status = int64_t(sizeof(l0cim_stats) / sizeof(int32_t));
  ms.it = 1;
#define L0_TRY(x)                  \
  do {                             \
    l0cim_status _s = (x);         \
    if (_s != L0CIM_OK) return _s; \
  } while (0)
  for (int k = 0; k < count; ++k) {
    hipLaunchKernelGGL(mri_stats_init_kernel, dim3(1), dim3(1), 0, s, stats + k);
    L0_LAUNCHED("mri_stats_init_kernel");
    L0_TRY(launch_mri_aty_colnorm(m, n, Ak(k), lda, yk(k), b + size_t(k) * n, D0 + size_t(k) * n, s));
    if (mp->gamma != 0.0)
      L0_TRY(launch_mri_l2_diag(mp->size, mp->levels, mp->gamma, D0 + size_t(k) * n, 1, D + size_t(k) * n, s));
    if (mp->lasso_iters <= 0)
      L0_TRY(launch_mri_r_init(n, b + size_t(k) * n, D + size_t(k) * n, R_out + size_t(k) * n, &stats[k].status_bits,
                               s));
  }
  if (mp->lasso_iters > 0)
    L0_TRY(launch_mri_lasso(mp->size, mp->levels, mp->gamma, mask, b, mp->lasso_lam1, mp->lasso_iters, R_out, s,
                            count, ms));
  double eta = sp->eta_init;
  for (int i = 0; i < sp->n_outer; ++i) {
    const double v = sp->eta_init * (1.0 - double(i) / double(sp->velo));
    eta = v > sp->eta_end ? v : sp->eta_end;
    for (int k = 0; k < count; ++k)
      L0_TRY(launch_init_state(L0CIM_F32, n, P, seeds[k], i, cim->c0_std, c + k * pn, e + k * pn, s));
    const CimArgs a = mri_args(n, P, cim, eta, 0);
    L0_TRY(launch_mri_mfcim(mp->size, mp->levels, P, mask, R_out, D, 1, b, mp->gamma, a, c, e, sig, H, nullptr,
                            &stats[0].status_bits, s, count, ms));
    for (int k = 0; k < count; ++k)
      L0_TRY(launch_select(n, P, H + size_t(k) * P, sig + k * pn, sigma_out + size_t(k) * n,
                           &stats[k].selected_replica, &stats[k].H, s));
    if (mp->cdp == L0CIM_CDP_CG)
      L0_TRY(launch_mri_cg(mp->size, mp->levels, mp->gamma, mask, D, 1, b, sigma_out, R_out, mp->cg_max_iter,
                           mp->cg_tol, its, &stats[0].status_bits, s, count, ms));
    else
      L0_TRY(launch_mri_jacobi(mp->size, mp->levels, mp->gamma, mask, D, 1, b, sigma_out, R_out, sp->cdp_iters,
                               sp->dtc, &stats[0].status_bits, s, count, ms));
  }
  const int64_t spin_steps = int64_t(n) * P * cim->n_steps * sp->n_outer;
  for (int k = 0; k < count; ++k) {
    float* Rk = R_out + size_t(k) * n;
    uint8_t* sk = sigma_out + size_t(k) * n;
    if (refit)
      L0_TRY(launch_chol_refit_a(L0CIM_F32, m, n, Ak(k), lda, yk(k), sk, Rk, &stats[k].status_bits,
                                 base + L.chol, L.schol, s));
    L0_TRY(launch_objective(L0CIM_F32, m, n, Ak(k), lda, yk(k), sk, Rk, 0.5 * eta * eta, stats + k, spin_steps,
                            sp->n_outer, base + L.obj + k * L.sobj, L.sobj, s));
  }
#undef L0_TRY
  return L0CIM_OK;
}

}  // extern "C"
