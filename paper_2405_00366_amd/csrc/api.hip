// C ABI of the l0cim library: argument checking, workspace carving and the
// host-side sequence of Algorithm 1.  All device work is enqueued on the
// caller's stream; nothing here synchronises except l0cim_profile_end.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "kernels.h"

namespace l0 {

namespace {
thread_local char g_err[512] = "";

struct ProfState {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
};
thread_local ProfState g_prof;

std::mutex g_dev_mu;
DeviceInfo g_dev_cache[64];
bool g_dev_valid[64] = {};
}  // namespace

l0cim_status set_error(l0cim_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

l0cim_status hip_fail(hipError_t e, const char* what) {
  return set_error(L0CIM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

l0cim_status device_info(DeviceInfo* out) {
  int dev = 0;
  L0_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return set_error(L0CIM_ERR_HIP, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_dev_mu);
  if (!g_dev_valid[dev]) {
    DeviceInfo d;
    d.device = dev;
    L0_HIP(hipDeviceGetAttribute(&d.cu_count, hipDeviceAttributeMultiprocessorCount, dev));
    int lds = 0;
    L0_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    d.max_lds = lds < kMaxLdsBytes ? lds : kMaxLdsBytes;
    g_dev_cache[dev] = d;
    g_dev_valid[dev] = true;
  }
  *out = g_dev_cache[dev];
  return L0CIM_OK;
}

ProfileScope::ProfileScope(hipStream_t s) : stream(s), ev0(nullptr) {
  if (!g_prof.on) return;
  hipEvent_t e;
  if (hipEventCreate(&e) == hipSuccess && hipEventRecord(e, s) == hipSuccess) ev0 = e;
}

ProfileScope::~ProfileScope() {
  if (!ev0) return;
  hipEvent_t e1;
  if (hipEventCreate(&e1) == hipSuccess && hipEventRecord(e1, stream) == hipSuccess)
    g_prof.events.emplace_back(static_cast<hipEvent_t>(ev0), e1);
}

namespace {

__global__ void stats_init_kernel(l0cim_stats* st) {
  st->status_bits = 0;
  st->selected_replica = 0;
  st->support_size = 0;
  st->n_outer_done = 0;
  st->H = 0.0;
  st->E = 0.0;
  st->spin_steps = 0;
}

bool is_state_dtype(l0cim_dtype d) { return d == L0CIM_F32 || d == L0CIM_F64; }

l0cim_status check_jdtype(l0cim_dtype dt, l0cim_dtype jdt) {
  if (dt == L0CIM_F32 && (jdt == L0CIM_F32 || jdt == L0CIM_BF16 || jdt == L0CIM_FP8E4M3)) return L0CIM_OK;
  if (dt == L0CIM_F64 && jdt == L0CIM_F64) return L0CIM_OK;
  return set_error(L0CIM_ERR_UNSUPPORTED, "coupling dtype %d with arithmetic dtype %d", int(jdt), int(dt));
}

l0cim_status check_cim(const l0cim_cim_params* p) {
  if (!p) return set_error(L0CIM_ERR_ARG, "cim params is NULL");
  if (p->n_steps < 0) return set_error(L0CIM_ERR_ARG, "n_steps < 0");
  if (p->n_steps > (1 << 30)) return set_error(L0CIM_ERR_ARG, "n_steps too large");
  if (p->field != L0CIM_FIELD_CN && p->field != L0CIM_FIELD_BN)
    return set_error(L0CIM_ERR_ARG, "unknown field %d", p->field);
  if (!(p->dt > 0.0) || !(p->tau > 0.0) || !(p->t_w > 0.0))
    return set_error(L0CIM_ERR_ARG, "dt, tau and t_w must be positive");
  if (p->spin_limit < 0) return set_error(L0CIM_ERR_ARG, "spin_limit < 0");
  if (p->launch < L0CIM_LAUNCH_AUTO || p->launch > L0CIM_LAUNCH_MATRIX)
    return set_error(L0CIM_ERR_ARG, "unknown launch shape %d", p->launch);
  return L0CIM_OK;
}

CimArgs make_args(int n, int P, const l0cim_cim_params* p, double eta, int trace_steps) {
  CimArgs a;
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

double eta_at(const l0cim_solve_params* sp, int i) {
  double v = sp->eta_init * (1.0 - double(i) / double(sp->velo));
  return v > sp->eta_end ? v : sp->eta_end;
}

struct SolveLayout {
  size_t G, b, J, rs, z, c, e, sig, H, run, cdp, obj, total;
  size_t run_bytes, cdp_bytes, obj_bytes;
};

SolveLayout solve_layout(l0cim_dtype dt, int m, int n, int P, l0cim_dtype jdt, bool chol) {
  SolveLayout L;
  const size_t ts = dtype_size(dt);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  L.G = take(size_t(n) * n * ts);
  L.b = take(size_t(n) * ts);
  L.J = take(size_t(n) * n * dtype_size(jdt));
  L.rs = take(size_t(n) * sizeof(float));
  L.z = take(size_t(n) * ts);
  L.c = take(size_t(P) * n * ts);
  L.e = take(size_t(P) * n * ts);
  L.sig = take(size_t(P) * n);
  L.H = take(size_t(P) * sizeof(double));
  L.run_bytes = mfcim_ws_bytes(dt, n, P);
  L.run = take(L.run_bytes);
  L.cdp_bytes = jacobi_ws_bytes(dt, n);
  if (chol && chol_a_ws_bytes(n, m) > L.cdp_bytes) L.cdp_bytes = chol_a_ws_bytes(n, m);
  L.cdp = take(L.cdp_bytes);
  L.obj_bytes = objective_ws_bytes(m);
  L.obj = take(L.obj_bytes);
  L.total = o;
  return L;
}

}  // namespace

l0cim_status mfcim_run_checked(l0cim_dtype dtype, int n, int P, l0cim_dtype j_dtype, const void* J, int64_t ldj,
                               const float* row_scale, const void* z, double eta, const l0cim_cim_params* prm,
                               void* c, void* e, uint8_t* sigma, double* H, void* trace, int trace_steps,
                               int* status, void* ws, size_t ws_bytes, bool allow_matrix, hipStream_t s) {
  if (!is_state_dtype(dtype)) return set_error(L0CIM_ERR_UNSUPPORTED, "mfcim_run: dtype %d", int(dtype));
  l0cim_status st = check_jdtype(dtype, j_dtype);
  if (st != L0CIM_OK) return st;
  st = check_cim(prm);
  if (st != L0CIM_OK) return st;
  if (!J || !z || !c || !e || !sigma) return set_error(L0CIM_ERR_ARG, "mfcim_run: NULL pointer");
  if ((j_dtype == L0CIM_BF16 || j_dtype == L0CIM_FP8E4M3) && !row_scale)
    return set_error(L0CIM_ERR_ARG, "mfcim_run: row_scale required for BF16/FP8");
  if (n <= 0 || P <= 0 || ldj < n) return set_error(L0CIM_ERR_SHAPE, "mfcim_run: bad shape");
  if (trace_steps < 0 || (trace_steps > 0 && !trace))
    return set_error(L0CIM_ERR_ARG, "mfcim_run: trace_steps > 0 needs a trace buffer");
  const size_t need = allow_matrix ? mfcim_ws_bytes(dtype, n, P) : mfcim_base_ws_bytes(dtype, n, P);
  if (!ws || ws_bytes < need) return set_error(L0CIM_ERR_WORKSPACE, "mfcim_run: workspace needs %zu bytes", need);
  CimArgs a = make_args(n, P, prm, eta, trace_steps < prm->n_steps ? trace_steps : prm->n_steps);
  return launch_mfcim(dtype, n, P, j_dtype, J, ldj,
                      j_dtype == L0CIM_F32 || j_dtype == L0CIM_F64 ? nullptr : row_scale, z, a, c, e, sigma, H,
                      trace, status, ws, ws_bytes, s, allow_matrix);
}

}  // namespace l0

using namespace l0;

namespace {

// Pools of the many-instance solve: every array holds `count` per-instance
// blocks at a fixed stride, so that one launch can address all instances.
struct ManyLayout {
  size_t G, b, J, rs, z, c, e, sig, H, run, cdp, obj, total;
  size_t sG, sb, sv, sJ, sH, srun, scdp, sobj;   // per-instance strides (bytes; sv in elements)
};

ManyLayout many_layout(l0cim_dtype dt, int count, int m, int n, int P, l0cim_dtype jdt, bool chol) {
  ManyLayout L;
  const size_t ts = dtype_size(dt);
  L.sG = align_up(size_t(n) * n * ts);
  L.sb = align_up(size_t(n) * ts);
  L.sv = align_up(size_t(P) * n * 8) / 8;          // elements, the same for float and double vectors
  L.sJ = size_t(n) * n;                            // elements (ldj = n)
  L.sH = align_up(size_t(P) * sizeof(double));
  L.srun = align_up(mfcim_ws_bytes(dt, n, P));
  size_t cdp = jacobi_ws_bytes(dt, n);
  if (chol && chol_a_ws_bytes(n, m) > cdp) cdp = chol_a_ws_bytes(n, m);
  L.scdp = align_up(cdp);
  L.sobj = align_up(objective_ws_bytes(m));
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  L.G = take(count * L.sG);
  L.b = take(count * L.sb);
  L.J = take(count * L.sJ * dtype_size(jdt));
  L.rs = take(count * L.sv * sizeof(float));
  L.z = take(count * L.sv * ts);
  L.c = take(count * L.sv * ts);
  L.e = take(count * L.sv * ts);
  L.sig = take(count * L.sv);
  L.H = take(count * L.sH);
  L.run = take(count * L.srun);
  L.cdp = take(count * L.scdp);
  L.obj = take(count * L.sobj);
  L.total = o;
  return L;
}

}  // namespace

extern "C" {

int l0cim_version(void) { return L0CIM_VERSION; }

const char* l0cim_status_string(l0cim_status s) {
  switch (s) {
    case L0CIM_OK: return "ok";
    case L0CIM_ERR_ARG: return "invalid argument";
    case L0CIM_ERR_SHAPE: return "invalid shape or leading dimension";
    case L0CIM_ERR_WORKSPACE: return "workspace missing or too small";
    case L0CIM_ERR_HIP: return "HIP runtime error";
    case L0CIM_ERR_UNSUPPORTED: return "unsupported combination";
  }
  return "unknown status";
}

const char* l0cim_last_error(void) { return g_err; }

void l0cim_cim_params_default(l0cim_cim_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->dt = 0.02;
  p->n_steps = 1000;
  p->field = L0CIM_FIELD_CN;
  p->p_thr = 1.0;
  p->d = 0.4;
  p->t_c = 4.0;
  p->t_w = 2.0;
  p->K = 1.0;
  p->j = 0.2;
  p->beta = 0.3;
  p->tau = 1.0;
  p->c0_std = 1e-2;
}

void l0cim_solve_params_default(l0cim_solve_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->eta_init = 0.8;
  p->eta_end = 0.18;
  p->velo = 51;
  p->n_outer = 51;
  p->cdp = L0CIM_CDP_JACOBI;
  p->cdp_iters = 100;
  p->dtc = 0.1;
  p->replicas = 1;
  p->j_dtype = L0CIM_F32;
}

l0cim_status l0cim_gram(l0cim_dtype dtype, int32_t m, int32_t n, const void* A, int64_t lda,
                        const void* y, void* G, int64_t ldg, void* b, void* stream) {
  if (!is_state_dtype(dtype)) return set_error(L0CIM_ERR_UNSUPPORTED, "gram: dtype %d", int(dtype));
  if (!A || !y || !G || !b) return set_error(L0CIM_ERR_ARG, "gram: NULL pointer");
  if (m <= 0 || n <= 0 || lda < n || ldg < n) return set_error(L0CIM_ERR_SHAPE, "gram: bad shape");
  return launch_gram(dtype, m, n, A, lda, y, G, ldg, b, static_cast<hipStream_t>(stream));
}

l0cim_status l0cim_build_couplings(l0cim_dtype dtype, int32_t n, const void* G, int64_t ldg,
                                   const void* b, const void* R, l0cim_dtype j_dtype, void* J,
                                   int64_t ldj, float* row_scale, void* z, void* stream) {
  if (!is_state_dtype(dtype)) return set_error(L0CIM_ERR_UNSUPPORTED, "couplings: dtype %d", int(dtype));
  l0cim_status st = check_jdtype(dtype, j_dtype);
  if (st != L0CIM_OK) return st;
  if (!G || !b || !R || !J || !z) return set_error(L0CIM_ERR_ARG, "couplings: NULL pointer");
  if ((j_dtype == L0CIM_BF16 || j_dtype == L0CIM_FP8E4M3) && !row_scale)
    return set_error(L0CIM_ERR_ARG, "couplings: row_scale required for BF16/FP8");
  if (n <= 0 || ldg < n || ldj < n) return set_error(L0CIM_ERR_SHAPE, "couplings: bad shape");
  return launch_couplings(dtype, n, G, ldg, b, R, j_dtype, J, ldj, row_scale, z,
                          static_cast<hipStream_t>(stream));
}

l0cim_status l0cim_init_r(l0cim_dtype dtype, int32_t n, const void* G, int64_t ldg, const void* b,
                          void* R, void* D_out, int32_t* status, void* stream) {
  if (!is_state_dtype(dtype)) return set_error(L0CIM_ERR_UNSUPPORTED, "init_r: dtype %d", int(dtype));
  if (!G || !b || !R) return set_error(L0CIM_ERR_ARG, "init_r: NULL pointer");
  if (n <= 0 || ldg < n) return set_error(L0CIM_ERR_SHAPE, "init_r: bad shape");
  return launch_r_init_diag(dtype, n, G, ldg, b, nullptr, R, D_out, status, static_cast<hipStream_t>(stream));
}

l0cim_status l0cim_init_state(l0cim_dtype dtype, int32_t n, int32_t P, uint64_t seed, int32_t alt,
                              double c0_std, void* c, void* e, void* stream) {
  if (!is_state_dtype(dtype)) return set_error(L0CIM_ERR_UNSUPPORTED, "init_state: dtype %d", int(dtype));
  if (!c || !e) return set_error(L0CIM_ERR_ARG, "init_state: NULL pointer");
  if (n <= 0 || n > (1 << 24) || P <= 0 || P > (1 << 16))
    return set_error(L0CIM_ERR_SHAPE, "init_state: n or P out of range");
  if (alt < 0 || alt >= (1 << 24)) return set_error(L0CIM_ERR_ARG, "init_state: alternation out of range");
  return launch_init_state(dtype, n, P, seed, alt, c0_std, c, e, static_cast<hipStream_t>(stream));
}

size_t l0cim_mfcim_run_workspace_bytes(l0cim_dtype dtype, int32_t n, int32_t P, l0cim_dtype j_dtype) {
  (void)j_dtype;
  if (n <= 0 || P <= 0 || !is_state_dtype(dtype)) return 0;
  return mfcim_ws_bytes(dtype, n, P);
}

l0cim_status l0cim_mfcim_run(l0cim_dtype dtype, int32_t n, int32_t P, l0cim_dtype j_dtype,
                             const void* J, int64_t ldj, const float* row_scale, const void* z,
                             double eta, const l0cim_cim_params* prm, void* c, void* e,
                             uint8_t* sigma, double* H, void* trace, int32_t trace_steps,
                             int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  return mfcim_run_checked(dtype, n, P, j_dtype, J, ldj, row_scale, z, eta, prm, c, e, sigma, H, trace, trace_steps,
                           status, ws, ws_bytes, true, static_cast<hipStream_t>(stream));
}

l0cim_status l0cim_select_replica(int32_t n, int32_t P, const double* H, const uint8_t* sigma,
                                  uint8_t* sigma_out, int32_t* q_out, void* stream) {
  if (!H || !sigma || !sigma_out) return set_error(L0CIM_ERR_ARG, "select_replica: NULL pointer");
  if (n <= 0 || P <= 0) return set_error(L0CIM_ERR_SHAPE, "select_replica: bad shape");
  return launch_select(n, P, H, sigma, sigma_out, q_out, nullptr, static_cast<hipStream_t>(stream));
}

size_t l0cim_update_r_workspace_bytes(l0cim_dtype dtype, int32_t n, l0cim_cdp cdp) {
  if (n <= 0 || !is_state_dtype(dtype)) return 0;
  return cdp == L0CIM_CDP_CHOL_F64 ? chol_ws_bytes(n) : jacobi_ws_bytes(dtype, n);
}

l0cim_status l0cim_update_r(l0cim_dtype dtype, int32_t n, const void* G, int64_t ldg, const void* b,
                            const uint8_t* sigma, l0cim_cdp cdp, double dtc, int32_t iters,
                            void* R, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  if (!is_state_dtype(dtype)) return set_error(L0CIM_ERR_UNSUPPORTED, "update_r: dtype %d", int(dtype));
  if (!G || !b || !sigma || !R) return set_error(L0CIM_ERR_ARG, "update_r: NULL pointer");
  if (n <= 0 || ldg < n) return set_error(L0CIM_ERR_SHAPE, "update_r: bad shape");
  if (cdp != L0CIM_CDP_JACOBI && cdp != L0CIM_CDP_CHOL_F64)
    return set_error(L0CIM_ERR_ARG, "update_r: unknown cdp %d", int(cdp));
  if (cdp == L0CIM_CDP_JACOBI && iters < 0) return set_error(L0CIM_ERR_ARG, "update_r: iters < 0");
  size_t need = l0cim_update_r_workspace_bytes(dtype, n, cdp);
  if (!ws || ws_bytes < need) return set_error(L0CIM_ERR_WORKSPACE, "update_r: workspace needs %zu bytes", need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (cdp == L0CIM_CDP_CHOL_F64) return launch_chol_refit(dtype, n, G, ldg, b, sigma, R, status, ws, ws_bytes, s);
  return launch_jacobi(dtype, n, G, ldg, b, sigma, dtc, iters, R, status, ws, ws_bytes, s, kDefaultSpinLimit);
}

size_t l0cim_refit_f64_workspace_bytes(int32_t m, int32_t n) {
  if (m <= 0 || n <= 0) return 0;
  return chol_a_ws_bytes(n, m);
}

l0cim_status l0cim_refit_f64(l0cim_dtype dtype, int32_t m, int32_t n, const void* A, int64_t lda, const void* y,
                             const uint8_t* sigma, void* R, int32_t* status, void* ws, size_t ws_bytes,
                             void* stream) {
  if (!is_state_dtype(dtype)) return set_error(L0CIM_ERR_UNSUPPORTED, "refit_f64: dtype %d", int(dtype));
  if (!A || !y || !sigma || !R) return set_error(L0CIM_ERR_ARG, "refit_f64: NULL pointer");
  if (m <= 0 || n <= 0 || lda < n) return set_error(L0CIM_ERR_SHAPE, "refit_f64: bad shape");
  const size_t need = chol_a_ws_bytes(n, m);
  if (!ws || ws_bytes < need) return set_error(L0CIM_ERR_WORKSPACE, "refit_f64: workspace needs %zu bytes", need);
  return launch_chol_refit_a(dtype, m, n, A, lda, y, sigma, R, status, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

size_t l0cim_solve_workspace_bytes(l0cim_dtype dtype, int32_t m, int32_t n, const l0cim_cim_params* cim,
                                   const l0cim_solve_params* sp) {
  (void)cim;
  if (!sp || m <= 0 || n <= 0 || !is_state_dtype(dtype) || sp->replicas <= 0) return 0;
  bool chol = sp->final_refit_f64 || sp->cdp == L0CIM_CDP_CHOL_F64;
  return solve_layout(dtype, m, n, sp->replicas, l0cim_dtype(sp->j_dtype), chol).total;
}

l0cim_status l0cim_solve(l0cim_dtype dtype, int32_t m, int32_t n, const void* A, int64_t lda,
                         const void* y, const void* R_init, const l0cim_cim_params* cim,
                         const l0cim_solve_params* sp, void* R_out, uint8_t* sigma_out,
                         l0cim_stats* stats, void* ws, size_t ws_bytes, void* stream) {
  if (!is_state_dtype(dtype)) return set_error(L0CIM_ERR_UNSUPPORTED, "solve: dtype %d", int(dtype));
  l0cim_status st = check_cim(cim);
  if (st != L0CIM_OK) return st;
  if (!sp) return set_error(L0CIM_ERR_ARG, "solve: solve params is NULL");
  const l0cim_dtype jdt = l0cim_dtype(sp->j_dtype);
  st = check_jdtype(dtype, jdt);
  if (st != L0CIM_OK) return st;
  if (!A || !y || !R_out || !sigma_out || !stats) return set_error(L0CIM_ERR_ARG, "solve: NULL pointer");
  if (m <= 0 || n <= 0 || lda < n) return set_error(L0CIM_ERR_SHAPE, "solve: bad shape");
  if (n > (1 << 24)) return set_error(L0CIM_ERR_SHAPE, "solve: n above 2^24");
  const int P = sp->replicas;
  if (P <= 0 || P > (1 << 16)) return set_error(L0CIM_ERR_ARG, "solve: replicas out of range");
  if (sp->n_outer <= 0 || sp->n_outer >= (1 << 24) || sp->velo <= 0)
    return set_error(L0CIM_ERR_ARG, "solve: n_outer and velo must be positive");
  if (sp->cdp != L0CIM_CDP_JACOBI && sp->cdp != L0CIM_CDP_CHOL_F64)
    return set_error(L0CIM_ERR_ARG, "solve: unknown cdp %d", sp->cdp);
  if (sp->cdp_iters < 0) return set_error(L0CIM_ERR_ARG, "solve: cdp_iters < 0");
  const bool chol = sp->final_refit_f64 || sp->cdp == L0CIM_CDP_CHOL_F64;
  const SolveLayout L = solve_layout(dtype, m, n, P, jdt, chol);
  if (!ws || ws_bytes < L.total)
    return set_error(L0CIM_ERR_WORKSPACE, "solve: workspace needs %zu bytes", L.total);

  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  void* G = base + L.G;
  void* b = base + L.b;
  void* J = base + L.J;
  float* rs = reinterpret_cast<float*>(base + L.rs);
  void* z = base + L.z;
  void* c = base + L.c;
  void* e = base + L.e;
  uint8_t* sig = reinterpret_cast<uint8_t*>(base + L.sig);
  double* H = reinterpret_cast<double*>(base + L.H);
  void* run_ws = base + L.run;
  void* cdp_ws = base + L.cdp;
  void* obj_ws = base + L.obj;
  int* status = &stats->status_bits;
  const bool quant = (jdt == L0CIM_BF16 || jdt == L0CIM_FP8E4M3);

  hipLaunchKernelGGL(stats_init_kernel, dim3(1), dim3(1), 0, s, stats);
  L0_LAUNCHED("stats_init_kernel");
#define L0_TRY(x)                      \
  do {                                 \
    l0cim_status _s = (x);             \
    if (_s != L0CIM_OK) return _s;     \
  } while (0)
  L0_TRY(launch_gram(dtype, m, n, A, lda, y, G, n, b, s));
  L0_TRY(launch_r_init(dtype, n, G, n, b, R_init, R_out, status, s));
  double eta = eta_at(sp, 0);
  for (int i = 0; i < sp->n_outer; ++i) {
    eta = eta_at(sp, i);
    L0_TRY(launch_couplings(dtype, n, G, n, b, R_out, jdt, J, n, rs, z, s));
    L0_TRY(launch_init_state(dtype, n, P, sp->seed, i, cim->c0_std, c, e, s));
    CimArgs a = make_args(n, P, cim, eta, 0);
    L0_TRY(launch_mfcim(dtype, n, P, jdt, J, n, quant ? rs : nullptr, z, a, c, e, sig, H, nullptr,
                        status, run_ws, L.run_bytes, s));
    L0_TRY(launch_select(n, P, H, sig, sigma_out, &stats->selected_replica, &stats->H, s));
    if (sp->cdp == L0CIM_CDP_CHOL_F64)
      L0_TRY(launch_chol_refit_a(dtype, m, n, A, lda, y, sigma_out, R_out, status, cdp_ws, L.cdp_bytes, s));
    else
      L0_TRY(launch_jacobi(dtype, n, G, n, b, sigma_out, sp->dtc, sp->cdp_iters, R_out, status, cdp_ws,
                           L.cdp_bytes, s, a.spin_limit));
  }
  if (sp->final_refit_f64)
    L0_TRY(launch_chol_refit_a(dtype, m, n, A, lda, y, sigma_out, R_out, status, cdp_ws, L.cdp_bytes, s));
  const int64_t spin_steps = int64_t(n) * P * cim->n_steps * sp->n_outer;
  L0_TRY(launch_objective(dtype, m, n, A, lda, y, sigma_out, R_out, 0.5 * eta * eta, stats, spin_steps,
                          sp->n_outer, obj_ws, L.obj_bytes, s));
#undef L0_TRY
  return L0CIM_OK;
}

size_t l0cim_solve_many_workspace_bytes(l0cim_dtype dtype, int32_t count, int32_t m, int32_t n,
                                        const l0cim_solve_params* sp) {
  if (!sp || count <= 0 || m <= 0 || n <= 0 || !is_state_dtype(dtype) || sp->replicas <= 0) return 0;
  const bool chol = sp->final_refit_f64 || sp->cdp == L0CIM_CDP_CHOL_F64;
  return many_layout(dtype, count, m, n, sp->replicas, l0cim_dtype(sp->j_dtype), chol).total;
}

l0cim_status l0cim_solve_many(l0cim_dtype dtype, int32_t count, int32_t m, int32_t n, const void* A, int64_t lda,
                              int64_t strideA, const void* y, int64_t stridey, const uint64_t* seeds,
                              const l0cim_cim_params* cim, const l0cim_solve_params* sp, void* R_out,
                              uint8_t* sigma_out, l0cim_stats* stats, void* ws, size_t ws_bytes, void* stream) {
  if (!is_state_dtype(dtype)) return set_error(L0CIM_ERR_UNSUPPORTED, "solve_many: dtype %d", int(dtype));
  l0cim_status st = check_cim(cim);
  if (st != L0CIM_OK) return st;
  if (!sp || !seeds) return set_error(L0CIM_ERR_ARG, "solve_many: NULL parameters or seeds");
  const l0cim_dtype jdt = l0cim_dtype(sp->j_dtype);
  st = check_jdtype(dtype, jdt);
  if (st != L0CIM_OK) return st;
  if (!A || !y || !R_out || !sigma_out || !stats) return set_error(L0CIM_ERR_ARG, "solve_many: NULL pointer");
  if (count <= 0 || count > 4096) return set_error(L0CIM_ERR_ARG, "solve_many: count must be 1..4096");
  if (m <= 0 || n <= 0 || n > (1 << 24) || lda < n || strideA < int64_t(m) * lda || stridey < m)
    return set_error(L0CIM_ERR_SHAPE, "solve_many: bad shape or stride");
  const int P = sp->replicas;
  if (P <= 0 || P > (1 << 16)) return set_error(L0CIM_ERR_ARG, "solve_many: replicas out of range");
  if (sp->n_outer <= 0 || sp->n_outer >= (1 << 24) || sp->velo <= 0)
    return set_error(L0CIM_ERR_ARG, "solve_many: n_outer and velo must be positive");
  if (sp->cdp != L0CIM_CDP_JACOBI && sp->cdp != L0CIM_CDP_CHOL_F64)
    return set_error(L0CIM_ERR_ARG, "solve_many: unknown cdp %d", sp->cdp);
  if (sp->cdp_iters < 0) return set_error(L0CIM_ERR_ARG, "solve_many: cdp_iters < 0");
  const bool chol = sp->final_refit_f64 || sp->cdp == L0CIM_CDP_CHOL_F64;
  const ManyLayout L = many_layout(dtype, count, m, n, P, jdt, chol);
  if (!ws || ws_bytes < L.total) return set_error(L0CIM_ERR_WORKSPACE, "solve_many: workspace needs %zu bytes", L.total);

  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  const size_t ts = dtype_size(dtype);
  const size_t jsz = dtype_size(jdt);
  const bool quant = (jdt == L0CIM_BF16 || jdt == L0CIM_FP8E4M3);
  auto Ak = [&](int k) { return static_cast<const char*>(A) + size_t(k) * strideA * ts; };
  auto yk = [&](int k) { return static_cast<const char*>(y) + size_t(k) * stridey * ts; };
  auto Gk = [&](int k) { return base + L.G + k * L.sG; };
  auto bk = [&](int k) { return base + L.b + k * L.sb; };
  auto Jk = [&](int k) { return base + L.J + k * L.sJ * jsz; };
  auto rsk = [&](int k) { return reinterpret_cast<float*>(base + L.rs) + k * L.sv; };
  auto zk = [&](int k) { return base + L.z + k * L.sv * ts; };
  auto ck = [&](int k) { return base + L.c + k * L.sv * ts; };
  auto ek = [&](int k) { return base + L.e + k * L.sv * ts; };
  auto sigk = [&](int k) { return reinterpret_cast<uint8_t*>(base + L.sig) + k * L.sv; };
  auto Hk = [&](int k) { return reinterpret_cast<double*>(base + L.H + k * L.sH); };
  auto runk = [&](int k) { return base + L.run + k * L.srun; };
  auto cdpk = [&](int k) { return base + L.cdp + k * L.scdp; };
  auto Rk = [&](int k) { return static_cast<char*>(R_out) + size_t(k) * n * ts; };
  auto sok = [&](int k) { return sigma_out + size_t(k) * n; };
#define L0_TRY(x)                  \
  do {                             \
    l0cim_status _s = (x);         \
    if (_s != L0CIM_OK) return _s; \
  } while (0)
  for (int k = 0; k < count; ++k) {
    hipLaunchKernelGGL(stats_init_kernel, dim3(1), dim3(1), 0, s, stats + k);
    L0_LAUNCHED("stats_init_kernel");
    L0_TRY(launch_gram(dtype, m, n, Ak(k), lda, yk(k), Gk(k), n, bk(k), s));
    L0_TRY(launch_r_init(dtype, n, Gk(k), n, bk(k), nullptr, Rk(k), &stats[k].status_bits, s));
  }
  // one register-resident launch for all instances where that form applies
  bool together = dtype == L0CIM_F32 && P == 1 && count > 1;
  double eta = eta_at(sp, 0);
  for (int i = 0; i < sp->n_outer; ++i) {
    eta = eta_at(sp, i);
    for (int k = 0; k < count; ++k) {
      L0_TRY(launch_couplings(dtype, n, Gk(k), n, bk(k), Rk(k), jdt, Jk(k), n, rsk(k), zk(k), s));
      L0_TRY(launch_init_state(dtype, n, P, seeds[k], i, cim->c0_std, ck(k), ek(k), s));
    }
    const CimArgs a = make_args(n, P, cim, eta, 0);
    if (together) {
      const int64_t sst = int64_t(sizeof(l0cim_stats) / sizeof(int32_t));
      l0cim_status ms = launch_mfcim_many(jdt, count, n, Jk(0), n, int64_t(L.sJ), quant ? rsk(0) : nullptr,
                                          reinterpret_cast<const float*>(zk(0)), int64_t(L.sv), a,
                                          reinterpret_cast<float*>(ck(0)), reinterpret_cast<float*>(ek(0)), sigk(0),
                                          Hk(0), int64_t(L.sH / sizeof(double)), &stats[0].status_bits, sst, runk(0),
                                          int64_t(L.srun), s);
      if (ms == L0CIM_ERR_UNSUPPORTED) together = false;
      else if (ms != L0CIM_OK) return ms;
    }
    if (!together)
      for (int k = 0; k < count; ++k)
        L0_TRY(launch_mfcim(dtype, n, P, jdt, Jk(k), n, quant ? rsk(k) : nullptr, zk(k), a, ck(k), ek(k), sigk(k),
                            Hk(k), nullptr, &stats[k].status_bits, runk(k), L.srun, s));
    for (int k = 0; k < count; ++k) {
      L0_TRY(launch_select(n, P, Hk(k), sigk(k), sok(k), &stats[k].selected_replica, &stats[k].H, s));
      if (sp->cdp == L0CIM_CDP_CHOL_F64)
        L0_TRY(launch_chol_refit_a(dtype, m, n, Ak(k), lda, yk(k), sok(k), Rk(k), &stats[k].status_bits, cdpk(k),
                                   L.scdp, s));
      else
        L0_TRY(launch_jacobi(dtype, n, Gk(k), n, bk(k), sok(k), sp->dtc, sp->cdp_iters, Rk(k), &stats[k].status_bits,
                             cdpk(k), L.scdp, s, a.spin_limit));
    }
  }
  const int64_t spin_steps = int64_t(n) * P * cim->n_steps * sp->n_outer;
  for (int k = 0; k < count; ++k) {
    if (sp->final_refit_f64)
      L0_TRY(launch_chol_refit_a(dtype, m, n, Ak(k), lda, yk(k), sok(k), Rk(k), &stats[k].status_bits, cdpk(k),
                                 L.scdp, s));
    L0_TRY(launch_objective(dtype, m, n, Ak(k), lda, yk(k), sok(k), Rk(k), 0.5 * eta * eta, stats + k, spin_steps,
                            sp->n_outer, base + L.obj + k * L.sobj, L.sobj, s));
  }
#undef L0_TRY
  return L0CIM_OK;
}

l0cim_status l0cim_profile_begin(void) {
  for (auto& pr : g_prof.events) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  g_prof.events.clear();
  g_prof.on = true;
  return L0CIM_OK;
}

l0cim_status l0cim_profile_end(double* cim_ms, int64_t* cim_launches) {
  g_prof.on = false;
  double total = 0.0;
  l0cim_status st = L0CIM_OK;
  for (auto& pr : g_prof.events) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(pr.second);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
    if (e != hipSuccess && st == L0CIM_OK) st = hip_fail(e, "profile events");
    total += ms;
  }
  if (cim_ms) *cim_ms = total;
  if (cim_launches) *cim_launches = int64_t(g_prof.events.size());
  for (auto& pr : g_prof.events) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  g_prof.events.clear();
  return st;
}

}  // extern "C"
