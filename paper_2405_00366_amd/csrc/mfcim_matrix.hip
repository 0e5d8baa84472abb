// Single-instance CIM run on the matrix cores: the batched MFMA step kernel
// applied to a one-instance table.  Used when several replicas make J X a
// dense product and the couplings are streamed every step (for example the
// MRI-shaped workload, N = 16384 with 64 replicas).  The caller's row-major
// couplings are copied once into the panel layout; the instance and tile
// tables and the padded copies of the state are written by a setup kernel,
// so the whole run is a sequence of kernel launches on the caller's stream.
#include <map>
#include <mutex>

#include "batch.h"

namespace l0 {
namespace {

constexpr int kLd = 32;

__global__ void __launch_bounds__(256)
mat_setup_kernel(BInst I, BTile* __restrict__ tiles, int ntiles, int tr, BInst* __restrict__ inst_out,
                 double* __restrict__ eta_out, double eta, const float* __restrict__ rscale,
                 float* __restrict__ rs, const float* __restrict__ z_in, float* __restrict__ z,
                 const float* __restrict__ c_in, const float* __restrict__ e_in, float* __restrict__ c,
                 float* __restrict__ c2, float* __restrict__ e, int n, int P, int ld) {
  const size_t gid = blockIdx.x * size_t(256) + threadIdx.x;
  const size_t stride = size_t(gridDim.x) * 256;
  if (gid == 0) {
    *inst_out = I;
    *eta_out = eta;
  }
  for (size_t t = gid; t < size_t(ntiles); t += stride) tiles[t] = BTile{0, int(t) * tr};
  for (size_t i = gid; i < size_t(ld); i += stride) {
    rs[i] = (i < size_t(n) && rscale) ? rscale[i] : 1.0f;
    z[i] = i < size_t(n) ? z_in[i] : 0.0f;
  }
  for (size_t i = gid; i < size_t(P) * ld; i += stride) {
    const size_t q = i / ld, r = i - q * ld;
    const bool in = r < size_t(n);
    c[i] = in ? c_in[q * n + r] : 0.0f;
    c2[i] = 0.0f;
    e[i] = in ? e_in[q * n + r] : 0.0f;
  }
}

// Row r (< n16) of the caller's couplings into the panel layout, zero padded.
// A thread moves columns 8 g .. 8 g + 7, which land in the panel as one
// contiguous run (two runs of 4 for 4-byte elements): one wide store each.
template <typename JT>
__global__ void __launch_bounds__(256)
mat_copyJ_kernel(const JT* __restrict__ J, int64_t ldj, JT* __restrict__ Jp, int n, int ld) {
  const int r = blockIdx.y, np = (n + 15) / 16;
  for (int j0 = 8 * (blockIdx.x * 256 + threadIdx.x); j0 < ld; j0 += 8 * gridDim.x * 256) {
    JT v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = (r < n && j0 + t < n) ? J[size_t(r) * ldj + j0 + t] : JT(0.0f);
    if constexpr (sizeof(JT) == 4) {
      *reinterpret_cast<float4*>(Jp + jpanel_offset(r, j0, ld, np, 4)) =
          make_float4(float(v[0]), float(v[1]), float(v[2]), float(v[3]));
      *reinterpret_cast<float4*>(Jp + jpanel_offset(r, j0 + 4, ld, np, 4)) =
          make_float4(float(v[4]), float(v[5]), float(v[6]), float(v[7]));
    } else {
      struct alignas(8 * sizeof(JT)) Run { JT e[8]; };
      Run run;
#pragma unroll
      for (int t = 0; t < 8; ++t) run.e[t] = v[t];
      *reinterpret_cast<Run*>(Jp + jpanel_offset(r, j0, ld, np, int(sizeof(JT)))) = run;
    }
  }
}

__global__ void __launch_bounds__(256)
mat_finish_kernel(const float* __restrict__ cf, const float* __restrict__ ef, float* __restrict__ c,
                  float* __restrict__ e, int n, int P, int ld) {
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < size_t(P) * n; i += size_t(gridDim.x) * 256) {
    const size_t q = i / n, r = i - q * n;
    c[i] = cf[q * ld + r];
    e[i] = ef[q * ld + r];
  }
}

// H_q = sum over spins of the eq. 4 terms of replica q: one workgroup per
// replica, 256 contiguous runs of spins summed in order, then a fixed tree.
__global__ void __launch_bounds__(256)
mat_hsum_kernel(const double* __restrict__ hrow, int n, double* __restrict__ H) {
  __shared__ double part[256];
  const int q = blockIdx.x, t = threadIdx.x;
  const int chunk = (n + 255) / 256;
  const int lo = min(n, t * chunk), hi = min(n, lo + chunk);
  double h = 0.0;
  for (int r = lo; r < hi; ++r) h += hrow[size_t(q) * n + r];
  part[t] = h;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) part[t] += part[t + w];
    __syncthreads();
  }
  if (t == 0) H[q] = part[0];
}

struct MatLayout {
  size_t inst, tiles, eta, rs, z, c, c2, e, xb, xb2, hrow, J, total;
};

MatLayout mat_layout(int n, int P, size_t jsize) {
  const int ld = (n + kLd - 1) / kLd * kLd;
  const size_t ntiles = size_t((n + 15) / 16);
  MatLayout L;
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t at = o;
    o += align_up(b);
    return at;
  };
  L.inst = take(sizeof(BInst));
  L.tiles = take(ntiles * sizeof(BTile));
  L.eta = take(sizeof(double));
  L.rs = take(size_t(ld) * 4);
  L.z = take(size_t(ld) * 4);
  L.c = take(size_t(P) * ld * 4);
  L.c2 = take(size_t(P) * ld * 4);
  L.e = take(size_t(P) * ld * 4);
  L.xb = take(xbits_words(ld, P) * 4);
  L.xb2 = take(xbits_words(ld, P) * 4);
  L.hrow = take(size_t(P) * n * 8);
  L.J = take(size_t(round_up16(n)) * ld * jsize);
  L.total = o;
  return L;
}

struct MatKey {
  int n, P, jdt, field;
  bool operator<(const MatKey& o) const {
    return n != o.n ? n < o.n : (P != o.P ? P < o.P : (jdt != o.jdt ? jdt < o.jdt : field < o.field));
  }
};

std::mutex g_shape_mu;
std::map<MatKey, int> g_shape;

int tuned_shape(const MatKey& k) {
  std::lock_guard<std::mutex> lk(g_shape_mu);
  auto it = g_shape.find(k);
  return it == g_shape.end() ? 0 : it->second;
}

void remember_shape(const MatKey& k, int rb) {
  std::lock_guard<std::mutex> lk(g_shape_mu);
  if (rb) g_shape[k] = rb;
  else g_shape.erase(k);
}

}  // namespace

size_t matrix_ws_bytes(int n, int P, size_t jsize) { return mat_layout(n, P, jsize).total; }

bool matrix_supported(int n, int P, int64_t ldj) { return P >= 1 && P <= 64 && n >= 1 && ldj >= n; }

l0cim_status launch_matrix_run(int n, int P, l0cim_dtype jdt, const void* J, int64_t ldj, const float* rscale,
                               const float* z, const CimArgs& a, float* c, float* e, uint8_t* sigma, double* H,
                               float* trace, int* status, void* ws, hipStream_t s, int rb_hint) {
  DeviceInfo dev;
  l0cim_status st = device_info(&dev);
  if (st != L0CIM_OK) return st;
  const int ld = (n + kLd - 1) / kLd * kLd;
  const size_t jsize = dtype_size(jdt);
  const MatLayout Lw = mat_layout(n, P, jsize);
  char* b = static_cast<char*>(ws);
  BInst* dinst = reinterpret_cast<BInst*>(b + Lw.inst);
  BTile* dtiles = reinterpret_cast<BTile*>(b + Lw.tiles);
  double* deta = reinterpret_cast<double*>(b + Lw.eta);
  float* drs = reinterpret_cast<float*>(b + Lw.rs);
  float* dz = reinterpret_cast<float*>(b + Lw.z);
  float* dc = reinterpret_cast<float*>(b + Lw.c);
  float* dc2 = reinterpret_cast<float*>(b + Lw.c2);
  float* de = reinterpret_cast<float*>(b + Lw.e);
  double* dh = reinterpret_cast<double*>(b + Lw.hrow);
  uint32_t* dxb = reinterpret_cast<uint32_t*>(b + Lw.xb);
  uint32_t* dxb2 = reinterpret_cast<uint32_t*>(b + Lw.xb2);
  void* Jp = b + Lw.J;
  {
    dim3 g((ld / 8 + 255) / 256, round_up16(n));
    if (jdt == L0CIM_F32)
      hipLaunchKernelGGL(mat_copyJ_kernel<float>, g, dim3(256), 0, s, (const float*)J, ldj, (float*)Jp, n, ld);
    else if (jdt == L0CIM_BF16)
      hipLaunchKernelGGL(mat_copyJ_kernel<__hip_bfloat16>, g, dim3(256), 0, s, (const __hip_bfloat16*)J, ldj,
                         (__hip_bfloat16*)Jp, n, ld);
    else
      hipLaunchKernelGGL(mat_copyJ_kernel<__hip_fp8_e4m3>, g, dim3(256), 0, s, (const __hip_fp8_e4m3*)J, ldj,
                         (__hip_fp8_e4m3*)Jp, n, ld);
    L0_LAUNCHED("mat_copyJ_kernel");
  }
  const int qb = P <= 16 ? 1 : (P <= 32 ? 2 : 4);
  BStepArgs sa;
  sa.P = P;
  sa.n_steps = a.n_steps;
  sa.linear_j = a.linear_j;
  sa.field = a.field;
  sa.dt = a.dt;
  sa.p_thr = a.p_thr;
  sa.d = a.d;
  sa.t_c = a.t_c;
  sa.t_w = a.t_w;
  sa.K = a.K;
  sa.j = a.j;
  sa.beta = a.beta;
  sa.tau = a.tau;
  sa.trace = trace;
  sa.trace_steps = a.trace_steps;
  BatchDev d{};
  d.count = 1;
  d.insts = dinst;
  d.tiles = dtiles;
  d.eta = deta;
  // Tables and padded state for tile shape rb (RB panels per workgroup).
  auto setup = [&](int rb, int* ntiles_out) -> l0cim_status {
    const int tr = 16 * rb;
    const int ntiles = (n + tr - 1) / tr;
    BInst I{};
    I.n = n;
    I.ld = ld;
    I.ldj = ld;
    I.tile0 = 0;
    I.ntiles = ntiles;
    I.J = Jp;
    I.xb = dxb;
    I.xb2 = dxb2;
    I.z = dz;
    I.rs = drs;
    I.c = dc;
    I.c2 = dc2;
    I.e = de;
    I.sig_all = sigma;
    I.hpart = dh;
    I.status = status;
    size_t work = size_t(P) * ld;
    int blocks = int((work + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(mat_setup_kernel, dim3(blocks), dim3(256), 0, s, I, dtiles, ntiles, tr, dinst, deta, a.eta,
                       rscale, drs, z, dz, c, e, dc, dc2, de, n, P, ld);
    L0_LAUNCHED("mat_setup_kernel");
    if (a.field == L0CIM_FIELD_BN) {
      l0cim_status r = launch_bbits(d, qb, int64_t(P) * ld / 32, s);
      if (r != L0CIM_OK) return r;
    }
    *ntiles_out = ntiles;
    return L0CIM_OK;
  };
  // Tile shape: the caller's, else the fastest of the candidates timed once
  // per (n, P, coupling type, field) in this process, else the largest row
  // block that still gives every CU four tiles.  Trial steps touch only the
  // padded copies of the state, which the final setup rewrites.
  int rb = 0;
  if (step_shape_ok(qb, rb_hint)) rb = rb_hint;
  const MatKey key{n, P, int(jdt), a.field};
  if (!rb) rb = tuned_shape(key);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  L0_HIP(hipStreamIsCapturing(s, &cap));
  if (!rb && a.n_steps >= 16 && cap == hipStreamCaptureStatusNone) {
    BStepArgs ta = sa;
    ta.trace = nullptr;
    ta.trace_steps = 0;
    hipEvent_t e0, e1;
    L0_HIP(hipEventCreate(&e0));
    L0_HIP(hipEventCreate(&e1));
    // two rounds over the candidates, each candidate's best of its 12-step
    // timings (single short timings picked a slower shape now and then)
    float cand_ms[9] = {1e30f, 1e30f, 1e30f, 1e30f, 1e30f, 1e30f, 1e30f, 1e30f, 1e30f};
    for (int round = 0; round < 2; ++round) {
      for (int cand : {1, 2, 4, 8}) {
        if (!step_shape_ok(qb, cand)) continue;
        int nt = 0;
        st = setup(cand, &nt);
        if (st != L0CIM_OK) return st;
        const StepKernel fc = batch_step_kernel(jdt, a.field, qb, cand);
        if (!fc.fn) return set_error(L0CIM_ERR_UNSUPPORTED, "matrix run: no kernel for this shape");
        st = enqueue_bsteps(d, fc, ta, nt, 0, 1, s);
        if (st != L0CIM_OK) return st;
        L0_HIP(hipEventRecord(e0, s));
        st = enqueue_bsteps(d, fc, ta, nt, 2, 13, s);
        if (st != L0CIM_OK) return st;
        L0_HIP(hipEventRecord(e1, s));
        L0_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        L0_HIP(hipEventElapsedTime(&ms, e0, e1));
        cand_ms[cand] = std::min(cand_ms[cand], ms);
      }
    }
    float best = 1e30f;
    int best_rb = 1;
    for (int cand : {1, 2, 4, 8})
      if (step_shape_ok(qb, cand) && cand_ms[cand] < best) {
        best = cand_ms[cand];
        best_rb = cand;
      }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    rb = best_rb;
    remember_shape(key, rb);
  }
  if (!rb) {
    rb = 1;
    for (int cand : {8, 4, 2}) {
      if (step_shape_ok(qb, cand) && (n + 16 * cand - 1) / (16 * cand) >= 4 * dev.cu_count) {
        rb = cand;
        break;
      }
    }
  }
  int ntiles = 0;
  st = setup(rb, &ntiles);
  if (st != L0CIM_OK) return st;
  const StepKernel fn = batch_step_kernel(jdt, a.field, qb, rb);
  if (!fn.fn) return set_error(L0CIM_ERR_UNSUPPORTED, "matrix run: no kernel for this shape");
  {
    ProfileScope prof(s);
    st = enqueue_bsteps(d, fn, sa, ntiles, 0, a.n_steps, s);
    if (st != L0CIM_OK) return st;
  }
  const float* cf = (a.n_steps & 1) ? dc2 : dc;
  {
    size_t work = size_t(P) * n;
    int blocks = int((work + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(mat_finish_kernel, dim3(blocks), dim3(256), 0, s, cf, de, c, e, n, P, ld);
    L0_LAUNCHED("mat_finish_kernel");
  }
  if (H) {
    hipLaunchKernelGGL(mat_hsum_kernel, dim3(P), dim3(256), 0, s, dh, n, H);
    L0_LAUNCHED("mat_hsum_kernel");
  }
  return L0CIM_OK;
}

}  // namespace l0

extern "C" {

l0cim_status l0cim_matrix_tile_get(int32_t n, int32_t P, l0cim_dtype j_dtype, int32_t field, int32_t* rows) {
  if (!rows) return l0::set_error(L0CIM_ERR_ARG, "matrix_tile_get: NULL pointer");
  *rows = 16 * l0::tuned_shape(l0::MatKey{n, P, int(j_dtype), field});
  return L0CIM_OK;
}

l0cim_status l0cim_matrix_tile_set(int32_t n, int32_t P, l0cim_dtype j_dtype, int32_t field, int32_t rows) {
  const int qb = P <= 16 ? 1 : (P <= 32 ? 2 : 4);
  if (rows != 0 && (rows % 16 != 0 || !l0::step_shape_ok(qb, rows / 16)))
    return l0::set_error(L0CIM_ERR_ARG, "matrix_tile_set: %d rows per workgroup is not a shape for %d replicas",
                         rows, P);
  l0::remember_shape(l0::MatKey{n, P, int(j_dtype), field}, rows / 16);
  return L0CIM_OK;
}

}  // extern "C"
