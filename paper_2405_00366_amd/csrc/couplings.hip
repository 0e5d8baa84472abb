// Per-alternation preparation of the Ising problem:
//  * couplings J_rr' = -G_rr' R_r R_r' with a zero diagonal and the Zeeman
//    term z_r = R_r b_r (eq. 4 with R fixed; eq. 15 / 16 use R_r h_r);
//  * optional BF16 / FP8-e4m3 storage of J with one FP32 scale per row;
//  * the initial CIM state c ~ N(0, c0_std^2), e = 1 (after eq. 16), drawn
//    from a counter-based SplitMix64 + Box-Muller generator;
//  * R_init = b_r / G_rr.
#include "kernels.h"

namespace l0 {
namespace {

template <typename T>
__global__ void __launch_bounds__(256)
couplings_kernel(int n, const T* __restrict__ G, int64_t ldg, const T* __restrict__ b,
                 const T* __restrict__ R, T* __restrict__ J, int64_t ldj, T* __restrict__ z) {
  const int r = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const T Rr = R[r];
  J[size_t(r) * ldj + j] = (j == r) ? T(0) : -(G[size_t(r) * ldg + j] * (Rr * R[j]));
  if (blockIdx.x == 0 && threadIdx.x == 0) z[r] = Rr * b[r];
}

template <typename Q> struct QTraits;
template <> struct QTraits<__hip_bfloat16> {
  static constexpr float kMax = 1.0f;
  __device__ static inline __hip_bfloat16 enc(float v) { return __float2bfloat16(v); }
};
template <> struct QTraits<__hip_fp8_e4m3> {
  static constexpr float kMax = 448.0f;
  __device__ static inline __hip_fp8_e4m3 enc(float v) {
    v = fminf(fmaxf(v, -448.0f), 448.0f);
    return __hip_fp8_e4m3(v);
  }
};

// One workgroup per row: amax of the row, then RNE(J / scale).
template <typename Q>
__global__ void __launch_bounds__(256)
couplings_quant_kernel(int n, const float* __restrict__ G, int64_t ldg, const float* __restrict__ b,
                       const float* __restrict__ R, Q* __restrict__ J, int64_t ldj,
                       float* __restrict__ rscale, float* __restrict__ z) {
  __shared__ float red[256];
  constexpr int kRowRegs = 64;   // rows of up to 256 * 64 couplings stay in registers between the passes
  const int r = blockIdx.x;
  const float Rr = R[r];
  const float* Gr = G + size_t(r) * ldg;
  const bool in_regs = n <= 256 * kRowRegs;
  float vals[kRowRegs];
  float amax = 0.0f;
  if (in_regs) {
#pragma unroll
    for (int u = 0; u < kRowRegs; ++u) {
      const int j = threadIdx.x + 256 * u;
      vals[u] = (j < n && j != r) ? -(Gr[j] * (Rr * R[j])) : 0.0f;
      amax = fmaxf(amax, fabsf(vals[u]));
    }
  } else {
    for (int j = threadIdx.x; j < n; j += 256) {
      float v = (j == r) ? 0.0f : -(Gr[j] * (Rr * R[j]));
      amax = fmaxf(amax, fabsf(v));
    }
  }
  red[threadIdx.x] = amax;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  amax = red[0];
  const float scale = amax > 0.0f ? amax / QTraits<Q>::kMax : 1.0f;
  if (in_regs) {
#pragma unroll
    for (int u = 0; u < kRowRegs; ++u) {
      const int j = threadIdx.x + 256 * u;
      if (j < n) J[size_t(r) * ldj + j] = QTraits<Q>::enc(vals[u] / scale);
    }
  } else {
    for (int j = threadIdx.x; j < n; j += 256) {
      float v = (j == r) ? 0.0f : -(Gr[j] * (Rr * R[j]));
      J[size_t(r) * ldj + j] = QTraits<Q>::enc(v / scale);
    }
  }
  if (threadIdx.x == 0) {
    rscale[r] = scale;
    z[r] = Rr * b[r];
  }
}

// SplitMix64 (Steele, Lea, Flood 2014): output n of the stream keyed by seed
// is mix64(seed + n * GAMMA).
__device__ inline uint64_t mix64(uint64_t x) {
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

template <typename T>
__global__ void __launch_bounds__(256)
init_state_kernel(int n, int P, uint64_t seed, int alt, double std, T* __restrict__ c,
                  T* __restrict__ e) {
  const size_t total = size_t(n) * P;
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < total; i += size_t(gridDim.x) * 256) {
    const uint64_t q = i / n, r = i - q * n;
    const uint64_t ctr = (uint64_t(alt) << 40) | (q << 24) | r;
    const uint64_t g = 0x9E3779B97F4A7C15ull;
    const uint64_t w1 = mix64(seed + (2 * ctr + 1) * g);
    const uint64_t w2 = mix64(seed + (2 * ctr + 2) * g);
    const double u1 = double(w1 >> 11) * 0x1.0p-53;
    const double u2 = double(w2 >> 11) * 0x1.0p-53;
    const double nrm = sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586 * u2);
    c[i] = T(std * nrm);
    e[i] = T(1);
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
r_init_kernel(int n, const T* __restrict__ G, int64_t ldg, const T* __restrict__ b,
              const T* __restrict__ Rin, T* __restrict__ R, T* __restrict__ Dout, int* __restrict__ status) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  const T d = G[size_t(r) * ldg + r];
  if (Dout) Dout[r] = d;
  const bool tiny = !(d >= T(1e-12));
  if (tiny) raise_status(status, L0CIM_ST_TINY_DIAG);
  if (Rin) R[r] = tiny ? T(0) : Rin[r];
  else R[r] = tiny ? T(0) : b[r] / d;
}

}  // namespace

l0cim_status launch_couplings(l0cim_dtype dt, int n, const void* G, int64_t ldg, const void* b,
                              const void* R, l0cim_dtype jdt, void* J, int64_t ldj, float* rscale,
                              void* z, hipStream_t s) {
  dim3 grid((n + 255) / 256, n);
  if (dt == L0CIM_F32 && jdt == L0CIM_F32) {
    hipLaunchKernelGGL(couplings_kernel<float>, grid, dim3(256), 0, s, n, (const float*)G, ldg,
                       (const float*)b, (const float*)R, (float*)J, ldj, (float*)z);
  } else if (dt == L0CIM_F64 && jdt == L0CIM_F64) {
    hipLaunchKernelGGL(couplings_kernel<double>, grid, dim3(256), 0, s, n, (const double*)G, ldg,
                       (const double*)b, (const double*)R, (double*)J, ldj, (double*)z);
  } else if (dt == L0CIM_F32 && jdt == L0CIM_BF16) {
    hipLaunchKernelGGL(couplings_quant_kernel<__hip_bfloat16>, dim3(n), dim3(256), 0, s, n,
                       (const float*)G, ldg, (const float*)b, (const float*)R, (__hip_bfloat16*)J, ldj,
                       rscale, (float*)z);
  } else if (dt == L0CIM_F32 && jdt == L0CIM_FP8E4M3) {
    hipLaunchKernelGGL(couplings_quant_kernel<__hip_fp8_e4m3>, dim3(n), dim3(256), 0, s, n,
                       (const float*)G, ldg, (const float*)b, (const float*)R, (__hip_fp8_e4m3*)J, ldj,
                       rscale, (float*)z);
  } else {
    return set_error(L0CIM_ERR_UNSUPPORTED, "build_couplings: dtype %d with coupling dtype %d",
                     int(dt), int(jdt));
  }
  L0_LAUNCHED("couplings kernel");
  return L0CIM_OK;
}

l0cim_status launch_init_state(l0cim_dtype dt, int n, int P, uint64_t seed, int alt, double std,
                               void* c, void* e, hipStream_t s) {
  size_t total = size_t(n) * P;
  int blocks = int((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (dt == L0CIM_F32)
    hipLaunchKernelGGL(init_state_kernel<float>, dim3(blocks), dim3(256), 0, s, n, P, seed, alt, std,
                       (float*)c, (float*)e);
  else if (dt == L0CIM_F64)
    hipLaunchKernelGGL(init_state_kernel<double>, dim3(blocks), dim3(256), 0, s, n, P, seed, alt, std,
                       (double*)c, (double*)e);
  else
    return set_error(L0CIM_ERR_UNSUPPORTED, "init_state: dtype %d", int(dt));
  L0_LAUNCHED("init_state_kernel");
  return L0CIM_OK;
}

l0cim_status launch_r_init_diag(l0cim_dtype dt, int n, const void* G, int64_t ldg, const void* b,
                                const void* R_init, void* R, void* D_out, int* status, hipStream_t s) {
  dim3 grid((n + 255) / 256);
  if (dt == L0CIM_F32)
    hipLaunchKernelGGL(r_init_kernel<float>, grid, dim3(256), 0, s, n, (const float*)G, ldg,
                       (const float*)b, (const float*)R_init, (float*)R, (float*)D_out, status);
  else if (dt == L0CIM_F64)
    hipLaunchKernelGGL(r_init_kernel<double>, grid, dim3(256), 0, s, n, (const double*)G, ldg,
                       (const double*)b, (const double*)R_init, (double*)R, (double*)D_out, status);
  else
    return set_error(L0CIM_ERR_UNSUPPORTED, "r_init: dtype %d", int(dt));
  L0_LAUNCHED("r_init_kernel");
  return L0CIM_OK;
}

l0cim_status launch_r_init(l0cim_dtype dt, int n, const void* G, int64_t ldg, const void* b,
                           const void* R_init, void* R, int* status, hipStream_t s) {
  return launch_r_init_diag(dt, n, G, ldg, b, R_init, R, nullptr, status, s);
}

}  // namespace l0
