// Gram and Zeeman preparation: G = A^T A, b = A^T y (the negated couplings
// and the Zeeman term over sqrt(tau), stated after eq. 11 and eq. 15).
//
// G is computed with an LDS-tiled outer-product kernel; every output element
// accumulates over k in the same order with explicit FMAs, so G_ij and G_ji
// are bitwise equal.
#include "kernels.h"

namespace l0 {
namespace {

constexpr int kTile = 64;
constexpr int kK = 16;

template <typename T>
__device__ inline T fma_t(T a, T b, T c);
template <>
__device__ inline float fma_t<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ inline double fma_t<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__global__ void __launch_bounds__(256)
gram_kernel(int m, int n, const T* __restrict__ A, int64_t lda, T* __restrict__ G, int64_t ldg) {
  __shared__ T As[kK][kTile];
  __shared__ T Bs[kK][kTile];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.y * kTile, j0 = blockIdx.x * kTile;
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = T(0);

  for (int k0 = 0; k0 < m; k0 += kK) {
    // 16 x 64 elements of each operand, 4 per thread, coalesced along the row.
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int idx = threadIdx.x + u * 256;
      int kk = idx >> 6, cc = idx & 63;
      int k = k0 + kk;
      int gi = i0 + cc, gj = j0 + cc;
      As[kk][cc] = (k < m && gi < n) ? A[size_t(k) * lda + gi] : T(0);
      Bs[kk][cc] = (k < m && gj < n) ? A[size_t(k) * lda + gj] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kK; ++kk) {
      T av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[kk][ty + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma_t(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int i = i0 + ty + 16 * a;
    if (i >= n) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int j = j0 + tx + 16 * b;
      if (j < n) G[size_t(i) * ldg + j] = acc[a][b];
    }
  }
}

// b_j = sum_k A_kj y_k: 64 columns per workgroup, four k-phases summed in a
// fixed order.
template <typename T>
__global__ void __launch_bounds__(256)
aty_kernel(int m, int n, const T* __restrict__ A, int64_t lda, const T* __restrict__ y, T* __restrict__ b) {
  __shared__ T part[4][64];
  const int col = threadIdx.x & 63, ph = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + col;
  T acc = T(0);
  if (j < n)
    for (int k = ph; k < m; k += 4) acc = fma_t(A[size_t(k) * lda + j], y[k], acc);
  part[ph][col] = acc;
  __syncthreads();
  if (ph == 0 && j < n) b[j] = ((part[0][col] + part[1][col]) + part[2][col]) + part[3][col];
}

template <typename T>
l0cim_status gram_typed(int m, int n, const T* A, int64_t lda, const T* y, T* G, int64_t ldg, T* b,
                        hipStream_t s) {
  dim3 grid((n + kTile - 1) / kTile, (n + kTile - 1) / kTile);
  hipLaunchKernelGGL(gram_kernel<T>, grid, dim3(256), 0, s, m, n, A, lda, G, ldg);
  L0_LAUNCHED("gram_kernel");
  hipLaunchKernelGGL(aty_kernel<T>, dim3((n + 63) / 64), dim3(256), 0, s, m, n, A, lda, y, b);
  L0_LAUNCHED("aty_kernel");
  return L0CIM_OK;
}

}  // namespace

l0cim_status launch_gram(l0cim_dtype dt, int m, int n, const void* A, int64_t lda, const void* y,
                         void* G, int64_t ldg, void* b, hipStream_t s) {
  if (dt == L0CIM_F32)
    return gram_typed<float>(m, n, static_cast<const float*>(A), lda, static_cast<const float*>(y),
                             static_cast<float*>(G), ldg, static_cast<float*>(b), s);
  if (dt == L0CIM_F64)
    return gram_typed<double>(m, n, static_cast<const double*>(A), lda, static_cast<const double*>(y),
                              static_cast<double*>(G), ldg, static_cast<double*>(b), s);
  return set_error(L0CIM_ERR_UNSUPPORTED, "gram: dtype %d", int(dt));
}

}  // namespace l0
