// Gram and Zeeman preparation: G = A^T A, b = A^T y (the negated couplings
// and the Zeeman term over sqrt(tau), stated after eq. 11 and eq. 15).
//
// FP32: the matrix cores compute the 128 x 128 tiles on and above the
// diagonal and each value is written to G_ij and G_ji, so G is bitwise
// symmetric and half the products are formed.  FP64: an LDS-tiled
// outer-product kernel in which every element accumulates over k in the same
// order with explicit FMAs (again G_ij and G_ji bitwise equal).
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

typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kMT = 128;        // output tile
constexpr int kMK = 32;         // rows of A per chunk
constexpr int kLdsK = kMK + 4;  // padded LDS row: 16 consecutive rows fall in distinct banks

// One workgroup per tile (I, J), I <= J, of the upper triangle; 4 wavefronts
// of 64 x 64 (4 x 4 blocks of 16 x 16).  A chunk of 32 rows of A is staged
// in LDS column-major (the 32 values of a column contiguous, padded to 36),
// each thread loading four consecutive rows of one column per quad (the
// wavefront's loads are coalesced along the row) and storing them with one
// 16-byte write.  In half h of a chunk the matrix-core step s of lane group g
// uses row 16 h + 4 g + s on both operands, so each lane reads its 4 values
// of a column with one 16-byte load, and every G entry accumulates its
// products in the same order for any chunk length.
__global__ void __launch_bounds__(256)
gram_mfma_kernel(int m, int n, const float* __restrict__ A, int64_t lda, float* __restrict__ G, int64_t ldg,
                 int tiles) {
  __shared__ __align__(16) float As[kMT][kLdsK];
  __shared__ __align__(16) float Bs[kMT][kLdsK];
  // tile (I, J) of the upper triangle, row by row
  int I = 0, rem = blockIdx.x;
  while (rem >= tiles - I) {
    rem -= tiles - I;
    ++I;
  }
  const int J = I + rem;
  const bool diag = I == J;
  const int i0 = I * kMT, j0 = J * kMT;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int c = lane & 15, g = lane >> 4;
  v4f acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  // loader: thread t moves column t % 128 of the tile, row quads t / 128 + 2 q (q < kMK / 8)
  constexpr int NQ = kMK / 8;
  const int lcol = t & (kMT - 1), lq = t >> 7;
  auto fetch = [&](int k0, int col0, v4f (&v)[NQ]) {
    const int col = col0 + lcol;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = k0 + 4 * (lq + 2 * q);
#pragma unroll
      for (int u = 0; u < 4; ++u) v[q][u] = (k + u < m && col < n) ? A[size_t(k + u) * lda + col] : 0.0f;
    }
  };
  v4f va[NQ], vb[NQ];
  fetch(0, i0, va);
  if (!diag) fetch(0, j0, vb);
  for (int k0 = 0; k0 < m; k0 += kMK) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      *reinterpret_cast<v4f*>(&As[lcol][4 * (lq + 2 * q)]) = va[q];
      if (!diag) *reinterpret_cast<v4f*>(&Bs[lcol][4 * (lq + 2 * q)]) = vb[q];
    }
    __syncthreads();
    if (k0 + kMK < m) {
      fetch(k0 + kMK, i0, va);
      if (!diag) fetch(k0 + kMK, j0, vb);
    }
    const float(*Bp)[kLdsK] = diag ? As : Bs;
#pragma unroll
    for (int h = 0; h < kMK / 16; ++h) {
      v4f ra[4], rb[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) ra[a] = *reinterpret_cast<const v4f*>(&As[wr * 64 + a * 16 + c][16 * h + 4 * g]);
#pragma unroll
      for (int b = 0; b < 4; ++b) rb[b] = *reinterpret_cast<const v4f*>(&Bp[wc * 64 + b * 16 + c][16 * h + 4 * g]);
#pragma unroll
      for (int st = 0; st < 4; ++st)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra[a][st], rb[b][st], acc[a][b], 0, 0, 0);
    }
  }
  // lane holds D[4 g + v][c] of block (a, b): row i0 + 64 wr + 16 a + 4 g + v, column j0 + 64 wc + 16 b + c
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = j0 + wc * 64 + b * 16 + c;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wr * 64 + a * 16 + 4 * g + v;
        if (i < n && j < n && (!diag || i <= j)) {
          G[size_t(i) * ldg + j] = acc[a][b][v];
          G[size_t(j) * ldg + i] = acc[a][b][v];
        }
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
  if constexpr (sizeof(T) == 4) {
    const int tiles = (n + kMT - 1) / kMT;
    hipLaunchKernelGGL(gram_mfma_kernel, dim3(unsigned(int64_t(tiles) * (tiles + 1) / 2)), dim3(256), 0, s, m, n,
                       A, lda, G, ldg, tiles);
    L0_LAUNCHED("gram_mfma_kernel");
  } else {
    dim3 grid((n + kTile - 1) / kTile, (n + kTile - 1) / kTile);
    hipLaunchKernelGGL(gram_kernel<T>, grid, dim3(256), 0, s, m, n, A, lda, G, ldg);
    L0_LAUNCHED("gram_kernel");
  }
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
