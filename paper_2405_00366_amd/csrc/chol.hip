// FP64 least-squares refit of R on the support (the R-minimisation of eq. 3
// with sigma fixed): R_S = G_SS^-1 b_S through a Cholesky factor, and
// R_r = (b_r - G_rS R_S) / G_rr off the support.
//
// The support size is only known on the device, so the whole refit is one
// cooperative launch: the support is compacted, G_SS is placed in an FP64
// buffer padded to a multiple of 64 with identity, and a blocked
// right-looking factorisation (64 x 64 tiles: diagonal block in one
// workgroup, panel rows and trailing tiles spread over all workgroups) is
// followed by blocked forward and back substitution.  Phases are separated
// by a bounded grid barrier.  A pivot <= 1e-12 * max diag(G_SS) restarts the
// factorisation once with a ridge of 1e-10 * tr(G_SS) / |S|.
//
// Two sources of G_SS and b_S:
//  * from G and b as given (l0cim_update_r with the Cholesky CDP): the
//    entries are widened to FP64, so an FP32 G carries its rounding into the
//    factor;
//  * from A and y (l0cim_refit_f64 and the final refit of every solve form):
//    G_SS = A_S^T A_S, b_S = A_S^T y and, off the support,
//    R_r = a_r^T (y - A_S R_S) / a_r^T a_r, all accumulated in FP64 from the
//    stored A (products of FP32 values are exact in FP64), so the refit does
//    not inherit the cond(G_SS) * 2^-24 error of an FP32 Gram.
#include "kernels.h"

namespace l0 {
namespace {

constexpr int NB = 64;
constexpr int BS = 256;
constexpr int64_t kBarrierLimit = int64_t(1) << 24;

// control words: barrier generation, abort, k, and one failure flag per
// attempt (never reset, so no workgroup can miss a flag)
enum { C_GEN = 1, C_ABORT = 2, C_K = 3, C_BAD0 = 4, C_BAD1 = 5 };

// Phases are separated by the bounded grid barrier of common.h.
#define L0_GRID_SYNC()                                                                  \
  do {                                                                                  \
    if (!grid_barrier<BS>(&ctl[C_GEN], &ctl[C_ABORT], arrive, nwg, gen, kBarrierLimit)) { \
      if (tid == 0) raise_status(status, L0CIM_ST_TIMEOUT);                             \
      return;                                                                           \
    }                                                                                   \
  } while (0)

// max and sum of diag(L) over the first k rows; every workgroup computes the
// same values in the same order
__device__ void diag_stats(const double* L, int kp, int k, double* sh, double& dmax, double& tr) {
  constexpr int NW = BS / 64;
  double mx = 0.0, sm = 0.0;
  for (int i = threadIdx.x; i < k; i += BS) {
    const double d = L[size_t(i) * kp + i];
    mx = fmax(mx, d);
    sm += d;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, off, 64));
    sm += __shfl_xor(sm, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x >> 6] = mx;
    sh[NW + (threadIdx.x >> 6)] = sm;
  }
  __syncthreads();
  dmax = sh[0];
  tr = sh[NW];
  for (int v = 1; v < NW; ++v) {
    dmax = fmax(dmax, sh[v]);
    tr += sh[NW + v];
  }
  __syncthreads();
}

// FROM_A: G_SS, b_S and the off-support rows from A (mrows x n, leading
// dimension lda) and y in FP64; otherwise from G and b.  rho (mrows doubles)
// may alias L: it is written only after the last read of the factor.
template <typename T, bool FROM_A>
__global__ void __launch_bounds__(BS)
chol_kernel(int n, const T* __restrict__ G, int64_t ldg, const T* __restrict__ b,
            int mrows, const T* __restrict__ A, int64_t lda, const T* __restrict__ yv,
            const uint8_t* __restrict__ sigma, T* __restrict__ R, int* __restrict__ status,
            int* __restrict__ idx, double* __restrict__ L, double* __restrict__ w, int* __restrict__ ctl,
            int* __restrict__ arrive) {
  int gen = 0;
  __shared__ double sA[NB][NB + 1];
  __shared__ double sB[NB][NB + 1];
  __shared__ double sv[NB];
  __shared__ double sred[2 * (BS / 64)];
  __shared__ int sIa[NB], sIb[NB];
  __shared__ int cnt[BS];
  __shared__ int flag;
  const int tid = threadIdx.x, wg = blockIdx.x, nwg = gridDim.x;
  const int lane = tid & 63, wv = tid >> 6;

  // 1. compact the support (workgroup 0), max and sum of its diagonal
  if (wg == 0) {
    const int chunk = (n + BS - 1) / BS;
    const int lo = min(n, tid * chunk), hi = min(n, lo + chunk);
    int c = 0;
    for (int i = lo; i < hi; ++i) c += sigma[i] ? 1 : 0;
    int ks = 0;
    int pos = block_exclusive_scan<BS>(c, cnt, &ks);
    if (tid == 0) ctl[C_K] = ks;
    for (int i = lo; i < hi; ++i)
      if (sigma[i]) idx[pos++] = i;
  }
  L0_GRID_SYNC();
  const int k = ctl[C_K];
  const int kp = (k + NB - 1) / NB * NB;
  const int m = kp / NB;
  double dmax = 0.0, trace = 0.0;
  double ridge = 0.0;
  bool ridged = false;

  for (int attempt = 0; attempt < 2 && m > 0; ++attempt) {
    // 2. L <- G_SS (+ ridge I), padded with identity; lower triangle
    if constexpr (FROM_A) {
      // lower 64 x 64 tiles of A_S^T A_S, 64 rows of A per pass through LDS;
      // the diagonal tiles also accumulate w = A_S^T y
      const int ntile = m * (m + 1) / 2;
      for (int t = wg; t < ntile; t += nwg) {
        int bi = 0;
        while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
        const int bj = t - bi * (bi + 1) / 2;
        if (tid < NB) {
          sIa[tid] = bi * NB + tid < k ? idx[bi * NB + tid] : -1;
          sIb[tid] = bj * NB + tid < k ? idx[bj * NB + tid] : -1;
        }
        __syncthreads();
        const int tr = tid / 16, tc = tid % 16;
        double acc[4][4] = {};
        double accb = 0.0;
        for (int q0 = 0; q0 < mrows; q0 += NB) {
          for (int e = tid; e < NB * NB; e += BS) {
            const int r = e % NB, c = e / NB, q = q0 + c;
            const int ia = sIa[r], ja = sIb[r];
            sA[r][c] = (q < mrows && ia >= 0) ? double(A[size_t(q) * lda + ia]) : 0.0;
            sB[r][c] = (q < mrows && ja >= 0) ? double(A[size_t(q) * lda + ja]) : 0.0;
          }
          if (bi == bj && tid < NB) sv[tid] = q0 + tid < mrows ? double(yv[q0 + tid]) : 0.0;
          __syncthreads();
          for (int l = 0; l < NB; ++l) {
            double a4[4], b4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              a4[u] = sA[tr + 16 * u][l];
              b4[u] = sB[tc + 16 * u][l];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
              for (int v = 0; v < 4; ++v) acc[u][v] = fma(a4[u], b4[v], acc[u][v]);
          }
          if (bi == bj && tid < NB)
            for (int l = 0; l < NB; ++l) accb = fma(sA[tid][l], sv[l], accb);
          __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = tr + 16 * u, c = tc + 16 * v;
            const int gi = bi * NB + r, gj = bj * NB + c;
            if (bi == bj && c > r) continue;
            double x;
            if (gi < k && gj < k) x = acc[u][v] + (gi == gj ? ridge : 0.0);
            else x = (gi == gj) ? 1.0 : 0.0;
            L[size_t(gi) * kp + gj] = x;
          }
        if (bi == bj && tid < NB) w[bi * NB + tid] = bi * NB + tid < k ? accb : 0.0;
      }
    } else {
      for (size_t e = size_t(wg) * BS + tid; e < size_t(kp) * kp; e += size_t(nwg) * BS) {
        const int i = int(e / kp), j = int(e - size_t(i) * kp);
        if (j > i) continue;
        double v;
        if (i < k && j < k) v = double(G[size_t(idx[i]) * ldg + idx[j]]) + (i == j ? ridge : 0.0);
        else v = (i == j) ? 1.0 : 0.0;
        L[size_t(i) * kp + j] = v;
      }
    }
    L0_GRID_SYNC();
    if (attempt == 0) diag_stats(L, kp, k, sred, dmax, trace);
    bool bad = false;
    for (int kb = 0; kb < m; ++kb) {
      const int k0 = kb * NB;
      // 3a. diagonal block, one workgroup
      if (wg == 0) {
        for (int e = tid; e < NB * NB; e += BS) {
          const int i = e / NB, j = e % NB;
          sA[i][j] = j <= i ? L[size_t(k0 + i) * kp + k0 + j] : 0.0;
        }
        if (tid == 0) flag = 0;
        __syncthreads();
        for (int j = 0; j < NB; ++j) {
          if (tid == 0) {
            const double piv = sA[j][j];
            if (!(piv > 1e-12 * dmax) && k0 + j < k) flag = 1;
            sA[j][j] = sqrt(fmax(piv, 1e-300));
          }
          __syncthreads();
          if (flag) break;
          for (int i = j + 1 + tid; i < NB; i += BS) sA[i][j] /= sA[j][j];
          __syncthreads();
          const int r = NB - j - 1;
          for (int e = tid; e < r * r; e += BS) {
            const int i = j + 1 + e / r, l = j + 1 + e % r;
            if (l <= i) sA[i][l] -= sA[i][j] * sA[l][j];
          }
          __syncthreads();
        }
        if (flag) {
          if (tid == 0) ctl[C_BAD0 + attempt] = 1;
        } else {
          for (int e = tid; e < NB * NB; e += BS) {
            const int i = e / NB, j = e % NB;
            if (j <= i) L[size_t(k0 + i) * kp + k0 + j] = sA[i][j];
          }
        }
      }
      L0_GRID_SYNC();
      if (ctl[C_BAD0 + attempt]) {
        bad = true;
        break;
      }
      // 3b. panel: X L_kk^T = A_ik for every row block below
      for (int ib = kb + 1 + wg; ib < m; ib += nwg) {
        for (int e = tid; e < NB * NB; e += BS) {
          const int i = e / NB, j = e % NB;
          sA[i][j] = j <= i ? L[size_t(k0 + i) * kp + k0 + j] : 0.0;
          sB[i][j] = L[size_t(ib * NB + i) * kp + k0 + j];
        }
        __syncthreads();
        if (tid < NB) {
          const int i = tid;
          for (int j = 0; j < NB; ++j) {
            double x = sB[i][j];
            for (int l = 0; l < j; ++l) x -= sB[i][l] * sA[j][l];
            sB[i][j] = x / sA[j][j];
          }
        }
        __syncthreads();
        for (int e = tid; e < NB * NB; e += BS) {
          const int i = e / NB, j = e % NB;
          L[size_t(ib * NB + i) * kp + k0 + j] = sB[i][j];
        }
        __syncthreads();
      }
      L0_GRID_SYNC();
      // 3c. trailing update of the lower blocks (i, j), kb < j <= i < m
      const int mt = m - kb - 1;
      const int ntile = mt * (mt + 1) / 2;
      for (int t = wg; t < ntile; t += nwg) {
        int i = 0;
        while ((i + 1) * (i + 2) / 2 <= t) ++i;
        const int j = t - i * (i + 1) / 2;
        const int bi = kb + 1 + i, bj = kb + 1 + j;
        for (int e = tid; e < NB * NB; e += BS) {
          const int r = e / NB, c = e % NB;
          sA[r][c] = L[size_t(bi * NB + r) * kp + k0 + c];
          sB[r][c] = L[size_t(bj * NB + r) * kp + k0 + c];
        }
        __syncthreads();
        const int tr = tid / 16, tc = tid % 16;
        double acc[4][4] = {};
        for (int l = 0; l < NB; ++l) {
          double a4[4], b4[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            a4[u] = sA[tr + 16 * u][l];
            b4[u] = sB[tc + 16 * u][l];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = fma(a4[u], b4[v], acc[u][v]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = tr + 16 * u, c = tc + 16 * v;
            if (bi != bj || c <= r) L[size_t(bi * NB + r) * kp + bj * NB + c] -= acc[u][v];
          }
        __syncthreads();
      }
      L0_GRID_SYNC();
    }
    if (!bad) break;
    // ridge and retry once
    ridged = true;
    ridge = 1e-10 * trace / double(k);
  }

  // 4. forward substitution L v = b_S, then back substitution L^T x = v
  if constexpr (!FROM_A) {
    for (size_t a = size_t(wg) * BS + tid; a < size_t(kp); a += size_t(nwg) * BS)
      w[a] = a < size_t(k) ? double(b[idx[a]]) : 0.0;
  }
  L0_GRID_SYNC();
  for (int kb = 0; kb < m; ++kb) {
    const int k0 = kb * NB;
    if (wg == 0) {
      for (int e = tid; e < NB * NB; e += BS) {
        const int i = e / NB, j = e % NB;
        sA[i][j] = j <= i ? L[size_t(k0 + i) * kp + k0 + j] : 0.0;
      }
      if (tid < NB) sv[tid] = w[k0 + tid];
      __syncthreads();
      for (int j = 0; j < NB; ++j) {
        if (tid == 0) sv[j] /= sA[j][j];
        __syncthreads();
        for (int i = j + 1 + tid; i < NB; i += BS) sv[i] -= sA[i][j] * sv[j];
        __syncthreads();
      }
      if (tid < NB) w[k0 + tid] = sv[tid];
    }
    L0_GRID_SYNC();
    for (int ib = kb + 1 + wg; ib < m; ib += nwg) {
      if (tid < NB) sv[tid] = w[k0 + tid];
      __syncthreads();
      if (tid < NB) {
        double acc = 0.0;
        const double* Lr = L + size_t(ib * NB + tid) * kp + k0;
        for (int l = 0; l < NB; ++l) acc = fma(Lr[l], sv[l], acc);
        w[ib * NB + tid] -= acc;
      }
      __syncthreads();
    }
    L0_GRID_SYNC();
  }
  for (int kb = m - 1; kb >= 0; --kb) {
    const int k0 = kb * NB;
    if (wg == 0) {
      for (int e = tid; e < NB * NB; e += BS) {
        const int i = e / NB, j = e % NB;
        sA[i][j] = j <= i ? L[size_t(k0 + i) * kp + k0 + j] : 0.0;
      }
      if (tid < NB) sv[tid] = w[k0 + tid];
      __syncthreads();
      for (int j = NB - 1; j >= 0; --j) {
        if (tid == 0) sv[j] /= sA[j][j];
        __syncthreads();
        for (int i = tid; i < j; i += BS) sv[i] -= sA[j][i] * sv[j];
        __syncthreads();
      }
      if (tid < NB) w[k0 + tid] = sv[tid];
    }
    L0_GRID_SYNC();
    for (int ib = wg; ib < kb; ib += nwg) {
      if (tid < NB) sv[tid] = w[k0 + tid];
      __syncthreads();
      if (tid < NB) {
        double acc = 0.0;
        for (int l = 0; l < NB; ++l) acc = fma(L[size_t(k0 + l) * kp + ib * NB + tid], sv[l], acc);
        w[ib * NB + tid] -= acc;
      }
      __syncthreads();
    }
    L0_GRID_SYNC();
  }

  // 5. R on the support, and the off-support rows
  for (size_t a = size_t(wg) * BS + tid; a < size_t(k); a += size_t(nwg) * BS) R[idx[a]] = T(w[a]);
  int bits = 0;
  if constexpr (FROM_A) {
    // residual rho = y - A_S R_S (one wavefront per row of A), into the
    // factor's storage, which is no longer read
    double* rho = L;
    for (int q = wg * (BS / 64) + wv; q < mrows; q += nwg * (BS / 64)) {
      double acc = 0.0;
      for (int a = lane; a < k; a += 64) acc = fma(double(A[size_t(q) * lda + idx[a]]), w[a], acc);
      acc = wave_sum(acc);
      if (lane == 0) rho[q] = double(yv[q]) - acc;
    }
    L0_GRID_SYNC();
    // R_r = a_r^T rho / a_r^T a_r: 64 columns per workgroup, the rows of A
    // split over its wavefronts and their partial sums added in order
    double* part = &sA[0][0];
    for (int c0 = wg * 64; c0 < n; c0 += nwg * 64) {
      const int r = c0 + lane;
      double num = 0.0, den = 0.0;
      if (r < n)
        for (int q = wv; q < mrows; q += BS / 64) {
          const double a = double(A[size_t(q) * lda + r]);
          num = fma(a, rho[q], num);
          den = fma(a, a, den);
        }
      part[wv * 64 + lane] = num;
      part[BS + wv * 64 + lane] = den;
      __syncthreads();
      if (wv == 0) {
        bool tiny = false;
        if (r < n) {
          for (int v = 1; v < BS / 64; ++v) {
            num += part[v * 64 + lane];
            den += part[BS + v * 64 + lane];
          }
          tiny = !(den >= 1e-12);
          if (!sigma[r]) R[r] = tiny ? T(0) : T(num / den);
        }
        if (__any(tiny)) bits |= L0CIM_ST_TINY_DIAG;   // lane 0 raises the wave's bits
      }
      __syncthreads();
    }
  } else for (int r = wg * (BS / 64) + wv; r < n; r += nwg * (BS / 64)) {
    const T d = G[size_t(r) * ldg + r];
    const bool tiny = !(d >= T(1e-12));
    if (tiny) bits |= L0CIM_ST_TINY_DIAG;
    if (sigma[r]) continue;
    double acc = 0.0;
    for (int a = lane; a < k; a += 64) acc += double(G[size_t(r) * ldg + idx[a]]) * w[a];
    acc = wave_sum(acc);
    if (lane == 0) R[r] = tiny ? T(0) : T((double(b[r]) - acc) / double(d));
  }
  if (ridged && wg == 0 && tid == 0) bits |= L0CIM_ST_CHOL_RIDGE;
  if (bits && lane == 0) raise_status(status, bits);
}

struct CholLayout {
  size_t idx, L, w, ctl, arrive, total;
};

// The factor's storage also holds the residual of the A-based refit, so it
// is at least `mrows` doubles.
CholLayout chol_layout(int n, int mrows) {
  const size_t np = size_t(n + NB - 1) / NB * NB;
  size_t lsz = np * np;
  if (size_t(mrows) > lsz) lsz = size_t(mrows);
  CholLayout c;
  size_t o = 0;
  auto take = [&](size_t bb) {
    size_t at = o;
    o += align_up(bb);
    return at;
  };
  c.idx = take(size_t(n) * sizeof(int));
  c.L = take(lsz * sizeof(double));
  c.w = take(np * sizeof(double));
  c.ctl = take(8 * sizeof(int));
  c.arrive = take(size_t(kGridMaxWg) * kGridSlot * sizeof(int));
  c.total = o;
  return c;
}

__global__ void chol_ctl_clear_kernel(int* ctl, int* arrive) {
  if (threadIdx.x < 8) ctl[threadIdx.x] = 0;
  for (int i = threadIdx.x; i < kGridMaxWg; i += blockDim.x) arrive[i * kGridSlot] = 0;
}

template <typename T, bool FROM_A>
l0cim_status chol_typed(int n, const T* G, int64_t ldg, const T* b, int mrows, const T* A, int64_t lda,
                        const T* y, const uint8_t* sigma, T* R, int* status, void* ws, hipStream_t s) {
  DeviceInfo dev;
  l0cim_status st = device_info(&dev);
  if (st != L0CIM_OK) return st;
  const CholLayout c = chol_layout(n, FROM_A ? mrows : 0);
  char* base = static_cast<char*>(ws);
  int* idx = reinterpret_cast<int*>(base + c.idx);
  double* L = reinterpret_cast<double*>(base + c.L);
  double* w = reinterpret_cast<double*>(base + c.w);
  int* ctl = reinterpret_cast<int*>(base + c.ctl);
  int* arrive = reinterpret_cast<int*>(base + c.arrive);
  hipLaunchKernelGGL(chol_ctl_clear_kernel, dim3(1), dim3(256), 0, s, ctl, arrive);
  L0_LAUNCHED("chol_ctl_clear_kernel");
  const void* fn = reinterpret_cast<const void*>(chol_kernel<T, FROM_A>);
  int per_cu = 0;
  L0_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, BS, 0));
  int grid = dev.cu_count * (per_cu > 0 ? 1 : 0);
  if (grid > kGridMaxWg) grid = kGridMaxWg;
  if (grid < 1) return set_error(L0CIM_ERR_HIP, "chol refit: kernel does not fit on a CU");
  int nn = n, mm = mrows;
  void* args[] = {&nn, &G, &ldg, &b, &mm, &A, &lda, &y, &sigma, &R, &status, &idx, &L, &w, &ctl, &arrive};
  L0_HIP(hipLaunchCooperativeKernel(fn, dim3(grid), dim3(BS), args, 0, s));
  return L0CIM_OK;
}

}  // namespace

size_t chol_ws_bytes(int n) { return chol_layout(n, 0).total; }
size_t chol_a_ws_bytes(int n, int m) { return chol_layout(n, m).total; }

l0cim_status launch_chol_refit(l0cim_dtype dt, int n, const void* G, int64_t ldg, const void* b,
                               const uint8_t* sigma, void* R, int* status, void* ws, size_t ws_bytes,
                               hipStream_t s) {
  if (!ws || ws_bytes < chol_ws_bytes(n)) return set_error(L0CIM_ERR_WORKSPACE, "chol refit: workspace too small");
  if (dt == L0CIM_F32)
    return chol_typed<float, false>(n, (const float*)G, ldg, (const float*)b, 0, nullptr, 0, nullptr, sigma,
                                    (float*)R, status, ws, s);
  if (dt == L0CIM_F64)
    return chol_typed<double, false>(n, (const double*)G, ldg, (const double*)b, 0, nullptr, 0, nullptr, sigma,
                                     (double*)R, status, ws, s);
  return set_error(L0CIM_ERR_UNSUPPORTED, "chol refit: dtype %d", int(dt));
}

l0cim_status launch_chol_refit_a(l0cim_dtype dt, int m, int n, const void* A, int64_t lda, const void* y,
                                 const uint8_t* sigma, void* R, int* status, void* ws, size_t ws_bytes,
                                 hipStream_t s) {
  if (!ws || ws_bytes < chol_a_ws_bytes(n, m))
    return set_error(L0CIM_ERR_WORKSPACE, "FP64 refit: workspace too small");
  if (dt == L0CIM_F32)
    return chol_typed<float, true>(n, nullptr, 0, nullptr, m, (const float*)A, lda, (const float*)y, sigma,
                                   (float*)R, status, ws, s);
  if (dt == L0CIM_F64)
    return chol_typed<double, true>(n, nullptr, 0, nullptr, m, (const double*)A, lda, (const double*)y, sigma,
                                    (double*)R, status, ws, s);
  return set_error(L0CIM_ERR_UNSUPPORTED, "FP64 refit: dtype %d", int(dt));
}

}  // namespace l0
