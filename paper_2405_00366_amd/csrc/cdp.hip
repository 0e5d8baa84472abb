// Classical digital processing (CDP): the R-minimisation of Algorithm 1.
//  * Jacobi relaxation with time increment dtc over every r, synchronously
//    (parameter paragraph of the numerical experiments: dtc = 0.1, 100
//    iterations).  Resident form: rows of G stay in LDS and the vector
//    s = sigma o R travels through flag-carrying words, as in the CIM run.
//  * Support form (FP32, support of at most 256 spins): only the support's
//    R enter the sums, so its sweeps run in one workgroup with G_SS in
//    registers; an off-support R is an affine function of the support's R
//    history, R_r(K) = f R_r(0) + (1 - f) b_r / G_rr - (dtc / G_rr) G_rS V
//    with f = (1 - dtc)^K and V = sum_k (1 - dtc)^(K-1-k) R_S(k), which is
//    the same K synchronous sweeps unrolled.
//  * eq. 3 objective and the per-solve report.
#include "kernels.h"

namespace l0 {
namespace {

__host__ __device__ inline size_t a16(size_t x) { return (x + 15) & ~size_t(15); }

template <typename T>
__host__ __device__ inline size_t jacobi_lds(int n, int rpw) {
  return a16(size_t(rpw) * n * sizeof(T)) + a16(size_t(n) * sizeof(T)) + 4 * a16(size_t(rpw) * sizeof(T)) + 16;
}

template <typename T>
__device__ inline void jacobi_update(T& R, T off, T br, T d, T dtc, bool tiny) {
  R = tiny ? T(0) : R + dtc * ((br - off) / d - R);
}

constexpr int kSupportMax = 256;

// Control block of the support form: [0] = 1 when it has done the update,
// [1] = support size; then the support list and V.
struct SupportCtl {
  int* flag;
  int* list;
  float* V;
};

// flag words at 0, the support list at 256, V at 256 + 4 kSupportMax
constexpr size_t kCtlList = 256, kCtlV = kCtlList + 4 * kSupportMax;

inline size_t support_ctl_bytes() { return kCtlV + 4 * kSupportMax; }

__device__ inline SupportCtl support_ctl(void* p) {
  char* c = static_cast<char*>(p);
  return SupportCtl{reinterpret_cast<int*>(c), reinterpret_cast<int*>(c + kCtlList),
                    reinterpret_cast<float*>(c + kCtlV)};
}

// One workgroup of 1024 threads: thread t holds the 4 x 16 block of G_SS at
// rows 4 (t / 16) + i, columns 16 (t % 16) + u in registers (diagonal
// zeroed).  Per sweep each thread reads its 16 amplitudes from LDS, the 16
// lanes of a row group reduce their 4 row sums with a transposed butterfly,
// and lane 4 i of the group owns row i.  R_S is double-buffered in LDS.
__global__ void __launch_bounds__(1024)
jacobi_support_kernel(int n, const float* __restrict__ G, int64_t ldg, const float* __restrict__ b,
                      const uint8_t* __restrict__ sigma, float dtc, int iters, float* __restrict__ R,
                      int* __restrict__ status, void* ctl_p) {
  __shared__ int scan_sh[1024 / kWave + 1];
  __shared__ int S[kSupportMax];
  __shared__ __align__(16) float Rb[2][kSupportMax];
  const SupportCtl ctl = support_ctl(ctl_p);
  const int t = threadIdx.x, lane = t & (kWave - 1);
  const int chunk = (n + 1023) / 1024;
  const int lo = min(n, t * chunk), hi = min(n, lo + chunk);
  int c = 0;
  for (int i = lo; i < hi; ++i) c += sigma[i] ? 1 : 0;
  int ks = 0;
  int at = block_exclusive_scan<1024>(c, scan_sh, &ks);
  if (t == 0) {
    ctl.flag[0] = ks <= kSupportMax ? 1 : 0;
    ctl.flag[1] = ks;
  }
  if (ks > kSupportMax || ks == 0) return;   // too large: the resident form runs; empty: nothing here
  for (int i = lo; i < hi; ++i)
    if (sigma[i]) {
      S[at] = i;
      ctl.list[at] = i;
      ++at;
    }
  for (int j = ks + t; j < kSupportMax; j += 1024) {
    Rb[0][j] = 0.0f;
    Rb[1][j] = 0.0f;
  }
  __syncthreads();
  const int rg = t >> 4, cg = t & 15;
  float g[4][16];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = 4 * rg + i;
    const int r = row < ks ? S[row] : 0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int col = 16 * cg + u;
      g[i][u] = (row < ks && col < ks && col != row) ? G[size_t(r) * ldg + S[col < ks ? col : 0]] : 0.0f;
    }
  }
  // row owned by this lane (lanes 4 i of each 16-lane group), see wave_sum_rows_level
  const int orow = 4 * rg + ((lane >> 2) & 3);
  const bool own = (lane & 3) == 0 && orow < ks;
  const int r = own ? S[orow] : 0;
  const float d = own ? G[size_t(r) * ldg + r] : 1.0f;
  const bool tiny = !(d >= 1e-12f);
  const float br = own ? b[r] : 0.0f;
  if (own) Rb[0][orow] = tiny ? 0.0f : R[r];
  float V = 0.0f;
  // wavefront w holds rows 16 w .. 16 w + 15: the ones past the support skip the sweeps
  const bool wave_on = 16 * (t / kWave) < ks;
  __syncthreads();
  for (int it = 0; it < iters; ++it) {
    if (wave_on) {
      const float4* x4 = reinterpret_cast<const float4*>(Rb[it & 1] + 16 * cg);
      float x[16];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 v = x4[q];
        x[4 * q] = v.x;
        x[4 * q + 1] = v.y;
        x[4 * q + 2] = v.z;
        x[4 * q + 3] = v.w;
      }
      float acc[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        acc[i] = 0.0f;
#pragma unroll
        for (int u = 0; u < 16; ++u) acc[i] += g[i][u] * x[u];
      }
      wave_sum_rows_level<float, 4, 4, 8>(acc, lane);
      if (own) {
        const float Rv = Rb[it & 1][orow];
        V = (1.0f - dtc) * V + Rv;
        Rb[(it + 1) & 1][orow] = tiny ? 0.0f : Rv + dtc * ((br - acc[0]) / d - Rv);
      }
    }
    __syncthreads();
  }
  if (own) {
    R[r] = Rb[iters & 1][orow];
    ctl.V[orow] = V;
    if (tiny) raise_status(status, L0CIM_ST_TINY_DIAG);
  }
}

// Off-support rows after the support form: one wavefront per row.
__global__ void __launch_bounds__(256)
jacobi_offsupport_kernel(int n, const float* __restrict__ G, int64_t ldg, const float* __restrict__ b,
                         const uint8_t* __restrict__ sigma, float dtc, int iters, float* __restrict__ R,
                         int* __restrict__ status, void* ctl_p) {
  const SupportCtl ctl = support_ctl(ctl_p);
  if (ctl.flag[0] == 0) return;
  const int ks = ctl.flag[1];
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n || sigma[r]) return;
  float acc = 0.0f;
  for (int s = lane; s < ks; s += kWave) acc += G[size_t(r) * ldg + ctl.list[s]] * ctl.V[s];
  acc = wave_sum(acc);
  if (lane == 0) {
    const float d = G[size_t(r) * ldg + r];
    const bool tiny = !(d >= 1e-12f);
    float f = 1.0f;
    for (int k = 0; k < iters; ++k) f *= (1.0f - dtc);
    R[r] = tiny ? 0.0f : f * R[r] + (1.0f - f) * (b[r] / d) - (dtc / d) * acc;
    if (tiny) raise_status(status, L0CIM_ST_TINY_DIAG);
  }
}

template <typename T>
__global__ void __launch_bounds__(512)
jacobi_resident_kernel(int n, const T* __restrict__ G, int64_t ldg, const T* __restrict__ b,
                       const uint8_t* __restrict__ sigma, T dtc, int iters, T* __restrict__ R,
                       uint64_t* __restrict__ ll, int* __restrict__ abort_word, int* __restrict__ status,
                       int64_t limit, int rpw, const int* __restrict__ done) {
  if (done && done[0]) return;   // the support form has already updated R
  constexpr int W = LL<T>::kWords;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, bs = blockDim.x;
  const int lane = tid & (kWave - 1), wv = tid / kWave, nwv = bs / kWave;
  const int r0 = blockIdx.x * rpw;
  const int nr = max(0, min(n, r0 + rpw) - r0);
  const bool solo = gridDim.x == 1;
  const size_t slot_words = size_t(n) * W;

  size_t o = 0;
  T* Gl = reinterpret_cast<T*>(smem + o); o += a16(size_t(rpw) * n * sizeof(T));
  T* X = reinterpret_cast<T*>(smem + o);  o += a16(size_t(n) * sizeof(T));
  T* Rs = reinterpret_cast<T*>(smem + o); o += a16(size_t(rpw) * sizeof(T));
  T* Ds = reinterpret_cast<T*>(smem + o); o += a16(size_t(rpw) * sizeof(T));
  T* Bs = reinterpret_cast<T*>(smem + o); o += a16(size_t(rpw) * sizeof(T));
  T* Sg = reinterpret_cast<T*>(smem + o); o += a16(size_t(rpw) * sizeof(T));
  int* lds_abort = reinterpret_cast<int*>(smem + o);

  for (size_t i = tid; i < size_t(nr) * n; i += bs) {
    size_t rl = i / n, j = i - rl * n;
    Gl[i] = G[size_t(r0 + rl) * ldg + j];
  }
  int bits = 0;
  for (int i = tid; i < nr; i += bs) {
    const int r = r0 + i;
    const T d = G[size_t(r) * ldg + r];
    const bool tiny = !(d >= T(1e-12));
    if (tiny) bits |= L0CIM_ST_TINY_DIAG;
    Ds[i] = d;
    Bs[i] = b[r];
    Sg[i] = sigma[r] ? T(1) : T(0);
    Rs[i] = tiny ? T(0) : R[r];
  }
  if (tid == 0) *lds_abort = 0;
  __syncthreads();
  if (!solo)
    for (int i = tid; i < nr; i += bs) LL<T>::put(ll + size_t(r0 + i) * W, Sg[i] * Rs[i], 1u);

  bool aborted = false;
  for (int it = 0; it < iters; ++it) {
    if (solo) {
      for (int i = tid; i < n; i += bs) X[i] = Sg[i] * Rs[i];
    } else {
      bool ok = ll_gather<T>(ll + size_t(it & 1) * slot_words, n, uint32_t(it + 1), limit,
                             abort_word, [&](int idx, T v) { X[idx] = v; });
      if (!ok) {
        *lds_abort = 1;
        __hip_atomic_store(abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
    if (*lds_abort) {
      aborted = true;
      break;
    }
    for (int rl = wv; rl < nr; rl += nwv) {
      const int r = r0 + rl;
      const T* gr = Gl + size_t(rl) * n;
      T acc = T(0);
      for (int j = lane; j < n; j += kWave)
        if (j != r) acc += gr[j] * X[j];
      acc = wave_sum(acc);
      if (lane == 0) {
        T Rv = Rs[rl];
        jacobi_update(Rv, acc, Bs[rl], Ds[rl], dtc, !(Ds[rl] >= T(1e-12)));
        Rs[rl] = Rv;
        if (!solo)
          LL<T>::put(ll + size_t((it + 1) & 1) * slot_words + size_t(r) * W, Sg[rl] * Rv,
                     uint32_t(it + 2));
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < nr; i += bs) R[r0 + i] = Rs[i];
  if (aborted) bits |= L0CIM_ST_TIMEOUT;
  if (bits) raise_status(status, bits);
}

// Streamed Jacobi sweep (G too large for the resident form): one launch per
// sweep, one wavefront per row.
// Streamed sweeps in one cooperative launch (when the support form did not
// run): s = sigma o R (R held at 0 where G_rr is tiny), then K synchronous
// sweeps, one wavefront per row reading its row of G, with a grid barrier
// before each.  Returns at once in every workgroup when the support form has
// updated R.
template <typename T>
__global__ void __launch_bounds__(256)
jacobi_streamed_kernel(int n, const T* __restrict__ G, int64_t ldg, const T* __restrict__ b,
                       const uint8_t* __restrict__ sigma, T dtc, int iters, T* __restrict__ s0, T* __restrict__ s1,
                       T* __restrict__ R, int* __restrict__ status, const int* __restrict__ done, int* __restrict__ bar,
                       int64_t limit) {
  if (done[0]) return;
  int gen = 0;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) {
    const T d = G[size_t(r) * ldg + r];
    if (!(d >= T(1e-12))) R[r] = T(0);
    s0[r] = sigma[r] ? R[r] : T(0);
  }
  const int lane = threadIdx.x & (kWave - 1);
  for (int it = 0; it < iters; ++it) {
    if (!grid_barrier<256>(bar, bar + 1, bar + 64, gridDim.x, gen, limit)) {
      if (threadIdx.x == 0) raise_status(status, L0CIM_ST_TIMEOUT);
      return;
    }
    const T* sin = (it & 1) ? s1 : s0;
    T* sout = (it & 1) ? s0 : s1;
    for (int r = blockIdx.x * 4 + threadIdx.x / kWave; r < n; r += gridDim.x * 4) {
      const T* gr = G + size_t(r) * ldg;
      const T d = gr[r];
      const bool tiny = !(d >= T(1e-12));
      T acc = T(0);
      for (int j = lane; j < n; j += kWave)
        if (j != r) acc += gr[j] * sin[j];
      acc = wave_sum(acc);
      if (lane == 0) {
        T Rv = R[r];
        if (it == 0 && tiny) raise_status(status, L0CIM_ST_TINY_DIAG);
        jacobi_update(Rv, acc, b[r], d, dtc, tiny);
        R[r] = Rv;
        sout[r] = sigma[r] ? Rv : T(0);
      }
    }
  }
}

// Zeroes the words of the streamed sweeps' grid barrier.
__global__ void grid_bar_clear_kernel(int* __restrict__ bar, size_t words) {
  for (size_t i = threadIdx.x; i < words; i += blockDim.x) bar[i] = 0;
}

// ---------------------------------------------------------------------------
// Support form for large N (G too large for the resident kernel): the
// support's block G_SS is compacted once, the sweeps run over the support
// rows only (one launch each), and one pass sets every R with the affine form
// above.  Used while |S| <= sup_kmax<T>(n); otherwise the streamed sweeps run
// (they check the flag and return at once when this form has run).
// ---------------------------------------------------------------------------
template <typename T>
__host__ __device__ inline int sup_kmax(int n) {
  const int cap = sizeof(T) == 4 ? 8192 : 4096;
  return n < cap ? n : cap;
}

template <typename T>
struct SupWs {
  int* ctl;      // [0] 1 when the support form runs, [1] |S|
  int* S;        // support list (n)
  int* pos;      // position in the list or -1 (n)
  T* sR;         // R on the support, two parities (2 kmax)
  T* V;          // sum_k (1 - dtc)^(K-1-k) R_S(k) (kmax)
  T* Gss;        // |S| x |S| (kmax^2)
};

template <typename T>
__host__ __device__ inline size_t sup_ws_bytes(int n) {
  const size_t k = size_t(sup_kmax<T>(n));
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  return al(2 * sizeof(int)) + 2 * al(size_t(n) * sizeof(int)) + al(2 * k * sizeof(T)) + al(k * sizeof(T)) +
         al(k * k * sizeof(T));
}

template <typename T>
__host__ __device__ inline SupWs<T> sup_ws(void* p, int n) {
  const size_t k = size_t(sup_kmax<T>(n));
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  char* c = static_cast<char*>(p);
  SupWs<T> w;
  w.ctl = reinterpret_cast<int*>(c);
  c += al(2 * sizeof(int));
  w.S = reinterpret_cast<int*>(c);
  c += al(size_t(n) * sizeof(int));
  w.pos = reinterpret_cast<int*>(c);
  c += al(size_t(n) * sizeof(int));
  w.sR = reinterpret_cast<T*>(c);
  c += al(2 * k * sizeof(T));
  w.V = reinterpret_cast<T*>(c);
  c += al(k * sizeof(T));
  w.Gss = reinterpret_cast<T*>(c);
  return w;
}

// One workgroup: support list, its inverse, R on the support, V = 0.
template <typename T>
__global__ void __launch_bounds__(1024)
sup_prep_kernel(int n, const T* __restrict__ G, int64_t ldg, const uint8_t* __restrict__ sigma,
                T* __restrict__ R, int* __restrict__ status, SupWs<T> w) {
  __shared__ int scan_sh[1024 / kWave + 1];
  const int t = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int lo = min(n, t * chunk), hi = min(n, lo + chunk);
  int c = 0;
  for (int i = lo; i < hi; ++i) c += sigma[i] ? 1 : 0;
  int ks = 0;
  int at = block_exclusive_scan<1024>(c, scan_sh, &ks);
  const bool run = ks <= sup_kmax<T>(n);
  if (t == 0) {
    w.ctl[0] = run ? 1 : 0;
    w.ctl[1] = ks;
  }
  if (!run) return;
  int bits = 0;
  for (int i = lo; i < hi; ++i) {
    const T d = G[size_t(i) * ldg + i];
    const bool tiny = !(d >= T(1e-12));
    if (tiny) bits |= L0CIM_ST_TINY_DIAG;
    const T r = tiny ? T(0) : R[i];
    R[i] = r;
    if (sigma[i]) {
      w.S[at] = i;
      w.pos[i] = at;
      w.sR[at] = r;
      w.V[at] = T(0);
      ++at;
    } else {
      w.pos[i] = -1;
    }
  }
  if (bits) raise_status(status, bits);
}

// G_SS[i][j] = G[S_i][S_j], one wavefront per row, rows strided over the grid.
template <typename T>
__global__ void __launch_bounds__(256)
sup_compact_kernel(const T* __restrict__ G, int64_t ldg, SupWs<T> w) {
  if (!w.ctl[0]) return;
  const int ks = w.ctl[1];
  const int lane = threadIdx.x & (kWave - 1);
  for (int i = blockIdx.x * 4 + threadIdx.x / kWave; i < ks; i += gridDim.x * 4) {
    const T* g = G + size_t(w.S[i]) * ldg;
    T* o = w.Gss + size_t(i) * ks;
    for (int j = lane; j < ks; j += kWave) o[j] = g[w.S[j]];
  }
}

// The K synchronous sweeps over the support rows in one cooperative launch
// without grid barriers: the support's R travel as step-tagged words (as in
// the resident runs), every workgroup gathers all of them into LDS, and
// wavefront gw = 4 blockIdx + wave updates rows i = gw, gw + 4 gridDim, ...
// of the compacted block G_SS, accumulating V from each sweep's input.  (A
// grid barrier between sweeps measured 28 us per sweep, as its device-scope
// release and acquire write back and invalidate L2; one launch per sweep
// 13.9 us.)  Two word slots suffice: a wavefront can only overwrite slot
// it & 1 after gathering every row's sweep-it word, which each owner
// publishes after its own gather of slot it & 1.
// Sleep (units of 64 clocks) before the first poll of a sweep.
constexpr int kFirstPollSleepCdp = 15;

template <typename T>
__global__ void __launch_bounds__(256)
sup_ll_kernel(const T* __restrict__ b, T dtc, int iters, SupWs<T> w, uint64_t* __restrict__ ll,
              int* __restrict__ abort_word, int* __restrict__ status, int64_t limit) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int lds_abort;
  if (!w.ctl[0]) return;   // the same in every workgroup
  constexpr int W = LL<T>::kWords;
  T* sx = reinterpret_cast<T*>(smem);
  const int ks = w.ctl[1];
  const size_t slot = size_t(ks) * W;
  const int lane = threadIdx.x & (kWave - 1);
  const int gw = blockIdx.x * 4 + threadIdx.x / kWave, nw = gridDim.x * 4;
  if (lane == 0)
    for (int i = gw; i < ks; i += nw) LL<T>::put(ll + size_t(i) * W, w.sR[i], 1u);
  // the wavefront's rows of G_SS stay in registers when they fit (at most two
  // rows of at most 64 kRegCols columns); otherwise they are read every sweep
  constexpr int kRegCols = 32;
  const bool in_regs = ks <= kRegCols * kWave && ks <= 2 * nw;
  T greg[2][kRegCols];
  if (in_regs) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int i = gw + r * nw;
#pragma unroll
      for (int u = 0; u < kRegCols; ++u) {
        const int j = lane + u * kWave;
        greg[r][u] = (i < ks && j < ks) ? w.Gss[size_t(i) * ks + j] : T(0);
      }
    }
  }
  auto finish = [&](int i, T acc, int it) {
    acc = wave_sum(acc);
    if (lane == 0) {
      const T d = w.Gss[size_t(i) * ks + i];
      T Rv = sx[i];
      w.V[i] = (T(1) - dtc) * w.V[i] + Rv;
      jacobi_update(Rv, acc, b[w.S[i]], d, dtc, !(d >= T(1e-12)));
      LL<T>::put(ll + size_t((it + 1) & 1) * slot + size_t(i) * W, Rv, uint32_t(it + 2));
      if (it + 1 == iters) w.sR[size_t(iters & 1) * ks + i] = Rv;
    }
  };
  if (threadIdx.x == 0) lds_abort = 0;
  __syncthreads();
  for (int it = 0; it < iters; ++it) {
    const uint64_t* src = ll + size_t(it & 1) * slot;
    const uint32_t flag = uint32_t(it + 1);
    bool ok = true;
    // 2048 words at a time, 8 per thread: issue them all, re-poll the late ones together
    if (it > 0) __builtin_amdgcn_s_sleep(kFirstPollSleepCdp);
    for (int base = 0; base < ks && ok; base += 8 * 256) {
      uint64_t wv[8][W];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = base + threadIdx.x + u * 256;
#pragma unroll
        for (int v = 0; v < W; ++v) wv[u][v] = j < ks ? ll_load(src + size_t(j) * W + v) : (uint64_t(flag) << 32);
      }
      int64_t polls = 0;
      for (;;) {
        bool ready = true;
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int v = 0; v < W; ++v) ready = ready && (uint32_t(wv[u][v] >> 32) == flag);
        if (ready) break;
        if (++polls > limit || ((polls & 1023) == 0 && abort_seen(abort_word))) {
          ok = false;
          break;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int j = base + threadIdx.x + u * 256;
#pragma unroll
          for (int v = 0; v < W; ++v)
            if (uint32_t(wv[u][v] >> 32) != flag) wv[u][v] = ll_load(src + size_t(j) * W + v);
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = base + threadIdx.x + u * 256;
        if (j < ks) sx[j] = ll_decode<T>(wv[u]);
      }
    }
    if (!ok) lds_abort = 1;
    __syncthreads();
    if (lds_abort) {
      if (threadIdx.x == 0) {
        __hip_atomic_store(abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        raise_status(status, L0CIM_ST_TIMEOUT);
      }
      return;
    }
    if (in_regs) {
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int i = gw + r * nw;
        if (i >= ks) break;
        T acc = T(0);
#pragma unroll
        for (int u = 0; u < kRegCols; ++u) {
          const int j = lane + u * kWave;
          if (j < ks && j != i) acc += greg[r][u] * sx[j];
        }
        finish(i, acc, it);
      }
    } else {
      for (int i = gw; i < ks; i += nw) {
        const T* g = w.Gss + size_t(i) * ks;
        // the row's loads issued eight at a time, the products added in column order
        T acc = T(0);
        int j = lane;
        for (; j + 7 * kWave < ks; j += 8 * kWave) {
          T gv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) gv[u] = g[j + u * kWave];
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (j + u * kWave != i) acc += gv[u] * sx[j + u * kWave];
        }
        for (; j < ks; j += kWave)
          if (j != i) acc += g[j] * sx[j];
        finish(i, acc, it);
      }
    }
    __syncthreads();   // sx is gathered again
  }
}

// Every R after K sweeps: the support's from the last sweep, the others from
// the affine form (one wavefront per row).
template <typename T>
__global__ void __launch_bounds__(256)
sup_final_kernel(int n, const T* __restrict__ G, int64_t ldg, const T* __restrict__ b, T dtc, int iters,
                 T* __restrict__ R, SupWs<T> w) {
  if (!w.ctl[0]) return;
  const int ks = w.ctl[1];
  const int lane = threadIdx.x & (kWave - 1);
  const int r = blockIdx.x * 4 + threadIdx.x / kWave;
  if (r >= n) return;
  const int pr = w.pos[r];
  if (pr >= 0) {
    if (lane == 0) R[r] = w.sR[size_t(iters & 1) * ks + pr];
    return;
  }
  const T* g = G + size_t(r) * ldg;
  T acc = T(0);
  for (int s = lane; s < ks; s += kWave) acc += g[w.S[s]] * w.V[s];
  acc = wave_sum(acc);
  if (lane == 0) {
    const T d = g[r];
    const bool tiny = !(d >= T(1e-12));
    T f = T(1);
    for (int k = 0; k < iters; ++k) f *= (T(1) - dtc);
    R[r] = tiny ? T(0) : f * R[r] + (T(1) - f) * (b[r] / d) - (dtc / d) * acc;
  }
}

// eq. 3 residual: one wavefront per measurement row.
template <typename T>
__global__ void __launch_bounds__(256)
residual_kernel(int m, int n, const T* __restrict__ A, int64_t lda, const T* __restrict__ y,
                const uint8_t* __restrict__ sigma, const T* __restrict__ R, double* __restrict__ part) {
  __shared__ double rs[4];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int k = blockIdx.x * 4 + wv;
  double acc = 0.0;
  if (k < m) {
    for (int j = lane; j < n; j += kWave)
      if (sigma[j]) acc += double(A[size_t(k) * lda + j]) * double(R[j]);
    acc = wave_sum(acc);
  }
  if (lane == 0) {
    double res = (k < m) ? double(y[k]) - acc : 0.0;
    rs[wv] = res * res;
  }
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((rs[0] + rs[1]) + rs[2]) + rs[3];
}

__global__ void finalize_kernel(int n, int nparts, const double* __restrict__ part,
                                const uint8_t* __restrict__ sigma, double lam, l0cim_stats* stats,
                                int64_t spin_steps, int n_outer) {
  __shared__ int cnt[256];
  int c = 0;
  for (int i = threadIdx.x; i < n; i += 256) c += sigma[i] ? 1 : 0;
  cnt[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int t = 0; t < 256; ++t) s += cnt[t];
    double r2 = 0.0;
    for (int p = 0; p < nparts; ++p) r2 += part[p];
    stats->support_size = s;
    stats->E = 0.5 * r2 + lam * double(s);
    stats->spin_steps = spin_steps;
    stats->n_outer_done = n_outer;
  }
}

}  // namespace

size_t jacobi_ws_bytes(l0cim_dtype dt, int n) {
  size_t words = (dt == L0CIM_F64) ? 2 : 1;
  return align_up(size_t(2) * n * words * sizeof(uint64_t)) + kAlign + 2 * align_up(size_t(n) * dtype_size(dt)) +
         support_ctl_bytes() + align_up(grid_barrier_bytes()) +
         (dt == L0CIM_F64 ? sup_ws_bytes<double>(n) : sup_ws_bytes<float>(n));
}

namespace {
template <typename T>
l0cim_status jacobi_typed(int n, const T* G, int64_t ldg, const T* b, const uint8_t* sigma, double dtc,
                          int iters, T* R, int* status, void* ws, hipStream_t s, int64_t limit) {
  DeviceInfo dev;
  l0cim_status st = device_info(&dev);
  if (st != L0CIM_OK) return st;
  char* p = static_cast<char*>(ws);
  uint64_t* ll = reinterpret_cast<uint64_t*>(p);
  p += align_up(size_t(2) * n * LL<T>::kWords * sizeof(uint64_t));
  int* abort_word = reinterpret_cast<int*>(p);
  p += kAlign;
  T* s0 = reinterpret_cast<T*>(p);
  p += align_up(size_t(n) * sizeof(T));
  T* s1 = reinterpret_cast<T*>(p);
  p += align_up(size_t(n) * sizeof(T));
  void* ctl = p;
  p += align_up(support_ctl_bytes());
  int* bar = reinterpret_cast<int*>(p);   // grid barrier of the streamed sweeps
  const size_t bar_words = align_up(grid_barrier_bytes()) / sizeof(int);
  p += align_up(grid_barrier_bytes());
  const SupWs<T> sw = sup_ws<T>(p, n);
  if (iters <= 0) return L0CIM_OK;

  int rpw = 0, grid = 0;
  size_t lds = 0;
  if (n <= 256 && jacobi_lds<T>(n, n) <= size_t(dev.max_lds)) {
    rpw = n;
    grid = 1;
    lds = jacobi_lds<T>(n, n);
  } else {
    int r = (n + dev.cu_count - 1) / dev.cu_count;
    if (jacobi_lds<T>(n, r) <= size_t(dev.max_lds)) {
      rpw = r;
      grid = (n + r - 1) / r;
      lds = jacobi_lds<T>(n, r);
    }
  }
  if (rpw) {
    auto kern = jacobi_resident_kernel<T>;
    const int* done = nullptr;
    if constexpr (sizeof(T) == 4) {
      // support form first; the resident kernel returns at once when it succeeded
      hipLaunchKernelGGL(jacobi_support_kernel, dim3(1), dim3(1024), 0, s, n, G, ldg, b, sigma, float(dtc), iters,
                         R, status, ctl);
      L0_LAUNCHED("jacobi_support_kernel");
      hipLaunchKernelGGL(jacobi_offsupport_kernel, dim3((n + 3) / 4), dim3(256), 0, s, n, G, ldg, b, sigma,
                         float(dtc), iters, R, status, ctl);
      L0_LAUNCHED("jacobi_offsupport_kernel");
      done = static_cast<const int*>(ctl);
    }
    if (grid > 1) {
      hipLaunchKernelGGL(ll_clear_kernel, dim3(64), dim3(256), 0, s, ll, size_t(2) * n * LL<T>::kWords,
                         abort_word);
      L0_LAUNCHED("clear exchange buffer");
    }
    L0_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    const int block = (rpw >= 8) ? 512 : 256;
    T dtcT = T(dtc);
    int nn = n, itn = iters, rp = rpw;
    int64_t lim = limit;
    void* kargs[] = {&nn, &G, &ldg, &b, &sigma, &dtcT, &itn, &R, &ll, &abort_word, &status, &lim, &rp, &done};
    if (grid > 1) {
      L0_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(block),
                                        kargs, unsigned(lds), s));
    } else {
      hipLaunchKernelGGL(kern, dim3(1), dim3(block), lds, s, nn, G, ldg, b, sigma, dtcT, itn, R, ll,
                         abort_word, status, lim, rp, done);
      L0_LAUNCHED("jacobi_resident_kernel");
    }
    return L0CIM_OK;
  }
  // support form first; the streamed sweeps return at once when it ran
  hipLaunchKernelGGL(grid_bar_clear_kernel, dim3(1), dim3(256), 0, s, bar, bar_words);
  L0_LAUNCHED("grid_bar_clear_kernel");
  T dtcT = T(dtc);
  int64_t lim = limit;
  int itn = iters;
  {
    const int kmax = sup_kmax<T>(n);
    int grid = (kmax + 3) / 4;
    if (grid > 4 * dev.cu_count) grid = 4 * dev.cu_count;
    hipLaunchKernelGGL(sup_prep_kernel<T>, dim3(1), dim3(1024), 0, s, n, G, ldg, sigma, R, status, sw);
    L0_LAUNCHED("sup_prep_kernel");
    hipLaunchKernelGGL(sup_compact_kernel<T>, dim3(grid), dim3(256), 0, s, G, ldg, sw);
    L0_LAUNCHED("sup_compact_kernel");
    hipLaunchKernelGGL(ll_clear_kernel, dim3(64), dim3(256), 0, s, ll, size_t(2) * kmax * LL<T>::kWords,
                       abort_word);
    L0_LAUNCHED("clear exchange buffer");
    const unsigned lds = unsigned(size_t(kmax) * sizeof(T));
    L0_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(sup_ll_kernel<T>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    int per_cu = 0;
    L0_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(sup_ll_kernel<T>), 256, lds));
    const int cgrid = std::min(dev.cu_count * std::max(per_cu, 1), dev.cu_count);
    SupWs<T> swa = sw;
    void* args[] = {&b, &dtcT, &itn, &swa, &ll, &abort_word, &status, &lim};
    L0_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(sup_ll_kernel<T>), dim3(cgrid), dim3(256),
                                      args, lds, s));
    hipLaunchKernelGGL(sup_final_kernel<T>, dim3((n + 3) / 4), dim3(256), 0, s, n, G, ldg, b, T(dtc), iters, R, sw);
    L0_LAUNCHED("sup_final_kernel");
  }
  {
    const int* done = sw.ctl;
    int per_cu = 0;
    L0_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(jacobi_streamed_kernel<T>), 256, 0));
    int cgrid = std::min({(n + 3) / 4, dev.cu_count * std::max(per_cu, 1), 4 * dev.cu_count, kGridMaxWg});
    int nn = n;
    int* b1 = bar;
    void* args[] = {&nn, &G, &ldg, &b, &sigma, &dtcT, &itn, &s0, &s1, &R, &status, &done, &b1, &lim};
    L0_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(jacobi_streamed_kernel<T>), dim3(cgrid),
                                      dim3(256), args, 0, s));
  }
  return L0CIM_OK;
}
}  // namespace

l0cim_status launch_jacobi(l0cim_dtype dt, int n, const void* G, int64_t ldg, const void* b,
                           const uint8_t* sigma, double dtc, int iters, void* R, int* status,
                           void* ws, size_t ws_bytes, hipStream_t s, int64_t spin_limit) {
  (void)ws_bytes;
  if (dt == L0CIM_F32)
    return jacobi_typed<float>(n, (const float*)G, ldg, (const float*)b, sigma, dtc, iters, (float*)R,
                               status, ws, s, spin_limit);
  if (dt == L0CIM_F64)
    return jacobi_typed<double>(n, (const double*)G, ldg, (const double*)b, sigma, dtc, iters,
                                (double*)R, status, ws, s, spin_limit);
  return set_error(L0CIM_ERR_UNSUPPORTED, "update_r: dtype %d", int(dt));
}

size_t objective_ws_bytes(int m) { return align_up(size_t((m + 3) / 4) * sizeof(double)); }

l0cim_status launch_objective(l0cim_dtype dt, int m, int n, const void* A, int64_t lda, const void* y,
                              const uint8_t* sigma, const void* R, double lam, l0cim_stats* stats,
                              int64_t spin_steps, int n_outer, void* ws, size_t ws_bytes,
                              hipStream_t s) {
  (void)ws_bytes;
  double* part = static_cast<double*>(ws);
  const int nb = (m + 3) / 4;
  if (dt == L0CIM_F32)
    hipLaunchKernelGGL(residual_kernel<float>, dim3(nb), dim3(256), 0, s, m, n, (const float*)A, lda,
                       (const float*)y, sigma, (const float*)R, part);
  else if (dt == L0CIM_F64)
    hipLaunchKernelGGL(residual_kernel<double>, dim3(nb), dim3(256), 0, s, m, n, (const double*)A, lda,
                       (const double*)y, sigma, (const double*)R, part);
  else
    return set_error(L0CIM_ERR_UNSUPPORTED, "objective: dtype %d", int(dt));
  L0_LAUNCHED("residual_kernel");
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, n, nb, part, sigma, lam, stats,
                     spin_steps, n_outer);
  L0_LAUNCHED("finalize_kernel");
  return L0CIM_OK;
}

}  // namespace l0
