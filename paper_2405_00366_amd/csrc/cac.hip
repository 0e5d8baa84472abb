// CAC-CIM (Positive-P) support estimation, eq. 5-11: the stochastic CIM the
// paper compares the mean-field model against, on the same couplings
// contraction.  Per spin and replica: the normalised mean amplitude mu
// (eq. 5), the fluctuation variances n and m (eq. 6, 7) and the amplitude
// control e (eq. 9); the local field (eq. 11) is built from the measured
// amplitudes mu~ = mu + sqrt(g^2/(4j)) W (eq. 10) of the other spins:
//
//   R_r h_r = 1/2 (J (mu~ + sqrt(tau)))_r + sqrt(tau) z_r,  J = -G o R R^T, z = R o b.
//
// Forward Euler-Maruyama with the time increment dt: one standard normal xi
// per spin, replica and step, the white noise of the step taken as its step
// average xi / sqrt(dt) (so the eq. 5 noise increment is
// sqrt(j g^2)(m + n) xi sqrt(dt)); every right-hand side at step k.
//
// The normals are counter-based: SplitMix64 (Steele, Lea and Flood, 2014)
// keyed by mix64(seed ^ kNoiseTag), outputs 2 ctr + 1 and 2 ctr + 2 with
// ctr = (alt << 52) | (k << 32) | (q << 24) | r, as two 53-bit uniforms, and
// Box-Muller sqrt(-2 ln(1 - u1)) cos(2 pi u2) in FP64.
//
// One launch per Euler step (the measured amplitudes of step k must be
// complete before any field of step k is formed): each wavefront owns one
// row of J and contracts it with the measured amplitudes of every replica,
// then updates that spin.  The measured amplitudes of step k + 1 are drawn at
// the end of step k into the other of two buffers.
#include "kernels.h"

namespace l0 {
namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kNoiseTag = 0x6E6F6973655F7764ull;
constexpr int kRows = 4;   // rows (wavefronts) per 256-thread workgroup
constexpr int kQB = 8;     // replicas per pass over a row of J
constexpr int kLdsRows = 8;   // rows (wavefronts) per workgroup of the LDS form
constexpr int kJU = 16;       // loads of a row of J in flight per lane
// The LDS form holds a whole row of J in registers and the kQB replicas'
// amplitudes in LDS: n up to 2048 (FP32) / 1024 (FP64), 64 KB of LDS.
template <typename T>
constexpr int kCacMaxN() { return sizeof(T) == 4 ? 2048 : 1024; }

__device__ inline uint64_t smix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ inline double step_normal(uint64_t s, int alt, int k, int q, int r) {
  const uint64_t ctr = (uint64_t(alt) << 52) | (uint64_t(k) << 32) | (uint64_t(q) << 24) | uint64_t(r);
  const uint64_t w1 = smix(s + (2 * ctr + 1) * kGolden);
  const uint64_t w2 = smix(s + (2 * ctr + 2) * kGolden);
  const double u1 = double(w1 >> 11) * 0x1.0p-53;
  const double u2 = double(w2 >> 11) * 0x1.0p-53;
  return sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586 * u2);
}

struct CacArgs {
  int n, P, n_steps, trace_steps, alt;
  uint64_t noise_seed;
  double dt, p_thr, d, t_c, t_w, K, j, beta, tau, g2, eta;
};

__device__ inline double cac_pump(const CacArgs& a, int k) {
  const double t = double(k) * a.dt;
  return (a.p_thr - a.d) + 2.0 * a.d / (1.0 + exp(-(t - a.t_c) / a.t_w));
}

// mu = n = m = 0, e = 1 and the measured amplitudes of step 0.
template <typename T>
__global__ void cac_init_kernel(CacArgs a, T* __restrict__ mu, T* __restrict__ nv, T* __restrict__ mv,
                                T* __restrict__ e, T* __restrict__ mum) {
  const size_t total = size_t(a.n) * a.P;
  const double s = sqrt(a.g2 / (4.0 * a.j)) / sqrt(a.dt);
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < total; i += size_t(gridDim.x) * blockDim.x) {
    const int q = int(i / a.n), r = int(i - size_t(q) * a.n);
    mu[i] = T(0);
    nv[i] = T(0);
    mv[i] = T(0);
    e[i] = T(1);
    mum[i] = T(s * step_normal(a.noise_seed, a.alt, 0, q, r));
  }
}

// Constants of one Euler-Maruyama step k (eq. 5-11).
template <typename T>
struct CacStep {
  T st, p, dt, jj, g2, KK, beta, tau, theta, noise_mu;
  double s_meas;
  __device__ CacStep(const CacArgs& a, int k) {
    st = T(sqrt(a.tau));
    p = T(cac_pump(a, k));
    dt = T(a.dt);
    jj = T(a.j);
    g2 = T(a.g2);
    KK = T(a.K);
    beta = T(a.beta);
    tau = T(a.tau);
    theta = T(sqrt(a.tau) * a.eta * a.eta * 0.25);
    noise_mu = T(sqrt(a.j * a.g2) * sqrt(a.dt));
    s_meas = sqrt(a.g2 / (4.0 * a.j)) / sqrt(a.dt);
  }
};

// One Euler-Maruyama step of (mu, n, m, e) of one spin and replica from its
// field sum acc = sum_c J_rc (m_c + sqrt(tau)), its Zeeman term zr, its
// measured amplitude m_t and the normal xi of the step (eq. 5-11).
template <typename T>
__device__ inline void cac_advance(const CacStep<T>& c, T acc, T zr, T m_t, T xi, T& u, T& nn, T& mm, T& ee) {
  const T phi = T(0.5) * acc + c.st * zr;
  const T inj = c.jj * ee * (phi - c.theta);
  const T u2 = u * u;
  const T p = c.p, jj = c.jj, g2 = c.g2;
  const T du = -(T(1) - p + jj) * u - u * (u2 + T(2) * g2 * nn + g2 * mm) + c.KK * inj;
  const T dn = -T(2) * (T(1) + jj) * nn + T(2) * p * mm - T(2) * u2 * (T(2) * nn + mm) - jj * (mm + nn) * (mm + nn);
  const T dm = -T(2) * (T(1) + jj) * mm + T(2) * p * nn - T(2) * u2 * (T(2) * mm + nn) + p - (u2 + g2 * mm) -
               jj * (mm + nn) * (mm + nn);
  const T de = -c.beta * (m_t * m_t - c.tau) * ee;
  const T un = u + c.dt * du + c.noise_mu * (mm + nn) * xi;
  const T nn1 = nn + c.dt * dn, mm1 = mm + c.dt * dm, ee1 = ee + c.dt * de;
  u = un;
  nn = nn1;
  mm = mm1;
  ee = ee1;
}

template <typename T>
__device__ inline void cac_trace(const CacArgs& a, int k, size_t g, T u, T nn, T mm, T ee, T* __restrict__ trace) {
  if (k < a.trace_steps) {
    const size_t base = (size_t(k) * 4) * a.P * a.n + g;
    trace[base] = u;
    trace[base + size_t(a.P) * a.n] = nn;
    trace[base + size_t(2) * a.P * a.n] = mm;
    trace[base + size_t(3) * a.P * a.n] = ee;
  }
}

// The update of spin r of replica q, state read from and written to memory.
template <typename T>
__device__ inline void cac_update(const CacArgs& a, const CacStep<T>& c, int k, int q, int r, T acc,
                                  const T* __restrict__ z, const T* __restrict__ mum_in, T* __restrict__ mum_out,
                                  T* __restrict__ mu, T* __restrict__ nv, T* __restrict__ mv, T* __restrict__ e,
                                  T* __restrict__ trace) {
  const size_t g = size_t(q) * a.n + r;
  const T xi = T(step_normal(a.noise_seed, a.alt, k, q, r));
  T u = mu[g], nn = nv[g], mm = mv[g], ee = e[g];
  cac_advance(c, acc, z[r], mum_in[g], xi, u, nn, mm, ee);
  mu[g] = u;
  nv[g] = nn;
  mv[g] = mm;
  e[g] = ee;
  mum_out[g] = u + T(c.s_meas * step_normal(a.noise_seed, a.alt, k + 1, q, r));
  cac_trace(a, k, g, u, nn, mm, ee, trace);
}

// Lane 0's total of each of the kQB sums to lane qq (every lane's butterfly
// total may differ in its last bits; lane 0's is the one used).
template <typename T>
__device__ inline T lane_total(T (&acc)[kQB], int lane) {
  T mine = T(0);
#pragma unroll
  for (int qq = 0; qq < kQB; ++qq) {
    const T tot = __shfl(wave_sum(acc[qq]), 0, kWave);
    if (lane == qq) mine = tot;
  }
  return mine;
}

// One Euler-Maruyama step of every spin and replica, a wavefront per row of J:
// kQB replicas per pass, the row of J read once for all of them, lane qq
// then runs the update of replica q0 + qq.  The measured amplitudes are read
// from memory (any n; the LDS form below covers n up to a limit).
template <typename T>
__global__ void __launch_bounds__(256)
cac_step_kernel(const T* __restrict__ J, int64_t ldj, const T* __restrict__ z, CacArgs a, int k,
                const T* __restrict__ mum_in, T* __restrict__ mum_out, T* __restrict__ mu, T* __restrict__ nv,
                T* __restrict__ mv, T* __restrict__ e, T* __restrict__ trace) {
  const int n = a.n, P = a.P;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int r = blockIdx.x * kRows + wv;
  if (r >= n) return;
  const CacStep<T> c(a, k);
  const T* jr = J + size_t(r) * ldj;
  for (int q0 = 0; q0 < P; q0 += kQB) {
    const int nq = P - q0 < kQB ? P - q0 : kQB;
    T acc[kQB];
#pragma unroll
    for (int qq = 0; qq < kQB; ++qq) acc[qq] = T(0);
    for (int c0 = lane; c0 < n; c0 += kWave * kJU) {
      T jv[kJU];   // kJU loads of the row in flight, then the sums in the same column order
#pragma unroll
      for (int u = 0; u < kJU; ++u) jv[u] = c0 + u * kWave < n ? jr[c0 + u * kWave] : T(0);
#pragma unroll
      for (int u = 0; u < kJU; ++u) {
        const int cc = c0 + u * kWave;
        if (cc < n) {
#pragma unroll
          for (int qq = 0; qq < kQB; ++qq)
            if (qq < nq) acc[qq] += jv[u] * (mum_in[size_t(q0 + qq) * n + cc] + c.st);
        }
      }
    }
    const T mine = lane_total(acc, lane);
    if (lane < nq) cac_update(a, c, k, q0 + lane, r, mine, z, mum_in, mum_out, mu, nv, mv, e, trace);
  }
}

// The same step with the measured amplitudes of kQB replicas (plus sqrt(tau),
// the same rounding as above) staged in LDS once per workgroup of kLdsRows
// rows, so that every row reads them from LDS instead of the caches.
template <typename T>
__global__ void __launch_bounds__(kLdsRows * kWave)
cac_step_lds_kernel(const T* __restrict__ J, int64_t ldj, const T* __restrict__ z, CacArgs a, int k,
                    const T* __restrict__ mum_in, T* __restrict__ mum_out, T* __restrict__ mu, T* __restrict__ nv,
                    T* __restrict__ mv, T* __restrict__ e, T* __restrict__ trace) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* xs = reinterpret_cast<T*>(smem);
  const int n = a.n, P = a.P;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int r = blockIdx.x * kLdsRows + wv;
  const CacStep<T> c(a, k);
  // the whole row of J in registers (columns lane + 64 u), requested before
  // the staging so that its latency is spent under it; it serves every pass
  constexpr int kCols = kCacMaxN<T>() / kWave;
  const T* jr = J + size_t(r < n ? r : 0) * ldj;
  T jv[kCols];
#pragma unroll
  for (int u = 0; u < kCols; ++u) jv[u] = lane + u * kWave < n ? jr[lane + u * kWave] : T(0);
  for (int q0 = 0; q0 < P; q0 += kQB) {
    const int nq = P - q0 < kQB ? P - q0 : kQB;
    __syncthreads();   // the previous block's reads of xs are done
    const int tot = nq * n;
    constexpr int kThreads = kLdsRows * kWave;
    for (int i0 = tid; i0 < tot; i0 += kThreads * kJU) {   // kJU loads in flight per lane
      T v[kJU];
#pragma unroll
      for (int u = 0; u < kJU; ++u) v[u] = i0 + u * kThreads < tot ? mum_in[size_t(q0) * n + i0 + u * kThreads] : T(0);
#pragma unroll
      for (int u = 0; u < kJU; ++u)
        if (i0 + u * kThreads < tot) xs[i0 + u * kThreads] = v[u] + c.st;
    }
    __syncthreads();
    if (r < n) {
      T acc[kQB];
#pragma unroll
      for (int qq = 0; qq < kQB; ++qq) acc[qq] = T(0);
      if (nq == kQB) {
        // a full block, one replica at a time: the LDS reads of its columns
        // issue together (the same column order per lane as below); a lane
        // past the row's end adds J = 0 times a valid entry (its index
        // clamped), which leaves the sum unchanged
        const int uend = (n + kWave - 1) / kWave;
#pragma unroll
        for (int qq = 0; qq < kQB; ++qq) {
          const T* xq = xs + qq * n;
#pragma unroll
          for (int u = 0; u < kCols; ++u) {
            if (u >= uend) break;
            const int cc = lane + u * kWave < n ? lane + u * kWave : n - 1;
            acc[qq] += jv[u] * xq[cc];
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < kCols; ++u) {
          const int cc = lane + u * kWave;
          if (cc < n) {
#pragma unroll
            for (int qq = 0; qq < kQB; ++qq)
              if (qq < nq) acc[qq] += jv[u] * xs[qq * n + cc];
          }
        }
      }
      const T mine = lane_total(acc, lane);
      if (lane < nq) cac_update(a, c, k, q0 + lane, r, mine, z, mum_in, mum_out, mu, nv, mv, e, trace);
    }
  }
}

// The whole run in one cooperative launch (every workgroup resident), for
// P <= kQB replicas and n up to kCacMaxN: each workgroup keeps its kLdsRows
// rows of J in registers and lane q of wavefront w the state (mu, n, m, e)
// of row w, replica q; the measured amplitudes of step k travel between
// workgroups as step-tagged words (flag k + 1, two slots by step parity).
// Per step every workgroup gathers all P n of them into LDS (plus
// sqrt(tau)), forms its rows' sums exactly as cac_step_lds_kernel does,
// advances its owned states and publishes the measured amplitudes of step
// k + 1.  A slot is rewritten only after every workgroup has gathered the
// step it held (a workgroup cannot finish step k + 1 before every other has
// published it).  Every wait is bounded; a timeout raises the abort word
// and every workgroup leaves the loop.
template <typename T>
__global__ void __launch_bounds__(kLdsRows * kWave)
cac_resident_kernel(const T* __restrict__ J, int64_t ldj, const T* __restrict__ z, CacArgs a,
                    const T* __restrict__ mum0, T* __restrict__ mu, T* __restrict__ nv, T* __restrict__ mv,
                    T* __restrict__ e, T* __restrict__ trace, uint64_t* __restrict__ ll, int* __restrict__ abort_word,
                    int* __restrict__ status) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* xs = reinterpret_cast<T*>(smem);
  __shared__ int lds_abort;
  constexpr int W = LL<T>::kWords;
  constexpr int kThreads = kLdsRows * kWave;
  constexpr int kCols = kCacMaxN<T>() / kWave;
  const int n = a.n, P = a.P;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int r = blockIdx.x * kLdsRows + wv;
  const bool valid = r < n;
  const size_t slot = size_t(P) * n * W;
  const T* jr = J + size_t(valid ? r : 0) * ldj;
  T jv[kCols];
#pragma unroll
  for (int u = 0; u < kCols; ++u) jv[u] = lane + u * kWave < n ? jr[lane + u * kWave] : T(0);
  const bool own = valid && lane < P;
  const size_t g = own ? size_t(lane) * n + r : 0;
  T su = T(0), sn = T(0), sm = T(0), se = T(0), mt = T(0), zr = T(0);
  if (own) {
    su = mu[g];
    sn = nv[g];
    sm = mv[g];
    se = e[g];
    mt = mum0[g];
    zr = z[r];
    LL<T>::put(ll + g * W, mt, 1u);
  }
  if (tid == 0) lds_abort = 0;
  __syncthreads();
  bool aborted = false;
  const int tot = P * n;
  for (int k = 0; k < a.n_steps; ++k) {
    const CacStep<T> c(a, k);
    const uint64_t* src = ll + size_t(k & 1) * slot;
    const uint32_t flag = uint32_t(k + 1);
    bool ok = true;
    for (int i0 = tid; i0 < tot && ok; i0 += kThreads * kJU) {   // kJU words in flight per lane
      uint64_t w[kJU][W];
#pragma unroll
      for (int u = 0; u < kJU; ++u) {
        const int idx = i0 + u * kThreads;
#pragma unroll
        for (int v = 0; v < W; ++v) w[u][v] = idx < tot ? ll_load(src + size_t(idx) * W + v) : (uint64_t(flag) << 32);
      }
#pragma unroll
      for (int u = 0; u < kJU; ++u) {
        const int idx = i0 + u * kThreads;
        if (idx < tot && ok) {
#pragma unroll
          for (int v = 0; v < W; ++v)
            if (ok) ok = ll_wait(src + size_t(idx) * W + v, flag, w[u][v], kDefaultSpinLimit, abort_word);
          if (ok) xs[idx] = ll_decode<T>(w[u]) + c.st;
        }
      }
    }
    if (!ok) {
      lds_abort = 1;
      __hip_atomic_store(abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (lds_abort) {
      aborted = true;
      break;
    }
    if (valid) {
      T acc[kQB];
#pragma unroll
      for (int qq = 0; qq < kQB; ++qq) acc[qq] = T(0);
      if (P == kQB) {
        const int uend = (n + kWave - 1) / kWave;
#pragma unroll
        for (int qq = 0; qq < kQB; ++qq) {
          const T* xq = xs + qq * n;
#pragma unroll
          for (int u = 0; u < kCols; ++u) {
            if (u >= uend) break;
            const int cc = lane + u * kWave < n ? lane + u * kWave : n - 1;
            acc[qq] += jv[u] * xq[cc];
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < kCols; ++u) {
          const int cc = lane + u * kWave;
          if (cc < n) {
#pragma unroll
            for (int qq = 0; qq < kQB; ++qq)
              if (qq < P) acc[qq] += jv[u] * xs[qq * n + cc];
          }
        }
      }
      const T mine = lane_total(acc, lane);
      if (own) {
        const T xi = T(step_normal(a.noise_seed, a.alt, k, lane, r));
        cac_advance(c, mine, zr, mt, xi, su, sn, sm, se);
        mt = su + T(c.s_meas * step_normal(a.noise_seed, a.alt, k + 1, lane, r));
        LL<T>::put(ll + size_t((k + 1) & 1) * slot + g * W, mt, uint32_t(k + 2));
        cac_trace(a, k, g, su, sn, sm, se, trace);
      }
    }
    __syncthreads();   // every read of xs is done before the next gather
  }
  if (own) {
    mu[g] = su;
    nv[g] = sn;
    mv[g] = sm;
    e[g] = se;
  }
  if (aborted && tid == 0) raise_status(status, L0CIM_ST_TIMEOUT);
}

// sigma = H(mu) and the per-row terms of the eq. 4 energy
// sigma_r (-1/2 (J sigma)_r - z_r + lambda) of every replica.
template <typename T>
__global__ void __launch_bounds__(256)
cac_sigma_energy_kernel(const T* __restrict__ J, int64_t ldj, const T* __restrict__ z, int n, int P, double lam,
                        const T* __restrict__ mu, const T* __restrict__ e, uint8_t* __restrict__ sigma,
                        double* __restrict__ hrow, int* __restrict__ status) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int r = blockIdx.x * kRows + wv;
  if (r >= n) return;
  const T* jr = J + size_t(r) * ldj;
  int bits = 0;
  for (int q = 0; q < P; ++q) {
    const T* uq = mu + size_t(q) * n;
    double acc = 0.0;
    for (int c = lane; c < n; c += kWave) acc += uq[c] > T(0) ? double(jr[c]) : 0.0;
    acc = wave_sum(acc);
    if (lane == 0) {
      const size_t g = size_t(q) * n + r;
      const bool on = uq[r] > T(0);
      sigma[g] = on ? 1 : 0;
      hrow[g] = on ? (-0.5 * acc - double(z[r]) + lam) : 0.0;
      if (!(isfinite(double(uq[r])) && isfinite(double(e[g])))) bits |= L0CIM_ST_NONFINITE;
      else if (fabs(double(uq[r])) > 1e3) bits |= L0CIM_ST_BLOWUP;
    }
  }
  if (lane == 0 && bits) raise_status(status, bits);
}

// H[q] = sum_r hrow[q][r] in a fixed order.
__global__ void cac_energy_reduce_kernel(int n, const double* __restrict__ hrow, double* __restrict__ H) {
  __shared__ double part[256];
  const int q = blockIdx.x, t = threadIdx.x;
  double h = 0.0;
  for (int r = t; r < n; r += 256) h += hrow[size_t(q) * n + r];
  part[t] = h;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) part[t] += part[t + s];
    __syncthreads();
  }
  if (t == 0) H[q] = part[0];
}

uint64_t host_mix64(uint64_t zz) {
  zz = (zz ^ (zz >> 30)) * 0xBF58476D1CE4E5B9ull;
  zz = (zz ^ (zz >> 27)) * 0x94D049BB133111EBull;
  return zz ^ (zz >> 31);
}

struct CacWs {
  void *mum0, *mum1;
  double* hrow;
  uint64_t* ll;     // exchange words of the resident form: 2 slots x P n values
  int* abort_word;
};

size_t cac_ll_words(l0cim_dtype dt, int n, int P) { return 2 * size_t(n) * P * (dt == L0CIM_F64 ? 2 : 1); }

CacWs cac_ws(void* ws, l0cim_dtype dt, int n, int P) {
  char* b = static_cast<char*>(ws);
  const size_t v = align_up(size_t(n) * P * dtype_size(dt));
  const size_t h = align_up(size_t(n) * P * sizeof(double));
  const size_t l = align_up(cac_ll_words(dt, n, P) * sizeof(uint64_t));
  CacWs w;
  w.mum0 = b;
  w.mum1 = b + v;
  w.hrow = reinterpret_cast<double*>(b + 2 * v);
  w.ll = reinterpret_cast<uint64_t*>(b + 2 * v + h);
  w.abort_word = reinterpret_cast<int*>(b + 2 * v + h + l);
  return w;
}

template <typename T>
l0cim_status cac_run_typed(int n, int P, const T* J, int64_t ldj, const T* z, const CacArgs& a, T* mu, T* nv, T* mv,
                           T* e, uint8_t* sigma, double* H, T* trace, int* status, void* ws, l0cim_dtype dt,
                           hipStream_t s) {
  const CacWs w = cac_ws(ws, dt, n, P);
  const size_t total = size_t(n) * P;
  int blocks = int((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(cac_init_kernel<T>, dim3(blocks), dim3(256), 0, s, a, mu, nv, mv, e, static_cast<T*>(w.mum0));
  L0_LAUNCHED("cac_init_kernel");
  const int grid = (n + kRows - 1) / kRows;
  T* bufs[2] = {static_cast<T*>(w.mum0), static_cast<T*>(w.mum1)};
  // the whole run in one launch when every workgroup can be resident
  if (P <= kQB && n <= kCacMaxN<T>()) {
    const size_t rlds = size_t(P) * n * sizeof(T);
    const int rgrid = (n + kLdsRows - 1) / kLdsRows;
    const void* rk = reinterpret_cast<const void*>(cac_resident_kernel<T>);
    L0_HIP(hipFuncSetAttribute(rk, hipFuncAttributeMaxDynamicSharedMemorySize, int(rlds)));
    DeviceInfo dev;
    l0cim_status st = device_info(&dev);
    if (st != L0CIM_OK) return st;
    int per_cu = 0;
    L0_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, rk, kLdsRows * kWave, rlds));
    if (int64_t(per_cu) * dev.cu_count >= rgrid) {
      hipLaunchKernelGGL(ll_clear_kernel, dim3(64), dim3(256), 0, s, w.ll, cac_ll_words(dt, n, P), w.abort_word);
      L0_LAUNCHED("clear exchange buffer");
      const T* m0 = static_cast<const T*>(w.mum0);
      CacArgs aa = a;
      uint64_t* llp = w.ll;
      int* abw = w.abort_word;
      void* kargs[] = {&J, &ldj, &z, &aa, &m0, &mu, &nv, &mv, &e, &trace, &llp, &abw, &status};
      {
        ProfileScope prof(s);
        L0_HIP(hipLaunchCooperativeKernel(rk, dim3(rgrid), dim3(kLdsRows * kWave), kargs, unsigned(rlds), s));
      }
      hipLaunchKernelGGL(cac_sigma_energy_kernel<T>, dim3(grid), dim3(256), 0, s, J, ldj, z, n, P,
                         0.5 * a.eta * a.eta, mu, e, sigma, w.hrow, status);
      L0_LAUNCHED("cac_sigma_energy_kernel");
      if (H) {
        hipLaunchKernelGGL(cac_energy_reduce_kernel, dim3(P), dim3(256), 0, s, n, w.hrow, H);
        L0_LAUNCHED("cac_energy_reduce_kernel");
      }
      return L0CIM_OK;
    }
  }
  const size_t lds = size_t(kQB) * n * sizeof(T);
  const bool staged = n <= kCacMaxN<T>();
  if (staged)
    L0_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(cac_step_lds_kernel<T>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  {
    ProfileScope prof(s);
    for (int k = 0; k < a.n_steps; ++k) {
      if (staged)
        hipLaunchKernelGGL(cac_step_lds_kernel<T>, dim3((n + kLdsRows - 1) / kLdsRows), dim3(kLdsRows * kWave), lds,
                           s, J, ldj, z, a, k, bufs[k & 1], bufs[(k + 1) & 1], mu, nv, mv, e, trace);
      else
        hipLaunchKernelGGL(cac_step_kernel<T>, dim3(grid), dim3(256), 0, s, J, ldj, z, a, k, bufs[k & 1],
                           bufs[(k + 1) & 1], mu, nv, mv, e, trace);
      L0_LAUNCHED("cac_step_kernel");
    }
  }
  hipLaunchKernelGGL(cac_sigma_energy_kernel<T>, dim3(grid), dim3(256), 0, s, J, ldj, z, n, P, 0.5 * a.eta * a.eta,
                     mu, e, sigma, w.hrow, status);
  L0_LAUNCHED("cac_sigma_energy_kernel");
  if (H) {
    hipLaunchKernelGGL(cac_energy_reduce_kernel, dim3(P), dim3(256), 0, s, n, w.hrow, H);
    L0_LAUNCHED("cac_energy_reduce_kernel");
  }
  return L0CIM_OK;
}

CacArgs cac_args(int n, int P, const l0cim_cac_params* p, double eta, uint64_t seed, int alt, int trace_steps) {
  CacArgs a{};
  a.n = n;
  a.P = P;
  a.n_steps = p->n_steps;
  a.trace_steps = trace_steps;
  a.alt = alt;
  a.noise_seed = host_mix64(seed ^ kNoiseTag);
  a.dt = p->dt;
  a.p_thr = p->p_thr;
  a.d = p->d;
  a.t_c = p->t_c;
  a.t_w = p->t_w;
  a.K = p->K;
  a.j = p->j;
  a.beta = p->beta;
  a.tau = p->tau;
  a.g2 = p->g2;
  a.eta = eta;
  return a;
}

l0cim_status check_cac(const l0cim_cac_params* p, const char* who) {
  if (!p) return set_error(L0CIM_ERR_ARG, "%s: CAC params is NULL", who);
  if (p->n_steps < 0 || p->n_steps >= (1 << 20) - 1)
    return set_error(L0CIM_ERR_ARG, "%s: n_steps must be 0 .. 2^20 - 2", who);
  if (!(p->dt > 0.0) || !(p->j > 0.0) || !(p->t_w > 0.0) || !(p->tau > 0.0) || !(p->g2 >= 0.0) || !(p->beta >= 0.0))
    return set_error(L0CIM_ERR_ARG, "%s: dt, j, t_w, tau must be positive and g2, beta >= 0", who);
  return L0CIM_OK;
}

size_t cac_run_ws_bytes(l0cim_dtype dt, int n, int P) {
  return 2 * align_up(size_t(n) * P * dtype_size(dt)) + align_up(size_t(n) * P * sizeof(double)) +
         align_up(cac_ll_words(dt, n, P) * sizeof(uint64_t)) + align_up(sizeof(int));
}

l0cim_status launch_cac_run(l0cim_dtype dt, int n, int P, const void* J, int64_t ldj, const void* z, const CacArgs& a,
                            void* mu, void* nv, void* mv, void* e, uint8_t* sigma, double* H, void* trace,
                            int* status, void* ws, hipStream_t s) {
  if (dt == L0CIM_F32)
    return cac_run_typed<float>(n, P, (const float*)J, ldj, (const float*)z, a, (float*)mu, (float*)nv, (float*)mv,
                                (float*)e, sigma, H, (float*)trace, status, ws, dt, s);
  if (dt == L0CIM_F64)
    return cac_run_typed<double>(n, P, (const double*)J, ldj, (const double*)z, a, (double*)mu, (double*)nv,
                                 (double*)mv, (double*)e, sigma, H, (double*)trace, status, ws, dt, s);
  return set_error(L0CIM_ERR_UNSUPPORTED, "cac_run: dtype %d", int(dt));
}

__global__ void cac_stats_init_kernel(l0cim_stats* st) {
  st->status_bits = 0;
  st->selected_replica = 0;
  st->support_size = 0;
  st->n_outer_done = 0;
  st->H = 0.0;
  st->E = 0.0;
  st->spin_steps = 0;
}

struct CacSolveLayout {
  size_t G, b, J, rs, z, mu, nv, mv, e, sig, H, run, cdp, obj, total;
};

CacSolveLayout cac_solve_layout(l0cim_dtype dt, int m, int n, int P) {
  CacSolveLayout L;
  const size_t ts = dtype_size(dt);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  L.G = take(size_t(n) * n * ts);
  L.b = take(size_t(n) * ts);
  L.J = take(size_t(n) * n * ts);
  L.rs = take(size_t(n) * sizeof(float));
  L.z = take(size_t(n) * ts);
  L.mu = take(size_t(P) * n * ts);
  L.nv = take(size_t(P) * n * ts);
  L.mv = take(size_t(P) * n * ts);
  L.e = take(size_t(P) * n * ts);
  L.sig = take(size_t(P) * n);
  L.H = take(size_t(P) * sizeof(double));
  L.run = take(cac_run_ws_bytes(dt, n, P));
  L.cdp = take(jacobi_ws_bytes(dt, n));
  L.obj = take(objective_ws_bytes(m));
  L.total = o;
  return L;
}

}  // namespace
}  // namespace l0

using namespace l0;

extern "C" {

void l0cim_cac_params_default(l0cim_cac_params* p) {
  if (!p) return;
  p->dt = 0.02;
  p->n_steps = 1000;
  p->p_thr = 1.0;
  p->d = 0.4;
  p->t_c = 4.0;
  p->t_w = 2.0;
  p->K = 1.0;
  p->j = 0.2;
  p->beta = 0.3;
  p->tau = 0.21;
  p->g2 = 1e-7;
}

size_t l0cim_cac_run_workspace_bytes(l0cim_dtype dtype, int32_t n, int32_t P) {
  if (n <= 0 || P <= 0 || (dtype != L0CIM_F32 && dtype != L0CIM_F64)) return 0;
  return cac_run_ws_bytes(dtype, n, P);
}

l0cim_status l0cim_cac_run(l0cim_dtype dtype, int32_t n, int32_t P, const void* J, int64_t ldj, const void* z,
                           double eta, const l0cim_cac_params* prm, uint64_t seed, int32_t alt, void* mu,
                           void* nvar, void* mvar, void* e, uint8_t* sigma, double* H, void* trace,
                           int32_t trace_steps, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  if (dtype != L0CIM_F32 && dtype != L0CIM_F64) return set_error(L0CIM_ERR_UNSUPPORTED, "cac_run: dtype %d", int(dtype));
  l0cim_status st = check_cac(prm, "cac_run");
  if (st != L0CIM_OK) return st;
  if (!J || !z || !mu || !nvar || !mvar || !e || !sigma) return set_error(L0CIM_ERR_ARG, "cac_run: NULL pointer");
  if (n <= 0 || n > (1 << 24) || P <= 0 || P > 256 || ldj < n) return set_error(L0CIM_ERR_SHAPE, "cac_run: bad shape");
  if (alt < 0 || alt >= (1 << 11)) return set_error(L0CIM_ERR_ARG, "cac_run: alternation must be 0 .. 2047");
  if (trace_steps < 0 || (trace_steps > 0 && !trace))
    return set_error(L0CIM_ERR_ARG, "cac_run: trace_steps > 0 needs a trace buffer");
  if (!ws || ws_bytes < cac_run_ws_bytes(dtype, n, P))
    return set_error(L0CIM_ERR_WORKSPACE, "cac_run: workspace needs %zu bytes", cac_run_ws_bytes(dtype, n, P));
  const CacArgs a = cac_args(n, P, prm, eta, seed, alt, trace_steps < prm->n_steps ? trace_steps : prm->n_steps);
  return launch_cac_run(dtype, n, P, J, ldj, z, a, mu, nvar, mvar, e, sigma, H, trace, status, ws,
                        static_cast<hipStream_t>(stream));
}

size_t l0cim_cac_solve_workspace_bytes(l0cim_dtype dtype, int32_t m, int32_t n, int32_t P) {
  if (m <= 0 || n <= 0 || P <= 0 || (dtype != L0CIM_F32 && dtype != L0CIM_F64)) return 0;
  return cac_solve_layout(dtype, m, n, P).total;
}

l0cim_status l0cim_cac_solve(l0cim_dtype dtype, int32_t m, int32_t n, const void* A, int64_t lda, const void* y,
                             const l0cim_cac_params* prm, const l0cim_solve_params* sp, void* R_out,
                             uint8_t* sigma_out, l0cim_stats* stats, void* ws, size_t ws_bytes, void* stream) {
  if (dtype != L0CIM_F32 && dtype != L0CIM_F64) return set_error(L0CIM_ERR_UNSUPPORTED, "cac_solve: dtype %d", int(dtype));
  l0cim_status st = check_cac(prm, "cac_solve");
  if (st != L0CIM_OK) return st;
  if (!sp) return set_error(L0CIM_ERR_ARG, "cac_solve: solve params is NULL");
  if (!A || !y || !R_out || !sigma_out || !stats) return set_error(L0CIM_ERR_ARG, "cac_solve: NULL pointer");
  if (m <= 0 || n <= 0 || n > (1 << 24) || lda < n) return set_error(L0CIM_ERR_SHAPE, "cac_solve: bad shape");
  const int P = sp->replicas;
  if (P <= 0 || P > 256) return set_error(L0CIM_ERR_ARG, "cac_solve: replicas must be 1 .. 256");
  if (sp->n_outer <= 0 || sp->n_outer > (1 << 11) || sp->velo <= 0 || sp->cdp_iters < 0)
    return set_error(L0CIM_ERR_ARG, "cac_solve: n_outer must be 1 .. 2048, velo > 0, cdp_iters >= 0");
  const CacSolveLayout L = cac_solve_layout(dtype, m, n, P);
  if (!ws || ws_bytes < L.total) return set_error(L0CIM_ERR_WORKSPACE, "cac_solve: workspace needs %zu bytes", L.total);
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  void* G = base + L.G;
  void* b = base + L.b;
  void* J = base + L.J;
  void* z = base + L.z;
  uint8_t* sig = reinterpret_cast<uint8_t*>(base + L.sig);
  double* H = reinterpret_cast<double*>(base + L.H);
  int* status = &stats->status_bits;
#define L0_TRY(x)                  \
  do {                             \
    l0cim_status _s = (x);         \
    if (_s != L0CIM_OK) return _s; \
  } while (0)
  hipLaunchKernelGGL(cac_stats_init_kernel, dim3(1), dim3(1), 0, s, stats);
  L0_LAUNCHED("cac_stats_init_kernel");
  L0_TRY(launch_gram(dtype, m, n, A, lda, y, G, n, b, s));
  L0_TRY(launch_r_init(dtype, n, G, n, b, nullptr, R_out, status, s));
  double eta = sp->eta_init;
  for (int i = 0; i < sp->n_outer; ++i) {
    const double v = sp->eta_init * (1.0 - double(i) / double(sp->velo));
    eta = v > sp->eta_end ? v : sp->eta_end;
    L0_TRY(launch_couplings(dtype, n, G, n, b, R_out, dtype, J, n, reinterpret_cast<float*>(base + L.rs), z, s));
    const CacArgs a = cac_args(n, P, prm, eta, sp->seed, i, 0);
    L0_TRY(launch_cac_run(dtype, n, P, J, n, z, a, base + L.mu, base + L.nv, base + L.mv, base + L.e, sig, H, nullptr,
                          status, base + L.run, s));
    L0_TRY(launch_select(n, P, H, sig, sigma_out, &stats->selected_replica, &stats->H, s));
    L0_TRY(launch_jacobi(dtype, n, G, n, b, sigma_out, sp->dtc, sp->cdp_iters, R_out, status, base + L.cdp,
                         jacobi_ws_bytes(dtype, n), s, kDefaultSpinLimit));
  }
  const int64_t spin_steps = int64_t(n) * P * prm->n_steps * sp->n_outer;
  L0_TRY(launch_objective(dtype, m, n, A, lda, y, sigma_out, R_out, 0.5 * eta * eta, stats, spin_steps, sp->n_outer,
                          base + L.obj, objective_ws_bytes(m), s));
#undef L0_TRY
  return L0CIM_OK;
}

}  // extern "C"
