// MFZ-CIM run kernels: eq. 12-14 with the local field of eq. 15 (CN) or
// eq. 16 (BN), pump schedule eq. 21, forward Euler.
//
// Two launch shapes:
//  * cim_resident_kernel: one persistent cooperative launch for the whole run.
//    Each workgroup keeps a block of rows of J in LDS for all n_steps steps,
//    computes its rows' local fields with wavefront-reduced dot products,
//    applies the Euler update to the amplitudes it owns and publishes them
//    through flag-carrying 64-bit words (see LL in common.h).  Every
//    workgroup gathers the full amplitude vector of the step from those words,
//    so no grid-wide barrier is needed.  With a single workgroup (small n) the
//    exchange stays in LDS.
//  * cim_stream_step_kernel: one launch per Euler step, J streamed from HBM,
//    for couplings too large to stay on chip.
#include <type_traits>

#include "kernels.h"

namespace l0 {
namespace {

constexpr int kCN = 0;
constexpr int kBN = 1;

template <typename T> struct AccT { using type = float; };
template <> struct AccT<double> { using type = double; };

__host__ __device__ inline size_t a16(size_t x) { return (x + 15) & ~size_t(15); }

struct ResidentLayout {
  size_t j, x, cs, es, zs, sc, hc, flag, total;
};

template <typename T, typename JT>
__host__ __device__ inline ResidentLayout resident_layout(int n, int P, int rpw) {
  ResidentLayout L;
  size_t o = 0;
  L.j = o;    o += a16(size_t(rpw) * n * sizeof(JT));
  L.x = o;    o += a16(size_t(P) * n * sizeof(T));
  L.cs = o;   o += a16(size_t(P) * rpw * sizeof(T));
  L.es = o;   o += a16(size_t(P) * rpw * sizeof(T));
  L.zs = o;   o += a16(size_t(rpw) * sizeof(T));
  L.sc = o;   o += a16(size_t(rpw) * sizeof(float));
  L.hc = o;   o += a16(size_t(P) * rpw * sizeof(double));
  L.flag = o; o += 16;
  L.total = o;
  return L;
}

// Euler update of one (spin, replica) from its local-field dot product y.
template <typename T, int FIELD>
__device__ inline void euler_update(T& c, T& e, T y, T zr, T lin, T theta, T half_st, T jj, T KK,
                                    T beta, T tau, T dt) {
  T phi = (FIELD == kCN) ? (y + half_st * zr) : (half_st * (y + zr));
  T inj = jj * e * (phi - theta);
  T c2 = c * c;
  T dc = (lin - c2) * c + KK * inj;
  T de = -beta * (c2 - tau) * e;
  c = c + dt * dc;
  e = e + dt * de;
}

template <typename T, int FIELD>
__device__ inline T xform(T c, T st, bool binary) {
  if (binary || FIELD == kBN) return c > T(0) ? T(1) : T(0);
  return (c + st) * T(0.25);
}

template <typename T, typename JT, int FIELD>
__global__ void __launch_bounds__(512)
cim_resident_kernel(const JT* __restrict__ J, int64_t ldj, const float* __restrict__ rscale,
                    const T* __restrict__ z, CimArgs a, T* __restrict__ c, T* __restrict__ e,
                    uint8_t* __restrict__ sigma, double* __restrict__ Hpart, T* __restrict__ trace,
                    uint64_t* __restrict__ ll, int* __restrict__ abort_word, int* __restrict__ status,
                    int rpw) {
  using Acc = typename AccT<T>::type;
  constexpr int W = LL<T>::kWords;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = a.n, P = a.P;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int lane = tid & (kWave - 1), wv = tid / kWave, nwv = bs / kWave;
  const int r0 = blockIdx.x * rpw;
  const int nr = max(0, min(n, r0 + rpw) - r0);
  const bool solo = gridDim.x == 1;
  const size_t slot_words = size_t(P) * n * W;

  const ResidentLayout L = resident_layout<T, JT>(n, P, rpw);
  JT* Jl = reinterpret_cast<JT*>(smem + L.j);
  T* X = reinterpret_cast<T*>(smem + L.x);
  T* cs = reinterpret_cast<T*>(smem + L.cs);
  T* es = reinterpret_cast<T*>(smem + L.es);
  T* zs = reinterpret_cast<T*>(smem + L.zs);
  float* sc = reinterpret_cast<float*>(smem + L.sc);
  double* hc = reinterpret_cast<double*>(smem + L.hc);
  int* lds_abort = reinterpret_cast<int*>(smem + L.flag);

  // Stage the owned rows of J and the owned state.
  for (size_t i = tid; i < size_t(nr) * n; i += bs) {
    size_t rl = i / n, jj = i - rl * n;
    Jl[i] = J[size_t(r0 + rl) * ldj + jj];
  }
  for (int i = tid; i < P * nr; i += bs) {
    int q = i / nr, rl = i - q * nr;
    cs[q * rpw + rl] = c[size_t(q) * n + r0 + rl];
    es[q * rpw + rl] = e[size_t(q) * n + r0 + rl];
  }
  for (int i = tid; i < nr; i += bs) {
    zs[i] = z[r0 + i];
    sc[i] = rscale ? rscale[r0 + i] : 1.0f;
  }
  if (tid == 0) *lds_abort = 0;
  __syncthreads();
  if (!solo) {
    for (int i = tid; i < P * nr; i += bs) {
      int q = i / nr, rl = i - q * nr;
      LL<T>::put(ll + (size_t(q) * n + r0 + rl) * W, cs[q * rpw + rl], 1u);
    }
  }

  const T st = T(sqrt(a.tau));
  const T half_st = T(0.5 * sqrt(a.tau));
  const T theta = T(a.eta * a.eta * sqrt(a.tau) * 0.25);
  const T jj = T(a.j), KK = T(a.K), beta = T(a.beta), tau = T(a.tau), dt = T(a.dt);
  const double lam = 0.5 * a.eta * a.eta;
  const int pairs = nr * P;
  bool aborted = false;

  for (int k = 0; k <= a.n_steps; ++k) {
    const bool last = (k == a.n_steps);
    // 1. amplitudes of step k -> field operand X (H(c) at the end, for eq. 4)
    if (solo) {
      for (int i = tid; i < P * n; i += bs) {
        int q = i / n, r = i - q * n;
        X[i] = xform<T, FIELD>(cs[q * rpw + r], st, last);
      }
    } else {
      const uint64_t* src = ll + size_t(k & 1) * slot_words;
      bool ok = ll_gather<T>(src, P * n, uint32_t(k + 1), a.spin_limit, abort_word,
                             [&](int idx, T v) { X[idx] = xform<T, FIELD>(v, st, last); });
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
    const T lin = T(pump_at(a, k) - 1.0 - (a.linear_j ? a.j : 0.0));
    // 2. one wavefront per (row, replica): dot product, reduction, update
    for (int pr = wv; pr < pairs; pr += nwv) {
      const int q = pr / nr, rl = pr - q * nr;
      const JT* jr = Jl + size_t(rl) * n;
      const T* xq = X + size_t(q) * n;
      Acc acc = Acc(0);
      for (int j = lane; j < n; j += kWave) acc += Acc(JLoad<JT>::get(jr[j])) * Acc(xq[j]);
      acc = wave_sum(acc);
      if (lane == 0) {
        const T y = T(acc) * T(sc[rl]);
        T cv = cs[q * rpw + rl];
        if (!last) {
          T ev = es[q * rpw + rl];
          euler_update<T, FIELD>(cv, ev, y, zs[rl], lin, theta, half_st, jj, KK, beta, tau, dt);
          cs[q * rpw + rl] = cv;
          es[q * rpw + rl] = ev;
          if (!solo)
            LL<T>::put(ll + size_t((k + 1) & 1) * slot_words + (size_t(q) * n + r0 + rl) * W, cv,
                       uint32_t(k + 2));
          if (k < a.trace_steps) {
            trace[(size_t(2 * k) * P + q) * n + r0 + rl] = cv;
            trace[(size_t(2 * k + 1) * P + q) * n + r0 + rl] = ev;
          }
        } else {
          // eq. 4 contribution of spin r: s_r (-1/2 (J s)_r - z_r + lambda)
          hc[q * rpw + rl] = cv > T(0) ? (-0.5 * double(y) - double(zs[rl]) + lam) : 0.0;
        }
      }
    }
    __syncthreads();
  }

  // Final state, support and status.
  int bits = 0;
  for (int i = tid; i < P * nr; i += bs) {
    int q = i / nr, rl = i - q * nr;
    T cv = cs[q * rpw + rl], ev = es[q * rpw + rl];
    size_t g = size_t(q) * n + r0 + rl;
    c[g] = cv;
    e[g] = ev;
    sigma[g] = cv > T(0) ? 1 : 0;
    if (!(isfinite(double(cv)) && isfinite(double(ev)))) bits |= L0CIM_ST_NONFINITE;
    else if (fabs(double(cv)) > 1e3) bits |= L0CIM_ST_BLOWUP;
  }
  if (aborted) bits |= L0CIM_ST_TIMEOUT;
  if (bits) raise_status(status, bits);
  if (Hpart && tid < P) {
    double h = 0.0;
    if (!aborted)
      for (int rl = 0; rl < nr; ++rl) h += hc[tid * rpw + rl];
    Hpart[size_t(blockIdx.x) * P + tid] = aborted ? NAN : h;
  }
}

// One Euler step over all rows, J streamed from global memory.  Rows are
// owned by wavefronts; each wavefront loops over the replicas.  On the call
// with k == n_steps it only evaluates the eq. 4 partial energies.
template <typename T, typename JT, int FIELD>
__global__ void __launch_bounds__(256)
cim_stream_step_kernel(const JT* __restrict__ J, int64_t ldj, const float* __restrict__ rscale,
                       const T* __restrict__ z, CimArgs a, int k, const T* __restrict__ cin,
                       T* __restrict__ cout, T* __restrict__ e, uint8_t* __restrict__ sigma,
                       double* __restrict__ Hpart, T* __restrict__ trace, int* __restrict__ status) {
  using Acc = typename AccT<T>::type;
  constexpr int kRows = 4;  // one row per wavefront
  __shared__ double hsum[kRows];
  const int n = a.n, P = a.P;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int r = blockIdx.x * kRows + wv;
  const bool last = (k == a.n_steps);
  const T st = T(sqrt(a.tau));
  const T half_st = T(0.5 * sqrt(a.tau));
  const T theta = T(a.eta * a.eta * sqrt(a.tau) * 0.25);
  const T lin = T(pump_at(a, k) - 1.0 - (a.linear_j ? a.j : 0.0));
  const double lam = 0.5 * a.eta * a.eta;
  for (int q = 0; q < P; ++q) {
    double hterm = 0.0;
    if (r < n) {
      const JT* jr = J + size_t(r) * ldj;
      const T* cq = cin + size_t(q) * n;
      Acc acc = Acc(0);
      for (int j = lane; j < n; j += kWave)
        acc += Acc(JLoad<JT>::get(jr[j])) * Acc(xform<T, FIELD>(cq[j], st, last));
      acc = wave_sum(acc);
      if (lane == 0) {
        const T y = T(acc) * T(rscale ? rscale[r] : 1.0f);
        const size_t g = size_t(q) * n + r;
        T cv = cq[r];
        if (!last) {
          T ev = e[g];
          euler_update<T, FIELD>(cv, ev, y, z[r], lin, theta, half_st, T(a.j), T(a.K), T(a.beta),
                                 T(a.tau), T(a.dt));
          cout[g] = cv;
          e[g] = ev;
          if (k < a.trace_steps) {
            trace[(size_t(2 * k) * P + q) * n + r] = cv;
            trace[(size_t(2 * k + 1) * P + q) * n + r] = ev;
          }
        } else {
          hterm = cv > T(0) ? (-0.5 * double(y) - double(z[r]) + lam) : 0.0;
          T ev = e[g];
          sigma[g] = cv > T(0) ? 1 : 0;
          int bits = 0;
          if (!(isfinite(double(cv)) && isfinite(double(ev)))) bits |= L0CIM_ST_NONFINITE;
          else if (fabs(double(cv)) > 1e3) bits |= L0CIM_ST_BLOWUP;
          if (bits) raise_status(status, bits);
        }
      }
    }
    if (last && Hpart) {
      if (lane == 0) hsum[wv] = hterm;
      __syncthreads();
      if (threadIdx.x == 0) {
        double h = 0.0;
        for (int w = 0; w < kRows; ++w) h += hsum[w];
        Hpart[size_t(blockIdx.x) * P + q] = h;
      }
      __syncthreads();
    }
  }
}

// One workgroup per replica: 256 contiguous runs of the G partials summed in
// order, then a fixed tree.
__global__ void __launch_bounds__(256)
reduce_h_kernel(const double* __restrict__ Hpart, int G, int P, double* __restrict__ H) {
  __shared__ double part[256];
  const int q = blockIdx.x, t = threadIdx.x;
  const int chunk = (G + 255) / 256;
  const int lo = min(G, t * chunk), hi = min(G, lo + chunk);
  double h = 0.0;
  for (int w = lo; w < hi; ++w) h += Hpart[size_t(w) * P + q];
  part[t] = h;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) part[t] += part[t + s];
    __syncthreads();
  }
  if (t == 0) H[q] = part[0];
}

// argmin over replicas (first on ties), then copy that replica's sigma.
__global__ void select_kernel(int n, int P, const double* __restrict__ H,
                              const uint8_t* __restrict__ sigma, uint8_t* __restrict__ out,
                              int32_t* __restrict__ q_out, double* __restrict__ H_out) {
  __shared__ int qs;
  if (threadIdx.x == 0) {
    int best = 0;
    double hb = H ? H[0] : 0.0;
    for (int q = 1; q < P && H; ++q) {
      double h = H[q];
      if (h < hb || (isnan(hb) && !isnan(h))) {
        hb = h;
        best = q;
      }
    }
    qs = best;
    if (q_out) *q_out = best;
    if (H_out) *H_out = hb;
  }
  __syncthreads();
  const uint8_t* src = sigma + size_t(qs) * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = src[i];
}

// Sleep (units of 64 clocks) before the first poll of each step of the
// register-resident run.
constexpr int kFirstPollSleep = 17;

// Single-replica resident run with the couplings held in registers.  Thread t
// of a 512-thread workgroup keeps J[r0 + rho][t + u*512] for its rows rho < R
// and columns u < C, gathers exactly the amplitudes of those columns from the
// exchange words, multiplies, and the row sums are reduced across the
// workgroup through LDS.  Wavefront 0 owns the state of the workgroup's rows.
//
// Several independent instances of the same n may share one launch (their
// exchange round trips then overlap): instance i owns workgroups
// [i G, (i + 1) G), and its couplings, per-spin vectors, run workspace and
// status word sit at the strides of `mb` from the first instance's.  A single
// instance has G = the grid and zero strides.
struct RegsBatch {
  int G;           // workgroups per instance
  int64_t sJ;      // elements between the instances' couplings
  int64_t sv;      // elements between the instances' per-spin vectors (c, e, z, row scales, sigma)
  int64_t sws;     // bytes between the instances' run workspaces (exchange words, abort word, energies)
  int64_t sst;     // ints between the instances' status words
};

template <typename T, typename JT, int FIELD, int R, int C>
__global__ void __launch_bounds__(512)
cim_regs_kernel(const JT* __restrict__ J, int64_t ldj, const float* __restrict__ rscale,
                const T* __restrict__ z, CimArgs a, T* __restrict__ c, T* __restrict__ e,
                uint8_t* __restrict__ sigma, double* __restrict__ Hpart, T* __restrict__ trace,
                uint64_t* __restrict__ ll, int* __restrict__ abort_word, int* __restrict__ status,
                int rpw, RegsBatch mb) {
  using Acc = typename AccT<T>::type;
  constexpr int BS = 512, NW = BS / kWave;
  constexpr int W = LL<T>::kWords;
  __shared__ Acc part[2][NW][R];
  __shared__ int lds_abort;
  const int n = a.n;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int inst = blockIdx.x / mb.G, bx = blockIdx.x - inst * mb.G;
  if (inst > 0) {
    J += inst * mb.sJ;
    if (rscale) rscale += inst * mb.sv;
    z += inst * mb.sv;
    c += inst * mb.sv;
    e += inst * mb.sv;
    sigma += inst * mb.sv;
    ll = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(ll) + inst * mb.sws);
    abort_word = reinterpret_cast<int*>(reinterpret_cast<char*>(abort_word) + inst * mb.sws);
    if (Hpart) Hpart = reinterpret_cast<double*>(reinterpret_cast<char*>(Hpart) + inst * mb.sws);
    status += inst * mb.sst;
  }
  const int r0 = bx * rpw;
  const int nr = max(0, min(n, r0 + rpw) - r0);
  const size_t slot_words = size_t(n) * W;

  Acc Jr[R][C];
#pragma unroll
  for (int u = 0; u < C; ++u) {
    const int j = tid + u * BS;
#pragma unroll
    for (int rho = 0; rho < R; ++rho)
      Jr[rho][u] = (rho < nr && j < n) ? Acc(JLoad<JT>::get(J[size_t(r0 + rho) * ldj + j])) : Acc(0);
  }
  const bool owner = (wv == 0 && lane < nr);
  T cv = T(0), ev = T(0), zr = T(0);
  float scl = 1.0f;
  if (owner) {
    cv = c[r0 + lane];
    ev = e[r0 + lane];
    zr = z[r0 + lane];
    scl = rscale ? rscale[r0 + lane] : 1.0f;
    LL<T>::put(ll + size_t(r0 + lane) * W, cv, 1u);
  }
  if (tid == 0) lds_abort = 0;
  __syncthreads();

  const T st = T(sqrt(a.tau));
  const T half_st = T(0.5 * sqrt(a.tau));
  const T theta = T(a.eta * a.eta * sqrt(a.tau) * 0.25);
  const T jj = T(a.j), KK = T(a.K), beta = T(a.beta), tau = T(a.tau), dt = T(a.dt);
  const double lam = 0.5 * a.eta * a.eta;
  bool aborted = false;

  for (int k = 0; k <= a.n_steps; ++k) {
    // Every workgroup publishes its spins about the same time after its own
    // barrier, and a poll that reaches memory before the words do comes back
    // stale and costs a second round trip (about 0.3 us): the first poll of a
    // step waits kFirstPollSleep x 64 clocks (about 0.45 us).  At N = 2000 on
    // MI355X, 2000 steps took 2.90 ms with 17 units, 3.20 / 2.92 / 2.96 ms with
    // 15 / 18 / 19, and 3.8 ms with no sleep.  A second poll issued a little
    // after the first, to catch late words without a round trip, and several
    // copies of the exchange words, to spread the polls, were both slower: the
    // polls of all workgroups arrive together and extra requests queue.
    if (k > 0) __builtin_amdgcn_s_sleep(kFirstPollSleep);
    const bool last = (k == a.n_steps);
    const uint64_t* src = ll + size_t(k & 1) * slot_words;
    const uint32_t flag = uint32_t(k + 1);
    // 1. gather this thread's columns: issue every load, then re-poll the late ones together
    uint64_t w[C][W];
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int j = tid + u * BS;
#pragma unroll
      for (int v = 0; v < W; ++v) w[u][v] = (j < n) ? ll_load(src + size_t(j) * W + v) : (uint64_t(flag) << 32);
    }
    // The pump value of this step (an FP64 exp and two divisions) is evaluated
    // after the loads are issued, in their shadow: before them it delayed the
    // owner wavefront's gather, and with it the whole step.
    T lin = T(0);
    if (owner && !last) lin = T(pump_at(a, k) - 1.0 - (a.linear_j ? a.j : 0.0));
    int64_t polls = 0;
    bool ok = true;
    for (;;) {
      bool ready = true;
#pragma unroll
      for (int u = 0; u < C; ++u)
#pragma unroll
        for (int v = 0; v < W; ++v) ready = ready && (uint32_t(w[u][v] >> 32) == flag);
      if (ready) break;
      if (++polls > a.spin_limit || ((polls & 1023) == 0 && abort_seen(abort_word))) {
        ok = false;
        break;
      }
#pragma unroll
      for (int u = 0; u < C; ++u) {
        const int j = tid + u * BS;
#pragma unroll
        for (int v = 0; v < W; ++v)
          if (uint32_t(w[u][v] >> 32) != flag) w[u][v] = ll_load(src + size_t(j) * W + v);
      }
    }
    if (!ok) {
      lds_abort = 1;
      __hip_atomic_store(abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // 2. partial row sums of this thread's columns, reduced per wavefront
    Acc acc[R];
#pragma unroll
    for (int rho = 0; rho < R; ++rho) acc[rho] = Acc(0);
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const Acc x = Acc(xform<T, FIELD>(ll_decode<T>(w[u]), st, last));
#pragma unroll
      for (int rho = 0; rho < R; ++rho) acc[rho] += Jr[rho][u] * x;
    }
    wave_sum_rows<Acc, R>(acc, lane);
    if ((lane & (kWave / R - 1)) == 0) part[k & 1][wv][wave_row_of<R>(lane)] = acc[0];
    __syncthreads();
    if (lds_abort) {
      aborted = true;
      break;
    }
    // 3. owners: row sums in a fixed order, Euler update, publish
    if (wv == 0) {
      double hterm = 0.0;
      if (owner) {
        Acc yacc = Acc(0);
        for (int q = 0; q < NW; ++q) yacc += part[k & 1][q][lane];
        const T y = T(yacc) * T(scl);
        if (!last) {
          euler_update<T, FIELD>(cv, ev, y, zr, lin, theta, half_st, jj, KK, beta, tau, dt);
          LL<T>::put(ll + size_t((k + 1) & 1) * slot_words + size_t(r0 + lane) * W, cv, uint32_t(k + 2));
          if (k < a.trace_steps) {
            trace[size_t(2 * k) * n + r0 + lane] = cv;
            trace[size_t(2 * k + 1) * n + r0 + lane] = ev;
          }
        } else {
          hterm = cv > T(0) ? (-0.5 * double(y) - double(zr) + lam) : 0.0;
        }
      }
      if (last && Hpart) {
        // fixed-order sum over the owned rows
        __shared__ double hrow[kWave];
        hrow[lane] = hterm;
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
          double h = 0.0;
          for (int q = 0; q < nr; ++q) h += hrow[q];
          Hpart[bx] = h;
        }
      }
    }
  }
  if (owner) {
    c[r0 + lane] = cv;
    e[r0 + lane] = ev;
    sigma[r0 + lane] = cv > T(0) ? 1 : 0;
    int bits = 0;
    if (!(isfinite(double(cv)) && isfinite(double(ev)))) bits |= L0CIM_ST_NONFINITE;
    else if (fabs(double(cv)) > 1e3) bits |= L0CIM_ST_BLOWUP;
    if (aborted) bits |= L0CIM_ST_TIMEOUT;
    if (bits) raise_status(status, bits);
  }
  if (aborted && tid == 0 && Hpart) Hpart[bx] = NAN;
}

struct RunWs {
  uint64_t* ll;
  int* abort_word;
  double* hpart;
  void* cbuf;
};

template <typename T>
RunWs carve_run_ws(void* ws, int n, int P) {
  RunWs w;
  char* p = static_cast<char*>(ws);
  size_t ll_bytes = align_up(size_t(2) * P * n * LL<T>::kWords * sizeof(uint64_t));
  w.ll = reinterpret_cast<uint64_t*>(p);
  p += ll_bytes;
  w.abort_word = reinterpret_cast<int*>(p);
  p += kAlign;
  w.hpart = reinterpret_cast<double*>(p);
  p += align_up(size_t(n) * P * sizeof(double));
  w.cbuf = p;
  return w;
}

template <typename T, typename JT, int FIELD>
l0cim_status run_typed(int n, int P, const JT* J, int64_t ldj, const float* rscale, const T* z,
                       const CimArgs& a, T* c, T* e, uint8_t* sigma, double* H, T* trace,
                       int* status, void* ws, bool allow_matrix, hipStream_t s) {
  DeviceInfo dev;
  l0cim_status st = device_info(&dev);
  if (st != L0CIM_OK) return st;
  RunWs w = carve_run_ws<T>(ws, n, P);

  // Launch shape.  Small problems run in one workgroup with everything in
  // LDS; one FP32 replica keeps its couplings in registers; a few replicas
  // keep rows of J in LDS when they fit; many FP32 replicas stream J through
  // the matrix cores; otherwise J is streamed every step by the vector units.
  int rpw = 0, grid = 0, block = 256;
  size_t lds = 0;
  const int rpw_cu = (n + dev.cu_count - 1) / dev.cu_count;
  if constexpr (sizeof(T) == 4) {
    const bool small = n <= 256 && resident_layout<T, JT>(n, P, n).total <= size_t(dev.max_lds);
    const bool lds_fits = resident_layout<T, JT>(n, P, rpw_cu).total <= size_t(dev.max_lds);
    const bool want = allow_matrix && (a.launch == L0CIM_LAUNCH_MATRIX ||
                                       (a.launch == L0CIM_LAUNCH_AUTO && P >= 2 && !small && !(lds_fits && P <= 4)));
    if (want) {
      l0cim_dtype jdt = std::is_same<JT, float>::value ? L0CIM_F32
                        : (sizeof(JT) == 2 ? L0CIM_BF16 : L0CIM_FP8E4M3);
      if (matrix_supported(n, P, ldj))
        return launch_matrix_run(n, P, jdt, J, ldj, rscale, z, a, c, e, sigma, H, trace, status,
                                 static_cast<char*>(ws) + matrix_ws_offset(n, P), s, 0);
      if (a.launch == L0CIM_LAUNCH_MATRIX)
        return set_error(L0CIM_ERR_UNSUPPORTED, "mfcim_run: matrix launch needs P <= 64 and ldj %% 32 == 0");
    }
  } else {
    if (a.launch == L0CIM_LAUNCH_MATRIX)
      return set_error(L0CIM_ERR_UNSUPPORTED, "mfcim_run: matrix launch needs FP32 state");
  }
  if (a.launch != L0CIM_LAUNCH_STREAMED) {
    const size_t whole = resident_layout<T, JT>(n, P, n).total;
    if (n <= 256 && whole <= size_t(dev.max_lds)) {
      rpw = n;
      grid = 1;
      lds = whole;
    }
    if constexpr (sizeof(T) == 4) {
      if (!rpw && P == 1) {
        const int cols = (n + 511) / 512;
        void (*rk)(const JT*, int64_t, const float*, const T*, CimArgs, T*, T*, uint8_t*, double*, T*,
                   uint64_t*, int*, int*, int, RegsBatch) = nullptr;
        if (rpw_cu <= 8 && cols <= 4) rk = cim_regs_kernel<T, JT, FIELD, 8, 4>;
        else if (rpw_cu <= 16 && cols <= 8) rk = cim_regs_kernel<T, JT, FIELD, 16, 8>;
        if (rk) {
          const int g = (n + rpw_cu - 1) / rpw_cu;
          size_t words = size_t(2) * n * LL<T>::kWords;
          hipLaunchKernelGGL(ll_clear_kernel, dim3(256), dim3(256), 0, s, w.ll, words, w.abort_word);
          L0_LAUNCHED("clear exchange buffer");
          CimArgs args = a;
          const JT* Jp = J;
          int rp = rpw_cu;
          RegsBatch mb{g, 0, 0, 0, 0};
          void* kargs[] = {&Jp, &ldj, &rscale, &z, &args, &c, &e, &sigma, &w.hpart, &trace,
                           &w.ll, &w.abort_word, &status, &rp, &mb};
          {
            ProfileScope prof(s);
            L0_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(rk), dim3(g), dim3(512),
                                              kargs, 0u, s));
          }
          if (H) {
            hipLaunchKernelGGL(reduce_h_kernel, dim3(P), dim3(256), 0, s, w.hpart, g, P, H);
            L0_LAUNCHED("reduce_h_kernel");
          }
          return L0CIM_OK;
        }
      }
    }
    if (!rpw) {
      size_t need = resident_layout<T, JT>(n, P, rpw_cu).total;
      if (need <= size_t(dev.max_lds)) {
        rpw = rpw_cu;
        grid = (n + rpw_cu - 1) / rpw_cu;
        lds = need;
      }
    }
    if (rpw) block = (rpw * P >= 8) ? 512 : 256;
    if (!rpw && a.launch == L0CIM_LAUNCH_RESIDENT)
      return set_error(L0CIM_ERR_UNSUPPORTED, "mfcim_run: n=%d P=%d does not fit the resident launch", n, P);
  }

  if (rpw) {
    auto kern = cim_resident_kernel<T, JT, FIELD>;
    if (grid > 1) {
      size_t words = size_t(2) * P * n * LL<T>::kWords;
      hipLaunchKernelGGL(ll_clear_kernel, dim3(256), dim3(256), 0, s, w.ll, words, w.abort_word);
      L0_LAUNCHED("clear exchange buffer");
    }
    L0_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    CimArgs args = a;
    const JT* Jp = J;
    int rp = rpw;
    void* kargs[] = {&Jp, &ldj, &rscale, &z, &args, &c, &e, &sigma, &w.hpart, &trace,
                     &w.ll, &w.abort_word, &status, &rp};
    ProfileScope prof(s);
    if (grid > 1) {
      L0_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(block),
                                        kargs, unsigned(lds), s));
    } else {
      hipLaunchKernelGGL(kern, dim3(1), dim3(block), lds, s, Jp, ldj, rscale, z, args, c, e, sigma,
                         w.hpart, trace, w.ll, w.abort_word, status, rp);
      L0_LAUNCHED("cim_resident_kernel");
    }
  } else {
    // Streamed: ping-pong amplitudes between c and the workspace copy.
    T* cb = static_cast<T*>(w.cbuf);
    grid = (n + 3) / 4;
    T* cur = c;
    T* nxt = cb;
    ProfileScope prof(s);
    for (int k = 0; k <= a.n_steps; ++k) {
      hipLaunchKernelGGL((cim_stream_step_kernel<T, JT, FIELD>), dim3(grid), dim3(256), 0, s, J, ldj,
                         rscale, z, a, k, cur, nxt, e, sigma, w.hpart, trace, status);
      L0_LAUNCHED("cim_stream_step_kernel");
      if (k < a.n_steps) {
        T* t = cur;
        cur = nxt;
        nxt = t;
      }
    }
    if (cur != c) {
      L0_HIP(hipMemcpyAsync(c, cur, size_t(P) * n * sizeof(T), hipMemcpyDeviceToDevice, s));
    }
  }
  if (H) {
    hipLaunchKernelGGL(reduce_h_kernel, dim3(P), dim3(256), 0, s, w.hpart, grid, P, H);
    L0_LAUNCHED("reduce_h_kernel");
  }
  return L0CIM_OK;
}

template <typename T, typename JT>
l0cim_status run_field(int n, int P, const void* J, int64_t ldj, const float* rscale, const void* z,
                       const CimArgs& a, void* c, void* e, uint8_t* sigma, double* H, void* trace,
                       int* status, void* ws, bool allow_matrix, hipStream_t s) {
  auto Jp = static_cast<const JT*>(J);
  auto zp = static_cast<const T*>(z);
  auto cp = static_cast<T*>(c);
  auto ep = static_cast<T*>(e);
  auto tp = static_cast<T*>(trace);
  if (a.field == L0CIM_FIELD_BN)
    return run_typed<T, JT, kBN>(n, P, Jp, ldj, rscale, zp, a, cp, ep, sigma, H, tp, status, ws, allow_matrix, s);
  return run_typed<T, JT, kCN>(n, P, Jp, ldj, rscale, zp, a, cp, ep, sigma, H, tp, status, ws, allow_matrix, s);
}

// Several single-replica FP32 runs of the same n in one cooperative launch
// of the register-resident kernel (RegsBatch strides); UNSUPPORTED when the
// shape has no register-resident form or the instances do not all fit on
// the device at once.
template <typename JT, int FIELD>
l0cim_status regs_many_typed(int count, int n, const JT* J, int64_t ldj, int64_t sJ, const float* rscale,
                             const float* z, int64_t sv, const CimArgs& a, float* c, float* e, uint8_t* sigma,
                             double* H, int64_t sh, int* status, int64_t sst, void* ws, int64_t sws, hipStream_t s) {
  DeviceInfo dev;
  l0cim_status st = device_info(&dev);
  if (st != L0CIM_OK) return st;
  const int rpw_cu = (n + dev.cu_count - 1) / dev.cu_count;
  const int cols = (n + 511) / 512;
  // the form l0cim_mfcim_run takes for one such instance (run_typed)
  const bool small = n <= 256 && resident_layout<float, JT>(n, 1, n).total <= size_t(dev.max_lds);
  const bool regs_ok = !small && (a.launch == L0CIM_LAUNCH_AUTO || a.launch == L0CIM_LAUNCH_RESIDENT);
  void (*rk)(const JT*, int64_t, const float*, const float*, CimArgs, float*, float*, uint8_t*, double*, float*,
             uint64_t*, int*, int*, int, RegsBatch) = nullptr;
  if (regs_ok && rpw_cu <= 8 && cols <= 4) rk = cim_regs_kernel<float, JT, FIELD, 8, 4>;
  else if (regs_ok && rpw_cu <= 16 && cols <= 8) rk = cim_regs_kernel<float, JT, FIELD, 16, 8>;
  if (!rk) return set_error(L0CIM_ERR_UNSUPPORTED, "mfcim_run_many: n = %d has no register-resident form", n);
  const int g = (n + rpw_cu - 1) / rpw_cu;
  int per_cu = 0;
  L0_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(rk), 512, 0));
  if (int64_t(per_cu) * dev.cu_count < int64_t(count) * g)
    return set_error(L0CIM_ERR_UNSUPPORTED, "mfcim_run_many: %d instances of %d workgroups exceed %d resident", count,
                     g, per_cu * dev.cu_count);
  for (int i = 0; i < count; ++i) {
    RunWs w = carve_run_ws<float>(static_cast<char*>(ws) + i * sws, n, 1);
    hipLaunchKernelGGL(ll_clear_kernel, dim3(64), dim3(256), 0, s, w.ll, size_t(2) * n, w.abort_word);
    L0_LAUNCHED("clear exchange buffer");
  }
  RunWs w0 = carve_run_ws<float>(ws, n, 1);
  CimArgs args = a;
  args.trace_steps = 0;
  float* trace = nullptr;
  int rp = rpw_cu;
  RegsBatch mb{g, sJ, sv, sws, sst};
  void* kargs[] = {&J, &ldj, &rscale, &z, &args, &c, &e, &sigma, &w0.hpart, &trace, &w0.ll, &w0.abort_word, &status,
                   &rp, &mb};
  {
    ProfileScope prof(s);
    L0_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(rk), dim3(g * count), dim3(512), kargs, 0u, s));
  }
  if (H) {
    for (int i = 0; i < count; ++i) {
      RunWs w = carve_run_ws<float>(static_cast<char*>(ws) + i * sws, n, 1);
      hipLaunchKernelGGL(reduce_h_kernel, dim3(1), dim3(256), 0, s, w.hpart, g, 1, H + i * sh);
      L0_LAUNCHED("reduce_h_kernel");
    }
  }
  return L0CIM_OK;
}

}  // namespace

// Workspace of a run: the exchange words, the abort word, per-workgroup
// energies and the streamed ping-pong copy, followed (FP32 state) by the
// matrix-core run's tables and padded state.
size_t mfcim_base_ws_bytes(l0cim_dtype dt, int n, int P) {
  size_t ts = dtype_size(dt);
  size_t words = (dt == L0CIM_F64) ? 2 : 1;
  return align_up(size_t(2) * P * n * words * sizeof(uint64_t)) + kAlign +
         align_up(size_t(n) * P * sizeof(double)) + align_up(size_t(P) * n * ts);
}

size_t matrix_ws_offset(int n, int P) { return mfcim_base_ws_bytes(L0CIM_F32, n, P); }

size_t mfcim_ws_bytes(l0cim_dtype dt, int n, int P) {
  size_t b = mfcim_base_ws_bytes(dt, n, P);
  if (dt == L0CIM_F32 && P <= 64) b += matrix_ws_bytes(n, P, 4);
  return b;
}

l0cim_status launch_mfcim(l0cim_dtype dt, int n, int P, l0cim_dtype jdt, const void* J, int64_t ldj,
                          const float* rscale, const void* z, const CimArgs& a, void* c, void* e,
                          uint8_t* sigma, double* H, void* trace, int* status, void* ws,
                          size_t ws_bytes, hipStream_t s, bool allow_matrix) {
  (void)ws_bytes;
  const bool am = allow_matrix;
  if (dt == L0CIM_F32) {
    switch (jdt) {
      case L0CIM_F32:
        return run_field<float, float>(n, P, J, ldj, rscale, z, a, c, e, sigma, H, trace, status, ws, am, s);
      case L0CIM_BF16:
        return run_field<float, __hip_bfloat16>(n, P, J, ldj, rscale, z, a, c, e, sigma, H, trace,
                                                status, ws, am, s);
      case L0CIM_FP8E4M3:
        return run_field<float, __hip_fp8_e4m3>(n, P, J, ldj, rscale, z, a, c, e, sigma, H, trace,
                                                status, ws, am, s);
      default: break;
    }
  } else if (dt == L0CIM_F64 && jdt == L0CIM_F64) {
    return run_field<double, double>(n, P, J, ldj, rscale, z, a, c, e, sigma, H, trace, status, ws, am, s);
  }
  return set_error(L0CIM_ERR_UNSUPPORTED, "mfcim_run: dtype %d with coupling dtype %d", int(dt), int(jdt));
}

l0cim_status launch_mfcim_many(l0cim_dtype jdt, int count, int n, const void* J, int64_t ldj, int64_t sJ,
                               const float* rscale, const float* z, int64_t sv, const CimArgs& a, float* c, float* e,
                               uint8_t* sigma, double* H, int64_t sh, int* status, int64_t sst, void* ws,
                               int64_t sws, hipStream_t s) {
  const bool bn = a.field == L0CIM_FIELD_BN;
  switch (jdt) {
    case L0CIM_F32:
      return bn ? regs_many_typed<float, kBN>(count, n, (const float*)J, ldj, sJ, nullptr, z, sv, a, c, e, sigma, H,
                                              sh, status, sst, ws, sws, s)
                : regs_many_typed<float, kCN>(count, n, (const float*)J, ldj, sJ, nullptr, z, sv, a, c, e, sigma, H,
                                              sh, status, sst, ws, sws, s);
    case L0CIM_BF16:
      return bn ? regs_many_typed<__hip_bfloat16, kBN>(count, n, (const __hip_bfloat16*)J, ldj, sJ, rscale, z, sv, a, c,
                                                       e, sigma, H, sh, status, sst, ws, sws, s)
                : regs_many_typed<__hip_bfloat16, kCN>(count, n, (const __hip_bfloat16*)J, ldj, sJ, rscale, z, sv, a, c,
                                                       e, sigma, H, sh, status, sst, ws, sws, s);
    case L0CIM_FP8E4M3:
      return bn ? regs_many_typed<__hip_fp8_e4m3, kBN>(count, n, (const __hip_fp8_e4m3*)J, ldj, sJ, rscale, z, sv, a,
                                                       c, e, sigma, H, sh, status, sst, ws, sws, s)
                : regs_many_typed<__hip_fp8_e4m3, kCN>(count, n, (const __hip_fp8_e4m3*)J, ldj, sJ, rscale, z, sv, a,
                                                       c, e, sigma, H, sh, status, sst, ws, sws, s);
    default: break;
  }
  return set_error(L0CIM_ERR_UNSUPPORTED, "mfcim_run_many: coupling dtype %d", int(jdt));
}

l0cim_status launch_select(int n, int P, const double* H, const uint8_t* sigma, uint8_t* out,
                           int32_t* q_out, double* H_out, hipStream_t s) {
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(256), 0, s, n, P, H, sigma, out, q_out, H_out);
  L0_LAUNCHED("select_kernel");
  return L0CIM_OK;
}

}  // namespace l0
