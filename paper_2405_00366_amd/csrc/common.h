// Internal declarations shared by the l0cim HIP translation units (gfx950).
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp8.h>
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#include "l0cim.h"

namespace l0 {

constexpr int kWave = 64;
constexpr size_t kAlign = 256;
constexpr int kMaxLdsBytes = 160 * 1024;   // LDS per workgroup on gfx950
constexpr int64_t kDefaultSpinLimit = int64_t(1) << 22;

inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// Host-side error plumbing
// ---------------------------------------------------------------------------
l0cim_status set_error(l0cim_status s, const char* fmt, ...);
l0cim_status hip_fail(hipError_t e, const char* what);
#define L0_HIP(call)                                         \
  do {                                                       \
    hipError_t _e = (call);                                  \
    if (_e != hipSuccess) return ::l0::hip_fail(_e, #call);  \
  } while (0)
#define L0_LAUNCHED(what)                                    \
  do {                                                       \
    hipError_t _e = hipGetLastError();                       \
    if (_e != hipSuccess) return ::l0::hip_fail(_e, what);   \
  } while (0)

struct DeviceInfo {
  int device;
  int cu_count;
  int max_lds;
};
l0cim_status device_info(DeviceInfo* out);

// Profiling hook: brackets CIM-kernel launches with events when enabled.
struct ProfileScope {
  hipStream_t stream;
  void* ev0;
  ProfileScope(hipStream_t s);
  ~ProfileScope();
};

inline size_t dtype_size(l0cim_dtype t) {
  switch (t) {
    case L0CIM_F32: return 4;
    case L0CIM_F64: return 8;
    case L0CIM_BF16: return 2;
    case L0CIM_FP8E4M3: return 1;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Kernel argument blocks
// ---------------------------------------------------------------------------
struct CimArgs {
  int n, P;
  int n_steps, trace_steps;
  int field, linear_j;
  int launch;
  double dt, p_thr, d, t_c, t_w;
  double K, j, beta, tau;
  double eta;
  int64_t spin_limit;
};

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

// Pump rate of eq. 21 at t = k dt, evaluated in FP64.
__device__ inline double pump_at(const CimArgs& a, int k) {
  double t = double(k) * a.dt;
  return (a.p_thr - a.d) + 2.0 * a.d / (1.0 + exp(-(t - a.t_c) / a.t_w));
}

// Bounded grid barrier for a cooperative launch (every workgroup resident).
// Workgroup w publishes its arrival in a slot of its own, arrive[w *
// kGridSlot] (no contended atomic); workgroup 0 waits for every slot and then
// publishes the generation in *gen_word, which the others wait for.  `gen`
// counts the barriers passed and is the same in every workgroup; the words
// start at zero for each launch.  Arrival is one device-scope release (the
// workgroup's writes, ordered before it by the workgroup barrier, become
// visible first); waits poll with relaxed loads and acquire once they
// succeed (an acquire per poll would invalidate the poller's L2 on every
// iteration).  A wait beyond `limit` polls, or one that sees *abort_word set,
// raises the abort word and returns false.
constexpr int kGridSlot = 16;      // ints between arrival slots (64 bytes)
constexpr int kGridMaxWg = 1024;   // arrival slots
inline size_t grid_barrier_bytes() { return 256 + size_t(kGridMaxWg) * kGridSlot * sizeof(int); }

template <int BS>
__device__ bool grid_barrier(int* gen_word, int* abort_word, int* arrive, int nblocks, int& gen, int64_t limit) {
  __shared__ int ok_sh;
  ++gen;
  if (threadIdx.x == 0) ok_sh = 1;
  __syncthreads();
  const int tid = threadIdx.x, wg = blockIdx.x;
  if (tid == 0) __hip_atomic_store(&arrive[wg * kGridSlot], gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  auto give_up = [&]() {
    ok_sh = 0;
    __hip_atomic_store(abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  if (wg == 0) {
    for (int w = tid; w < nblocks; w += BS) {
      int64_t polls = 0;
      while (__hip_atomic_load(&arrive[w * kGridSlot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gen) {
        if (++polls > limit ||
            ((polls & 255) == 0 && __hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
          give_up();
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __syncthreads();
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (ok_sh) __hip_atomic_store(gen_word, gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else if (tid == 0) {
    int64_t polls = 0;
    while (__hip_atomic_load(gen_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gen) {
      if (++polls > limit || __hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        give_up();
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return ok_sh != 0;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Value of `v` held by this lane's partner across lane bit OFF.  Partners
// differ in lane bit OFF: lane ^ 32 and lane ^ 16 through the LDS crossbar,
// the mirrored lane of the 16- or 8-lane row (i <-> 15 - i, i <-> 7 - i) and
// lane ^ 2, lane ^ 1 through DPP.
template <int OFF>
__device__ inline float lane_partner(float v) {
  const int x = __float_as_int(v);
  if constexpr (OFF == 32) return __shfl_xor(v, 32, kWave);
  else if constexpr (OFF == 16) return __int_as_float(__builtin_amdgcn_ds_swizzle(x, 0x401F));
  else if constexpr (OFF == 8) return __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false));
  else if constexpr (OFF == 4) return __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false));
  else if constexpr (OFF == 2) return __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false));
  else return __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false));
}

template <int OFF>
__device__ inline double lane_partner(double v) {
  return __shfl_xor(v, OFF, kWave);
}

// Sum each of R values over the 64 lanes of a wavefront with a transposed
// butterfly: at each of the first log2(R) levels a lane keeps half of its
// values and adds its partner's copy of them, so R - 1 + (6 - log2 R)
// exchanges replace 6 R.  Afterwards v[0] of lane l holds the full sum of
// value number wave_row_of<R>(l); the order of additions is fixed.
template <int R>
__device__ inline int wave_row_of(int lane) {
  static_assert(R >= 1 && R <= 64 && (R & (R - 1)) == 0, "R must be a power of two <= 64");
  return R == 1 ? 0 : (lane / (64 / R)) & (R - 1);
}

// a' + b' after swapping a's upper half-rows with b's lower ones gives, in
// every lane, own + partner of a (lower lanes) or of b (upper lanes).
template <int OFF>
__device__ inline float swap_pair_sum(float a, float b) {
  if constexpr (OFF == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
}

template <typename T, int R, int COUNT, int OFF>
__device__ inline void wave_sum_rows_level(T (&v)[R], int lane) {
  if constexpr (OFF > 0) {
    if constexpr (std::is_same<T, float>::value && (OFF == 32 || OFF == 16)) {
      constexpr int H = COUNT > 1 ? COUNT / 2 : 1;
#pragma unroll
      for (int i = 0; i < H; ++i) v[i] = swap_pair_sum<OFF>(v[i], COUNT > 1 ? v[i + H] : v[i]);
      wave_sum_rows_level<T, R, (COUNT > 1 ? COUNT / 2 : 1), OFF / 2>(v, lane);
    } else if constexpr (COUNT > 1) {
      constexpr int H = COUNT / 2;
      const bool hi = (lane & OFF) != 0;
      T recv[H];
#pragma unroll
      for (int i = 0; i < H; ++i) recv[i] = lane_partner<OFF>(hi ? v[i] : v[i + H]);
#pragma unroll
      for (int i = 0; i < H; ++i) v[i] = (hi ? v[i + H] : v[i]) + recv[i];
      wave_sum_rows_level<T, R, H, OFF / 2>(v, lane);
    } else {
      v[0] += lane_partner<OFF>(v[0]);
      wave_sum_rows_level<T, R, 1, OFF / 2>(v, lane);
    }
  }
}

template <typename T, int R>
__device__ inline void wave_sum_rows(T (&v)[R], int lane) {
  wave_sum_rows_level<T, R, R, 32>(v, lane);
}

// Exclusive prefix sum of one int per thread over a workgroup of BS threads
// (a multiple of 64, at most 1024): wavefront scans, then the wavefront
// totals in order.  `sh` is LDS scratch of BS / 64 + 1 ints; every thread
// gets its exclusive prefix and the total.  Ends with a barrier.
template <int BS>
__device__ inline int block_exclusive_scan(int v, int* sh, int* total) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  int x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) sh[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < BS / kWave; ++w) {
      const int t = sh[w];
      sh[w] = acc;
      acc += t;
    }
    sh[BS / kWave] = acc;
  }
  __syncthreads();
  *total = sh[BS / kWave];
  const int r = sh[wv] + x - v;
  __syncthreads();
  return r;
}

// Coupling storage decoding.  Integer-exact for bf16 and fp8 (e4m3, OCP).
template <typename JT> struct JLoad;
template <> struct JLoad<float> {
  __device__ static inline float get(float v) { return v; }
};
template <> struct JLoad<double> {
  __device__ static inline double get(double v) { return v; }
};
template <> struct JLoad<__hip_bfloat16> {
  __device__ static inline float get(__hip_bfloat16 v) { return __bfloat162float(v); }
};
template <> struct JLoad<__hip_fp8_e4m3> {
  __device__ static inline float get(__hip_fp8_e4m3 v) { return float(v); }
};

// ---------------------------------------------------------------------------
// Low-latency exchange: each published value travels in 64-bit words whose
// upper half is a flag (the producer's step number + 1) and whose lower half
// is 32 bits of payload.  Stores and loads are relaxed atomics at device
// scope, so a reader sees either the old word or the new one, never a mix,
// and needs no separate barrier.  A float uses one word, a double two.
// ---------------------------------------------------------------------------
template <typename T> struct LL;
template <> struct LL<float> {
  static constexpr int kWords = 1;
  __device__ static inline void put(uint64_t* p, float v, uint32_t flag) {
    uint64_t w = (uint64_t(flag) << 32) | uint64_t(__float_as_uint(v));
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};
template <> struct LL<double> {
  static constexpr int kWords = 2;
  __device__ static inline void put(uint64_t* p, double v, uint32_t flag) {
    uint64_t bits = uint64_t(__double_as_longlong(v));
    uint64_t w0 = (uint64_t(flag) << 32) | (bits & 0xffffffffull);
    uint64_t w1 = (uint64_t(flag) << 32) | (bits >> 32);
    __hip_atomic_store(p, w0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p + 1, w1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};

__device__ inline uint64_t ll_load(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int abort_seen(const int* abort_word) {
  return __hip_atomic_load(const_cast<int*>(abort_word), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void raise_status(int* status, int bits) {
  if (status && bits) __hip_atomic_fetch_or(status, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until word p carries `flag`; returns false after `limit` polls or once
// another workgroup has raised the abort word.
__device__ inline bool ll_wait(const uint64_t* p, uint32_t flag, uint64_t& w, int64_t limit,
                               const int* abort_word) {
  int64_t polls = 0;
  while (uint32_t(w >> 32) != flag) {
    if (++polls > limit) return false;
    if ((polls & 1023) == 0 && abort_seen(abort_word)) return false;
    w = ll_load(p);
  }
  return true;
}

template <typename T>
__device__ inline T ll_decode(const uint64_t* w);
template <>
__device__ inline float ll_decode<float>(const uint64_t* w) {
  return __uint_as_float(uint32_t(w[0]));
}
template <>
__device__ inline double ll_decode<double>(const uint64_t* w) {
  uint64_t bits = (w[0] & 0xffffffffull) | (w[1] << 32);
  return __longlong_as_double(int64_t(bits));
}

// Gather `count` published values carrying `flag` from `src`, storing
// store(idx, value).  Loads of several words are issued before any wait.
template <typename T, typename F>
__device__ inline bool ll_gather(const uint64_t* src, int count, uint32_t flag, int64_t limit,
                                 const int* abort_word, F store) {
  constexpr int W = LL<T>::kWords;
  constexpr int E = 4;
  bool ok = true;
  const int bs = blockDim.x;
  for (int base = threadIdx.x; base < count; base += bs * E) {
    uint64_t w[E][W];
#pragma unroll
    for (int u = 0; u < E; ++u) {
      int idx = base + u * bs;
      if (idx < count) {
#pragma unroll
        for (int v = 0; v < W; ++v) w[u][v] = ll_load(src + size_t(idx) * W + v);
      }
    }
#pragma unroll
    for (int u = 0; u < E; ++u) {
      int idx = base + u * bs;
      if (idx < count && ok) {
#pragma unroll
        for (int v = 0; v < W; ++v)
          if (ok) ok = ll_wait(src + size_t(idx) * W + v, flag, w[u][v], limit, abort_word);
        if (ok) store(idx, ll_decode<T>(w[u]));
      }
    }
  }
  return ok;
}


// Zero `count` exchange words and the abort word before a resident launch
// (a kernel rather than a memset, so that the sequence may be graph-captured).
__global__ static void ll_clear_kernel(uint64_t* p, size_t count, int* abort_word) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < count;
       i += size_t(gridDim.x) * blockDim.x)
    p[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0 && abort_word) *abort_word = 0;
}

}  // namespace l0
