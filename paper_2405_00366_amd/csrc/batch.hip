// Batched form: many instances of uneven size, each with P replicas, solved
// together (Algorithm 1 for every instance in lock step).  With several
// replicas the local-field contraction of eq. 15 / 16 is a dense product
// Y = J X (N x N times N x P) per instance, done on the matrix cores:
//   * FP32 couplings: v_mfma_f32_16x16x4_f32,
//   * BF16 couplings: v_mfma_f32_16x16x32_bf16 (binarised field exact;
//     continuous field as a bf16 hi + lo pair of the operand),
//   * FP8 e4m3 couplings: widened to bf16 in registers (exact: every e4m3
//     value is a bf16 value) and multiplied on the bf16 matrix cores as above,
// with FP32 accumulation, the per-row scale and the Euler update of eq. 12-14
// fused into the epilogue.  One launch per Euler step covers every row tile
// of every instance; the launches of one CIM run form a HIP graph.
#include <vector>

#include "batch.h"

namespace l0 {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kCN = 0;
constexpr int kBN = 1;

// FP8 couplings are widened to bf16 in registers with the hardware e4m3 ->
// bf16 pair conversion (exact for every e4m3 code, subnormals included) and
// multiplied on the bf16 matrix cores, so products and FP32 sums are those of
// the dequantised definition; HBM still serves one byte per coupling.  (The
// FP8 matrix cores themselves are not used: their results on these codes
// differ from the exact products' FP32 sums by more than the FP32 state
// tolerance.)

__device__ inline v4f mfma_f32(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline v4f mfma_bf16(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Field operand of a spin: (c + sqrt(tau))/4 for the continuous field,
// H(c) for the binarised one and for the eq. 4 energy after the last step.
template <int FIELD>
__device__ inline float xf(float c, float st, bool binary) {
  return (FIELD == kBN || binary) ? (c > 0.0f ? 1.0f : 0.0f) : (c + st) * 0.25f;
}

__device__ inline int find_inst(const int64_t* prefix, int count, int64_t g) {
  // largest k with prefix[k] <= g  (prefix has count + 1 entries, prefix[0] = 0)
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Per-alternation preparation over all instances
// ---------------------------------------------------------------------------

// One workgroup per (instance, row of the 16-padded row range): J row (zero
// diagonal, zero padding) written into the panel layout, z, and for narrow
// storage the row scale amax / Q_max and RNE(J / scale).  Padding rows are
// written as zeros.
template <typename JT>
__global__ void __launch_bounds__(256)
bcouplings_kernel(const BInst* __restrict__ insts, const int64_t* __restrict__ row_prefix, int count) {
  __shared__ float red[256];
  const int k = find_inst(row_prefix, count, blockIdx.x);
  const BInst I = insts[k];
  const int r = int(blockIdx.x - row_prefix[k]);
  const int n = I.n, ld = I.ld, np = (n + 15) / 16;
  JT* J = static_cast<JT*>(I.J);
  if (r >= n) {
    for (int j = threadIdx.x; j < ld; j += 256) J[jpanel_offset(r, j, ld, np, int(sizeof(JT)))] = JT(0.0f);
    return;
  }
  const float* G = I.G + size_t(r) * ld;
  const float* R = I.R;
  const float Rr = R[r];
  if constexpr (sizeof(JT) == 4) {
    for (int j = threadIdx.x; j < ld; j += 256)
      J[jpanel_offset(r, j, ld, np, 4)] = (j < n && j != r) ? -(G[j] * (Rr * R[j])) : 0.0f;
    if (threadIdx.x == 0) {
      I.z[r] = Rr * I.b[r];
      I.rs[r] = 1.0f;
    }
  } else {
    constexpr float qmax = sizeof(JT) == 2 ? 1.0f : 448.0f;
    float amax = 0.0f;
    for (int j = threadIdx.x; j < n; j += 256) {
      float v = (j == r) ? 0.0f : -(G[j] * (Rr * R[j]));
      amax = fmaxf(amax, fabsf(v));
    }
    red[threadIdx.x] = amax;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
      __syncthreads();
    }
    const float scale = red[0] > 0.0f ? red[0] / qmax : 1.0f;
    for (int j = threadIdx.x; j < ld; j += 256) {
      float v = (j < n && j != r) ? -(G[j] * (Rr * R[j])) / scale : 0.0f;
      const size_t o = jpanel_offset(r, j, ld, np, int(sizeof(JT)));
      if constexpr (sizeof(JT) == 2) J[o] = __float2bfloat16(v);
      else J[o] = __hip_fp8_e4m3(fminf(fmaxf(v, -448.0f), 448.0f));
    }
    if (threadIdx.x == 0) {
      I.z[r] = Rr * I.b[r];
      I.rs[r] = scale;
    }
  }
}

__device__ inline uint64_t bmix64(uint64_t x) {
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// Initial state of alternation `alt` (each instance's own index when alt < 0)
// for every instance: the same counter generator as the single-instance path,
// keyed by the instance's seed.
__global__ void __launch_bounds__(256)
binit_kernel(const BInst* __restrict__ insts, const int64_t* __restrict__ st_prefix, int count, int P,
             int alt, double std) {
  const int64_t total = st_prefix[count];
  for (int64_t g = blockIdx.x * int64_t(256) + threadIdx.x; g < total; g += int64_t(gridDim.x) * 256) {
    const int k = find_inst(st_prefix, count, g);
    const BInst I = insts[k];
    const int64_t li = g - st_prefix[k];          // index inside P x ld
    const uint64_t q = uint64_t(li / I.ld), r = uint64_t(li % I.ld);
    const uint64_t ia = uint64_t(alt >= 0 ? alt : I.alt);
    float cv = 0.0f, ev = 0.0f;
    if (r < uint64_t(I.n)) {
      const uint64_t ctr = (ia << 40) | (q << 24) | r;
      const uint64_t gm = 0x9E3779B97F4A7C15ull;
      const uint64_t w1 = bmix64(I.seed + (2 * ctr + 1) * gm);
      const uint64_t w2 = bmix64(I.seed + (2 * ctr + 2) * gm);
      const double u1 = double(w1 >> 11) * 0x1.0p-53;
      const double u2 = double(w2 >> 11) * 0x1.0p-53;
      cv = float(std * (sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586 * u2)));
      ev = 1.0f;
    }
    I.c[li] = cv;
    I.c2[li] = 0.0f;
    I.e[li] = ev;
  }
}

// ---------------------------------------------------------------------------
// The Euler step over all row tiles of all instances
// ---------------------------------------------------------------------------
//
// A workgroup owns 16 * RB rows (RB panels) of one instance for all its
// replicas (16 * QB columns of X) and its NW wavefronts split the columns of
// J into NW contiguous ranges of 32-column chunks (boundaries fixed by the
// instance's ld).  Each wavefront keeps D chunks of operands in flight, sums
// its range on the matrix cores, and the NW partial sums are added in LDS in
// wavefront order before the fused Euler epilogue.  Every output row's
// arithmetic is therefore a function of its instance only.
//
// Operands of one chunk for lane (li = lane % 16, lk = lane / 16):
//   A: J[16 p + li][32 c + 8 lk + t], t < 8, from the panel block (p, c);
//   B: X[q = 16 qb + li][32 c + 8 lk + t]: amplitudes (continuous field) or
//      bits 8 lk + t of the support word (binarised field).

// Loads through the global address space: pointers read from the instance
// table are generic, and generic (flat) loads would also hold the LDS/scalar
// counter, so a wait for one chunk would drain every chunk in flight.
template <typename T>
__device__ inline T gload(const void* p) {
  return *(const __attribute__((address_space(1))) T*)(p);
}

typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));

// Non-temporal variant for the couplings stream, which no other workgroup
// reads in the same step: measured faster for BF16 and for FP32 (batched
// form: 599 against 638 us per Euler step; within 2% either way for one
// instance with 64 replicas) and slower for FP8, which keeps plain loads.
template <typename T>
__device__ inline T gload_nt(const void* p) {
  return __builtin_nontemporal_load((const __attribute__((address_space(1))) T*)(p));
}

template <typename JT> struct ARaw;
template <> struct ARaw<float> { v4f v0, v1; };
template <> struct ARaw<__hip_bfloat16> { v4u v; };
template <> struct ARaw<__hip_fp8_e4m3> { v2u v; };

template <int FIELD> struct BRaw { v4f v0, v1; };
template <> struct BRaw<kBN> { uint32_t v; };

template <typename JT, int FIELD, int RB, int QB>
struct Stage {
  ARaw<JT> a[RB];
  BRaw<FIELD> b[QB];
};

// Chunks in flight per wavefront: about 96 registers of operands, 2 to 12.
constexpr int pipe_depth(int jsize, int field, int RB, int QB) {
  const int v = RB * (jsize == 4 ? 8 : (jsize == 2 ? 4 : 2)) + QB * (field == kBN ? 1 : 8);
  const int d = 96 / v;
  return d < 2 ? 2 : (d > 12 ? 12 : d);
}

// 8 support bits (bits pos .. pos + 7 of the word; bit pos + t is column
// 8 lk + t) -> 8 bf16 values 0 / 1.  Each nibble is spread to the low bit of
// four bytes by one multiply (the four shifted copies occupy disjoint bit
// ranges, so nothing carries), which makes e4m3 codes 0 / 0x01 (2^-9); the
// hardware pair conversion scales them by 2^9 to bf16 0 / 1, exactly.
__device__ inline v8bf bits_to_bf16(uint32_t word, int pos) {
  const uint32_t lo = (((word >> pos) & 0xFu) * 0x00204081u) & 0x01010101u;
  const uint32_t hi = (((word >> (pos + 4)) & 0xFu) * 0x00204081u) & 0x01010101u;
  v4u w;
  w.x = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(int(lo), 512.0f, false));
  w.y = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(int(lo), 512.0f, true));
  w.z = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(int(hi), 512.0f, false));
  w.w = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(int(hi), 512.0f, true));
  return __builtin_bit_cast(v8bf, w);
}

// 8 e4m3 codes -> 8 bf16 with the hardware pair conversion at scale 1
// (exact: every e4m3 value, subnormals included, is a bf16 value).
__device__ inline v8bf fp8_to_bf16(v2u v) {
  v4u w;
  w.x = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(int(v.x), 1.0f, false));
  w.y = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(int(v.x), 1.0f, true));
  w.z = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(int(v.y), 1.0f, false));
  w.w = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(int(v.y), 1.0f, true));
  return __builtin_bit_cast(v8bf, w);
}

// Wavefronts per workgroup: eight for FP8 couplings (their fastest tile at
// the MRI shape, 64 rows, leaves one workgroup per CU: 47.4 against 49.9 us
// per step with four), four for the others (eight measured slower for FP32).
template <typename JT>
constexpr int step_waves() {
  return sizeof(JT) == 1 ? 8 : 4;
}

template <typename JT, int FIELD, int QB, int RB>
__global__ void __launch_bounds__(64 * step_waves<JT>())
bstep_kernel(const BTile* __restrict__ tiles, const BInst* __restrict__ insts, BStepArgs a, int k,
             const double* __restrict__ etap) {
  constexpr bool kF32 = sizeof(JT) == 4;
  constexpr int NW = step_waves<JT>();
  constexpr int D = pipe_depth(int(sizeof(JT)), FIELD, RB, QB);
  static_assert(RB * QB * NW <= 128, "partial sums must fit in 128 KB of LDS");
  __shared__ v4f red[NW][RB * QB][64];
  const BTile tl = tiles[blockIdx.x];
  if (tl.inst < 0) return;
  const BInst I = insts[tl.inst];
  const int n = I.n, ld = I.ld, P = a.P, nch = ld >> 5;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int p0 = tl.row0 >> 4;
  const bool last = (k == a.n_steps);
  const float st = float(sqrt(a.tau));
  const float* cin = (k & 1) ? I.c2 : I.c;
  const uint32_t* xin = (k & 1) ? I.xb2 : I.xb;
  const JT* J = static_cast<const JT*>(I.J);
  constexpr int kNwLog = NW == 8 ? 3 : 2;
  static_assert(NW == (1 << kNwLog), "four or eight wavefronts");
  const int c0 = (w * nch) >> kNwLog, c1 = ((w + 1) * nch) >> kNwLog;
  const int lane_off = kF32 ? (li * 4 + lk) * 4 : (li * 4 + lk) * 8;

  // Rows of panels past the instance and replicas past P read valid
  // addresses of panel p0 / replica 0 instead; their sums are never used.
  // The tile's panels lie in one panel group (RB divides kPanelGroup and p0
  // is a multiple of RB): chunk c of panel p0 + rb is block gs c + rb of the
  // group, after the group's base.
  static_assert(kPanelGroup % RB == 0, "row tiles within one panel group");
  const int np = (n + 15) / 16;
  const int cstride = jpanel_group_size(p0, np) * 512;
  const JT* gbase = J + jpanel_group_base(p0, nch);
  int poff[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int pp = (p0 + rb) * 16 < n ? p0 + rb : p0;
    poff[rb] = (pp % kPanelGroup) * 512 + lane_off;
  }
  bool qon[QB];
  const float* cbase[QB];
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    const int q = qb * 16 + li;
    qon[qb] = q < P;
    cbase[qb] = cin + size_t(q < P ? q : 0) * ld + 8 * lk;
  }
  // support words of this lane's 16 QB-replica block row: adjacent, one load per chunk
  const uint32_t* xbase = xin + size_t(li) * QB;

  v4f acc[RB][QB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) acc[rb][qb] = v4f{0.f, 0.f, 0.f, 0.f};

  using St = Stage<JT, FIELD, RB, QB>;
  auto load = [&](int c, St& S) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const JT* src = gbase + (size_t(c * cstride) + poff[rb]);
      if constexpr (kF32) {
        S.a[rb].v0 = gload_nt<v4f>(src);
        S.a[rb].v1 = gload_nt<v4f>(src + 256);
      } else if constexpr (sizeof(JT) == 2) {
        S.a[rb].v = gload_nt<v4u>(src);
      } else {
        S.a[rb].v = gload<v2u>(src);
      }
    }
    if constexpr (FIELD == kBN) {
      const uint32_t* xw = xbase + size_t(c) * (16 * QB);
      if constexpr (QB == 1) {
        S.b[0].v = gload<uint32_t>(xw);
      } else if constexpr (QB == 2) {
        const v2u w2 = gload<v2u>(xw);
        S.b[0].v = w2.x;
        S.b[1].v = w2.y;
      } else {
        const v4u w4 = gload<v4u>(xw);
        S.b[0].v = w4.x;
        S.b[1].v = w4.y;
        S.b[2].v = w4.z;
        S.b[3].v = w4.w;
      }
    }
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
      if constexpr (FIELD == kBN) {
      } else {
        const float* cs = cbase[qb] + c * 32;
        S.b[qb].v0 = gload<v4f>(cs);
        S.b[qb].v1 = gload<v4f>(cs + 4);
      }
    }
  };
  auto compute = [&](const St& S) {
    if constexpr (kF32) {
#pragma unroll
      for (int qb = 0; qb < QB; ++qb) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          float x[4];
          if constexpr (FIELD == kBN) {
            const uint32_t byte = (S.b[qb].v >> (8 * lk)) & 0xFFu;
#pragma unroll
            for (int u = 0; u < 4; ++u) x[u] = float((byte >> (4 * h + u)) & 1u);
          } else {
            const v4f c4 = h ? S.b[qb].v1 : S.b[qb].v0;
            const bool on = qon[qb];
            x[0] = on ? xf<FIELD>(c4.x, st, last) : 0.f;
            x[1] = on ? xf<FIELD>(c4.y, st, last) : 0.f;
            x[2] = on ? xf<FIELD>(c4.z, st, last) : 0.f;
            x[3] = on ? xf<FIELD>(c4.w, st, last) : 0.f;
          }
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            const v4f a4 = h ? S.a[rb].v1 : S.a[rb].v0;
            acc[rb][qb] = mfma_f32(a4.x, x[0], acc[rb][qb]);
            acc[rb][qb] = mfma_f32(a4.y, x[1], acc[rb][qb]);
            acc[rb][qb] = mfma_f32(a4.z, x[2], acc[rb][qb]);
            acc[rb][qb] = mfma_f32(a4.w, x[3], acc[rb][qb]);
          }
        }
      }
    } else {
      v8bf av[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        if constexpr (sizeof(JT) == 2) av[rb] = __builtin_bit_cast(v8bf, S.a[rb].v);
        else av[rb] = fp8_to_bf16(S.a[rb].v);
      }
#pragma unroll
      for (int qb = 0; qb < QB; ++qb) {
        if constexpr (FIELD == kBN) {
          const v8bf bx = bits_to_bf16(S.b[qb].v, 8 * lk);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) acc[rb][qb] = mfma_bf16(av[rb], bx, acc[rb][qb]);
        } else {
          const float cc[8] = {S.b[qb].v0.x, S.b[qb].v0.y, S.b[qb].v0.z, S.b[qb].v0.w,
                               S.b[qb].v1.x, S.b[qb].v1.y, S.b[qb].v1.z, S.b[qb].v1.w};
          v8bf bh, bl;
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const float xv = qon[qb] ? xf<FIELD>(cc[t], st, last) : 0.f;
            const __bf16 hv = __bf16(xv);
            bh[t] = hv;
            bl[t] = __bf16(xv - float(hv));
          }
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            acc[rb][qb] = mfma_bf16(av[rb], bh, acc[rb][qb]);
            if (!last) acc[rb][qb] = mfma_bf16(av[rb], bl, acc[rb][qb]);
          }
        }
      }
    }
  };

  // D chunks in flight: a branch-free steady state, then the last 2 D - 1 at most
  St buf[D];
  if (c1 - c0 >= D) {
#pragma unroll
    for (int s = 0; s < D; ++s) load(c0 + s, buf[s]);
    int c = c0;
    for (; c + 2 * D <= c1; c += D) {
#pragma unroll
      for (int s = 0; s < D; ++s) {
        compute(buf[s]);
        load(c + D + s, buf[s]);
      }
    }
    const int rem = c1 - c - D;
#pragma unroll
    for (int s = 0; s < D; ++s) {
      compute(buf[s]);
      if (s < rem) load(c + D + s, buf[s]);
    }
#pragma unroll
    for (int s = 0; s < D; ++s)
      if (s < rem) compute(buf[s]);
  } else {
    for (int c = c0; c < c1; ++c) {
      load(c, buf[0]);
      compute(buf[0]);
    }
  }

#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) red[w][rb * QB + qb][lane] = acc[rb][qb];
  __syncthreads();

  // Epilogue: lane holds rows 16 (p0 + rb) + 4 lk + v (v < 4) of replica 16 qb + li.
  const double eta = etap ? *etap : I.eta;
  const float theta = float(eta * eta * sqrt(a.tau) * 0.25);
  const float half_st = float(0.5 * sqrt(a.tau));
  const double lam = 0.5 * eta * eta;
  const float lin = float((a.p_thr - a.d) + 2.0 * a.d / (1.0 + exp(-(double(k) * a.dt - a.t_c) / a.t_w)) -
                          1.0 - (a.linear_j ? a.j : 0.0));
  const float jj = float(a.j), KK = float(a.K), beta = float(a.beta), tau = float(a.tau), dt = float(a.dt);
  const float* z = I.z;
  const float* rs = I.rs;
  float* e = I.e;
  float* cout = (k & 1) ? I.c : I.c2;
  uint16_t* xout = reinterpret_cast<uint16_t*>((k & 1) ? I.xb : I.xb2);
  int bits = 0;
  for (int b = w; b < RB * QB; b += NW) {
    const int rb = b / QB, qb = b - (b / QB) * QB;
    v4f sacc = red[0][b][lane];
    sacc += red[1][b][lane];
    sacc += red[2][b][lane];
    sacc += red[3][b][lane];
    if constexpr (NW == 8) {
      sacc += red[4][b][lane];
      sacc += red[5][b][lane];
      sacc += red[6][b][lane];
      sacc += red[7][b][lane];
    }
    const int q = qb * 16 + li;
    const int r0 = (p0 + rb) * 16 + 4 * lk;
    uint32_t nib = 0;
    if (q < P && r0 < n) {
      const size_t off = size_t(q) * ld + r0;
      float4 c4 = *reinterpret_cast<const float4*>(cin + off);
      float4 e4 = *reinterpret_cast<const float4*>(e + off);
      float cvs[4] = {c4.x, c4.y, c4.z, c4.w};
      float evs[4] = {e4.x, e4.y, e4.z, e4.w};
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + v;
        if (r >= n) continue;
        const float y = sacc[v] * rs[r];
        float cv = cvs[v], ev = evs[v];
        if (!last) {
          const float phi = (FIELD == kCN) ? (y + half_st * z[r]) : (half_st * (y + z[r]));
          const float inj = jj * ev * (phi - theta);
          const float c2 = cv * cv;
          const float dc = (lin - c2) * cv + KK * inj;
          const float de = -beta * (c2 - tau) * ev;
          cvs[v] = cv + dt * dc;
          evs[v] = ev + dt * de;
          nib |= (cvs[v] > 0.0f ? 1u : 0u) << v;
          if (k < a.trace_steps) {
            a.trace[(size_t(2 * k) * P + q) * n + r] = cvs[v];
            a.trace[(size_t(2 * k + 1) * P + q) * n + r] = evs[v];
          }
        } else {
          const bool sg = cv > 0.0f;
          I.hpart[size_t(q) * n + r] = sg ? (-0.5 * double(y) - double(z[r]) + lam) : 0.0;
          I.sig_all[size_t(q) * n + r] = sg ? 1 : 0;
          if (!(isfinite(cv) && isfinite(ev))) bits |= L0CIM_ST_NONFINITE;
          else if (fabsf(cv) > 1e3f) bits |= L0CIM_ST_BLOWUP;
        }
      }
      if (!last) {
        *reinterpret_cast<float4*>(cout + off) = make_float4(cvs[0], cvs[1], cvs[2], cvs[3]);
        *reinterpret_cast<float4*>(e + off) = make_float4(evs[0], evs[1], evs[2], evs[3]);
      }
    }
    if constexpr (FIELD == kBN) {
      // support bits of the panel for the next step: 4 rows per lane, 16 per replica
      uint32_t word = nib << (4 * lk);
      word |= uint32_t(__shfl_xor(int(word), 16, kWave));
      word |= uint32_t(__shfl_xor(int(word), 32, kWave));
      const int pp = p0 + rb;
      if (!last && lk == 0 && q < P && pp * 16 < n)
        xout[2 * ((size_t(pp >> 1) * 16 + li) * QB + qb) + (pp & 1)] = uint16_t(word);
    }
  }
  if (last && bits) raise_status(I.status, bits);
}

// Support bits of the initial amplitudes (binarised field), in the chunk
// block layout: the word of (replica q, chunk c) holds c_q[32 c + t] > 0 in
// bit t; the other buffer starts at zero.  With no prefix table the launch
// covers instance 0 alone.
__global__ void __launch_bounds__(256)
bbits_kernel(const BInst* __restrict__ insts, const int64_t* __restrict__ st_prefix, int count, int QB,
             int64_t total_words) {
  for (int64_t g = blockIdx.x * int64_t(256) + threadIdx.x; g < total_words; g += int64_t(gridDim.x) * 256) {
    const int64_t e0 = g * 32;
    const int k = st_prefix ? find_inst(st_prefix, count, e0) : 0;
    const BInst I = insts[k];
    const int64_t li = e0 - (st_prefix ? st_prefix[k] : 0);
    const int64_t q = li / I.ld, r0 = li - q * I.ld;
    const float* c = I.c + q * I.ld + r0;
    uint32_t wv = 0;
    for (int t = 0; t < 32; ++t) wv |= (c[t] > 0.0f ? 1u : 0u) << t;
    const int64_t wi = ((r0 >> 5) * 16 + (q & 15)) * QB + (q >> 4);
    I.xb[wi] = wv;
    I.xb2[wi] = 0u;
  }
}

// Per instance: H_q = sum of the per-spin eq. 4 terms (256 contiguous runs
// of spins summed in order, then a fixed tree, so the result depends only on
// the instance), lowest-energy replica (first on ties, NaN last), copy of its
// support.
__global__ void __launch_bounds__(256)
bselect_kernel(const BInst* __restrict__ insts, int P) {
  __shared__ double part[256];
  __shared__ double hq[64];
  __shared__ int qs;
  const BInst I = insts[blockIdx.x];
  const int t = threadIdx.x, n = I.n;
  const int chunk = (n + 255) / 256;
  const int lo = min(n, t * chunk), hi = min(n, lo + chunk);
  for (int q = 0; q < P; ++q) {
    const double* hr = I.hpart + size_t(q) * n;
    double h = 0.0;
    for (int r = lo; r < hi; ++r) h += hr[r];
    part[t] = h;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w) part[t] += part[t + w];
      __syncthreads();
    }
    if (t == 0) hq[q] = part[0];
    __syncthreads();
  }
  if (t == 0) {
    int best = 0;
    double hb = hq[0];
    for (int q = 1; q < P; ++q) {
      const double h = hq[q];
      if (h < hb || (isnan(hb) && !isnan(h))) {
        hb = h;
        best = q;
      }
    }
    qs = best;
    I.st->selected_replica = best;
    I.st->H = hb;
  }
  __syncthreads();
  const uint8_t* src = I.sig_all + size_t(qs) * n;
  for (int i = t; i < n; i += 256) I.sig[i] = src[i];
}

// ---------------------------------------------------------------------------
// CDP for every instance (synchronous damped Jacobi over all r, the same
// update as the single-instance path).  Only the support's R enter the sums,
// so the sweeps run over the support rows and every other R follows at the
// end from the affine form R_r(K) = f R_r(0) + (1 - f) b_r / G_rr -
// (dtc / G_rr) G_rS V, f = (1 - dtc)^K, V = sum_k (1 - dtc)^(K-1-k) R_S(k)
// (the K sweeps unrolled).  Per alternation: a preparation kernel per
// instance (support list, its inverse, R on the support), one pass that
// gathers G's support columns into a compact block, one launch per sweep, one
// final pass; all over the row tiles of every instance (a tile's rows double
// as support indices in the sweeps).  Each sum runs over the support in index
// order split by lane, so the result depends only on the instance.
// Per-instance scratch (words of 4 bytes, ld = padded row length):
//   [0, ld) V                       [ld, 3 ld) R on the support, two parities
//   [3 ld, 4 ld) support list       [4 ld, 5 ld) position in the list or -1
//   [5 ld, 5 ld + 64) counters      [5 ld + 64, 5 ld + 192) 64 FP64 partial sums
// ---------------------------------------------------------------------------
constexpr int kObjChunks = 64;

__global__ void __launch_bounds__(256)
bjac_prep_kernel(const BInst* __restrict__ insts) {
  __shared__ int scan_sh[256 / kWave + 1];
  const BInst I = insts[blockIdx.x];
  const int n = I.n, ld = I.ld, tid = threadIdx.x;
  float* V = I.jw;
  float* sR0 = I.jw + ld;
  int* S = reinterpret_cast<int*>(I.jw + 3 * ld);
  int* pos = reinterpret_cast<int*>(I.jw + 4 * ld);
  int* misc = reinterpret_cast<int*>(I.jw + 5 * ld);
  const int chunk = (n + 255) / 256;
  const int lo = min(n, tid * chunk), hi = min(n, lo + chunk);
  int c = 0;
  for (int i = lo; i < hi; ++i) c += I.sig[i] ? 1 : 0;
  int ks = 0;
  int at = block_exclusive_scan<256>(c, scan_sh, &ks);
  if (tid == 0) misc[0] = ks;
  int bits = 0;
  for (int i = lo; i < hi; ++i) {
    const float d = I.G[size_t(i) * ld + i];
    const bool tiny = !(d >= 1e-12f);
    if (tiny) bits |= L0CIM_ST_TINY_DIAG;
    const float r = tiny ? 0.0f : I.R[i];
    I.R[i] = r;
    if (I.sig[i]) {
      S[at] = i;
      sR0[at] = r;
      V[at] = 0.0f;
      pos[i] = at++;
    } else {
      pos[i] = -1;
    }
  }
  if (bits) raise_status(I.status, bits);
}

// Threads of the batched Jacobi kernels: a wavefront per row, sixteen rows of
// a tile at a time (the step tiles hold 16 to 128 rows).
constexpr int kJacThreads = 1024;
constexpr int kJacWaves = kJacThreads / kWave;

// Gc[r][s] = G[r][S[s]] for the rows of one tile (a wavefront per row).
__global__ void __launch_bounds__(kJacThreads)
bjac_compact_kernel(const BTile* __restrict__ tiles, const BInst* __restrict__ insts, int rows_per_tile) {
  const BTile tl = tiles[blockIdx.x];
  if (tl.inst < 0) return;
  const BInst I = insts[tl.inst];
  const int ld = I.ld;
  const int* S = reinterpret_cast<const int*>(I.jw + 3 * ld);
  const int ks = reinterpret_cast<const int*>(I.jw + 5 * ld)[0];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r1 = min(I.n, tl.row0 + rows_per_tile);
  for (int r = tl.row0 + w; r < r1; r += kJacWaves) {
    const float* g = I.G + size_t(r) * ld;
    float* gc = I.Gc + size_t(r) * ks;
    for (int s = lane; s < ks; s += kWave) gc[s] = g[S[s]];
  }
}

// One synchronous sweep over the support rows (support indices of the tile).
__global__ void __launch_bounds__(kJacThreads)
bjac_sweep_kernel(const BTile* __restrict__ tiles, const BInst* __restrict__ insts, int rows_per_tile, float dtc,
                  int it) {
  const BTile tl = tiles[blockIdx.x];
  if (tl.inst < 0) return;
  const BInst I = insts[tl.inst];
  const int ld = I.ld;
  const int ks = reinterpret_cast<const int*>(I.jw + 5 * ld)[0];
  if (tl.row0 >= ks) return;
  float* V = I.jw;
  const float* sRi = I.jw + ld + (it & 1) * ld;
  float* sRo = I.jw + ld + ((it + 1) & 1) * ld;
  const int* S = reinterpret_cast<const int*>(I.jw + 3 * ld);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i1 = min(ks, tl.row0 + rows_per_tile);
  for (int i = tl.row0 + w; i < i1; i += kJacWaves) {
    const int r = S[i];
    const float* gc = I.Gc + size_t(r) * ks;
    float acc = 0.0f;
    for (int s = lane; s < ks; s += kWave)
      if (s != i) acc += gc[s] * sRi[s];
    acc = wave_sum(acc);
    if (lane == 0) {
      const float d = I.G[size_t(r) * ld + r];
      const bool tiny = !(d >= 1e-12f);
      const float Rv = sRi[i];
      V[i] = (1.0f - dtc) * V[i] + Rv;
      sRo[i] = tiny ? 0.0f : Rv + dtc * ((I.b[r] - acc) / d - Rv);
    }
  }
}

// Every R after K sweeps: the support's from the last sweep, the others from
// the affine form.
__global__ void __launch_bounds__(kJacThreads)
bjac_final_kernel(const BTile* __restrict__ tiles, const BInst* __restrict__ insts, int rows_per_tile, float dtc,
                  int iters) {
  const BTile tl = tiles[blockIdx.x];
  if (tl.inst < 0) return;
  const BInst I = insts[tl.inst];
  const int ld = I.ld;
  const int ks = reinterpret_cast<const int*>(I.jw + 5 * ld)[0];
  const float* V = I.jw;
  const float* sRK = I.jw + ld + (iters & 1) * ld;
  const int* pos = reinterpret_cast<const int*>(I.jw + 4 * ld);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r1 = min(I.n, tl.row0 + rows_per_tile);
  float f = 1.0f;
  for (int k = 0; k < iters; ++k) f *= (1.0f - dtc);
  for (int r = tl.row0 + w; r < r1; r += kJacWaves) {
    const int pr = pos[r];
    if (pr >= 0) {
      if (lane == 0) I.R[r] = sRK[pr];
      continue;
    }
    const float* gc = I.Gc + size_t(r) * ks;
    float acc = 0.0f;
    for (int s = lane; s < ks; s += kWave) acc += gc[s] * V[s];
    acc = wave_sum(acc);
    if (lane == 0) {
      const float d = I.G[size_t(r) * ld + r];
      const bool tiny = !(d >= 1e-12f);
      I.R[r] = tiny ? 0.0f : f * I.R[r] + (1.0f - f) * (I.b[r] / d) - (dtc / d) * acc;
    }
  }
}

// eq. 3 objective and the per-instance report.  Phase 1: FP64 partial sums
// of squared residuals over fixed row chunks of A; phase 2: their ordered sum.
__global__ void __launch_bounds__(256)
bobj_partial_kernel(const BInst* __restrict__ insts) {
  __shared__ double wpart[4];
  const int k = blockIdx.x / kObjChunks, ch = blockIdx.x % kObjChunks;
  const BInst I = insts[k];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double r2 = 0.0;
  for (int row = ch * 4 + w; row < I.m; row += kObjChunks * 4) {
    double acc = 0.0;
    const float* a = I.A + size_t(row) * I.lda;
    for (int j = lane; j < I.n; j += kWave)
      if (I.sig[j]) acc += double(a[j]) * double(I.R[j]);
    acc = wave_sum(acc);
    const double res = double(I.y[row]) - acc;
    r2 += res * res;
  }
  if (lane == 0) wpart[w] = r2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double* part = reinterpret_cast<double*>(I.jw + 5 * I.ld + 64);
    part[ch] = ((wpart[0] + wpart[1]) + wpart[2]) + wpart[3];
  }
}

__global__ void __launch_bounds__(256)
bobj_final_kernel(const BInst* __restrict__ insts, double lam, int64_t steps_per_alt, int n_outer, int P) {
  __shared__ int scan_sh[256 / kWave + 1];
  const BInst I = insts[blockIdx.x];
  int c = 0;
  for (int j = threadIdx.x; j < I.n; j += 256) c += I.sig[j] ? 1 : 0;
  int s = 0;
  (void)block_exclusive_scan<256>(c, scan_sh, &s);
  if (threadIdx.x == 0) {
    const double* part = reinterpret_cast<const double*>(I.jw + 5 * I.ld + 64);
    double rr = 0.0;
    for (int ch = 0; ch < kObjChunks; ++ch) rr += part[ch];
    const bool own = lam < 0.0;
    const double lm = own ? 0.5 * I.eta * I.eta : lam;
    const int no = own ? I.alt + 1 : n_outer;
    I.st->support_size = s;
    I.st->E = 0.5 * rr + lm * double(s);
    I.st->spin_steps = int64_t(I.n) * P * steps_per_alt * no;
    I.st->n_outer_done = no;
  }
}

__global__ void bstats_init_kernel(const BInst* __restrict__ insts, int count) {
  int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  l0cim_stats* st = insts[i].st - i;
  st[i].status_bits = 0;
  st[i].selected_replica = 0;
  st[i].support_size = 0;
  st[i].n_outer_done = 0;
  st[i].H = 0.0;
  st[i].E = 0.0;
  st[i].spin_steps = 0;
}

__global__ void bfill_kernel(float* p, int64_t count) {
  for (int64_t i = blockIdx.x * int64_t(256) + threadIdx.x; i < count; i += int64_t(gridDim.x) * 256) p[i] = 0.0f;
}

__global__ void bset_scalar_kernel(double* p, double v) { *p = v; }

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

template <typename JT, int FIELD, int QB, int RB>
static const void* step_kernel_ptr() {
  return reinterpret_cast<const void*>(bstep_kernel<JT, FIELD, QB, RB>);
}

template <typename JT, int FIELD>
static const void* step_kernel_q(int qb, int rb) {
  if (qb == 1) {
    if (rb == 1) return step_kernel_ptr<JT, FIELD, 1, 1>();
    if (rb == 2) return step_kernel_ptr<JT, FIELD, 1, 2>();
    if (rb == 4) return step_kernel_ptr<JT, FIELD, 1, 4>();
    if (rb == 8) return step_kernel_ptr<JT, FIELD, 1, 8>();
  } else if (qb == 2) {
    if (rb == 1) return step_kernel_ptr<JT, FIELD, 2, 1>();
    if (rb == 2) return step_kernel_ptr<JT, FIELD, 2, 2>();
    if (rb == 4) return step_kernel_ptr<JT, FIELD, 2, 4>();
    if (rb == 8) return step_kernel_ptr<JT, FIELD, 2, 8>();
  } else if (qb == 4) {
    if (rb == 1) return step_kernel_ptr<JT, FIELD, 4, 1>();
    if (rb == 2) return step_kernel_ptr<JT, FIELD, 4, 2>();
    if (rb == 4) return step_kernel_ptr<JT, FIELD, 4, 4>();
  }
  return nullptr;
}

StepKernel batch_step_kernel(l0cim_dtype jdt, int field, int qb, int rb) {
  if (jdt == L0CIM_F32)
    return {field == L0CIM_FIELD_BN ? step_kernel_q<float, kBN>(qb, rb) : step_kernel_q<float, kCN>(qb, rb),
            64 * step_waves<float>()};
  if (jdt == L0CIM_BF16)
    return {field == L0CIM_FIELD_BN ? step_kernel_q<__hip_bfloat16, kBN>(qb, rb)
                                    : step_kernel_q<__hip_bfloat16, kCN>(qb, rb),
            64 * step_waves<__hip_bfloat16>()};
  if (jdt == L0CIM_FP8E4M3)
    return {field == L0CIM_FIELD_BN ? step_kernel_q<__hip_fp8_e4m3, kBN>(qb, rb)
                                    : step_kernel_q<__hip_fp8_e4m3, kCN>(qb, rb),
            64 * step_waves<__hip_fp8_e4m3>()};
  return {nullptr, 0};
}

l0cim_status enqueue_bsteps(const BatchDev& d, StepKernel sk, const BStepArgs& a, int ntiles, int k0, int k1,
                            hipStream_t s) {
  for (int k = k0; k <= k1; ++k) {
    const BTile* tiles = d.tiles;
    const BInst* insts = d.insts;
    BStepArgs aa = a;
    int kk = k;
    const double* eta = d.eta;
    void* args[] = {&tiles, &insts, &aa, &kk, &eta};
    L0_HIP(hipLaunchKernel(sk.fn, dim3(ntiles), dim3(sk.threads), args, 0, s));
  }
  return L0CIM_OK;
}

l0cim_status launch_bcouplings(const BatchDev& d, l0cim_dtype jdt, int64_t total_rows, hipStream_t s) {
  if (jdt == L0CIM_F32)
    hipLaunchKernelGGL(bcouplings_kernel<float>, dim3(unsigned(total_rows)), dim3(256), 0, s, d.insts,
                       d.row_prefix, d.count);
  else if (jdt == L0CIM_BF16)
    hipLaunchKernelGGL(bcouplings_kernel<__hip_bfloat16>, dim3(unsigned(total_rows)), dim3(256), 0, s,
                       d.insts, d.row_prefix, d.count);
  else
    hipLaunchKernelGGL(bcouplings_kernel<__hip_fp8_e4m3>, dim3(unsigned(total_rows)), dim3(256), 0, s,
                       d.insts, d.row_prefix, d.count);
  L0_LAUNCHED("bcouplings_kernel");
  return L0CIM_OK;
}

l0cim_status launch_binit(const BatchDev& d, int P, int alt, double std, int64_t total_state, hipStream_t s) {
  int blocks = int((total_state + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(binit_kernel, dim3(blocks), dim3(256), 0, s, d.insts, d.st_prefix, d.count, P, alt, std);
  L0_LAUNCHED("binit_kernel");
  return L0CIM_OK;
}

l0cim_status launch_bbits(const BatchDev& d, int QB, int64_t total_words, hipStream_t s) {
  int blocks = int((total_words + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(bbits_kernel, dim3(blocks), dim3(256), 0, s, d.insts, d.st_prefix, d.count, QB, total_words);
  L0_LAUNCHED("bbits_kernel");
  return L0CIM_OK;
}

l0cim_status launch_bselect(const BatchDev& d, int P, hipStream_t s) {
  hipLaunchKernelGGL(bselect_kernel, dim3(d.count), dim3(256), 0, s, d.insts, P);
  L0_LAUNCHED("bselect_kernel");
  return L0CIM_OK;
}

l0cim_status launch_bjacobi(const BatchDev& d, int ntiles, int rows_per_tile, double dtc, int iters,
                           hipStream_t s) {
  hipLaunchKernelGGL(bjac_prep_kernel, dim3(d.count), dim3(256), 0, s, d.insts);
  L0_LAUNCHED("bjac_prep_kernel");
  if (iters <= 0) return L0CIM_OK;
  hipLaunchKernelGGL(bjac_compact_kernel, dim3(ntiles), dim3(kJacThreads), 0, s, d.tiles, d.insts, rows_per_tile);
  L0_LAUNCHED("bjac_compact_kernel");
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(bjac_sweep_kernel, dim3(ntiles), dim3(kJacThreads), 0, s, d.tiles, d.insts, rows_per_tile,
                       float(dtc), it);
    L0_LAUNCHED("bjac_sweep_kernel");
  }
  hipLaunchKernelGGL(bjac_final_kernel, dim3(ntiles), dim3(kJacThreads), 0, s, d.tiles, d.insts, rows_per_tile, float(dtc),
                     iters);
  L0_LAUNCHED("bjac_final_kernel");
  return L0CIM_OK;
}

l0cim_status launch_bobjective(const BatchDev& d, double lam, int64_t steps_per_alt, int n_outer, int P,
                               hipStream_t s) {
  hipLaunchKernelGGL(bobj_partial_kernel, dim3(d.count * kObjChunks), dim3(256), 0, s, d.insts);
  L0_LAUNCHED("bobj_partial_kernel");
  hipLaunchKernelGGL(bobj_final_kernel, dim3(d.count), dim3(256), 0, s, d.insts, lam, steps_per_alt, n_outer, P);
  L0_LAUNCHED("bobj_final_kernel");
  return L0CIM_OK;
}

l0cim_status launch_bstats_init(const BatchDev& d, hipStream_t s) {
  hipLaunchKernelGGL(bstats_init_kernel, dim3((d.count + 255) / 256), dim3(256), 0, s, d.insts, d.count);
  L0_LAUNCHED("bstats_init_kernel");
  return L0CIM_OK;
}

l0cim_status launch_bfill(float* p, int64_t count, hipStream_t s) {
  int blocks = int((count + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(bfill_kernel, dim3(blocks), dim3(256), 0, s, p, count);
  L0_LAUNCHED("bfill_kernel");
  return L0CIM_OK;
}

l0cim_status launch_bset_scalar(double* p, double v, hipStream_t s) {
  hipLaunchKernelGGL(bset_scalar_kernel, dim3(1), dim3(1), 0, s, p, v);
  L0_LAUNCHED("bset_scalar_kernel");
  return L0CIM_OK;
}

}  // namespace l0
