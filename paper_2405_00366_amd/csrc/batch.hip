// Batched form: many instances of uneven size, each with P replicas, solved
// together (Algorithm 1 for every instance in lock step).  With several
// replicas the local-field contraction of eq. 15 / 16 is a dense product
// Y = J X (N x N times N x P) per instance, done on the matrix cores:
//   * FP32 couplings: v_mfma_f32_16x16x4_f32,
//   * BF16 couplings: v_mfma_f32_16x16x32_bf16 (binarised field exact;
//     continuous field as a bf16 hi + lo pair of the operand),
//   * FP8 e4m3 couplings: v_mfma_f32_16x16x32_fp8_fp8 for the binarised field
//     (sigma in {0,1} is exact in fp8); continuous field through the bf16 path
//     (e4m3 values are exact in bf16),
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

// FP8 couplings are widened to bf16 in registers (every e4m3 value is exact
// in bf16) and multiplied on the bf16 matrix cores, so the products and their
// FP32 sums are the ones the dequantised definition gives; the bytes read from
// HBM are still one per coupling.  The direct fp8 x fp8 instruction path below
// is kept switched off: its trajectories drifted from the dequantised
// definition by about 5e-3 after a full run, while a single-instruction check
// on normal e4m3 values summed exactly, so the cause is not pinned down.
constexpr bool kFp8Matrix = false;

__device__ inline v4f mfma_f32(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline v4f mfma_bf16(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline v4f mfma_fp8(long a, long b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
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

// One workgroup per (instance, row): J row (zero diagonal, zero padding), z,
// and for narrow storage the row scale amax / Q_max and RNE(J / scale).
template <typename JT>
__global__ void __launch_bounds__(256)
bcouplings_kernel(const BInst* __restrict__ insts, const int64_t* __restrict__ row_prefix, int count) {
  __shared__ float red[256];
  const int k = find_inst(row_prefix, count, blockIdx.x);
  const BInst I = insts[k];
  const int r = int(blockIdx.x - row_prefix[k]);
  const int n = I.n, ld = I.ld;
  const float* G = I.G + size_t(r) * ld;
  const float* R = I.R;
  const float Rr = R[r];
  JT* J = static_cast<JT*>(I.J) + size_t(r) * I.ldj;
  if constexpr (sizeof(JT) == 4) {
    for (int j = threadIdx.x; j < ld; j += 256)
      J[j] = (j < n && j != r) ? -(G[j] * (Rr * R[j])) : 0.0f;
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
      if constexpr (sizeof(JT) == 2) J[j] = __float2bfloat16(v);
      else J[j] = __hip_fp8_e4m3(fminf(fmaxf(v, -448.0f), 448.0f));
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

// Operand loaders: lane (li = lane % 16, lk = lane / 16).  A: row li of the
// 16-row block, columns [j0 + KW*lk, +KW).  B: replica li, the same columns.
// Both sides map the lane's KW values to the same k indices, so the product
// sums every column of the chunk exactly once.
template <typename JT, int FIELD, int QB, int RB>
__global__ void __launch_bounds__(256)
bstep_kernel(const BTile* __restrict__ tiles, const BInst* __restrict__ insts, BStepArgs a, int k,
             const double* __restrict__ etap) {
  const BTile tl = tiles[blockIdx.x];
  const BInst I = insts[tl.inst];
  const int n = I.n, ld = I.ld, P = a.P;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int rbase = tl.row0 + wv * 16 * RB;
  const JT* J = static_cast<const JT*>(I.J);
  const float* cin = (k & 1) ? I.c2 : I.c;
  const bool last = (k == a.n_steps);
  const float st = float(sqrt(a.tau));

  v4f acc[RB][QB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) acc[rb][qb] = v4f{0.f, 0.f, 0.f, 0.f};

  if constexpr (sizeof(JT) == 4) {
    // FP32: per 32-column chunk each lane loads two float4 of A (per row
    // block) and of B (per replica block), feeding 8 MFMA steps of k = 4.
    // The next chunk's loads are issued before this chunk's MFMAs.
    auto loadA = [&](int j0, float4 (&av)[RB][2]) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int row = rbase + rb * 16 + li;
        const float* src = J + size_t(row) * I.ldj + j0 + 8 * lk;
        av[rb][0] = row < n ? *reinterpret_cast<const float4*>(src) : make_float4(0.f, 0.f, 0.f, 0.f);
        av[rb][1] = row < n ? *reinterpret_cast<const float4*>(src + 4) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    };
    auto loadB = [&](int j0, float4 (&bv)[QB][2]) {
#pragma unroll
      for (int qb = 0; qb < QB; ++qb) {
        const int q = qb * 16 + li;
        const float* src = cin + size_t(q) * ld + j0 + 8 * lk;
        bv[qb][0] = q < P ? *reinterpret_cast<const float4*>(src) : make_float4(0.f, 0.f, 0.f, 0.f);
        bv[qb][1] = q < P ? *reinterpret_cast<const float4*>(src + 4) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    };
    float4 a0[RB][2], b0[QB][2], a1[RB][2], b1[QB][2];
    loadA(0, a0);
    loadB(0, b0);
    auto compute = [&](float4 (&av)[RB][2], float4 (&bv)[QB][2]) {
#pragma unroll
      for (int qb = 0; qb < QB; ++qb) {
        const bool on = (qb * 16 + li) < P;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const float4 c4 = bv[qb][h];
          const float x0 = on ? xf<FIELD>(c4.x, st, last) : 0.f, x1 = on ? xf<FIELD>(c4.y, st, last) : 0.f;
          const float x2 = on ? xf<FIELD>(c4.z, st, last) : 0.f, x3 = on ? xf<FIELD>(c4.w, st, last) : 0.f;
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            acc[rb][qb] = mfma_f32(av[rb][h].x, x0, acc[rb][qb]);
            acc[rb][qb] = mfma_f32(av[rb][h].y, x1, acc[rb][qb]);
            acc[rb][qb] = mfma_f32(av[rb][h].z, x2, acc[rb][qb]);
            acc[rb][qb] = mfma_f32(av[rb][h].w, x3, acc[rb][qb]);
          }
        }
      }
    };
    int j0 = 0;
    for (; j0 + 32 < ld; j0 += 64) {
      loadA(j0 + 32, a1);
      loadB(j0 + 32, b1);
      compute(a0, b0);
      if (j0 + 64 < ld) {
        loadA(j0 + 64, a0);
        loadB(j0 + 64, b0);
      }
      compute(a1, b1);
    }
    if (j0 < ld) compute(a0, b0);
  } else if constexpr (kFp8Matrix && sizeof(JT) == 1 && FIELD == kBN) {
    // FP8 couplings, binarised operand: 8 e4m3 values per lane, k = 32.
    for (int j0 = 0; j0 < ld; j0 += 32) {
      long av[RB], bv[QB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int row = rbase + rb * 16 + li;
        av[rb] = row < n ? *reinterpret_cast<const long*>(J + size_t(row) * I.ldj + j0 + 8 * lk) : 0l;
      }
#pragma unroll
      for (int qb = 0; qb < QB; ++qb) {
        const int q = qb * 16 + li;
        uint64_t bits = 0;
        if (q < P) {
          const float4 c0 = *reinterpret_cast<const float4*>(cin + size_t(q) * ld + j0 + 8 * lk);
          const float4 c1 = *reinterpret_cast<const float4*>(cin + size_t(q) * ld + j0 + 8 * lk + 4);
          const float cc[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
          for (int t = 0; t < 8; ++t) bits |= (cc[t] > 0.0f ? uint64_t(0x38) : uint64_t(0)) << (8 * t);
        }
        bv[qb] = long(bits);   // 0x38 is 1.0 in OCP e4m3
      }
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) acc[rb][qb] = mfma_fp8(av[rb], bv[qb], acc[rb][qb]);
    }
  } else {
    // BF16 couplings (or FP8 widened to bf16 exactly): 8 values per lane,
    // k = 32; the continuous operand is split into bf16 hi + lo.
    for (int j0 = 0; j0 < ld; j0 += 32) {
      v8bf av[RB], bh[QB], bl[QB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int row = rbase + rb * 16 + li;
        if constexpr (sizeof(JT) == 2) {
          if (row < n) {
            av[rb] = *reinterpret_cast<const v8bf*>(J + size_t(row) * I.ldj + j0 + 8 * lk);
          } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) av[rb][t] = __bf16(0.0f);
          }
        } else {
          const JT* src = J + size_t(row) * I.ldj + j0 + 8 * lk;
#pragma unroll
          for (int t = 0; t < 8; ++t) av[rb][t] = __bf16(row < n ? float(src[t]) : 0.0f);
        }
      }
#pragma unroll
      for (int qb = 0; qb < QB; ++qb) {
        const int q = qb * 16 + li;
        float cc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (q < P) {
          const float4 c0 = *reinterpret_cast<const float4*>(cin + size_t(q) * ld + j0 + 8 * lk);
          const float4 c1 = *reinterpret_cast<const float4*>(cin + size_t(q) * ld + j0 + 8 * lk + 4);
          cc[0] = xf<FIELD>(c0.x, st, last); cc[1] = xf<FIELD>(c0.y, st, last);
          cc[2] = xf<FIELD>(c0.z, st, last); cc[3] = xf<FIELD>(c0.w, st, last);
          cc[4] = xf<FIELD>(c1.x, st, last); cc[5] = xf<FIELD>(c1.y, st, last);
          cc[6] = xf<FIELD>(c1.z, st, last); cc[7] = xf<FIELD>(c1.w, st, last);
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const __bf16 h = __bf16(cc[t]);
          bh[qb][t] = h;
          bl[qb][t] = __bf16(cc[t] - float(h));
        }
      }
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
          acc[rb][qb] = mfma_bf16(av[rb], bh[qb], acc[rb][qb]);
          if (FIELD == kCN && !last) acc[rb][qb] = mfma_bf16(av[rb], bl[qb], acc[rb][qb]);
        }
    }
  }

  // Epilogue: lane holds rows rbase + rb*16 + 4*lk + v (v < 4) of replica qb*16 + li.
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
  int bits = 0;
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    const int q = qb * 16 + li;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int r0 = rbase + rb * 16 + 4 * lk;
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
          const float y = acc[rb][qb][v] * rs[r];
          float cv = cvs[v], ev = evs[v];
          if (!last) {
            const float phi = (FIELD == kCN) ? (y + half_st * z[r]) : (half_st * (y + z[r]));
            const float inj = jj * ev * (phi - theta);
            const float c2 = cv * cv;
            const float dc = (lin - c2) * cv + KK * inj;
            const float de = -beta * (c2 - tau) * ev;
            cvs[v] = cv + dt * dc;
            evs[v] = ev + dt * de;
            if (k < a.trace_steps) {
              a.trace[(size_t(2 * k) * P + q) * n + r] = cvs[v];
              a.trace[(size_t(2 * k + 1) * P + q) * n + r] = evs[v];
            }
          } else {
            const bool s = cv > 0.0f;
            I.hpart[size_t(q) * n + r] = s ? (-0.5 * double(y) - double(z[r]) + lam) : 0.0;
            I.sig_all[size_t(q) * n + r] = s ? 1 : 0;
            if (!(isfinite(cv) && isfinite(ev))) bits |= L0CIM_ST_NONFINITE;
            else if (fabsf(cv) > 1e3f) bits |= L0CIM_ST_BLOWUP;
          }
        }
        if (!last) {
          *reinterpret_cast<float4*>(cout + off) = make_float4(cvs[0], cvs[1], cvs[2], cvs[3]);
          *reinterpret_cast<float4*>(e + off) = make_float4(evs[0], evs[1], evs[2], evs[3]);
        }
      }
    }
  }
  if (last && bits) raise_status(I.status, bits);
}

// Per instance: H_q = sum of the per-spin eq. 4 terms in spin order (so the
// result does not depend on the tile shape or on the rest of the batch),
// lowest-energy replica (first on ties, NaN last), copy of its support.
__global__ void __launch_bounds__(256)
bselect_kernel(const BInst* __restrict__ insts, int P) {
  __shared__ int qs;
  __shared__ double hq[64];
  const BInst I = insts[blockIdx.x];
  if (threadIdx.x < P) {
    const double* hr = I.hpart + size_t(threadIdx.x) * I.n;
    double h = 0.0;
    for (int r = 0; r < I.n; ++r) h += hr[r];
    hq[threadIdx.x] = h;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
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
  const uint8_t* src = I.sig_all + size_t(qs) * I.n;
  for (int i = threadIdx.x; i < I.n; i += 256) I.sig[i] = src[i];
}

// ---------------------------------------------------------------------------
// CDP for every instance: one workgroup per instance.  The support's columns
// of G are gathered once into a compact block, then `iters` synchronous
// Jacobi sweeps update every r (same update as the single-instance path).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024)
bjacobi_kernel(const BInst* __restrict__ insts, float dtc, int iters) {
  extern __shared__ __align__(16) unsigned char smem[];
  const BInst I = insts[blockIdx.x];
  const int n = I.n, ld = I.ld;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6, nwv = bs >> 6;
  int* S = reinterpret_cast<int*>(smem);                  // n
  float* Rl = reinterpret_cast<float*>(smem + 4 * size_t(ld));   // n
  float* sR = Rl + ld;                                     // |S|
  __shared__ int cnt[1024];
  __shared__ int sh_k;
  const uint8_t* sg = I.sig;
  const float* G = I.G;
  const float* b = I.b;
  float* R = I.R;
  float* Gc = I.Gc;
  // support list in index order
  const int chunk = (n + bs - 1) / bs;
  const int lo = min(n, tid * chunk), hi = min(n, lo + chunk);
  int c = 0;
  for (int i = lo; i < hi; ++i) c += sg[i] ? 1 : 0;
  cnt[tid] = c;
  __syncthreads();
  if (tid == 0) {
    int s = 0;
    for (int t = 0; t < bs; ++t) {
      int v = cnt[t];
      cnt[t] = s;
      s += v;
    }
    sh_k = s;
  }
  __syncthreads();
  int pos = cnt[tid];
  for (int i = lo; i < hi; ++i)
    if (sg[i]) S[pos++] = i;
  int bits = 0;
  for (int i = tid; i < n; i += bs) {
    const float d = G[size_t(i) * ld + i];
    const bool tiny = !(d >= 1e-12f);
    if (tiny) bits |= L0CIM_ST_TINY_DIAG;
    Rl[i] = tiny ? 0.0f : R[i];
  }
  __syncthreads();
  const int ks = sh_k;
  // compact columns: Gc[r][s] = G[r][S[s]]
  for (size_t e = tid; e < size_t(n) * ks; e += bs) {
    const int r = int(e / ks), s = int(e - size_t(r) * ks);
    Gc[size_t(r) * ks + s] = G[size_t(r) * ld + S[s]];
  }
  for (int s = tid; s < ks; s += bs) sR[s] = Rl[S[s]];
  __syncthreads();
  for (int it = 0; it < iters; ++it) {
    for (int r = wv; r < n; r += nwv) {
      const float* gr = Gc + size_t(r) * ks;
      float acc = 0.0f;
      for (int s = lane; s < ks; s += kWave)
        if (S[s] != r) acc += gr[s] * sR[s];
      acc = wave_sum(acc);
      if (lane == 0) {
        const float d = G[size_t(r) * ld + r];
        const bool tiny = !(d >= 1e-12f);
        const float Rv = Rl[r];
        Rl[r] = tiny ? 0.0f : Rv + dtc * ((b[r] - acc) / d - Rv);
      }
    }
    __syncthreads();
    for (int s = tid; s < ks; s += bs) sR[s] = Rl[S[s]];
    __syncthreads();
  }
  for (int i = tid; i < n; i += bs) R[i] = Rl[i];
  if (bits && tid == 0) raise_status(I.status, bits);
  (void)cnt;
}

// eq. 3 objective and the per-instance report: one workgroup per instance.
__global__ void __launch_bounds__(256)
bobjective_kernel(const BInst* __restrict__ insts, double lam, int64_t steps_per_alt, int n_outer, int P) {
  __shared__ double part[4];
  __shared__ int cnt[256];
  const BInst I = insts[blockIdx.x];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const float* A = I.A;
  const float* y = I.y;
  const uint8_t* sg = I.sig;
  const float* R = I.R;
  double r2 = 0.0;
  for (int row = wv; row < I.m; row += 4) {
    double acc = 0.0;
    for (int j = lane; j < I.n; j += kWave)
      if (sg[j]) acc += double(A[size_t(row) * I.lda + j]) * double(R[j]);
    acc = wave_sum(acc);
    const double res = double(y[row]) - acc;
    r2 += res * res;
  }
  if (lane == 0) part[wv] = r2;
  int c = 0;
  for (int j = threadIdx.x; j < I.n; j += 256) c += sg[j] ? 1 : 0;
  cnt[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int t = 0; t < 256; ++t) s += cnt[t];
    const double rr = ((part[0] + part[1]) + part[2]) + part[3];
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
#define L0_RB(Q)                                               \
  switch (rb) {                                                \
    case 1: return step_kernel_ptr<JT, FIELD, Q, 1>();         \
    case 2: return step_kernel_ptr<JT, FIELD, Q, 2>();         \
    case 4: return step_kernel_ptr<JT, FIELD, Q, 4>();         \
  }                                                            \
  return nullptr;
  switch (qb) {
    case 1: { L0_RB(1) }
    case 2: { L0_RB(2) }
    case 4: { L0_RB(4) }
  }
#undef L0_RB
  return nullptr;
}

const void* batch_step_kernel(l0cim_dtype jdt, int field, int qb, int rb) {
  if (jdt == L0CIM_F32)
    return field == L0CIM_FIELD_BN ? step_kernel_q<float, kBN>(qb, rb) : step_kernel_q<float, kCN>(qb, rb);
  if (jdt == L0CIM_BF16)
    return field == L0CIM_FIELD_BN ? step_kernel_q<__hip_bfloat16, kBN>(qb, rb)
                                   : step_kernel_q<__hip_bfloat16, kCN>(qb, rb);
  if (jdt == L0CIM_FP8E4M3)
    return field == L0CIM_FIELD_BN ? step_kernel_q<__hip_fp8_e4m3, kBN>(qb, rb)
                                   : step_kernel_q<__hip_fp8_e4m3, kCN>(qb, rb);
  return nullptr;
}

l0cim_status enqueue_bsteps(const BatchDev& d, const void* fn, const BStepArgs& a, int ntiles, int k0, int k1,
                            hipStream_t s) {
  for (int k = k0; k <= k1; ++k) {
    const BTile* tiles = d.tiles;
    const BInst* insts = d.insts;
    BStepArgs aa = a;
    int kk = k;
    const double* eta = d.eta;
    void* args[] = {&tiles, &insts, &aa, &kk, &eta};
    L0_HIP(hipLaunchKernel(fn, dim3(ntiles), dim3(256), args, 0, s));
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

l0cim_status launch_bselect(const BatchDev& d, int P, hipStream_t s) {
  hipLaunchKernelGGL(bselect_kernel, dim3(d.count), dim3(256), 0, s, d.insts, P);
  L0_LAUNCHED("bselect_kernel");
  return L0CIM_OK;
}

l0cim_status launch_bjacobi(const BatchDev& d, int max_ld, double dtc, int iters, hipStream_t s) {
  const size_t lds = size_t(max_ld) * 4 * 3;
  L0_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(bjacobi_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  hipLaunchKernelGGL(bjacobi_kernel, dim3(d.count), dim3(1024), lds, s, d.insts, float(dtc), iters);
  L0_LAUNCHED("bjacobi_kernel");
  return L0CIM_OK;
}

l0cim_status launch_bobjective(const BatchDev& d, double lam, int64_t steps_per_alt, int n_outer, int P,
                               hipStream_t s) {
  hipLaunchKernelGGL(bobjective_kernel, dim3(d.count), dim3(256), 0, s, d.insts, lam, steps_per_alt, n_outer, P);
  L0_LAUNCHED("bobjective_kernel");
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
