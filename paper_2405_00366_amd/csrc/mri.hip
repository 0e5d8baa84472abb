// MF-CIM run for an MRI-shaped observation matrix A = S C Psi^T (a subset S
// of the frequencies of the orthonormal 2-D DCT-II C of a 2-D image, Psi the
// orthonormal multi-level 2-D Haar analysis in Mallat layout), with the
// couplings J = -(A^T A) o R R^T (zero diagonal) applied in factored form:
//
//   (J x)_r = -R_r (G (R o x))_r + G_rr R_r^2 x_r,
//   G v     = Psi C^T M C Psi^T v        (M: 0/1 mask of the sampled frequencies)
//
// which is the product with the dense couplings (eq. 13, 15, 16) without the
// N x N matrix: per replica and Euler step an inverse Haar transform, a 2-D
// DCT-II, the mask, a 2-D DCT-III and a Haar transform of the 128 x 128 image,
// O(N log N) FP32 work instead of N^2 coupling bytes.
//
// One workgroup of 512 threads owns one replica for the whole run (512 rather
// than 1024 so that a thread may hold 256 registers).  The image lives in LDS
// (two 128 x 136 float buffers); thread t keeps c, e and R of spins t + 512 i,
// i < 32, in registers.  The Haar transforms take one pass each (an aligned
// 2^levels square of pixels depends only on its own coefficients).  Each
// length-128 DCT is the length-128 complex FFT of a reordered sequence with a
// phase factor (Makhoul's algorithm), and each 8-lane group transforms rows
// (or columns) g and g + 64 with one FFT of v_a + i v_b: the forward results
// are separated with Z[k] and Z[N - k]; the inverse uses the Hermitian form
// of the coefficients, whose inverse FFT is real, so the two rows are its
// real and imaginary parts.  The FFT is split 128 = 16 x 8: a 16-point DFT in
// the registers of each of 8 lanes, a twiddle, a transpose through the rows'
// own LDS storage within the wavefront, and 8-point DFTs; the inverse runs
// the same steps backwards, so the forward output layout feeds it without
// reordering.
#include <cmath>
#include <cstdint>

#include "kernels.h"

namespace l0 {
namespace {

constexpr int kS = 128;            // image side
// LDS row stride (floats).  The lanes of one instruction touch up to eight
// rows (the 8-lane groups of a wavefront); with a stride of 8 mod 64 those
// rows fall in different banks in the transposes, which were most of the
// bank conflicts (61% of LDS cycles at a stride of 129).  Per Euler step of
// 64 replicas on MI355X: 129 -> 27.1 us, 132 -> 27.2, 136 -> 24.2, 137 -> 26.0.
constexpr int kLd = kS + 8;
constexpr int kBS = 512;           // threads per workgroup
constexpr int kPer = kS * kS / kBS; // spins per thread
constexpr int kRows = kS / (kBS / 8);   // rows an 8-lane group transforms per pass
constexpr int kQuads = (kS / 2) * (kS / 2) / kBS;   // Haar quads per thread at the finest level
static_assert(kRows * 16 <= 32, "mask bits of a thread's column frequencies fit one word");

struct MriLds {
  float A[kS * kLd];   // the image; the row pass's output is stored back into it transposed
  float Rv[kS * kS];   // R of the run's spins (read-only), in LDS rather than registers
  float2 tw[kS];     // exp(-2 pi i m / 128)
  float2 ph[kS];     // exp(-i pi k / 256)
  double red[kBS / kWave];
  float lam2[kS];    // (4 sin^2(pi k / 256))^2: D^T D of the reflecting second difference in the DCT-II basis
  float lin[4096];   // p_k - 1 (- j) of the first steps (eq. 21)
};
constexpr int kLinSteps = 4096;

// cos and sin of 2 pi m / 16
__device__ constexpr float kCos16[16] = {
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
__device__ constexpr float kSin16[16] = {
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f};

template <int BITS>
__host__ __device__ constexpr int brev(int p) {
  int r = 0;
  for (int i = 0; i < BITS; ++i) r |= ((p >> i) & 1) << (BITS - 1 - i);
  return r;
}

// In-place radix-2 decimation-in-frequency DFT of length L <= 16 with kernel
// exp(SIGN 2 pi i n k / L): natural-order input, bit-reversed output.
template <int L, int SIGN>
__device__ __forceinline__ void dif(float (&re)[L], float (&im)[L]) {
#pragma unroll
  for (int half = L / 2; half >= 1; half >>= 1) {
#pragma unroll
    for (int base = 0; base < L; base += 2 * half) {
#pragma unroll
      for (int q = 0; q < half; ++q) {
        const int i0 = base + q, i1 = i0 + half;
        const float ar = re[i0], ai = im[i0], br = re[i1], bi = im[i1];
        re[i0] = ar + br;
        im[i0] = ai + bi;
        const float dr = ar - br, di = ai - bi;
        const int m = q * (L / (2 * half));
        if (m == 0) {
          re[i1] = dr;
          im[i1] = di;
        } else if (4 * m == L) {
          re[i1] = -float(SIGN) * di;
          im[i1] = float(SIGN) * dr;
        } else {
          const float cr = kCos16[m * (16 / L)], ci = float(SIGN) * kSin16[m * (16 / L)];
          re[i1] = dr * cr - di * ci;
          im[i1] = dr * ci + di * cr;
        }
      }
    }
  }
}

// Orders the LDS accesses of the lanes of one wavefront (a transpose within
// an 8-lane group) without a workgroup barrier.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int opaque_tid() {
  int t;
  asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"(int(threadIdx.x)));
  return t;
}

// Slot of element (k1, n2) of the FFT transpose in a row's storage: 16 groups
// of 8, group k1 shifted by k1 / 2 slots (at most slot 134, inside the row's
// 136-float stride).  Lane n2 of an 8-lane group writes (k1, n2) for one k1
// at a time and reads (2 n2 + h, q) for one q at a time; unshifted, those
// reads put the 64 lanes of a wavefront (8 groups, rows 8 banks apart) on 8
// banks, shifted on 64 distinct ones, and both sides keep one address per
// lane plus constant offsets.
__device__ __forceinline__ int tslot(int k1, int n2) { return k1 * 8 + n2 + (k1 >> 1); }
static_assert(15 * 8 + 7 + 15 / 2 < kLd, "transpose slots stay inside the row's stride");

// Position in a length-128 row of element m of the reordered DCT sequence:
// v[m] = x[2m] for m < 64, x[255 - 2m] otherwise.
__device__ __forceinline__ int perm_col(int m) { return m < kS / 2 ? 2 * m : 2 * kS - 1 - 2 * m; }

__device__ __forceinline__ float dct_gain(int k) {
  return k == 0 ? 0.08838834764831845f : 0.125f;   // sqrt(1/128), sqrt(2/128)
}

// Forward orthonormal DCT-II of two rows at once: the reordered sequences
// v_a[m] = a[perm_col(m)], v_b[m] = b[perm_col(m)] (one 8-lane group, lane n2)
// go through one complex FFT of z = v_a + i v_b; with Z[k] and Z[N - k],
// V_a = (Z[k] + conj Z[N-k]) / 2 and V_b = (Z[k] - conj Z[N-k]) / 2i, and
// y[k] = g_k Re(exp(-i pi k / 256) V[k]).  scr_re / scr_im: 128 floats of the
// group's scratch each (the two input rows may serve, once read).  Output:
// ya/yb[h * 8 + p] = coefficient k = 2 j + h + 16 brev3(p), j = n2.
__device__ __forceinline__ void dct_fwd2(const float* srca, const float* srcb, float* scr_re, float* scr_im,
                                         int n2, const MriLds& s, float (&ya)[16], float (&yb)[16]) {
  float re[16], im[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) {
    re[n1] = srca[perm_col(8 * n1 + n2)];
    im[n1] = srcb[perm_col(8 * n1 + n2)];
  }
  wave_sync();
  dif<16, -1>(re, im);
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int k1 = brev<4>(p);
    const float2 t = s.tw[(n2 * k1) & (kS - 1)];
    scr_re[tslot(k1, n2)] = re[p] * t.x - im[p] * t.y;
    scr_im[tslot(k1, n2)] = re[p] * t.y + im[p] * t.x;
  }
  wave_sync();
  float zr[16], zi[16];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k1 = 2 * n2 + h;
    float r8[8], i8[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      r8[q] = scr_re[tslot(k1, q)];
      i8[q] = scr_im[tslot(k1, q)];
    }
    dif<8, -1>(r8, i8);
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      zr[h * 8 + p] = r8[p];
      zi[h * 8 + p] = i8[p];
    }
  }
  wave_sync();
  // Z[k] of every k of the row, then each lane reads its partners Z[N - k]
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int k = 2 * n2 + h + 16 * brev<3>(p);
      scr_re[k] = zr[h * 8 + p];
      scr_im[k] = zi[h * 8 + p];
    }
  wave_sync();
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int k = 2 * n2 + h + 16 * brev<3>(p);
      const int kp = (kS - k) & (kS - 1);
      const float rr = scr_re[kp], ri = scr_im[kp];
      const float Ar = 0.5f * (zr[h * 8 + p] + rr), Ai = 0.5f * (zi[h * 8 + p] - ri);
      const float Br = 0.5f * (zi[h * 8 + p] + ri), Bi = -0.5f * (zr[h * 8 + p] - rr);
      const float2 f = s.ph[k];
      const float gk = dct_gain(k);
      ya[h * 8 + p] = gk * (f.x * Ar - f.y * Ai);
      yb[h * 8 + p] = gk * (f.x * Br - f.y * Bi);
    }
  wave_sync();
  __builtin_amdgcn_sched_barrier(0);
}

// Inverse (orthonormal DCT-III) of two rows at once.  For each row the
// coefficients y[k] and their partners y[N - k] are held as
// w[h * 8 + k2] / wp[h * 8 + k2] for k = 2 j + h + 16 k2 (natural k2), j = n2
// (wp of k = 0 unused).  With Z = g y, W[0] = Z[0] and
// W[k] = exp(i pi k / 256) (Z[k] - i Z[N-k]) / 2 is Hermitian, so the inverse
// FFT of W_a + i W_b is v_a + i v_b.  Output: xa/xb[p] = value at position
// perm_col(8 brev4(p) + n2) of the row.
__device__ __forceinline__ void dct_inv2(const float (&wa)[16], const float (&wpa)[16], const float (&wb)[16],
                                         const float (&wpb)[16], float* scr_re, float* scr_im, int n2,
                                         const MriLds& s, float (&xa)[16], float (&xb)[16]) {
  wave_sync();   // the caller may have read its input from the scratch rows
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k1 = 2 * n2 + h;
    float r8[8], i8[8];
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
      const int k = k1 + 16 * k2;
      const int kp = (kS - k) & (kS - 1);
      const float2 f = s.ph[k];
      const float cx = f.x, sx = -f.y;                 // exp(+i pi k / 256)
      const float za = dct_gain(k) * wa[h * 8 + k2], zna = dct_gain(kp) * wpa[h * 8 + k2];
      const float zb = dct_gain(k) * wb[h * 8 + k2], znb = dct_gain(kp) * wpb[h * 8 + k2];
      float War, Wai, Wbr, Wbi;
      if (k == 0) {
        War = za; Wai = 0.0f; Wbr = zb; Wbi = 0.0f;
      } else {
        War = 0.5f * (cx * za + sx * zna);
        Wai = 0.5f * (sx * za - cx * zna);
        Wbr = 0.5f * (cx * zb + sx * znb);
        Wbi = 0.5f * (sx * zb - cx * znb);
      }
      r8[k2] = War - Wbi;
      i8[k2] = Wai + Wbr;
    }
    dif<8, 1>(r8, i8);
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int q = brev<3>(p);          // n2 of this output
      const float2 t = s.tw[(q * k1) & (kS - 1)];   // conj twiddle
      scr_re[tslot(k1, q)] = r8[p] * t.x + i8[p] * t.y;
      scr_im[tslot(k1, q)] = i8[p] * t.x - r8[p] * t.y;
    }
  }
  wave_sync();
  float re[16], im[16];
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) {
    re[k1] = scr_re[tslot(k1, n2)];
    im[k1] = scr_im[tslot(k1, n2)];
  }
  wave_sync();
  dif<16, 1>(re, im);
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    xa[p] = re[p];
    xb[p] = im[p];
  }
  __builtin_amdgcn_sched_barrier(0);
}

// Inverse Haar of LV levels on the image in A, in one pass: with LV levels an
// aligned block of 2^LV x 2^LV pixels depends only on its own coefficients
// (at level lev, the (2^LV >> lev)/2 square of quads at block position (a, b)
// of each subband), so a thread gathers them for each of its blocks, runs the
// levels in registers, and after one barrier writes the pixels.
// out(2i+p, 2j+q) = 1/2 sum (-1)^(ap+bq) c(i+ah, j+bh).
template <int LV>
__device__ __forceinline__ void ihaar_fused(MriLds& s, int t) {
  constexpr int Bk = 1 << LV, NB = kS / Bk, NBLK = NB * NB;
  constexpr int PER = (NBLK + kBS - 1) / kBS;
  float x[PER][Bk][Bk];
#pragma unroll
  for (int w = 0; w < PER; ++w) {
    const int blk = t + w * kBS;
    if (blk >= NBLK) break;
    const int a = blk / NB, b = blk - a * NB;
    x[w][0][0] = s.A[a * kLd + b];
#pragma unroll
    for (int lev = LV - 1; lev >= 0; --lev) {
      const int half = (Bk >> lev) / 2, hg = (kS >> lev) / 2;
      float nx[Bk][Bk];
#pragma unroll
      for (int i = 0; i < half; ++i)
#pragma unroll
        for (int j = 0; j < half; ++j) {
          const int gi = a * half + i, gj = b * half + j;
          const float c00 = x[w][i][j], c01 = s.A[gi * kLd + gj + hg];
          const float c10 = s.A[(gi + hg) * kLd + gj], c11 = s.A[(gi + hg) * kLd + gj + hg];
          nx[2 * i][2 * j] = 0.5f * ((c00 + c10) + (c01 + c11));
          nx[2 * i][2 * j + 1] = 0.5f * ((c00 + c10) - (c01 + c11));
          nx[2 * i + 1][2 * j] = 0.5f * ((c00 - c10) + (c01 - c11));
          nx[2 * i + 1][2 * j + 1] = 0.5f * ((c00 - c10) - (c01 - c11));
        }
#pragma unroll
      for (int i = 0; i < 2 * half; ++i)
#pragma unroll
        for (int j = 0; j < 2 * half; ++j) x[w][i][j] = nx[i][j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < PER; ++w) {
    const int blk = t + w * kBS;
    if (blk >= NBLK) break;
    const int a = blk / NB, b = blk - a * NB;
#pragma unroll
    for (int i = 0; i < Bk; ++i)
#pragma unroll
      for (int j = 0; j < Bk; ++j) s.A[(a * Bk + i) * kLd + b * Bk + j] = x[w][i][j];
  }
  __syncthreads();
}

// Haar analysis of LV levels in one pass (the inverse of ihaar_fused):
// out(i+ah, j+bh) = 1/2 sum (-1)^(ap+bq) x(2i+p, 2j+q), level by level on the
// block's low-pass part; after one barrier every coefficient is written where
// it belongs.
template <int LV>
__device__ __forceinline__ void haar_fused(MriLds& s, int t) {
  constexpr int Bk = 1 << LV, NB = kS / Bk, NBLK = NB * NB;
  constexpr int PER = (NBLK + kBS - 1) / kBS;
  float x[PER][Bk][Bk];
#pragma unroll
  for (int w = 0; w < PER; ++w) {
    const int blk = t + w * kBS;
    if (blk >= NBLK) break;
    const int a = blk / NB, b = blk - a * NB;
#pragma unroll
    for (int i = 0; i < Bk; ++i)
#pragma unroll
      for (int j = 0; j < Bk; ++j) x[w][i][j] = s.A[(a * Bk + i) * kLd + b * Bk + j];
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < PER; ++w) {
    const int blk = t + w * kBS;
    if (blk >= NBLK) break;
    const int a = blk / NB, b = blk - a * NB;
#pragma unroll
    for (int lev = 0; lev < LV; ++lev) {
      const int half = (Bk >> lev) / 2, hg = (kS >> lev) / 2;
#pragma unroll
      for (int i = 0; i < half; ++i)
#pragma unroll
        for (int j = 0; j < half; ++j) {
          const float x00 = x[w][2 * i][2 * j], x01 = x[w][2 * i][2 * j + 1];
          const float x10 = x[w][2 * i + 1][2 * j], x11 = x[w][2 * i + 1][2 * j + 1];
          const int gi = a * half + i, gj = b * half + j;
          s.A[gi * kLd + gj + hg] = 0.5f * ((x00 - x01) + (x10 - x11));
          s.A[(gi + hg) * kLd + gj] = 0.5f * ((x00 + x01) - (x10 + x11));
          s.A[(gi + hg) * kLd + gj + hg] = 0.5f * ((x00 - x01) - (x10 - x11));
          x[w][i][j] = 0.5f * ((x00 + x01) + (x10 + x11));   // (i, j) <= (2i, 2j): already read
        }
    }
    s.A[a * kLd + b] = x[w][0][0];
  }
  __syncthreads();
}

// G v for the workgroup's replica: the values u (R o x) of the thread's spins
// go in, (Psi C^T M C Psi^T u) of the same spins comes out.  mbits: the mask
// bits of the (kr, kc) the thread holds in the column pass.  t is the thread
// index, passed as a value the compiler cannot see through (opaque_tid) so
// that the few hundred LDS addresses derived from it are formed inside each
// call rather than hoisted out of the step loop and kept live (which spilled).
__device__ void gram_apply(MriLds& s, float (&u)[kPer], int levels, uint32_t mbits, float gamma, int t,
                           const float* __restrict__ D, int64_t incd, const float* __restrict__ bv,
                           float (&dq)[kPer], float (&zb)[kPer]) {
  const int g = t >> 3, n2 = t & 7;
  const int col = t & (kS - 1), row0 = t / kS;
  constexpr int kRowStep = kBS / kS;
#pragma unroll
  for (int i = 0; i < kPer; ++i) s.A[(row0 + kRowStep * i) * kLd + col] = u[i];
  __syncthreads();
  // inverse Haar, coarsest level first: out(2i+p, 2j+q) = 1/2 sum (-1)^(ap+bq) c(i+ah, j+bh)
  if (levels == 3) ihaar_fused<3>(s, t);
  else if (levels == 2) ihaar_fused<2>(s, t);
  else if (levels == 1) ihaar_fused<1>(s, t);
  else for (int lev = levels - 1; lev >= 0; --lev) {
    const int h = (kS >> lev) >> 1;
    float v[kQuads][4];
#pragma unroll
    for (int nq = 0; nq < kQuads; ++nq) {
      const int q = t + nq * kBS;
      if (q >= h * h) break;
      const int i = q / h, j = q - i * h;
      const float c00 = s.A[i * kLd + j], c01 = s.A[i * kLd + j + h];
      const float c10 = s.A[(i + h) * kLd + j], c11 = s.A[(i + h) * kLd + j + h];
      v[nq][0] = 0.5f * ((c00 + c10) + (c01 + c11));
      v[nq][1] = 0.5f * ((c00 + c10) - (c01 + c11));
      v[nq][2] = 0.5f * ((c00 - c10) + (c01 - c11));
      v[nq][3] = 0.5f * ((c00 - c10) - (c01 - c11));
    }
    __syncthreads();
#pragma unroll
    for (int nq = 0; nq < kQuads; ++nq) {
      const int q = t + nq * kBS;
      if (q >= h * h) break;
      const int i = q / h, j = q - i * h;
      s.A[(2 * i) * kLd + 2 * j] = v[nq][0];
      s.A[(2 * i) * kLd + 2 * j + 1] = v[nq][1];
      s.A[(2 * i + 1) * kLd + 2 * j] = v[nq][2];
      s.A[(2 * i + 1) * kLd + 2 * j + 1] = v[nq][3];
    }
    __syncthreads();
  }
  // rows: DCT-II along each image row, rows g and g + 64 as one complex FFT;
  // once every row is in registers the result is stored transposed in A
  constexpr int H = kS / 2;
  static_assert(kBS / 8 == H, "one 8-lane group per row pair");
  {
    float ya[16], yb[16];
    dct_fwd2(s.A + g * kLd, s.A + (g + H) * kLd, s.A + g * kLd, s.A + (g + H) * kLd, n2, s, ya, yb);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const int k = 2 * n2 + h + 16 * brev<3>(p);
        s.A[k * kLd + g] = ya[h * 8 + p];
        s.A[k * kLd + g + H] = yb[h * 8 + p];
      }
    __syncthreads();
  }
  // columns kc = g and g + 64 (rows of the transposed A): DCT-II, mask, DCT-III
  {
    float ya[16], yb[16];
    float* ra = s.A + g * kLd;
    float* rb = s.A + (g + H) * kLd;
    dct_fwd2(ra, rb, ra, rb, n2, s, ya, yb);
    if (gamma == 0.0f) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int p = 0; p < 8; ++p) {
          const int k = 2 * n2 + h + 16 * brev<3>(p);
          ra[k] = ((mbits >> (h * 8 + p)) & 1u) ? ya[h * 8 + p] : 0.0f;
          rb[k] = ((mbits >> (16 + h * 8 + p)) & 1u) ? yb[h * 8 + p] : 0.0f;
        }
    } else {
      // the L2 term of eq. 20 is diagonal in this basis: weight mask(kr, kc)
      // + gamma (lam2[kr] + lam2[kc]), kr = k, kc = g (row a) or g + 64 (row b)
      const float la = s.lam2[g], lb = s.lam2[g + H];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int p = 0; p < 8; ++p) {
          const int k = 2 * n2 + h + 16 * brev<3>(p);
          const float lk = s.lam2[k];
          const float ma = ((mbits >> (h * 8 + p)) & 1u) ? 1.0f : 0.0f;
          const float mb = ((mbits >> (16 + h * 8 + p)) & 1u) ? 1.0f : 0.0f;
          ra[k] = ya[h * 8 + p] * (ma + gamma * (lk + la));
          rb[k] = yb[h * 8 + p] * (mb + gamma * (lk + lb));
        }
    }
    wave_sync();
    float wa[16], wpa[16], wb[16], wpb[16];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k2 = 0; k2 < 8; ++k2) {
        const int k = 2 * n2 + h + 16 * k2, kp = (kS - k) & (kS - 1);
        wa[h * 8 + k2] = ra[k];
        wpa[h * 8 + k2] = ra[kp];
        wb[h * 8 + k2] = rb[k];
        wpb[h * 8 + k2] = rb[kp];
      }
    float xa[16], xb[16];
    dct_inv2(wa, wpa, wb, wpb, ra, rb, n2, s, xa, xb);
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 16; ++p) {
      const int r = perm_col(8 * brev<4>(p) + n2);
      s.A[r * kLd + g] = xa[p];
      s.A[r * kLd + g + H] = xb[p];
    }
    __syncthreads();
  }
  // rows: DCT-III along image rows g and g + 64
  {
    float* ra = s.A + g * kLd;
    float* rb = s.A + (g + H) * kLd;
    float wa[16], wpa[16], wb[16], wpb[16];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k2 = 0; k2 < 8; ++k2) {
        const int k = 2 * n2 + h + 16 * k2, kp = (kS - k) & (kS - 1);
        wa[h * 8 + k2] = ra[k];
        wpa[h * 8 + k2] = ra[kp];
        wb[h * 8 + k2] = rb[k];
        wpb[h * 8 + k2] = rb[kp];
      }
    float xa[16], xb[16];
    dct_inv2(wa, wpa, wb, wpb, ra, rb, n2, s, xa, xb);
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 16; ++p) {
      const int c = perm_col(8 * brev<4>(p) + n2);
      ra[c] = xa[p];
      rb[c] = xb[p];
    }
    __syncthreads();
  }
  // D and b of the thread's spins for the epilogue, requested here so that
  // their latency is spent under the Haar transform
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int r = t + kBS * i;
    dq[i] = D[r * incd];
    zb[i] = bv[r];
  }
  // Haar analysis, finest level first: out(i+ah, j+bh) = 1/2 sum (-1)^(ap+bq) x(2i+p, 2j+q)
  if (levels == 3) haar_fused<3>(s, t);
  else if (levels == 2) haar_fused<2>(s, t);
  else if (levels == 1) haar_fused<1>(s, t);
  else for (int lev = 0; lev < levels; ++lev) {
    const int h = (kS >> lev) >> 1;
    float v[kQuads][4];
#pragma unroll
    for (int nq = 0; nq < kQuads; ++nq) {
      const int q = t + nq * kBS;
      if (q >= h * h) break;
      const int i = q / h, j = q - i * h;
      const float x00 = s.A[(2 * i) * kLd + 2 * j], x01 = s.A[(2 * i) * kLd + 2 * j + 1];
      const float x10 = s.A[(2 * i + 1) * kLd + 2 * j], x11 = s.A[(2 * i + 1) * kLd + 2 * j + 1];
      v[nq][0] = 0.5f * ((x00 + x01) + (x10 + x11));
      v[nq][1] = 0.5f * ((x00 - x01) + (x10 - x11));
      v[nq][2] = 0.5f * ((x00 + x01) - (x10 + x11));
      v[nq][3] = 0.5f * ((x00 - x01) - (x10 - x11));
    }
    __syncthreads();
#pragma unroll
    for (int nq = 0; nq < kQuads; ++nq) {
      const int q = t + nq * kBS;
      if (q >= h * h) break;
      const int i = q / h, j = q - i * h;
      s.A[i * kLd + j] = v[nq][0];
      s.A[i * kLd + j + h] = v[nq][1];
      s.A[(i + h) * kLd + j] = v[nq][2];
      s.A[(i + h) * kLd + j + h] = v[nq][3];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < kPer; ++i) u[i] = s.A[(row0 + kRowStep * i) * kLd + col];
  __syncthreads();
}

// p_k - 1 (- j) of eq. 21 for steps k0 .. k0 + kLinSteps - 1 into LDS (its own
// function, so that the FP64 exp is not part of the step loop's code).
__device__ __noinline__ void fill_lin(float* lin, int k0, int n_steps, double dt, double p_thr, double d,
                                     double t_c, double t_w, double lj) {
  for (int k = k0 + int(threadIdx.x); k < n_steps && k < k0 + kLinSteps; k += kBS) {
    const double tk = double(k) * dt;
    lin[k - k0] = float((p_thr - d) + 2.0 * d / (1.0 + exp(-(tk - t_c) / t_w)) - 1.0 - lj);
  }
}

// Twiddle, phase and L2-weight tables in LDS; returns the mask bits of the
// frequencies (kr, kc = g) this thread holds in the column pass.
__device__ uint32_t init_tables(MriLds& s, const uint8_t* __restrict__ mask, int t) {
  const int g = t >> 3, n2 = t & 7;
  if (t < kS) {
    double sn, cs;
    sincospi(-2.0 * t / kS, &sn, &cs);
    s.tw[t] = make_float2(float(cs), float(sn));
    sincospi(-double(t) / (2 * kS), &sn, &cs);
    s.ph[t] = make_float2(float(cs), float(sn));
    const double sq = sinpi(double(t) / (2 * kS));
    const double lam = 4.0 * sq * sq;
    s.lam2[t] = float(lam * lam);
  }
  uint32_t mbits = 0;
#pragma unroll
  for (int rr = 0; rr < kRows; ++rr)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const int kr = 2 * n2 + h + 16 * brev<3>(p);
        if (mask[kr * kS + g + (kBS / 8) * rr]) mbits |= 1u << (16 * rr + h * 8 + p);
      }
  return mbits;
}

template <int FIELD>
__global__ void __launch_bounds__(kBS)
mri_cim_kernel(const uint8_t* __restrict__ mask, const float* __restrict__ R, const float* __restrict__ D, int64_t incd,
               const float* __restrict__ b, float gamma, CimArgs a, int levels, float* __restrict__ c,
               float* __restrict__ e, uint8_t* __restrict__ sigma, double* __restrict__ H,
               float* __restrict__ trace, int* __restrict__ status, MriStrides ms) {
  extern __shared__ __align__(16) unsigned char smem[];
  MriLds& s = *reinterpret_cast<MriLds*>(smem);
  const int t = threadIdx.x, q = blockIdx.x, n = kS * kS;
  if (const int k = blockIdx.y) {   // instance k of a many-instance launch
    mask += k * ms.mask;
    R += k * ms.vec;
    b += k * ms.vec;
    D += k * ms.D;
    c += k * ms.state;
    e += k * ms.state;
    sigma += k * ms.state;
    if (H) H += k * ms.H;
    status += k * ms.status;
  }
  const uint32_t mbits = init_tables(s, mask, t);
  const double lj = a.linear_j ? a.j : 0.0;
  fill_lin(s.lin, 0, a.n_steps, a.dt, a.p_thr, a.d, a.t_c, a.t_w, lj);
  float cv[kPer], ev[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int r = t + kBS * i;
    cv[i] = c[size_t(q) * n + r];
    ev[i] = e[size_t(q) * n + r];
    s.Rv[r] = R[r];
  }
  __syncthreads();
  const float st = float(sqrt(a.tau)), half_st = float(0.5 * sqrt(a.tau));
  const float theta = float(a.eta * a.eta * sqrt(a.tau) * 0.25);
  const float jj = float(a.j), KK = float(a.K), beta = float(a.beta), tau = float(a.tau), dt = float(a.dt);
  const bool bn = (FIELD == int(L0CIM_FIELD_BN));
  for (int k = 0; k < a.n_steps; ++k) {
    if (k > 0 && k % kLinSteps == 0) {
      __syncthreads();
      fill_lin(s.lin, k, a.n_steps, a.dt, a.p_thr, a.d, a.t_c, a.t_w, lj);
      __syncthreads();
    }
    float u[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const float x = bn ? (cv[i] > 0.0f ? 1.0f : 0.0f) : (cv[i] + st) * 0.25f;
      u[i] = s.Rv[t + kBS * i] * x;
    }
    float dq[kPer], zb[kPer];
    gram_apply(s, u, levels, mbits, gamma, opaque_tid(), D, incd, b, dq, zb);
    const float lin = s.lin[k % kLinSteps];
    // D and b were read again in this step (from the caches, through an
    // opaque index): held across the steps they would take 64 more registers
    const int tk = opaque_tid();
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int r = tk + kBS * i;
      const float x = bn ? (cv[i] > 0.0f ? 1.0f : 0.0f) : (cv[i] + st) * 0.25f;
      const float Rr = s.Rv[r];
      const float y = -Rr * u[i] + (dq[i] * Rr * Rr) * x;    // (J x)_r, zero diagonal
      const float zr = Rr * zb[i];                           // z = R o b
      const float phi = bn ? half_st * (y + zr) : y + half_st * zr;
      const float inj = jj * ev[i] * (phi - theta);
      const float c2 = cv[i] * cv[i];
      const float dc = (lin - c2) * cv[i] + KK * inj;
      const float de = -beta * (c2 - tau) * ev[i];
      cv[i] = cv[i] + dt * dc;
      ev[i] = ev[i] + dt * de;
      if (k < a.trace_steps) {
        trace[(size_t(2 * k) * a.P + q) * n + r] = cv[i];
        trace[(size_t(2 * k + 1) * a.P + q) * n + r] = ev[i];
      }
    }
  }
  // final state, support and the eq. 4 energy of the support (addresses from
  // an opaque index again, so that they are not shared with the loads at the
  // start and kept live through the run)
  float u[kPer];
  int bits = 0;
  const int tf = opaque_tid();
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int r = tf + kBS * i;
    c[size_t(q) * n + r] = cv[i];
    e[size_t(q) * n + r] = ev[i];
    sigma[size_t(q) * n + r] = cv[i] > 0.0f ? 1 : 0;
    u[i] = cv[i] > 0.0f ? s.Rv[r] : 0.0f;
    if (!(isfinite(cv[i]) && isfinite(ev[i]))) bits |= L0CIM_ST_NONFINITE;
    else if (fabsf(cv[i]) > 1e3f) bits |= L0CIM_ST_BLOWUP;
  }
  if (bits) raise_status(status, bits);
  if (H) {
    float dq[kPer], zb[kPer];
    gram_apply(s, u, levels, mbits, gamma, opaque_tid(), D, incd, b, dq, zb);
    const double lam = 0.5 * a.eta * a.eta;
    double hs = 0.0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int r = tf + kBS * i;
      if (cv[i] > 0.0f) {
        const double Rr = s.Rv[r];
        const double js = -Rr * double(u[i]) + double(D[r * incd]) * Rr * Rr;   // (J sigma)_r
        hs += -0.5 * js - double(s.Rv[r] * b[r]) + lam;
      }
    }
    // fixed-order reduction: wavefront partials, then wavefront 0
    for (int off = kWave / 2; off > 0; off >>= 1) hs += __shfl_down(hs, off, kWave);
    if ((t & (kWave - 1)) == 0) s.red[t / kWave] = hs;
    __syncthreads();
    if (t == 0) {
      double tot = 0.0;
      for (int w = 0; w < kBS / kWave; ++w) tot += s.red[w];
      H[q] = tot;
    }
  }
}

// ---- the MRI pipeline around the run: L2 diagonal, LASSO start, CG CDP ----

// ||D f||^2 of the unit-norm 1-D Haar function of `len` = 2^l samples at
// offset lo (high: + on its first half, - on its second), D the second
// difference with the reflecting boundary f[-1] = f[0], f[S] = f[S-1].
__device__ double d2_norm2(int lo, int len, bool high) {
  const double v = rsqrt(double(len));
  auto f = [&](int i) -> double {
    i = i < 0 ? 0 : (i >= kS ? kS - 1 : i);
    if (i < lo || i >= lo + len) return 0.0;
    return (high && i - lo >= len / 2) ? -v : v;
  };
  double acc = 0.0;
  const int i0 = lo > 0 ? lo - 1 : 0, i1 = lo + len < kS ? lo + len : kS - 1;
  for (int i = i0; i <= i1; ++i) {
    const double d = f(i - 1) - 2.0 * f(i) + f(i + 1);
    acc += d * d;
  }
  return acc;
}

// D_out[r] = D_in[r * incd] + gamma [Psi (D_v^T D_v + D_h^T D_h) Psi^T]_rr.  The
// Haar basis image of coefficient r is a product v(row) h(col) of unit-norm
// 1-D Haar functions, so the diagonal entry is ||D v||^2 + ||D h||^2.
__global__ void mri_l2_diag_kernel(int levels, double gamma, const float* __restrict__ D_in, int64_t incd,
                                   float* __restrict__ D_out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= kS * kS) return;
  const int i = r / kS, j = r - i * kS;
  int lev = levels, pi = i, pj = j;
  bool hv = false, hh = false;
  for (int l = 1; l <= levels; ++l) {
    const int h = kS >> l;
    if (i < 2 * h && j < 2 * h && (i >= h || j >= h)) {
      lev = l;
      hv = i >= h;
      hh = j >= h;
      pi = hv ? i - h : i;
      pj = hh ? j - h : j;
      break;
    }
  }
  const int len = 1 << lev;
  const double dl = d2_norm2(pi * len, len, hv) + d2_norm2(pj * len, len, hh);
  D_out[r] = float(double(D_in[size_t(r) * incd]) + gamma * dl);
}

// FP64 sum over the workgroup of per-thread partials; every thread gets it.
__device__ double block_sum(MriLds& s, double v) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) s.red[threadIdx.x / kWave] = v;
  __syncthreads();
  double tot = 0.0;
  for (int w = 0; w < kBS / kWave; ++w) tot += s.red[w];
  return tot;
}

// LASSO start of the MRI pipeline by FISTA: x minimises
// (1/2) x^T G_gamma x - b^T x + lam1 ||x||_1 after `iters` iterations from 0,
// step 1 / (1 + 32 gamma), G_gamma applied in factored form.  One workgroup.
__global__ void __launch_bounds__(kBS)
mri_lasso_kernel(const uint8_t* __restrict__ mask, int levels, float gamma, const float* __restrict__ b,
                 double lam1, int iters, float* __restrict__ R_out, MriStrides ms) {
  extern __shared__ __align__(16) unsigned char smem[];
  MriLds& s = *reinterpret_cast<MriLds*>(smem);
  const int t = threadIdx.x;
  if (const int k = blockIdx.x) {   // instance k
    mask += k * ms.mask;
    b += k * ms.vec;
    R_out += k * ms.vec;
  }
  const uint32_t mbits = init_tables(s, mask, t);
  __syncthreads();
  const double stepd = 1.0 / (1.0 + 32.0 * double(gamma));
  const float step = float(stepd), thr = float(stepd * lam1);
  float x[kPer], yk[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) x[i] = yk[i] = 0.0f;
  double tk = 1.0;
  for (int it = 0; it < iters; ++it) {
    float u[kPer], dq[kPer], zb[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) u[i] = yk[i];
    gram_apply(s, u, levels, mbits, gamma, opaque_tid(), b, 1, b, dq, zb);
    const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * tk * tk));
    const float mom = float((tk - 1.0) / tn);
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const float v = yk[i] - step * (u[i] - zb[i]);
      const float xn = v > thr ? v - thr : (v < -thr ? v + thr : 0.0f);
      yk[i] = xn + mom * (xn - x[i]);
      x[i] = xn;
    }
    tk = tn;
  }
  const int tf = opaque_tid();
#pragma unroll
  for (int i = 0; i < kPer; ++i) R_out[tf + kBS * i] = x[i];
}

// CG CDP of the MRI pipeline: (G_gamma)_SS R_S = b_S from the current R_S
// until ||r|| <= tol ||b_S|| or max_iter iterations, then off the support
// R_r = (b_r - (G_gamma R_S)_r) / D_r (held at 0 where D_r < 1e-12).  Dot
// products are accumulated in FP64 in a fixed order.  One workgroup.
__global__ void __launch_bounds__(kBS)
mri_cg_kernel(const uint8_t* __restrict__ mask, int levels, float gamma, const float* __restrict__ D, int64_t incd,
              const float* __restrict__ b, const uint8_t* __restrict__ sigma, float* __restrict__ R, int max_iter,
              double tol, int* __restrict__ iters_out, int* __restrict__ status, MriStrides ms) {
  extern __shared__ __align__(16) unsigned char smem[];
  MriLds& s = *reinterpret_cast<MriLds*>(smem);
  const int t = threadIdx.x;
  if (const int k = blockIdx.x) {   // instance k
    mask += k * ms.mask;
    D += k * ms.D;
    b += k * ms.vec;
    sigma += k * ms.vec;
    R += k * ms.vec;
    if (iters_out) iters_out += k * ms.it;
    status += k * ms.status;
  }
  const uint32_t mbits = init_tables(s, mask, t);
  __syncthreads();
  uint32_t sb = 0;
  float x[kPer], r[kPer], p[kPer];
  double bb = 0.0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int k = t + kBS * i;
    const bool on = sigma[k] != 0;
    sb |= on ? (1u << i) : 0u;
    x[i] = on ? R[k] : 0.0f;
  }
  {
    float u[kPer], dq[kPer], zb[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) u[i] = x[i];
    gram_apply(s, u, levels, mbits, gamma, opaque_tid(), D, incd, b, dq, zb);
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const bool on = (sb >> i) & 1u;
      r[i] = on ? zb[i] - u[i] : 0.0f;
      p[i] = r[i];
      bb += on ? double(zb[i]) * double(zb[i]) : 0.0;
    }
  }
  double rr = 0.0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) rr += double(r[i]) * double(r[i]);
  rr = block_sum(s, rr);
  bb = block_sum(s, bb);
  const double stop = tol * tol * bb;
  int it = 0;
  while (it < max_iter && rr > stop) {
    float u[kPer], dq[kPer], zb[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) u[i] = p[i];
    gram_apply(s, u, levels, mbits, gamma, opaque_tid(), D, incd, b, dq, zb);
    double pap = 0.0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      u[i] = ((sb >> i) & 1u) ? u[i] : 0.0f;
      pap += double(p[i]) * double(u[i]);
    }
    pap = block_sum(s, pap);
    if (!(pap > 0.0)) break;     // a breakdown (the support system is singular in FP32): keep x
    const float alpha = float(rr / pap);
    double rn = 0.0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      x[i] += alpha * p[i];
      r[i] -= alpha * u[i];
      rn += double(r[i]) * double(r[i]);
    }
    rn = block_sum(s, rn);
    const float beta = float(rn / rr);
#pragma unroll
    for (int i = 0; i < kPer; ++i) p[i] = r[i] + beta * p[i];
    rr = rn;
    ++it;
  }
  float u[kPer], dq[kPer], zb[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) u[i] = x[i];
  gram_apply(s, u, levels, mbits, gamma, opaque_tid(), D, incd, b, dq, zb);
  int bits = 0;
  const int tf = opaque_tid();
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int k = tf + kBS * i;
    const bool tiny = !(dq[i] >= 1e-12f);
    if (tiny) bits |= L0CIM_ST_TINY_DIAG;
    const float off = tiny ? 0.0f : (zb[i] - (u[i] - dq[i] * x[i])) / dq[i];
    R[k] = ((sb >> i) & 1u) ? x[i] : off;
  }
  if (bits) raise_status(status, bits);
  if (t == 0 && iters_out) *iters_out = it;
}

// Jacobi CDP with the couplings in factored form: `iters` synchronous sweeps
// R_r <- R_r + dtc [(b_r - ((G_gamma s)_r - D_r s_r)) / D_r - R_r], s = sigma o R,
// over every r (held at 0 where D_r < 1e-12).  One workgroup.
__global__ void __launch_bounds__(kBS)
mri_jacobi_kernel(const uint8_t* __restrict__ mask, int levels, float gamma, const float* __restrict__ D,
                  int64_t incd, const float* __restrict__ b, const uint8_t* __restrict__ sigma, float* __restrict__ R,
                  int iters, float dtc, int* __restrict__ status, MriStrides ms) {
  extern __shared__ __align__(16) unsigned char smem[];
  MriLds& s = *reinterpret_cast<MriLds*>(smem);
  const int t = threadIdx.x;
  if (const int k = blockIdx.x) {   // instance k
    mask += k * ms.mask;
    D += k * ms.D;
    b += k * ms.vec;
    sigma += k * ms.vec;
    R += k * ms.vec;
    status += k * ms.status;
  }
  const uint32_t mbits = init_tables(s, mask, t);
  __syncthreads();
  uint32_t sb = 0;
  float x[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int k = t + kBS * i;
    sb |= sigma[k] ? (1u << i) : 0u;
    x[i] = R[k];
  }
  int bits = 0;
  for (int it = 0; it < iters; ++it) {
    float u[kPer], dq[kPer], zb[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) u[i] = ((sb >> i) & 1u) ? x[i] : 0.0f;
    gram_apply(s, u, levels, mbits, gamma, opaque_tid(), D, incd, b, dq, zb);
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const float si = ((sb >> i) & 1u) ? x[i] : 0.0f;
      const bool tiny = !(dq[i] >= 1e-12f);
      if (tiny) bits |= L0CIM_ST_TINY_DIAG;
      x[i] = tiny ? 0.0f : x[i] + dtc * ((zb[i] - (u[i] - dq[i] * si)) / dq[i] - x[i]);
    }
  }
  const int tf = opaque_tid();
#pragma unroll
  for (int i = 0; i < kPer; ++i) R[tf + kBS * i] = x[i];
  if (bits) raise_status(status, bits);
}

// b = A^T y and D_r = sum_k A_kr^2 (FP64 accumulation), one column per thread.
__global__ void mri_aty_colnorm_kernel(int m, int n, const float* __restrict__ A, int64_t lda,
                                       const float* __restrict__ y, float* __restrict__ b, float* __restrict__ D) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double sb = 0.0, sd = 0.0;
  for (int k = 0; k < m; ++k) {
    const double a = A[size_t(k) * lda + r];
    sb = fma(a, double(y[k]), sb);
    sd = fma(a, a, sd);
  }
  b[r] = float(sb);
  D[r] = float(sd);
}

// R_r = b_r / D_r (0 where D_r < 1e-12).
__global__ void mri_r_init_kernel(int n, const float* __restrict__ b, const float* __restrict__ D,
                                  float* __restrict__ R, int* __restrict__ status) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const bool tiny = !(D[r] >= 1e-12f);
  R[r] = tiny ? 0.0f : b[r] / D[r];
  if (tiny) raise_status(status, L0CIM_ST_TINY_DIAG);
}

}  // namespace

size_t mri_lds_bytes() { return sizeof(MriLds); }

l0cim_status launch_mri_mfcim(int size, int levels, int P, const uint8_t* mask, const float* R,
                              const float* D, int64_t incd, const float* b, double gamma, const CimArgs& a, float* c,
                              float* e, uint8_t* sigma, double* H, float* trace, int* status, hipStream_t s,
                              int count, const MriStrides& ms) {
  if (size != kS) return set_error(L0CIM_ERR_UNSUPPORTED, "mri_mfcim_run: image side %d (128 supported)", size);
  if (count < 1 || count > 65535 || (count > 1 && trace))
    return set_error(L0CIM_ERR_ARG, "mri_mfcim_run: %d instances (a trace needs one)", count);
  const size_t lds = sizeof(MriLds);
  void (*k)(const uint8_t*, const float*, const float*, int64_t, const float*, float, CimArgs, int, float*, float*,
            uint8_t*, double*, float*, int*, MriStrides) =
      a.field == L0CIM_FIELD_BN ? mri_cim_kernel<int(L0CIM_FIELD_BN)> : mri_cim_kernel<int(L0CIM_FIELD_CN)>;
  L0_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(lds)));
  {
    ProfileScope prof(s);
    hipLaunchKernelGGL(k, dim3(P, count), dim3(kBS), lds, s, mask, R, D, incd, b, float(gamma), a, levels, c, e,
                       sigma, H, trace, status, ms);
  }
  L0_LAUNCHED("mri_cim_kernel");
  return L0CIM_OK;
}

l0cim_status launch_mri_l2_diag(int size, int levels, double gamma, const float* D_in, int64_t incd, float* D_out,
                                hipStream_t s) {
  if (size != kS) return set_error(L0CIM_ERR_UNSUPPORTED, "mri_l2_diag: image side %d (128 supported)", size);
  hipLaunchKernelGGL(mri_l2_diag_kernel, dim3(kS * kS / 256), dim3(256), 0, s, levels, gamma, D_in, incd, D_out);
  L0_LAUNCHED("mri_l2_diag_kernel");
  return L0CIM_OK;
}

l0cim_status launch_mri_lasso(int size, int levels, double gamma, const uint8_t* mask, const float* b, double lam1,
                              int iters, float* R_out, hipStream_t s, int count, const MriStrides& ms) {
  if (size != kS) return set_error(L0CIM_ERR_UNSUPPORTED, "mri_lasso: image side %d (128 supported)", size);
  const size_t lds = sizeof(MriLds);
  L0_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(mri_lasso_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  hipLaunchKernelGGL(mri_lasso_kernel, dim3(count), dim3(kBS), lds, s, mask, levels, float(gamma), b, lam1, iters,
                     R_out, ms);
  L0_LAUNCHED("mri_lasso_kernel");
  return L0CIM_OK;
}

l0cim_status launch_mri_jacobi(int size, int levels, double gamma, const uint8_t* mask, const float* D,
                               int64_t incd, const float* b, const uint8_t* sigma, float* R, int iters, double dtc,
                               int* status, hipStream_t s, int count, const MriStrides& ms) {
  if (size != kS) return set_error(L0CIM_ERR_UNSUPPORTED, "mri_cdp: image side %d (128 supported)", size);
  const size_t lds = sizeof(MriLds);
  L0_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(mri_jacobi_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  hipLaunchKernelGGL(mri_jacobi_kernel, dim3(count), dim3(kBS), lds, s, mask, levels, float(gamma), D, incd, b, sigma,
                     R, iters, float(dtc), status, ms);
  L0_LAUNCHED("mri_jacobi_kernel");
  return L0CIM_OK;
}

l0cim_status launch_mri_aty_colnorm(int m, int n, const float* A, int64_t lda, const float* y, float* b, float* D,
                                    hipStream_t s) {
  hipLaunchKernelGGL(mri_aty_colnorm_kernel, dim3((n + 255) / 256), dim3(256), 0, s, m, n, A, lda, y, b, D);
  L0_LAUNCHED("mri_aty_colnorm_kernel");
  return L0CIM_OK;
}

l0cim_status launch_mri_r_init(int n, const float* b, const float* D, float* R, int* status, hipStream_t s) {
  hipLaunchKernelGGL(mri_r_init_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, b, D, R, status);
  L0_LAUNCHED("mri_r_init_kernel");
  return L0CIM_OK;
}

l0cim_status launch_mri_cg(int size, int levels, double gamma, const uint8_t* mask, const float* D, int64_t incd,
                           const float* b, const uint8_t* sigma, float* R, int max_iter, double tol, int* iters_out,
                           int* status, hipStream_t s, int count, const MriStrides& ms) {
  if (size != kS) return set_error(L0CIM_ERR_UNSUPPORTED, "mri_cdp_cg: image side %d (128 supported)", size);
  const size_t lds = sizeof(MriLds);
  L0_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(mri_cg_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(lds)));
  hipLaunchKernelGGL(mri_cg_kernel, dim3(count), dim3(kBS), lds, s, mask, levels, float(gamma), D, incd, b, sigma, R,
                     max_iter, tol, iters_out, status, ms);
  L0_LAUNCHED("mri_cg_kernel");
  return L0CIM_OK;
}

}  // namespace l0
