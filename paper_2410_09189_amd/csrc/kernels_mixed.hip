// Mixed-precision grid contractions for gfx950: BF16x3 split products on the
// matrix cores with FP32 accumulation, FP64 partial-sum reduction.
//
// A value x is carried as hi = bf16(x), lo = bf16(x - hi); a product is
// approximated by hi*hi' + hi*lo' + lo*hi' (the lo*lo' term, ~2^-16 relative,
// is dropped), which keeps about 16 significant bits per product.  These
// kernels only ever see perturbations from the ground state (density-matrix
// change, potential change), whose static parts stay in FP64 elsewhere.
#include "kernels.h"
#include "kernels_mixed.h"

#include <hip/hip_runtime.h>

namespace rtk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__host__ __device__ static inline int cdivm(long a, long b) { return (int)((a + b - 1) / b); }

// Round-to-nearest-even float -> bf16 bits (finite inputs).
__device__ __forceinline__ unsigned short f2bf(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

__device__ __forceinline__ void split2(float x, unsigned short& hi, unsigned short& lo) {
  hi = f2bf(x);
  lo = f2bf(x - bf2f(hi));
}

__global__ void k_split_bf16(const double* __restrict__ x, unsigned short* __restrict__ hi,
                             unsigned short* __restrict__ lo, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double v = x[i];
    unsigned short h = f2bf((float)v);
    double r = v - (double)bf2f(h);
    hi[i] = h;
    lo[i] = f2bf((float)r);
  }
}

hipError_t split_bf16(hipStream_t s, const double* x, unsigned short* hi, unsigned short* lo, long n) {
  long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_split_bf16, dim3((int)b), dim3(256), 0, s, x, hi, lo, n);
  return hipGetLastError();
}

// W_ij = (S_ij - S0_ij) * (2 if i < j, 1 if i == j, 0 if i > j), split to bf16 hi/lo,
// padded to ld >= N (rows and columns N..ld-1 zero).  blockIdx.y = trajectory:
// S_t = S + t sstride, hi/lo_t = + t ld^2, S0 shared.
// frag = 0: row-major [ld][ld].  frag = 1 (ld % 32 == 0): 32x32x16 A-fragment order,
// one contiguous 64-lane x 8 block per (32-row block I, 16-column step c):
//   offset = ((I (ld/16) + c) 64 + (i % 32) + 32 ((j % 16) / 8)) 8 + j % 8.
__global__ void k_upper_weighted_delta_bf16(const double* S, const double* S0, unsigned short* hi,
                                            unsigned short* lo, int N, int ld, long sstride, const int* active,
                                            int frag) {
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)ld * ld) return;
  S += t * sstride;
  hi += t * (long)ld * ld;
  lo += t * (long)ld * ld;
  int i = (int)(e / ld), j = (int)(e - (long)i * ld);
  double w = 0.0;
  if (i < N && j < N) {
    long f = (long)i * N + j;
    w = i < j ? 2.0 * (S[f] - S0[f]) : (i == j ? S[f] - S0[f] : 0.0);
  }
  unsigned short h = f2bf((float)w);
  long o = e;
  if (frag) o = (((long)(i >> 5) * (ld >> 4) + (j >> 4)) * 64 + (i & 31) + 32 * ((j & 15) >> 3)) * 8 + (j & 7);
  hi[o] = h;
  lo[o] = f2bf((float)(w - (double)bf2f(h)));
}

hipError_t upper_weighted_delta_bf16(hipStream_t s, const double* S, const double* S0, unsigned short* hi,
                                     unsigned short* lo, int N, int ld, long sstride, int T, const int* active,
                                     int frag) {
  if (frag && ld % 32) return hipErrorInvalidValue;
  long n = (long)ld * ld;
  hipLaunchKernelGGL(k_upper_weighted_delta_bf16, dim3(cdivm(n, 256), T), dim3(256), 0, s, S, S0, hi, lo, N, ld,
                     sstride, active, frag);
  return hipGetLastError();
}

// Point-major split of the orbitals: hiT/loT[r][j] (pitch ld) = bf16 hi/lo of psi[j][r]
// for j < N, zero for N <= j < ld.  64-point x 32-orbital tiles transposed through LDS.
__global__ __launch_bounds__(256) void k_split_bf16_t(const double* __restrict__ psi, unsigned short* __restrict__ hiT,
                                                      unsigned short* __restrict__ loT, int N, int ld, long ng) {
  __shared__ unsigned short sh[32][66], sl[32][66];
  const long p0 = (long)blockIdx.x * 64;
  const int j0 = blockIdx.y * 32, tid = threadIdx.x;
  for (int e = tid; e < 32 * 64; e += 256) {
    int jj = e >> 6, pp = e & 63;
    int j = j0 + jj;
    long r = p0 + pp;
    double v = (j < N && r < ng) ? psi[(long)j * ng + r] : 0.0;
    unsigned short h = f2bf((float)v);
    sh[jj][pp] = h;
    sl[jj][pp] = f2bf((float)(v - (double)bf2f(h)));
  }
  __syncthreads();
  for (int e = tid; e < 32 * 64; e += 256) {
    int pp = e >> 5, jj = e & 31;
    long r = p0 + pp;
    if (r < ng) {
      hiT[r * ld + j0 + jj] = sh[jj][pp];
      loT[r * ld + j0 + jj] = sl[jj][pp];
    }
  }
}

hipError_t split_bf16_t(hipStream_t s, const double* psi, unsigned short* hiT, unsigned short* loT, int N, int ld,
                        long ng) {
  if (ld % 32 || ld < N) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_split_bf16_t, dim3(cdivm(ng, 64), ld / 32), dim3(256), 0, s, psi, hiT, loT, N, ld, ng);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Symmetric weighted projection: part[s][m][n] = sum_{k in split s} A[m][k] w[k] A[n][k]
// over upper tiles (tn >= tm), A given as bf16 hi/lo rows [N][ng] (ng % 8 == 0).
// Block 256 threads = 2 x 2 waves, tile 128 x 128, K chunk 64; each wave owns a
// 64 x 64 sub-tile = 4 x 4 MFMA 16x16x32 blocks, 3 MFMAs per block per K/32.
// Fragment layout of v_mfma_f32_16x16x32_bf16: lane l holds row (l & 15) and
// k = 8 (l >> 4) .. 8 (l >> 4) + 7 of each operand; the result row is
// 4 (l >> 4) + r, column l & 15.
// ---------------------------------------------------------------------------
constexpr int XB = 128, XK = 64, XPAD = 8;

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

typedef float f32x2 __attribute__((ext_vector_type(2)));

// (hi + lo) * w of two packed bf16 pairs, re-split to packed bf16 hi/lo (round to
// nearest even on the hardware converter, both halves in one conversion).
__device__ __forceinline__ void split_scaled2(unsigned int h, unsigned int l, float w0, float w1, unsigned int& oh,
                                              unsigned int& ol) {
  const float x0 = (__uint_as_float(h << 16) + __uint_as_float(l << 16)) * w0;
  const float x1 = (__uint_as_float(h & 0xFFFF0000u) + __uint_as_float(l & 0xFFFF0000u)) * w1;
  const f32x2 x = {x0, x1};
  const unsigned int hb = __builtin_bit_cast(unsigned int, __builtin_convertvector(x, bf16x2));
  const f32x2 r = {x0 - __uint_as_float(hb << 16), x1 - __uint_as_float(hb & 0xFFFF0000u)};
  oh = hb;
  ol = __builtin_bit_cast(unsigned int, __builtin_convertvector(r, bf16x2));
}

// Raw buffer resource over [base, base + bytes): loads at offsets >= bytes return 0.
// Word 3 is the gfx9 raw-buffer format word.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ uint4 buf_ld16(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Fragment layout of v_mfma_f32_32x32x16_bf16: lane l holds row (A) / column (B)
// l & 31 and k = 8 (l >> 5) .. 8 (l >> 5) + 7; result register r of lane l is
// row 8 (r >> 2) + 4 (l >> 5) + (r & 3), column l & 31.  It retires twice the
// products of the 16x16x32 form per issue cycle.
__device__ __forceinline__ f32x16 mfma32(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Projection kernel: per thread one 32-bit row offset for the whole loop (the K
// position rides in the scalar offset of buffer loads), rows >= N read as zero
// through the resource bound, the weights fetched once per K chunk (all four
// vectors a thread stages share its K columns), the next chunk in flight in
// registers during the MFMAs, XCD-aware block order.  Each wave owns 64 x 64 of
// the 128 x 128 tile as 2 x 2 blocks of 32x32x16 products.  Needs 256 ng < 2^31.
__global__ __launch_bounds__(256, 2) void k_proj_bf16x3(int N, long ng, const unsigned short* __restrict__ Ahi,
                                                        const unsigned short* __restrict__ Alo,
                                                        const float* __restrict__ w, float* __restrict__ part,
                                                        long kps, int ntm, int T, const int* active) {
  __shared__ __attribute__((aligned(16))) unsigned short sAh[XB][XK + XPAD], sAl[XB][XK + XPAD];
  __shared__ __attribute__((aligned(16))) unsigned short sBh[XB][XK + XPAD], sBl[XB][XK + XPAD];
  const long h = blockIdx.x + (long)gridDim.x * blockIdx.y;
  const long lid = xcd_logical(h, (long)gridDim.x * gridDim.y);
  const int bx = (int)(lid % gridDim.x), by = (int)(lid / gridDim.x);
  const int tb = bx % T;
  if (active && !active[tb]) return;
  part += (long)tb * gridDim.y * N * N;
  int tm = 0, tn;
  {
    int t = bx / T, rowlen = ntm;
    while (t >= rowlen) { t -= rowlen; ++tm; --rowlen; }
    tn = tm + t;
  }
  const long k0 = (long)by * kps;
  const long k1 = min(ng, k0 + kps);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const long m0 = (long)tm * XB, n0 = (long)tn * XB;
  const long va = min((long)XB, N - m0), vb = min((long)XB, N - n0);
  // matrix work only where the upper triangle has entries: on a diagonal tile the
  // wave below the diagonal idles and the diagonal waves skip their strictly lower
  // 16 x 16 blocks; 16-row / 16-column blocks past N are skipped everywhere
  const bool idle = (tm == tn) && (wm > wn);
  const bool lowdiag = (tm == tn) && (wm == wn);
  const int nib = (int)min(2L, max(0L, (N - m0 - wm * 64 + 31) / 32));
  const int njb = (int)min(2L, max(0L, (N - n0 - wn * 64 + 31) / 32));
  const auto rAh = buf_rsrc(Ahi + m0 * ng + k0, (int)((va * ng - k0) * 2));
  const auto rAl = buf_rsrc(Alo + m0 * ng + k0, (int)((va * ng - k0) * 2));
  const auto rBh = buf_rsrc(Ahi + n0 * ng + k0, (int)((vb * ng - k0) * 2));
  const auto rBl = buf_rsrc(Alo + n0 * ng + k0, (int)((vb * ng - k0) * 2));
  const auto rW = buf_rsrc(w + (long)tb * ng + k0, (int)((ng - k0) * 4));
  const int c8 = (tid & 7) * 8, r0 = tid >> 3;  // vector u covers row r0 + 32 u, columns c8..c8+7
  int vo[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) vo[u] = (int)(((long)(r0 + 32 * u) * ng + c8) * 2);
  uint4 rah[4], ral[4], rbh[4], rbl[4];
  uint4 rw0, rw1;
  auto fetch = [&](long kb) {
    const int so = (int)((kb - k0) * 2);
    int v[4];
    const bool tail = kb + XK > k1;
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = (tail && kb + c8 >= k1) ? (int)0x80000000 : vo[u];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      rah[u] = buf_ld16(rAh, v[u], so);
      ral[u] = buf_ld16(rAl, v[u], so);
      rbh[u] = buf_ld16(rBh, v[u], so);
      rbl[u] = buf_ld16(rBl, v[u], so);
    }
    // the range check covers the vector offset only, so columns past the end of the
    // split take an out-of-range vector offset (zero, no memory access) as the rows do
    const int wv = (tail && kb + c8 >= k1) ? (int)0x80000000 : c8 * 4;
    rw0 = buf_ld16(rW, wv, 2 * so);
    rw1 = buf_ld16(rW, wv + 16, 2 * so);
  };
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  fetch(k0);
  for (long kb = k0; kb < k1; kb += XK) {
    const float w0 = __uint_as_float(rw0.x), w1 = __uint_as_float(rw0.y), w2 = __uint_as_float(rw0.z),
                w3 = __uint_as_float(rw0.w), w4 = __uint_as_float(rw1.x), w5 = __uint_as_float(rw1.y),
                w6 = __uint_as_float(rw1.z), w7 = __uint_as_float(rw1.w);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + 32 * u;
      *reinterpret_cast<uint4*>(&sAh[r][c8]) = rah[u];
      *reinterpret_cast<uint4*>(&sAl[r][c8]) = ral[u];
      uint4 bh, bl;
      split_scaled2(rbh[u].x, rbl[u].x, w0, w1, bh.x, bl.x);
      split_scaled2(rbh[u].y, rbl[u].y, w2, w3, bh.y, bl.y);
      split_scaled2(rbh[u].z, rbl[u].z, w4, w5, bh.z, bl.z);
      split_scaled2(rbh[u].w, rbl[u].w, w6, w7, bh.w, bl.w);
      *reinterpret_cast<uint4*>(&sBh[r][c8]) = bh;
      *reinterpret_cast<uint4*>(&sBl[r][c8]) = bl;
    }
    __syncthreads();
    if (kb + XK < k1) fetch(kb + XK);
#pragma unroll
    for (int kk = 0; kk < XK && !idle; kk += 16) {
      bf16x8 fah[2], fal[2], fbh[2], fbl[2];
      const int kc = kk + 8 * (lane >> 5);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        int r = wm * 64 + i * 32 + (lane & 31);
        fah[i] = *reinterpret_cast<const bf16x8*>(&sAh[r][kc]);
        fal[i] = *reinterpret_cast<const bf16x8*>(&sAl[r][kc]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        int r = wn * 64 + j * 32 + (lane & 31);
        fbh[j] = *reinterpret_cast<const bf16x8*>(&sBh[r][kc]);
        fbl[j] = *reinterpret_cast<const bf16x8*>(&sBl[r][kc]);
      }
      // the three BF16x3 terms outermost: consecutive products update different tiles
#pragma unroll
      for (int term = 0; term < 3; ++term)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            if (i >= nib || j >= njb || (lowdiag && i > j)) continue;
            acc[i][j] = mfma32(term == 0 ? fal[i] : fah[i], term == 1 ? fbl[j] : fbh[j], acc[i][j]);
          }
    }
    __syncthreads();
  }
  if (idle) return;
  float* P = part + (long)by * N * N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        long row = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        long col = n0 + wn * 64 + j * 32 + (lane & 31);
        if (row < N && col < N) P[row * N + col] = acc[i][j][r];
      }
}

// ---------------------------------------------------------------------------
// Projection for N <= 256 (block grid NB = ceil(N / 32) <= 8).  One block owns
// one trajectory and one range of grid points and accumulates every 32 x 32 block
// of the upper triangle with v_mfma_f32_32x32x16_bf16.  The block's eight waves
// have two roles, one of each on every SIMD:
//  * four matrix waves: wave W owns block rows W and NB - 1 - W (row r holds
//    NB - r blocks, so a pair holds NB + 1: at NB = 8 every wave 9 blocks); its
//    blocks are compile-time parameters of its code, so the accumulators are
//    indexed statically;
//  * four staging waves: global loads one chunk ahead, the weighted copy of the
//    orbitals re-split to bf16 hi/lo, LDS writes.
// Points pass through LDS TKC at a time, double buffered with one barrier per
// chunk, so the staging of chunk c + 1 runs beside the matrix work on chunk c.
// LDS holds the raw orbital hi/lo (A side) and the weighted copy (B side), each
// 16-byte piece XOR-swizzled by row so fragment reads and staging writes are free
// of bank conflicts.  Each block covers a long range of points (about one block
// per CU in one round), so few FP32 partials are written.
// ---------------------------------------------------------------------------
constexpr int TKC = 32;       // points per staged chunk
constexpr int TMW = 4;        // matrix waves
constexpr int TSW = 4;        // staging waves
constexpr int TTH = 64 * (TMW + TSW);

// element offset of (row r, 16-byte piece q) in a staged [rows][TKC] bf16 array
// (the XOR of bits 1 and 2 of the row keeps any 16 consecutive rows of one piece
// column, a fragment read's quarter wave, on 16 distinct 16-byte bank groups)
__device__ __forceinline__ int tri_off(int r, int q) { return r * TKC + 8 * (q ^ (((r >> 1) ^ (r >> 2)) & 3)); }

// Matrix wave W: block rows I0 = W and I1 = NB - 1 - W (used when I0 <= I1, the
// second only when I1 > I0); acc[J - I0] holds (I0, J), acc[NB - W + J - I1]
// holds (I1, J).
template <int NB, int W>
struct TriWave {
  static constexpr int I0 = W, I1 = NB - 1 - W;
  static constexpr bool one = I0 <= I1, two = I0 < I1;
};

template <int NB, int W>
__device__ __forceinline__ void tri_mfma(f32x16 (&acc)[NB + 1], const unsigned short* __restrict__ sm, int lane) {
  using TW = TriWave<NB, W>;
  constexpr int I0 = TW::I0, I1 = TW::I1;
  constexpr int R = NB * 32 * TKC;  // elements per staged array
  const unsigned short* sAh = sm;
  const unsigned short* sAl = sm + R;
  const unsigned short* sBh = sm + 2 * R;
  const unsigned short* sBl = sm + 3 * R;
  const int l32 = lane & 31, hk = lane >> 5;
#pragma unroll 1
  for (int st = 0; st < TKC / 16; ++st) {
    const int q = 2 * st + hk;
    bf16x8 a0h, a0l, a1h, a1l;
    a0h = *reinterpret_cast<const bf16x8*>(sAh + tri_off(32 * I0 + l32, q));
    a0l = *reinterpret_cast<const bf16x8*>(sAl + tri_off(32 * I0 + l32, q));
    if constexpr (TW::two) {
      a1h = *reinterpret_cast<const bf16x8*>(sAh + tri_off(32 * I1 + l32, q));
      a1l = *reinterpret_cast<const bf16x8*>(sAl + tri_off(32 * I1 + l32, q));
    }
#pragma unroll
    for (int J = I0; J < NB; ++J) {
      const bf16x8 bh = *reinterpret_cast<const bf16x8*>(sBh + tri_off(32 * J + l32, q));
      const bf16x8 bl = *reinterpret_cast<const bf16x8*>(sBl + tri_off(32 * J + l32, q));
      if constexpr (TW::two) {
        if (J >= I1) {
          // two independent accumulation chains interleaved
          acc[J - I0] = mfma32(a0l, bh, acc[J - I0]);
          acc[NB - W + J - I1] = mfma32(a1l, bh, acc[NB - W + J - I1]);
          acc[J - I0] = mfma32(a0h, bl, acc[J - I0]);
          acc[NB - W + J - I1] = mfma32(a1h, bl, acc[NB - W + J - I1]);
          acc[J - I0] = mfma32(a0h, bh, acc[J - I0]);
          acc[NB - W + J - I1] = mfma32(a1h, bh, acc[NB - W + J - I1]);
          continue;
        }
      }
      acc[J - I0] = mfma32(a0l, bh, acc[J - I0]);
      acc[J - I0] = mfma32(a0h, bl, acc[J - I0]);
      acc[J - I0] = mfma32(a0h, bh, acc[J - I0]);
    }
  }
}

template <int NB, int W>
__device__ __forceinline__ void tri_store(const f32x16 (&acc)[NB + 1], float* __restrict__ P, int N, int lane) {
  using TW = TriWave<NB, W>;
  constexpr int I0 = TW::I0, I1 = TW::I1;
  const int c0 = lane & 31, r0 = 4 * (lane >> 5);
#pragma unroll
  for (int J = I0; J < NB; ++J) {
    const int col = 32 * J + c0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 32 * I0 + 8 * (r >> 2) + r0 + (r & 3);
      if (row < N && col < N) P[(long)row * N + col] = acc[J - I0][r];
    }
  }
  if constexpr (TW::two) {
#pragma unroll
    for (int J = I1; J < NB; ++J) {
      const int col = 32 * J + c0;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * I1 + 8 * (r >> 2) + r0 + (r & 3);
        if (row < N && col < N) P[(long)row * N + col] = acc[NB - W + J - I1][r];
      }
    }
  }
}

// Matrix wave: nc chunks, one barrier before the first and one after each (a wave
// without blocks, at small NB, only takes part in the barriers).
template <int NB, int W>
__device__ __forceinline__ void tri_matrix(int N, int nc, unsigned short (*sm)[4 * NB * 32 * TKC],
                                           float* __restrict__ P) {
  const int lane = threadIdx.x & 63;
  f32x16 acc[NB + 1];
#pragma unroll
  for (int a = 0; a < NB + 1; ++a)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[a][r] = 0.f;
  __syncthreads();
  for (int c = 0; c < nc; ++c) {
    if constexpr (TriWave<NB, W>::one) tri_mfma<NB, W>(acc, sm[c & 1], lane);
    __syncthreads();
  }
  if constexpr (TriWave<NB, W>::one) tri_store<NB, W>(acc, P, N, lane);
}

// one staging thread's share of a chunk: U pieces of A hi/lo and the 8 weights
template <int U>
struct TriRegs {
  uint4 h[U], l[U], w0, w1;
};

// Staging waves: the same barrier sequence as the matrix waves.  Chunk c is
// loaded into registers while the matrix waves work on chunk c - 2 and written
// to LDS buffer c & 1 while they work on chunk c - 1; its loads are issued once
// the registers are free (after the previous chunk was written), so each wait
// covers exactly the loads of the chunk being staged.  (With two register sets in
// flight the compiler's wait counts serialise the loads of both sets.)
template <int NB>
__device__ __forceinline__ void tri_stage(int N, const __amdgpu_buffer_rsrc_t& rAh,
                                          const __amdgpu_buffer_rsrc_t& rAl, const __amdgpu_buffer_rsrc_t& rW,
                                          int nc, unsigned short (*sm)[4 * NB * 32 * TKC]) {
  constexpr int R = NB * 32 * TKC;             // elements per staged array
  constexpr int PIECES = NB * 32 * TKC / 8;    // 16-byte pieces per staged array
  constexpr int NS = 64 * TSW;                 // staging threads
  constexpr int U = (PIECES + NS - 1) / NS;    // pieces per staging thread
  const int tid = threadIdx.x - 64 * TMW;
  const int q = tid & 3;  // every piece of this thread sits at piece column q
  // piece (row r, column q) of chunk c sits at byte (c N + r) 2 TKC + 16 q of the
  // K-blocked orbitals (rows >= N read zero through an out-of-range offset)
  int vo[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = tid + NS * u;
    vo[u] = (e < PIECES && (e >> 2) < N) ? (e >> 2) * 2 * TKC + 16 * q : (int)0x80000000;
  }
  const int stride = N * 2 * TKC;  // bytes per chunk of K-blocked orbitals
  auto fetch = [&](TriRegs<U>& g, int c) {
    // the chunk offset is uniform (readfirstlane keeps it in a scalar register);
    // the weights carry it in the vector offset so that points past ng, the
    // resource's end, read zero
    const int so = __builtin_amdgcn_readfirstlane(c * stride);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      g.h[u] = buf_ld16(rAh, vo[u], so);
      g.l[u] = buf_ld16(rAl, vo[u], so);
    }
    const int wv = 32 * q + c * 4 * TKC;
    g.w0 = buf_ld16(rW, wv, 0);
    g.w1 = buf_ld16(rW, wv + 16, 0);
  };
  auto stage = [&](const TriRegs<U>& g, unsigned short* s) {
    const float w0 = __uint_as_float(g.w0.x), w1 = __uint_as_float(g.w0.y), w2 = __uint_as_float(g.w0.z),
                w3 = __uint_as_float(g.w0.w), w4 = __uint_as_float(g.w1.x), w5 = __uint_as_float(g.w1.y),
                w6 = __uint_as_float(g.w1.z), w7 = __uint_as_float(g.w1.w);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = tid + NS * u;
      if (PIECES % NS != 0 && e >= PIECES) break;  // (no divergent branch when every thread has U)
      const int o = tri_off(e >> 2, q);
      *reinterpret_cast<uint4*>(s + o) = g.h[u];
      *reinterpret_cast<uint4*>(s + R + o) = g.l[u];
      uint4 bh, bl;
      split_scaled2(g.h[u].x, g.l[u].x, w0, w1, bh.x, bl.x);
      split_scaled2(g.h[u].y, g.l[u].y, w2, w3, bh.y, bl.y);
      split_scaled2(g.h[u].z, g.l[u].z, w4, w5, bh.z, bl.z);
      split_scaled2(g.h[u].w, g.l[u].w, w6, w7, bh.w, bl.w);
      *reinterpret_cast<uint4*>(s + 2 * R + o) = bh;
      *reinterpret_cast<uint4*>(s + 3 * R + o) = bl;
    }
  };
  TriRegs<U> g;
  fetch(g, 0);
  stage(g, sm[0]);
  if (nc > 1) fetch(g, 1);
  __syncthreads();
  for (int c = 0; c < nc; ++c) {
    // the matrix waves work on buffer c & 1: stage chunk c + 1 into the other one
    if (c + 1 < nc) {
      stage(g, sm[(c + 1) & 1]);
      if (c + 2 < nc) fetch(g, c + 2);
    }
    __syncthreads();
  }
}

template <int NB>
__global__ __launch_bounds__(TTH, 1) void k_proj_tri(int N, long ng, const unsigned short* __restrict__ Ahi,
                                                     const unsigned short* __restrict__ Alo,
                                                     const float* __restrict__ w, float* __restrict__ part, long kps,
                                                     int T, const int* active) {
  __shared__ __attribute__((aligned(16))) unsigned short sm[2][4 * NB * 32 * TKC];
  const long lid = xcd_logical(blockIdx.x, gridDim.x);
  const int tb = (int)(lid % T), sp = (int)(lid / T);
  if (active && !active[tb]) return;
  const long k0 = (long)sp * kps;
  const long k1 = min(ng, k0 + kps);
  const int nc = (int)((k1 - k0 + TKC - 1) / TKC);
  float* P = part + ((long)tb * (gridDim.x / T) + sp) * N * N;
  // every role below runs 1 + nc barriers; the role index is wave-uniform
  // (readfirstlane), so each wave executes only its own branch
  switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
    case 0: tri_matrix<NB, 0>(N, nc, sm, P); break;
    case 1: tri_matrix<NB, 1>(N, nc, sm, P); break;
    case 2: tri_matrix<NB, 2>(N, nc, sm, P); break;
    case 3: tri_matrix<NB, 3>(N, nc, sm, P); break;
    default: {
      // K-blocked orbitals from this block's first chunk on
      const long e0 = k0 / TKC * N * TKC, ne = (ng + TKC - 1) / TKC * N * TKC;
      const auto rAh = buf_rsrc(Ahi + e0, (int)((ne - e0) * 2));
      const auto rAl = buf_rsrc(Alo + e0, (int)((ne - e0) * 2));
      const auto rW = buf_rsrc(w + (long)tb * ng + k0, (int)((ng - k0) * 4));
      tri_stage<NB>(N, rAh, rAl, rW, nc, sm);
      break;
    }
  }
}

// K-blocked bf16 hi/lo orbitals for the triangle projection: piece q (8 points)
// of row r in chunk c (TKC points) at element (c N + r) TKC + 8 q, zero past ng.
__global__ void k_split_bf16_kb(const double* __restrict__ psi, unsigned short* __restrict__ hi,
                                unsigned short* __restrict__ lo, int N, long ng, long n_pieces) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pieces) return;
  const int q = (int)(p & 3);
  const long rc = p >> 2;  // c N + r
  const long c = rc / N;
  const int r = (int)(rc - c * N);
  const long k = c * TKC + 8 * q;
  unsigned short h[8], l[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const double v = k + i < ng ? psi[(long)r * ng + k + i] : 0.0;
    h[i] = f2bf((float)v);
    l[i] = f2bf((float)(v - (double)bf2f(h[i])));
  }
  uint4 vh, vl;
  vh.x = h[0] | ((unsigned)h[1] << 16); vh.y = h[2] | ((unsigned)h[3] << 16);
  vh.z = h[4] | ((unsigned)h[5] << 16); vh.w = h[6] | ((unsigned)h[7] << 16);
  vl.x = l[0] | ((unsigned)l[1] << 16); vl.y = l[2] | ((unsigned)l[3] << 16);
  vl.z = l[4] | ((unsigned)l[5] << 16); vl.w = l[6] | ((unsigned)l[7] << 16);
  *reinterpret_cast<uint4*>(hi + rc * TKC + 8 * q) = vh;
  *reinterpret_cast<uint4*>(lo + rc * TKC + 8 * q) = vl;
}

long proj_tri_elems(int N, long ng) { return (ng + TKC - 1) / TKC * N * TKC; }

hipError_t split_bf16_kb(hipStream_t s, const double* psi, unsigned short* hi, unsigned short* lo, int N, long ng) {
  const long n_pieces = proj_tri_elems(N, ng) / 8;
  hipLaunchKernelGGL(k_split_bf16_kb, dim3(cdivm(n_pieces, 256)), dim3(256), 0, s, psi, hi, lo, N, ng, n_pieces);
  return hipGetLastError();
}

int proj_tri_max_n() { return 256; }
int proj_tri_chunk() { return TKC; }

hipError_t proj_tri_bf16x3(hipStream_t s, int N, long ng, const unsigned short* hi, const unsigned short* lo,
                           const float* w, float* part, long kps, int n_split, int T, const int* active) {
  if (N < 1 || N > 256 || 2 * proj_tri_elems(N, ng) >= (1L << 31) || 4 * ng >= (1L << 31) || kps % TKC || kps < TKC || n_split < 1 ||
      (long)(n_split - 1) * kps >= ng || (long)n_split * kps < ng)
    return hipErrorInvalidValue;
  const dim3 grid(T * n_split), blk(TTH);
  switch ((N + 31) / 32) {
#define RT_TRI_NB(nb)                                                                                            \
  case nb:                                                                                                       \
    hipLaunchKernelGGL(k_proj_tri<nb>, grid, blk, 0, s, N, ng, hi, lo, w, part, kps, T, active);                \
    break;
    RT_TRI_NB(1) RT_TRI_NB(2) RT_TRI_NB(3) RT_TRI_NB(4) RT_TRI_NB(5) RT_TRI_NB(6) RT_TRI_NB(7) RT_TRI_NB(8)
#undef RT_TRI_NB
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t proj_bf16x3(hipStream_t s, int N, long ng, const unsigned short* hi, const unsigned short* lo,
                       const float* w, float* part, long kps, int n_split, int T, const int* active) {
  if (ng % 8 || 256 * ng >= (1L << 31) || kps % XK) return hipErrorInvalidValue;
  int ntm = cdivm(N, XB);
  int nt = ntm * (ntm + 1) / 2;
  hipLaunchKernelGGL(k_proj_bf16x3, dim3(nt * T, n_split), dim3(256), 0, s, N, ng, hi, lo, w, part, kps, ntm, T,
                     active);
  return hipGetLastError();
}

// C[m][n] = alpha * sum_s part[s][m][n] (FP64 sum of FP32 partials), upper kept and mirrored, plus base.
// Block = 64 consecutive elements x 4 wave groups; group g adds splits g, g + 4, ... in
// order, the four group sums are combined in group order (deterministic).
__global__ __launch_bounds__(256) void k_reduce_parts_f32(const float* __restrict__ part, int n_split, int N,
                                                          double alpha, const double* base, double* C,
                                                          const int* active, long sbase) {
  __shared__ double sh[4][64];
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  const long NN = (long)N * N;
  part += (long)t * n_split * NN;
  C += t * NN;
  base += t * sbase;
  const int x = threadIdx.x & 63, g = threadIdx.x >> 6;
  const long e = (long)blockIdx.x * 64 + x;
  double acc = 0.0;
  if (e < NN)
    for (int q = g; q < n_split; q += 4) acc += (double)part[(long)q * NN + e];
  sh[g][x] = acc;
  __syncthreads();
  if (g != 0 || e >= NN) return;
  const int m = (int)(e / N), n = (int)(e - (long)m * N);
  if (m > n) return;
  const double v = alpha * (((sh[0][x] + sh[1][x]) + sh[2][x]) + sh[3][x]);
  C[e] = base[e] + v;
  if (m < n) C[(long)n * N + m] = base[(long)n * N + m] + v;
}

hipError_t reduce_parts_f32(hipStream_t s, const float* part, int n_split, int N, double alpha,
                            const double* base, double* C, int T, const int* active, long sbase) {
  long n = (long)N * N;
  hipLaunchKernelGGL(k_reduce_parts_f32, dim3(cdivm(n, 64), T), dim3(256), 0, s, part, n_split, N, alpha, base, C,
                     active, sbase);
  return hipGetLastError();
}

// Resident-tile density for N <= 256.  One block owns BN grid points and every
// trajectory: the point-major hi/lo orbital tile [BN][NP] (NP = 32 NC, zero padded)
// is loaded into LDS once; for each trajectory Z = W Psi_tile is accumulated with
// 32x32x16 matrix instructions, W (upper triangular, stored in A-fragment order) read
// straight from L2, j-chunks of 32 outermost so each B fragment read from LDS serves
// all of a wave's row blocks, lower-triangle blocks skipped; then
// rho_t = rho0 + sum_i psi_i Z_i with psi_i again from the LDS tile.
// Waves: 4 row groups x WP point groups; row group g owns the 32-row blocks g and
// 7 - g (equal triangular work), a point group owns BN / WP points.
// The chunk loop is unrolled (NC is a template argument) so the W fragments of chunk
// c + PF load into a fixed register slot while chunks c + 1 .. c + PF - 1 compute:
// no register rotation, hence no wait for loads still in flight.  With 64-point tiles
// (67 KB of LDS) two blocks share a CU, so one block's tile load overlaps the other's
// matrix work.
template <int BN, int WP, int NC, int PF, int MINB>
__global__ __launch_bounds__(256 * WP, MINB) void k_density_tile32(long ng, const unsigned short* __restrict__ whi,
                                                             const unsigned short* __restrict__ wlo,
                                                             const unsigned short* __restrict__ pth,
                                                             const unsigned short* __restrict__ ptl,
                                                             const double* __restrict__ rho0,
                                                             double* __restrict__ rho, int T, const int* active) {
  constexpr int NP = 32 * NC;
  constexpr int LDP = NP + 8;  // LDS row pitch (bf16)
  constexpr int RB = 2, PC = BN / 32 / WP, NTH = 256 * WP;
  __shared__ __attribute__((aligned(16))) unsigned short sT[2][BN][LDP];
  __shared__ float red[4][BN];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave & 3, wp = wave >> 2;
  const long p0 = (long)blockIdx.x * BN;
  {
    constexpr int QN = NP / 8, U = BN * QN / NTH;  // 16-byte pieces per tile row, per thread
    static_assert(BN * QN % NTH == 0, "tile pieces must divide over the block");
    uint4 vh[U], vl[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = tid + NTH * u;
      const long r = p0 + e / QN;
      vh[u] = vl[u] = make_uint4(0u, 0u, 0u, 0u);
      if (r < ng) {
        vh[u] = *reinterpret_cast<const uint4*>(pth + r * NP + 8 * (e % QN));
        vl[u] = *reinterpret_cast<const uint4*>(ptl + r * NP + 8 * (e % QN));
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = tid + NTH * u;
      *reinterpret_cast<uint4*>(&sT[0][e / QN][8 * (e % QN)]) = vh[u];
      *reinterpret_cast<uint4*>(&sT[1][e / QN][8 * (e % QN)]) = vl[u];
    }
  }
  __syncthreads();
  const int Ib[RB] = {wr, 7 - wr};
  const int kq = 8 * (lane >> 5), l32 = lane & 31;
  const int pb = wp * (BN / WP);
  for (int t = 0; t < T; ++t) {
    if (active && !active[t]) continue;
    const unsigned short* Wh = whi + (long)t * NP * NP;
    const unsigned short* Wl = wlo + (long)t * NP * NP;
    f32x16 acc[RB][PC];
#pragma unroll
    for (int k = 0; k < RB; ++k)
#pragma unroll
      for (int p = 0; p < PC; ++p)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[k][p][r] = 0.f;
    // W fragments through a buffer resource over W_t: one coalesced 1 KB block per
    // load; blocks below the diagonal (or past NC) get an out-of-range offset and read
    // zero without memory traffic.
    const auto rWh = buf_rsrc(Wh, NP * NP * 2), rWl = buf_rsrc(Wl, NP * NP * 2);
    auto wofs = [&](int k, int cc, int s2) -> int {
      return (Ib[k] <= cc && Ib[k] < NC) ? ((Ib[k] * (NP >> 4) + 2 * cc + s2) * 64 + lane) * 16 : (int)0x80000000;
    };
    uint4 wh[PF][RB][2], wl[PF][RB][2];
#pragma unroll
    for (int d = 0; d < PF && d < NC; ++d)
#pragma unroll
      for (int k = 0; k < RB; ++k)
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
          const int o = wofs(k, d, s2);
          wh[d][k][s2] = buf_ld16(rWh, o, 0);
          wl[d][k][s2] = buf_ld16(rWl, o, 0);
        }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int sl = c % PF;
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        bf16x8 bh[PC], bl[PC];
#pragma unroll
        for (int p = 0; p < PC; ++p) {
          const int pt = pb + 32 * p + l32;
          bh[p] = *reinterpret_cast<const bf16x8*>(&sT[0][pt][32 * c + 16 * s2 + kq]);
          bl[p] = *reinterpret_cast<const bf16x8*>(&sT[1][pt][32 * c + 16 * s2 + kq]);
        }
#pragma unroll
        for (int k = 0; k < RB; ++k) {
          if (Ib[k] > c) continue;
          const bf16x8 ah = __builtin_bit_cast(bf16x8, wh[sl][k][s2]);
          const bf16x8 al = __builtin_bit_cast(bf16x8, wl[sl][k][s2]);
#pragma unroll
          for (int p = 0; p < PC; ++p) {
            acc[k][p] = mfma32(al, bh[p], acc[k][p]);
            acc[k][p] = mfma32(ah, bl[p], acc[k][p]);
            acc[k][p] = mfma32(ah, bh[p], acc[k][p]);
          }
        }
      }
      if (c + PF < NC) {
#pragma unroll
        for (int k = 0; k < RB; ++k)
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2) {
            const int o = wofs(k, c + PF, s2);
            wh[sl][k][s2] = buf_ld16(rWh, o, 0);
            wl[sl][k][s2] = buf_ld16(rWl, o, 0);
          }
      }
    }
    float part[PC];
#pragma unroll
    for (int p = 0; p < PC; ++p) part[p] = 0.f;
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      if (Ib[k] >= NC) continue;
#pragma unroll
      for (int p = 0; p < PC; ++p) {
        const int pt = pb + 32 * p + l32;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int i0 = 32 * Ib[k] + 8 * g + 4 * (lane >> 5);
          uint2 hh = *reinterpret_cast<const uint2*>(&sT[0][pt][i0]);
          uint2 ll = *reinterpret_cast<const uint2*>(&sT[1][pt][i0]);
          float v0 = __uint_as_float(hh.x << 16) + __uint_as_float(ll.x << 16);
          float v1 = __uint_as_float(hh.x & 0xFFFF0000u) + __uint_as_float(ll.x & 0xFFFF0000u);
          float v2 = __uint_as_float(hh.y << 16) + __uint_as_float(ll.y << 16);
          float v3 = __uint_as_float(hh.y & 0xFFFF0000u) + __uint_as_float(ll.y & 0xFFFF0000u);
          part[p] += v0 * acc[k][p][4 * g] + v1 * acc[k][p][4 * g + 1] + v2 * acc[k][p][4 * g + 2] +
                     v3 * acc[k][p][4 * g + 3];
        }
      }
    }
#pragma unroll
    for (int p = 0; p < PC; ++p) {
      part[p] += __shfl_xor(part[p], 32);
      if (lane < 32) red[wr][pb + 32 * p + lane] = part[p];
    }
    __syncthreads();
    for (int x = tid; x < BN; x += NTH) {
      long r = p0 + x;
      if (r < ng) {
        double a = (double)red[0][x] + (double)red[1][x] + (double)red[2][x] + (double)red[3][x];
        rho[(long)t * ng + r] = rho0[r] + a;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Density for N > 256 (orbital-major hi/lo psi [N][ng], W row-major [ld][ld], ld a
// multiple of 32, zero past N).  rho = rho0 + sum_i psi_i Z_i, Z = W Psi, as a tiled
// product: one block per (128-row block I of W, trajectory, 128 grid points), I
// fastest so the blocks sharing a tile of points run together and read its orbital
// rows once from HBM, the rest from L2.  K runs over the orbitals j >= 128 I in
// chunks of 32: the block stages W[I rows][chunk] and psi[chunk][points] into LDS
// (the latter transposed to [point][j] by packing row pairs into 32-bit words,
// 16-byte pieces XOR-swizzled by bits 2-3 of the row), double buffered, the next
// chunk's loads in flight during the matrix instructions; four waves each own 64
// rows x 64 points as 2 x 2 tiles of 32x32x16 BF16x3 products.  The epilogue
// reads psi_i at the block's rows and points, reduces sum_i psi_i Z_i over the
// rows, and writes one FP32 partial density per row block; k_density_sum adds
// the partials in row-block order (deterministic).
constexpr int DBM = 128, DBN = 128;
__device__ __forceinline__ int dsw32(int r, int q) { return r * 32 + 8 * (q ^ ((r >> 2) & 3)); }

__global__ __launch_bounds__(256, 2) void k_density_big(int N, long ng, int ld, const unsigned short* __restrict__ whi,
                                                        const unsigned short* __restrict__ wlo,
                                                        const unsigned short* __restrict__ phi,
                                                        const unsigned short* __restrict__ plo,
                                                        float* __restrict__ part, int nI, int T, const int* active) {
  __shared__ __attribute__((aligned(16))) unsigned short sA[2][2][DBM * 32];
  __shared__ __attribute__((aligned(16))) unsigned short sB[2][2][DBN * 32];
  __shared__ float red[2][DBN];
  const long lid = xcd_logical(blockIdx.x, gridDim.x);
  const int I = (int)(lid % nI);
  const long rest = lid / nI;
  const int t = (int)(rest % T);
  const long pt0 = (rest / T) * DBN;
  if (active && !active[t]) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int i0 = I * DBM;
  const int nk = (N - i0 + 31) / 32;
  const long npt = min((long)DBN, ng - pt0);  // valid points of this tile (a multiple of 8)
  const auto rWh = buf_rsrc(whi + (long)t * ld * ld, ld * ld * 2);
  const auto rWl = buf_rsrc(wlo + (long)t * ld * ld, ld * ld * 2);
  // staging roles: W pieces p = tid, tid + 256 (row p >> 2, piece p & 3); orbital rows
  // 2 jp, 2 jp + 1 (jp = tid & 15) at points 8 pc .. 8 pc + 7 (pc = tid >> 4)
  const int jp = tid & 15, pc = tid >> 4;
  const int pv = 8 * pc < npt ? 16 * pc : (int)0x80000000;  // byte offset of the piece, or out of range
  uint4 ah[2], al[2], bh[2], bl[2];
  auto fetch = [&](int c) {
    const int j0 = i0 + 32 * c;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int p = tid + 256 * u, row = p >> 2, q = p & 3;
      const int off = ((i0 + row) * ld + j0 + 8 * q) * 2;
      ah[u] = buf_ld16(rWh, off, 0);
      al[u] = buf_ld16(rWl, off, 0);
    }
    const int rows = __builtin_amdgcn_readfirstlane(min(32, N - j0));
    const int bytes = (int)(((long)(rows - 1) * ng + npt) * 2);
    const auto rBh = buf_rsrc(phi + (long)j0 * ng + pt0, bytes);
    const auto rBl = buf_rsrc(plo + (long)j0 * ng + pt0, bytes);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int o = pv < 0 ? pv : (int)((long)(2 * jp + u) * ng * 2) + pv;
      bh[u] = buf_ld16(rBh, o, 0);
      bl[u] = buf_ld16(rBl, o, 0);
    }
  };
  auto stage = [&](int b) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int p = tid + 256 * u, row = p >> 2, q = p & 3;
      *reinterpret_cast<uint4*>(&sA[b][0][dsw32(row, q)]) = ah[u];
      *reinterpret_cast<uint4*>(&sA[b][1][dsw32(row, q)]) = al[u];
    }
    // transpose: word u of the point pair (rows 2 jp, 2 jp + 1) at point 8 pc + u
    const unsigned int h0[4] = {bh[0].x, bh[0].y, bh[0].z, bh[0].w}, h1[4] = {bh[1].x, bh[1].y, bh[1].z, bh[1].w};
    const unsigned int l0[4] = {bl[0].x, bl[0].y, bl[0].z, bl[0].w}, l1[4] = {bl[1].x, bl[1].y, bl[1].z, bl[1].w};
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int pt = 8 * pc + u, sh = 16 * (u & 1), w = u >> 1;
      const unsigned int vh = ((h0[w] >> sh) & 0xFFFFu) | (((h1[w] >> sh) & 0xFFFFu) << 16);
      const unsigned int vl = ((l0[w] >> sh) & 0xFFFFu) | (((l1[w] >> sh) & 0xFFFFu) << 16);
      const int e = dsw32(pt, jp >> 2) + 2 * (jp & 3);
      *reinterpret_cast<unsigned int*>(&sB[b][0][e]) = vh;
      *reinterpret_cast<unsigned int*>(&sB[b][1][e]) = vl;
    }
  };
  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;
  const int l32 = lane & 31, k8 = lane >> 5;
  fetch(0);
  stage(0);
  __syncthreads();
  for (int c = 0; c < nk; ++c) {
    const int b = c & 1;
    if (c + 1 < nk) fetch(c + 1);
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      bf16x8 fah[2], fal[2], fbh[2], fbl[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const int ra = 64 * wr + 32 * x + l32, rb = 64 * wc + 32 * x + l32;
        fah[x] = *reinterpret_cast<const bf16x8*>(&sA[b][0][dsw32(ra, 2 * s2 + k8)]);
        fal[x] = *reinterpret_cast<const bf16x8*>(&sA[b][1][dsw32(ra, 2 * s2 + k8)]);
        fbh[x] = *reinterpret_cast<const bf16x8*>(&sB[b][0][dsw32(rb, 2 * s2 + k8)]);
        fbl[x] = *reinterpret_cast<const bf16x8*>(&sB[b][1][dsw32(rb, 2 * s2 + k8)]);
      }
      // the three BF16x3 terms outermost: consecutive products update different tiles
#pragma unroll
      for (int term = 0; term < 3; ++term)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            acc[x][y] = mfma32(term == 0 ? fal[x] : fah[x], term == 1 ? fbl[y] : fbh[y], acc[x][y]);
    }
    if (c + 1 < nk) stage(b ^ 1);
    __syncthreads();
  }
  // epilogue: sum over the block's rows of psi_i Z_i at each point
  const int rowsI = min(DBM, N - i0);
  const int ebytes = (int)(((long)(rowsI - 1) * ng + npt) * 2);
  const auto rEh = buf_rsrc(phi + (long)i0 * ng + pt0, ebytes);
  const auto rEl = buf_rsrc(plo + (long)i0 * ng + pt0, ebytes);
  float pr[2] = {0.f, 0.f};
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    const int col = 64 * wc + 32 * y + l32;
    const bool cok = col < npt;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 64 * wr + 32 * x + 8 * (r >> 2) + 4 * k8 + (r & 3);
        const int o = cok ? (int)(((long)row * ng + col) * 2) : (int)0x80000000;
        const unsigned short vh = __builtin_amdgcn_raw_buffer_load_b16(rEh, o, 0, 0);
        const unsigned short vl = __builtin_amdgcn_raw_buffer_load_b16(rEl, o, 0, 0);
        pr[y] += (bf2f(vh) + bf2f(vl)) * acc[x][y][r];
      }
  }
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    pr[y] += __shfl_xor(pr[y], 32);
    if (lane < 32) red[wr][64 * wc + 32 * y + lane] = pr[y];
  }
  __syncthreads();
  if (tid < npt) part[((long)t * nI + I) * ng + pt0 + tid] = red[0][tid] + red[1][tid];
}

// rho_t = rho0 + sum_I part_t[I] (row-block order)
__global__ void k_density_sum(const float* __restrict__ part, int nI, long ng, const double* __restrict__ rho0,
                              double* __restrict__ rho, const int* active) {
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  part += (long)t * nI * ng;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < ng; p += (long)gridDim.x * blockDim.x) {
    double a = rho0[p];
    for (int I = 0; I < nI; ++I) a += (double)part[(long)I * ng + p];
    rho[(long)t * ng + p] = a;
  }
}

int density_big_rows() { return DBM; }

int density_tile_ld(int N) { return (N + 31) / 32 * 32; }

hipError_t density_bf16x3(hipStream_t s, int N, long ng, const unsigned short* whi, const unsigned short* wlo,
                          const unsigned short* phi, const unsigned short* plo, const unsigned short* pthi,
                          const unsigned short* ptlo, const double* rho0, double* rho, int T, const int* active,
                          float* dpart) {
  if (N <= 256) {
    if (!pthi || !ptlo) return hipErrorInvalidValue;
    const dim3 grid(cdivm(ng, 64)), blk(256);
    switch (density_tile_ld(N) / 32) {
#define RT_DENSITY_NC(nc)                                                                                         \
  case nc:                                                                                                        \
    hipLaunchKernelGGL((k_density_tile32<64, 1, nc, 2, 2>), grid, blk, 0, s, ng, whi, wlo, pthi, ptlo, rho0, rho, T, \
                       active);                                                                                   \
    break;
      RT_DENSITY_NC(1) RT_DENSITY_NC(2) RT_DENSITY_NC(3) RT_DENSITY_NC(4)
      RT_DENSITY_NC(5) RT_DENSITY_NC(6) RT_DENSITY_NC(7) RT_DENSITY_NC(8)
#undef RT_DENSITY_NC
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (!dpart || ng % 8) return hipErrorInvalidValue;
  const int ld = density_tile_ld(N), nI = cdivm(N, DBM);
  if ((long)ld * ld * 2 >= (1L << 31) || (long)DBM * ng * 2 >= (1L << 31) || 32L * ng * 2 >= (1L << 31))
    return hipErrorInvalidValue;
  const long blocks = (long)nI * T * cdivm(ng, DBN);
  hipLaunchKernelGGL(k_density_big, dim3((unsigned)blocks), dim3(256), 0, s, N, ng, ld, whi, wlo, phi, plo, dpart, nI,
                     T, active);
  long b = (ng + 255) / 256;
  if (b > 2048) b = 2048;
  hipLaunchKernelGGL(k_density_sum, dim3((unsigned)b, T), dim3(256), 0, s, dpart, nI, ng, rho0, rho, active);
  return hipGetLastError();
}

// dv32_t = (float)(vloc_t - vloc_gs); blockIdx.y = t
__global__ void k_delta_f32(float* d, const double* a, const double* b, long n, const int* active) {
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    d[t * n + i] = (float)(a[t * n + i] - b[i]);
}
hipError_t delta_f32(hipStream_t s, float* d, const double* a, const double* b, long n, int T, const int* active) {
  long bl = (n + 255) / 256;
  if (bl > 1024) bl = 1024;
  hipLaunchKernelGGL(k_delta_f32, dim3((int)bl, T), dim3(256), 0, s, d, a, b, n, active);
  return hipGetLastError();
}

}  // namespace rtk
