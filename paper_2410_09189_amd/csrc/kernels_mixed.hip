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
// stored with leading dimension ld >= N (rows and columns N..ld-1 zero).
// blockIdx.y = trajectory: S_t = S + t sstride, hi/lo_t = + t ld^2, S0 shared.
__global__ void k_upper_weighted_delta_bf16(const double* S, const double* S0, unsigned short* hi,
                                            unsigned short* lo, int N, int ld, long sstride, const int* active) {
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
  hi[e] = h;
  lo[e] = f2bf((float)(w - (double)bf2f(h)));
}

hipError_t upper_weighted_delta_bf16(hipStream_t s, const double* S, const double* S0, unsigned short* hi,
                                     unsigned short* lo, int N, int ld, long sstride, int T, const int* active) {
  long n = (long)ld * ld;
  hipLaunchKernelGGL(k_upper_weighted_delta_bf16, dim3(cdivm(n, 256), T), dim3(256), 0, s, S, S0, hi, lo, N, ld,
                     sstride, active);
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

__global__ __launch_bounds__(256) void k_proj_bf16x3(int N, long ng, const unsigned short* __restrict__ Ahi,
                                                     const unsigned short* __restrict__ Alo,
                                                     const float* __restrict__ w, float* __restrict__ part,
                                                     long kps, int ntm, int T, const int* active) {
  __shared__ unsigned short sAh[XB][XK + XPAD], sAl[XB][XK + XPAD];
  __shared__ unsigned short sBh[XB][XK + XPAD], sBl[XB][XK + XPAD];
  const int tb = blockIdx.x % T;
  if (active && !active[tb]) return;
  w += (long)tb * ng;
  part += (long)tb * gridDim.y * N * N;
  int tm = 0, tn;
  {
    int t = blockIdx.x / T, rowlen = ntm;
    while (t >= rowlen) { t -= rowlen; ++tm; --rowlen; }
    tn = tm + t;
  }
  const long k0 = (long)blockIdx.y * kps;
  const long k1 = min(ng, k0 + kps);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
  const long m0 = (long)tm * XB, n0 = (long)tn * XB;
  for (long kb = k0; kb < k1; kb += XK) {
    // 128 rows x 64 k = 1024 vectors of 8 bf16 per array
    for (int v = tid; v < XB * XK / 8; v += 256) {
      int r = v >> 3, c8 = (v & 7) * 8;
      long gk = kb + c8;
      long ga = m0 + r, gb = n0 + r;
      uint4 ah = make_uint4(0, 0, 0, 0), al = ah, bh = ah, bl = ah;
      if (gk + 8 <= k1) {
        if (ga < N) {
          ah = *reinterpret_cast<const uint4*>(Ahi + ga * ng + gk);
          al = *reinterpret_cast<const uint4*>(Alo + ga * ng + gk);
        }
        if (gb < N) {
          uint4 xh = *reinterpret_cast<const uint4*>(Ahi + gb * ng + gk);
          uint4 xl = *reinterpret_cast<const uint4*>(Alo + gb * ng + gk);
          const unsigned short* ph = reinterpret_cast<const unsigned short*>(&xh);
          const unsigned short* pl = reinterpret_cast<const unsigned short*>(&xl);
          unsigned short oh[8], ol[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) split2((bf2f(ph[q]) + bf2f(pl[q])) * w[gk + q], oh[q], ol[q]);
          bh = *reinterpret_cast<uint4*>(oh);
          bl = *reinterpret_cast<uint4*>(ol);
        }
      } else if (gk < k1) {
        unsigned short th[8] = {0}, tl[8] = {0}, uh[8] = {0}, ul[8] = {0};
        for (int q = 0; q < 8 && gk + q < k1; ++q) {
          if (ga < N) { th[q] = Ahi[ga * ng + gk + q]; tl[q] = Alo[ga * ng + gk + q]; }
          if (gb < N) split2((bf2f(Ahi[gb * ng + gk + q]) + bf2f(Alo[gb * ng + gk + q])) * w[gk + q], uh[q], ul[q]);
        }
        ah = *reinterpret_cast<uint4*>(th);
        al = *reinterpret_cast<uint4*>(tl);
        bh = *reinterpret_cast<uint4*>(uh);
        bl = *reinterpret_cast<uint4*>(ul);
      }
      *reinterpret_cast<uint4*>(&sAh[r][c8]) = ah;
      *reinterpret_cast<uint4*>(&sAl[r][c8]) = al;
      *reinterpret_cast<uint4*>(&sBh[r][c8]) = bh;
      *reinterpret_cast<uint4*>(&sBl[r][c8]) = bl;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < XK; kk += 32) {
      bf16x8 fah[4], fal[4], fbh[4], fbl[4];
      const int kc = kk + 8 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int r = wm * 64 + i * 16 + (lane & 15);
        fah[i] = *reinterpret_cast<const bf16x8*>(&sAh[r][kc]);
        fal[i] = *reinterpret_cast<const bf16x8*>(&sAl[r][kc]);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int r = wn * 64 + j * 16 + (lane & 15);
        fbh[j] = *reinterpret_cast<const bf16x8*>(&sBh[r][kc]);
        fbl[j] = *reinterpret_cast<const bf16x8*>(&sBl[r][kc]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fal[i], fbh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[i], fbl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[i], fbh[j], acc[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  float* P = part + (long)blockIdx.y * N * N;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        long row = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        long col = n0 + wn * 64 + j * 16 + (lane & 15);
        if (row < N && col < N) P[row * N + col] = acc[i][j][r];
      }
}

hipError_t proj_bf16x3(hipStream_t s, int N, long ng, const unsigned short* hi, const unsigned short* lo,
                       const float* w, float* part, long kps, int n_split, int T, const int* active) {
  int ntm = cdivm(N, XB);
  int nt = ntm * (ntm + 1) / 2;
  hipLaunchKernelGGL(k_proj_bf16x3, dim3(nt * T, n_split), dim3(256), 0, s, N, ng, hi, lo, w, part, kps, ntm, T,
                     active);
  return hipGetLastError();
}

// C[m][n] = alpha * sum_s part[s][m][n] (FP64 sum of FP32 partials), upper kept and mirrored, plus base.
__global__ void k_reduce_parts_f32(const float* __restrict__ part, int n_split, int N, double alpha,
                                   const double* base, double* C, const int* active, long sbase) {
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  part += (long)t * n_split * N * N;
  C += (long)t * N * N;
  base += t * sbase;
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)N * N) return;
  int m = (int)(e / N), n = (int)(e - (long)m * N);
  if (m > n) return;
  double acc = 0.0;
  for (int sI = 0; sI < n_split; ++sI) acc += (double)part[(long)sI * N * N + e];
  acc *= alpha;
  C[e] = base[e] + acc;
  if (m < n) C[(long)n * N + m] = base[(long)n * N + m] + acc;
}

hipError_t reduce_parts_f32(hipStream_t s, const float* part, int n_split, int N, double alpha,
                            const double* base, double* C, int T, const int* active, long sbase) {
  long n = (long)N * N;
  hipLaunchKernelGGL(k_reduce_parts_f32, dim3(cdivm(n, 256), T), dim3(256), 0, s, part, n_split, N, alpha, base, C,
                     active, sbase);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Density change from the density-matrix change, fused:
//   rho[r] = rho0[r] + sum_i psi_i(r) sum_{j >= i} W_ij psi_j(r)
// with W (upper-weighted change, bf16 hi/lo) and Psi (bf16 hi/lo).  One block
// owns 64 grid points and loops over 64-row blocks of W; Phi = W Psi is never
// stored.  Psi columns are staged transposed in LDS (k = orbital contiguous).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_density_bf16x3(int N, long ng, const unsigned short* __restrict__ Whi,
                                                        const unsigned short* __restrict__ Wlo,
                                                        const unsigned short* __restrict__ Phi_,
                                                        const unsigned short* __restrict__ Plo_,
                                                        const double* __restrict__ rho0,
                                                        double* __restrict__ rho, int T, const int* active,
                                                        int ld) {
  constexpr int BM = 64, BN = 64, BK = 32, PD = 8;
  const int tb = blockIdx.x % T;
  if (active && !active[tb]) return;
  Whi += (long)tb * ld * ld;
  Wlo += (long)tb * ld * ld;
  rho += (long)tb * ng;
  __shared__ unsigned short sWh[BM][BK + PD], sWl[BM][BK + PD];
  __shared__ unsigned short sPh[BN][BK + PD], sPl[BN][BK + PD];
  __shared__ float red[2][4][BN];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const long r0 = (long)(blockIdx.x / T) * BN;
  float part[2] = {0.f, 0.f};
  const int nI = cdivm(N, BM);
  for (int I = 0; I < nI; ++I) {
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int jb = I * BM; jb < N; jb += BK) {
      for (int e = tid; e < BM * BK; e += 256) {
        int r = e / BK, c = e - r * BK;
        int gi = I * BM + r, gj = jb + c;
        bool ok = gi < N && gj < N;
        sWh[r][c] = ok ? Whi[(long)gi * ld + gj] : (unsigned short)0;
        sWl[r][c] = ok ? Wlo[(long)gi * ld + gj] : (unsigned short)0;
      }
      for (int e = tid; e < BK * BN; e += 256) {
        int kj = e / BN, c = e - kj * BN;
        int gj = jb + kj;
        long gr = r0 + c;
        bool ok = gj < N && gr < ng;
        sPh[c][kj] = ok ? Phi_[(long)gj * ng + gr] : (unsigned short)0;
        sPl[c][kj] = ok ? Plo_[(long)gj * ng + gr] : (unsigned short)0;
      }
      __syncthreads();
      const int kc = 8 * (lane >> 4);
      bf16x8 fwh[2], fwl[2], fph[2], fpl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        int r = wm * 32 + i * 16 + (lane & 15);
        fwh[i] = *reinterpret_cast<const bf16x8*>(&sWh[r][kc]);
        fwl[i] = *reinterpret_cast<const bf16x8*>(&sWl[r][kc]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        int c = wn * 32 + j * 16 + (lane & 15);
        fph[j] = *reinterpret_cast<const bf16x8*>(&sPh[c][kc]);
        fpl[j] = *reinterpret_cast<const bf16x8*>(&sPl[c][kc]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fwl[i], fph[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fwh[i], fpl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fwh[i], fph[j], acc[i][j], 0, 0, 0);
        }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int row = I * BM + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
          long col = r0 + wn * 32 + j * 16 + (lane & 15);
          if (row < N && col < ng) {
            float p = bf2f(Phi_[(long)row * ng + col]) + bf2f(Plo_[(long)row * ng + col]);
            part[j] += p * acc[i][j][r];
          }
        }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) red[wm][lane >> 4][wn * 32 + j * 16 + (lane & 15)] = part[j];
  __syncthreads();
  if (tid < BN && r0 + tid < ng) {
    double a = 0.0;
    for (int x = 0; x < 2; ++x)
      for (int y = 0; y < 4; ++y) a += (double)red[x][y][tid];
    rho[r0 + tid] = rho0[r0 + tid] + a;
  }
}

// Resident-tile density for N <= 256.  One block owns BN grid points and every
// trajectory: the point-major hi/lo orbital tile [BN][NP] (NP = N rounded up to 32,
// zero padded) is loaded into LDS once; for each trajectory Z = W Psi_tile is
// accumulated on the matrix cores with W (upper triangular, leading dimension NP)
// read as A fragments straight from L2, j-chunks of 32 outermost so each B fragment
// read from LDS serves all of a wave's row blocks, triangular blocks skipped; then
// rho_t = rho0 + sum_i psi_i Z_i with psi_i again from the LDS tile.
// Waves: 4 row groups x WP point groups; row group g owns the 16-row blocks
// g, 7-g, 8+g, 15-g, which balances the triangular work.
template <int BN, int WP>
__global__ __launch_bounds__(256 * WP) void k_density_tile(int NP, long ng, const unsigned short* __restrict__ whi,
                                                           const unsigned short* __restrict__ wlo,
                                                           const unsigned short* __restrict__ pth,
                                                           const unsigned short* __restrict__ ptl,
                                                           const double* __restrict__ rho0,
                                                           double* __restrict__ rho, int T, const int* active) {
  constexpr int LDP = 256 + 8;  // LDS row pitch (bf16)
  constexpr int RB = 4, PC = BN / 16 / WP, NTH = 256 * WP;
  __shared__ __attribute__((aligned(16))) unsigned short sT[2][BN][LDP];
  __shared__ float red[4][BN];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave & 3, wp = wave >> 2;
  const long p0 = (long)blockIdx.x * BN;
  const int c8 = NP >> 3;
  for (int e = tid; e < BN * c8; e += NTH) {
    int row = e / c8, q = e - row * c8;
    long r = p0 + row;
    uint4 vh = {0u, 0u, 0u, 0u}, vl = {0u, 0u, 0u, 0u};
    if (r < ng) {
      vh = *reinterpret_cast<const uint4*>(pth + r * NP + 8 * q);
      vl = *reinterpret_cast<const uint4*>(ptl + r * NP + 8 * q);
    }
    *reinterpret_cast<uint4*>(&sT[0][row][8 * q]) = vh;
    *reinterpret_cast<uint4*>(&sT[1][row][8 * q]) = vl;
  }
  __syncthreads();
  const int NB = NP >> 4, NC = NP >> 5;
  int Ib[RB] = {wr, 7 - wr, 8 + wr, 15 - wr};
  const int kq = 8 * (lane >> 4), l16 = lane & 15;
  const int pb = wp * (BN / WP);
  for (int t = 0; t < T; ++t) {
    if (active && !active[t]) continue;
    const unsigned short* Wh = whi + (long)t * NP * NP;
    const unsigned short* Wl = wlo + (long)t * NP * NP;
    f32x4 acc[RB][PC];
#pragma unroll
    for (int k = 0; k < RB; ++k)
#pragma unroll
      for (int p = 0; p < PC; ++p) acc[k][p] = (f32x4){0.f, 0.f, 0.f, 0.f};
    bf16x8 ah[RB], al[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      ah[k] = (bf16x8){};
      al[k] = (bf16x8){};
      if (Ib[k] <= 1 && Ib[k] < NB) {
        long off = (long)(16 * Ib[k] + l16) * NP + kq;
        ah[k] = *reinterpret_cast<const bf16x8*>(Wh + off);
        al[k] = *reinterpret_cast<const bf16x8*>(Wl + off);
      }
    }
    for (int c = 0; c < NC; ++c) {
      bf16x8 nh[RB], nl[RB];
#pragma unroll
      for (int k = 0; k < RB; ++k) {
        nh[k] = (bf16x8){};
        nl[k] = (bf16x8){};
        if (c + 1 < NC && Ib[k] <= 2 * c + 3 && Ib[k] < NB) {
          long off = (long)(16 * Ib[k] + l16) * NP + 32 * (c + 1) + kq;
          nh[k] = *reinterpret_cast<const bf16x8*>(Wh + off);
          nl[k] = *reinterpret_cast<const bf16x8*>(Wl + off);
        }
      }
      bf16x8 bh[PC], bl[PC];
#pragma unroll
      for (int p = 0; p < PC; ++p) {
        int pt = pb + 16 * p + l16;
        bh[p] = *reinterpret_cast<const bf16x8*>(&sT[0][pt][32 * c + kq]);
        bl[p] = *reinterpret_cast<const bf16x8*>(&sT[1][pt][32 * c + kq]);
      }
#pragma unroll
      for (int k = 0; k < RB; ++k) {
        if (Ib[k] > 2 * c + 1 || Ib[k] >= NB) continue;
#pragma unroll
        for (int p = 0; p < PC; ++p) {
          acc[k][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[k], bh[p], acc[k][p], 0, 0, 0);
          acc[k][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[k], bl[p], acc[k][p], 0, 0, 0);
          acc[k][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[k], bh[p], acc[k][p], 0, 0, 0);
        }
      }
#pragma unroll
      for (int k = 0; k < RB; ++k) {
        ah[k] = nh[k];
        al[k] = nl[k];
      }
    }
    float part[PC];
#pragma unroll
    for (int p = 0; p < PC; ++p) part[p] = 0.f;
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      if (Ib[k] >= NB) continue;
      const int i0 = 16 * Ib[k] + 4 * (lane >> 4);
#pragma unroll
      for (int p = 0; p < PC; ++p) {
        int pt = pb + 16 * p + l16;
        uint2 hh = *reinterpret_cast<const uint2*>(&sT[0][pt][i0]);
        uint2 ll = *reinterpret_cast<const uint2*>(&sT[1][pt][i0]);
        float v0 = __uint_as_float(hh.x << 16) + __uint_as_float(ll.x << 16);
        float v1 = __uint_as_float(hh.x & 0xFFFF0000u) + __uint_as_float(ll.x & 0xFFFF0000u);
        float v2 = __uint_as_float(hh.y << 16) + __uint_as_float(ll.y << 16);
        float v3 = __uint_as_float(hh.y & 0xFFFF0000u) + __uint_as_float(ll.y & 0xFFFF0000u);
        part[p] += v0 * acc[k][p][0] + v1 * acc[k][p][1] + v2 * acc[k][p][2] + v3 * acc[k][p][3];
      }
    }
#pragma unroll
    for (int p = 0; p < PC; ++p) {
      part[p] += __shfl_xor(part[p], 16);
      part[p] += __shfl_xor(part[p], 32);
      if (lane < 16) red[wr][pb + 16 * p + lane] = part[p];
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

int density_tile_ld(int N) { return N <= 256 ? (N + 31) / 32 * 32 : N; }

hipError_t density_bf16x3(hipStream_t s, int N, long ng, const unsigned short* whi, const unsigned short* wlo,
                          const unsigned short* phi, const unsigned short* plo, const unsigned short* pthi,
                          const unsigned short* ptlo, const double* rho0, double* rho, int T, const int* active) {
  if (N <= 256) {
    if (!pthi || !ptlo) return hipErrorInvalidValue;
    const int NP = density_tile_ld(N);
    hipLaunchKernelGGL((k_density_tile<128, 2>), dim3(cdivm(ng, 128)), dim3(512), 0, s, NP, ng, whi, wlo, pthi,
                       ptlo, rho0, rho, T, active);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_density_bf16x3, dim3(cdivm(ng, 64) * T), dim3(256), 0, s, N, ng, whi, wlo, phi, plo, rho0,
                     rho, T, active, N);
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
