// Learned first guess of the self-consistent loop: feature extraction from
// the density change, a small tanh MLP (forward, backward, Adam) in FP32, and
// the coarse-to-fine transfer of its predicted potential correction.
//
// Network: x (n_in) -> tanh(W1 x + b1) (n_h) -> tanh(W2 a1 + b2) (n_h) -> W3 a2 + b3
// (n_out), on standardised inputs/outputs.  Packed parameter layout (floats):
//   x_mean[n_in] x_scale[n_in] y_mean[n_out] y_scale[n_out]
//   W1[n_h][n_in] b1[n_h] W2[n_h][n_h] b2[n_h] W3[n_out][n_h] b3[n_out]
// The trainable part starts at offset 2 n_in + 2 n_out.
#include "kernels_mlp.h"

#include <hip/hip_runtime.h>

namespace rtk {

__host__ __device__ static inline int cdivl(long a, long b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Strided FP32 GEMM: C[i][j] = alpha sum_k A(i,k) B(k,j) + beta C[i][j] (+ bias[j]),
// A(i,k) = A[i sai + k sak], B(k,j) = B[k sbk + j sbj].  64 x 64 tile, K chunk 16,
// 256 threads with 4 x 4 outputs each.  Sizes here are small (batch x 8264 x 256).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gemm_f32(int M, int N, int K, float alpha, const float* __restrict__ A,
                                                  long sai, long sak, const float* __restrict__ B, long sbk,
                                                  long sbj, float beta, float* __restrict__ C, long ldc,
                                                  const float* __restrict__ bias) {
  __shared__ float As[16][64 + 1];
  __shared__ float Bs[16][64 + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      int kk = e >> 6, r = e & 63;
      int gi = i0 + r, gk = k0 + kk, gj = j0 + r;
      As[kk][r] = (gi < M && gk < K) ? A[gi * sai + gk * sak] : 0.f;
      Bs[kk][r] = (gj < N && gk < K) ? B[gk * sbk + gj * sbj] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][ty * 4 + q];
        b[q] = Bs[kk][tx * 4 + q];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int gi = i0 + ty * 4 + p, gj = j0 + tx * 4 + q;
      if (gi < M && gj < N) {
        float v = alpha * acc[p][q];
        if (beta != 0.f) v += beta * C[gi * ldc + gj];
        if (bias) v += bias[gj];
        C[gi * ldc + gj] = v;
      }
    }
}

// Few rows (M <= kGemvRows, e.g. the network evaluated for a handful of
// trajectories): one wave per output column j, the lanes striding K (contiguous
// for the weight matrices), all M rows accumulated together, then a fixed
// shuffle tree.  The tiled kernel above would run a few blocks with the whole K
// loop each.
constexpr int kGemvRows = 8;

__global__ __launch_bounds__(256) void k_gemv_f32(int M, int N, int K, float alpha, const float* __restrict__ A,
                                                  long sai, long sak, const float* __restrict__ B, long sbk,
                                                  long sbj, float beta, float* __restrict__ C, long ldc,
                                                  const float* __restrict__ bias) {
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (j >= N) return;
  float acc[kGemvRows];
#pragma unroll
  for (int i = 0; i < kGemvRows; ++i) acc[i] = 0.f;
  for (int k = lane; k < K; k += 64) {
    const float b = B[k * sbk + j * sbj];
#pragma unroll
    for (int i = 0; i < kGemvRows; ++i)
      if (i < M) acc[i] += A[i * sai + k * sak] * b;
  }
#pragma unroll
  for (int i = 0; i < kGemvRows; ++i)
    for (int o = 32; o > 0; o >>= 1) acc[i] += __shfl_xor(acc[i], o);
  if (lane == 0)
    for (int i = 0; i < M && i < kGemvRows; ++i) {
      float v = alpha * acc[i];
      if (beta != 0.f) v += beta * C[i * ldc + j];
      if (bias) v += bias[j];
      C[i * ldc + j] = v;
    }
}

hipError_t gemm_f32(hipStream_t s, int M, int N, int K, float alpha, const float* A, long sai, long sak,
                    const float* B, long sbk, long sbj, float beta, float* C, long ldc, const float* bias) {
  if (M <= kGemvRows) {
    hipLaunchKernelGGL(k_gemv_f32, dim3(cdivl(N, 4)), dim3(256), 0, s, M, N, K, alpha, A, sai, sak, B, sbk, sbj,
                       beta, C, ldc, bias);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_gemm_f32, dim3(cdivl(N, 64), cdivl(M, 64)), dim3(256), 0, s, M, N, K, alpha, A, sai, sak,
                     B, sbk, sbj, beta, C, ldc, bias);
  return hipGetLastError();
}

__global__ void k_tanh_inplace(float* x, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    x[i] = tanhf(x[i]);
}
// dZ = dA * (1 - A^2)
__global__ void k_tanh_bwd(float* dz, const float* a, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dz[i] = dz[i] * (1.f - a[i] * a[i]);
}
// db[j] = sum_i dZ[i][j]  (one thread per column, fixed order)
__global__ void k_colsum(const float* dz, int M, int N, float* db) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float acc = 0.f;
  for (int i = 0; i < M; ++i) acc += dz[(long)i * N + j];
  db[j] = acc;
}
// dY = (Y - T) / (B n_out); per-block partial sums of (Y - T)^2
__global__ __launch_bounds__(256) void k_mse_grad(const float* y, const float* t, float* dy, long n, float inv,
                                                  float* part) {
  __shared__ float sh[256];
  float acc = 0.f;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    float d = y[i] - t[i];
    dy[i] = d * inv;
    acc += d * d;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void k_loss_final(const float* part, int nb, float scale, float* loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float a = 0.f;
    for (int b = 0; b < nb; ++b) a += part[b];
    *loss = a * scale;
  }
}
// Adam (Kingma & Ba 2015) with bias correction.
__global__ void k_adam(float* p, const float* g, float* m, float* v, long n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}
// column mean and 1/std (floored) of X [M][N]
__global__ void k_colstats(const float* X, int M, int N, float* mean, float* scale, float floor_std) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double s = 0.0, s2 = 0.0;
  for (int i = 0; i < M; ++i) {
    double v = X[(long)i * N + j];
    s += v;
    s2 += v * v;
  }
  double mu = s / M;
  double var = s2 / M - mu * mu;
  double sd = var > 0 ? sqrt(var) : 0.0;
  mean[j] = (float)mu;
  scale[j] = (float)(1.0 / (sd > floor_std ? sd : floor_std));
}
// Z[i][j] = (X[i][j] - mean[j]) * scale[j]
__global__ void k_standardize(const float* X, const float* mean, const float* scale, float* Z, int M, int N) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)M * N) return;
  int j = (int)(e % N);
  Z[e] = (X[e] - mean[j]) * scale[j];
}
// Y[i][j] = mean[j] + U[i][j] / scale[j]
__global__ void k_unstandardize(const float* U, const float* mean, const float* scale, float* Y, int M, int N) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)M * N) return;
  int j = (int)(e % N);
  Y[e] = mean[j] + U[e] / scale[j];
}

static int ewb(long n) {
  long b = (n + 255) / 256;
  return (int)(b > 2048 ? 2048 : (b < 1 ? 1 : b));
}

long mlp_n_params(MlpDims d) {
  return 2L * d.n_in + 2L * d.n_out + (long)d.n_h * d.n_in + d.n_h + (long)d.n_h * d.n_h + d.n_h +
         (long)d.n_out * d.n_h + d.n_out;
}
long mlp_n_train(MlpDims d) { return mlp_n_params(d) - 2L * d.n_in - 2L * d.n_out; }
long mlp_work_floats(MlpDims d, int B) {
  return (long)B * d.n_in + 4L * B * d.n_h + 2L * B * d.n_out + 2048;
}

struct P {
  const float *xm, *xs, *ym, *ys, *W1, *b1, *W2, *b2, *W3, *b3;
};
static P unpack(const float* p, MlpDims d) {
  P q;
  q.xm = p; p += d.n_in;
  q.xs = p; p += d.n_in;
  q.ym = p; p += d.n_out;
  q.ys = p; p += d.n_out;
  q.W1 = p; p += (long)d.n_h * d.n_in;
  q.b1 = p; p += d.n_h;
  q.W2 = p; p += (long)d.n_h * d.n_h;
  q.b2 = p; p += d.n_h;
  q.W3 = p; p += (long)d.n_out * d.n_h;
  q.b3 = p;
  return q;
}

// work layout: Xs [B][n_in], a1 [B][n_h], a2 [B][n_h], d1, d2 [B][n_h], U [B][n_out], dU [B][n_out], part[2048]
hipError_t mlp_forward(hipStream_t s, MlpDims d, const float* params, const float* X, float* Y, int B,
                       float* work, bool standardized_out) {
  P q = unpack(params, d);
  float* Xs = work;
  float* a1 = Xs + (long)B * d.n_in;
  float* a2 = a1 + (long)B * d.n_h;
  float* U = a2 + 3L * B * d.n_h;
  long nx = (long)B * d.n_in;
  hipLaunchKernelGGL(k_standardize, dim3(cdivl(nx, 256)), dim3(256), 0, s, X, q.xm, q.xs, Xs, B, d.n_in);
  hipError_t e;
  if ((e = gemm_f32(s, B, d.n_h, d.n_in, 1.f, Xs, d.n_in, 1, q.W1, 1, d.n_in, 0.f, a1, d.n_h, q.b1)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_tanh_inplace, dim3(ewb((long)B * d.n_h)), dim3(256), 0, s, a1, (long)B * d.n_h);
  if ((e = gemm_f32(s, B, d.n_h, d.n_h, 1.f, a1, d.n_h, 1, q.W2, 1, d.n_h, 0.f, a2, d.n_h, q.b2)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_tanh_inplace, dim3(ewb((long)B * d.n_h)), dim3(256), 0, s, a2, (long)B * d.n_h);
  float* out = standardized_out ? Y : U;
  if ((e = gemm_f32(s, B, d.n_out, d.n_h, 1.f, a2, d.n_h, 1, q.W3, 1, d.n_h, 0.f, out, d.n_out, q.b3)) != hipSuccess)
    return e;
  if (!standardized_out) {
    long ny = (long)B * d.n_out;
    hipLaunchKernelGGL(k_unstandardize, dim3(cdivl(ny, 256)), dim3(256), 0, s, U, q.ym, q.ys, Y, B, d.n_out);
  }
  return hipGetLastError();
}

// Loss (on standardised targets) and gradients of the trainable parameters.
hipError_t mlp_loss_grad(hipStream_t s, MlpDims d, const float* params, const float* X, const float* Tgt, int B,
                         float* grads, float* work, float* loss_dev) {
  P q = unpack(params, d);
  float* Xs = work;
  float* a1 = Xs + (long)B * d.n_in;
  float* a2 = a1 + (long)B * d.n_h;
  float* d1 = a2 + (long)B * d.n_h;
  float* d2 = d1 + (long)B * d.n_h;
  float* U = d2 + (long)B * d.n_h;
  float* dU = U + (long)B * d.n_out;
  float* part = dU + (long)B * d.n_out;
  hipError_t e;
  if ((e = mlp_forward(s, d, params, X, U, B, work, true)) != hipSuccess) return e;
  // standardised targets into dU, then dU <- (U - Ts) / (B n_out)
  long ny = (long)B * d.n_out;
  hipLaunchKernelGGL(k_standardize, dim3(cdivl(ny, 256)), dim3(256), 0, s, Tgt, q.ym, q.ys, dU, B, d.n_out);
  const int nb = 512;
  hipLaunchKernelGGL(k_mse_grad, dim3(nb), dim3(256), 0, s, U, dU, dU, ny, 1.f / (float)ny, part);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, part, nb, 0.5f / (float)ny, loss_dev);
  float* gW1 = grads;
  float* gb1 = gW1 + (long)d.n_h * d.n_in;
  float* gW2 = gb1 + d.n_h;
  float* gb2 = gW2 + (long)d.n_h * d.n_h;
  float* gW3 = gb2 + d.n_h;
  float* gb3 = gW3 + (long)d.n_out * d.n_h;
  // layer 3: gW3 = dU^T a2, gb3 = colsum dU, d2 = (dU W3) * (1 - a2^2)
  if ((e = gemm_f32(s, d.n_out, d.n_h, B, 1.f, dU, 1, d.n_out, a2, d.n_h, 1, 0.f, gW3, d.n_h, nullptr)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_colsum, dim3(cdivl(d.n_out, 256)), dim3(256), 0, s, dU, B, d.n_out, gb3);
  if ((e = gemm_f32(s, B, d.n_h, d.n_out, 1.f, dU, d.n_out, 1, q.W3, d.n_h, 1, 0.f, d2, d.n_h, nullptr)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_tanh_bwd, dim3(ewb((long)B * d.n_h)), dim3(256), 0, s, d2, a2, (long)B * d.n_h);
  // layer 2
  if ((e = gemm_f32(s, d.n_h, d.n_h, B, 1.f, d2, 1, d.n_h, a1, d.n_h, 1, 0.f, gW2, d.n_h, nullptr)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_colsum, dim3(cdivl(d.n_h, 256)), dim3(256), 0, s, d2, B, d.n_h, gb2);
  if ((e = gemm_f32(s, B, d.n_h, d.n_h, 1.f, d2, d.n_h, 1, q.W2, d.n_h, 1, 0.f, d1, d.n_h, nullptr)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_tanh_bwd, dim3(ewb((long)B * d.n_h)), dim3(256), 0, s, d1, a1, (long)B * d.n_h);
  // layer 1
  if ((e = gemm_f32(s, d.n_h, d.n_in, B, 1.f, d1, 1, d.n_h, Xs, d.n_in, 1, 0.f, gW1, d.n_in, nullptr)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_colsum, dim3(cdivl(d.n_h, 256)), dim3(256), 0, s, d1, B, d.n_h, gb1);
  return hipGetLastError();
}

hipError_t mlp_adam(hipStream_t s, float* p, const float* g, float* m, float* v, long n, int t, float lr) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(ewb(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t mlp_colstats(hipStream_t s, const float* X, int M, int N, float* mean, float* scale, float floor_std) {
  hipLaunchKernelGGL(k_colstats, dim3(cdivl(N, 256)), dim3(256), 0, s, X, M, N, mean, scale, floor_std);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Features and transfers (fine grid [nz][ny][nx], coarse 16^3)
// ---------------------------------------------------------------------------
// coarse_t[c] = mean over the fine block of c of (f_t - ref) (ref nullable); blockIdx.y = t
template <typename TO>
__global__ void k_restrict(const double* f, const double* ref, TO* coarse, int nx, int ny, int nz, long fstride,
                           long cstride) {
  const int t = blockIdx.y;
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= 4096) return;
  int cx = c % 16, cy = (c / 16) % 16, cz = c / 256;
  int bx = nx / 16, by = ny / 16, bz = nz / 16;
  const double* ft = f + t * fstride;
  double acc = 0.0;
  for (int z = cz * bz; z < (cz + 1) * bz; ++z)
    for (int y = cy * by; y < (cy + 1) * by; ++y)
      for (int x = cx * bx; x < (cx + 1) * bx; ++x) {
        long g = ((long)z * ny + y) * nx + x;
        acc += ref ? ft[g] - ref[g] : ft[g];
      }
  coarse[t * cstride + c] = (TO)(acc / ((double)bx * by * bz));
}
hipError_t restrict16(hipStream_t s, const double* f, const double* ref, float* coarse, int nx, int ny, int nz,
                      long fstride, long cstride, int T) {
  hipLaunchKernelGGL(k_restrict<float>, dim3(16, T), dim3(256), 0, s, f, ref, coarse, nx, ny, nz, fstride, cstride);
  return hipGetLastError();
}
hipError_t restrict16_f64(hipStream_t s, const double* f, const double* ref, double* coarse, int nx, int ny, int nz,
                          long fstride, long cstride, int T) {
  hipLaunchKernelGGL(k_restrict<double>, dim3(16, T), dim3(256), 0, s, f, ref, coarse, nx, ny, nz, fstride, cstride);
  return hipGetLastError();
}

// fine_t = trilinear periodic interpolation of coarse_t (cell centres at (c + 1/2) b - 1/2)
__global__ void k_prolong(const float* coarse, double* fine, int nx, int ny, int nz, long cstride, long fstride) {
  const int t = blockIdx.y;
  long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long ng = (long)nx * ny * nz;
  if (g >= ng) return;
  int ix = (int)(g % nx), iy = (int)((g / nx) % ny), iz = (int)(g / ((long)nx * ny));
  double px = (ix + 0.5) / (nx / 16) - 0.5, py = (iy + 0.5) / (ny / 16) - 0.5, pz = (iz + 0.5) / (nz / 16) - 0.5;
  int x0 = (int)floor(px), y0 = (int)floor(py), z0 = (int)floor(pz);
  double wx = px - x0, wy = py - y0, wz = pz - z0;
  const float* ct = coarse + t * cstride;
  double acc = 0.0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        int cx = ((x0 + dx) % 16 + 16) % 16, cy = ((y0 + dy) % 16 + 16) % 16, cz = ((z0 + dz) % 16 + 16) % 16;
        double w = (dx ? wx : 1 - wx) * (dy ? wy : 1 - wy) * (dz ? wz : 1 - wz);
        acc += w * (double)ct[(cz * 16 + cy) * 16 + cx];
      }
  fine[t * fstride + g] = acc;
}
hipError_t prolong16(hipStream_t s, const float* coarse, double* fine, int nx, int ny, int nz, long cstride,
                     long fstride, int T) {
  long ng = (long)nx * ny * nz;
  hipLaunchKernelGGL(k_prolong, dim3(cdivl(ng, 256), T), dim3(256), 0, s, coarse, fine, nx, ny, nz, cstride, fstride);
  return hipGetLastError();
}

// 9 moments of d = f_t - ref with the centred sawtooth coordinates; partials per block.
__global__ __launch_bounds__(256) void k_moments_part(const double* f, const double* ref, int nx, int ny, int nz,
                                                      double h, long fstride, double* part) {
  __shared__ double sh[256];
  const int t = blockIdx.y;
  const double* ft = f + t * fstride;
  long ng = (long)nx * ny * nz;
  double m[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (long g = (long)blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += (long)gridDim.x * blockDim.x) {
    int ix = (int)(g % nx), iy = (int)((g / nx) % ny), iz = (int)(g / ((long)nx * ny));
    double q[3] = {(ix - 0.5 * (nx - 1)) * h, (iy - 0.5 * (ny - 1)) * h, (iz - 0.5 * (nz - 1)) * h};
    double d = ft[g] - ref[g];
    m[0] += d * q[0];
    m[1] += d * q[1];
    m[2] += d * q[2];
    m[3] += d * q[0] * q[0];
    m[4] += d * q[0] * q[1];
    m[5] += d * q[0] * q[2];
    m[6] += d * q[1] * q[1];
    m[7] += d * q[1] * q[2];
    m[8] += d * q[2] * q[2];
  }
  for (int k = 0; k < 9; ++k) {
    sh[threadIdx.x] = m[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[((long)t * gridDim.x + blockIdx.x) * 9 + k] = sh[0];
    __syncthreads();
  }
}
__global__ void k_moments_final(const double* part, int nb, double h3, float* out, long ostride) {
  const int t = blockIdx.x;
  int k = threadIdx.x;
  if (k >= 9) return;
  double a = 0.0;
  for (int b = 0; b < nb; ++b) a += part[((long)t * nb + b) * 9 + k];
  out[t * ostride + k] = (float)(a * h3);
}
hipError_t moments9(hipStream_t s, const double* f, const double* ref, int nx, int ny, int nz, double h, long fstride,
                    double* part, float* out, long ostride, int T) {
  const int nb = 256;
  hipLaunchKernelGGL(k_moments_part, dim3(nb, T), dim3(256), 0, s, f, ref, nx, ny, nz, h, fstride, part);
  hipLaunchKernelGGL(k_moments_final, dim3(T), dim3(64), 0, s, part, nb, h * h * h, out, ostride);
  return hipGetLastError();
}

// x_t = [mom ring (oldest first, 8 x 9), coarse ring slot `cur`, coarse ring slot `prev`]
__global__ void k_assemble(const float* mom_ring, int mom_head, const float* cd_ring, int cur, int prev, float* X,
                           int n_in, long mom_stride, long cd_stride) {
  const int t = blockIdx.y;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_in) return;
  float v;
  if (i < 72) {
    int slot = (mom_head + 1 + i / 9) % 8;  // mom_head = newest; oldest first
    v = mom_ring[t * mom_stride + slot * 9 + i % 9];
  } else if (i < 72 + 4096) {
    v = cd_ring[t * cd_stride + cur * 4096 + (i - 72)];
  } else {
    v = cd_ring[t * cd_stride + prev * 4096 + (i - 72 - 4096)];
  }
  X[(long)t * n_in + i] = v;
}
hipError_t assemble_features(hipStream_t s, const float* mom_ring, int mom_head, const float* cd_ring, int cur,
                             int prev, float* X, int n_in, long mom_stride, long cd_stride, int T) {
  hipLaunchKernelGGL(k_assemble, dim3(cdivl(n_in, 256), T), dim3(256), 0, s, mom_ring, mom_head, cd_ring, cur, prev, X,
                     n_in, mom_stride, cd_stride);
  return hipGetLastError();
}

// y_t = c_new - 2 c_mid + c_old (second difference of coarse potentials, FP64, stored FP32)
__global__ void k_second_diff(const double* ring, int inew, int imid, int iold, float* Y, long rstride, long ystride) {
  const int t = blockIdx.y;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 4096) return;
  const double* r = ring + t * rstride;
  Y[t * ystride + i] = (float)((r[inew * 4096 + i] - 2.0 * r[imid * 4096 + i]) + r[iold * 4096 + i]);
}
hipError_t second_diff(hipStream_t s, const double* ring, int inew, int imid, int iold, float* Y, long rstride,
                       long ystride, int T) {
  hipLaunchKernelGGL(k_second_diff, dim3(16, T), dim3(256), 0, s, ring, inew, imid, iold, Y, rstride, ystride);
  return hipGetLastError();
}

// rows dst[t] = src[t] for t < T (float), row length n
__global__ void k_copy_rows_f(const float* src, float* dst, long n, long sstride, long dstride) {
  const int t = blockIdx.y;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[t * dstride + i] = src[t * sstride + i];
}
hipError_t copy_rows_f(hipStream_t s, const float* src, float* dst, long n, long sstride, long dstride, int T) {
  hipLaunchKernelGGL(k_copy_rows_f, dim3(ewb(n), T), dim3(256), 0, s, src, dst, n, sstride, dstride);
  return hipGetLastError();
}

}  // namespace rtk
