// Ground-state kernels for gfx950: the dense symmetric eigensolver of the
// Rayleigh-Ritz step (parallel cyclic Jacobi), block residuals, the occupied
// density of an orbital block, sign normalisation and Pulay (DIIS) mixing.
//
// Every reduction has a fixed partition and combination order (the one atomic is
// a max of non-negative doubles), so repeated runs are bitwise identical.
#include "kernels_gs.h"

#include <hip/hip_runtime.h>
#include <cmath>

namespace rtk {
namespace {

__host__ __device__ inline int gs_cdiv(long a, long b) { return (int)((a + b - 1) / b); }

__device__ double gs_block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) sh[t] += sh[t + o];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// Parallel cyclic Jacobi (Golub & Van Loan, Matrix Computations, Sec. 8.5,
// with the round-robin ("chess tournament") ordering of Brent & Luk): in each
// of the ld - 1 rounds of a sweep the ld/2 index pairs are disjoint, so all
// their rotations commute and one launch applies them together.  A 2x2 block
// (rows of pair i, columns of pair j) of J^T A J only needs the same block of
// A and the two rotations, so every block is an independent thread; the
// (i, j) and (j, i) blocks are written by one thread, which keeps the iterate
// exactly symmetric.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void rr_pair(int ld, int round, int k, int& p, int& q) {
  const int m = ld - 1;
  if (k == 0) {
    p = m;
    q = round;
  } else {
    p = (round + k) % m;
    q = (round - k + m) % m;
  }
}

// Rotation (c, s) with t = s / c the root of smaller modulus of
// t^2 + 2 theta t - 1 = 0, theta = (a_qq - a_pp) / (2 a_pq): it zeroes a_pq of J^T A J,
// J = [[c, s], [-s, c]] on (p, q).
__device__ __forceinline__ void jrot(const double* A, int ld, int p, int q, double& c, double& s, double& t) {
  const double apq = A[(long)p * ld + q];
  if (apq == 0.0) {
    c = 1.0;
    s = 0.0;
    t = 0.0;
    return;
  }
  const double th = (A[(long)q * ld + q] - A[(long)p * ld + p]) / (2.0 * apq);
  const double at = fabs(th);
  t = at > 1e150 ? 0.5 / th : copysign(1.0, th) / (at + sqrt(at * at + 1.0));
  c = 1.0 / sqrt(t * t + 1.0);
  s = t * c;
}

__global__ void k_jacobi_setup(const double* __restrict__ A, int n, int ld, double* __restrict__ W,
                               double* __restrict__ V) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)ld * ld) return;
  const int i = (int)(e / ld), j = (int)(e - (long)i * ld);
  W[e] = (i < n && j < n) ? 0.5 * (A[(long)i * n + j] + A[(long)j * n + i]) : 0.0;
  V[e] = i == j ? 1.0 : 0.0;
}

__global__ __launch_bounds__(256) void k_jacobi_round(const double* __restrict__ A, double* __restrict__ Ao,
                                                      double* __restrict__ V, int ld, int round) {
  const int h = ld >> 1;
  const long nA = (long)h * h;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nA) {
    const int i = (int)(e / h), j = (int)(e - (long)i * h);
    if (i > j) return;
    int pi, qi;
    rr_pair(ld, round, i, pi, qi);
    double ci, si, ti;
    jrot(A, ld, pi, qi, ci, si, ti);
    if (i == j) {
      const double apq = A[(long)pi * ld + qi];
      Ao[(long)pi * ld + pi] = A[(long)pi * ld + pi] - ti * apq;
      Ao[(long)qi * ld + qi] = A[(long)qi * ld + qi] + ti * apq;
      Ao[(long)pi * ld + qi] = 0.0;
      Ao[(long)qi * ld + pi] = 0.0;
      return;
    }
    int pj, qj;
    rr_pair(ld, round, j, pj, qj);
    double cj, sj, tj;
    jrot(A, ld, pj, qj, cj, sj, tj);
    const double b00 = A[(long)pi * ld + pj], b01 = A[(long)pi * ld + qj];
    const double b10 = A[(long)qi * ld + pj], b11 = A[(long)qi * ld + qj];
    const double m00 = ci * b00 - si * b10, m01 = ci * b01 - si * b11;
    const double m10 = si * b00 + ci * b10, m11 = si * b01 + ci * b11;
    const double r00 = cj * m00 - sj * m01, r01 = sj * m00 + cj * m01;
    const double r10 = cj * m10 - sj * m11, r11 = sj * m10 + cj * m11;
    Ao[(long)pi * ld + pj] = r00;
    Ao[(long)pi * ld + qj] = r01;
    Ao[(long)qi * ld + pj] = r10;
    Ao[(long)qi * ld + qj] = r11;
    Ao[(long)pj * ld + pi] = r00;
    Ao[(long)qj * ld + pi] = r01;
    Ao[(long)pj * ld + qi] = r10;
    Ao[(long)qj * ld + qi] = r11;
    return;
  }
  // eigenvector columns: V <- V J, one (row, pair) per thread
  const long e2 = e - nA;
  if (e2 >= (long)ld * h) return;
  const int r = (int)(e2 / h), j = (int)(e2 - (long)r * h);
  int pj, qj;
  rr_pair(ld, round, j, pj, qj);
  double cj, sj, tj;
  jrot(A, ld, pj, qj, cj, sj, tj);
  const double vp = V[(long)r * ld + pj], vq = V[(long)r * ld + qj];
  V[(long)r * ld + pj] = cj * vp - sj * vq;
  V[(long)r * ld + qj] = sj * vp + cj * vq;
}

// The whole eigensolve of a matrix of order ld <= kSmallLd in one block: A in LDS,
// V in global memory (each (row, pair) is owned by one thread), the rotations of a
// round computed into LDS first, then every 2x2 block rotated in place by the thread
// that owns it.  The same stopping rule as the multi-launch path, tested after every
// sweep; stat = (sweeps, off-diagonal norm^2, total norm^2).
constexpr int kSmallLd = 128;

__global__ __launch_bounds__(1024) void k_jacobi_small(double* __restrict__ Ag, double* __restrict__ V, int ld,
                                                       int max_sweeps, double* __restrict__ stat) {
  __shared__ double A[kSmallLd * kSmallLd];
  __shared__ double cs[kSmallLd / 2], sn[kSmallLd / 2], tn[kSmallLd / 2];
  __shared__ double red[1024 / 64];
  __shared__ int flag;
  const int tid = threadIdx.x, nt = blockDim.x, h = ld >> 1;
  const int LL = ld * ld;
  for (int e = tid; e < LL; e += nt) A[e] = Ag[e];
  __syncthreads();
  // Frobenius norms: off-diagonal and total (fixed order: per-thread strided, then waves, then lanes)
  auto norms = [&](double& off, double& tot) {
    double o = 0.0, d = 0.0;
    for (int e = tid; e < LL; e += nt) {
      const int i = e / ld, j = e - i * ld;
      const double a = A[e];
      if (i == j) d += a * a;
      else o += a * a;
    }
    double v2[2] = {o, d};
    for (int k = 0; k < 2; ++k) {
      double v = v2[k];
      for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
      if ((tid & 63) == 0) red[tid >> 6] = v;
      __syncthreads();
      double r = 0.0;
      for (int w = 0; w < nt / 64; ++w) r += red[w];
      __syncthreads();
      v2[k] = r;
    }
    off = v2[0];
    tot = v2[0] + v2[1];
  };
  double off, total;
  norms(off, total);
  double prev = off;
  int sw = 0;
  while (off > 1e-30 * total && sw < max_sweeps) {
    for (int r = 0; r < ld - 1; ++r) {
      for (int k = tid; k < h; k += nt) {
        int p, q;
        rr_pair(ld, r, k, p, q);
        double c, s, t;
        jrot(A, ld, p, q, c, s, t);
        cs[k] = c;
        sn[k] = s;
        tn[k] = t;
      }
      __syncthreads();
      for (long e = tid; e < (long)h * h + (long)ld * h; e += nt) {
        if (e < (long)h * h) {
          const int i = (int)(e / h), j = (int)(e - (long)i * h);
          if (i > j) continue;
          int pi, qi;
          rr_pair(ld, r, i, pi, qi);
          const double ci = cs[i], si = sn[i];
          if (i == j) {
            const double apq = A[pi * ld + qi], ti = tn[i];
            A[pi * ld + pi] -= ti * apq;
            A[qi * ld + qi] += ti * apq;
            A[pi * ld + qi] = 0.0;
            A[qi * ld + pi] = 0.0;
            continue;
          }
          int pj, qj;
          rr_pair(ld, r, j, pj, qj);
          const double cj = cs[j], sj = sn[j];
          const double b00 = A[pi * ld + pj], b01 = A[pi * ld + qj];
          const double b10 = A[qi * ld + pj], b11 = A[qi * ld + qj];
          const double m00 = ci * b00 - si * b10, m01 = ci * b01 - si * b11;
          const double m10 = si * b00 + ci * b10, m11 = si * b01 + ci * b11;
          const double r00 = cj * m00 - sj * m01, r01 = sj * m00 + cj * m01;
          const double r10 = cj * m10 - sj * m11, r11 = sj * m10 + cj * m11;
          A[pi * ld + pj] = r00;
          A[pi * ld + qj] = r01;
          A[qi * ld + pj] = r10;
          A[qi * ld + qj] = r11;
          A[pj * ld + pi] = r00;
          A[qj * ld + pi] = r01;
          A[pj * ld + qi] = r10;
          A[qj * ld + qi] = r11;
        } else {
          const long e2 = e - (long)h * h;
          const int row = (int)(e2 / h), j = (int)(e2 - (long)row * h);
          int pj, qj;
          rr_pair(ld, r, j, pj, qj);
          const double cj = cs[j], sj = sn[j];
          const double vp = V[(long)row * ld + pj], vq = V[(long)row * ld + qj];
          V[(long)row * ld + pj] = cj * vp - sj * vq;
          V[(long)row * ld + qj] = sj * vp + cj * vq;
        }
      }
      __syncthreads();
    }
    ++sw;
    norms(off, total);
    if (tid == 0) flag = (off <= 1e-26 * total && off > 0.25 * prev) ? 1 : 0;
    __syncthreads();
    const int stop = flag;
    __syncthreads();
    if (stop) break;
    prev = off;
  }
  for (int e = tid; e < LL; e += nt) Ag[e] = A[e];
  if (tid == 0) {
    stat[0] = (double)sw;
    stat[1] = off;
    stat[2] = total;
  }
}

// L = chol(A) (lower) in LDS, then Linv = L^-1 by forward substitution, one
// column per thread, for n <= kSmallLd; info = first failing column + 1.  For
// 2 n^2 <= kSmallLd^2 the inverse is built in LDS next to L and copied out at
// the end, otherwise in global memory.
__global__ __launch_bounds__(256) void k_chol_inv_small(const double* __restrict__ Ag, double* __restrict__ Linv,
                                                        int n, int* info) {
  __shared__ double sm[kSmallLd * kSmallLd];
  __shared__ double djj;
  double* const L = sm;
  const bool lds_x = 2 * n * n <= kSmallLd * kSmallLd;
  double* const X = lds_x ? sm + n * n : Linv;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < n * n; e += nt) L[e] = Ag[e];
  if (tid == 0) *info = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    // d = A_jj - sum_k<j L_jk^2 (one wave, fixed shuffle tree)
    if (tid < 64) {
      double acc = 0.0;
      for (int k = tid; k < j; k += 64) acc += L[j * n + k] * L[j * n + k];
      for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
      if (tid == 0) {
        double d = L[j * n + j] - acc;
        if (!(d > 0.0)) {
          if (*info == 0) *info = j + 1;
          d = 1.0;
        }
        djj = sqrt(d);
        L[j * n + j] = djj;
      }
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < n; i += nt) {
      double t = L[i * n + j];
      for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / djj;
    }
    __syncthreads();
  }
  for (int c = tid; c < n; c += nt) {
    for (int i = 0; i < c; ++i) X[i * n + c] = 0.0;
    for (int i = c; i < n; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) t -= L[i * n + k] * X[k * n + c];
      X[i * n + c] = t / L[i * n + i];
    }
  }
  if (lds_x) {
    __syncthreads();
    for (int e = tid; e < n * n; e += nt) Linv[e] = X[e];
  }
}

__global__ __launch_bounds__(256) void k_jacobi_offdiag(const double* __restrict__ A, int ld, double* out) {
  __shared__ double sh[256];
  double off = 0.0, dg = 0.0;
  for (long e = threadIdx.x; e < (long)ld * ld; e += 256) {
    const int i = (int)(e / ld), j = (int)(e - (long)i * ld);
    const double a = A[e];
    if (i == j) dg += a * a;
    else off += a * a;
  }
  off = gs_block_sum(off, sh);
  dg = gs_block_sum(dg, sh);
  if (threadIdx.x == 0) {
    out[0] = off;
    out[1] = dg;
  }
}

__global__ void k_jacobi_rank(const double* __restrict__ A, int n, int ld, double* __restrict__ evals,
                              int* __restrict__ rank) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double li = A[(long)i * ld + i];
  int r = 0;
  for (int j = 0; j < n; ++j) {
    const double lj = A[(long)j * ld + j];
    r += (lj < li || (lj == li && j < i)) ? 1 : 0;
  }
  rank[i] = r;
  evals[r] = li;
}

__global__ void k_jacobi_perm(const double* __restrict__ V, int n, int ld, const int* __restrict__ rank,
                              double* __restrict__ vecs) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const int r = (int)(e / n), i = (int)(e - (long)r * n);
  vecs[(long)rank[i] * n + r] = V[(long)r * ld + i];
}

// ---------------------------------------------------------------------------
// Block kernels
// ---------------------------------------------------------------------------
// res[i] = sqrt(h3 sum_r (HX[i][r] - ev[i] X[i][r])^2): kResChunks blocks per row
// write partial sums, then one thread per row adds them in order.
constexpr int kResChunks = 16;

__global__ __launch_bounds__(256) void k_row_residual_parts(const double* __restrict__ HX,
                                                            const double* __restrict__ X,
                                                            const double* __restrict__ ev, long ng,
                                                            double* __restrict__ part) {
  __shared__ double sh[256];
  const int i = blockIdx.x, ch = blockIdx.y;
  const double l = ev[i];
  const double* hx = HX + (long)i * ng;
  const double* x = X + (long)i * ng;
  double acc = 0.0;
  for (long r = (long)ch * 256 + threadIdx.x; r < ng; r += (long)kResChunks * 256) {
    const double d = hx[r] - l * x[r];
    acc += d * d;
  }
  acc = gs_block_sum(acc, sh);
  if (threadIdx.x == 0) part[(long)i * kResChunks + ch] = acc;
}

__global__ void k_row_residual_final(const double* __restrict__ part, int n, double h3, double* __restrict__ res) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = 0.0;
  for (int c = 0; c < kResChunks; ++c) a += part[(long)i * kResChunks + c];
  res[i] = sqrt(h3 * a);
}

__global__ void k_occ_density(const double* __restrict__ X, const double* __restrict__ occ, int n, long ng,
                              double* __restrict__ rho) {
  for (long r = (long)blockIdx.x * blockDim.x + threadIdx.x; r < ng; r += (long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int i = 0; i < n; ++i) {
      const double f = occ[i];
      if (f != 0.0) {
        const double x = X[(long)i * ng + r];
        acc += f * (x * x);
      }
    }
    rho[r] = acc;
  }
}

__global__ __launch_bounds__(256) void k_abs_max(const double* __restrict__ v, long n, unsigned long long* slot) {
  __shared__ double sh[256];
  double m = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    m = fmax(m, fabs(v[i]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(slot, (unsigned long long)__double_as_longlong(sh[0]));
}

__global__ __launch_bounds__(256) void k_count_nonfinite(const double* __restrict__ v, long n,
                                                         unsigned long long* count) {
  unsigned long long k = 0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    k += isfinite(v[i]) ? 0ull : 1ull;
  if (k) atomicAdd(count, k);
}

// First index of the largest |x| in the row, then the row times the sign there.
__global__ __launch_bounds__(256) void k_fix_signs(double* __restrict__ X, long ng) {
  __shared__ double sv[256];
  __shared__ long si[256];
  double* x = X + (long)blockIdx.x * ng;
  double best = -1.0;
  long bi = 0;
  for (long r = threadIdx.x; r < ng; r += 256) {
    const double a = fabs(x[r]);
    if (a > best) {  // r increases per thread: ties keep the first
      best = a;
      bi = r;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double a = sv[threadIdx.x + o];
      const long ia = si[threadIdx.x + o];
      if (a > sv[threadIdx.x] || (a == sv[threadIdx.x] && ia < si[threadIdx.x])) {
        sv[threadIdx.x] = a;
        si[threadIdx.x] = ia;
      }
    }
    __syncthreads();
  }
  const double sg = x[si[0]] < 0.0 ? -1.0 : 1.0;
  __syncthreads();
  if (sg < 0.0)
    for (long r = threadIdx.x; r < ng; r += 256) x[r] = -x[r];
}

// ---------------------------------------------------------------------------
// Pulay mixing (P. Pulay, Chem. Phys. Lett. 73, 393 (1980)): the coefficients
// minimise the norm of the combined density residual under sum c_k = 1.
// ---------------------------------------------------------------------------
constexpr int kDotBlocks = 256;
constexpr int kMaxDepth = 8;

__global__ __launch_bounds__(256) void k_pulay_dots(const double* __restrict__ res, int snew, long ng,
                                                    double* __restrict__ part) {
  __shared__ double sh[256];
  const int k = blockIdx.y, b = blockIdx.x;
  const double* a = res + (long)k * ng;
  const double* z = res + (long)snew * ng;
  double acc = 0.0;
  for (long r = (long)b * 256 + threadIdx.x; r < ng; r += (long)kDotBlocks * 256) acc += a[r] * z[r];
  acc = gs_block_sum(acc, sh);
  if (threadIdx.x == 0) part[(long)k * kDotBlocks + b] = acc;
}

// One wave per stored residual sums its kDotBlocks partial dot products (fixed
// lane order and shuffle tree), then one thread solves the small system.
__global__ __launch_bounds__(64 * kMaxDepth) void k_pulay_solve(const double* __restrict__ part, int m, int snew,
                                                                int depth, double* __restrict__ B,
                                                                double* __restrict__ coef) {
  __shared__ double dk[kMaxDepth];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (w < m) {
    double d = 0.0;
    for (int b = lane; b < kDotBlocks; b += 64) d += part[(long)w * kDotBlocks + b];
    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o);
    if (lane == 0) dk[w] = d;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 0; k < m; ++k) {
    B[k * depth + snew] = dk[k];
    B[snew * depth + k] = dk[k];
  }
  // bordered system [B 1; 1^T 0] [c; lambda] = [0; 1]
  const int n = m + 1;
  double M[kMaxDepth + 1][kMaxDepth + 2];
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) M[i][j] = (i < m && j < m) ? B[i * depth + j] : ((i < m || j < m) ? 1.0 : 0.0);
    M[i][n] = i == m ? 1.0 : 0.0;
  }
  bool ok = true;
  for (int col = 0; col < n && ok; ++col) {
    int piv = col;
    for (int i = col + 1; i < n; ++i)
      if (fabs(M[i][col]) > fabs(M[piv][col])) piv = i;
    if (!(fabs(M[piv][col]) > 1e-300)) {
      ok = false;
      break;
    }
    if (piv != col)
      for (int j = 0; j <= n; ++j) {
        const double t = M[col][j];
        M[col][j] = M[piv][j];
        M[piv][j] = t;
      }
    for (int i = col + 1; i < n; ++i) {
      const double f = M[i][col] / M[col][col];
      for (int j = col; j <= n; ++j) M[i][j] -= f * M[col][j];
    }
  }
  double c[kMaxDepth + 1];
  if (ok) {
    for (int i = n - 1; i >= 0; --i) {
      double t = M[i][n];
      for (int j = i + 1; j < n; ++j) t -= M[i][j] * c[j];
      c[i] = t / M[i][i];
    }
    for (int k = 0; k < m; ++k) ok = ok && isfinite(c[k]);
  }
  for (int k = 0; k < m; ++k) coef[k] = ok ? c[k] : (k == snew ? 1.0 : 0.0);
}

__global__ void k_pulay_mix(const double* __restrict__ in, const double* __restrict__ res,
                            const double* __restrict__ coef, int m, double beta, long ng, double* __restrict__ rho) {
  for (long r = (long)blockIdx.x * blockDim.x + threadIdx.x; r < ng; r += (long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int k = 0; k < m; ++k) acc += coef[k] * (in[(long)k * ng + r] + beta * res[(long)k * ng + r]);
    rho[r] = acc;
  }
}

int grid_blocks(long n) {
  const long b = (n + 255) / 256;
  return (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

}  // namespace

hipError_t jacobi_setup(hipStream_t s, const double* A, int n, int ld, double* W, double* V) {
  hipLaunchKernelGGL(k_jacobi_setup, dim3(gs_cdiv((long)ld * ld, 256)), dim3(256), 0, s, A, n, ld, W, V);
  return hipGetLastError();
}

hipError_t jacobi_round(hipStream_t s, const double* A, double* Aout, double* V, int ld, int round) {
  const long h = ld / 2;
  const long threads = h * h + (long)ld * h;
  hipLaunchKernelGGL(k_jacobi_round, dim3(gs_cdiv(threads, 256)), dim3(256), 0, s, A, Aout, V, ld, round);
  return hipGetLastError();
}

int jacobi_small_max() { return kSmallLd; }

hipError_t jacobi_small(hipStream_t s, double* A, double* V, int ld, int max_sweeps, double* stat) {
  if (ld > kSmallLd || ld < 2 || (ld & 1)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_jacobi_small, dim3(1), dim3(1024), 0, s, A, V, ld, max_sweeps, stat);
  return hipGetLastError();
}

hipError_t chol_inv_small(hipStream_t s, const double* A, double* Linv, int n, int* info) {
  if (n > kSmallLd || n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chol_inv_small, dim3(1), dim3(256), 0, s, A, Linv, n, info);
  return hipGetLastError();
}

hipError_t jacobi_offdiag(hipStream_t s, const double* A, int ld, double* out) {
  hipLaunchKernelGGL(k_jacobi_offdiag, dim3(1), dim3(256), 0, s, A, ld, out);
  return hipGetLastError();
}

hipError_t jacobi_sort(hipStream_t s, const double* A, const double* V, int n, int ld, double* evals, double* vecs,
                       int* rank) {
  hipLaunchKernelGGL(k_jacobi_rank, dim3(gs_cdiv(n, 256)), dim3(256), 0, s, A, n, ld, evals, rank);
  hipLaunchKernelGGL(k_jacobi_perm, dim3(gs_cdiv((long)n * n, 256)), dim3(256), 0, s, V, n, ld, rank, vecs);
  return hipGetLastError();
}

int row_residual_parts() { return kResChunks; }

hipError_t row_residuals(hipStream_t s, const double* HX, const double* X, const double* ev, int n, long ng,
                         double h3, double* res, double* part) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_residual_parts, dim3(n, kResChunks), dim3(256), 0, s, HX, X, ev, ng, part);
  hipLaunchKernelGGL(k_row_residual_final, dim3(gs_cdiv(n, 256)), dim3(256), 0, s, part, n, h3, res);
  return hipGetLastError();
}

hipError_t occ_density(hipStream_t s, const double* X, const double* occ, int n, long ng, double* rho) {
  hipLaunchKernelGGL(k_occ_density, dim3(grid_blocks(ng)), dim3(256), 0, s, X, occ, n, ng, rho);
  return hipGetLastError();
}

hipError_t abs_max(hipStream_t s, const double* v, long n, unsigned long long* slot) {
  const int nb = grid_blocks(n) > 256 ? 256 : grid_blocks(n);
  hipLaunchKernelGGL(k_abs_max, dim3(nb), dim3(256), 0, s, v, n, slot);
  return hipGetLastError();
}

hipError_t count_nonfinite(hipStream_t s, const double* v, long n, unsigned long long* count) {
  const int nb = grid_blocks(n) > 1024 ? 1024 : grid_blocks(n);
  hipLaunchKernelGGL(k_count_nonfinite, dim3(nb), dim3(256), 0, s, v, n, count);
  return hipGetLastError();
}

hipError_t fix_signs(hipStream_t s, double* X, int n, long ng) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fix_signs, dim3(n), dim3(256), 0, s, X, ng);
  return hipGetLastError();
}

hipError_t pulay_dots(hipStream_t s, const double* res, int m, int snew, long ng, double* part) {
  hipLaunchKernelGGL(k_pulay_dots, dim3(kDotBlocks, m), dim3(256), 0, s, res, snew, ng, part);
  return hipGetLastError();
}

hipError_t pulay_solve(hipStream_t s, const double* part, int m, int snew, int depth, double* B, double* coef) {
  if (m < 1 || m > kMaxDepth || depth > kMaxDepth || snew >= m) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pulay_solve, dim3(1), dim3(64 * kMaxDepth), 0, s, part, m, snew, depth, B, coef);
  return hipGetLastError();
}

hipError_t pulay_mix(hipStream_t s, const double* in, const double* res, const double* coef, int m, double beta,
                     long ng, double* rho) {
  hipLaunchKernelGGL(k_pulay_mix, dim3(grid_blocks(ng)), dim3(256), 0, s, in, res, coef, m, beta, ng, rho);
  return hipGetLastError();
}

}  // namespace rtk
