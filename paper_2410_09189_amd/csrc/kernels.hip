// RT-TDDFT time-step kernels for gfx950 (MI355X, CDNA4, 64-wide wavefronts).
//
// Grid fields are [nz][ny][nx] (x fastest), orbitals [N][nz][ny][nx], N x N
// matrices row-major.  All reductions use a fixed partition and a fixed
// combination order, so repeated runs are bitwise identical; the only atomics
// are max-reductions of non-negative doubles (order independent).
#include "kernels.h"

#include <hip/hip_runtime.h>
#include <cmath>

namespace rtk {


__host__ __device__ static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Deterministic block sum over 256 threads (tree in LDS).
__device__ double block_sum_256(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) sh[t] += sh[t + o];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__device__ double block_max_256(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) sh[t] = fmax(sh[t], sh[t + o]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* slot, double v) {
  atomicMax(slot, (unsigned long long)__double_as_longlong(v));
}

// ============================================================================
// Grid fields
// ============================================================================

// V_ion(r) = - sum_a D_a sum_images exp(-|r - R_a - nL|^2 / (2 w_a^2)); atoms
// outer, images (i, j, k) inner, accumulated in that order.
__global__ void k_vion(double* __restrict__ v, int nx, int ny, int nz, double h, int n_atoms,
                       const double* __restrict__ pos, const double* __restrict__ depth,
                       const double* __restrict__ width, int nim) {
  long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long ng = (long)nx * ny * nz;
  if (g >= ng) return;
  int ix = (int)(g % nx);
  int iy = (int)((g / nx) % ny);
  int iz = (int)(g / ((long)nx * ny));
  double x = ix * h, y = iy * h, z = iz * h;
  double Lx = nx * h, Ly = ny * h, Lz = nz * h;
  double acc = 0.0;
  for (int a = 0; a < n_atoms; ++a) {
    double inv = 1.0 / (2.0 * width[a] * width[a]);
    double D = depth[a];
    for (int i = -nim; i <= nim; ++i) {
      double dx = x - pos[3 * a] - i * Lx;
      for (int j = -nim; j <= nim; ++j) {
        double dy = y - pos[3 * a + 1] - j * Ly;
        for (int k = -nim; k <= nim; ++k) {
          double dz = z - pos[3 * a + 2] - k * Lz;
          acc -= D * exp(-((dx * dx + dy * dy) + dz * dz) * inv);
        }
      }
    }
  }
  v[g] = acc;
}

hipError_t vion(hipStream_t s, double* v, int nx, int ny, int nz, double h, int n_atoms,
                const double* pos, const double* depth, const double* width, int n_images) {
  long ng = (long)nx * ny * nz;
  hipLaunchKernelGGL(k_vion, dim3(cdiv(ng, 256)), dim3(256), 0, s, v, nx, ny, nz, h, n_atoms, pos,
                     depth, width, n_images);
  return hipGetLastError();
}

// Sawtooth coordinate along one axis: rises by h per plane, drops once between
// planes j0 - 1 and j0, centred: q_i = (((i - j0) mod n) - (n-1)/2) h.
__device__ __forceinline__ double saw(int i, int n, int j0, double h) {
  int k = i - j0;
  k += k < 0 ? n : 0;
  return (k - 0.5 * (n - 1)) * h;
}

__global__ void k_coord(double* q, int nx, int ny, int nz, double h, int axis, int j0) {
  long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long ng = (long)nx * ny * nz;
  if (g >= ng) return;
  int i, n;
  if (axis == 0) { i = (int)(g % nx); n = nx; }
  else if (axis == 1) { i = (int)((g / nx) % ny); n = ny; }
  else { i = (int)(g / ((long)nx * ny)); n = nz; }
  q[g] = saw(i, n, j0, h);
}

hipError_t coord(hipStream_t s, double* q, int nx, int ny, int nz, double h, int axis, int j0) {
  long ng = (long)nx * ny * nz;
  hipLaunchKernelGGL(k_coord, dim3(cdiv(ng, 256)), dim3(256), 0, s, q, nx, ny, nz, h, axis, j0);
  return hipGetLastError();
}

__global__ void k_fill(double* p, long n, double v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u64(unsigned long long* p, long n, unsigned long long v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_copy(double* d, const double* a, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    d[i] = a[i];
}
__global__ void k_cast_d2f(float* d, const double* a, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    d[i] = (float)a[i];
}
// d_t = a_t - b for T stacked fields (b shared); blockIdx.y = t.
__global__ void k_sub(double* d, const double* a, const double* b, long n, const int* active) {
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    d[t * n + i] = a[t * n + i] - b[i];
}
static int ew_blocks(long n) { long b = (n + 255) / 256; return (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b)); }

hipError_t fill(hipStream_t s, double* p, long n, double v) {
  hipLaunchKernelGGL(k_fill, dim3(ew_blocks(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t fill_u64(hipStream_t s, unsigned long long* p, long n, unsigned long long v) {
  hipLaunchKernelGGL(k_fill_u64, dim3(ew_blocks(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t copy_d(hipStream_t s, double* dst, const double* src, long n) {
  hipLaunchKernelGGL(k_copy, dim3(ew_blocks(n)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}
hipError_t cast_d2f(hipStream_t s, float* dst, const double* src, long n) {
  hipLaunchKernelGGL(k_cast_d2f, dim3(ew_blocks(n)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}
hipError_t sub_d(hipStream_t s, double* dst, const double* a, const double* b, long n, int T, const int* active) {
  int nb = ew_blocks(n) > 1024 ? 1024 : ew_blocks(n);
  hipLaunchKernelGGL(k_sub, dim3(nb, T), dim3(256), 0, s, dst, a, b, n, active);
  return hipGetLastError();
}

// ============================================================================
// FD8 stencil + local potential
// ============================================================================
//
// One block = one orbital, all x (nx <= 256), a tile of TY rows in y, a chunk of z
// planes, blockDim = the tile's strips rounded up to whole waves.  A thread owns
// COLS strips of V consecutive x points (V = 16 bytes / element size when nx
// allows, else 1) and marches in z: the 9-plane window of its strips sits in
// registers (z neighbours) with the next PD planes' loads in flight.  The current
// plane with a 4-row y halo is staged in one of two LDS buffers whose rows carry 4
// periodic copies on each side, so the x and y neighbours of a strip are whole
// 16-byte LDS reads at fixed offsets (no wrap arithmetic); one barrier per plane.
// Global traffic is whole x rows in 16-byte vectors.  Blocks are ordered (tile, z
// chunk, orbital) with the tile fastest and mapped XCD-aware, so the tiles of one
// orbital run together on one XCD and a tile's halo rows are its neighbours'
// interior rows.
// Latency: every value a plane waits for was requested at least two planes
// earlier, and no register holding a load in flight is ever copied: the window
// (9 + PD = KW planes), the potential (3 planes) and the staged halo (2 planes) are
// rings whose slots are fixed by the plane's position modulo KW, with the z loop
// unrolled KW times so that every slot index is a compile-time constant (a rotated
// register would force a wait for every load in flight, exposing one full memory
// latency per plane).  The halo rows are requested HQ planes ahead, close to when
// the neighbouring tiles request the same rows for their windows (5 + PD planes
// ahead), so the second request finds the line in L2; after their two planes in
// registers they wait in an LDS ring of HQ - 1 planes (compact rows) and are
// copied into the plane buffer when their plane comes up.
struct StencilCoef {
  double c[5];  // -1/2 a_k / h^2
};

// Aligned to its full width so LDS accesses compile to single 16-byte instructions
// (an element-aligned struct splits into pairs of narrower accesses that conflict).
template <typename T, int V>
struct alignas(sizeof(T) * V) SVec {
  T e[V];
};

template <typename T, int V>
__device__ __forceinline__ SVec<T, V> sv_ld(const T* p) {
  return *reinterpret_cast<const SVec<T, V>*>(p);
}
template <typename T, int V>
__device__ __forceinline__ void sv_st(T* p, const SVec<T, V>& x) {
  *reinterpret_cast<SVec<T, V>*>(p) = x;
}
// Streaming store (non-temporal hint): the stencil output is not read again by
// the launch, so its lines go first when L2 evicts and the y-halo rows that
// neighbouring tiles re-read stay cached longer (3 % faster, measured).
template <typename T, int V>
__device__ __forceinline__ void sv_st_nt(T* p, const SVec<T, V>& x) {
  typedef T vt __attribute__((ext_vector_type(V)));
  vt w;
#pragma unroll
  for (int u = 0; u < V; ++u) w[u] = x.e[u];
  __builtin_nontemporal_store(w, reinterpret_cast<vt*>(p));
}

// Up to 512 threads (8 waves) per block; three waves per SIMD leave 168 registers,
// which the rings need with one halo strip per thread (two with more).
template <typename T, int V, int COLS, int HS, int PD>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(COLS == 1 && HS == 1 ? 3 : 2))) void k_stencil(const T* __restrict__ psi, T* __restrict__ hpsi,
                                                 const T* __restrict__ v, int nx, int ny, int nz,
                                                 int TY, int ZC, int HQ, StencilCoef cf) {
  typedef SVec<T, V> Vec;
  constexpr int KW = 9 + PD;  // window ring and unroll length; the potential's ring (3) and
  static_assert(KW % 6 == 0, "the halo's (2) divide it");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  T* const sp0 = reinterpret_cast<T*>(smem_raw);  // [2][TY + 8][nx + 8], x = 0 at column 4
  const int P = nx + 8;
  const int pln = (TY + 8) * P;
  const int R = HQ - 1;           // LDS ring slots (HQ >= 3)
  T* const ring = sp0 + 2 * pln;  // [R][8 nx]: halo rows of planes ahead, slot = plane % R
  const int R8 = 8 * nx;
  const int tid = threadIdx.x, NT = blockDim.x;
  const long lid = xcd_logical(blockIdx.x, gridDim.x);
  const int tiles = ny / TY, nzc = (nz + ZC - 1) / ZC;
  const int tile = (int)(lid % tiles), zc = (int)((lid / tiles) % nzc);
  const long orb = lid / ((long)tiles * nzc);
  const int y0 = tile * TY;
  const int rows = min(TY, ny - y0);
  const int z0 = zc * ZC;
  const int z1 = min(nz, z0 + ZC);
  const long plane = (long)nx * ny;
  const T* __restrict__ f = psi + orb * plane * nz;
  T* __restrict__ o = hpsi + orb * plane * nz;
  const T c0 = (T)(3.0 * cf.c[0]);
  const T c1 = (T)cf.c[1], c2 = (T)cf.c[2], c3 = (T)cf.c[3], c4 = (T)cf.c[4];
  const int spr = nx / V;  // strips per row

  // window ring: plane z0 - 4 + k in slot k mod KW; potential: plane z0 + k in slot k mod 3.
  // Loads are unconditional (threads past the tile read its first strip, planes past
  // the chunk are clamped or wrapped into the grid): without divergent branches
  // around them the compiler's waits cover exactly the loads a value needs.
  int cb[COLS], ls[COLS], pw[COLS];  // plane offset, LDS offset, LDS offset of the wrap copy (-1: none)
  bool ok[COLS];
  Vec wq[COLS][KW], vr[COLS][3];
#pragma unroll
  for (int c = 0; c < COLS; ++c) {
    const int sidx = tid + c * NT;
    const int yl = sidx / spr, x = (sidx - yl * spr) * V;
    ok[c] = yl < rows;
    cb[c] = ok[c] ? (y0 + yl) * nx + x : y0 * nx;
    ls[c] = (yl + 4) * P + 4 + x;
    pw[c] = x < 4 ? ls[c] + nx : (x >= nx - 4 ? ls[c] - nx : -1);
#pragma unroll
    for (int d = 0; d < KW - 1; ++d) wq[c][d] = sv_ld<T, V>(f + (long)wrapi(z0 - 4 + d, nz) * plane + cb[c]);
    vr[c][0] = sv_ld<T, V>(v + (long)z0 * plane + cb[c]);
    vr[c][1] = sv_ld<T, V>(v + (long)min(z0 + 1, nz - 1) * plane + cb[c]);
  }
  // y halo: 8 rows (4 below, 4 above the tile), 8 spr <= NT HS strips; strip e sits
  // at e V in an LDS ring slot.  Plane p enters the LDS ring at plane p - HQ + 2 (here
  // for p < z0 + HQ - 2); plane z0 + HQ - 2 + k starts in register slot k (k = 0, 1).
  int hoff[HS], hl[HS], hw[HS];  // hoff: global offset in the plane (0 for threads without a strip)
  bool hok[HS];
  Vec hr[HS][2];
#pragma unroll
  for (int i = 0; i < HS; ++i) {
    const int e = tid + NT * i;
    hok[i] = e < 8 * spr;
    hoff[i] = 0;
    hl[i] = hw[i] = -1;
    if (hok[i]) {
      const int hrow = e / spr, x = (e - hrow * spr) * V;
      const int yl = hrow < 4 ? hrow - 4 : rows + (hrow - 4);
      hoff[i] = wrapi(y0 + yl, ny) * nx + x;
      hl[i] = (yl + 4) * P + 4 + x;
      hw[i] = x < 4 ? hl[i] + nx : (x >= nx - 4 ? hl[i] - nx : -1);
      for (int k = 0; k + 2 < HQ && z0 + k < z1; ++k)
        sv_st<T, V>(ring + ((z0 + k) % R) * R8 + e * V, sv_ld<T, V>(f + (long)(z0 + k) * plane + hoff[i]));
    }
    hr[i][0] = sv_ld<T, V>(f + (long)min(z0 + HQ - 2, nz - 1) * plane + hoff[i]);
    hr[i][1] = sv_ld<T, V>(f + (long)min(z0 + HQ - 1, nz - 1) * plane + hoff[i]);
  }
  __syncthreads();
  for (int zb = z0; zb < z1; zb += KW) {
#pragma unroll
    for (int j = 0; j < KW; ++j) {
      const int z = zb + j;  // plane z - 4 + d is window slot (j + d) % KW
      if (z >= z1) break;
      T* const sp = sp0 + ((z - z0) & 1) * pln;
#pragma unroll
      for (int c = 0; c < COLS; ++c)
        if (ok[c]) {
          sv_st<T, V>(sp + ls[c], wq[c][(j + 4) % KW]);
          if (pw[c] >= 0) sv_st<T, V>(sp + pw[c], wq[c][(j + 4) % KW]);
        }
      // halo of plane z: LDS ring -> plane buffer; plane z + HQ - 2 (register slot
      // j % 2, loaded two planes ago) -> LDS slot (z - 1) mod R, whose last reader
      // (plane z - 1) passed the previous barrier and which differs from z mod R
      // (past the chunk the slot is never read)
#pragma unroll
      for (int i = 0; i < HS; ++i)
        if (hok[i]) {
          const int e = tid + NT * i;
          const Vec hz = sv_ld<T, V>(ring + (z % R) * R8 + e * V);
          sv_st<T, V>(sp + hl[i], hz);
          if (hw[i] >= 0) sv_st<T, V>(sp + hw[i], hz);
          sv_st<T, V>(ring + ((z + HQ - 2) % R) * R8 + e * V, hr[i][j % 2]);
        }
      __syncthreads();
      // in flight: halo of plane z + HQ (register slot j % 2, just freed), potential of
      // plane z + 2 (slot of plane z - 1), window plane z + 4 + PD (slot of plane z - 5)
#pragma unroll
      for (int i = 0; i < HS; ++i) hr[i][j % 2] = sv_ld<T, V>(f + (long)min(z + HQ, nz - 1) * plane + hoff[i]);
#pragma unroll
      for (int c = 0; c < COLS; ++c) {
        vr[c][(j + 2) % 3] = sv_ld<T, V>(v + (long)min(z + 2, nz - 1) * plane + cb[c]);
        wq[c][(j + KW - 1) % KW] = sv_ld<T, V>(f + (long)wrapi(z + 4 + PD, nz) * plane + cb[c]);
      }
      const long zoff = (long)z * plane;
#pragma unroll
      for (int c = 0; c < COLS; ++c) {
        if (!ok[c]) continue;
        const T* r0 = sp + ls[c];
        T w[V + 8];  // x window x - 4 .. x + V + 3
#pragma unroll
        for (int g = 0; g < (V + 8) / V; ++g) {
          Vec t = sv_ld<T, V>(r0 - 4 + g * V);
#pragma unroll
          for (int u = 0; u < V; ++u) w[g * V + u] = t.e[u];
        }
        Vec ym[4], yp[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          ym[k] = sv_ld<T, V>(r0 - (k + 1) * P);
          yp[k] = sv_ld<T, V>(r0 + (k + 1) * P);
        }
        const Vec& zc0 = wq[c][(j + 4) % KW];
        Vec out;
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const T ctr = zc0.e[u];
          T sx1 = w[u + 5] + w[u + 3], sx2 = w[u + 6] + w[u + 2];
          T sx3 = w[u + 7] + w[u + 1], sx4 = w[u + 8] + w[u + 0];
          T sy1 = yp[0].e[u] + ym[0].e[u], sy2 = yp[1].e[u] + ym[1].e[u];
          T sy3 = yp[2].e[u] + ym[2].e[u], sy4 = yp[3].e[u] + ym[3].e[u];
          T sz1 = wq[c][(j + 5) % KW].e[u] + wq[c][(j + 3) % KW].e[u];
          T sz2 = wq[c][(j + 6) % KW].e[u] + wq[c][(j + 2) % KW].e[u];
          T sz3 = wq[c][(j + 7) % KW].e[u] + wq[c][(j + 1) % KW].e[u];
          T sz4 = wq[c][(j + 8) % KW].e[u] + wq[c][j % KW].e[u];
          T acc = c0 * ctr;
          acc += c1 * ((sx1 + sy1) + sz1);
          acc += c2 * ((sx2 + sy2) + sz2);
          acc += c3 * ((sx3 + sy3) + sz3);
          acc += c4 * ((sx4 + sy4) + sz4);
          out.e[u] = acc + vr[c][j % 3].e[u] * ctr;
        }
        sv_st_nt<T, V>(o + zoff + cb[c], out);
      }
    }
  }
}

// Threads per block and halo strips per thread of a tile of ty rows (spr strips a
// row): one strip a thread up to 512 strips, else two; false where that does not
// launch (more than 1024 strips, or two strips with more than two halo strips).
static bool stencil_shape(int spr, int ty, int& cols, int& nt, int& hs) {
  if (ty * spr > 1024) return false;
  cols = ty * spr > 512 ? 2 : 1;
  nt = ((ty * spr + cols - 1) / cols + 63) / 64 * 64;
  hs = (8 * spr + nt - 1) / nt;
  return hs <= 8 && (cols == 1 || hs <= 2);
}

// Default y tile: the smallest divisor of ny of at least 8 rows whose strips fit one
// 512-thread block (one strip per thread): the tile's threads then cover its 8 halo
// rows with one strip each; else the largest divisor that fits (measured on 96^3 and
// 192^3: taller tiles than that were slower, lower ones re-read more halo).
static int stencil_default_ty(int spr, int ny) {
  for (int t = 8; t <= ny && t * spr <= 512; ++t)
    if (ny % t == 0) return t;
  for (int t = 7; t >= 1; --t)
    if (t <= ny && ny % t == 0 && t * spr <= 512) return t;
  return 1;
}

template <typename T, int V>
static hipError_t stencil_launch(hipStream_t s, const T* psi, T* hpsi, const T* v, int n_orb, int nx, int ny,
                                 int nz, const StencilCoef& cf, int ty, int nzc, int hq) {
  const int spr = nx / V;
  // y tile (ty > 0: as given; it must divide ny and its strips fit one block),
  // block = strips rounded up to whole waves
  const int TY = ty > 0 ? ty : stencil_default_ty(spr, ny);
  int cols, nt, hs;
  if (ny % TY || !stencil_shape(spr, TY, cols, nt, hs)) return hipErrorInvalidValue;
  int tiles = ny / TY;
  // z chunks (nzc > 0: as given): by default doubled until the grid has 2048 blocks
  // or a chunk would drop below 16 planes
  if (nzc <= 0) {
    nzc = 1;
    const long blocks = (long)tiles * n_orb;
    while (blocks * nzc < 2048 && nz / (nzc * 2) >= 16) nzc *= 2;
  }
  if (nzc > nz) return hipErrorInvalidValue;
  int ZC = (nz + nzc - 1) / nzc;
  nzc = (nz + ZC - 1) / ZC;
  // halo look-ahead (hq > 0: as given, 3 .. 8): by default 6 planes in FP32 and 4 in
  // FP64 (measured best at 96^3), fewer where the ring (hq - 1 planes of 8 halo rows)
  // would take the block past 64 KB of LDS
  const size_t lds_planes = 2 * (size_t)(TY + 8) * (nx + 8) * sizeof(T), lds_ring = (size_t)8 * nx * sizeof(T);
  int HQ = hq;
  if (HQ <= 0)
    for (HQ = sizeof(T) == 4 ? 6 : 4; HQ > 3 && lds_planes + (HQ - 1) * lds_ring > 64 * 1024; --HQ) {
    }
  if (HQ < 3 || HQ > 8) return hipErrorInvalidValue;
  const size_t lds = lds_planes + (HQ - 1) * lds_ring;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  dim3 grid((unsigned)((long)tiles * nzc * n_orb));
#define RT_STENCIL(C, H) \
  hipLaunchKernelGGL((k_stencil<T, V, C, H, 3>), grid, dim3(nt), lds, s, psi, hpsi, v, nx, \
                     ny, nz, TY, ZC, HQ, cf)
  if (cols == 1) {
    if (hs <= 1) RT_STENCIL(1, 1);
    else if (hs <= 2) RT_STENCIL(1, 2);
    else if (hs <= 4) RT_STENCIL(1, 4);
    else RT_STENCIL(1, 8);
  } else {
    // (two strips and more than two halo strips a thread would not fit the registers)
    if (hs <= 1) RT_STENCIL(2, 1);
    else RT_STENCIL(2, 2);
  }
#undef RT_STENCIL
  return hipGetLastError();
}

template <typename T>
hipError_t stencil(hipStream_t s, const T* psi, T* hpsi, const T* v, int n_orb, int nx, int ny,
                   int nz, double h, const double* a, int ty, int nzc, int hq) {
  if (nx > 256 || ny > 256 || nz > 256) return hipErrorInvalidValue;
  StencilCoef cf;
  for (int k = 0; k < 5; ++k) cf.c[k] = -0.5 * a[k] / (h * h);
  constexpr int VV = 16 / sizeof(T);
  if (nx % VV == 0) return stencil_launch<T, VV>(s, psi, hpsi, v, n_orb, nx, ny, nz, cf, ty, nzc, hq);
  return stencil_launch<T, 1>(s, psi, hpsi, v, n_orb, nx, ny, nz, cf, ty, nzc, hq);
}

template <typename T>
void stencil_tiles(int nx, int ny, int nz, int n_orb, std::vector<int>& ty, std::vector<int>& nzc) {
  constexpr int VV = 16 / sizeof(T);
  const int spr = nx % VV == 0 ? nx / VV : nx;
  ty.clear();
  nzc.clear();
  int cols, nt, hs;
  for (int t = 1; t <= ny && t * spr <= 1024; ++t)  // up to two strips per thread
    if (ny % t == 0 && stencil_shape(spr, t, cols, nt, hs)) ty.push_back(t);
  for (int z = 1; z <= 16 && z <= nz; z *= 2) nzc.push_back(z);
  (void)n_orb;
}
void stencil_halo_ahead(std::vector<int>& hq) { hq = {3, 4, 5, 6, 8}; }
template void stencil_tiles<double>(int, int, int, int, std::vector<int>&, std::vector<int>&);
template void stencil_tiles<float>(int, int, int, int, std::vector<int>&, std::vector<int>&);
template hipError_t stencil<double>(hipStream_t, const double*, double*, const double*, int, int, int,
                                    int, double, const double*, int, int, int);
template hipError_t stencil<float>(hipStream_t, const float*, float*, const float*, int, int, int, int,
                                   double, const double*, int, int, int);

// ============================================================================
// Separable nonlocal projectors
// ============================================================================
// gather: one block per (atom, group of 4 orbitals).
template <typename T>
__global__ __launch_bounds__(256) void k_nl_gather(const T* __restrict__ psi, long ng, int n_orb,
                                                   int rank, const int* __restrict__ atom_off,
                                                   const int* __restrict__ sph_idx,
                                                   const double* __restrict__ beta, double h3,
                                                   double* __restrict__ c, int n_proj) {
  __shared__ double sh[256];
  const int a = blockIdx.x;
  const int s0 = atom_off[a], s1 = atom_off[a + 1];
  for (int jj = 0; jj < 4; ++jj) {
    const int j = blockIdx.y * 4 + jj;
    if (j >= n_orb) break;
    const T* f = psi + (long)j * ng;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int sp = s0 + threadIdx.x; sp < s1; sp += 256) {
      double val = (double)f[sph_idx[sp]];
      for (int p = 0; p < rank; ++p) acc[p] += beta[(long)sp * rank + p] * val;
    }
    for (int p = 0; p < rank; ++p) {
      double t = block_sum_256(acc[p], sh);
      if (threadIdx.x == 0) c[(long)j * n_proj + a * rank + p] = h3 * t;
    }
  }
}

template <typename T>
hipError_t nl_gather(hipStream_t s, const T* psi, long ng, int n_orb, int n_atoms, int rank,
                     const int* atom_off, const int* sph_idx, const double* beta, double h3,
                     double* c) {
  dim3 grid(n_atoms, cdiv(n_orb, 4));
  hipLaunchKernelGGL((k_nl_gather<T>), grid, dim3(256), 0, s, psi, ng, n_orb, rank, atom_off, sph_idx,
                     beta, h3, c, n_atoms * rank);
  return hipGetLastError();
}
template hipError_t nl_gather<double>(hipStream_t, const double*, long, int, int, int, const int*,
                                      const int*, const double*, double, double*);
template hipError_t nl_gather<float>(hipStream_t, const float*, long, int, int, int, const int*,
                                     const int*, const double*, double, double*);

template <typename T>
__global__ void k_nl_scatter(T* __restrict__ hpsi, long ng, int n_union, const int* __restrict__ u_idx,
                             const int* __restrict__ u_ptr, const int* __restrict__ ent_pt,
                             const int* __restrict__ ent_atom, int rank, const double* __restrict__ beta,
                             const double* __restrict__ D, const double* __restrict__ c, int n_proj) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n_union) return;
  const long j = blockIdx.y;
  const double* cj = c + j * n_proj;
  double acc = 0.0;
  for (int e = u_ptr[u]; e < u_ptr[u + 1]; ++e) {
    const int a = ent_atom[e];
    const long sp = ent_pt[e];
    for (int p = 0; p < rank; ++p) acc += beta[sp * rank + p] * (D[a * rank + p] * cj[a * rank + p]);
  }
  T* o = hpsi + j * ng + u_idx[u];
  *o = (T)((double)*o + acc);
}

template <typename T>
hipError_t nl_scatter(hipStream_t s, T* hpsi, long ng, int n_orb, int n_union, const int* u_idx,
                      const int* u_ptr, const int* ent_pt, const int* ent_atom, int rank,
                      const double* beta, const double* D, const double* c, int n_proj) {
  dim3 grid(cdiv(n_union, 256), n_orb);
  hipLaunchKernelGGL((k_nl_scatter<T>), grid, dim3(256), 0, s, hpsi, ng, n_union, u_idx, u_ptr, ent_pt,
                     ent_atom, rank, beta, D, c, n_proj);
  return hipGetLastError();
}
template hipError_t nl_scatter<double>(hipStream_t, double*, long, int, int, const int*, const int*,
                                       const int*, const int*, int, const double*, const double*,
                                       const double*, int);
template hipError_t nl_scatter<float>(hipStream_t, float*, long, int, int, const int*, const int*,
                                      const int*, const int*, int, const double*, const double*,
                                      const double*, int);

// ============================================================================
// FP64 GEMM, C = A . B^T with both operands K-contiguous (tall-skinny
// projections over the grid and the N x N series products).  K is split across
// blockIdx.y into fixed ranges whose partial tiles are summed afterwards in a
// fixed order.
// ============================================================================
// Trajectory batching: T independent problems share one launch.  The
// trajectory index is the fastest-varying part of blockIdx.x, so blocks of
// different trajectories working on the same tile run together and share the
// orbital reads through L2.
struct SeriesSkip {
  const unsigned long long* slots;  // [T][stride]: max |dP_k| per term (bits of a non-negative double)
  const double* kmin;               // [T]
  const int* done;                  // [T][2]
  double thrs;
  int k;       // term this launch computes (1-based); 0 = not a series launch
  int stride;  // slots per trajectory
};

__device__ __forceinline__ bool series_stopped(const SeriesSkip& sk, int t) {
  if (sk.k <= 1) return false;
  if (sk.done[2 * t]) return true;
  double prev = __longlong_as_double((long long)sk.slots[(long)t * sk.stride + sk.k - 1]);
  return prev <= sk.thrs && (double)(sk.k - 1) >= sk.kmin[t];
}

// FP64 register-blocked GEMM on the vector units (MI355X: FP64 vector and
// matrix peaks are equal).  Tile BM x BN = 128 x 128 (big) or 64 x 64, K chunk
// 16, 256 threads each owning a TM x TN = BM/16 x BN/16 block of outputs.
// Operands are staged k-major in LDS (As[k][m], Bs[k][n]) so each thread reads
// contiguous runs of its rows/columns.
// FP64 matrix instructions: v_mfma_f64_16x16x4f64, lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16] (one double each), result register r is D[l / 16 + 4 r][l % 16]
// (lane layout probed on the device).  Block = 2 x 2 waves, each owning a
// (BM/2) x (BN/2) sub-tile of (BM/32) x (BN/32) 16 x 16 blocks; K in chunks of 16
// staged row-major in LDS (pitch 17: the fragment reads hit distinct banks) from
// coalesced loads (consecutive threads walk k along a row), the next chunk held in
// registers during the MFMAs.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int BM, int BN>
__global__ __launch_bounds__(256) void k_gemm_nt_f64(int M, int N, long K, const double* __restrict__ A,
                                                     long lda, const double* __restrict__ B, long ldb,
                                                     const double* __restrict__ w,
                                                     double* __restrict__ part, long kps, int upper,
                                                     int n_tn, Batch bt, SeriesSkip sk) {
  constexpr int BK = 16, PK = BK + 1, UA = BM * BK / 256, UB = BN * BK / 256;
  constexpr int WM = BM / 2, WN = BN / 2, FI = WM / 16, FJ = WN / 16;
  // XCD-aware order: consecutive logical blocks (the tiles of one K split, which
  // share their rows of A and B) run on one XCD and read those rows through its L2
  const long lid = xcd_logical(blockIdx.x + (long)gridDim.x * blockIdx.y, (long)gridDim.x * gridDim.y);
  const int bx = (int)(lid % gridDim.x), by = (int)(lid / gridDim.x);
  const int tb = bx % bt.T;
  if (bt.active && !bt.active[tb]) return;
  if (sk.k > 0 && series_stopped(sk, tb)) return;
  A += tb * bt.sa;
  B += tb * bt.sb;
  if (w) w += tb * bt.sw;
  part += tb * bt.sp;
  __shared__ double As[BM][PK];
  __shared__ double Bs[BN][PK];
  int tm, tn;
  {
    int t = bx / bt.T;
    if (upper) {
      tm = 0;
      int rowlen = n_tn;
      while (t >= rowlen) { t -= rowlen; ++tm; --rowlen; }
      tn = tm + t;
    } else {
      tm = t / n_tn;
      tn = t - tm * n_tn;
    }
  }
  const long k0 = (long)by * kps;
  const long k1 = min(K, k0 + kps);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int lc = tid & 15, lr = tid >> 4;  // loader: column k, row (of 16 per pass)
  const long am0 = (long)tm * BM, bn0 = (long)tn * BN;
  double ra[UA], rb[UB];
  auto fetch = [&](long kb) {
    const long gk = kb + lc;
    const bool kok = gk < k1;
    const double wk = (w && kok) ? w[gk] : 1.0;
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      const long gm = am0 + lr + 16 * u;
      ra[u] = (kok && gm < M) ? A[gm * lda + gk] * wk : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const long gn = bn0 + lr + 16 * u;
      rb[u] = (kok && gn < N) ? B[gn * ldb + gk] : 0.0;
    }
  };
  f64x4 acc[FI][FJ];
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FJ; ++j) acc[i][j] = (f64x4){0.0, 0.0, 0.0, 0.0};
  fetch(k0);
  for (long kb = k0; kb < k1; kb += BK) {
#pragma unroll
    for (int u = 0; u < UA; ++u) As[lr + 16 * u][lc] = ra[u];
#pragma unroll
    for (int u = 0; u < UB; ++u) Bs[lr + 16 * u][lc] = rb[u];
    __syncthreads();
    if (kb + BK < k1) fetch(kb + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double fa[FI], fb[FJ];
#pragma unroll
      for (int i = 0; i < FI; ++i) fa[i] = As[wm * WM + 16 * i + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < FJ; ++j) fb[j] = Bs[wn * WN + 16 * j + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < FJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  double* P = part + (long)by * M * N;
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long row = am0 + wm * WM + 16 * i + (lane >> 4) + 4 * r;
        const long col = bn0 + wn * WN + 16 * j + (lane & 15);
        if (row < M && col < N) P[row * N + col] = acc[i][j][r];
      }
}

static hipError_t gemm_launch(hipStream_t s, int M, int N, long K, const double* A, long lda,
                              const double* B, long ldb, const double* w, double* part, long kps,
                              int n_split, int upper, int big, Batch bt, SeriesSkip sk) {
  // 64 x 64 tiles for every shape: 4 waves per SIMD hide the load latency that the
  // 128 x 128 tile (one wave per SIMD, 275 registers) leaves exposed.
  (void)big;
  int ntm = cdiv(M, 64), ntn = cdiv(N, 64);
  int nt = upper ? ntm * (ntm + 1) / 2 : ntm * ntn;
  hipLaunchKernelGGL((k_gemm_nt_f64<64, 64>), dim3(nt * bt.T, n_split), dim3(256), 0, s, M, N, K, A, lda, B, ldb,
                     w, part, kps, upper, ntn, bt, sk);
  return hipGetLastError();
}

hipError_t gemm_nt_f64(hipStream_t s, int M, int N, long K, const double* A, long lda,
                       const double* B, long ldb, const double* w, double* part, long kps,
                       int n_split, int upper, int big, Batch bt) {
  SeriesSkip sk{nullptr, nullptr, nullptr, 0.0, 0, 0};
  return gemm_launch(s, M, N, K, A, lda, B, ldb, w, part, kps, n_split, upper, big, bt, sk);
}

// K = N split into series_splits(N) ranges of 16-aligned length so that a series
// term, a latency-bound N x 2N x N product, spreads over several times more blocks.
int series_splits(int N) { return N <= 64 ? 1 : (N <= 128 ? 2 : (N <= 192 ? 3 : 4)); }
static long series_kps(int N) {
  const int S = series_splits(N);
  return ((N + S - 1) / S + 15) / 16 * 16;
}
hipError_t gemm_nt_f64_series(hipStream_t s, int N, int T, const double* Hbar, const double* dP, double* C,
                              int k, const unsigned long long* slots, int stride, const double* kmin,
                              double thrs, const int* done, const int* active) {
  SeriesSkip sk{slots, kmin, done, thrs, k, stride};
  const long NN = (long)N * N;
  const long kps = series_kps(N);
  const int S = (int)((N + kps - 1) / kps);
  Batch bt{T, active, NN, 2 * NN, 0, (long)series_splits(N) * 2 * NN};
  return gemm_launch(s, N, 2 * N, N, Hbar, N, dP, N, nullptr, C, kps, S, 0, 0, bt, sk);
}

// C_t[m][n] = base_t[m][n] + alpha * sum_s part_t[s][m][n]; with mirror the upper
// part is kept and copied to the lower one.  blockIdx.y = trajectory.
__global__ void k_reduce_parts(const double* __restrict__ part, int n_split, int M, int N, double alpha,
                               const double* base, double* C, int mirror,
                               long sp, long sbase, long sc, const int* active) {
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)M * N) return;
  int m = (int)(e / N), n = (int)(e - (long)m * N);
  if (mirror && m > n) return;
  part += t * sp;
  C += t * sc;
  if (base) base += t * sbase;
  double acc = 0.0;
  for (int sI = 0; sI < n_split; ++sI) acc += part[(long)sI * M * N + e];
  acc *= alpha;
  C[e] = base ? base[e] + acc : acc;
  if (mirror && m < n) {
    long f = (long)n * N + m;
    C[f] = base ? base[f] + acc : acc;
  }
}

hipError_t reduce_parts(hipStream_t s, const double* part, int n_split, int M, int N, double alpha,
                        double* C, int mirror, const double* base, int T, long sp, long sbase, long sc,
                        const int* active) {
  long n = (long)M * N;
  hipLaunchKernelGGL(k_reduce_parts, dim3(cdiv(n, 256), T), dim3(256), 0, s, part, n_split, M, N, alpha, base,
                     C, mirror, sp, sbase, sc, active);
  return hipGetLastError();
}

// ============================================================================
// Small x tall FP64 MFMA product over grid columns: Phi = W . Psi with either
// Phi stored (orthonormalisation) or rho[r] = sum_i Psi[i][r] Phi[i][r]
// reduced in the epilogue (density from a density matrix), Phi never stored.
// Batched over trajectories: W_t = W + t N^2, out_t = out + t * (N ng | ng).
// ============================================================================
template <int MODE>
__global__ __launch_bounds__(256) void k_smalltall_f64(int N, long ng, const double* __restrict__ W,
                                                       const double* __restrict__ psi,
                                                       double* __restrict__ out, int tri, int T,
                                                       const int* active) {
  // Tile: 64 rows of W x 128 grid points on FP64 matrix instructions (layout as in
  // k_gemm_nt_f64); 2 x 2 waves, wave (wm, wn) owns rows 32 wm.. and points 64 wn..
  // as 2 x 4 blocks of 16 x 16; K chunk 16 over orbitals j, loaded coalesced (W along
  // its rows, psi along the grid) and prefetched one chunk ahead.
  constexpr int BM = 64, BN = 128, BK = 16;
  __shared__ double Ws[BM][BK + 1];
  __shared__ double Ps[BK][BN + 2];
  __shared__ double red[2][BN];
  // XCD-aware order: the T blocks of one column range (trajectory fastest) run on one
  // XCD and read its Psi columns through one L2
  const long lid = xcd_logical(blockIdx.x, gridDim.x);
  const int tb = (int)(lid % T);
  if (active && !active[tb]) return;
  W += (long)tb * N * N;
  out += MODE == 0 ? (long)tb * N * ng : (long)tb * ng;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const long r0 = (lid / T) * BN;
  double rho_part[4] = {0.0, 0.0, 0.0, 0.0};
  const int nI = cdiv(N, BM);
  for (int I = 0; I < nI; ++I) {
    f64x4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = (f64x4){0.0, 0.0, 0.0, 0.0};
    int jlo = 0, jhi = N;
    if (tri == 1) jlo = I * BM;
    if (tri == 2) jhi = min(N, (I + 1) * BM);
    double rw[4], rp[8];
    auto fetch = [&](int jb) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {  // W rows (tid >> 4) + 16 u, column jb + (tid & 15)
        const int gi = I * BM + (tid >> 4) + 16 * u, gj = jb + (tid & 15);
        rw[u] = (gi < N && gj < jhi) ? W[(long)gi * N + gj] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {  // psi row jb + (tid >> 7) + 2 u, point r0 + (tid & 127)
        const int gj = jb + (tid >> 7) + 2 * u;
        const long gr = r0 + (tid & 127);
        rp[u] = (gj < jhi && gr < ng) ? psi[(long)gj * ng + gr] : 0.0;
      }
    };
    if (jlo < jhi) fetch(jlo);
    for (int jb = jlo; jb < jhi; jb += BK) {
#pragma unroll
      for (int u = 0; u < 4; ++u) Ws[(tid >> 4) + 16 * u][tid & 15] = rw[u];
#pragma unroll
      for (int u = 0; u < 8; ++u) Ps[(tid >> 7) + 2 * u][tid & 127] = rp[u];
      __syncthreads();
      if (jb + BK < jhi) fetch(jb + BK);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        double fa[2], fb[4];
#pragma unroll
        for (int i = 0; i < 2; ++i) fa[i] = Ws[wm * 32 + 16 * i + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < 4; ++j) fb[j] = Ps[kk + (lane >> 4)][wn * 64 + 16 * j + (lane & 15)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = I * BM + wm * 32 + 16 * i + (lane >> 4) + 4 * r;
          const long col = r0 + wn * 64 + 16 * j + (lane & 15);
          if (row < N && col < ng) {
            if (MODE == 0) out[(long)row * ng + col] = acc[i][j][r];
            else rho_part[j] += psi[(long)row * ng + col] * acc[i][j][r];
          }
        }
  }
  if (MODE == 1) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      rho_part[j] += __shfl_xor(rho_part[j], 16);
      rho_part[j] += __shfl_xor(rho_part[j], 32);
      if (lane < 16) red[wm][wn * 64 + 16 * j + lane] = rho_part[j];
    }
    __syncthreads();
    if (tid < BN && r0 + tid < ng) out[r0 + tid] = red[0][tid] + red[1][tid];
  }
}
hipError_t smalltall_f64(hipStream_t s, int N, long ng, const double* W, const double* psi,
                         double* out, int mode, int tri, int T, const int* active) {
  dim3 grid(cdiv(ng, 128) * T);
  if (mode == 0)
    hipLaunchKernelGGL((k_smalltall_f64<0>), grid, dim3(256), 0, s, N, ng, W, psi, out, tri, T, active);
  else
    hipLaunchKernelGGL((k_smalltall_f64<1>), grid, dim3(256), 0, s, N, ng, W, psi, out, tri, T, active);
  return hipGetLastError();
}

// ============================================================================
// Spectral Poisson: discrete Fourier transforms along each axis in LDS
// ============================================================================
__global__ void k_twiddles(double2* tw, int n) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double sv, cv;
  sincospi(2.0 * p / n, &sv, &cv);
  tw[p] = make_double2(cv, sv);
}
hipError_t twiddles(hipStream_t s, double2* tw, int n) {
  hipLaunchKernelGGL(k_twiddles, dim3(cdiv(n, 256)), dim3(256), 0, s, tw, n);
  return hipGetLastError();
}

__global__ void k_pack_real(double2* z, const double* r, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    z[i] = make_double2(r[i], 0.0);
}
__global__ void k_real_part(double* r, const double2* z, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    r[i] = z[i].x;
}
hipError_t pack_real(hipStream_t s, double2* z, const double* r, long n) {
  hipLaunchKernelGGL(k_pack_real, dim3(ew_blocks(n)), dim3(256), 0, s, z, r, n);
  return hipGetLastError();
}
hipError_t real_part(hipStream_t s, double* r, const double2* z, long n) {
  hipLaunchKernelGGL(k_real_part, dim3(ew_blocks(n)), dim3(256), 0, s, r, z, n);
  return hipGetLastError();
}

// Mixed-radix (4, 2, 3, 5) self-sorting Stockham FFT of lines held in LDS
// (ping-pong buffers).  Pass with radix R after passes whose radices multiply
// to Ns: butterfly j reads x[j + r n/R], r < R, multiplies by the twiddle
// w^(r (j mod Ns) n / (Ns R)), takes an R-point DFT and writes element
// (j div Ns) Ns R + (j mod Ns) + r Ns.  After the last pass the line is in
// natural order.  X[m] = sum_p x[p] exp(-+ 2 pi i m p / n).
struct FftPlan {
  int np;
  int r[12];
};

static FftPlan fft_plan(int n) {
  FftPlan pl{};
  int m = n;
  const int order[4] = {4, 2, 3, 5};
  for (int q = 0; q < 4; ++q) {
    int rr = order[q];
    while (m % rr == 0 && !(rr == 2 && m % 4 == 0)) {
      pl.r[pl.np++] = rr;
      m /= rr;
    }
  }
  if (m != 1) pl.np = -1;  // not 2,3,5-smooth
  return pl;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// out[k] = sum_q v[q] exp(sgn 2 pi i q k / R), R in {2, 3, 4, 5}; the radix is a
// compile-time constant so v stays in registers.
template <int R>
__device__ __forceinline__ void small_dft(double2 (&v)[R], double sgn) {
  if constexpr (R == 2) {
    double2 a = v[0], b = v[1];
    v[0] = make_double2(a.x + b.x, a.y + b.y);
    v[1] = make_double2(a.x - b.x, a.y - b.y);
  } else if constexpr (R == 4) {
    double2 a = v[0], b = v[1], c = v[2], d = v[3];
    double2 s0 = make_double2(a.x + c.x, a.y + c.y), d0 = make_double2(a.x - c.x, a.y - c.y);
    double2 s1 = make_double2(b.x + d.x, b.y + d.y), d1 = make_double2(b.x - d.x, b.y - d.y);
    // w = exp(sgn i pi/2) = sgn i;  w * d1 = (-sgn d1.y, sgn d1.x)
    double2 wd1 = make_double2(-sgn * d1.y, sgn * d1.x);
    v[0] = make_double2(s0.x + s1.x, s0.y + s1.y);
    v[1] = make_double2(d0.x + wd1.x, d0.y + wd1.y);
    v[2] = make_double2(s0.x - s1.x, s0.y - s1.y);
    v[3] = make_double2(d0.x - wd1.x, d0.y - wd1.y);
  } else {
    // R = 3 or 5: direct sum with cos/sin of 2 pi m / R correctly rounded
    constexpr double c3[3] = {1.0, -0.5, -0.5};
    constexpr double s3[3] = {0.0, 0.86602540378443864676, -0.86602540378443864676};
    constexpr double c5[5] = {1.0, 0.30901699437494742410, -0.80901699437494742410, -0.80901699437494742410,
                              0.30901699437494742410};
    constexpr double s5[5] = {0.0, 0.95105651629515357212, 0.58778525229247312917, -0.58778525229247312917,
                              -0.95105651629515357212};
    double2 o[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int m = (q * k) % R;
        const double wr = R == 3 ? c3[m] : c5[m], wi = sgn * (R == 3 ? s3[m] : s5[m]);
        re += v[q].x * wr - v[q].y * wi;
        im += v[q].x * wi + v[q].y * wr;
      }
      o[k] = make_double2(re, im);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = o[k];
  }
}

// LAYOUT 0: element (line c, position p) at p * L + c (lines interleaved, L = lines);
// LAYOUT 1: at c * n + p (lines contiguous).
template <int LAYOUT>
__device__ __forceinline__ int lidx(int c, int p, int n, int L) {
  return LAYOUT == 0 ? p * L + c : c * n + p;
}

// One radix-R Stockham pass over L lines in LDS (twiddle index k r n / (Ns R) < n).
template <int LAYOUT, int R>
__device__ __forceinline__ void fft_pass(const double2* src, double2* dst, const double2* tws, int n, int L, int Ns,
                                         double sgn) {
  const int nb = n / R;
  const int tstep = n / (Ns * R);
  for (int e = threadIdx.x; e < nb * L; e += blockDim.x) {
    // neighbouring threads take neighbouring LDS elements: along the line for
    // line-major data (LAYOUT 1), across lines for column-major data
    int j, c;
    if (LAYOUT == 1) {
      c = e / nb;
      j = e - c * nb;
    } else {
      j = e / L;
      c = e - j * L;
    }
    const int k = j % Ns;
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double2 x = src[lidx<LAYOUT>(c, j + r * nb, n, L)];
      if (r > 0) {
        double2 t = tws[k * r * tstep];
        t.y *= sgn;
        x = cmul(x, t);
      }
      v[r] = x;
    }
    small_dft<R>(v, sgn);
    const int base = (j - k) * R + k;  // (j / Ns) Ns R + k
#pragma unroll
    for (int r = 0; r < R; ++r) dst[lidx<LAYOUT>(c, base + r * Ns, n, L)] = v[r];
  }
}

template <int LAYOUT>
__device__ double2* fft_lds(double2* A, double2* B, const double2* tws, int n, int L, const FftPlan& pl,
                            double sgn) {
  int Ns = 1;
  double2* src = A;
  double2* dst = B;
  for (int ps = 0; ps < pl.np; ++ps) {
    const int R = pl.r[ps];
    switch (R) {
      case 2: fft_pass<LAYOUT, 2>(src, dst, tws, n, L, Ns, sgn); break;
      case 3: fft_pass<LAYOUT, 3>(src, dst, tws, n, L, Ns, sgn); break;
      case 4: fft_pass<LAYOUT, 4>(src, dst, tws, n, L, Ns, sgn); break;
      default: fft_pass<LAYOUT, 5>(src, dst, tws, n, L, Ns, sgn); break;
    }
    __syncthreads();
    double2* t = src;
    src = dst;
    dst = t;
    Ns *= R;
  }
  return src;
}

// Lines along y or z: element p of line (o, c) at o*os + p*st + c, c in [c0, c0 + TC);
// blockIdx.z = trajectory (field stride fs).  mode 0: one transform (sign by
// inverse); mode 1: forward transform, multiply by the Poisson kernel
// 4 pi / (|G|^2 Ng) (G = 0 dropped), inverse transform -- used on z lines,
// the last forward and first inverse axis, so the k-space field never leaves LDS.
// px: row pitch of the k-space layout, nx for full rows, nx / 2 + 1 for the
// half spectrum of real fields (kx = 0 .. nx / 2, all with mx = ix).
struct PoissonGeom {
  int nx, ny, nz;
  double h;
  int px;
};

__device__ __forceinline__ double poisson_factor(const PoissonGeom& g, long gidx) {
  int ix = (int)(gidx % g.px), iy = (int)((gidx / g.px) % g.ny), iz = (int)(gidx / ((long)g.px * g.ny));
  int mx = ix < (g.nx + 1) / 2 || g.px != g.nx ? ix : ix - g.nx;
  int my = iy < (g.ny + 1) / 2 ? iy : iy - g.ny;
  int mz = iz < (g.nz + 1) / 2 ? iz : iz - g.nz;
  double gx = 2.0 * M_PI * mx / (g.nx * g.h), gy = 2.0 * M_PI * my / (g.ny * g.h), gz = 2.0 * M_PI * mz / (g.nz * g.h);
  double g2 = (gz * gz + gy * gy) + gx * gx;
  return g2 > 0.0 ? 4.0 * M_PI / (g2 * ((double)g.nx * g.ny * g.nz)) : 0.0;
}

__global__ __launch_bounds__(256) void k_fft_strided(double2* __restrict__ z, int n, long st, long os, int C, int TC,
                                                     const double2* __restrict__ tw, int inverse, FftPlan pl,
                                                     long fs, int mode, PoissonGeom pg) {
  extern __shared__ unsigned char smem_raw[];
  double2* tws = reinterpret_cast<double2*>(smem_raw);
  double2* A = tws + n;
  double2* B = A + n * TC;
  const int c0 = blockIdx.x * TC;
  const long base = (long)blockIdx.y * os;
  z += (long)blockIdx.z * fs;
  for (int p = threadIdx.x; p < n; p += blockDim.x) tws[p] = tw[p];
  const int cw = min(TC, C - c0);
  for (int e = threadIdx.x; e < n * TC; e += blockDim.x) {
    int p = e / TC, c = e - p * TC;
    A[e] = c < cw ? z[base + p * st + c0 + c] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  double2* out;
  if (mode == 0) {
    out = fft_lds<0>(A, B, tws, n, TC, pl, inverse ? 1.0 : -1.0);
  } else {
    double2* k = fft_lds<0>(A, B, tws, n, TC, pl, -1.0);
    for (int e = threadIdx.x; e < n * TC; e += blockDim.x) {
      int p = e / TC, c = e - p * TC;
      double f = c < cw ? poisson_factor(pg, base + p * st + c0 + c) : 0.0;
      k[e] = make_double2(k[e].x * f, k[e].y * f);
    }
    __syncthreads();
    double2* other = (k == A) ? B : A;
    out = fft_lds<0>(k, other, tws, n, TC, pl, 1.0);
  }
  for (int e = threadIdx.x; e < n * TC; e += blockDim.x) {
    int p = e / TC, c = e - p * TC;
    if (c < cw) z[base + p * st + c0 + c] = out[e];
  }
}

// Lines along x (contiguous), lpb lines per block, blockIdx.y = trajectory.
// real_in: read the real field rin (stride rs) instead of z; real_out: write the
// real part to rout (stride rs) instead of z.
__global__ __launch_bounds__(256) void k_fft_x(double2* __restrict__ z, int n, long n_lines, int lpb,
                                               const double2* __restrict__ tw, int inverse, FftPlan pl, long fs,
                                               const double* __restrict__ rin, double* __restrict__ rout, long rs) {
  extern __shared__ unsigned char smem_raw[];
  double2* tws = reinterpret_cast<double2*>(smem_raw);
  double2* A = tws + n;
  double2* B = A + n * lpb;
  const long l0 = (long)blockIdx.x * lpb;
  const int t = blockIdx.y;
  z += (long)t * fs;
  for (int p = threadIdx.x; p < n; p += blockDim.x) tws[p] = tw[p];
  const int nl = (int)min((long)lpb, n_lines - l0);
  for (int e = threadIdx.x; e < lpb * n; e += blockDim.x) {
    double2 v = make_double2(0.0, 0.0);
    if (e < nl * n) v = rin ? make_double2(rin[t * rs + l0 * n + e], 0.0) : z[l0 * n + e];
    A[e] = v;
  }
  __syncthreads();
  double2* out = fft_lds<1>(A, B, tws, n, lpb, pl, inverse ? 1.0 : -1.0);
  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    if (rout) rout[t * rs + l0 * n + e] = out[e].x;
    else z[l0 * n + e] = out[e];
  }
}

// Real fields along x (n even, M = n / 2): one complex transform of length M per
// line on z_m = x_2m + i x_2m+1, then the half spectrum X_k, k = 0 .. M, from
// X_k = E_k + e^(-2 pi i k / n) O_k, E_k = (Z_k + conj Z_(M-k)) / 2,
// O_k = -i (Z_k - conj Z_(M-k)) / 2 (Z_M = Z_0), written with row pitch M + 1.
// inverse: the reverse, Z'_k = (X_k + conj X_(M-k)) + i e^(2 pi i k / n) (X_k - conj X_(M-k)),
// x_2m + i x_2m+1 = IDFT_M(Z')_m (unnormalised, as the full-row transform).  Each
// line is a transform of its own (nothing mixes fields or lines).
__global__ __launch_bounds__(256) void k_fft_x_half(double2* __restrict__ z, int n, long n_lines, int lpb,
                                                    const double2* __restrict__ tw, int inverse, FftPlan pl,
                                                    long fs, const double* __restrict__ rin,
                                                    double* __restrict__ rout, long rs) {
  extern __shared__ unsigned char smem_raw[];
  const int M = n / 2, H = M + 1;
  double2* tn = reinterpret_cast<double2*>(smem_raw);  // e^(2 pi i p / n), p < n
  double2* tm = tn + n;                                // e^(2 pi i p / M), p < M
  double2* A = tm + M;
  double2* B = A + M * lpb;
  const long l0 = (long)blockIdx.x * lpb;
  const int t = blockIdx.y;
  z += (long)t * fs;
  for (int p = threadIdx.x; p < n; p += blockDim.x) tn[p] = tw[p];
  for (int p = threadIdx.x; p < M; p += blockDim.x) tm[p] = tw[2 * p];
  const int nl = (int)min((long)lpb, n_lines - l0);
  __syncthreads();
  for (int e = threadIdx.x; e < lpb * M; e += blockDim.x) {
    const int c = e / M, m = e - c * M;
    double2 v = make_double2(0.0, 0.0);
    if (c < nl) {
      if (!inverse) {
        const double* x = rin + t * rs + (l0 + c) * n;
        v = make_double2(x[2 * m], x[2 * m + 1]);
      } else {
        const double2* X = z + (l0 + c) * H;
        const double2 a = X[m], b = X[M - m];  // X_k, X_(M-k)
        const double2 s = make_double2(a.x + b.x, a.y - b.y);   // X_k + conj X_(M-k)
        const double2 d = make_double2(a.x - b.x, a.y + b.y);   // X_k - conj X_(M-k)
        const double2 w = tn[m];
        const double2 wd = make_double2(d.x * w.x - d.y * w.y, d.x * w.y + d.y * w.x);
        v = make_double2(s.x - wd.y, s.y + wd.x);  // s + i wd
      }
    }
    A[e] = v;
  }
  __syncthreads();
  double2* out = fft_lds<1>(A, B, tm, M, lpb, pl, inverse ? 1.0 : -1.0);
  if (!inverse) {
    for (int e = threadIdx.x; e < nl * H; e += blockDim.x) {
      const int c = e / H, k = e - c * H;
      const double2 a = out[c * M + (k == M ? 0 : k)];
      const double2 b = out[c * M + (k == 0 ? 0 : M - k)];
      // E = (a + conj b) / 2, O = -i (a - conj b) / 2
      const double2 E = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
      const double2 O = make_double2(0.5 * (a.y + b.y), -0.5 * (a.x - b.x));
      const double2 w = tn[k];  // conj is the forward twiddle
      const double2 wo = make_double2(O.x * w.x + O.y * w.y, O.y * w.x - O.x * w.y);
      z[(l0 + c) * H + k] = make_double2(E.x + wo.x, E.y + wo.y);
    }
  } else {
    for (int e = threadIdx.x; e < nl * M; e += blockDim.x) {
      const int c = e / M, m = e - c * M;
      const double2 v = out[e];
      double* x = rout + t * rs + (l0 + c) * n;
      x[2 * m] = v.x;
      x[2 * m + 1] = v.y;
    }
  }
}

// nr real fields (stride ng) to / from their half spectra in z (field stride ng).
static hipError_t fft_x_half_launch(hipStream_t s, double2* z, int nx, int ny, int nz, const double2* tw,
                                    int inverse, int T, const double* rin, double* rout) {
  const int n = nx, M = nx / 2;
  FftPlan pl = fft_plan(M);
  if (nx % 2 || pl.np < 0) return hipErrorInvalidValue;
  long n_lines = (long)ny * nz;
  int lpb = std::max(1, std::min(16, 1536 / M));
  lpb = std::max(1, std::min(lpb, (4096 - n - M) / (2 * M)));  // at most 64 KB of LDS
  size_t lds = (size_t)(n + M + 2 * lpb * M) * sizeof(double2);
  long ng = (long)nx * ny * nz;
  hipLaunchKernelGGL(k_fft_x_half, dim3(cdiv(n_lines, lpb), T), dim3(256), lds, s, z, n, n_lines, lpb, tw, inverse,
                     pl, ng, rin, rout, ng);
  return hipGetLastError();
}

static hipError_t fft_x_launch(hipStream_t s, double2* z, int nx, int ny, int nz, const double2* tw, int inverse,
                               int T, const double* rin, double* rout) {
  const int n = nx;
  FftPlan pl = fft_plan(n);
  if (pl.np < 0) return hipErrorInvalidValue;
  long n_lines = (long)ny * nz;
  // about 1536 elements per block (as the strided passes), at most 16 lines
  int lpb = std::max(1, std::min(16, 1536 / n));
  size_t lds = (size_t)(n + 2 * lpb * n) * sizeof(double2);
  long ng = (long)nx * ny * nz;
  hipLaunchKernelGGL(k_fft_x, dim3(cdiv(n_lines, lpb), T), dim3(256), lds, s, z, n, n_lines, lpb, tw, inverse, pl, ng,
                     rin, rout, ng);
  return hipGetLastError();
}

// px: row pitch of z (nx, or nx / 2 + 1 for half spectra)
static hipError_t fft_strided_launch(hipStream_t s, double2* z, int nx, int ny, int nz, int axis, const double2* tw,
                                     int inverse, int T, int mode, double h, int px = 0) {
  if (px == 0) px = nx;
  const int n = axis == 1 ? ny : nz;
  FftPlan pl = fft_plan(n);
  if (pl.np < 0) return hipErrorInvalidValue;
  int TC = n <= 96 ? 16 : (n <= 192 ? 8 : 4);
  long st = axis == 1 ? px : (long)px * ny;
  int C = axis == 1 ? px : px * ny;
  int n_outer = axis == 1 ? nz : 1;
  long os = axis == 1 ? (long)px * ny : 0;
  size_t lds = (size_t)(n + 2 * n * TC) * sizeof(double2);
  PoissonGeom pg{nx, ny, nz, h, px};
  long ng = (long)nx * ny * nz;
  hipLaunchKernelGGL(k_fft_strided, dim3(cdiv(C, TC), n_outer, T), dim3(256), lds, s, z, n, st, os, C, TC, tw, inverse,
                     pl, ng, mode, pg);
  return hipGetLastError();
}

hipError_t dft_axis(hipStream_t s, double2* z, int nx, int ny, int nz, int axis, const double2* tw,
                    int inverse) {
  if (axis == 0) return fft_x_launch(s, z, nx, ny, nz, tw, inverse, 1, nullptr, nullptr);
  return fft_strided_launch(s, z, nx, ny, nz, axis, tw, inverse, 1, 0, 0.0);
}

// V_H,t = IFFT[4 pi FFT[rho_t] / |G|^2] for T stacked densities: five launches
// (x fwd from the real field, y fwd, z fwd * kernel * z inv, y inv, x inv to the real field);
// for even nx the x passes are real-to-half-spectrum transforms.
hipError_t poisson_fft(hipStream_t s, const double* rho, double* vh, double2* z, int nx, int ny, int nz, double h,
                       const double2* twx, const double2* twy, const double2* twz, int T) {
  hipError_t e;
  if (nx % 2 == 0) {
    // real fields: half spectra along x, so the y and z passes see nx / 2 + 1 columns
    const int px = nx / 2 + 1;
    if ((e = fft_x_half_launch(s, z, nx, ny, nz, twx, 0, T, rho, nullptr)) != hipSuccess) return e;
    if ((e = fft_strided_launch(s, z, nx, ny, nz, 1, twy, 0, T, 0, h, px)) != hipSuccess) return e;
    if ((e = fft_strided_launch(s, z, nx, ny, nz, 2, twz, 0, T, 1, h, px)) != hipSuccess) return e;
    if ((e = fft_strided_launch(s, z, nx, ny, nz, 1, twy, 1, T, 0, h, px)) != hipSuccess) return e;
    return fft_x_half_launch(s, z, nx, ny, nz, twx, 1, T, nullptr, vh);
  }
  if ((e = fft_x_launch(s, z, nx, ny, nz, twx, 0, T, rho, nullptr)) != hipSuccess) return e;
  if ((e = fft_strided_launch(s, z, nx, ny, nz, 1, twy, 0, T, 0, h)) != hipSuccess) return e;
  if ((e = fft_strided_launch(s, z, nx, ny, nz, 2, twz, 0, T, 1, h)) != hipSuccess) return e;
  if ((e = fft_strided_launch(s, z, nx, ny, nz, 1, twy, 1, T, 0, h)) != hipSuccess) return e;
  return fft_x_launch(s, z, nx, ny, nz, twx, 1, T, nullptr, vh);
}

// V_H(G) = 4 pi rho(G) / |G|^2 / Ng (inverse-transform normalisation folded in), V_H(0) = 0.
__global__ void k_poisson_scale(double2* z, int nx, int ny, int nz, double h) {
  long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long ng = (long)nx * ny * nz;
  if (g >= ng) return;
  int ix = (int)(g % nx), iy = (int)((g / nx) % ny), iz = (int)(g / ((long)nx * ny));
  int mx = ix < (nx + 1) / 2 ? ix : ix - nx;
  int my = iy < (ny + 1) / 2 ? iy : iy - ny;
  int mz = iz < (nz + 1) / 2 ? iz : iz - nz;
  double gx = 2.0 * M_PI * mx / (nx * h), gy = 2.0 * M_PI * my / (ny * h), gz = 2.0 * M_PI * mz / (nz * h);
  double g2 = (gz * gz + gy * gy) + gx * gx;
  double f = g2 > 0.0 ? 4.0 * M_PI / (g2 * (double)ng) : 0.0;
  double2 v = z[g];
  z[g] = make_double2(v.x * f, v.y * f);
}
hipError_t poisson_scale(hipStream_t s, double2* z, int nx, int ny, int nz, double h) {
  long ng = (long)nx * ny * nz;
  hipLaunchKernelGGL(k_poisson_scale, dim3(cdiv(ng, 256)), dim3(256), 0, s, z, nx, ny, nz, h);
  return hipGetLastError();
}

// ============================================================================
// LDA exchange, local potential and energy partial sums
// ============================================================================
// Sawtooth values of one grid point, x fastest.
struct SawPoint {
  double x, y, z;
};
__device__ __forceinline__ SawPoint saw_point(unsigned g, const SawGeom& sg) {
  const unsigned ix = g % (unsigned)sg.nx;
  const unsigned r = g / (unsigned)sg.nx;
  const unsigned iy = r % (unsigned)sg.ny;
  const unsigned iz = r / (unsigned)sg.ny;
  return SawPoint{saw((int)ix, sg.nx, sg.jx, sg.h), saw((int)iy, sg.ny, sg.jy, sg.h), saw((int)iz, sg.nz, sg.jz, sg.h)};
}

// Dipole partial sums of each trajectory's density about the sawtooth:
// part3[t][blk][q] = sum over the block's points of rho s_q.
__global__ __launch_bounds__(256) void k_saw_dipole(const double* __restrict__ rho, SawGeom sg, long n,
                                                    double* part3, const int* active) {
  __shared__ double sh[256];
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  rho += t * n;
  part3 += (long)t * 3 * gridDim.x;
  double ax = 0.0, ay = 0.0, az = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double r = rho[i];
    const SawPoint p = saw_point((unsigned)i, sg);
    ax += r * p.x;
    ay += r * p.y;
    az += r * p.z;
  }
  ax = block_sum_256(ax, sh);
  ay = block_sum_256(ay, sh);
  az = block_sum_256(az, sh);
  if (threadIdx.x == 0) {
    part3[3 * blockIdx.x] = ax;
    part3[3 * blockIdx.x + 1] = ay;
    part3[3 * blockIdx.x + 2] = az;
  }
}
hipError_t saw_dipole(hipStream_t s, const double* rho, const SawGeom& sg, long n, double* part3, int T,
                      const int* active) {
  hipLaunchKernelGGL(k_saw_dipole, dim3(kRedBlocks, T), dim3(256), 0, s, rho, sg, n, part3, active);
  return hipGetLastError();
}

// vx, V_loc = V_ion + V_H (+ sum_q g_q s_q, the dipole correction, when DC) + v_x,
// and the per-block exchange and electrostatic energy sums (the latter weighs
// rho by V_H plus the correction, with the ions' energy term in block 0).
template <bool DC>
__global__ __launch_bounds__(256) void k_lda_vloc(const double* __restrict__ rho,
                                                  const double* __restrict__ vh,
                                                  const double* __restrict__ vion, double* __restrict__ vx,
                                                  double* __restrict__ vloc, long n, double* part2,
                                                  const int* active, SawGeom sg, const double* gfield) {
  __shared__ double sh[256];
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  rho += t * n;
  vh += t * n;
  vx += t * n;
  vloc += t * n;
  part2 += (long)t * 2 * gridDim.x;
  double gx = 0.0, gy = 0.0, gz = 0.0;
  if (DC) {
    gx = gfield[3 * t] - sg.gion[0];
    gy = gfield[3 * t + 1] - sg.gion[1];
    gz = gfield[3 * t + 2] - sg.gion[2];
  }
  const double cx = cbrt(3.0 / M_PI);
  double ex_sum = 0.0, eh_sum = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double r = rho[i];
    double rc = r > 0.0 ? r : 0.0;
    double c = cbrt(rc);
    double v = -cx * c;
    vx[i] = v;
    double h = vh[i];
    if (DC) {
      const SawPoint p = saw_point((unsigned)i, sg);
      h += (gx * p.x + gy * p.y) + gz * p.z;
    }
    vloc[i] = (vion[i] + h) + v;
    ex_sum += -0.75 * cx * rc * c;
    eh_sum += r * h;
  }
  double a = block_sum_256(ex_sum, sh);
  double b = block_sum_256(eh_sum, sh);
  if (threadIdx.x == 0) {
    // E_dc = 1/2 sum_q g_q (d_el,q - d_ion,q): the ions' part once per trajectory
    if (DC && blockIdx.x == 0) b -= (gx * sg.dion[0] + gy * sg.dion[1]) + gz * sg.dion[2];
    part2[2 * blockIdx.x] = a;
    part2[2 * blockIdx.x + 1] = b;
  }
}
hipError_t lda_vloc(hipStream_t s, const double* rho, const double* vh, const double* vion, double* vx,
                    double* vloc, long n, double* part2, int T, const int* active, const SawGeom* sg,
                    const double* gfield) {
  if (sg && gfield)
    hipLaunchKernelGGL(k_lda_vloc<true>, dim3(kRedBlocks, T), dim3(256), 0, s, rho, vh, vion, vx, vloc, n, part2,
                       active, *sg, gfield);
  else
    hipLaunchKernelGGL(k_lda_vloc<false>, dim3(kRedBlocks, T), dim3(256), 0, s, rho, vh, vion, vx, vloc, n, part2,
                       active, SawGeom{}, nullptr);
  return hipGetLastError();
}

// blockIdx.x = trajectory: part_t = part + t nblk ncol, out_t = out + t ncol
__global__ __launch_bounds__(256) void k_reduce_cols(const double* part, int nblk, int ncol,
                                                     const double* scale, double* out, const int* active) {
  __shared__ double sh[256];
  const int t = blockIdx.x;
  if (active && !active[t]) return;
  part += (long)t * nblk * ncol;
  out += (long)t * ncol;
  for (int c = 0; c < ncol; ++c) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) acc += part[(long)b * ncol + c];
    double t = block_sum_256(acc, sh);
    if (threadIdx.x == 0) out[c] = t * scale[c];
  }
}
hipError_t reduce_cols(hipStream_t s, const double* part, int nblk, int ncol, const double* scale,
                       double* out, int T, const int* active) {
  hipLaunchKernelGGL(k_reduce_cols, dim3(T), dim3(256), 0, s, part, nblk, ncol, scale, out, active);
  return hipGetLastError();
}

// ============================================================================
// N x N kernels
// ============================================================================
__global__ void k_lincomb(double* out, double a, const double* x, double b, const double* y, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = a * x[i] + b * y[i];
}
hipError_t lincomb(hipStream_t s, double* out, double a, const double* x, double b, const double* y,
                   long n) {
  hipLaunchKernelGGL(k_lincomb, dim3(ew_blocks(n)), dim3(256), 0, s, out, a, x, b, y, n);
  return hipGetLastError();
}

__global__ void k_lincomb3(double* out, double a, const double* x, double b, const double* y, double c,
                           const double* z, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = (a * x[i] + b * y[i]) + c * z[i];
}
hipError_t lincomb3(hipStream_t s, double* out, double a, const double* x, double b, const double* y, double c,
                    const double* z, long n) {
  hipLaunchKernelGGL(k_lincomb3, dim3(ew_blocks(n)), dim3(256), 0, s, out, a, x, b, y, c, z, n);
  return hipGetLastError();
}

// dst_t = src_t for active trajectories (blockIdx.y = t), n elements each.
__global__ void k_copy_masked(double* dst, const double* src, long n, const int* active) {
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[t * n + i] = src[t * n + i];
}
hipError_t copy_masked(hipStream_t s, double* dst, const double* src, long n, int T, const int* active) {
  int nb = ew_blocks(n) > 256 ? 256 : ew_blocks(n);
  hipLaunchKernelGGL(k_copy_masked, dim3(nb, T), dim3(256), 0, s, dst, src, n, active);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_max_abs_diff(const double* a, const double* b, long n,
                                                      unsigned long long* slot, const int* active) {
  __shared__ double sh[256];
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  a += t * n;
  b += t * n;
  double m = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    m = fmax(m, fabs(a[i] - b[i]));
  m = block_max_256(m, sh);
  if (threadIdx.x == 0) atomic_max_nonneg(slot + t, m);
}
hipError_t max_abs_diff(hipStream_t s, const double* a, const double* b, long n, unsigned long long* slot,
                        int T, const int* active) {
  int nb = ew_blocks(n) > 256 ? 256 : ew_blocks(n);
  hipLaunchKernelGGL(k_max_abs_diff, dim3(nb, T), dim3(256), 0, s, a, b, n, slot, active);
  return hipGetLastError();
}

// k_min = ceil(dt * (max_i (a_ii + r_i) - min_i (a_ii - r_i))), r_i = sum_{j != i} |a_ij|;
// one block per trajectory (A_t = A + t N^2).
// Gershgorin rows of A_t (or of (A_t + A2_t)/2 when A2 != nullptr, the value the
// series uses for Hbar): rows[t][i] = (a_ii + r_i, a_ii - r_i), r_i = sum_{j != i} |a_ij|.
// One wave per row (lanes stride the row, fixed shuffle tree), blockIdx.y = t.
// With Bm (Omega_2, real antisymmetric) the rows are those of i Omega / dt = Hbar + i Bm / dt:
// off-diagonal moduli sqrt(h_ij^2 + (b_ij / dt)^2).
__global__ __launch_bounds__(256) void k_gersh_rows(const double* __restrict__ A, const double* __restrict__ A2,
                                                    int N, double* __restrict__ rows, const int* active,
                                                    const double* __restrict__ Bm, double inv_dt) {
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= N) return;
  const long NN = (long)N * N;
  const double* a = A + t * NN + (long)i * N;
  const double* a2 = A2 ? A2 + t * NN + (long)i * N : nullptr;
  const double* b = Bm ? Bm + t * NN + (long)i * N : nullptr;
  double r = 0.0, dg = 0.0;
  for (int j = lane; j < N; j += 64) {
    const double v = a2 ? 0.5 * a[j] + 0.5 * a2[j] : a[j];
    if (j == i) dg = v;
    else if (b) r += sqrt(v * v + (b[j] * inv_dt) * (b[j] * inv_dt));
    else r += fabs(v);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    r += __shfl_xor(r, o);
    dg += __shfl_xor(dg, o);
  }
  if (lane == 0) {
    rows[(t * (long)N + i) * 2] = dg + r;
    rows[(t * (long)N + i) * 2 + 1] = dg - r;
  }
}

// kmin_t = ceil(|dt| (max_i rows[t][i][0] - min_i rows[t][i][1])), one block per t.
__global__ __launch_bounds__(256) void k_gersh_final(const double* __restrict__ rows, int N, double dt, double* kmin,
                                                     const int* active) {
  __shared__ double sh[256];
  const int t = blockIdx.x;
  if (active && !active[t]) return;
  double hi = -1e300, lo = 1e300;
  for (int i = threadIdx.x; i < N; i += 256) {
    hi = fmax(hi, rows[(t * (long)N + i) * 2]);
    lo = fmin(lo, rows[(t * (long)N + i) * 2 + 1]);
  }
  hi = block_max_256(hi, sh);
  lo = -block_max_256(-lo, sh);
  if (threadIdx.x == 0) kmin[t] = ceil(fabs(dt) * (hi - lo));
}

static hipError_t gersh_launch(hipStream_t s, const double* A, const double* A2, int N, double dt, double* kmin,
                               double* rows, int T, const int* active, const double* Bm = nullptr) {
  hipLaunchKernelGGL(k_gersh_rows, dim3(cdiv(N, 4), T), dim3(256), 0, s, A, A2, N, rows, active, Bm, 1.0 / dt);
  hipLaunchKernelGGL(k_gersh_final, dim3(T), dim3(256), 0, s, rows, N, dt, kmin, active);
  return hipGetLastError();
}

hipError_t gershgorin(hipStream_t s, const double* A, int N, double dt, double* kmin_out, double* rows, int T,
                      const int* active) {
  return gersh_launch(s, A, nullptr, N, dt, kmin_out, rows, T, active);
}

// Start of a series for T trajectories (blockIdx.y = t): Pout = dP = Pin (stacked,
// 2 N^2 each); when H0 != nullptr also Hbar = (H0 + H1)/2; block 0 of each
// trajectory zeroes its term slots, stop flags and residual slot.  kmin =
// ceil(|dt| (max_i (h_ii + r_i) - min_i (h_ii - r_i))) of Hbar (Gershgorin) follows
// from the row kernels, reading (H0 + H1)/2 directly when given.  With pulse
// parameters (fieldp[t] = a, omega, tau, phase, d_x, d_y, d_z), Hbar also takes the
// external field (V(t_a) + V(t_b))/2, V(t) = sum_q E_q(t) M_q (Algorithm 1).
__device__ __forceinline__ double pulse_env(const double* f, double t) {
  if (!(t >= 0.0 && t <= f[2])) return 0.0;
  const double s = sin(M_PI * t / f[2]);
  return f[0] * s * s * sin(f[1] * t + f[3]);
}

__global__ __launch_bounds__(256) void k_series_begin(const double* __restrict__ Pin, double* __restrict__ Pout,
                                                      double* __restrict__ dP, const double* __restrict__ H0,
                                                      const double* __restrict__ H1, double* Hbar, int N,
                                                      unsigned long long* slots, int stride, int* done,
                                                      unsigned long long* resid, const int* active,
                                                      const double* __restrict__ fieldp,
                                                      const double* __restrict__ M3, const double* tptr, double dt) {
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  const double t_a = tptr ? *tptr : 0.0, t_b = t_a + dt;
  const long NN = (long)N * N;
  Pin += t * 2 * NN;
  Pout += t * 2 * NN;
  dP += t * 2 * NN;
  Hbar += t * NN;
  if (H0) {
    H0 += t * NN;
    H1 += t * NN;
  }
  double cq[3] = {0.0, 0.0, 0.0};
  if (fieldp) {
    const double* f = fieldp + 7L * t;
    const double s = 0.5 * (pulse_env(f, t_a) + pulse_env(f, t_b));
    cq[0] = s * f[4];
    cq[1] = s * f[5];
    cq[2] = s * f[6];
  }
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < 2 * NN; e += (long)gridDim.x * blockDim.x) {
    double v = Pin[e];
    Pout[e] = v;
    dP[e] = v;
    if (H0 && e < NN) {
      double hb = 0.5 * H0[e] + 0.5 * H1[e];
      if (fieldp) hb += (cq[0] * M3[e] + cq[1] * M3[NN + e]) + cq[2] * M3[2 * NN + e];
      Hbar[e] = hb;
    }
  }
  if (blockIdx.x != 0) return;
  for (int q = threadIdx.x; q < stride; q += 256) slots[(long)t * stride + q] = 0ULL;
  if (threadIdx.x == 0) {
    done[2 * t] = 0;
    done[2 * t + 1] = 0;
    if (resid) resid[t] = 0ULL;
  }
}
hipError_t series_begin(hipStream_t s, const double* Pin, double* Pout, double* dP, const double* H0,
                        const double* H1, double* Hbar, int N, double dt, double* kmin, unsigned long long* slots,
                        int stride, int* done, unsigned long long* resid, double* rows, int T, const int* active,
                        const double* fieldp, const double* M3, const double* tptr, const double* Bm) {
  if (fieldp && !(H0 && M3)) return hipErrorInvalidValue;
  long n2 = 2L * N * N;
  int nb = ew_blocks(n2) > 256 ? 256 : ew_blocks(n2);
  hipLaunchKernelGGL(k_series_begin, dim3(nb, T), dim3(256), 0, s, Pin, Pout, dP, H0, H1, Hbar, N, slots, stride,
                     done, resid, active, fieldp, M3, tptr, dt);
  // Gershgorin floor of the Hbar the series uses (read back when the field is in it)
  const bool direct = H0 && !fieldp;
  return gersh_launch(s, direct ? H0 : Hbar, direct ? H1 : nullptr, N, dt, kmin, rows, T, active, Bm);
}

// Fourth-order Magnus term Omega_2 = (dt^2/12)[A0, A1] for the endpoint Hamiltonians
// A0 = H0 + V(t_a), A1 = H1 + V(t_a + dt) (V from the pulse parameters, or none):
// endpoints into A0/A1 (only with a field), X = A0 . A1^T = A0 A1 by the FP64 GEMM,
// B = (dt^2/12)(X - X^T).
__global__ void k_magnus2_ends(const double* __restrict__ H0, const double* __restrict__ H1,
                               const double* __restrict__ fieldp, const double* __restrict__ M3, const double* tptr,
                               double dt, double* __restrict__ A0, double* __restrict__ A1, int N,
                               const int* active) {
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  const double t_a = tptr ? *tptr : 0.0, t_b = t_a + dt;
  const long NN = (long)N * N;
  const double* f = fieldp + 7L * t;
  const double ea = pulse_env(f, t_a), eb = pulse_env(f, t_b);
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < NN; e += (long)gridDim.x * blockDim.x) {
    const double v = (f[4] * M3[e] + f[5] * M3[NN + e]) + f[6] * M3[2 * NN + e];
    A0[t * NN + e] = H0[t * NN + e] + ea * v;
    A1[t * NN + e] = H1[t * NN + e] + eb * v;
  }
}
__global__ void k_antisym_scale(const double* __restrict__ X, double* __restrict__ B, int N, double c,
                                const int* active) {
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  const long NN = (long)N * N;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < NN; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e - (long)i * N);
    B[t * NN + e] = c * (X[t * NN + e] - X[t * NN + (long)j * N + i]);
  }
}
hipError_t magnus2(hipStream_t s, const double* H0, const double* H1, const double* fieldp, const double* M3,
                   const double* tptr, double dt, double* A0, double* A1, double* X, double* B, int N, int T,
                   const int* active) {
  const long NN = (long)N * N;
  const int nb = ew_blocks(NN) > 256 ? 256 : ew_blocks(NN);
  const double* e0 = H0;
  const double* e1 = H1;
  if (fieldp) {
    hipLaunchKernelGGL(k_magnus2_ends, dim3(nb, T), dim3(256), 0, s, H0, H1, fieldp, M3, tptr, dt, A0, A1, N,
                       active);
    e0 = A0;
    e1 = A1;
  }
  Batch bt{T, active, NN, NN, 0, NN};
  SeriesSkip sk{nullptr, nullptr, nullptr, 0.0, 0, 0};
  hipError_t err = gemm_launch(s, N, N, N, e0, N, e1, N, nullptr, X, N, 1, 0, 0, bt, sk);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_antisym_scale, dim3(nb, T), dim3(256), 0, s, X, B, N, dt * dt / 12.0, active);
  return hipGetLastError();
}

// max_t |a_t - b_t| into slot[t] (zeroed beforehand), then b_t = a_t.
__global__ __launch_bounds__(256) void k_max_diff_assign(const double* a, double* b, long n, unsigned long long* slot,
                                                         const int* active) {
  __shared__ double sh[256];
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  a += t * n;
  b += t * n;
  double m = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double x = a[i];
    m = fmax(m, fabs(x - b[i]));
    b[i] = x;
  }
  m = block_max_256(m, sh);
  if (threadIdx.x == 0) atomic_max_nonneg(slot + t, m);
}
hipError_t max_diff_assign(hipStream_t s, const double* a, double* b, long n, unsigned long long* slot, int T,
                           const int* active) {
  int nb = ew_blocks(n) > 256 ? 256 : ew_blocks(n);
  hipLaunchKernelGGL(k_max_diff_assign, dim3(nb, T), dim3(256), 0, s, a, b, n, slot, active);
  return hipGetLastError();
}

// dP_k = (1/k)(-i dt)[Hbar, S + iA]:  S_k = (dt/k)[Hbar, A],  A_k = -(dt/k)[Hbar, S].
// C = Hbar . [S; A]^T, so C[:, :N] = Hbar S and C[:, N:] = -Hbar A (S symmetric, A antisymmetric).
// blockIdx.y = trajectory; C, dPn, P1 have stride 2 N^2.
// With Omega_2 = B (real antisymmetric), C2 = B . [S; A]^T adds (1/k)[B, S] =
// (1/k)(C2_S + C2_S^T) to S_k and (1/k)[B, A] = (1/k)(-C2_A + C2_A^T) to A_k.
// One block per 16 x 16 tile (i, j) of a trajectory, one element per thread: the
// transposed entries (j, i) the update needs come from the mirror tile, read row-wise
// into LDS, so every global read is coalesced.
__global__ __launch_bounds__(256) void k_series_update(const double* __restrict__ C, const double* __restrict__ C2,
                                                       double* __restrict__ dPn, double* __restrict__ P1, int N,
                                                       double dt, SeriesSkip sk, int* done, const int* active,
                                                       int ns, int nsp) {
  __shared__ double sT[4][16][17];  // mirror tile: C_S, C_A, C2_S, C2_A at (j, i)
  __shared__ double sh[256];
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  if (series_stopped(sk, t)) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && done[2 * t] == 0) {
      done[2 * t] = 1;
      done[2 * t + 1] = sk.k - 1;
    }
    return;
  }
  const double f = dt / sk.k, f2 = 1.0 / sk.k;
  const long NN = (long)N * N;
  const long N2 = 2L * N;
  C += t * (long)nsp * 2 * NN;
  if (C2) C2 += t * (long)nsp * 2 * NN;
  // C (and C2) hold ns K-split partial products [s][N][2N]; summed in split order
  auto cs = [&](const double* X, long idx) {
    double v = X[idx];
    for (int q = 1; q < ns; ++q) v += X[q * 2 * NN + idx];
    return v;
  };
  dPn += t * 2 * NN;
  P1 += t * 2 * NN;
  const int nt = (N + 15) / 16;
  const int i0 = (blockIdx.x / nt) * 16, j0 = (blockIdx.x % nt) * 16;
  {
    const int r = threadIdx.x >> 4, q = threadIdx.x & 15;  // mirror element (j0 + r, i0 + q)
    const int j = j0 + r, i = i0 + q;
    double a = 0.0, b = 0.0, a2 = 0.0, b2 = 0.0;
    if (j < N && i < N) {
      a = cs(C, (long)j * N2 + i);
      b = cs(C, (long)j * N2 + N + i);
      if (C2) {
        a2 = cs(C2, (long)j * N2 + i);
        b2 = cs(C2, (long)j * N2 + N + i);
      }
    }
    sT[0][r][q] = a;
    sT[1][r][q] = b;
    sT[2][r][q] = a2;
    sT[3][r][q] = b2;
  }
  __syncthreads();
  double m = 0.0;
  {
    const int r = threadIdx.x >> 4, q = threadIdx.x & 15;  // element (i0 + r, j0 + q)
    const int i = i0 + r, j = j0 + q;
    if (i < N && j < N) {
      const double gS_ij = cs(C, (long)i * N2 + j), gA_ij = cs(C, (long)i * N2 + N + j);
      const double gS_ji = sT[0][q][r], gA_ji = sT[1][q][r];
      double sv = -f * (gA_ij + gA_ji);
      double av = -f * (gS_ij - gS_ji);
      if (C2) {
        sv += f2 * (cs(C2, (long)i * N2 + j) + sT[2][q][r]);
        av += f2 * (sT[3][q][r] - cs(C2, (long)i * N2 + N + j));
      }
      const long o = (long)i * N + j;
      dPn[o] = sv;
      dPn[NN + o] = av;
      P1[o] += sv;
      P1[NN + o] += av;
      m = fmax(m, sqrt(sv * sv + av * av));
    }
  }
  m = block_max_256(m, sh);
  if (threadIdx.x == 0)
    atomic_max_nonneg(const_cast<unsigned long long*>(sk.slots) + (long)t * sk.stride + sk.k, m);
}
hipError_t series_update(hipStream_t s, const double* C, const double* C2, double* dPn, double* P1, int N,
                         double dt, int k, unsigned long long* slots, int stride, const double* kmin, double thrs,
                         int* done, int T, const int* active) {
  SeriesSkip sk{slots, kmin, done, thrs, k, stride};
  const int nb = ((N + 15) / 16) * ((N + 15) / 16);
  const long kps = series_kps(N);
  const int ns = (int)((N + kps - 1) / kps);
  hipLaunchKernelGGL(k_series_update, dim3(nb, T), dim3(256), 0, s, C, C2, dPn, P1, N, dt, sk, done, active, ns,
                     series_splits(N));
  return hipGetLastError();
}

// One series term for N <= 64 in a single launch, one block per trajectory: the
// product C = G . [S; A]^T (N x 2N) on v_mfma_f64_16x16x4f64 with G and dP staged in
// LDS (zero padded to 64), C kept in LDS, then the same update as k_series_update
// (dP_k from C and its transpose, P1 += dP_k, max |dP_k| to the slot).  Lane layout
// of the matrix instruction: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16],
// result register r is D[l / 16 + 4 r][l % 16].  Row pitches of 4 mod 32 doubles
// keep each fragment read at two LDS passes.
constexpr int SMALL_N = 64, SP = 68, CP = 132;
__global__ __launch_bounds__(256) void k_series_term_small(const double* __restrict__ G,
                                                           const double* __restrict__ dP, double* __restrict__ dPn,
                                                           double* __restrict__ P1, int N, double dt, SeriesSkip sk,
                                                           int* done, const int* active) {
  __shared__ double sG[SMALL_N * SP];
  __shared__ double sB[2 * SMALL_N * SP];  // rows 0..63: S, 64..127: A; later C [64][CP]
  __shared__ double sh[256];
  static_assert(SMALL_N * CP <= 2 * SMALL_N * SP, "C fits where the operands were");
  const int t = blockIdx.x;
  if (active && !active[t]) return;
  if (series_stopped(sk, t)) {
    if (threadIdx.x == 0 && done[2 * t] == 0) {
      done[2 * t] = 1;
      done[2 * t + 1] = sk.k - 1;
    }
    return;
  }
  const long NN = (long)N * N;
  G += t * NN;
  dP += t * 2 * NN;
  dPn += t * 2 * NN;
  P1 += t * 2 * NN;
  for (int e = threadIdx.x; e < SMALL_N * SMALL_N; e += 256) {
    const int r = e >> 6, c = e & 63;
    const bool in = r < N && c < N;
    sG[r * SP + c] = in ? G[r * N + c] : 0.0;
    sB[r * SP + c] = in ? dP[r * N + c] : 0.0;
    sB[(SMALL_N + r) * SP + c] = in ? dP[NN + r * N + c] : 0.0;
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
  f64x4 acc[8];
#pragma unroll
  for (int cb = 0; cb < 8; ++cb) acc[cb] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int kp = (N + 3) & ~3;
  for (int k0 = 0; k0 < kp; k0 += 4) {
    const double a = sG[(16 * w + lr) * SP + k0 + lk];
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) {
      const double b = sB[(16 * cb + lr) * SP + k0 + lk];
      acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[cb], 0, 0, 0);
    }
  }
  __syncthreads();
  double* Cs = sB;
#pragma unroll
  for (int cb = 0; cb < 8; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) Cs[(16 * w + lk + 4 * r) * CP + 16 * cb + lr] = acc[cb][r];
  __syncthreads();
  const double f = dt / sk.k;
  double m = 0.0;
  for (int e = threadIdx.x; e < N * N; e += 256) {
    const int i = e / N, j = e - i * N;
    const double gS_ij = Cs[i * CP + j], gA_ij = Cs[i * CP + SMALL_N + j];
    const double gS_ji = Cs[j * CP + i], gA_ji = Cs[j * CP + SMALL_N + i];
    const double sv = -f * (gA_ij + gA_ji);
    const double av = -f * (gS_ij - gS_ji);
    dPn[e] = sv;
    dPn[NN + e] = av;
    P1[e] += sv;
    P1[NN + e] += av;
    m = fmax(m, sqrt(sv * sv + av * av));
  }
  m = block_max_256(m, sh);
  if (threadIdx.x == 0)
    atomic_max_nonneg(const_cast<unsigned long long*>(sk.slots) + (long)t * sk.stride + sk.k, m);
}

int series_small_max() { return SMALL_N; }

hipError_t series_term_small(hipStream_t s, int N, int T, const double* G, const double* dP, double* dPn, double* P1,
                             double dt, int k, unsigned long long* slots, int stride, const double* kmin,
                             double thrs, int* done, const int* active) {
  if (N < 1 || N > SMALL_N || T < 1) return hipErrorInvalidValue;
  SeriesSkip sk{slots, kmin, done, thrs, k, stride};
  hipLaunchKernelGGL(k_series_term_small, dim3(T), dim3(256), 0, s, G, dP, dPn, P1, N, dt, sk, done, active);
  return hipGetLastError();
}

__global__ void k_series_finish(SeriesSkip sk, int* done, int T, const int* active) {
  int t = threadIdx.x;
  if (t >= T || (active && !active[t])) return;
  if (done[2 * t] == 0 && series_stopped(sk, t)) {
    done[2 * t] = 1;
    done[2 * t + 1] = sk.k - 1;
  }
}
hipError_t series_finish(hipStream_t s, int kmax, const unsigned long long* slots, int stride,
                         const double* kmin, double thrs, int* done, int T, const int* active) {
  SeriesSkip sk{slots, kmin, done, thrs, kmax + 1, stride};
  hipLaunchKernelGGL(k_series_finish, dim3(1), dim3(256), 0, s, sk, done, T, active);
  return hipGetLastError();
}

__global__ void k_set_flags(int* dst, Flags256 f, int T) {
  const int t = threadIdx.x;
  if (t < T) dst[t] = (int)((f.w[t >> 6] >> (t & 63)) & 1ull);
}
hipError_t set_flags(hipStream_t s, int* dst, Flags256 f, int T) {
  if (T < 0 || T > 256) return hipErrorInvalidValue;
  if (T == 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_flags, dim3(1), dim3(256), 0, s, dst, f, T);
  return hipGetLastError();
}

// One lane copies the words into a slot of the host-mapped mailbox and then stores the
// slot's sequence number with a system-scope release: a host thread that reads seq also
// reads the words.  The sequence number is a device-side counter (ctr) of the slot's
// owner, advanced by every publish, so the same launch can be replayed from a graph.
__global__ void k_publish(const unsigned* src, int n, unsigned* box, int off, unsigned long long* ctr) {
  if (threadIdx.x != 0) return;
  const unsigned long long seq = *ctr + 1;
  *ctr = seq;
  for (int i = 0; i < n; ++i) box[off + 2 + i] = src[i];
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(box + off), seq, __ATOMIC_RELEASE,
                     __HIP_MEMORY_SCOPE_SYSTEM);
}
hipError_t publish(hipStream_t s, const void* src, int n32, unsigned* box, int off, unsigned long long* ctr) {
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, static_cast<const unsigned*>(src), n32, box, off, ctr);
  return hipGetLastError();
}

// mu_q = sum_ij S_ij M_q,ij ; E = sum_ij S_ij Hcore_ij + E_x + E_H ; TrP = sum_i S_ii.
// S_t = S + t 2N^2, eparts_t = eparts + t estride, row_t = rows + t rstride.  Stage 1:
// kObsBlocks blocks per trajectory write partial sums part[t][b][5]; stage 2 adds
// them in block order (deterministic, independent of T).
constexpr int kObsBlocks = 32;
__global__ __launch_bounds__(256) void k_observables_part(const double* S, const double* M3, const double* hc,
                                                          const double* ovl, int N, double* part) {
  __shared__ double sh[256];
  const int t = blockIdx.y;
  const long NN = (long)N * N;
  S += t * 2 * NN;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = 0.0;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < NN; e += (long)kObsBlocks * 256) {
    double sv = S[e];
    a0 += sv * M3[e];
    a1 += sv * M3[NN + e];
    a2 += sv * M3[2 * NN + e];
    a3 += sv * hc[e];
  }
  if (ovl) {
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < NN; e += (long)kObsBlocks * 256) a4 += S[e] * ovl[e];
  } else {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < N; i += kObsBlocks * 256) a4 += S[(long)i * N + i];
  }
  a0 = block_sum_256(a0, sh);
  a1 = block_sum_256(a1, sh);
  a2 = block_sum_256(a2, sh);
  a3 = block_sum_256(a3, sh);
  a4 = block_sum_256(a4, sh);
  if (threadIdx.x == 0) {
    double* p = part + ((long)t * kObsBlocks + blockIdx.x) * 5;
    p[0] = a0;
    p[1] = a1;
    p[2] = a2;
    p[3] = a3;
    p[4] = a4;
  }
}
__global__ void k_observables_final(const double* part, const double* eparts, int estride, double* rows,
                                    long rstride) {
  const int t = blockIdx.x, q = threadIdx.x;
  if (q >= 5) return;
  double a = 0.0;
  for (int b = 0; b < kObsBlocks; ++b) a += part[((long)t * kObsBlocks + b) * 5 + q];
  if (q == 3) a += eparts[(long)t * estride] + eparts[(long)t * estride + 1];
  rows[t * rstride + q] = a;
}
hipError_t observables(hipStream_t s, const double* S, const double* M3, const double* hcore, const double* ovl,
                       int N, const double* eparts, int estride, double* rows, long rstride, double* work, int T) {
  hipLaunchKernelGGL(k_observables_part, dim3(kObsBlocks, T), dim3(256), 0, s, S, M3, hcore, ovl, N, work);
  hipLaunchKernelGGL(k_observables_final, dim3(T), dim3(64), 0, s, work, eparts, estride, rows, rstride);
  return hipGetLastError();
}

// out = A^T (N x N)
__global__ void k_transpose(const double* __restrict__ A, double* __restrict__ out, int N) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)N * N) return;
  const int i = (int)(e / N), j = (int)(e - (long)i * N);
  out[(long)j * N + i] = A[e];
}
hipError_t transpose(hipStream_t s, const double* A, double* out, int N) {
  const long n = (long)N * N;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, out, N);
  return hipGetLastError();
}

// In-place Cholesky A = L L^T (lower part; upper part zeroed), one block, left-looking.
__global__ __launch_bounds__(256) void k_cholesky(double* A, int N, int* info) {
  __shared__ double sh[256];
  __shared__ double djj;
  if (threadIdx.x == 0) *info = 0;
  for (int j = 0; j < N; ++j) {
    double acc = 0.0;
    for (int k = threadIdx.x; k < j; k += 256) acc += A[(long)j * N + k] * A[(long)j * N + k];
    acc = block_sum_256(acc, sh);
    if (threadIdx.x == 0) {
      double d = A[(long)j * N + j] - acc;
      if (!(d > 0.0)) {
        if (*info == 0) *info = j + 1;
        d = 1.0;
      }
      djj = sqrt(d);
      A[(long)j * N + j] = djj;
    }
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < N; i += 256) {
      double t = A[(long)i * N + j];
      for (int k = 0; k < j; ++k) t -= A[(long)i * N + k] * A[(long)j * N + k];
      A[(long)i * N + j] = t / djj;
    }
    __syncthreads();
  }
  for (long e = threadIdx.x; e < (long)N * N; e += 256) {
    int i = (int)(e / N), j = (int)(e - (long)i * N);
    if (j > i) A[e] = 0.0;
  }
}
hipError_t cholesky(hipStream_t s, double* A, int N, int* info) {
  hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(256), 0, s, A, N, info);
  return hipGetLastError();
}

// Linv = L^-1 for lower-triangular L: one column per thread by forward substitution.
__global__ void k_tri_inverse_lower(const double* L, double* X, int N) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  for (int i = 0; i < c; ++i) X[(long)i * N + c] = 0.0;
  for (int i = c; i < N; ++i) {
    double t = (i == c) ? 1.0 : 0.0;
    for (int k = c; k < i; ++k) t -= L[(long)i * N + k] * X[(long)k * N + c];
    X[(long)i * N + c] = t / L[(long)i * N + i];
  }
}
hipError_t tri_inverse_lower(hipStream_t s, const double* L, double* Linv, int N) {
  hipLaunchKernelGGL(k_tri_inverse_lower, dim3(cdiv(N, 64)), dim3(64), 0, s, L, Linv, N);
  return hipGetLastError();
}

// W_ij = S_ij * (2 if i < j, 1 if i == j, 0 if i > j): rho = sum_i psi_i sum_{j >= i} W_ij psi_j.
// blockIdx.y = trajectory; S_t = S + t sstride, W_t = W + t N^2.
__global__ void k_upper_weighted(const double* S, double* W, int N, long sstride, const int* active) {
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)N * N) return;
  S += t * sstride;
  W += t * (long)N * N;
  int i = (int)(e / N), j = (int)(e - (long)i * N);
  W[e] = i < j ? 2.0 * S[e] : (i == j ? S[e] : 0.0);
}
hipError_t upper_weighted(hipStream_t s, const double* S, double* W, int N, long sstride, int T,
                          const int* active) {
  long n = (long)N * N;
  hipLaunchKernelGGL(k_upper_weighted, dim3(cdiv(n, 256), T), dim3(256), 0, s, S, W, N, sstride, active);
  return hipGetLastError();
}

}  // namespace rtk
