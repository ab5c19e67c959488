// Internal launcher declarations for the RT-TDDFT kernels (gfx950).
// Every launcher enqueues on the given stream and returns the launch status.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>
#include <cstdint>

namespace rtk {

constexpr int kRedBlocks = 512;  // fixed block count of deterministic grid reductions

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2) in
// linear-id order.  The logical id is the position in a contiguous per-XCD range, so
// blocks with neighbouring logical ids run on one XCD and share its L2.
__device__ __forceinline__ long xcd_logical(long h, long nblk) {
  const long full = nblk / 8 * 8;
  return h < full ? (h % 8) * (full / 8) + h / 8 : h;
}

// T independent problems in one launch (trajectory index fastest in blockIdx.x);
// per-trajectory element strides of the operands A, B, the weight w and the output.
struct Batch {
  int T;
  const int* active;  // [T] device flags, nullable = all active
  long sa, sb, sw, sp;
};
inline Batch single() { return Batch{1, nullptr, 0, 0, 0, 0}; }

// ---- grid fields -----------------------------------------------------------
hipError_t vion(hipStream_t s, double* v, int nx, int ny, int nz, double h, int n_atoms,
                const double* pos, const double* depth, const double* width, int n_images);
// sawtooth coordinate along one axis, jump between planes j0 - 1 and j0, centred
hipError_t coord(hipStream_t s, double* q, int nx, int ny, int nz, double h, int axis, int j0);
hipError_t fill(hipStream_t s, double* p, long n, double v);
hipError_t fill_u64(hipStream_t s, unsigned long long* p, long n, unsigned long long v);
hipError_t copy_d(hipStream_t s, double* dst, const double* src, long n);
hipError_t cast_d2f(hipStream_t s, float* dst, const double* src, long n);
// dst_t = a_t - b (b shared by the T stacked fields)
hipError_t sub_d(hipStream_t s, double* dst, const double* a, const double* b, long n, int T, const int* active);

// ---- Hamiltonian on the grid -------------------------------------------------
// hpsi[j] = -1/2 L psi[j] + v psi[j] (8th-order FD, periodic), j < n_orb.  Tiling:
// ty rows of y per block (a divisor of ny whose strips fit one block), nzc z chunks
// and hq planes of halo look-ahead (2 .. 8); 0 = the default choice.  The tiling
// changes no arithmetic.
template <typename T>
hipError_t stencil(hipStream_t s, const T* psi, T* hpsi, const T* v, int n_orb, int nx, int ny,
                   int nz, double h, const double* coef5, int ty = 0, int nzc = 0, int hq = 0);
// halo look-ahead candidates of stencil<T>
void stencil_halo_ahead(std::vector<int>& hq);
// the tilings stencil<T> accepts on this grid (candidate ty values, nzc values)
template <typename T>
void stencil_tiles(int nx, int ny, int nz, int n_orb, std::vector<int>& ty, std::vector<int>& nzc);
// c[j][p] = h^3 sum_s beta[s][p] psi_j[idx[s]] over atom spheres (rank 4 or 1..4).
template <typename T>
hipError_t nl_gather(hipStream_t s, const T* psi, long ng, int n_orb, int n_atoms, int rank,
                     const int* atom_off, const int* sph_idx, const double* beta, double h3,
                     double* c);
// hpsi_j[u] += sum_{entries e of u} beta[ent[e]][p] D[a p] c[j][a p].
template <typename T>
hipError_t nl_scatter(hipStream_t s, T* hpsi, long ng, int n_orb, int n_union, const int* u_idx,
                      const int* u_ptr, const int* ent_pt, const int* ent_atom, int rank,
                      const double* beta, const double* D, const double* c, int n_proj);

// ---- dense products -----------------------------------------------------------
// part[s][m][n] = sum_{k in split s} A[m][k] w[k] B[n][k]   (w nullable), batched by bt;
// tiles with tn < tm skipped when upper != 0 (M == N).  kps: k per split.
hipError_t gemm_nt_f64(hipStream_t s, int M, int N, long K, const double* A, long lda,
                       const double* B, long ldb, const double* w, double* part, long kps,
                       int n_split, int upper, int big, Batch bt);
// C_t = base_t + alpha * sum_s part_t[s] (base nullable); mirror keeps the upper part.
hipError_t reduce_parts(hipStream_t s, const double* part, int n_split, int M, int N, double alpha,
                        double* C, int mirror, const double* base, int T, long sp, long sbase, long sc,
                        const int* active);
// out = W . Psi (mode 0) or rho[r] = sum_i Psi[i][r] (W Psi)[i][r] (mode 1);
// tri: 0 full, 1 W upper triangular, 2 W lower triangular; batched over T weight matrices.
hipError_t smalltall_f64(hipStream_t s, int N, long ng, const double* W, const double* psi,
                         double* out, int mode, int tri, int T, const int* active);

// ---- Poisson (spectral) ---------------------------------------------------------
hipError_t twiddles(hipStream_t s, double2* tw, int n);
hipError_t pack_real(hipStream_t s, double2* z, const double* r, long n);
hipError_t dft_axis(hipStream_t s, double2* z, int nx, int ny, int nz, int axis, const double2* tw,
                    int inverse);
hipError_t poisson_scale(hipStream_t s, double2* z, int nx, int ny, int nz, double h);
// V_H,t = IFFT[4 pi FFT[rho_t] / |G|^2] (G = 0 dropped) for T stacked fields; z: T x ng scratch
hipError_t poisson_fft(hipStream_t s, const double* rho, double* vh, double2* z, int nx, int ny, int nz, double h,
                       const double2* twx, const double2* twy, const double2* twz, int T);
hipError_t real_part(hipStream_t s, double* r, const double2* z, long n);

// ---- exchange, local potential, energies -------------------------------------------
// Grid shape, spacing and sawtooth jump planes (ng < 2^32 points); for the dipole
// correction also the ions' part: gion[q] = (4 pi / Omega) d_ion,q (subtracted from the
// electrons' field) and dion[q] = d_ion,q / h^3 (its energy term).
struct SawGeom {
  int nx = 0, ny = 0, nz = 0, jx = 0, jy = 0, jz = 0;
  double h = 0.0;
  double gion[3] = {0.0, 0.0, 0.0};
  double dion[3] = {0.0, 0.0, 0.0};
};
// part3: [T][kRedBlocks][3] partial sums of rho s_q (s_q the sawtooth coordinates)
hipError_t saw_dipole(hipStream_t s, const double* rho, const SawGeom& sg, long n, double* part3, int T,
                      const int* active);
// vx = -(3 rho/pi)^(1/3), vloc = vion + vh + vx; part[b] = (sum e_x, sum rho vh) per block.
// With sg and gfield ([T][3], the electrons' (4 pi / Omega) h^3 sum rho s_q) both non-null,
// g_q = gfield_q - sg.gion[q] and vh is taken as vh + sum_q g_q s_q (the vacuum dipole
// correction) in vloc and in the energy sum; block 0 adds -sum_q g_q dion[q] to the latter,
// so that 1/2 h^3 times it is E_H + (2 pi / Omega) sum_q d_q^2.
// batched over T stacked fields (blockIdx.y), part2: [T][kRedBlocks][2]
hipError_t lda_vloc(hipStream_t s, const double* rho, const double* vh, const double* vion,
                    double* vx, double* vloc, long n, double* part2, int T, const int* active,
                    const SawGeom* sg = nullptr, const double* gfield = nullptr);
// out[0..ncol) = scale[c] * sum_b part[b][c]   (single block, fixed order)
hipError_t reduce_cols(hipStream_t s, const double* part, int nblk, int ncol, const double* scale3,
                       double* out, int T, const int* active);

// ---- N x N kernels (batched over T trajectories with stacked buffers) ----------
hipError_t lincomb(hipStream_t s, double* out, double a, const double* x, double b, const double* y,
                   long n);
// out = (a x + b y) + c z
hipError_t lincomb3(hipStream_t s, double* out, double a, const double* x, double b, const double* y, double c,
                    const double* z, long n);
hipError_t copy_masked(hipStream_t s, double* dst, const double* src, long n, int T, const int* active);
hipError_t max_abs_diff(hipStream_t s, const double* a, const double* b, long n,
                        unsigned long long* slot, int T, const int* active);
// kmin_t = ceil(|dt| Gershgorin width of A_t); rows: scratch [T][N][2]
hipError_t gershgorin(hipStream_t s, const double* A, int N, double dt, double* kmin_out, double* rows, int T,
                      const int* active);
// series start: Pout = dP = Pin; Hbar = (H0 + H1)/2 when H0 != nullptr; slots, stop flags and
// resid (nullable) zeroed; kmin from the Gershgorin width of Hbar (rows: scratch [T][N][2]).
// fieldp (nullable, needs H0): per-trajectory pulse parameters [T][7]; Hbar then also gets
// (V(t_a) + V(t_a + dt))/2 with V = sum_q E_q M_q (M3: [3][N^2]), t_a = *tptr (device scalar;
// nullptr: 0).
// Bm (nullable): Omega_2, whose i Bm / dt joins Hbar in the Gershgorin floor.
hipError_t series_begin(hipStream_t s, const double* Pin, double* Pout, double* dP, const double* H0,
                        const double* H1, double* Hbar, int N, double dt, double* kmin, unsigned long long* slots,
                        int stride, int* done, unsigned long long* resid, double* rows, int T, const int* active,
                        const double* fieldp, const double* M3, const double* tptr, const double* Bm);
// Omega_2 = (dt^2/12)[H0 + V(t_a), H1 + V(t_a + dt)] into B ([T][N^2]); A0, A1, X: scratch [T][N^2];
// t_a = *tptr (device scalar; nullptr: 0)
hipError_t magnus2(hipStream_t s, const double* H0, const double* H1, const double* fieldp, const double* M3,
                   const double* tptr, double dt, double* A0, double* A1, double* X, double* B, int N, int T,
                   const int* active);
// slot[t] = max |a_t - b_t| (atomic max; zeroed beforehand), then b_t = a_t
hipError_t max_diff_assign(hipStream_t s, const double* a, double* b, long n, unsigned long long* slot, int T,
                           const int* active);
// K splits of a series product; C and C2 take series_splits(N) x 2 N^2 doubles per trajectory
int series_splits(int N);
// series term k (1-based) for T trajectories: C_t = Hbar_t . [S;A]_t^T (N x 2N), dP_k -> dPn_t,
// P1_t += dP_k, max |dP_k| -> slots[t][k]; skips trajectories whose series stopped.
hipError_t gemm_nt_f64_series(hipStream_t s, int N, int T, const double* Hbar, const double* dP, double* C,
                              int k, const unsigned long long* slots, int stride, const double* kmin,
                              double thrs, const int* done, const int* active);
// C2 (nullable): B . [S;A]^T for Omega_2 = B
hipError_t series_update(hipStream_t s, const double* C, const double* C2, double* dPn, double* P1, int N,
                         double dt, int k, unsigned long long* slots, int stride, const double* kmin, double thrs,
                         int* done, int T, const int* active);
// series term k for N <= series_small_max() in one launch (product and update fused,
// one block per trajectory); same arguments and results as the two launches above
// without Omega_2
int series_small_max();
hipError_t series_term_small(hipStream_t s, int N, int T, const double* G, const double* dP, double* dPn, double* P1,
                             double dt, int k, unsigned long long* slots, int stride, const double* kmin,
                             double thrs, int* done, const int* active);
hipError_t series_finish(hipStream_t s, int kmax, const unsigned long long* slots, int stride,
                         const double* kmin, double thrs, int* done, int T, const int* active);
// dst[t] = bit t of f (t < T <= 256), flags passed by value
struct Flags256 {
  unsigned long long w[4];
};
hipError_t set_flags(hipStream_t s, int* dst, Flags256 f, int T);
// Copies n32 32-bit words of device memory to box[off + 2 ..] (host-mapped, coherent) and
// then stores seq = ++(*ctr) (device counter) into box[off .. off + 1] with system-scope
// release, so a host that sees seq sees the words.
hipError_t publish(hipStream_t s, const void* src, int n32, unsigned* box, int off, unsigned long long* ctr);
// rows_t = (mu_x, mu_y, mu_z, E, N_e) from S'_t (stride 2N^2) and eparts_t; work: [T][160].
// N_e = Tr P, or Tr(P ovl) for a non-orthogonal basis with overlap ovl (nullable).
hipError_t observables(hipStream_t s, const double* S, const double* M3, const double* hcore, const double* ovl,
                       int N, const double* eparts, int estride, double* rows, long rstride, double* work, int T);
hipError_t transpose(hipStream_t s, const double* A, double* out, int N);
hipError_t cholesky(hipStream_t s, double* A, int N, int* info);
hipError_t tri_inverse_lower(hipStream_t s, const double* L, double* Linv, int N);
hipError_t upper_weighted(hipStream_t s, const double* S, double* W, int N, long sstride, int T,
                          const int* active);

}  // namespace rtk
