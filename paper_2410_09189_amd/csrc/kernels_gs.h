// Launchers of the ground-state kernels: the symmetric eigensolver of the
// Rayleigh-Ritz step, block residuals, occupied density and Pulay density mixing.
#pragma once
#include <hip/hip_runtime.h>

namespace rtk {

// ---- symmetric eigensolver (parallel cyclic Jacobi) ------------------------------
// A: [n][n] (row-major) -> work [ld][ld], ld = n rounded up to even; the symmetric
// part (A + A^T)/2 is copied and the padding row/column zeroed.  V = I.
hipError_t jacobi_setup(hipStream_t s, const double* A, int n, int ld, double* W, double* V);
// One round of the round-robin ordering: the ld/2 disjoint pairs (p, q) of round r
// are rotated at once, Aout = J^T A J (J the product of the pair rotations that
// zero A_pq), V <- V J.  A and Aout must differ.
hipError_t jacobi_round(hipStream_t s, const double* A, double* Aout, double* V, int ld, int round);
// Largest order of the single-block (LDS-resident) eigensolve and Cholesky.
int jacobi_small_max();
// All sweeps in one block for even ld <= jacobi_small_max(): A (set up by
// jacobi_setup) iterated in LDS and written back, V updated in place; at most
// max_sweeps; stat[0..2] = sweeps, off-diagonal norm^2, total norm^2.
hipError_t jacobi_small(hipStream_t s, double* A, double* V, int ld, int max_sweeps, double* stat);
// Linv = L^-1 with A = L L^T (lower) for n <= jacobi_small_max(), one block, L in
// LDS; info = first non-positive pivot column + 1 (0: success).
hipError_t chol_inv_small(hipStream_t s, const double* A, double* Linv, int n, int* info);
// out[0] = sum_{i != j} A_ij^2, out[1] = sum_i A_ii^2 (one block, fixed order)
hipError_t jacobi_offdiag(hipStream_t s, const double* A, int ld, double* out);
// evals[k] = k-th smallest diag(A) over the first n indices (ties by index);
// vecs row k = column of V that belongs to it (vecs [n][n]); rank: scratch [n]
hipError_t jacobi_sort(hipStream_t s, const double* A, const double* V, int n, int ld, double* evals,
                       double* vecs, int* rank);

// ---- block kernels of the subspace iteration ----------------------------------------
// res[i] = sqrt(h3 sum_r (HX[i][r] - ev[i] X[i][r])^2); part: scratch
// [n][row_residual_parts()] of per-block partial sums (fixed combination order)
int row_residual_parts();
hipError_t row_residuals(hipStream_t s, const double* HX, const double* X, const double* ev, int n, long ng,
                         double h3, double* res, double* part);
// rho[r] = sum_{i < n} occ[i] X[i][r]^2 (rows in order)
hipError_t occ_density(hipStream_t s, const double* X, const double* occ, int n, long ng, double* rho);
// slot = max_r |v[r]| (slot zeroed beforehand; bits of a non-negative double)
hipError_t abs_max(hipStream_t s, const double* v, long n, unsigned long long* slot);
// count += number of entries of v that are NaN or infinite (count zeroed beforehand)
hipError_t count_nonfinite(hipStream_t s, const double* v, long n, unsigned long long* count);
// each row scaled by the sign of its entry of largest modulus (first such entry)
hipError_t fix_signs(hipStream_t s, double* X, int n, long ng);

// ---- Pulay (DIIS) density mixing ------------------------------------------------------
// part[k][b]: block b's share of <res_k, res_snew> for the m stored residuals
// (res: [depth][ng]); 256 blocks per k
hipError_t pulay_dots(hipStream_t s, const double* res, int m, int snew, long ng, double* part);
// B[k][snew] = B[snew][k] = sum_b part[k][b]; then c minimises |sum_k c_k res_k| with
// sum_k c_k = 1 (bordered system of B over the m slots, partial pivoting); a
// singular system falls back to c = e_snew.  B: [depth][depth], coef: [depth]
hipError_t pulay_solve(hipStream_t s, const double* part, int m, int snew, int depth, double* B, double* coef);
// rho[r] = sum_k coef[k] (in[k][r] + beta res[k][r])
hipError_t pulay_mix(hipStream_t s, const double* in, const double* res, const double* coef, int m, double beta,
                     long ng, double* rho);

}  // namespace rtk
