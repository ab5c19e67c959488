// Launchers of the BF16x3 mixed-precision grid contractions (gfx950).
#pragma once
#include <hip/hip_runtime.h>

namespace rtk {

// hi = bf16(x), lo = bf16(x - hi)
hipError_t split_bf16(hipStream_t s, const double* x, unsigned short* hi, unsigned short* lo, long n);
// upper-weighted (S - S0) split to bf16 hi/lo (density weights of the change), padded to ld;
// frag = 1 stores 32x32x16 A-fragment order (ld % 32 == 0), frag = 0 row-major
hipError_t upper_weighted_delta_bf16(hipStream_t s, const double* S, const double* S0, unsigned short* hi,
                                     unsigned short* lo, int N, int ld, long sstride, int T, const int* active,
                                     int frag);
// point-major split: hiT/loT[r][j] (pitch ld, multiple of 32, zero for j >= N) of psi[j][r]
hipError_t split_bf16_t(hipStream_t s, const double* psi, unsigned short* hiT, unsigned short* loT, int N, int ld,
                        long ng);
// leading dimension of the density weights and point-major orbitals for N orbitals
int density_tile_ld(int N);
// part[s] (FP32, N x N, upper tiles) = sum_k A[m][k] w[k] A[n][k] over K split s of kps
// points; requires ng % 8 == 0, kps % 64 == 0 and 256 ng < 2^31
hipError_t proj_bf16x3(hipStream_t s, int N, long ng, const unsigned short* hi, const unsigned short* lo,
                       const float* w, float* part, long kps, int n_split, int T, const int* active);
// The same product for N <= proj_tri_max_n(): one block per (trajectory, split of
// kps points) computes the whole upper triangle; kps a positive multiple of
// proj_tri_chunk(), n_split = ceil(ng / kps); part layout as above.  hi/lo are
// K-blocked ([ceil(ng / TKC)][N][TKC], TKC = proj_tri_chunk(), zero past ng;
// proj_tri_elems(N, ng) elements each), written by split_bf16_kb.
int proj_tri_max_n();
int proj_tri_chunk();
long proj_tri_elems(int N, long ng);
hipError_t split_bf16_kb(hipStream_t s, const double* psi, unsigned short* hi, unsigned short* lo, int N, long ng);
hipError_t proj_tri_bf16x3(hipStream_t s, int N, long ng, const unsigned short* hi, const unsigned short* lo,
                           const float* w, float* part, long kps, int n_split, int T, const int* active);
// C = base + alpha * sum_s part[s] (upper kept, mirrored)
hipError_t reduce_parts_f32(hipStream_t s, const float* part, int n_split, int N, double alpha,
                            const double* base, double* C, int T, const int* active, long sbase);
// rho = rho0 + sum_i psi_i sum_{j>=i} W_ij psi_j.  W: [T][ld][ld], ld = density_tile_ld(N)
// (a multiple of 32, zero past N).  N <= 256: resident-tile kernel on the point-major
// orbitals pthi/ptlo [ng][ld]; larger N: tiled product on the orbital-major phi/plo
// [N][ng] with FP32 partial densities dpart [T][ceil(N / density_big_rows())][ng]
// (scratch; ng % 8 == 0).
int density_big_rows();
hipError_t density_bf16x3(hipStream_t s, int N, long ng, const unsigned short* whi, const unsigned short* wlo,
                          const unsigned short* phi, const unsigned short* plo, const unsigned short* pthi,
                          const unsigned short* ptlo, const double* rho0, double* rho, int T, const int* active,
                          float* dpart);
hipError_t delta_f32(hipStream_t s, float* d, const double* a, const double* b, long n, int T, const int* active);

}  // namespace rtk
