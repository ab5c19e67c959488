// Launchers of the learned-predictor kernels (FP32 MLP, features, transfers).
#pragma once
#include <hip/hip_runtime.h>

namespace rtk {

struct MlpDims {
  int n_in, n_h, n_out;
};

long mlp_n_params(MlpDims d);                 // packed floats incl. standardisation
long mlp_n_train(MlpDims d);                  // trainable floats (W1 .. b3)
long mlp_work_floats(MlpDims d, int batch);   // scratch for forward / backward

hipError_t gemm_f32(hipStream_t s, int M, int N, int K, float alpha, const float* A, long sai, long sak,
                    const float* B, long sbk, long sbj, float beta, float* C, long ldc, const float* bias);
// Y = network(X) in physical units (standardised_out: raw network output)
hipError_t mlp_forward(hipStream_t s, MlpDims d, const float* params, const float* X, float* Y, int B,
                       float* work, bool standardized_out);
// loss_dev = mean (U - std(T))^2 / 2, grads of W1..b3 (layout of the trainable part)
hipError_t mlp_loss_grad(hipStream_t s, MlpDims d, const float* params, const float* X, const float* Tgt, int B,
                         float* grads, float* work, float* loss_dev);
hipError_t mlp_adam(hipStream_t s, float* p, const float* g, float* m, float* v, long n, int t, float lr);
hipError_t mlp_colstats(hipStream_t s, const float* X, int M, int N, float* mean, float* scale, float floor_std);

// coarse_t = block average over the 16^3 cells of (f_t - ref); grid edges divisible by 16
hipError_t restrict16(hipStream_t s, const double* f, const double* ref, float* coarse, int nx, int ny, int nz,
                      long fstride, long cstride, int T);
hipError_t restrict16_f64(hipStream_t s, const double* f, const double* ref, double* coarse, int nx, int ny, int nz,
                          long fstride, long cstride, int T);
hipError_t prolong16(hipStream_t s, const float* coarse, double* fine, int nx, int ny, int nz, long cstride,
                     long fstride, int T);
// 9 moments (dipole, second) of f_t - ref; part: scratch of T * 256 * 9 doubles
hipError_t moments9(hipStream_t s, const double* f, const double* ref, int nx, int ny, int nz, double h, long fstride,
                    double* part, float* out, long ostride, int T);
hipError_t assemble_features(hipStream_t s, const float* mom_ring, int mom_head, const float* cd_ring, int cur,
                             int prev, float* X, int n_in, long mom_stride, long cd_stride, int T);
hipError_t second_diff(hipStream_t s, const double* ring, int inew, int imid, int iold, float* Y, long rstride,
                       long ystride, int T);
hipError_t copy_rows_f(hipStream_t s, const float* src, float* dst, long n, long sstride, long dstride, int T);

}  // namespace rtk
