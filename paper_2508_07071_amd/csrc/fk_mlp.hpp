// fk_mlp.hpp -- launchers of the cost-model network kernels (fk_mlp.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace fk {

enum : int { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_RELU = 2, EPI_RELU_MASK = 3 };

// C[M x N] = op(A) op(B), then the epilogue: + bias[c] (and ReLU), or keep
// C only where mask[r][c] > 0 (ReLU backward).  op(X) = X^T when t* is set;
// all matrices row-major.
hipError_t mlp_gemm(bool ta, bool tb, const float *A, const float *B, float *C, int M, int N, int K,
                    const float *bias, const float *mask, int epilogue, hipStream_t s);
hipError_t mlp_colsum(const float *X, int rows, int cols, float *out, hipStream_t s);
hipError_t mlp_mse(const float *Y, const float *T, int64_t count, float *dY, float *loss,
                   hipStream_t s);
hipError_t mlp_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                    float b2, float eps, int step, hipStream_t s);
hipError_t mlp_gather(const float *src, int cols, const int32_t *idx, int rows, float *dst,
                      hipStream_t s);
// per-column mean and std (fp64 sums; std 1 for a constant column)
hipError_t mlp_colstats(const float *X, int rows, int cols, float *mean, float *stdv, hipStream_t s);
// (X - mean[c]) / std[c]
hipError_t mlp_standardize(const float *X, int64_t rows, int cols, const float *mean,
                           const float *stdv, float *out, hipStream_t s);
// out[0] = mean of x[0..n)
hipError_t mlp_mean(const float *x, int n, float *out, hipStream_t s);

}  // namespace fk
