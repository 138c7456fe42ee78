// fk_mlp.hip -- kernels of the launch-configuration cost model: a small
// fully connected ReLU network trained and run on the GPU.
//
//   gemm      C[M x N] = op(A) * op(B)  (+ bias[n], ReLU) or (* [mask > 0])
//             64x64 output tile per 256-thread block, 4x4 outputs per
//             thread, K-panels of 16 staged through LDS.  Each output sums
//             its K terms in a fixed order, so results are deterministic.
//   colsum    db[n] = sum over rows of dY[:, n]   (fixed row order)
//   mse       loss and dY = 2 (Y - T) / (rows * cols)
//   adam      one Adam step over a flat parameter array
//   gather    rows of a matrix by an index list (mini-batch assembly)
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "fk_mlp.hpp"

namespace fk {

constexpr int kTile = 64;
constexpr int kPanel = 16;
constexpr int kThreads = 256;

// element (r, c) of a row-major matrix with `ld` columns, optionally read
// transposed
template <bool T>
__device__ __forceinline__ float at(const float *m, int ld, int r, int c)
{
    return T ? m[(int64_t)c * ld + r] : m[(int64_t)r * ld + c];
}

// op(A) is M x K: A row-major M x K (TA = false) or K x M (TA = true).
// op(B) is K x N: B row-major K x N (TB = false) or N x K (TB = true).
template <bool TA, bool TB>
__global__ __launch_bounds__(kThreads) void k_gemm(const float *__restrict__ A,
                                                   const float *__restrict__ B,
                                                   float *__restrict__ C, int M, int N, int K,
                                                   const float *__restrict__ bias,
                                                   const float *__restrict__ mask, int epilogue)
{
    __shared__ float As[kPanel][kTile + 1];
    __shared__ float Bs[kPanel][kTile + 1];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int row0 = blockIdx.y * kTile, col0 = blockIdx.x * kTile;
    const int lda = TA ? M : K;
    const int ldb = TB ? K : N;
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            acc[i][j] = 0.0f;
    for (int k0 = 0; k0 < K; k0 += kPanel) {
        // stage op(A)[row0.., k0..] and op(B)[k0.., col0..]: 1024 values each
        for (int e = threadIdx.x; e < kPanel * kTile; e += kThreads) {
            const int kk = e / kTile, mm = e % kTile;
            const int r = row0 + mm, k = k0 + kk;
            As[kk][mm] = (r < M && k < K) ? at<TA>(A, lda, r, k) : 0.0f;
            const int c = col0 + mm;
            Bs[kk][mm] = (c < N && k < K) ? at<TB>(B, ldb, k, c) : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kPanel; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = As[kk][ty + 16 * i];
                b[i] = Bs[kk][tx + 16 * i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = row0 + ty + 16 * i;
        if (r >= M)
            continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = col0 + tx + 16 * j;
            if (c >= N)
                continue;
            float v = acc[i][j];
            if (epilogue == EPI_BIAS || epilogue == EPI_BIAS_RELU)
                v += bias[c];
            if (epilogue == EPI_BIAS_RELU)
                v = v > 0.0f ? v : 0.0f;
            if (epilogue == EPI_RELU_MASK)
                v = mask[(int64_t)r * N + c] > 0.0f ? v : 0.0f;
            C[(int64_t)r * N + c] = v;
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_colsum(const float *__restrict__ X, int rows, int cols,
                                                     float *__restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols)
        return;
    float s = 0.0f;
    for (int r = 0; r < rows; ++r)
        s += X[(int64_t)r * cols + c];
    out[c] = s;
}

// One block: loss = mean((Y - T)^2) over rows x cols, dY = 2 (Y - T) / count.
__global__ __launch_bounds__(1024) void k_mse(const float *__restrict__ Y, const float *__restrict__ T,
                                              int64_t count, float *__restrict__ dY,
                                              float *__restrict__ loss)
{
    __shared__ float part[1024];
    float s = 0.0f;
    const float scale = 2.0f / (float)count;
    for (int64_t i = threadIdx.x; i < count; i += blockDim.x) {
        const float d = Y[i] - T[i];
        s = fmaf(d, d, s);
        dY[i] = scale * d;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w /= 2) {
        if ((int)threadIdx.x < w)
            part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        loss[0] = part[0] / (float)count;
}

__global__ __launch_bounds__(kThreads) void k_adam(float *__restrict__ p, const float *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ v,
                                                   int64_t n, float lr, float b1, float b2, float eps,
                                                   float c1, float c2)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1;  // bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t
    const float vh = vi / c2;
    p[i] = p[i] - lr * mh / (sqrtf(vh) + eps);
}

__global__ __launch_bounds__(kThreads) void k_gather(const float *__restrict__ src, int cols,
                                                     const int32_t *__restrict__ idx, int rows,
                                                     float *__restrict__ dst)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cols)
        return;
    const int r = (int)(e / cols), c = (int)(e % cols);
    dst[e] = src[(int64_t)idx[r] * cols + c];
}

// Per-column mean and standard deviation of a rows x cols matrix: sums of
// x and x^2 in fp64 over the rows in order; var = max(0, s2/n - mu^2); a
// column with var <= 1e-12 gets std 1.  One thread per column.
__global__ __launch_bounds__(kThreads) void k_colstats(const float *__restrict__ X, int rows,
                                                       int cols, float *__restrict__ mean,
                                                       float *__restrict__ stdv)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols)
        return;
    double s1 = 0.0, s2 = 0.0;
    for (int r = 0; r < rows; ++r) {
        const double v = X[(int64_t)r * cols + c];
        s1 += v;
        s2 += v * v;
    }
    const double mu = s1 / rows;
    double var = s2 / rows - mu * mu;
    var = var > 0.0 ? var : 0.0;
    mean[c] = (float)mu;
    stdv[c] = var > 1e-12 ? (float)sqrt(var) : 1.0f;
}

// out = (X - mean[c]) / std[c], one fp32 subtraction and one IEEE division.
__global__ __launch_bounds__(kThreads) void k_standardize(const float *__restrict__ X, int64_t rows,
                                                          int cols, const float *__restrict__ mean,
                                                          const float *__restrict__ stdv,
                                                          float *__restrict__ out)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= rows * cols)
        return;
    const int c = (int)(e % cols);
    out[e] = (X[e] - mean[c]) / stdv[c];
}

// out[0] = mean of x[0..n) (fp64 sum in order, one thread).
__global__ void k_mean(const float *__restrict__ x, int n, float *__restrict__ out)
{
    double acc = 0.0;
    for (int i = 0; i < n; ++i)
        acc += x[i];
    out[0] = (float)(acc / n);
}

// ------------------------------------------------------------- launchers --

hipError_t mlp_gemm(bool ta, bool tb, const float *A, const float *B, float *C, int M, int N, int K,
                    const float *bias, const float *mask, int epilogue, hipStream_t s)
{
    if (M <= 0 || N <= 0)
        return hipSuccess;
    dim3 grid((N + kTile - 1) / kTile, (M + kTile - 1) / kTile);
    if (!ta && !tb)
        k_gemm<false, false><<<grid, kThreads, 0, s>>>(A, B, C, M, N, K, bias, mask, epilogue);
    else if (!ta && tb)
        k_gemm<false, true><<<grid, kThreads, 0, s>>>(A, B, C, M, N, K, bias, mask, epilogue);
    else if (ta && !tb)
        k_gemm<true, false><<<grid, kThreads, 0, s>>>(A, B, C, M, N, K, bias, mask, epilogue);
    else
        k_gemm<true, true><<<grid, kThreads, 0, s>>>(A, B, C, M, N, K, bias, mask, epilogue);
    return hipGetLastError();
}

hipError_t mlp_colsum(const float *X, int rows, int cols, float *out, hipStream_t s)
{
    k_colsum<<<(cols + kThreads - 1) / kThreads, kThreads, 0, s>>>(X, rows, cols, out);
    return hipGetLastError();
}

hipError_t mlp_mse(const float *Y, const float *T, int64_t count, float *dY, float *loss,
                   hipStream_t s)
{
    k_mse<<<1, 1024, 0, s>>>(Y, T, count, dY, loss);
    return hipGetLastError();
}

hipError_t mlp_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                    float b2, float eps, int step, hipStream_t s)
{
    const float c1 = 1.0f - powf(b1, (float)step);
    const float c2 = 1.0f - powf(b2, (float)step);
    k_adam<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(p, g, m, v, n, lr, b1, b2,
                                                                         eps, c1, c2);
    return hipGetLastError();
}

hipError_t mlp_gather(const float *src, int cols, const int32_t *idx, int rows, float *dst,
                      hipStream_t s)
{
    const int64_t n = (int64_t)rows * cols;
    if (n == 0)
        return hipSuccess;
    k_gather<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(src, cols, idx, rows, dst);
    return hipGetLastError();
}

hipError_t mlp_colstats(const float *X, int rows, int cols, float *mean, float *stdv, hipStream_t s)
{
    k_colstats<<<(cols + kThreads - 1) / kThreads, kThreads, 0, s>>>(X, rows, cols, mean, stdv);
    return hipGetLastError();
}

hipError_t mlp_standardize(const float *X, int64_t rows, int cols, const float *mean,
                           const float *stdv, float *out, hipStream_t s)
{
    const int64_t n = rows * cols;
    if (n == 0)
        return hipSuccess;
    k_standardize<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(X, rows, cols, mean,
                                                                               stdv, out);
    return hipGetLastError();
}

hipError_t mlp_mean(const float *x, int n, float *out, hipStream_t s)
{
    k_mean<<<1, 1, 0, s>>>(x, n, out);
    return hipGetLastError();
}

}  // namespace fk
