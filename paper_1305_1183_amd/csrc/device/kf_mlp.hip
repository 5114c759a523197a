// kf_mlp.hip -- training and inference kernels of the learned cost model: a
// d -> H -> H -> H -> 1 multilayer perceptron with ReLU, mean-squared error on
// log run time and Adam. The layer products are dense contractions and run on
// the matrix cores (v_mfma_f32_16x16x4f32, FP32 in and out, one 16 x 16 output
// tile per wave); the rest is element-wise. All reductions are in fixed order,
// so training is bit-reproducible.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "device/kf_blocks.h"

namespace kf {

typedef float f4v __attribute__((ext_vector_type(4)));

// C(i,j) = sum_k A(i,k) B(k,j) [+ bias(j)] [relu] [* (mask(i,j) > 0)], with
// element strides so that either operand can be read transposed:
// A(i,k) = A[i*sai + k*sak], B(k,j) = B[k*sbk + j*sbj], C(i,j) = C[i*ldc + j].
// Lane layout of the 16x16x4 FP32 MFMA on a 64-lane wave: lane l supplies
// A(l%16, l/16) and B(l/16, l%16) of the 16x4 / 4x16 slices and receives
// C(4*(l/16) + r, l%16) in accumulator register r.
__global__ void __launch_bounds__(64) mlp_gemm_kernel(int M, int N, int K, const float* __restrict__ A,
                                                      long sai, long sak, const float* __restrict__ B, long sbk,
                                                      long sbj, float* __restrict__ C, long ldc,
                                                      const float* __restrict__ bias, int relu,
                                                      const float* __restrict__ mask, long ldm) {
    const int lane = threadIdx.x;
    const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
    const int ia = i0 + (lane & 15), jb = j0 + (lane & 15), kk = lane >> 4;
    f4v acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 4) {
        const int k = k0 + kk;
        const float a = (ia < M && k < K) ? A[ia * sai + k * sak] : 0.f;
        const float b = (jb < N && k < K) ? B[k * sbk + jb * sbj] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
    const int j = j0 + (lane & 15);
    for (int r = 0; r < 4; ++r) {
        const int i = i0 + 4 * (lane >> 4) + r;
        if (i < M && j < N) {
            float v = acc[r];
            if (bias) v += bias[j];
            if (relu) v = v > 0.f ? v : 0.f;
            if (mask) v = mask[i * ldm + j] > 0.f ? v : 0.f;
            C[i * ldc + j] = v;
        }
    }
}

// db(j) = sum_i dY(i, j), rows in order.
__global__ void mlp_colsum_kernel(int M, int N, const float* __restrict__ dY, long ld, float* __restrict__ db) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.f;
    for (int i = 0; i < M; ++i) s += dY[i * ld + j];
    db[j] = s;
}

// loss = mean((p - y)^2); dp = 2 (p - y) / n. One workgroup of 256 threads.
__global__ void __launch_bounds__(256) mlp_mse_kernel(int n, const float* __restrict__ p, const float* __restrict__ y,
                                                      float* __restrict__ dp, float* __restrict__ loss) {
    __shared__ float part[256];
    const int t = threadIdx.x;
    float s = 0.f;
    for (int i = t; i < n; i += 256) {
        const float d = p[i] - y[i];
        s += d * d;
        dp[i] = 2.f * d / (float)n;
    }
    part[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) part[t] += part[t + w];
        __syncthreads();
    }
    if (t == 0 && loss) *loss = part[0] / (float)n;
}

// Adam (Kingma and Ba): m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
// p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ void mlp_adam_kernel(long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Per-column mean and standard deviation (population, floored at `floor`) of
// an n x d row-major matrix, for the standardisation of features and targets.
// One workgroup per column; thread t adds rows t, t + 256, ... with
// compensated sums, then the 256 pairs are merged by a fixed halving tree.
// Two passes: the mean, then the squared deviations from it.
__device__ __forceinline__ float mlp_block_total(kf_cs v, kf_cs* part) {
    const int t = threadIdx.x;
    part[t] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) part[t] = kf_cs_merge(part[t], part[t + w]);
        __syncthreads();
    }
    const float r = kf_cs_value(part[0]);
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(256) mlp_col_stats_kernel(long n, int d, const float* __restrict__ X,
                                                            float floor, float* __restrict__ mu,
                                                            float* __restrict__ sd) {
    __shared__ kf_cs part[256];
    const int j = blockIdx.x;
    kf_cs a = kf_cs_init(0.f);
    for (long i = threadIdx.x; i < n; i += 256) a = kf_cs_add(a, X[i * d + j]);
    const float mean = mlp_block_total(a, part) / (float)n;
    kf_cs q = kf_cs_init(0.f);
    for (long i = threadIdx.x; i < n; i += 256) {
        const float e = X[i * d + j] - mean;
        q = kf_cs_add(q, e * e);
    }
    const float var = mlp_block_total(q, part) / (float)n;
    if (threadIdx.x == 0) {
        mu[j] = mean;
        sd[j] = fmaxf(sqrtf(var), floor);
    }
}

// out(r, j) = (X(src, j) - mu(j)) / sd(j) for r < rows, with src = idx[r]
// (a minibatch in shuffled order) or row0 + r when idx is null.
__global__ void mlp_gather_std_kernel(int rows, int d, const float* __restrict__ X, const int* __restrict__ idx,
                                      long row0, const float* __restrict__ mu, const float* __restrict__ sd,
                                      float* __restrict__ out) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)rows * d) return;
    const int r = (int)(i / d), j = (int)(i % d);
    const long src = idx ? (long)idx[r] : row0 + r;
    out[i] = (X[src * d + j] - mu[j]) / sd[j];
}

// out(i) = p(i) sd + mu: a standardised prediction back to log microseconds.
__global__ void mlp_unstd_kernel(int n, const float* __restrict__ p, const float* __restrict__ mu,
                                 const float* __restrict__ sd, float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = __builtin_fmaf(p[i], *sd, *mu);
}

hipError_t mlp_col_stats(long n, int d, const float* X, float floor, float* mu, float* sd, hipStream_t st) {
    if (n <= 0 || d <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(mlp_col_stats_kernel, dim3(d), dim3(256), 0, st, n, d, X, floor, mu, sd);
    return hipGetLastError();
}

hipError_t mlp_gather_std(int rows, int d, const float* X, const int* idx, long row0, const float* mu,
                          const float* sd, float* out, hipStream_t st) {
    const long total = (long)rows * d;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_gather_std_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, rows, d, X,
                       idx, row0, mu, sd, out);
    return hipGetLastError();
}

hipError_t mlp_unstd(int n, const float* p, const float* mu, const float* sd, float* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_unstd_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, p, mu, sd, out);
    return hipGetLastError();
}

hipError_t mlp_gemm(int M, int N, int K, const float* A, long sai, long sak, const float* B, long sbk, long sbj,
                    float* C, long ldc, const float* bias, int relu, const float* mask, long ldm, hipStream_t st) {
    if (M <= 0 || N <= 0) return hipSuccess;
    dim3 grid((N + 15) / 16, (M + 15) / 16);
    hipLaunchKernelGGL(mlp_gemm_kernel, grid, dim3(64), 0, st, M, N, K, A, sai, sak, B, sbk, sbj, C, ldc, bias,
                       relu, mask, ldm);
    return hipGetLastError();
}

hipError_t mlp_colsum(int M, int N, const float* dY, long ld, float* db, hipStream_t st) {
    hipLaunchKernelGGL(mlp_colsum_kernel, dim3((N + 127) / 128), dim3(128), 0, st, M, N, dY, ld, db);
    return hipGetLastError();
}

hipError_t mlp_mse(int n, const float* p, const float* y, float* dp, float* loss, hipStream_t st) {
    hipLaunchKernelGGL(mlp_mse_kernel, dim3(1), dim3(256), 0, st, n, p, y, dp, loss);
    return hipGetLastError();
}

hipError_t mlp_adam(long n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, p, g, m, v, lr, b1,
                       b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace kf
