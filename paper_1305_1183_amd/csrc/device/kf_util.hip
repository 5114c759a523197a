// kf_util.hip -- ahead-of-time kernels of the runtime: counter reset and a
// plain streaming copy used to calibrate memory counters.
#include <hip/hip_runtime.h>

#include <cstddef>

namespace kf {

__global__ void kf_fill_u32_kernel(unsigned* __restrict__ p, size_t n, unsigned v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

typedef float f4_t __attribute__((ext_vector_type(4)));

// dst[i] = src[i] over n float4 elements, grid-stride.
__global__ void __launch_bounds__(256) kf_copy_f4_kernel(f4_t* __restrict__ dst,
                                                         const f4_t* __restrict__ src, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// Seeded uniform[-1, 1) input values: element (i, j) of a rows x cols block
// with row pitch ld is the SplitMix64 output number i * cols + j + 1 of the
// stream starting at `key` (Steele, Lea and Flood), mapped to
// (h >> 40) 2^-23 - 1, which is exact in float32; columns >= cols get `pad`.
__device__ __forceinline__ unsigned long long kf_splitmix(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256) kf_fill_uniform_kernel(float* __restrict__ dst, long rows, long cols, long ld,
                                                              unsigned long long key, float pad) {
    const long total = rows * ld;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const long i = e / ld, j = e - i * ld;
        float v = pad;
        if (j < cols) {
            const unsigned long long c = (unsigned long long)(i * cols + j) + 1ull;
            const unsigned long long h = kf_splitmix(key + c * 0x9E3779B97F4A7C15ull);
            v = (float)((long long)(h >> 40) - (1ll << 23)) * 0x1p-23f;
        }
        dst[e] = v;
    }
}

hipError_t launch_fill_uniform(float* dst, long rows, long cols, long ld, unsigned long long key, float pad,
                               hipStream_t st) {
    const long total = rows * ld;
    if (total <= 0) return hipSuccess;
    long grid = (total + 255) / 256;
    if (grid > 16384) grid = 16384;
    hipLaunchKernelGGL(kf_fill_uniform_kernel, dim3((unsigned)grid), dim3(256), 0, st, dst, rows, cols, ld, key, pad);
    return hipGetLastError();
}

hipError_t launch_fill_u32(void* p, size_t n, unsigned v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    int grid = (int)((n + 255) / 256);
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(kf_fill_u32_kernel, dim3(grid), dim3(256), 0, st, (unsigned*)p, n, v);
    return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
    size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    size_t grid = (n + 255) / 256;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(kf_copy_f4_kernel, dim3((unsigned)grid), dim3(256), 0, st, (f4_t*)dst,
                       (const f4_t*)src, n);
    return hipGetLastError();
}

}  // namespace kf
