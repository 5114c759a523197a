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
