// kf_util.hip -- ahead-of-time kernels of the runtime: counter reset, a plain
// streaming copy used to calibrate memory counters, streaming read and copy
// references for the attainable bandwidth, and seeded input generation.
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

// Streaming read reference: n float4 with non-temporal loads, grid-stride, eight
// loads in flight per lane; workgroup g writes the sum of its share to sink[g].
__global__ void __launch_bounds__(256) kf_read_f4_kernel(const f4_t* __restrict__ src, size_t n,
                                                         float* __restrict__ sink) {
    __shared__ float part[4];
    constexpr int U = 8;
    float acc = 0.f;
    const size_t step = (size_t)gridDim.x * 256 * U;
    for (size_t base = (size_t)blockIdx.x * 256 * U + threadIdx.x; base < n; base += step) {
        f4_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t i = base + (size_t)u * 256;
            v[u] = i < n ? __builtin_nontemporal_load(src + i) : f4_t{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) sink[blockIdx.x] = ((part[0] + part[1]) + part[2]) + part[3];
}

// Streaming copy reference in the layout of the strip kernels: the buffer is
// rows of 4096 float4 (64 KiB); workgroup (strip s, block b) copies the 2 KiB
// column strip s of rows b * 2048 ... with two waves, four rows per wave step.
__global__ void __launch_bounds__(128) kf_copy_strip_kernel(f4_t* __restrict__ dst, const f4_t* __restrict__ src,
                                                            long rows) {
    constexpr int G = 4, W = 2, K = 2, COLS4 = 4096, RPW = 2048, STRIPS = COLS4 / (64 * K);
    const int s = (int)(blockIdx.x % STRIPS);
    const long rb = blockIdx.x / STRIPS;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long r0 = rb * RPW, r1 = r0 + RPW < rows ? r0 + RPW : rows;
    for (long r = r0 + wave * G; r < r1; r += W * G) {
        f4_t v[G][K];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const long i = (r + g) * COLS4 + s * 64 * K + k * 64 + lane;
                v[g][k] = r + g < r1 ? __builtin_nontemporal_load(src + i) : f4_t{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const long i = (r + g) * COLS4 + s * 64 * K + k * 64 + lane;
                if (r + g < r1) __builtin_nontemporal_store(v[g][k], dst + i);
            }
    }
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

hipError_t launch_stream(int kind, void* dst, const void* src, size_t bytes, hipStream_t st) {
    const size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    if (kind == 0) {
        hipLaunchKernelGGL(kf_read_f4_kernel, dim3(2048), dim3(256), 0, st, (const f4_t*)src, n, (float*)dst);
    } else {
        const long rows = (long)(bytes / 65536);
        const long grid = 32 * ((rows + 2047) / 2048);
        hipLaunchKernelGGL(kf_copy_strip_kernel, dim3((unsigned)grid), dim3(128), 0, st, (f4_t*)dst,
                           (const f4_t*)src, rows);
    }
    return hipGetLastError();
}

}  // namespace kf
