// kf_quant.hip -- row-scaled reduced-precision storage of an FP32 matrix (the
// storage kf_matrix_q declares): BF16 with scale 1, or OCP FP8-E4M3 with one
// FP32 scale per row, scale_i = amax_i / 448 (448 is the largest finite E4M3
// value). Every code is the nearest value, ties to even, of the exact number
// it stands for (a_ij for BF16, the exact quotient a_ij / scale_i for FP8),
// with FP8 saturating at +-448.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace kf {
namespace {

constexpr int QT = 256;   // threads per workgroup; one row per workgroup

// BF16: round the binary32 value to 8 significant bits, ties to even (adding
// 0x7fff plus the kept lowest bit carries exactly when the dropped half is
// above one half, or equal to it with an odd kept part). NaN stays a quiet NaN.
__device__ __forceinline__ unsigned short bf16_code(float x) {
    const unsigned u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Magnitude of E4M3 code c (0 <= c <= 0x7e): c = e << 3 | m stands for
// m 2^-9 when e = 0 and (1 + m / 8) 2^(e - 7) otherwise.
__device__ __forceinline__ float e4m3_mag(unsigned c) {
    const unsigned e = c >> 3, m = c & 7u;
    return e == 0 ? (float)m * 0x1p-9f : __uint_as_float(((e + 120u) << 23) | (m << 20));
}

// E4M3 code of x / s (s > 0 finite). q = x / s in binary32 is within a few
// units in the last place of the exact quotient, far less than half the E4M3
// spacing, so its neighbours lo <= |q| < hi on the E4M3 grid bracket the exact
// quotient or the exact quotient lies within those few units of one of them
// (then that one is the nearest). The choice between lo and hi compares
// |x| with mid s, mid = (lo + hi) / 2 exact in binary32, by the sign of one
// fused multiply-add, so it is exact; both operands are first scaled by 2^64
// when s is small so that the difference cannot underflow to zero.
__device__ __forceinline__ unsigned char e4m3_code(float x, float s) {
    const unsigned sign = (__float_as_uint(x) >> 24) & 0x80u;
    if (x != x) return (unsigned char)(sign | 0x7fu);
    const float a = fabsf(x / s);
    if (!(a < 448.f)) return (unsigned char)(sign | 0x7eu);   // saturate (includes +inf)
    unsigned lo;
    if (a < 0x1p-6f) {
        lo = (unsigned)(a * 0x1p9f);                 // subnormal grid m 2^-9 (exact scaling)
    } else {
        const unsigned b = __float_as_uint(a);
        lo = ((((b >> 23) - 127u + 7u) << 3) | ((b >> 20) & 7u));
    }
    const float vlo = e4m3_mag(lo);
    if (vlo == a) return (unsigned char)(sign | lo);
    const float vhi = e4m3_mag(lo + 1u);
    const float mid = 0.5f * (vlo + vhi);
    const float k = s < 0x1p-60f ? 0x1p64f : 1.f;
    const float r = __builtin_fmaf(-mid, s * k, fabsf(x) * k);
    unsigned c;
    if (r > 0.f) c = lo + 1u;
    else if (r < 0.f) c = lo;
    else c = (lo & 1u) ? lo + 1u : lo;              // tie: the even code
    return (unsigned char)(sign | c);
}

template <int FP8>
__global__ void __launch_bounds__(QT) kf_quantize_rows_kernel(const float* __restrict__ A, long cols, long lda,
                                                               void* __restrict__ codes, long ldq,
                                                               float* __restrict__ scales) {
    __shared__ float red[QT / 64];
    const long i = blockIdx.x;
    const float* a = A + i * lda;
    const int tid = threadIdx.x;
    float s = 1.f;
    if (FP8) {
        float m = 0.f;
        for (long j = tid; j < cols; j += QT) m = fmaxf(m, fabsf(a[j]));   // NaN entries are skipped
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        if ((tid & 63) == 0) red[tid >> 6] = m;
        __syncthreads();
        m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        if (m > 0.f && m <= 3.4028235e38f) s = __fdiv_rn(m, 448.f);
    }
    if (tid == 0) scales[i] = s;
    if (FP8) {
        unsigned char* q = static_cast<unsigned char*>(codes) + i * ldq;
        for (long j = tid; j < ldq; j += QT) q[j] = j < cols ? e4m3_code(a[j], s) : (unsigned char)0;
    } else {
        unsigned short* q = static_cast<unsigned short*>(codes) + i * ldq;
        for (long j = tid; j < ldq; j += QT) q[j] = j < cols ? bf16_code(a[j]) : (unsigned short)0;
    }
}

}  // namespace

hipError_t launch_quantize_rows(const float* A, long rows, long cols, long lda, int fp8, void* codes, long ldq,
                                float* scales, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    if (fp8)
        hipLaunchKernelGGL(kf_quantize_rows_kernel<1>, dim3((unsigned)rows), dim3(QT), 0, st, A, cols, lda, codes, ldq,
                           scales);
    else
        hipLaunchKernelGGL(kf_quantize_rows_kernel<0>, dim3((unsigned)rows), dim3(QT), 0, st, A, cols, lda, codes, ldq,
                           scales);
    return hipGetLastError();
}

}  // namespace kf
