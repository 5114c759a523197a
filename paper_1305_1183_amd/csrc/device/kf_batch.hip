// kf_batch.hip -- one persistent launch over many uneven-size BiCGK and GEMVER
// instances.
//
// The paper fuses the calls of one script into kernels and notes that the
// only way to keep data on chip across a global reduction would be persistent
// threads (Section 5, discussion of ATAX and SGEMVT). Here a fixed grid of
// workgroups repeatedly takes the next item from a queue in the workspace and
// processes it with the fused tiles of Algorithm 3 (BiCGK: A read once for
// A p and A^T r) and of the GEMVER plan {ger, ger, gemtv}{gemv}:
//
//   * a whole small instance is one item; for GEMVER the workgroup completes
//     x = beta B^T y + z itself and then runs w = alpha B x, so the global
//     barrier between the two kernels of the plan becomes a workgroup barrier;
//   * a larger instance is cut into row blocks; every block writes a column
//     partial, the last block to arrive (a per-instance counter) adds the
//     partials in block order and, for GEMVER, publishes x with a flag;
//   * the K2 row blocks of split GEMVER instances come after every phase-1
//     item in the queue. A K2 block waits for its flag, which can only be
//     held back by phase-1 items already taken by running workgroups, so the
//     wait always ends; it is bounded all the same and reports an error bit.
//
// Every counter is returned to zero by the item or workgroup that uses it
// last, so the launch can be replayed (e.g. from a graph) without clearing.
//
// Tile shape by size bucket. Up to n = 512: TPR = 2^LTPR lanes share a row (K
// float4 chunks each), 256 / TPR rows are in flight per workgroup step, G =
// 2^LG steps are loaded before their row sums are reduced. Above, BiCGK uses
// the wide tiles, in which the four waves split the columns of each row
// (below); GEMVER keeps whole rows per wave group there, which measured faster
// for its B stores.
#include <hip/hip_runtime.h>

#include "device/kf_blocks.h"
#include "kf_batch_defs.h"

namespace {

// Row sums of G = 2^LG partials per lane over groups of TPR = 2^LTPR lanes:
// a transposing exchange over the top LG bits of the group, then a butterfly
// over the rest. Lane cl of a group returns the sum of row cl >> (LTPR - LG).
template <int LTPR, int LG>
__device__ __forceinline__ float kfb_rows_reduce(float* v) {
    constexpr int TPR = 1 << LTPR;
    constexpr int G = 1 << LG;
    const int lane = __lane_id();
#pragma unroll
    for (int t = 0; t < LG; ++t) {
        const int half = G >> (t + 1);
        const int mask = (TPR >> 1) >> t;
        const bool hi = (lane & mask) != 0;
#pragma unroll
        for (int j = 0; j < half; ++j) {
            const float send = hi ? v[j] : v[j + half];
            const float keep = hi ? v[j + half] : v[j];
            v[j] = keep + kf_xor(send, mask);
        }
    }
    float s = v[0];
#pragma unroll
    for (int mask = (TPR >> 1) >> LG; mask >= 1; mask >>= 1) s += kf_xor(s, mask);
    return s;
}

__device__ __forceinline__ kf_f4 kfb_xor4(kf_f4 v, int m) {
    kf_f4 r;
    r.x = kf_xor(v.x, m); r.y = kf_xor(v.y, m); r.z = kf_xor(v.z, m); r.w = kf_xor(v.w, m);
    return r;
}

// Sum of the column partials of a split instance's row blocks 0 .. nblk - 1
// (p points at block 0's chunk, blocks ld floats apart), compensated, in
// block order.
__device__ __forceinline__ kf_f4 kfb_block_partials(const float* p, long ld, int nblk) {
    kf_cs4 t = kf_cs4_init(kf_zero4());
    for (int b = 0; b < nblk; ++b) t = kf_cs4_add(t, kf_ld4(p + (long)b * ld));
    return kf_cs4_value(t);
}

// Column sums of acc[k] over the 256 / TPR row-lanes of the workgroup, in a
// fixed order (butterfly inside the wave, then waves 0..3, compensated). emit(c, v) runs in
// threads tid < TPR with chunk c = tid + k TPR (columns 4c .. 4c + 3).
template <int LTPR, int K, typename Emit>
__device__ __forceinline__ void kfb_colsum(kf_f4* acc, kf_f4* red, Emit emit) {
    constexpr int TPR = 1 << LTPR;
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int m = TPR; m < 64; m <<= 1) acc[k] += kfb_xor4(acc[k], m);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        __syncthreads();
        if (lane < TPR) red[wave * TPR + lane] = acc[k];
        __syncthreads();
        if (threadIdx.x < TPR) {
            const int t = threadIdx.x;
            kf_cs4 s = kf_cs4_init(red[t]);
            s = kf_cs4_add(s, red[TPR + t]);
            s = kf_cs4_add(s, red[2 * TPR + t]);
            s = kf_cs4_add(s, red[3 * TPR + t]);
            emit(t + k * TPR, kf_cs4_value(s));
        }
    }
}

// Device-scope release and acquire, separately: a release writes back this
// XCD's L2 so that other XCDs can read what the workgroup stored; an acquire
// invalidates the local caches so that this workgroup reads what other XCDs
// released. A full fence does both, and its invalidation drops lines every
// other workgroup on the XCD is still using, so each side is used only where
// it is needed.
__device__ __forceinline__ void kfb_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void kfb_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Arrival at a per-instance counter. Returns true in every thread of the
// workgroup that arrives last; that workgroup then sees the stores every
// earlier arrival made before arriving, and the counter is back at zero.
__device__ __forceinline__ bool kfb_arrive(unsigned* counter, unsigned count, int* s_flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        kfb_release();
        const unsigned old = atomicAdd(counter, 1u);
        const int last = old == count - 1;
        if (last) {
            kfb_acquire();
            __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        *s_flag = last;
    }
    __syncthreads();
    return *s_flag != 0;
}

// Arrival that publishes nothing (only counts): no fences. The K2 blocks of a
// split GEMVER instance use it to find the last one, which clears the
// instance's flag for the next launch; every block has passed its wait on the
// flag before it arrives, and the next launch starts after this one ends.
__device__ __forceinline__ bool kfb_count(unsigned* counter, unsigned count, int* s_flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned old = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int last = old == count - 1;
        if (last) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *s_flag = last;
    }
    __syncthreads();
    return *s_flag != 0;
}

// Chunk k of a thread covers columns col .. col + 3, col = 4 (cl + k TPR).
// Per chunk the thread keeps the load column clamped into the row (cc) and
// the number of its columns below n (nv, 0 .. 4), both 32-bit.
struct kfb_cols {
    int cc, nv;
};
__device__ __forceinline__ kfb_cols kfb_col(int col, int n, int ld) {
    kfb_cols c;
    c.cc = col < ld - 4 ? col : ld - 4;
    const int v = n - col;
    c.nv = v < 0 ? 0 : (v > 4 ? 4 : v);
    return c;
}
// Row `row` of a matrix block at one chunk, without branches: the address is
// clamped into the block (row r1 - 1, the row's last chunk) and entries of
// rows >= r1 or columns >= n are replaced by zero with a select (padding may
// hold NaN). Clamped loads fall on lines that other lanes fetch anyway.
__device__ __forceinline__ kf_f4 kfb_ldm(const float* M, long ld, int row, int r1, kfb_cols c) {
    const long rc = row < r1 ? row : r1 - 1;
    kf_f4 v = kf_ld4_nt(M + rc * ld + c.cc);
    const int lim = row < r1 ? c.nv : 0;
    v.x = lim > 0 ? v.x : 0.f;
    v.y = lim > 1 ? v.y : 0.f;
    v.z = lim > 2 ? v.z : 0.f;
    v.w = lim > 3 ? v.w : 0.f;
    return v;
}
// Vector entries at one chunk (the vector holds exactly n floats; entries
// at index >= n read as zero). 32-bit index arithmetic throughout.
__device__ __forceinline__ kf_f4 kfb_ldv(const float* v, int col, int n) {
    if (col + 4 <= n) return kf_ld4(v + col);
    kf_f4 r = kf_zero4();
    if (col + 0 < n) r.x = v[col + 0];
    if (col + 1 < n) r.y = v[col + 1];
    if (col + 2 < n) r.z = v[col + 2];
    return r;
}
__device__ __forceinline__ void kfb_stv(float* v, int col, int n, kf_f4 x) {
    if (col + 4 <= n) { kf_st4(v + col, x); return; }
    if (col + 0 < n) v[col + 0] = x.x;
    if (col + 1 < n) v[col + 1] = x.y;
    if (col + 2 < n) v[col + 2] = x.z;
}
__device__ __forceinline__ void kfb_stm(float* row, int col, int n, kf_f4 x) {
    if (col + 4 <= n) { kf_st4_nt(row + col, x); return; }
    if (col + 0 < n) row[col + 0] = x.x;
    if (col + 1 < n) row[col + 1] = x.y;
    if (col + 2 < n) row[col + 2] = x.z;
}

// threadIdx.x as an opaque value: per-thread column offsets are then
// recomputed for every item instead of being hoisted out of the persistent
// loop, where they would stay live across all buckets.
__device__ __forceinline__ int kfb_tid() {
    int t;
    asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
    return t;
}

// Column-indexed vectors (BiCGK p; GEMVER v1, v2, then x) are staged in LDS
// once per item and read from there at every row step: held in registers
// they would cost 2 K float4 per lane and halve the occupancy of the
// largest tiles.
// A compiler barrier at the top of each row step: the LDS copies of the
// column vectors are read again at every step instead of being hoisted into
// registers for the whole item.
__device__ __forceinline__ void kfb_reload_lds() { asm volatile("" ::: "memory"); }

struct Shared {
    kf_f4 red[KFB_THREADS];
    kf_f4 cv[2][KFB_MAX_N / 4];
    float rowp[2][4][16];   // wave partials of row sums, double-buffered (wide tiles)
    int flag;
    int item;
};

// Chunks 0 .. TPR K - 1 of a column vector into LDS (threads tid < TPR;
// entries >= n are zero). The caller synchronises before the first read.
template <int LTPR, int K>
__device__ __forceinline__ void kfb_stage(kf_f4* dst, const float* v, int n, int tid) {
    constexpr int TPR = 1 << LTPR;
    if (tid < TPR) {
#pragma unroll
        for (int k = 0; k < K; ++k) dst[tid + k * TPR] = kfb_ldv(v, 4 * (tid + k * TPR), n);
    }
}

// Wait (thread 0, bounded) until the instance's x is published, then acquire.
// Returns false in every thread if the wait ran out (error bit set).
__device__ __forceinline__ bool kfb_wait_x(unsigned* ctr, unsigned* sync, unsigned spin_limit, Shared& sh) {
    if (threadIdx.x == 0) {
        unsigned spins = 0;
        int ok = 1;
        while (__hip_atomic_load(ctr + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
            if (++spins > spin_limit) {
                atomicOr(sync + KFB_SYNC_ERROR, KFB_ERR_SPIN);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
        kfb_acquire();
        sh.flag = ok;
    }
    __syncthreads();
    const bool ready = sh.flag != 0;
    __syncthreads();
    return ready;
}

// w rows r0 .. r1 - 1 of alpha B x, x given per thread at its columns.
template <int LTPR, int K, int LG>
__device__ __forceinline__ void kfb_gemv_rows(const kfb_inst& I, const float* __restrict__ B,
                                              float* __restrict__ w, int r0, int r1, const kf_f4* xv) {
    // xv: x in LDS, chunk c at xv[c]
    constexpr int TPR = 1 << LTPR, G = 1 << LG, RL = KFB_THREADS / TPR, RI = RL * G;
    const int tid = kfb_tid(), cl = tid & (TPR - 1), rl = tid >> LTPR;
    const int n = I.n;
    const long ld = I.ld;
    kfb_cols cs[K];
#pragma unroll
    for (int k = 0; k < K; ++k) cs[k] = kfb_col(4 * (cl + k * TPR), n, I.ld);
#pragma unroll 1
    for (int i0 = r0; i0 < r1; i0 += RI) {
        kfb_reload_lds();
        kf_f4 b[G][K];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int row = i0 + g * RL + rl;
#pragma unroll
            for (int k = 0; k < K; ++k) b[g][k] = kfb_ldm(B, ld, row, r1, cs[k]);
        }
        float wp[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            wp[g] = 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k) wp[g] = kf_dot4(b[g][k], xv[cl + k * TPR], wp[g]);
        }
        const float ws = kfb_rows_reduce<LTPR, LG>(wp);
        const int g = cl >> (LTPR - LG);
        const int row = i0 + g * RL + rl;
        if ((cl & ((TPR >> LG) - 1)) == 0 && row < r1) w[row] = I.alpha * ws;
    }
}

template <int LTPR, int K, int LG>
__device__ void kfb_bicgk(const kfb_inst& I, int blk, float* __restrict__ arena, float* __restrict__ ws,
                          unsigned* sync, Shared& sh) {
    constexpr int TPR = 1 << LTPR, G = 1 << LG, RL = KFB_THREADS / TPR, RI = RL * G;
    const int tid = kfb_tid(), cl = tid & (TPR - 1), rl = tid >> LTPR;
    const int n = I.n;
    const long ld = I.ld;
    const int r0 = blk * I.rows, r1 = min(n, r0 + I.rows);
    const float* __restrict__ A = arena + I.a;
    const float* __restrict__ p = arena + I.v[0];
    const float* __restrict__ r = arena + I.v[1];
    float* __restrict__ q = arena + I.v[2];
    float* __restrict__ s = arena + I.v[3];
    kf_f4 acc[K];
    kfb_cols cs[K];
    kfb_stage<LTPR, K>(sh.cv[0], p, n, tid);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        cs[k] = kfb_col(4 * (cl + k * TPR), n, I.ld);
        acc[k] = kf_zero4();
    }
    __syncthreads();
    const kf_f4* pv = sh.cv[0] + cl;
#pragma unroll 1
    for (int i0 = r0; i0 < r1; i0 += RI) {
        kfb_reload_lds();
        kf_f4 a[G][K];
        float rr[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int row = i0 + g * RL + rl;
            const bool ok = row < r1;
            rr[g] = r[ok ? row : r1 - 1];
            rr[g] = ok ? rr[g] : 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k) a[g][k] = kfb_ldm(A, ld, row, r1, cs[k]);
        }
        float qp[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            qp[g] = 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k) qp[g] = kf_dot4(a[g][k], pv[k * TPR], qp[g]);
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] = kf_fma4s(rr[g], a[g][k], acc[k]);
        }
        const float qs = kfb_rows_reduce<LTPR, LG>(qp);
        const int g = cl >> (LTPR - LG);
        const int row = i0 + g * RL + rl;
        if ((cl & ((TPR >> LG) - 1)) == 0 && row < r1) q[row] = qs;
    }
    if (I.nblk == 1) {
        kfb_colsum<LTPR, K>(acc, sh.red, [&](int c, kf_f4 v) { kfb_stv(s, 4 * c, n, v); });
        return;
    }
    float* part = ws + I.ws + (long)blk * ld;
    kfb_colsum<LTPR, K>(acc, sh.red, [&](int c, kf_f4 v) {
        if (4 * c < ld) kf_st4(part + 4 * c, v);
    });
    unsigned* ctr = sync + KFB_SYNC_HEADER + KFB_SYNC_PER_INST * I.sync;
    if (kfb_arrive(ctr, (unsigned)I.nblk, &sh.flag)) {
        for (int c = threadIdx.x; 4 * c < n; c += KFB_THREADS) {
            kfb_stv(s, 4 * c, n, kfb_block_partials(ws + I.ws + 4 * c, ld, I.nblk));
        }
    }
}

template <int LTPR, int K, int LG>
__device__ void kfb_gemver_k1(const kfb_inst& I, int blk, float* __restrict__ arena, float* __restrict__ ws,
                              unsigned* sync, Shared& sh) {
    constexpr int TPR = 1 << LTPR, G = 1 << LG, RL = KFB_THREADS / TPR, RI = RL * G;
    const int tid = kfb_tid(), cl = tid & (TPR - 1), rl = tid >> LTPR;
    const int n = I.n;
    const long ld = I.ld;
    const int r0 = blk * I.rows, r1 = min(n, r0 + I.rows);
    const float* __restrict__ A = arena + I.a;
    float* __restrict__ B = arena + I.b;
    const float* __restrict__ u1 = arena + I.v[0];
    const float* __restrict__ v1 = arena + I.v[1];
    const float* __restrict__ u2 = arena + I.v[2];
    const float* __restrict__ v2 = arena + I.v[3];
    const float* __restrict__ y = arena + I.v[4];
    const float* __restrict__ z = arena + I.v[5];
    float* __restrict__ x = arena + I.v[6];
    float* __restrict__ w = arena + I.v[7];
    kf_f4 acc[K];
    kfb_cols cs[K];
    kfb_stage<LTPR, K>(sh.cv[0], v1, n, tid);
    kfb_stage<LTPR, K>(sh.cv[1], v2, n, tid);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        cs[k] = kfb_col(4 * (cl + k * TPR), n, I.ld);
        acc[k] = kf_zero4();
    }
    __syncthreads();
    const kf_f4* v1c = sh.cv[0] + cl;
    const kf_f4* v2c = sh.cv[1] + cl;
#pragma unroll 1
    for (int i0 = r0; i0 < r1; i0 += RI) {
        kfb_reload_lds();
        kf_f4 a[G][K];
        float u1r[G], u2r[G], yr[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int row = i0 + g * RL + rl;
            const bool ok = row < r1;
            const int rc = ok ? row : r1 - 1;
            u1r[g] = ok ? u1[rc] : 0.f;
            u2r[g] = ok ? u2[rc] : 0.f;
            yr[g] = ok ? y[rc] : 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k) a[g][k] = kfb_ldm(A, ld, row, r1, cs[k]);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int row = i0 + g * RL + rl;
            float* brow = B + (long)row * ld;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                kf_f4 b = kf_fma4s(u1r[g], v1c[k * TPR], a[g][k]);
                b = kf_fma4s(u2r[g], v2c[k * TPR], b);
                if (row < r1) kfb_stm(brow, 4 * (cl + k * TPR), n, b);
                acc[k] = kf_fma4s(yr[g], b, acc[k]);
            }
        }
    }
    if (I.nblk == 1) {
        // x is complete inside this workgroup: finish it, then run the gemv.
        kfb_colsum<LTPR, K>(acc, sh.red, [&](int c, kf_f4 v) {
            const kf_f4 xc = kf_fma4s(I.beta, v, kfb_ldv(z, 4 * c, n));
            kfb_stv(x, 4 * c, n, xc);
            sh.cv[0][c] = xc;
        });
        __syncthreads();
        kfb_gemv_rows<LTPR, K, LG>(I, B, w, 0, n, sh.cv[0]);
        return;
    }
    float* part = ws + I.ws + (long)blk * ld;
    kfb_colsum<LTPR, K>(acc, sh.red, [&](int c, kf_f4 v) {
        if (4 * c < ld) kf_st4(part + 4 * c, v);
    });
    unsigned* ctr = sync + KFB_SYNC_HEADER + KFB_SYNC_PER_INST * I.sync;
    if (kfb_arrive(ctr, (unsigned)I.nblk, &sh.flag)) {
        for (int c = threadIdx.x; 4 * c < n; c += KFB_THREADS) {
            const kf_f4 t = kfb_block_partials(ws + I.ws + 4 * c, ld, I.nblk);
            kfb_stv(x, 4 * c, n, kf_fma4s(I.beta, t, kfb_ldv(z, 4 * c, n)));
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            kfb_release();
            __hip_atomic_store(ctr + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int LTPR, int K, int LG>
__device__ void kfb_gemver_k2(const kfb_inst& I, int blk, float* __restrict__ arena, unsigned* sync,
                              unsigned spin_limit, Shared& sh) {
    const int n = I.n;
    unsigned* ctr = sync + KFB_SYNC_HEADER + KFB_SYNC_PER_INST * I.sync;
    if (!kfb_wait_x(ctr, sync, spin_limit, sh)) return;
    const float* __restrict__ B = arena + I.b;
    const float* __restrict__ x = arena + I.v[6];
    float* __restrict__ w = arena + I.v[7];
    kfb_stage<LTPR, K>(sh.cv[0], x, n, kfb_tid());
    __syncthreads();
    const int r0 = blk * I.rows, r1 = min(n, r0 + I.rows);
    kfb_gemv_rows<LTPR, K, LG>(I, B, w, r0, r1, sh.cv[0]);
    // the last K2 block of the instance clears the flag for the next launch
    if (kfb_count(ctr + 2, (unsigned)I.nblk, &sh.flag) && threadIdx.x == 0)
        __hip_atomic_store(ctr + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


// ---- wide BiCGK tiles (n > 512): the four waves split each row's columns ---
// Lane t of the workgroup owns chunks t + 256 k (k < K) of every row of the
// item, so the column result A^T r needs no cross-lane reduction; G rows
// are loaded per step, and a row sum is finished by a transposing reduction
// inside each wave and then the four wave partials, added in wave order after
// one barrier per step (double-buffered in LDS). This is the row-resident
// layout of the single-instance kernels at batch-instance size; it keeps the
// per-lane state small, so more waves are resident.

// Row-indexed scalars of the wide tiles: lanes 0 .. G - 1 load v[i0 + lane]
// (zero past r1) one step ahead; kfb_row_bcast reads each lane as a
// wave-uniform value once the load has long completed.
template <int G>
__device__ __forceinline__ float kfb_row_fetch(const float* v, int i0, int r1) {
    const int lane = __lane_id();
    return (lane < G && i0 + lane < r1) ? v[i0 + lane] : 0.f;
}
template <int G>
__device__ __forceinline__ void kfb_row_bcast(float x, float* out) {
#pragma unroll
    for (int g = 0; g < G; ++g) out[g] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), g));
}

template <int K, int LG>
__device__ __forceinline__ void kfb_w_rows_sum(const float* qp_in, float* __restrict__ out, float scale, int i0,
                                               int r1, Shared& sh, int& buf) {
    constexpr int G = 1 << LG;
    float qp[G];
#pragma unroll
    for (int g = 0; g < G; ++g) qp[g] = qp_in[g];
    const float sw = kfb_rows_reduce<6, LG>(qp);
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    if ((lane & ((64 >> LG) - 1)) == 0) sh.rowp[buf][wave][lane >> (6 - LG)] = sw;
    __syncthreads();
    if (threadIdx.x < G && i0 + (int)threadIdx.x < r1) {
        const int g = threadIdx.x;
        kf_cs t = kf_cs_init(sh.rowp[buf][0][g]);
        t = kf_cs_add(t, sh.rowp[buf][1][g]);
        t = kf_cs_add(t, sh.rowp[buf][2][g]);
        t = kf_cs_add(t, sh.rowp[buf][3][g]);
        out[i0 + g] = scale * kf_cs_value(t);
    }
    buf ^= 1;
}

template <int K, int LG>
__device__ void kfb_w_bicgk(const kfb_inst& I, int blk, float* __restrict__ arena, float* __restrict__ ws,
                            unsigned* sync, Shared& sh) {
    constexpr int G = 1 << LG;
    const int t = kfb_tid();
    const int n = I.n;
    const long ld = I.ld;
    const int r0 = blk * I.rows, r1 = min(n, r0 + I.rows);
    const float* __restrict__ A = arena + I.a;
    const float* __restrict__ r = arena + I.v[1];
    float* __restrict__ q = arena + I.v[2];
    float* __restrict__ s = arena + I.v[3];
    kf_f4 pv[K], acc[K];
    kfb_cols cs[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        cs[k] = kfb_col(4 * (t + 256 * k), n, I.ld);
        pv[k] = kfb_ldv(arena + I.v[0], 4 * (t + 256 * k), n);
        acc[k] = kf_zero4();
    }
    int buf = 0;
    float r_next = kfb_row_fetch<G>(r, r0, r1);
#pragma unroll 1
    for (int i0 = r0; i0 < r1; i0 += G) {
        const float r_cur = r_next;
        kf_f4 a[G][K];
        float rr[G];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int k = 0; k < K; ++k) a[g][k] = kfb_ldm(A, ld, i0 + g, r1, cs[k]);
        r_next = kfb_row_fetch<G>(r, i0 + G, r1);     // issued after this step's matrix loads
        kfb_row_bcast<G>(r_cur, rr);
        float qp[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            qp[g] = 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k) qp[g] = kf_dot4(a[g][k], pv[k], qp[g]);
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] = kf_fma4s(rr[g], a[g][k], acc[k]);
        }
        kfb_w_rows_sum<K, LG>(qp, q, 1.f, i0, r1, sh, buf);
    }
    if (I.nblk == 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) kfb_stv(s, 4 * (t + 256 * k), n, acc[k]);
        return;
    }
    float* part = ws + I.ws + (long)blk * ld;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (4 * (t + 256 * k) < I.ld) kf_st4(part + 4 * (t + 256 * k), acc[k]);
    unsigned* ctr = sync + KFB_SYNC_HEADER + KFB_SYNC_PER_INST * I.sync;
    if (kfb_arrive(ctr, (unsigned)I.nblk, &sh.flag)) {
        for (int c = threadIdx.x; 4 * c < n; c += KFB_THREADS) {
            kfb_stv(s, 4 * c, n, kfb_block_partials(ws + I.ws + 4 * c, ld, I.nblk));
        }
    }
}

// Tile T of the menu of (KIND, B), instantiated from the shared table.
template <int KIND, int B, int T>
__device__ __forceinline__ void kfb_tile_run(const kfb_inst& I, int phase, int blk, float* arena, float* ws,
                                             unsigned* sync, unsigned spin_limit, Shared& sh) {
    constexpr kfb_tile x = kfb_tile_menu[KIND][B][T];
    if constexpr (x.k == 0) {
        return;   // not on the menu (the host never selects it)
    } else if constexpr (x.wide) {
        kfb_w_bicgk<x.k, x.lg>(I, blk, arena, ws, sync, sh);
    } else if constexpr (KIND == 0) {
        kfb_bicgk<x.ltpr, x.k, x.lg>(I, blk, arena, ws, sync, sh);
    } else if (phase == KFB_GEMVER_K1) {
        kfb_gemver_k1<x.ltpr, x.k, x.lg>(I, blk, arena, ws, sync, sh);
    } else {
        kfb_gemver_k2<x.ltpr, x.k, x.lg>(I, blk, arena, sync, spin_limit, sh);
    }
}

template <int KIND, int B>
__device__ __forceinline__ void kfb_bucket_run(const kfb_inst& I, int phase, int blk, float* arena, float* ws,
                                               unsigned* sync, unsigned spin_limit, Shared& sh) {
    switch (I.tile) {
    case 1: kfb_tile_run<KIND, B, 1>(I, phase, blk, arena, ws, sync, spin_limit, sh); break;
    case 2: kfb_tile_run<KIND, B, 2>(I, phase, blk, arena, ws, sync, spin_limit, sh); break;
    default: kfb_tile_run<KIND, B, 0>(I, phase, blk, arena, ws, sync, spin_limit, sh); break;
    }
}

template <int KIND>
__device__ __forceinline__ void kfb_kind_run(const kfb_inst& I, int phase, int blk, float* arena, float* ws,
                                             unsigned* sync, unsigned spin_limit, Shared& sh) {
    switch (I.bucket) {
    case 0: kfb_bucket_run<KIND, 0>(I, phase, blk, arena, ws, sync, spin_limit, sh); break;
    case 1: kfb_bucket_run<KIND, 1>(I, phase, blk, arena, ws, sync, spin_limit, sh); break;
    case 2: kfb_bucket_run<KIND, 2>(I, phase, blk, arena, ws, sync, spin_limit, sh); break;
    case 3: kfb_bucket_run<KIND, 3>(I, phase, blk, arena, ws, sync, spin_limit, sh); break;
    case 4: kfb_bucket_run<KIND, 4>(I, phase, blk, arena, ws, sync, spin_limit, sh); break;
    default: kfb_bucket_run<KIND, 5>(I, phase, blk, arena, ws, sync, spin_limit, sh); break;
    }
}

// Three waves per SIMD (168 VGPRs, two of them spilled): the whole-row GEMVER
// tiles of the largest bucket keep eight 16-byte loads per lane in flight.
__global__ void __launch_bounds__(KFB_THREADS) __attribute__((amdgpu_waves_per_eu(3, 8)))
kfb_kernel(const kfb_inst* __restrict__ insts, const kfb_item* __restrict__ items, int nitems, int item0,
           int persistent, float* arena, float* ws, unsigned* sync, unsigned spin_limit) {
    __shared__ Shared sh;
    for (;;) {
        int it;
        if (persistent) {
            if (threadIdx.x == 0) sh.item = (int)atomicAdd(sync + KFB_SYNC_QUEUE, 1u);
            __syncthreads();
            it = sh.item;
            __syncthreads();
            if (it >= nitems) break;
        } else {
            it = item0 + (int)blockIdx.x;
        }
        const kfb_item item = items[it];
        const kfb_inst I = insts[item.inst];
        const int phase = item.phase_blk >> 24;
        const int blk = item.phase_blk & 0xffffff;
        // the instance's tile from the menu of its kind and size bucket (by
        // default BiCGK takes the wide tiles above n = 512; GEMVER keeps whole
        // rows per wave there, which stores B faster, measured per bucket)
        if (I.kind == 0) kfb_kind_run<0>(I, phase, blk, arena, ws, sync, spin_limit, sh);   // BiCGK
        else kfb_kind_run<1>(I, phase, blk, arena, ws, sync, spin_limit, sh);
        if (!persistent) break;
        __syncthreads();
    }
    if (persistent && threadIdx.x == 0) {
        if (atomicAdd(sync + KFB_SYNC_EXIT, 1u) == gridDim.x - 1) {
            __hip_atomic_store(sync + KFB_SYNC_QUEUE, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(sync + KFB_SYNC_EXIT, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace

// Persistent launch (grid workgroups draining the queue) or a direct launch of
// items item0 .. item0 + grid - 1, one per workgroup.
hipError_t kfb_launch(const kfb_inst* insts, const kfb_item* items, int nitems, int item0, int grid, int persistent,
                      float* arena, float* ws, unsigned* sync, unsigned spin_limit, hipStream_t st) {
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(kfb_kernel, dim3(grid), dim3(KFB_THREADS), 0, st, insts, items, nitems, item0, persistent,
                       arena, ws, sync, spin_limit);
    return hipGetLastError();
}

hipError_t kfb_resident_blocks(int* per_cu, int* cus) {
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kfb_kernel, KFB_THREADS, 0);
    if (e != hipSuccess) return e;
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    return hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
}
