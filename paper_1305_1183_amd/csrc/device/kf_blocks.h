// kf_blocks.h -- gfx950 building blocks that the generated kernels compose.
//
// These are the "routines" of the paper's elementary functions (Section 4.3:
// load, compute and store routines glued into one kernel), written for CDNA4:
// 64-lane wavefronts, 128-bit global loads and stores, cross-lane exchanges
// instead of shared-memory atomics, and a deterministic two-level reduction:
// workgroups write partial sums, and a second launch adds them in a fixed
// order (the "extra kernel" option of Section 3.2.2).
//
// This header is prepended verbatim to every run-time compiled source; it has
// no includes of its own (hipRTC provides the HIP device runtime).

typedef float kf_f4 __attribute__((ext_vector_type(4)));

// ---- B1/B2: 128-bit loads and stores ----------------------------------------
// Streamed matrix data is read once per plan, so it is loaded and stored with
// the non-temporal hint; vectors use ordinary cached accesses.
__device__ __forceinline__ kf_f4 kf_ld4_nt(const float* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const kf_f4*>(p));
}
__device__ __forceinline__ kf_f4 kf_ld4(const float* p) {
    return *reinterpret_cast<const kf_f4*>(p);
}
__device__ __forceinline__ void kf_st4_nt(float* p, kf_f4 v) {
    __builtin_nontemporal_store(v, reinterpret_cast<kf_f4*>(p));
}
__device__ __forceinline__ void kf_st4(float* p, kf_f4 v) {
    *reinterpret_cast<kf_f4*>(p) = v;
}
// Non-temporal 16-byte load and store at float offset `off` from a wave-uniform
// base: a 32-bit offset keeps the address one scalar base plus one lane
// register (off < 2^30).
__device__ __forceinline__ kf_f4 kf_ld4_nt_at(const float* base, unsigned off) {
    return __builtin_nontemporal_load(reinterpret_cast<const kf_f4*>(reinterpret_cast<const char*>(base) + 4u * off));
}
__device__ __forceinline__ void kf_st4_nt_at(float* base, unsigned off, kf_f4 v) {
    __builtin_nontemporal_store(v, reinterpret_cast<kf_f4*>(reinterpret_cast<char*>(base) + 4u * off));
}
__device__ __forceinline__ kf_f4 kf_zero4() { kf_f4 z = {0.f, 0.f, 0.f, 0.f}; return z; }

// Vector entries col..col+3, entries at index >= n read as zero (the vector
// buffer holds exactly n floats, so nothing past n is touched).
__device__ __forceinline__ kf_f4 kf_ld4_tail(const float* v, long col, long n) {
    if (col + 4 <= n) return kf_ld4(v + col);
    kf_f4 r = kf_zero4();
    if (col + 0 < n) r.x = v[col + 0];
    if (col + 1 < n) r.y = v[col + 1];
    if (col + 2 < n) r.z = v[col + 2];
    return r;
}
__device__ __forceinline__ void kf_st4_tail(float* v, long col, long n, kf_f4 x) {
    if (col + 4 <= n) { kf_st4(v + col, x); return; }
    if (col + 0 < n) v[col + 0] = x.x;
    if (col + 1 < n) v[col + 1] = x.y;
    if (col + 2 < n) v[col + 2] = x.z;
}

// Matrix row segment at the right edge: the row holds ld >= round_up(n, 4)
// floats, so a float4 starting below n is inside the row; entries >= n are
// padding and are replaced by zero with a select (padding may hold NaN).
__device__ __forceinline__ kf_f4 kf_ldm_edge(const float* row, long col, long n) {
    if (col >= n) return kf_zero4();
    kf_f4 r = kf_ld4_nt(row + col);
    if (col + 4 > n) {
        r.y = (col + 1 < n) ? r.y : 0.f;
        r.z = (col + 2 < n) ? r.z : 0.f;
        r.w = 0.f;
    }
    return r;
}
__device__ __forceinline__ void kf_stm_edge(float* row, long col, long n, kf_f4 x) {
    if (col >= n) return;
    if (col + 4 <= n) { kf_st4_nt(row + col, x); return; }
    row[col] = x.x;
    if (col + 1 < n) row[col + 1] = x.y;
    if (col + 2 < n) row[col + 2] = x.z;
}

// ---- quantised matrix storage (BF16, OCP FP8-E4M3) ---------------------------
typedef unsigned int kf_u4 __attribute__((ext_vector_type(4)));
typedef float kf_f2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ kf_u4 kf_ldu_nt(const unsigned char* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const kf_u4*>(p));
}
// 8 BF16 values (the upper halves of IEEE singles), lowest address first.
__device__ __forceinline__ void kf_dec_bf16(kf_u4 w, kf_f4* out) {
    out[0].x = __uint_as_float(w.x << 16); out[0].y = __uint_as_float(w.x & 0xffff0000u);
    out[0].z = __uint_as_float(w.y << 16); out[0].w = __uint_as_float(w.y & 0xffff0000u);
    out[1].x = __uint_as_float(w.z << 16); out[1].y = __uint_as_float(w.z & 0xffff0000u);
    out[1].z = __uint_as_float(w.w << 16); out[1].w = __uint_as_float(w.w & 0xffff0000u);
}
// 16 FP8-E4M3 values with the hardware conversion (two bytes per instruction).
__device__ __forceinline__ kf_f4 kf_dec_fp8_word(unsigned int x) {
    const kf_f2 a = __builtin_amdgcn_cvt_pk_f32_fp8((int)x, false);
    const kf_f2 b = __builtin_amdgcn_cvt_pk_f32_fp8((int)x, true);
    kf_f4 r;
    r.x = a.x; r.y = a.y; r.z = b.x; r.w = b.y;
    return r;
}
__device__ __forceinline__ void kf_dec_fp8(kf_u4 w, kf_f4* out) {
    out[0] = kf_dec_fp8_word(w.x);
    out[1] = kf_dec_fp8_word(w.y);
    out[2] = kf_dec_fp8_word(w.z);
    out[3] = kf_dec_fp8_word(w.w);
}
// Four quantised elements (one float4 group) with one 4- or 8-byte load.
typedef unsigned int kf_u2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ kf_f4 kf_ld4_fp8_nt(const unsigned char* p) {
    return kf_dec_fp8_word(__builtin_nontemporal_load(reinterpret_cast<const unsigned int*>(p)));
}
__device__ __forceinline__ kf_f4 kf_ld4_bf16_nt(const unsigned char* p) {
    const kf_u2 w = __builtin_nontemporal_load(reinterpret_cast<const kf_u2*>(p));
    kf_f4 r;
    r.x = __uint_as_float(w.x << 16); r.y = __uint_as_float(w.x & 0xffff0000u);
    r.z = __uint_as_float(w.y << 16); r.w = __uint_as_float(w.y & 0xffff0000u);
    return r;
}
// Zero the components of v at column index >= n (v holds columns col..col+3).
__device__ __forceinline__ kf_f4 kf_mask4(kf_f4 v, long col, long n) {
    v.x = (col + 0 < n) ? v.x : 0.f;
    v.y = (col + 1 < n) ? v.y : 0.f;
    v.z = (col + 2 < n) ? v.z : 0.f;
    v.w = (col + 3 < n) ? v.w : 0.f;
    return v;
}

// ---- B8: element-wise map arithmetic (explicit FMAs, no contraction) --------
__device__ __forceinline__ kf_f4 kf_fma4s(float s, kf_f4 v, kf_f4 c) {
    kf_f4 r;
    r.x = __builtin_fmaf(s, v.x, c.x); r.y = __builtin_fmaf(s, v.y, c.y);
    r.z = __builtin_fmaf(s, v.z, c.z); r.w = __builtin_fmaf(s, v.w, c.w);
    return r;
}
__device__ __forceinline__ kf_f4 kf_fma4v(kf_f4 a, kf_f4 b, kf_f4 c) {
    kf_f4 r;
    r.x = __builtin_fmaf(a.x, b.x, c.x); r.y = __builtin_fmaf(a.y, b.y, c.y);
    r.z = __builtin_fmaf(a.z, b.z, c.z); r.w = __builtin_fmaf(a.w, b.w, c.w);
    return r;
}
__device__ __forceinline__ kf_f4 kf_mul4s(float s, kf_f4 v) {
    kf_f4 r;
    r.x = s * v.x; r.y = s * v.y; r.z = s * v.z; r.w = s * v.w;
    return r;
}
// acc + a.b over the four components, in component order.
__device__ __forceinline__ float kf_dot4(kf_f4 a, kf_f4 b, float acc) {
    acc = __builtin_fmaf(a.x, b.x, acc);
    acc = __builtin_fmaf(a.y, b.y, acc);
    acc = __builtin_fmaf(a.z, b.z, acc);
    acc = __builtin_fmaf(a.w, b.w, acc);
    return acc;
}

// ---- B4: cross-lane reductions over the 64-lane wavefront --------------------
__device__ __forceinline__ float kf_xor(float v, int mask) {
    const int lane = __lane_id();
    const int src = (lane ^ mask) << 2;
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(v)));
}
// Butterfly: every lane ends with the sum of all 64 lanes (same value in all).
__device__ __forceinline__ float kf_wave_sum(float v) {
    v += kf_xor(v, 32);
    v += kf_xor(v, 16);
    v += kf_xor(v, 8);
    v += kf_xor(v, 4);
    v += kf_xor(v, 2);
    v += kf_xor(v, 1);
    return v;
}
// Transposing reduction of G = 2^LG row partials held by every lane. Stage t
// exchanges half of the remaining values with the lane whose bit (5 - t)
// differs, so after LG stages lane l holds one partial of row l >> (6 - LG);
// a butterfly over the low 6 - LG bits then completes the sum. G rows cost
// G - 1 + (6 - LG) exchanges instead of 6 G.
template <int LG>
__device__ __forceinline__ float kf_rows_reduce(float* v) {
    const int lane = __lane_id();
    constexpr int G = 1 << LG;
#pragma unroll
    for (int t = 0; t < LG; ++t) {
        const int half = G >> (t + 1);
        const int mask = 32 >> t;
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
    for (int mask = (32 >> LG); mask >= 1; mask >>= 1) s += kf_xor(s, mask);
    return s;
}

// ---- B6: workgroup sum in wave order -----------------------------------------
// Returns the workgroup total in thread 0 (other threads get an unspecified value).
template <int NW>
__device__ __forceinline__ float kf_block_sum(float v, float* lds) {
    v = kf_wave_sum(v);
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    float s = 0.f;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < NW; ++w) s += lds[w];
    }
    return s;
}

// ---- B7: compensated summation of partial sums ---------------------------------
// A partial sum travels as a pair (s, c): s is the rounded running sum and c
// collects the rounding errors of the additions that formed it. Each addition
// is Knuth's TwoSum, which gives the exact error of fl(a + b) for any finite a
// and b without a branch (six additions; it relies on strict IEEE evaluation,
// so no reassociation -- the kernels are built without fast-math); a sum that
// overflows or meets an infinity or NaN keeps error 0, so the pair's value is
// the plain sum's infinity or NaN. Two pairs merge
// with TwoSum of their leading parts, and the value of a pair is s + c. The
// merge is symmetric in its arguments (the error term is exact), so a
// butterfly leaves every lane with the same pair. Every final reduction that
// combines partial sums of different waves or workgroups goes through these,
// in a fixed order, so results stay bit-reproducible; sums whose partials
// cancel keep the small remainder that plain FP32 addition would round away.
struct kf_cs { float s, c; };
struct kf_cs4 { kf_f4 s, c; };
__device__ __forceinline__ void kf_two_sum(float a, float b, float* s, float* e) {
    const float t = a + b;
    const float z = t - a;
    const float err = (a - (t - z)) + (b - z);
    // an infinite or NaN sum carries no error term (inf - inf would make it NaN)
    *e = __builtin_fabsf(t) <= 3.40282347e38f ? err : 0.f;
    *s = t;
}
__device__ __forceinline__ kf_cs kf_cs_init(float x) { kf_cs r = {x, 0.f}; return r; }
__device__ __forceinline__ kf_cs kf_cs_add(kf_cs a, float x) {
    float t, e;
    kf_two_sum(a.s, x, &t, &e);
    kf_cs r = {t, a.c + e};
    return r;
}
__device__ __forceinline__ kf_cs kf_cs_merge(kf_cs a, kf_cs b) {
    float t, e;
    kf_two_sum(a.s, b.s, &t, &e);
    kf_cs r = {t, (a.c + b.c) + e};
    return r;
}
__device__ __forceinline__ float kf_cs_value(kf_cs a) { return a.s + a.c; }

__device__ __forceinline__ kf_cs4 kf_cs4_init(kf_f4 x) { kf_cs4 r = {x, kf_zero4()}; return r; }
__device__ __forceinline__ kf_cs4 kf_cs4_pack(kf_cs x, kf_cs y, kf_cs z, kf_cs w) {
    kf_cs4 r;
    r.s.x = x.s; r.s.y = y.s; r.s.z = z.s; r.s.w = w.s;
    r.c.x = x.c; r.c.y = y.c; r.c.z = z.c; r.c.w = w.c;
    return r;
}
__device__ __forceinline__ kf_cs4 kf_cs4_add(kf_cs4 a, kf_f4 v) {
    return kf_cs4_pack(kf_cs_add(kf_cs{a.s.x, a.c.x}, v.x), kf_cs_add(kf_cs{a.s.y, a.c.y}, v.y),
                       kf_cs_add(kf_cs{a.s.z, a.c.z}, v.z), kf_cs_add(kf_cs{a.s.w, a.c.w}, v.w));
}
__device__ __forceinline__ kf_cs4 kf_cs4_merge(kf_cs4 a, kf_cs4 b) {
    return kf_cs4_pack(kf_cs_merge(kf_cs{a.s.x, a.c.x}, kf_cs{b.s.x, b.c.x}),
                       kf_cs_merge(kf_cs{a.s.y, a.c.y}, kf_cs{b.s.y, b.c.y}),
                       kf_cs_merge(kf_cs{a.s.z, a.c.z}, kf_cs{b.s.z, b.c.z}),
                       kf_cs_merge(kf_cs{a.s.w, a.c.w}, kf_cs{b.s.w, b.c.w}));
}
__device__ __forceinline__ kf_f4 kf_cs4_value(kf_cs4 a) {
    kf_f4 r;
    r.x = a.s.x + a.c.x; r.y = a.s.y + a.c.y; r.z = a.s.z + a.c.z; r.w = a.s.w + a.c.w;
    return r;
}

// Butterfly over the 64 lanes on pairs: every lane ends with the same pair.
__device__ __forceinline__ kf_cs kf_wave_sum_cs(kf_cs v) {
#pragma unroll
    for (int mask = 32; mask >= 1; mask >>= 1) {
        kf_cs o;
        o.s = kf_xor(v.s, mask);
        o.c = kf_xor(v.c, mask);
        v = kf_cs_merge(v, o);
    }
    return v;
}
// The same butterfly within aligned groups of NL lanes (NL a power of two,
// at most 64): every lane of a group ends with the merge of the group's pairs.
template <int NL>
__device__ __forceinline__ kf_cs kf_group_sum_cs(kf_cs v) {
#pragma unroll
    for (int mask = NL / 2; mask >= 1; mask >>= 1) {
        kf_cs o;
        o.s = kf_xor(v.s, mask);
        o.c = kf_xor(v.c, mask);
        v = kf_cs_merge(v, o);
    }
    return v;
}
// Lane src's value of v (src wave-uniform), as a scalar in every lane.
__device__ __forceinline__ float kf_lane_bcast(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
// Workgroup sum of one float per thread, compensated from the wave level on:
// the wave pairs are merged in wave order by thread 0, which gets the value
// (other threads get an unspecified value). lds holds 2 NW floats.
template <int NW>
__device__ __forceinline__ float kf_block_sum_cs(kf_cs v, float* lds) {
    v = kf_wave_sum_cs(v);
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) { lds[2 * wave] = v.s; lds[2 * wave + 1] = v.c; }
    __syncthreads();
    float r = 0.f;
    if (threadIdx.x == 0) {
        kf_cs t = {lds[0], lds[1]};
#pragma unroll
        for (int w = 1; w < NW; ++w) {
            kf_cs o = {lds[2 * w], lds[2 * w + 1]};
            t = kf_cs_merge(t, o);
        }
        r = kf_cs_value(t);
    }
    return r;
}
