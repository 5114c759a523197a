// codegen.cpp -- HIP source for one fused (or single-call) kernel of a plan.
//
// The generated kernel follows the schema of Algorithm 1: shared (LDS) data
// first, then indices, invariant loads, cleared accumulators of reductions,
// the serial loop over rows (or over vector chunks) calling the load, compute
// and store routines of every call in script order (Algorithm 2), and last
// the stores of the accumulated reductions. Values that stay on chip are
// never stored or reloaded (Section 4.3: fusion removes the store of the
// producer and the load of the consumer); a value goes to HBM only when it is
// a script output or a later kernel reads it.
//
// BLAS-2 kernels (nesting depth 2) run on a 2D decomposition of the rows x
// cols iteration space: a workgroup owns a strip of C = 256 k columns (k
// float4 per lane, 64 lanes) and R rows; its W waves split the rows and walk
// them G at a time. Row reductions (gemv) are finished by a transposing
// cross-lane reduction per G rows; column reductions (gemtv) accumulate in
// registers and are merged across waves through LDS at the end. When a
// reduction spans several workgroups their partial sums go to the workspace
// and a second, small launch adds them in a fixed order and applies the
// alpha/beta epilogue (Section 3.2.2, final reduction "by extra kernel"):
// the kernel boundary is the global barrier, so the main pass needs no
// cross-XCD cache write-back per workgroup.
//
// BLAS-1 kernels (nesting depth 1) stream float4 chunks with a grid-stride
// loop; dot products reduce per thread, per wave and per workgroup, and the
// finishing launch adds the workgroup partials with a compensated sum.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <sstream>

#include "kf_internal.h"

namespace kf {

static std::string F(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    int n = vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (n < (int)sizeof buf) return std::string(buf, n);
    std::string s(n + 1, '\0');
    va_start(ap, fmt);
    vsnprintf(&s[0], n + 1, fmt, ap);
    va_end(ap);
    s.resize(n);
    return s;
}

static uint64_t fnv1a(const std::string& s) {
    uint64_t h = 1469598103934665603ULL;
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ULL;
    }
    return h;
}

// Does value v, produced in kernel kid, have to be written to HBM (R6)?
static bool must_store(const Script& s, const std::vector<int>& part, int kid, int v) {
    const Value& val = s.values[v];
    if (val.output) return true;
    for (int d : val.consumers)
        if (part[d] != kid) return true;
    return false;
}

static bool produced_in(const Script& s, const std::vector<int>& part, int kid, int v) {
    int p = s.values[v].producer;
    return p >= 0 && part[p] == kid;
}

struct Emitter {
    std::ostringstream o;
    int ind = 1;
    void l(const std::string& line) {
        for (int i = 0; i < ind; ++i) o << "  ";
        o << line << "\n";
    }
};

// Scalar operand expression: kernel-local names sc<v>.
static std::string scal_name(int v) { return F("sc%d", v); }

static void add_scalar_args(const Script& s, int v, std::vector<KArg>* args, std::vector<int>* seen) {
    if (v < 0) return;
    if (std::find(seen->begin(), seen->end(), v) != seen->end()) return;
    seen->push_back(v);
    if (s.values[v].kind == VK::Const) args->push_back({ArgKind::ConstScalar, v});
    else args->push_back({ArgKind::DevScalarIn, v});
}

void kernel_bytes(const Script& s, const std::vector<int>& calls, const std::vector<int>& part,
                  uint64_t* rd, uint64_t* wr) {
    const int kid = part[calls[0]];
    std::set<int> reads, writes;
    for (int c : calls) {
        const Call& k = s.calls[c];
        int ops[5] = {k.alpha, k.beta, k.in[0], k.in[1], k.in[2]};
        for (int v : ops) {
            if (v < 0) continue;
            if (s.values[v].kind == VK::Const) continue;
            if (!produced_in(s, part, kid, v)) {
                reads.insert(v);
                if (s.values[v].scale >= 0) reads.insert(s.values[v].scale);   // row scales of a quantised matrix
            }
        }
        if (must_store(s, part, kid, k.out)) writes.insert(k.out);
    }
    auto bytes = [&](int v) -> uint64_t {
        const Value& x = s.values[v];
        switch (x.kind) {
            case VK::Vec: return (uint64_t)x.n * 4;
            case VK::Mat: return (uint64_t)x.rows * (uint64_t)x.cols * (uint64_t)dtype_size(x.dtype);
            case VK::DevScalar: return 4;
            default: return 0;
        }
    };
    uint64_t r = 0, w = 0;
    for (int v : reads) r += bytes(v);
    for (int v : writes) w += bytes(v);
    *rd = r;
    *wr = w;
}

// Finishing launch of column partials (both BLAS-2 schedules): for columns
// cc .. cc + 3, wave `wave` of FW adds row blocks wave, wave + FW, ... of each
// gemtv call's partials, compensated; the FW wave pairs are merged in wave
// order through LDS (one buffer, reused call by call) and wave 0 ends with
// sum<c> (zero in the other waves). Expects lane, wave, cc, N, NB, NP, FW
// and ws in scope; every barrier is outside divergent code.
static void emit_colpart_finish(Emitter& f, const std::vector<int>& gemtv_calls,
                                const std::map<int, size_t>& ws_off) {
    f.l("__shared__ kf_f4 kf_fr[2][FW][64];");
    bool first = true;
    for (int c : gemtv_calls) {
        const size_t off = ws_off.at(c);
        // eight partials are loaded before they are added, so their loads are in
        // flight together rather than one latency per row block
        f.l(F("kf_cs4 pc%d = kf_cs4_init(kf_zero4());", c));
        f.l("if (cc < N) {");
        f.l("  for (long b0 = wave; b0 < NB; b0 += 8 * FW) {");
        f.l("    kf_f4 pv[8];");
        f.l(F("    for (int i = 0; i < 8; ++i) { const long b = b0 + (long)i * FW; pv[i] = b < NB ? kf_ld4(ws + %zuL + b * NP + cc) : kf_zero4(); }", off));
        f.l(F("    for (int i = 0; i < 8; ++i) if (b0 + (long)i * FW < NB) pc%d = kf_cs4_add(pc%d, pv[i]);", c, c));
        f.l("  }");
        f.l("}");
        if (!first) f.l("__syncthreads();");
        first = false;
        f.l(F("kf_fr[0][wave][lane] = pc%d.s; kf_fr[1][wave][lane] = pc%d.c;", c, c));
        f.l("__syncthreads();");
        f.l(F("kf_f4 sum%d = kf_zero4();", c));
        f.l("if (wave == 0) {");
        f.l("  kf_cs4 t = {kf_fr[0][0][lane], kf_fr[1][0][lane]};");
        f.l("  for (int w = 1; w < FW; ++w) { const kf_cs4 o = {kf_fr[0][w][lane], kf_fr[1][w][lane]}; t = kf_cs4_merge(t, o); }");
        f.l(F("  sum%d = kf_cs4_value(t);", c));
        f.l("}");
    }
}

// ============================================================================
// BLAS-2 kernels
// ============================================================================
static KernelCode gen_mat(const Script& s, const std::vector<int>& calls,
                          const std::vector<int>& part, const MatParams& p) {
    KernelCode kc;
    kc.mat = true;
    kc.calls = calls;
    const int kid = part[calls[0]];
    const Space sp = call_space(s, calls[0]);
    const long M = (long)sp.a, N = (long)sp.b;
    // E matrix elements per 16-byte load unit (4 FP32, 8 BF16, 16 FP8); a lane
    // takes p.k units per row, i.e. K = k E / 4 float4 column groups.
    const int E = kernel_unit_elems(s, calls, p.unit), EG = E / 4;
    const int U = p.k, K = p.k * EG, W = p.waves, G = p.group, R = p.rows, NT = 64 * W;
    int LG = 0;
    while ((1 << LG) < G) ++LG;
    const long C = 64L * E * U;
    const long S = (N + C - 1) / C, NB = (M + R - 1) / R;
    const long NP = (N + 3) / 4 * 4;

    // ---- classify operands
    std::vector<int> mat_in, mat_out, colv, rowv, vec_in, vec_out, gemv_calls, gemtv_calls;
    std::vector<int> scalars;
    auto push_u = [](std::vector<int>& v, int x) {
        if (std::find(v.begin(), v.end(), x) == v.end()) v.push_back(x);
    };
    for (int c : calls) {
        const Call& k = s.calls[c];
        int A = k.in[0];
        if (!produced_in(s, part, kid, A)) push_u(mat_in, A);
        if (k.op == Op::Ger) {
            push_u(rowv, k.in[1]);
            push_u(colv, k.in[2]);
            if (must_store(s, part, kid, k.out)) push_u(mat_out, k.out);
        } else if (k.op == Op::Gemv) {
            push_u(colv, k.in[1]);
            gemv_calls.push_back(c);
            if (k.in[2] >= 0 && !produced_in(s, part, kid, k.in[2])) push_u(vec_in, k.in[2]);
            if (must_store(s, part, kid, k.out)) push_u(vec_out, k.out);
        } else if (k.op == Op::Gemtv) {
            push_u(rowv, k.in[1]);
            gemtv_calls.push_back(c);
            if (k.in[2] >= 0 && !produced_in(s, part, kid, k.in[2])) push_u(vec_in, k.in[2]);
            if (must_store(s, part, kid, k.out)) push_u(vec_out, k.out);
        }
    }
    // quantised matrices bring their row scales (staged like other row vectors)
    for (int v : mat_in)
        if (s.values[v].scale >= 0) push_u(rowv, s.values[v].scale);
    for (int v : colv) push_u(vec_in, v);
    for (int v : rowv) push_u(vec_in, v);
    const bool row_part = !gemv_calls.empty() && S > 1;
    const bool col_part = !gemtv_calls.empty() && NB > 1;

    // ---- workspace layout (floats) and tickets
    std::map<int, size_t> ws_off;
    size_t wsz = 0;
    if (row_part)
        for (int c : gemv_calls) { ws_off[c] = wsz; wsz += (size_t)S * M; wsz = (wsz + 3) / 4 * 4; }
    if (col_part)
        for (int c : gemtv_calls) { ws_off[c] = wsz; wsz += (size_t)NB * NP; }
    kc.ws_floats = wsz;

    // ---- arguments
    std::vector<std::string> sig;
    for (int v : mat_in)
        sig.push_back(s.values[v].dtype == KF_F32 ? F("const float* __restrict__ M%d", v)
                                                  : F("const unsigned char* __restrict__ M%d", v));
    for (int v : mat_out) sig.push_back(F("float* __restrict__ O%d", v));
    for (int v : vec_in) sig.push_back(F("const float* __restrict__ V%d", v));
    // outputs the main pass writes itself (the rest are written by the finishing launch)
    std::vector<int> main_out;
    for (int v : vec_out) {
        Op op = s.calls[s.values[v].producer].op;
        if (!((op == Op::Gemv && row_part) || (op == Op::Gemtv && col_part))) main_out.push_back(v);
    }
    for (int v : main_out) sig.push_back(F("float* __restrict__ Y%d", v));
    std::vector<KArg> kc_scalar_args;
    {
        for (int c : calls) {
            add_scalar_args(s, s.calls[c].alpha, &kc_scalar_args, &scalars);
            if (s.calls[c].in[2] >= 0 && s.calls[c].op != Op::Ger)
                add_scalar_args(s, s.calls[c].beta, &kc_scalar_args, &scalars);
        }
        for (auto& a : kc_scalar_args) {
            if (a.kind == ArgKind::ConstScalar) sig.push_back(F("float P%d", a.value));
            else sig.push_back(F("const float* __restrict__ P%d", a.value));
        }
    }
    Launch mainl;
    for (int v : mat_in) mainl.args.push_back({ArgKind::MatIn, v});
    for (int v : mat_out) mainl.args.push_back({ArgKind::MatOut, v});
    for (int v : vec_in) mainl.args.push_back({ArgKind::VecIn, v});
    for (int v : main_out) mainl.args.push_back({ArgKind::VecOut, v});
    for (auto& a : kc_scalar_args) mainl.args.push_back(a);
    mainl.args.push_back({ArgKind::Workspace, -1});
    sig.push_back("float* __restrict__ ws");
    if (p.dyn) {
        // runtime shape: rows, cols and each matrix's leading dimension are arguments
        mainl.args.push_back({ArgKind::ShapeM, -1});
        mainl.args.push_back({ArgKind::ShapeN, -1});
        sig.push_back("long M_");
        sig.push_back("long N_");
        for (int v : mat_in) { mainl.args.push_back({ArgKind::MatLd, v}); sig.push_back(F("long LD%d", v)); }
        for (int v : mat_out) { mainl.args.push_back({ArgKind::MatLd, v}); sig.push_back(F("long LD%d", v)); }
    }

    // ---- body
    Emitter e;
    e.l(F("constexpr int K = %d, W = %d, G = %d, LG = %d, R = %d, NT = %d, E = %d, EG = %d;", K, W, G, LG, R, NT, E, EG));
    if (p.dyn) {
        e.l(F("constexpr long C = %ldL;", C));
        e.l("const long M = M_, N = N_, S = (N + C - 1) / C, NB = (M + R - 1) / R, NP = (N + 3) / 4 * 4;");
        e.l("(void)NB; (void)NP;");
    } else {
        e.l(F("constexpr long M = %ldL, N = %ldL, C = %ldL, S = %ldL, NB = %ldL, NP = %ldL;", M, N, C, S, NB, NP));
        for (int v : mat_in) e.l(F("constexpr long LD%d = %ldL;", v, (long)s.values[v].ld));
        for (int v : mat_out) e.l(F("constexpr long LD%d = %ldL;", v, (long)s.values[v].ld));
    }
    e.l("const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;");
    e.l("const long sidx = blockIdx.x % S, rb = blockIdx.x / S;");
    e.l("const long c0 = sidx * C, r0 = rb * R;");
    e.l("const long r1 = (r0 + R < M) ? r0 + R : M;");
    e.l("(void)ws;");
    for (int v : scalars) {
        if (s.values[v].kind == VK::Const) e.l(F("const float %s = P%d;", scal_name(v).c_str(), v));
        else e.l(F("const float %s = *P%d;", scal_name(v).c_str(), v));
    }
    e.l("long col[K];");
    e.l("#pragma unroll");
    e.l("for (int j = 0; j < K; ++j) col[j] = c0 + (long)((j / EG) * 64 + lane) * E + 4 * (j % EG);");
    // invariant column vectors (Algorithm 1, "load invariant data")
    for (int v : colv) {
        e.l(F("kf_f4 cv%d[K];", v));
        e.l("#pragma unroll");
        e.l(F("for (int j = 0; j < K; ++j) cv%d[j] = kf_ld4_tail(V%d, col[j], N);", v, v));
    }
    // row vectors staged in LDS; rows past the end read as zero
    for (int v : rowv) {
        e.l(F("__shared__ float rv%d[R];", v));
        e.l(F("for (int i = tid; i < R; i += NT) rv%d[i] = (r0 + i < M) ? V%d[r0 + i] : 0.f;", v, v));
    }
    // cleared accumulators (Algorithm 1, "clear outputs of accumulated reductions")
    for (int c : gemtv_calls) {
        e.l(F("kf_f4 acc%d[K];", c));
        e.l("#pragma unroll");
        e.l(F("for (int j = 0; j < K; ++j) acc%d[j] = kf_zero4();", c));
    }
    e.l("__syncthreads();");

    // Matrix value expression for matrix v at row gi.
    auto mexpr = [&](int v) -> std::string {
        if (produced_in(s, part, kid, v)) return F("m%d", v);
        return F("L%d[gi]", v);
    };
    // Row epilogue for all gemv calls at `row`, sums in sum<c>.
    auto row_epilogue = [&](const char* rowvar) {
        for (int c : gemv_calls) {
            const Call& k = s.calls[c];
            std::string val = F("%s * sum%d", scal_name(k.alpha).c_str(), c);
            if (k.in[2] >= 0) {
                std::string y0 = produced_in(s, part, kid, k.in[2]) ? F("f%d", s.values[k.in[2]].producer)
                                                                     : F("V%d[%s]", k.in[2], rowvar);
                val = F("__builtin_fmaf(%s, %s, %s)", scal_name(k.beta).c_str(), y0.c_str(), val.c_str());
            }
            e.l(F("const float f%d = %s;", c, val.c_str()));
            if (must_store(s, part, kid, k.out)) e.l(F("Y%d[%s] = f%d;", k.out, rowvar, c));
            else e.l(F("(void)f%d;", c));
        }
    };

    auto emit_loop = [&](bool edge) {
        e.l("for (long g0 = r0 + (long)wave * G; g0 < r1; g0 += (long)W * G) {");
        e.ind++;
        // loads of every matrix read from HBM (load routines)
        for (int v : mat_in) e.l(F("kf_f4 L%d[G][K];", v));
        e.l("#pragma unroll");
        e.l("for (int gi = 0; gi < G; ++gi) {");
        e.ind++;
        e.l("const long row = g0 + gi;");
        for (int v : mat_in) {
            e.l("#pragma unroll");
            const int dt = s.values[v].dtype;
            if (dt != KF_F32 && E == 4) {
                // narrow units: four elements (4 or 8 bytes) per float4 group, laid out like FP32
                const int es = dtype_size(dt);
                const char* ld4 = dt == KF_BF16 ? "kf_ld4_bf16_nt" : "kf_ld4_fp8_nt";
                if (!edge)
                    e.l(F("for (int j = 0; j < K; ++j) L%d[gi][j] = %s(M%d + (row * LD%d + col[j]) * %d);", v, ld4, v, v, es));
                else
                    e.l(F("for (int j = 0; j < K; ++j) L%d[gi][j] = (row < r1 && col[j] < N) ? kf_mask4(%s(M%d + (row * LD%d + col[j]) * %d), col[j], N) : kf_zero4();",
                          v, ld4, v, v, es));
            } else if (dt != KF_F32) {
                // one 16-byte unit per (row, u) decodes into 16/es elements = EQ float4 groups;
                // a BF16 matrix in a kernel with 16-element units takes two units per span
                const int es = dtype_size(dt), per = 16 / es, EQ = per / 4;
                const char* dec = dt == KF_BF16 ? "kf_dec_bf16" : "kf_dec_fp8";
                e.l(F("for (int u = 0; u < %d; ++u) {", U * (E / per)));
                e.ind++;
                e.l(F("const long cu0 = col[(u / %d) * EG] + (long)(u %% %d) * %d;", E / per, E / per, per));
                if (!edge) {
                    e.l(F("%s(kf_ldu_nt(M%d + (row * LD%d + cu0) * %d), &L%d[gi][u * %d]);", dec, v, v, es, v, EQ));
                } else {
                    e.l(F("if (row < r1 && cu0 < N) { %s(kf_ldu_nt(M%d + (row * LD%d + cu0) * %d), &L%d[gi][u * %d]);", dec, v, v, es, v, EQ));
                    e.l(F("  for (int q = 0; q < %d; ++q) L%d[gi][u * %d + q] = kf_mask4(L%d[gi][u * %d + q], cu0 + 4 * q, N); }", EQ, v, EQ, v, EQ));
                    e.l(F("else { for (int q = 0; q < %d; ++q) L%d[gi][u * %d + q] = kf_zero4(); }", EQ, v, EQ));
                }
                e.ind--;
                e.l("}");
            } else if (!edge)
                e.l(F("for (int j = 0; j < K; ++j) L%d[gi][j] = kf_ld4_nt(M%d + row * LD%d + col[j]);", v, v, v));
            else
                e.l(F("for (int j = 0; j < K; ++j) L%d[gi][j] = (row < r1) ? kf_ldm_edge(M%d + row * LD%d, col[j], N) : kf_zero4();", v, v, v));
        }
        e.ind--;
        e.l("}");
        for (int c : gemv_calls) e.l(F("float rp%d[G];", c));
        e.l("#pragma unroll");
        e.l("for (int gi = 0; gi < G; ++gi) {");
        e.ind++;
        e.l("const long row = g0 + gi;");
        e.l("const int rl = (int)(row - r0);");
        e.l("(void)rl;");
        // compute routines in script order
        for (int c : calls) {
            const Call& k = s.calls[c];
            std::string Min = mexpr(k.in[0]);
            const int qscale = s.values[k.in[0]].scale;   // row scale of a quantised matrix, or -1
            if (k.op == Op::Ger) {
                int o = k.out;
                e.l(F("const float cu%d = %s * rv%d[rl];", c, scal_name(k.alpha).c_str(), k.in[1]));
                e.l(F("kf_f4 m%d[K];", o));
                e.l("#pragma unroll");
                if (qscale >= 0)
                    e.l(F("for (int j = 0; j < K; ++j) m%d[j] = kf_fma4s(cu%d, cv%d[j], kf_mul4s(rv%d[rl], %s[j]));", o, c, k.in[2], qscale, Min.c_str()));
                else
                    e.l(F("for (int j = 0; j < K; ++j) m%d[j] = kf_fma4s(cu%d, cv%d[j], %s[j]);", o, c, k.in[2], Min.c_str()));
                if (must_store(s, part, kid, o)) {
                    if (!edge) {
                        e.l("#pragma unroll");
                        e.l(F("for (int j = 0; j < K; ++j) kf_st4_nt(O%d + row * LD%d + col[j], m%d[j]);", o, o, o));
                    } else {
                        e.l("if (row < r1) {");
                        e.l("#pragma unroll");
                        e.l(F("  for (int j = 0; j < K; ++j) kf_stm_edge(O%d + row * LD%d, col[j], N, m%d[j]);", o, o, o));
                        e.l("}");
                    }
                }
            } else if (k.op == Op::Gemtv) {
                if (qscale >= 0) e.l(F("const float xr%d = rv%d[rl] * rv%d[rl];", c, qscale, k.in[1]));
                else e.l(F("const float xr%d = rv%d[rl];", c, k.in[1]));
                e.l("#pragma unroll");
                e.l(F("for (int j = 0; j < K; ++j) acc%d[j] = kf_fma4s(xr%d, %s[j], acc%d[j]);", c, c, Min.c_str(), c));
            } else if (k.op == Op::Gemv) {
                e.l(F("float t%d = 0.f;", c));
                e.l("#pragma unroll");
                e.l(F("for (int j = 0; j < K; ++j) t%d = kf_dot4(%s[j], cv%d[j], t%d);", c, Min.c_str(), k.in[1], c));
                if (qscale >= 0) e.l(F("rp%d[gi] = rv%d[rl] * t%d;", c, qscale, c));
                else e.l(F("rp%d[gi] = t%d;", c, c));
            }
        }
        e.ind--;
        e.l("}");
        // row reductions of this group
        if (!gemv_calls.empty()) {
            for (int c : gemv_calls) e.l(F("const float sum%d = kf_rows_reduce<LG>(rp%d);", c, c));
            e.l("{");
            e.ind++;
            e.l("const long row = g0 + (lane >> (6 - LG));");
            if (edge) e.l("if ((lane & ((64 >> LG) - 1)) == 0 && row < r1) {");
            else e.l("if ((lane & ((64 >> LG) - 1)) == 0) {");
            e.ind++;
            if (!row_part) {
                row_epilogue("row");
            } else {
                for (int c : gemv_calls) e.l(F("ws[%zuL + sidx * M + row] = sum%d;", ws_off[c], c));
            }
            e.ind--;
            e.l("}");
            e.ind--;
            e.l("}");
        }
        e.ind--;
        e.l("}");
    };
    e.l("const bool edge = (c0 + C > N) || (r0 + R > M);");
    e.l("if (!edge) {");
    e.ind++;
    emit_loop(false);
    e.ind--;
    e.l("} else {");
    e.ind++;
    emit_loop(true);
    e.ind--;
    e.l("}");

    // column reductions: merge the waves in wave order through LDS
    if (!gemtv_calls.empty()) {
        const int ngt = (int)gemtv_calls.size();
        e.l(F("__shared__ kf_f4 kf_red[%d][W * (C / 4)];", ngt));
        for (int i = 0; i < ngt; ++i) {
            int c = gemtv_calls[i];
            e.l("#pragma unroll");
            e.l(F("for (int j = 0; j < K; ++j) kf_red[%d][wave * (C / 4) + (int)((col[j] - c0) >> 2)] = acc%d[j];", i, c));
        }
        e.l("__syncthreads();");
        e.l("for (int q = tid; q < C / 4; q += NT) {");
        e.ind++;
        e.l("const long cc = c0 + 4L * q;");
        for (int i = 0; i < ngt; ++i) {
            int c = gemtv_calls[i];
            e.l(F("kf_cs4 cs%d = kf_cs4_init(kf_red[%d][q]);", c, i));
            e.l(F("for (int w = 1; w < W; ++w) cs%d = kf_cs4_add(cs%d, kf_red[%d][w * (C / 4) + q]);", c, c, i));
            e.l(F("const kf_f4 sum%d = kf_cs4_value(cs%d);", c, c));
        }
        if (!col_part) {
            e.l("if (cc < N) {");
            e.ind++;
            for (int c : gemtv_calls) {
                const Call& k = s.calls[c];
                std::string val = F("kf_mul4s(%s, sum%d)", scal_name(k.alpha).c_str(), c);
                if (k.in[2] >= 0) {
                    std::string y0 = produced_in(s, part, kid, k.in[2]) ? F("f%d", s.values[k.in[2]].producer)
                                                                         : F("kf_ld4_tail(V%d, cc, N)", k.in[2]);
                    val = F("kf_fma4s(%s, %s, %s)", scal_name(k.beta).c_str(), y0.c_str(), val.c_str());
                }
                e.l(F("const kf_f4 f%d = %s;", c, val.c_str()));
                if (must_store(s, part, kid, k.out)) e.l(F("kf_st4_tail(Y%d, cc, N, f%d);", k.out, c));
                else e.l(F("(void)f%d;", c));
            }
            e.ind--;
            e.l("}");
        } else {
            e.l("if (cc < N) {");
            for (int c : gemtv_calls) e.l(F("  kf_st4(ws + %zuL + rb * NP + cc, sum%d);", ws_off[c], c));
            e.l("}");
        }
        e.ind--;
        e.l("}");
    }
    // ---- finishing launch: adds the partial sums in a fixed order, then the epilogue
    Emitter f;
    Launch finl;
    std::vector<std::string> fsig;
    if (row_part || col_part) {
        std::vector<int> fin_in;
        for (int c : calls) {
            const Call& k = s.calls[c];
            bool part_here = (k.op == Op::Gemv && row_part) || (k.op == Op::Gemtv && col_part);
            if (part_here && k.in[2] >= 0 && !produced_in(s, part, kid, k.in[2])) push_u(fin_in, k.in[2]);
        }
        std::vector<int> fin_out;
        for (int v : vec_out) {
            Op op = s.calls[s.values[v].producer].op;
            if ((op == Op::Gemv && row_part) || (op == Op::Gemtv && col_part)) fin_out.push_back(v);
        }
        for (int v : fin_in) { finl.args.push_back({ArgKind::VecIn, v}); fsig.push_back(F("const float* __restrict__ V%d", v)); }
        for (int v : fin_out) { finl.args.push_back({ArgKind::VecOut, v}); fsig.push_back(F("float* __restrict__ Y%d", v)); }
        for (auto& a : kc_scalar_args) {
            finl.args.push_back(a);
            if (a.kind == ArgKind::ConstScalar) fsig.push_back(F("float P%d", a.value));
            else fsig.push_back(F("const float* __restrict__ P%d", a.value));
        }
        finl.args.push_back({ArgKind::Workspace, -1});
        fsig.push_back("const float* __restrict__ ws");
        const int FWb = (col_part && NB >= 64) ? 1024 : 256;
        const long RBK = row_part ? (M + FWb - 1) / FWb : 0;
        const long CBK = col_part ? (NP / 4 + 63) / 64 : 0;
        const int FW = NB >= 64 ? 16 : 4;   // waves of the finishing pass that split the row blocks
        if (p.dyn) {
            finl.args.push_back({ArgKind::ShapeM, -1});
            finl.args.push_back({ArgKind::ShapeN, -1});
            fsig.push_back("long M_");
            fsig.push_back("long N_");
            f.l(F("constexpr long C = %ldL, R = %dL, FWB = %dL;", C, R, FWb));
            f.l("const long M = M_, N = N_, S = (N + C - 1) / C, NB = (M + R - 1) / R, NP = (N + 3) / 4 * 4;");
            f.l(row_part ? "const long RBK = (M + FWB - 1) / FWB;" : "const long RBK = 0;");
            f.l("(void)S; (void)NB; (void)NP; (void)RBK;");
        } else {
            f.l(F("constexpr long M = %ldL, N = %ldL, S = %ldL, NB = %ldL, NP = %ldL, RBK = %ldL;", M, N, S, NB, NP, RBK));
        }
        f.l(F("constexpr int FW = %d; (void)FW;", FW));
        for (int v : scalars) {
            if (s.values[v].kind == VK::Const) f.l(F("const float %s = P%d;", scal_name(v).c_str(), v));
            else f.l(F("const float %s = *P%d;", scal_name(v).c_str(), v));
        }
        if (row_part) {
            f.l("if (blockIdx.x < RBK) {");
            f.ind++;
            f.l("const long row = (long)blockIdx.x * blockDim.x + threadIdx.x;");
            f.l("if (row < M) {");
            f.ind++;
            // the S strip partials of a row, compensated, in strip order
            for (int c : gemv_calls) {
                f.l(F("kf_cs cs%d = kf_cs_init(ws[%zuL + row]);", c, ws_off[c]));
                f.l(F("for (long si = 1; si < S; ++si) cs%d = kf_cs_add(cs%d, ws[%zuL + si * M + row]);", c, c, ws_off[c]));
                f.l(F("const float sum%d = kf_cs_value(cs%d);", c, c));
            }
            for (int c : gemv_calls) {
                const Call& k = s.calls[c];
                std::string val = F("%s * sum%d", scal_name(k.alpha).c_str(), c);
                if (k.in[2] >= 0) {
                    std::string y0 = produced_in(s, part, kid, k.in[2]) ? F("f%d", s.values[k.in[2]].producer)
                                                                         : F("V%d[row]", k.in[2]);
                    val = F("__builtin_fmaf(%s, %s, %s)", scal_name(k.beta).c_str(), y0.c_str(), val.c_str());
                }
                f.l(F("const float f%d = %s;", c, val.c_str()));
                if (must_store(s, part, kid, k.out)) f.l(F("Y%d[row] = f%d;", k.out, c));
                else f.l(F("(void)f%d;", c));
            }
            f.ind--;
            f.l("}");
            f.ind--;
            f.l("}");
        }
        if (col_part) {
            // 64 float4 columns per workgroup; the FW waves split the row blocks
            // (wave w adds blocks w, w + FW, ...) and are merged in wave order,
            // all of it compensated.
            f.l("if (blockIdx.x >= RBK) {");
            f.ind++;
            f.l("const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;");
            f.l("const long cc = 4L * ((long)(blockIdx.x - RBK) * 64 + lane);");
            emit_colpart_finish(f, gemtv_calls, ws_off);
            f.l("if (wave == 0 && cc < N) {");
            f.ind++;
            for (int c : gemtv_calls) {
                const Call& k = s.calls[c];
                std::string val = F("kf_mul4s(%s, sum%d)", scal_name(k.alpha).c_str(), c);
                if (k.in[2] >= 0) {
                    std::string y0 = produced_in(s, part, kid, k.in[2]) ? F("f%d", s.values[k.in[2]].producer)
                                                                         : F("kf_ld4_tail(V%d, cc, N)", k.in[2]);
                    val = F("kf_fma4s(%s, %s, %s)", scal_name(k.beta).c_str(), y0.c_str(), val.c_str());
                }
                f.l(F("const kf_f4 f%d = %s;", c, val.c_str()));
                if (must_store(s, part, kid, k.out)) f.l(F("kf_st4_tail(Y%d, cc, N, f%d);", k.out, c));
                else f.l(F("(void)f%d;", c));
            }
            f.ind--;
            f.l("}");
            f.ind--;
            f.l("}");
        }
        finl.grid = (int)(RBK + CBK);
        finl.block = col_part ? 64 * FW : 256;
        if (p.dyn) {
            finl.dyn_grid = 2;
            finl.dyn_c = C;
            finl.dyn_r = R;
            finl.dyn_fwb = FWb;
            finl.dyn_rpart = row_part;
            finl.dyn_cpart = col_part;
        }
    }
    // the main pass no longer stores outputs that the finishing launch writes
    std::ostringstream head;
    std::string sigs, fsigs;
    for (size_t i = 0; i < sig.size(); ++i) sigs += (i ? ",\n    " : "    ") + sig[i];
    for (size_t i = 0; i < fsig.size(); ++i) fsigs += (i ? ",\n    " : "    ") + fsig[i];
    std::string key = F("mat K%d W%d G%d R%d E%d M%ld N%ld%s|", K, W, G, R, E, M, N, p.dyn ? " dyn" : "") + sigs +
                      e.o.str() + fsigs + f.o.str();
    kc.name = F("kf_mat_%016llx", (unsigned long long)fnv1a(key));
    head << "extern \"C\" __global__ void __launch_bounds__(" << NT << ") " << kc.name << "(\n"
         << sigs << ") {\n" << e.o.str() << "}\n";
    mainl.name = kc.name;
    mainl.grid = (int)(S * NB);
    mainl.block = NT;
    if (p.dyn) {
        mainl.dyn_grid = 1;
        mainl.dyn_c = C;
        mainl.dyn_r = R;
    }
    kc.launches.push_back(mainl);
    if (row_part || col_part) {
        finl.name = kc.name + "_fin";
        head << "extern \"C\" __global__ void __launch_bounds__(" << finl.block << ") " << finl.name << "(\n"
             << fsigs << ") {\n" << f.o.str() << "}\n";
        kc.launches.push_back(finl);
    }
    kc.source = head.str();
    kc.lds_bytes = 16 + rowv.size() * (size_t)R * 4 + gemtv_calls.size() * (size_t)W * (C / 4) * 16;
    kc.params_json = F("{\"k\": %d, \"waves\": %d, \"group\": %d, \"rows\": %d, \"unit_elems\": %d, \"strips\": %ld, \"row_blocks\": %ld}",
                       U, W, G, R, E, S, NB);
    kernel_bytes(s, calls, part, &kc.bytes_read, &kc.bytes_written);
    return kc;
}

// ============================================================================
// BLAS-1 kernels
// ============================================================================
static KernelCode gen_vec(const Script& s, const std::vector<int>& calls,
                          const std::vector<int>& part, const VecParams& p) {
    KernelCode kc;
    kc.mat = false;
    kc.calls = calls;
    const int kid = part[calls[0]];
    const Space sp = call_space(s, calls[0]);
    const long N = (long)sp.a, N4 = N / 4, T = N % 4;
    const int U = p.unroll, NT = p.threads, GRID = p.grid, NW = NT / 64;

    std::vector<int> vec_in, vec_out, dots, scalars;
    auto push_u = [](std::vector<int>& v, int x) {
        if (std::find(v.begin(), v.end(), x) == v.end()) v.push_back(x);
    };
    for (int c : calls) {
        const Call& k = s.calls[c];
        for (int i = 0; i < 2; ++i)
            if (k.in[i] >= 0 && !produced_in(s, part, kid, k.in[i])) push_u(vec_in, k.in[i]);
        if (k.op == Op::Dot) {
            dots.push_back(c);
            if (must_store(s, part, kid, k.out)) push_u(vec_out, k.out);
        } else if (must_store(s, part, kid, k.out)) {
            push_u(vec_out, k.out);
        }
    }
    const int ndot = (int)dots.size();
    const bool dot_part = GRID > 1 && ndot > 0;
    kc.ws_floats = dot_part ? (size_t)ndot * GRID : 0;

    std::vector<std::string> sig;
    Launch mainl;
    for (int v : vec_in) { mainl.args.push_back({ArgKind::VecIn, v}); sig.push_back(F("const float* __restrict__ V%d", v)); }
    std::vector<int> dot_out;
    for (int v : vec_out) {
        bool sc = s.values[v].kind == VK::DevScalar;
        if (sc && dot_part) { dot_out.push_back(v); continue; }
        mainl.args.push_back({sc ? ArgKind::DevScalarOut : ArgKind::VecOut, v});
        sig.push_back(F("float* __restrict__ Y%d", v));
    }
    {
        std::vector<KArg> sargs;
        for (int c : calls) add_scalar_args(s, s.calls[c].alpha, &sargs, &scalars);
        for (auto& a : sargs) {
            mainl.args.push_back(a);
            if (a.kind == ArgKind::ConstScalar) sig.push_back(F("float P%d", a.value));
            else sig.push_back(F("const float* __restrict__ P%d", a.value));
        }
    }
    mainl.args.push_back({ArgKind::Workspace, -1});
    sig.push_back("float* __restrict__ ws");

    Emitter e;
    e.l(F("constexpr long N = %ldL, N4 = %ldL, T = %ldL;", N, N4, T));
    e.l(F("constexpr int U = %d, NT = %d, GRID = %d, NW = %d;", U, NT, GRID, NW));
    e.l("constexpr long STEP = (long)NT * U;");
    e.l("const int tid = threadIdx.x;");
    e.l("__shared__ float kf_lds[2 * NW];");
    e.l("(void)kf_lds; (void)ws;");
    for (int v : scalars) {
        if (s.values[v].kind == VK::Const) e.l(F("const float %s = P%d;", scal_name(v).c_str(), v));
        else e.l(F("const float %s = *P%d;", scal_name(v).c_str(), v));
    }
    for (int c : dots) e.l(F("float dacc%d = 0.f;", c));

    // compute routines on one float4 chunk held in x<v>
    auto emit_compute = [&](const char* store_fmt_idx, bool tail) {
        for (int c : calls) {
            const Call& k = s.calls[c];
            if (k.op == Op::Scal) {
                e.l(F("const kf_f4 x%d = kf_mul4s(%s, x%d);", k.out, scal_name(k.alpha).c_str(), k.in[0]));
            } else if (k.op == Op::Axpy) {
                e.l(F("const kf_f4 x%d = kf_fma4s(%s, x%d, x%d);", k.out, scal_name(k.alpha).c_str(), k.in[0], k.in[1]));
            } else if (k.op == Op::Dot) {
                e.l(F("dacc%d = kf_dot4(x%d, x%d, dacc%d);", c, k.in[0], k.in[1], c));
            }
            if (k.op != Op::Dot && must_store(s, part, kid, k.out)) {
                if (!tail) e.l(F("kf_st4_nt(Y%d + 4 * %s, x%d);", k.out, store_fmt_idx, k.out));
                else e.l(F("Y%d[%s] = x%d.x;", k.out, store_fmt_idx, k.out));
            }
        }
    };
    auto emit_body = [&](bool guard) {
        for (int v : vec_in) e.l(F("kf_f4 in%d[U];", v));
        e.l("#pragma unroll");
        e.l("for (int u = 0; u < U; ++u) {");
        e.ind++;
        e.l("const long i4 = b + (long)u * NT + tid;");
        if (guard) e.l("if (i4 < N4) {");
        for (int v : vec_in) e.l(F("  in%d[u] = kf_ld4_nt(V%d + 4 * i4);", v, v));
        if (guard) e.l("}");
        e.ind--;
        e.l("}");
        e.l("#pragma unroll");
        e.l("for (int u = 0; u < U; ++u) {");
        e.ind++;
        e.l("const long i4 = b + (long)u * NT + tid;");
        if (guard) {
            e.l("if (i4 < N4) {");
            e.ind++;
        }
        for (int v : vec_in) e.l(F("const kf_f4 x%d = in%d[u];", v, v));
        emit_compute("i4", false);
        if (guard) {
            e.ind--;
            e.l("}");
        }
        e.ind--;
        e.l("}");
    };
    e.l("for (long b = (long)blockIdx.x * STEP; b < N4; b += (long)GRID * STEP) {");
    e.ind++;
    e.l("if (b + STEP <= N4) {");
    e.ind++;
    emit_body(false);
    e.ind--;
    e.l("} else {");
    e.ind++;
    emit_body(true);
    e.ind--;
    e.l("}");
    e.ind--;
    e.l("}");
    if (T) {
        e.l("if (blockIdx.x == 0 && tid < T) {");
        e.ind++;
        e.l("const long ix = 4 * N4 + tid;");
        for (int v : vec_in) e.l(F("kf_f4 x%d = kf_zero4(); x%d.x = V%d[ix];", v, v, v));
        emit_compute("ix", true);
        e.ind--;
        e.l("}");
    }
    // dot products: workgroup sums; the finishing launch adds them
    for (int i = 0; i < ndot; ++i) {
        int c = dots[i];
        const Call& k = s.calls[c];
        e.l(F("const float bs%d = kf_block_sum_cs<NW>(kf_cs_init(dacc%d), kf_lds);", c, c));
        if (!dot_part) {
            if (must_store(s, part, kid, k.out)) e.l(F("if (tid == 0) *Y%d = bs%d;", k.out, c));
        } else {
            e.l(F("if (tid == 0) ws[%dL * GRID + blockIdx.x] = bs%d;", i, c));
        }
    }
    Emitter f;
    Launch finl;
    std::vector<std::string> fsig;
    if (dot_part) {
        for (int v : dot_out) { finl.args.push_back({ArgKind::DevScalarOut, v}); fsig.push_back(F("float* __restrict__ Y%d", v)); }
        finl.args.push_back({ArgKind::Workspace, -1});
        fsig.push_back("const float* __restrict__ ws");
        // FT threads; thread t adds partials t, t + FT, ... in increasing order,
        // loading FU of them ahead of the dependent adds; the (sum, error)
        // pairs of the threads are then merged through the wave butterfly and
        // the waves in wave order, so the whole cross-workgroup sum is
        // compensated
        const int FT = GRID >= 4096 ? 1024 : 256, FU = 8;
        f.l(F("constexpr int GRID = %d, FT = %d, FU = %d;", GRID, FT, FU));
        f.l("__shared__ float kf_lds[2 * (FT / 64)];");
        f.l("const int tid = threadIdx.x;");
        for (int i = 0; i < ndot; ++i) {
            int c = dots[i];
            const Call& k = s.calls[c];
            f.l("{");
            f.ind++;
            f.l("kf_cs acc = kf_cs_init(0.f);");
            f.l("for (int g0 = tid; g0 < GRID; g0 += FT * FU) {");
            f.ind++;
            f.l("float yv[FU];");
            f.l("#pragma unroll");
            f.l(F("for (int u = 0; u < FU; ++u) yv[u] = g0 + u * FT < GRID ? ws[%dL * GRID + g0 + u * FT] : 0.f;", i));
            f.l("#pragma unroll");
            f.l("for (int u = 0; u < FU; ++u) acc = kf_cs_add(acc, yv[u]);");
            f.ind--;
            f.l("}");
            f.l("const float tot = kf_block_sum_cs<FT / 64>(acc, kf_lds);");
            if (must_store(s, part, kid, k.out)) f.l(F("if (tid == 0) *Y%d = tot;", k.out));
            else f.l("(void)tot;");
            f.ind--;
            f.l("}");
        }
        finl.grid = 1;
        finl.block = FT;
    }

    std::string sigs, fsigs;
    for (size_t i = 0; i < sig.size(); ++i) sigs += (i ? ",\n    " : "    ") + sig[i];
    for (size_t i = 0; i < fsig.size(); ++i) fsigs += (i ? ",\n    " : "    ") + fsig[i];
    std::string body = e.o.str();
    std::string key = F("vec U%d NT%d G%d N%ld|", U, NT, GRID, N) + sigs + body + fsigs + f.o.str();
    kc.name = F("kf_vec_%016llx", (unsigned long long)fnv1a(key));
    std::ostringstream src;
    src << "extern \"C\" __global__ void __launch_bounds__(" << NT << ") " << kc.name << "(\n"
        << sigs << ") {\n" << body << "}\n";
    mainl.name = kc.name;
    mainl.grid = GRID;
    mainl.block = NT;
    kc.launches.push_back(mainl);
    if (dot_part) {
        finl.name = kc.name + "_fin";
        src << "extern \"C\" __global__ void __launch_bounds__(" << finl.block << ") " << finl.name << "(\n"
            << fsigs << ") {\n" << f.o.str() << "}\n";
        kc.launches.push_back(finl);
    }
    kc.source = src.str();
    kc.lds_bytes = 16 + (size_t)NW * 8;
    kc.params_json = F("{\"unroll\": %d, \"threads\": %d, \"grid\": %d}", U, NT, GRID);
    kernel_bytes(s, calls, part, &kc.bytes_read, &kc.bytes_written);
    return kc;
}

// ============================================================================
// BLAS-2 kernels, row-resident schedule
// ============================================================================
// One workgroup owns R whole rows; its W waves split the columns (each wave a
// segment of CW = 256 kp columns, kp float4 per lane). A row dot is finished
// inside the workgroup -- a transposing cross-lane reduction per wave, then the
// W wave partials added in wave order after one barrier per group of G rows --
// so its result can feed, in the same pass over the row held in registers,
// the column accumulation of a gemtv: A^T (A x) reads A once. This is the row
// reuse the paper reports as impossible without a global barrier (Section
// 5.2); here the barrier is local because the row never leaves the workgroup.
bool needs_rowres(const Script& s, const std::vector<int>& calls) {
    for (int c : calls) {
        const Call& k = s.calls[c];
        if (k.op != Op::Gemtv) continue;
        int p = s.values[k.in[1]].producer;
        if (p >= 0 && std::find(calls.begin(), calls.end(), p) != calls.end()) return true;
    }
    return false;
}

RowresGeom rowres_geometry(int64_t rows, int64_t cols, const MatParams& p) {
    RowresGeom g;
    // enough waves to cover the row 256 columns each (at most 16); G rows per
    // group: two once a lane holds four or more float4 of a row (measured best
    // at 16384 columns), else up to four within the register budget
    g.W = p.waves > 0 ? p.waves : (int)std::min<int64_t>(16, std::max<int64_t>(1, (cols + 255) / 256));
    g.WP = 1;
    while (g.WP < g.W) g.WP *= 2;
    g.KP = (int)((cols + 256L * g.W - 1) / (256L * g.W));
    g.G = p.group > 0 ? p.group : std::max(1, std::min(g.KP >= 4 ? 2 : 4, 16 / g.KP));
    g.R = p.rows;
    if (g.R <= 0) {
        g.R = (rows + 255) / 256;
        g.R = (g.R + g.G - 1) / g.G * g.G;
        if (g.R < g.G) g.R = g.G;
    }
    return g;
}

// Register budget of a row-resident kernel, in VGPRs per lane, for the values
// that stay live through a row group: the group's rows that a gemv or gemtv
// reads (G kp float4 per matrix), the column vectors held in registers and the
// gemtv accumulators (kp float4 each). Workgroups of 16 waves leave 128 VGPRs per
// lane; the margin is for addresses, row partials and temporaries.
static constexpr int kRowresBudgetHeld = 64;   // a gemv and a gemtv: rows held through the group's barrier
static constexpr int kRowresBudget = 96;       // the others
static int rowres_pressure(int KP, int G, size_t nmat, size_t ncv_reg, size_t nacc) {
    return 4 * KP * (G * (int)nmat + (int)ncv_reg + (int)nacc);
}

static KernelCode gen_mat_rowres(const Script& s, const std::vector<int>& calls,
                                 const std::vector<int>& part, const MatParams& p0) {
    KernelCode kc;
    kc.mat = true;
    kc.calls = calls;
    const int kid = part[calls[0]];
    const Space sp = call_space(s, calls[0]);
    const long M = (long)sp.a, N = (long)sp.b;

    std::vector<int> mat_in, mat_out, colv, rowv, vec_in, vec_out, gemv_calls, gemtv_calls, scalars;
    auto push_u = [](std::vector<int>& v, int x) {
        if (std::find(v.begin(), v.end(), x) == v.end()) v.push_back(x);
    };
    for (int c : calls) {
        const Call& k = s.calls[c];
        if (!produced_in(s, part, kid, k.in[0])) push_u(mat_in, k.in[0]);
        if (k.op == Op::Ger) {
            push_u(rowv, k.in[1]);
            push_u(colv, k.in[2]);
            if (must_store(s, part, kid, k.out)) push_u(mat_out, k.out);
        } else if (k.op == Op::Gemv) {
            push_u(colv, k.in[1]);
            gemv_calls.push_back(c);
            if (k.in[2] >= 0 && !produced_in(s, part, kid, k.in[2])) push_u(rowv, k.in[2]);
            if (must_store(s, part, kid, k.out)) push_u(vec_out, k.out);
        } else {
            if (!produced_in(s, part, kid, k.in[1])) push_u(rowv, k.in[1]);
            gemtv_calls.push_back(c);
            if (k.in[2] >= 0 && !produced_in(s, part, kid, k.in[2])) push_u(vec_in, k.in[2]);
            if (must_store(s, part, kid, k.out)) push_u(vec_out, k.out);
        }
    }
    for (int v : colv) push_u(vec_in, v);
    for (int v : rowv) push_u(vec_in, v);

    RowresGeom geo = rowres_geometry(M, N, p0);
    const long CW = 256L * geo.KP;
    // Column-indexed vectors live in registers, KP float4 per lane each, or,
    // in kernels that also hold gemtv accumulators in registers, in LDS when
    // all of them fit 128 KiB (one copy per workgroup, zero past N), read at
    // each use: that keeps the loads of a row group in registers without
    // spills. (Column-major GEMVER's three vectors stay in registers: with two
    // of them staged it measured 2% slower.)
    const size_t vec_lds = (size_t)geo.W * CW * 4;   // bytes of one staged vector
    std::vector<int> colv_lds, colv_glob;
    if (!gemtv_calls.empty() && colv.size() * vec_lds <= 128 * 1024) colv_lds = colv;
    // Wider rows (more float4 per lane) or more operands than the registers
    // hold would spill to scratch memory, private to each lane and re-read
    // every group. Over the budget, G is halved first; then column vectors
    // are staged in LDS while they fit 128 KiB, and the rest are loaded from
    // global memory at each use (every workgroup reads the same vector: L2
    // hits). A kernel with both a gemv and a gemtv holds its rows through the
    // group's barrier, so its budget is lower.
    // Only a geometry the library picks itself is adjusted; requested
    // parameters are generated as asked.
    const bool auto_geo = p0.waves <= 0 && p0.group <= 0 && p0.rows <= 0;
    // rows a group holds: the matrices (loaded or made by ger) that a gemv or
    // a gemtv reads, and one more array while ger results are formed from
    // their loaded inputs
    std::vector<int> held;
    bool has_ger = false;
    for (int c : calls) {
        if (s.calls[c].op != Op::Ger) push_u(held, s.calls[c].in[0]);
        else has_ger = true;
    }
    const size_t nheld = std::max<size_t>(1, held.size() + (has_ger ? 1 : 0));
    auto ncv_reg = [&]() { return colv.size() - colv_lds.size() - colv_glob.size(); };
    auto pressure = [&]() { return rowres_pressure(geo.KP, geo.G, nheld, ncv_reg(), gemtv_calls.size()); };
    const int budget = !gemv_calls.empty() && !gemtv_calls.empty() ? kRowresBudgetHeld : kRowresBudget;
    if (auto_geo && pressure() > budget) {
        while (geo.G > 1 && pressure() > budget) {
            MatParams q = p0;
            q.group = geo.G / 2;
            geo = rowres_geometry(M, N, q);
        }
        for (int v : colv) {
            if (pressure() <= budget) break;
            if (std::find(colv_lds.begin(), colv_lds.end(), v) != colv_lds.end()) continue;
            if ((colv_lds.size() + 1) * vec_lds <= 128 * 1024) colv_lds.push_back(v);
            else colv_glob.push_back(v);
        }
    }
    const int W = geo.W, WP = geo.WP, KP = geo.KP, G = geo.G;
    int LG = 0;
    while ((1 << LG) < G) ++LG;
    const int NT = 64 * W;
    const long R = geo.R;
    const long NB = (M + R - 1) / R;
    const long NP = (N + 3) / 4 * 4;
    const bool edge_cols = (long)W * CW > N;
    // a row group's elements lie within 2^30 floats of its first row: 32-bit offsets
    long ld_max = 0;
    for (int c : calls) {
        const Call& k = s.calls[c];
        ld_max = std::max<long>(ld_max, (long)s.values[k.in[0]].ld);
        if (k.op == Op::Ger) ld_max = std::max<long>(ld_max, (long)s.values[k.out].ld);
    }
    const bool off32 = (long)G * ld_max + N < (1L << 30);
    auto cvx = [&](int v) {
        if (std::find(colv_lds.begin(), colv_lds.end(), v) != colv_lds.end()) return F("xs%d[(cb >> 2) + 64u * j]", v);
        if (std::find(colv_glob.begin(), colv_glob.end(), v) != colv_glob.end())
            return F("kf_ld4_tail(V%d, (long)(cbg + 256u * j), N)", v);
        return F("cv%d[j]", v);
    };
    const bool col_part = !gemtv_calls.empty() && NB > 1;
    std::map<int, size_t> ws_off;
    size_t wsz = 0;
    if (col_part)
        for (int c : gemtv_calls) { ws_off[c] = wsz; wsz += (size_t)NB * NP; }
    kc.ws_floats = wsz;

    std::vector<int> main_out;
    for (int v : vec_out) {
        Op op = s.calls[s.values[v].producer].op;
        if (!(op == Op::Gemtv && col_part)) main_out.push_back(v);
    }
    std::vector<std::string> sig;
    Launch mainl;
    for (int v : mat_in) { mainl.args.push_back({ArgKind::MatIn, v}); sig.push_back(F("const float* __restrict__ M%d", v)); }
    for (int v : mat_out) { mainl.args.push_back({ArgKind::MatOut, v}); sig.push_back(F("float* __restrict__ O%d", v)); }
    for (int v : vec_in) { mainl.args.push_back({ArgKind::VecIn, v}); sig.push_back(F("const float* __restrict__ V%d", v)); }
    for (int v : main_out) { mainl.args.push_back({ArgKind::VecOut, v}); sig.push_back(F("float* __restrict__ Y%d", v)); }
    std::vector<KArg> sargs;
    for (int c : calls) {
        add_scalar_args(s, s.calls[c].alpha, &sargs, &scalars);
        if (s.calls[c].in[2] >= 0 && s.calls[c].op != Op::Ger) add_scalar_args(s, s.calls[c].beta, &sargs, &scalars);
    }
    for (auto& a : sargs) {
        mainl.args.push_back(a);
        sig.push_back(a.kind == ArgKind::ConstScalar ? F("float P%d", a.value) : F("const float* __restrict__ P%d", a.value));
    }
    mainl.args.push_back({ArgKind::Workspace, -1});
    sig.push_back("float* __restrict__ ws");

    Emitter e;
    e.l(F("constexpr long M = %ldL, N = %ldL, NB = %ldL, NP = %ldL, CW = %ldL, R = %ldL;", M, N, NB, NP, CW, R));
    e.l(F("constexpr int KP = %d, W = %d, WP = %d, G = %d, LG = %d, NT = %d;", KP, W, WP, G, LG, NT));
    for (int v : mat_in) e.l(F("constexpr long LD%d = %ldL;", v, (long)s.values[v].ld));
    for (int v : mat_out) e.l(F("constexpr long LD%d = %ldL;", v, (long)s.values[v].ld));
    e.l("const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;");
    e.l("const long rb = blockIdx.x, r0 = rb * R, r1 = (r0 + R < M) ? r0 + R : M;");
    e.l("(void)ws;");
    for (int v : scalars)
        e.l(s.values[v].kind == VK::Const ? F("const float %s = P%d;", scal_name(v).c_str(), v)
                                          : F("const float %s = *P%d;", scal_name(v).c_str(), v));
    // column of lane's float4 j: cb + 256 j (32-bit: rows are at most 32768 columns)
    e.l("const unsigned cb = (unsigned)(wave * CW + lane * 4);");
    for (int v : colv) {
        if (std::find(colv_glob.begin(), colv_glob.end(), v) != colv_glob.end()) continue;
        if (std::find(colv_lds.begin(), colv_lds.end(), v) != colv_lds.end()) {
            e.l(F("__shared__ kf_f4 xs%d[W * KP * 64];", v));
            e.l(F("for (int i = tid; i < W * KP * 64; i += NT) xs%d[i] = kf_ld4_tail(V%d, 4L * i, N);", v, v));
        } else {
            e.l(F("kf_f4 cv%d[KP];", v));
            e.l(F("for (int j = 0; j < KP; ++j) cv%d[j] = kf_ld4_tail(V%d, (long)(cb + 256u * j), N);", v, v));
        }
    }
    for (int v : rowv) {
        e.l(F("__shared__ float rv%d[R];", v));
        e.l(F("for (long i = tid; i < R; i += NT) rv%d[i] = (r0 + i < M) ? V%d[r0 + i] : 0.f;", v, v));
    }
    const int ngv = (int)gemv_calls.size();
    if (ngv) e.l(F("__shared__ float kf_part[2][%d][G][WP];", ngv));
    for (int c : gemtv_calls) {
        e.l(F("kf_f4 acc%d[KP];", c));
        e.l(F("for (int j = 0; j < KP; ++j) acc%d[j] = kf_zero4();", c));
    }
    e.l("__syncthreads();");
    e.l("int slot = 0;");
    auto mexpr = [&](int v) { return produced_in(s, part, kid, v) ? F("m%d[gi]", v) : F("L%d[gi]", v); };
    auto emit_group = [&](bool edge) {
        for (int v : mat_in) e.l(F("kf_f4 L%d[G][KP];", v));
        e.l("for (int gi = 0; gi < G; ++gi) {");
        e.ind++;
        e.l("const long row = g0 + gi;");
        for (int v : mat_in) {
            if (!edge && off32) e.l(F("for (int j = 0; j < KP; ++j) L%d[gi][j] = kf_ld4_nt_at(M%d + g0 * LD%d, (unsigned)gi * (unsigned)LD%d + cb + 256u * j);", v, v, v, v));
            else if (!edge) e.l(F("for (int j = 0; j < KP; ++j) L%d[gi][j] = kf_ld4_nt(M%d + row * LD%d + (long)(cb + 256u * j));", v, v, v));
            else e.l(F("for (int j = 0; j < KP; ++j) L%d[gi][j] = (row < r1) ? kf_ldm_edge(M%d + row * LD%d, (long)(cb + 256u * j), N) : kf_zero4();", v, v, v));
        }
        e.ind--;
        e.l("}");
        for (int c : gemv_calls) e.l(F("float rp%d[G];", c));
        for (int c : calls)
            if (s.calls[c].op == Op::Ger) e.l(F("kf_f4 m%d[G][KP];", s.calls[c].out));
        // maps and row dots
        e.l("for (int gi = 0; gi < G; ++gi) {");
        e.ind++;
        e.l("const long row = g0 + gi; const int rl = (int)(row - r0); (void)rl;");
        for (int c : calls) {
            const Call& k = s.calls[c];
            std::string Min = mexpr(k.in[0]);
            if (k.op == Op::Ger) {
                e.l(F("const float cu%d = %s * rv%d[rl];", c, scal_name(k.alpha).c_str(), k.in[1]));
                e.l(F("for (int j = 0; j < KP; ++j) m%d[gi][j] = kf_fma4s(cu%d, %s, %s[j]);", k.out, c, cvx(k.in[2]).c_str(), Min.c_str()));
                if (must_store(s, part, kid, k.out)) {
                    if (!edge && off32) e.l(F("for (int j = 0; j < KP; ++j) kf_st4_nt_at(O%d + g0 * LD%d, (unsigned)gi * (unsigned)LD%d + cb + 256u * j, m%d[gi][j]);", k.out, k.out, k.out, k.out));
                    else if (!edge) e.l(F("for (int j = 0; j < KP; ++j) kf_st4_nt(O%d + row * LD%d + (long)(cb + 256u * j), m%d[gi][j]);", k.out, k.out, k.out));
                    else e.l(F("if (row < r1) for (int j = 0; j < KP; ++j) kf_stm_edge(O%d + row * LD%d, (long)(cb + 256u * j), N, m%d[gi][j]);", k.out, k.out, k.out));
                }
            } else if (k.op == Op::Gemv) {
                e.l(F("float t%d = 0.f;", c));
                e.l(F("for (int j = 0; j < KP; ++j) t%d = kf_dot4(%s[j], %s, t%d);", c, Min.c_str(), cvx(k.in[1]).c_str(), c));
                e.l(F("rp%d[gi] = t%d;", c, c));
            }
        }
        e.ind--;
        e.l("}");
        // finish the row dots inside the workgroup
        for (int i = 0; i < ngv; ++i) {
            int c = gemv_calls[i];
            e.l(F("{ const float sw = kf_rows_reduce<LG>(rp%d); if ((lane & ((64 >> LG) - 1)) == 0) kf_part[slot][%d][lane >> (6 - LG)][wave] = sw; }", c, i));
        }
        if (ngv) e.l("__syncthreads();");
        // lane l < G WP takes the partial of wave l % WP for row l / WP (zero
        // for l % WP >= W; WP is W rounded up to a power of two); a TwoSum
        // butterfly over each group of WP lanes merges them, in the same fixed
        // order for every row, and lane gi WP then holds row gi's sum
        for (int i = 0; i < ngv; ++i) {
            int c = gemv_calls[i];
            e.l(F("const float fl%d = kf_cs_value(kf_group_sum_cs<WP>(kf_cs_init((lane < G * WP && (lane & (WP - 1)) < W) ? (&kf_part[slot][%d][0][0])[lane] : 0.f)));", c, i));
        }
        // per row: gemv epilogues, gemtv accumulation (script order)
        e.l("for (int gi = 0; gi < G; ++gi) {");
        e.ind++;
        e.l("const long row = g0 + gi; const int rl = (int)(row - r0); (void)rl;");
        for (int i = 0; i < ngv; ++i) {
            int c = gemv_calls[i];
            e.l(F("const float sum%d = kf_lane_bcast(fl%d, gi * WP);", c, c));
        }
        for (int c : calls) {
            const Call& k = s.calls[c];
            std::string Min = mexpr(k.in[0]);
            if (k.op == Op::Gemv) {
                std::string val = F("%s * sum%d", scal_name(k.alpha).c_str(), c);
                if (k.in[2] >= 0) {
                    std::string y0 = produced_in(s, part, kid, k.in[2]) ? F("f%d", s.values[k.in[2]].producer)
                                                                         : F("rv%d[rl]", k.in[2]);
                    val = F("__builtin_fmaf(%s, %s, %s)", scal_name(k.beta).c_str(), y0.c_str(), val.c_str());
                }
                e.l(F("const float f%d = %s;", c, val.c_str()));
                if (must_store(s, part, kid, k.out))
                    e.l(edge ? F("if (tid == 0 && row < r1) Y%d[row] = f%d;", k.out, c) : F("if (tid == 0) Y%d[row] = f%d;", k.out, c));
                else e.l(F("(void)f%d;", c));
            } else if (k.op == Op::Gemtv) {
                std::string xr = produced_in(s, part, kid, k.in[1]) ? F("f%d", s.values[k.in[1]].producer)
                                                                     : F("rv%d[rl]", k.in[1]);
                if (edge && produced_in(s, part, kid, k.in[1])) xr = "((row < r1) ? " + xr + " : 0.f)";
                e.l(F("for (int j = 0; j < KP; ++j) acc%d[j] = kf_fma4s(%s, %s[j], acc%d[j]);", c, xr.c_str(), Min.c_str(), c));
            }
        }
        e.ind--;
        e.l("}");
        e.l("slot ^= 1;");
    };
    e.l("for (long g0 = r0; g0 < r1; g0 += G) {");
    e.ind++;
    // column vectors read from global memory: an offset the compiler cannot
    // prove constant across groups, so that it does not hoist their loads out
    // of the loop into registers (the spill this placement avoids)
    if (!colv_glob.empty()) e.l("unsigned cbg = cb; asm volatile(\"\" : \"+v\"(cbg));");
    e.l(edge_cols ? "if (false) {" : "if (g0 + G <= r1) {");
    e.ind++;
    emit_group(false);
    e.ind--;
    e.l("} else {");
    e.ind++;
    emit_group(true);
    e.ind--;
    e.l("}");
    e.ind--;
    e.l("}");
    // column results: each wave owns its columns (all gemtv calls in one loop so
    // that a chained y0 is at hand)
    if (!gemtv_calls.empty()) {
        e.l("for (int j = 0; j < KP; ++j) {");
        e.ind++;
        e.l("const long cc = (long)(cb + 256u * j);");
        e.l("if (cc < N) {");
        e.ind++;
        for (int c : gemtv_calls) {
            const Call& k = s.calls[c];
            if (!col_part) {
                std::string val = F("kf_mul4s(%s, acc%d[j])", scal_name(k.alpha).c_str(), c);
                if (k.in[2] >= 0) {
                    std::string y0 = produced_in(s, part, kid, k.in[2]) ? F("g%d", s.values[k.in[2]].producer)
                                                                         : F("kf_ld4_tail(V%d, cc, N)", k.in[2]);
                    val = F("kf_fma4s(%s, %s, %s)", scal_name(k.beta).c_str(), y0.c_str(), val.c_str());
                }
                e.l(F("const kf_f4 g%d = %s;", c, val.c_str()));
                if (must_store(s, part, kid, k.out)) e.l(F("kf_st4_tail(Y%d, cc, N, g%d);", k.out, c));
                else e.l(F("(void)g%d;", c));
            } else {
                e.l(F("kf_st4(ws + %zuL + rb * NP + cc, acc%d[j]);", ws_off[c], c));
            }
        }
        e.ind--;
        e.l("}");
        e.ind--;
        e.l("}");
    }

    // finishing launch (column partials), as in the strip schedule
    Emitter f;
    Launch finl;
    std::vector<std::string> fsig;
    if (col_part) {
        std::vector<int> fin_in, fin_out;
        for (int c : gemtv_calls) {
            const Call& k = s.calls[c];
            if (k.in[2] >= 0 && !produced_in(s, part, kid, k.in[2])) push_u(fin_in, k.in[2]);
            if (must_store(s, part, kid, k.out)) fin_out.push_back(k.out);
        }
        for (int v : fin_in) { finl.args.push_back({ArgKind::VecIn, v}); fsig.push_back(F("const float* __restrict__ V%d", v)); }
        for (int v : fin_out) { finl.args.push_back({ArgKind::VecOut, v}); fsig.push_back(F("float* __restrict__ Y%d", v)); }
        for (auto& a : sargs) {
            finl.args.push_back(a);
            fsig.push_back(a.kind == ArgKind::ConstScalar ? F("float P%d", a.value) : F("const float* __restrict__ P%d", a.value));
        }
        finl.args.push_back({ArgKind::Workspace, -1});
        fsig.push_back("const float* __restrict__ ws");
        f.l(F("constexpr long N = %ldL, NB = %ldL, NP = %ldL;", N, NB, NP));
        for (int v : scalars)
            f.l(s.values[v].kind == VK::Const ? F("const float %s = P%d;", scal_name(v).c_str(), v)
                                              : F("const float %s = *P%d;", scal_name(v).c_str(), v));
        const int FW = NB >= 64 ? 16 : 4;   // waves that split the row blocks
        f.l(F("constexpr int FW = %d;", FW));
        f.l("const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;");
        f.l("const long cc = 4L * ((long)blockIdx.x * 64 + lane);");
        emit_colpart_finish(f, gemtv_calls, ws_off);
        f.l("if (wave == 0 && cc < N) {");
        f.ind++;
        for (size_t i = 0; i < gemtv_calls.size(); ++i) {
            int c = gemtv_calls[i];
            const Call& k = s.calls[c];
            std::string val = F("kf_mul4s(%s, sum%d)", scal_name(k.alpha).c_str(), c);
            if (k.in[2] >= 0) {
                std::string y0 = produced_in(s, part, kid, k.in[2]) ? F("f%d", s.values[k.in[2]].producer)
                                                                     : F("kf_ld4_tail(V%d, cc, N)", k.in[2]);
                val = F("kf_fma4s(%s, %s, %s)", scal_name(k.beta).c_str(), y0.c_str(), val.c_str());
            }
            f.l(F("const kf_f4 f%d = %s;", c, val.c_str()));
            if (must_store(s, part, kid, k.out)) f.l(F("kf_st4_tail(Y%d, cc, N, f%d);", k.out, c));
            else f.l(F("(void)f%d;", c));
        }
        f.ind--;
        f.l("}");
        finl.grid = (int)((NP / 4 + 63) / 64);
        finl.block = 64 * FW;
    }
    std::string sigs, fsigs;
    for (size_t i = 0; i < sig.size(); ++i) sigs += (i ? ",\n    " : "    ") + sig[i];
    for (size_t i = 0; i < fsig.size(); ++i) fsigs += (i ? ",\n    " : "    ") + fsig[i];
    std::string key = F("rowres W%d G%d R%ld M%ld N%ld|", W, G, R, M, N) + sigs + e.o.str() + fsigs + f.o.str();
    kc.name = F("kf_row_%016llx", (unsigned long long)fnv1a(key));
    std::ostringstream head;
    head << "extern \"C\" __global__ void __launch_bounds__(" << NT << ") " << kc.name << "(\n" << sigs << ") {\n"
         << e.o.str() << "}\n";
    mainl.name = kc.name;
    mainl.grid = (int)NB;
    mainl.block = NT;
    kc.launches.push_back(mainl);
    if (col_part) {
        finl.name = kc.name + "_fin";
        head << "extern \"C\" __global__ void __launch_bounds__(" << finl.block << ") " << finl.name << "(\n" << fsigs
             << ") {\n" << f.o.str() << "}\n";
        kc.launches.push_back(finl);
    }
    kc.source = head.str();
    kc.lds_bytes = 16 + rowv.size() * (size_t)R * 4 + (size_t)ngv * 2 * G * WP * 4 + colv_lds.size() * (size_t)W * CW * 4;
    // vectors loaded from global memory count too: the loads of a group are
    // all in flight together
    kc.reg_estimate = rowres_pressure(KP, G, nheld, ncv_reg() + colv_glob.size(), gemtv_calls.size());
    kc.over_budget = kc.reg_estimate > budget;
    kc.params_json = F("{\"schedule\": \"row-resident\", \"waves\": %d, \"group\": %d, \"rows\": %ld, \"kp\": %d, \"row_blocks\": %ld, "
                       "\"register_estimate\": %d, \"over_register_budget\": %s}",
                       W, G, R, KP, NB, kc.reg_estimate, kc.over_budget ? "true" : "false");
    kernel_bytes(s, calls, part, &kc.bytes_read, &kc.bytes_written);
    return kc;
}

// Operand bytes one launch moves through HBM (workspace partials excluded).
static void launch_bytes(const Script& s, Launch* l) {
    l->bytes_read = l->bytes_written = 0;
    for (const KArg& a : l->args) {
        if (a.value < 0) continue;
        const Value& x = s.values[a.value];
        uint64_t b = x.kind == VK::Vec ? (uint64_t)x.n * 4
                   : x.kind == VK::Mat ? (uint64_t)x.rows * (uint64_t)x.cols * (uint64_t)dtype_size(x.dtype)
                   : x.kind == VK::DevScalar ? 4 : 0;
        switch (a.kind) {
            case ArgKind::MatIn: case ArgKind::VecIn: case ArgKind::DevScalarIn: l->bytes_read += b; break;
            case ArgKind::MatOut: case ArgKind::VecOut: case ArgKind::DevScalarOut: l->bytes_written += b; break;
            default: break;
        }
    }
}

KernelCode generate_kernel(const Script& s, const std::vector<int>& calls,
                           const std::vector<int>& part, const MatParams& mp,
                           const VecParams& vp) {
    Space sp = call_space(s, calls[0]);
    KernelCode kc;
    if (sp.mat && (mp.sched == 1 || needs_rowres(s, calls))) {
        MatParams q = mp;
        if (q.sched != 1) q.waves = q.group = q.rows = 0;   // strip-schedule parameters do not carry over
        kc = gen_mat_rowres(s, calls, part, q);
    } else {
        if (sp.mat) {
            MatParams q = default_mat_params(sp.a, sp.b, mp, kernel_unit_elems(s, calls, mp.unit));
            q.dyn = mp.dyn;
            kc = gen_mat(s, calls, part, q);
        } else {
            kc = gen_vec(s, calls, part, default_vec_params(sp.a, vp));
        }
    }
    for (Launch& l : kc.launches) launch_bytes(s, &l);
    return kc;
}

}  // namespace kf

namespace kf {

// ============================================================================
// Routine probes: one routine alone, in the workgroup geometry and serial
// iterations of a real kernel (Section 4.2: routine times are benchmarked in a
// simulated fusion environment and summed to predict a fusion).
// ============================================================================
// Extra LDS of a probe's environment: an array the workgroup holds (and
// touches, so that it is allocated) for the whole launch.
static void probe_extra_lds(Emitter& e, int extra_kb, int nt) {
    if (extra_kb <= 0) return;
    e.l(F("__shared__ float kf_xlds[%d];", extra_kb * 256));
    e.l(F("for (int i = threadIdx.x; i < %d; i += %d) kf_xlds[i] = 0.f;", extra_kb * 256, nt));
}

// Row-resident probe: a workgroup of W waves owns R whole rows and walks them
// G rows per group, as the row-resident kernels do; a row dot finishes inside
// the workgroup (transposing reduction, LDS, barrier, merge over the waves).
static std::string probe_rowres(Emitter& e, int routine, int64_t rows, int64_t cols, const MatParams& mp,
                                int extra_kb, Launch* l, std::string* params_json) {
    const RowresGeom g = rowres_geometry(rows, cols, mp);
    const long M = (long)rows, N = (long)cols;
    const int W = g.W, WP = g.WP, KP = g.KP, G = g.G, NT = 64 * W;
    int LG = 0;
    while ((1 << LG) < G) ++LG;
    const long R = g.R, NB = (M + R - 1) / R, CW = 256L * KP;
    const bool edge = (long)W * CW > N;
    e.l(F("constexpr long M = %ldL, N = %ldL, R = %ldL, LD = %ldL, CW = %ldL;", M, N, R, N, CW));
    e.l(F("constexpr int KP = %d, W = %d, WP = %d, G = %d, LG = %d, NT = %d;", KP, W, WP, G, LG, NT));
    e.l("const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;");
    e.l("const long r0 = (long)blockIdx.x * R, r1 = (r0 + R < M) ? r0 + R : M;");
    e.l("(void)src; (void)dst;");
    e.l("const unsigned cb = (unsigned)(wave * CW + lane * 4);");
    e.l("kf_f4 cv[KP], acc[KP];");
    e.l("for (int j = 0; j < KP; ++j) { cv[j] = kf_zero4() + (float)(lane + j); acc[j] = kf_zero4(); }");
    e.l("__shared__ kf_f4 tile[8 * KP * 64];");
    e.l("__shared__ float part[2][G][WP];");
    e.l("for (int i = tid; i < 8 * KP * 64; i += NT) tile[i] = kf_zero4() + 1e-3f * (float)i;");
    probe_extra_lds(e, extra_kb, NT);
    e.l("__syncthreads();");
    e.l("float s = 0.f; int slot = 0;");
    e.l("for (long g0 = r0; g0 < r1; g0 += G) {");
    e.ind++;
    // a lane's columns cb + 256 j; with edge columns only those below N are touched
    const std::string ok = edge ? "(long)(cb + 256u * j) + 4 <= N && g0 + gi < r1" : "g0 + gi < r1";
    std::string tag;
    switch (routine) {
        case KF_ROUTINE_LOAD_MAT:
            e.l("kf_f4 L[G][KP];");
            e.l(F("for (int gi = 0; gi < G; ++gi) for (int j = 0; j < KP; ++j) L[gi][j] = (%s) ? kf_ld4_nt_at(src + g0 * LD, (unsigned)gi * (unsigned)LD + cb + 256u * j) : kf_zero4();", ok.c_str()));
            e.l("for (int gi = 0; gi < G; ++gi) for (int j = 0; j < KP; ++j) acc[j] += L[gi][j];");
            tag = "load_mat";
            break;
        case KF_ROUTINE_STORE_MAT:
            e.l(F("for (int gi = 0; gi < G; ++gi) for (int j = 0; j < KP; ++j) if (%s) kf_st4_nt_at(dst + g0 * LD, (unsigned)gi * (unsigned)LD + cb + 256u * j, cv[j]);", ok.c_str()));
            tag = "store_mat";
            break;
        case KF_ROUTINE_COMPUTE_GEMV:
            e.l("float rp[G];");
            e.l("for (int gi = 0; gi < G; ++gi) { float t = 0.f; for (int j = 0; j < KP; ++j) t = kf_dot4(tile[(((g0 + gi) & 7) * KP + j) * 64 + lane], cv[j], t); rp[gi] = t; }");
            e.l("{ const float sw = kf_rows_reduce<LG>(rp); if ((lane & ((64 >> LG) - 1)) == 0) part[slot][lane >> (6 - LG)][wave] = sw; }");
            e.l("__syncthreads();");
            e.l("const float fl = kf_cs_value(kf_group_sum_cs<WP>(kf_cs_init((lane < G * WP && (lane & (WP - 1)) < W) ? (&part[slot][0][0])[lane] : 0.f)));");
            e.l("for (int gi = 0; gi < G; ++gi) s += kf_lane_bcast(fl, gi * WP);");
            e.l("slot ^= 1;");
            tag = "gemv";
            break;
        case KF_ROUTINE_COMPUTE_GEMTV:
            e.l("for (int gi = 0; gi < G; ++gi) { const float xr = 1e-7f * (float)(g0 + gi); for (int j = 0; j < KP; ++j) acc[j] = kf_fma4s(xr, tile[(((g0 + gi) & 7) * KP + j) * 64 + lane], acc[j]); }");
            tag = "gemtv";
            break;
        case KF_ROUTINE_COMPUTE_GER:
            e.l("for (int gi = 0; gi < G; ++gi) { const float cu = 1e-7f * (float)(g0 + gi); for (int j = 0; j < KP; ++j) acc[j] += kf_fma4s(cu, cv[j], tile[(((g0 + gi) & 7) * KP + j) * 64 + lane]); }");
            tag = "ger";
            break;
    }
    e.ind--;
    e.l("}");
    e.l("for (int j = 0; j < KP; ++j) s += (acc[j].x + acc[j].y) + (acc[j].z + acc[j].w);");
    if (extra_kb > 0) e.l(F("s += kf_xlds[tid %% %d];", extra_kb * 256));
    e.l("if (s == 1234.5678f) sink[tid] = s;");
    l->grid = (int)NB;
    l->block = NT;
    *params_json = F("{\"schedule\": \"row-resident\", \"waves\": %d, \"group\": %d, \"rows\": %ld, \"extra_lds_kb\": %d}",
                     W, G, R, extra_kb);
    return F("probe rowres %s W%d G%d R%ld M%ld N%ld X%d", tag.c_str(), W, G, R, M, N, extra_kb);
}

KernelCode generate_probe(int routine, int64_t rows, int64_t cols, const MatParams& mp0,
                          const VecParams& vp0, int extra_kb) {
    KernelCode kc;
    Emitter e;
    std::vector<std::string> sig = {"const float* __restrict__ src", "float* __restrict__ dst",
                                    "float* __restrict__ sink"};
    const bool mat = routine <= KF_ROUTINE_COMPUTE_GER;
    std::string tag;
    if (mat && mp0.sched == 1) {
        Launch l;
        const std::string key = probe_rowres(e, routine, rows, cols, mp0, extra_kb, &l, &kc.params_json) + e.o.str();
        kc.name = F("kf_probe_%016llx", (unsigned long long)fnv1a(key));
        l.name = kc.name;
        kc.launches.push_back(l);
        kc.mat = true;
    } else if (mat) {
        MatParams p = default_mat_params(rows, cols, mp0);
        const long M = (long)rows, N = (long)cols;
        const int K = p.k, W = p.waves, G = p.group, R = p.rows, NT = 64 * W;
        int LG = 0;
        while ((1 << LG) < G) ++LG;
        const long C = 256L * K, S = (N + C - 1) / C, NB = (M + R - 1) / R;
        e.l(F("constexpr long M = %ldL, N = %ldL, C = %ldL, S = %ldL, LD = %ldL;", M, N, C, S, N));
        e.l(F("constexpr int K = %d, W = %d, G = %d, LG = %d, R = %d, NT = %d;", K, W, G, LG, R, NT));
        e.l("const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;");
        e.l("const long sidx = blockIdx.x % S, rb = blockIdx.x / S;");
        e.l("const long c0 = sidx * C, r0 = rb * R, r1 = (r0 + R < M) ? r0 + R : M;");
        e.l("(void)src; (void)dst; (void)sidx;");
        e.l("long col[K]; kf_f4 cv[K]; kf_f4 acc[K];");
        e.l("for (int j = 0; j < K; ++j) { col[j] = c0 + (long)(j * 64 + lane) * 4; cv[j] = kf_zero4() + (float)(lane + j); acc[j] = kf_zero4(); }");
        e.l("__shared__ kf_f4 tile[8 * K * 64];");
        e.l("for (int i = tid; i < 8 * K * 64; i += NT) tile[i] = kf_zero4() + 1e-3f * (float)i;");
        probe_extra_lds(e, extra_kb, NT);
        e.l("__syncthreads();");
        e.l("float s = 0.f;");
        e.l("for (long g0 = r0 + (long)wave * G; g0 < r1; g0 += (long)W * G) {");
        e.ind++;
        switch (routine) {
            case KF_ROUTINE_LOAD_MAT:
                e.l("kf_f4 L[G][K];");
                e.l("for (int gi = 0; gi < G; ++gi) for (int j = 0; j < K; ++j) L[gi][j] = kf_ld4_nt(src + (g0 + gi) * LD + col[j]);");
                e.l("for (int gi = 0; gi < G; ++gi) for (int j = 0; j < K; ++j) acc[j] += L[gi][j];");
                tag = "load_mat";
                break;
            case KF_ROUTINE_STORE_MAT:
                e.l("for (int gi = 0; gi < G; ++gi) for (int j = 0; j < K; ++j) kf_st4_nt(dst + (g0 + gi) * LD + col[j], cv[j]);");
                tag = "store_mat";
                break;
            case KF_ROUTINE_COMPUTE_GEMV:
                e.l("float rp[G];");
                e.l("for (int gi = 0; gi < G; ++gi) { float t = 0.f; for (int j = 0; j < K; ++j) t = kf_dot4(tile[(((g0 + gi) & 7) * K + j) * 64 + lane], cv[j], t); rp[gi] = t; }");
                e.l("s += kf_rows_reduce<LG>(rp);");
                tag = "gemv";
                break;
            case KF_ROUTINE_COMPUTE_GEMTV:
                e.l("for (int gi = 0; gi < G; ++gi) { const float xr = 1e-7f * (float)(g0 + gi); for (int j = 0; j < K; ++j) acc[j] = kf_fma4s(xr, tile[(((g0 + gi) & 7) * K + j) * 64 + lane], acc[j]); }");
                tag = "gemtv";
                break;
            case KF_ROUTINE_COMPUTE_GER:
                e.l("for (int gi = 0; gi < G; ++gi) { const float cu = 1e-7f * (float)(g0 + gi); for (int j = 0; j < K; ++j) acc[j] += kf_fma4s(cu, cv[j], tile[(((g0 + gi) & 7) * K + j) * 64 + lane]); }");
                tag = "ger";
                break;
        }
        e.ind--;
        e.l("}");
        e.l("for (int j = 0; j < K; ++j) s += (acc[j].x + acc[j].y) + (acc[j].z + acc[j].w);");
        if (extra_kb > 0) e.l(F("s += kf_xlds[tid %% %d];", extra_kb * 256));
        e.l("if (s == 1234.5678f) sink[tid] = s;");
        std::string key = F("probe %s K%d W%d G%d R%d M%ld N%ld X%d", tag.c_str(), K, W, G, R, M, N, extra_kb) + e.o.str();
        kc.name = F("kf_probe_%016llx", (unsigned long long)fnv1a(key));
        Launch l;
        l.name = kc.name;
        l.grid = (int)(S * NB);
        l.block = NT;
        kc.launches.push_back(l);
        kc.params_json = F("{\"k\": %d, \"waves\": %d, \"group\": %d, \"rows\": %d, \"extra_lds_kb\": %d}", K, W, G, R,
                           extra_kb);
        kc.mat = true;
    } else {
        VecParams p = default_vec_params(rows, vp0);
        const long N = (long)rows, N4 = N / 4;
        const int U = p.unroll, NT = p.threads, GRID = p.grid;
        e.l(F("constexpr long N4 = %ldL; constexpr int U = %d, NT = %d, GRID = %d;", N4, U, NT, GRID));
        e.l("constexpr long STEP = (long)NT * U;");
        e.l("const int tid = threadIdx.x; (void)src; (void)dst;");
        e.l("kf_f4 acc = kf_zero4(); float d = 0.f; const float a = 1.0001f;");
        e.l("for (long b = (long)blockIdx.x * STEP; b < N4; b += (long)GRID * STEP) {");
        e.ind++;
        e.l("for (int u = 0; u < U; ++u) {");
        e.ind++;
        e.l("const long i4 = b + (long)u * NT + tid;");
        e.l("if (i4 < N4) {");
        e.ind++;
        e.l("const kf_f4 x = kf_zero4() + (float)(i4 & 1023);");
        switch (routine) {
            case KF_ROUTINE_LOAD_VEC: e.l("acc += kf_ld4_nt(src + 4 * i4);"); tag = "load_vec"; break;
            case KF_ROUTINE_STORE_VEC: e.l("kf_st4_nt(dst + 4 * i4, x);"); tag = "store_vec"; break;
            case KF_ROUTINE_COMPUTE_SCAL: e.l("acc += kf_mul4s(a, x);"); tag = "scal"; break;
            case KF_ROUTINE_COMPUTE_AXPY: e.l("acc = kf_fma4s(a, x, acc);"); tag = "axpy"; break;
            case KF_ROUTINE_COMPUTE_DOT: e.l("d = kf_dot4(x, x, d);"); tag = "dot"; break;
        }
        e.ind--;
        e.l("}");
        e.ind--;
        e.l("}");
        e.ind--;
        e.l("}");
        e.l("const float s = ((acc.x + acc.y) + (acc.z + acc.w)) + d;");
        e.l("if (s == 1234.5678f) sink[tid] = s;");
        std::string key = F("probe %s U%d NT%d G%d N%ld", tag.c_str(), U, NT, GRID, N) + e.o.str();
        kc.name = F("kf_probe_%016llx", (unsigned long long)fnv1a(key));
        Launch l;
        l.name = kc.name;
        l.grid = GRID;
        l.block = NT;
        kc.launches.push_back(l);
        kc.params_json = F("{\"unroll\": %d, \"threads\": %d, \"grid\": %d}", U, NT, GRID);
        kc.mat = false;
    }
    std::string sigs;
    for (size_t i = 0; i < sig.size(); ++i) sigs += (i ? ",\n    " : "    ") + sig[i];
    std::ostringstream src;
    src << "extern \"C\" __global__ void __launch_bounds__(" << kc.launches[0].block << ") " << kc.name
        << "(\n" << sigs << ") {\n" << e.o.str() << "}\n";
    kc.source = src.str();
    return kc;
}

// ---- features of one plan kernel (inputs of the learned cost model) --------
static float lg2(double x) { return (float)std::log2(x > 1.0 ? x : 1.0); }

void kernel_features(const Script& s, const KernelCode& kc, const std::vector<int>& part,
                     const MatParams& mp, const VecParams& vp, float* f) {
    for (int i = 0; i < KF_FEATURE_DIM; ++i) f[i] = 0.f;
    const Space sp = call_space(s, kc.calls[0]);
    const int kid = part[kc.calls[0]];
    f[0] = sp.mat ? 1.f : 0.f;
    f[1] = lg2((double)sp.a);
    f[2] = sp.mat ? lg2((double)sp.b) : 0.f;
    f[3] = lg2((double)kc.bytes_read + 1);
    f[4] = lg2((double)kc.bytes_written + 1);
    // bytes the same calls would move as separate kernels
    double alone = 0;
    auto vbytes = [&](int v) -> double {
        const Value& x = s.values[v];
        return x.kind == VK::Vec ? 4.0 * x.n : x.kind == VK::Mat ? (double)dtype_size(x.dtype) * x.rows * x.cols
                                                                 : x.kind == VK::DevScalar ? 4.0 : 0.0;
    };
    int chained = 0;
    for (int c : kc.calls) {
        const Call& k = s.calls[c];
        int ops[5] = {k.alpha, k.beta, k.in[0], k.in[1], k.in[2]};
        for (int v : ops)
            if (v >= 0) alone += vbytes(v);
        if (s.values[k.out].output || !s.values[k.out].consumers.empty()) alone += vbytes(k.out);
        f[6 + (int)k.op] += 1.f;
        if (k.in[2] >= 0 && k.op != Op::Ger && produced_in(s, part, kid, k.in[2])) chained = 1;
    }
    f[5] = lg2(alone - (double)(kc.bytes_read + kc.bytes_written) + 1);
    int mi = 0, mo = 0, vi = 0, vo = 0;
    for (const Launch& l : kc.launches)
        for (const KArg& a : l.args) {
            if (a.kind == ArgKind::MatIn) ++mi;
            else if (a.kind == ArgKind::MatOut) ++mo;
            else if (a.kind == ArgKind::VecIn || a.kind == ArgKind::DevScalarIn) ++vi;
            else if (a.kind == ArgKind::VecOut || a.kind == ArgKind::DevScalarOut) ++vo;
        }
    f[12] = (float)mi;
    f[13] = (float)mo;
    f[14] = (float)vi;
    f[15] = (float)vo;
    if (sp.mat) {
        MatParams p = default_mat_params(sp.a, sp.b, mp);
        f[16] = (float)p.k;
        f[17] = (float)p.waves;
        f[18] = lg2(p.group);
        f[19] = lg2(p.rows);
    } else {
        VecParams p = default_vec_params(sp.a, vp);
        f[20] = (float)p.unroll;
        f[21] = (float)p.threads / 256.f;
        f[22] = lg2(p.grid);
    }
    f[23] = lg2(kc.launches[0].grid);
    f[24] = lg2(kc.launches[0].block);
    f[25] = (float)kc.launches.size();
    f[26] = lg2((double)kc.ws_floats + 1);
    f[27] = (float)kc.lds_bytes / 4096.f;
    f[28] = (float)kc.calls.size();
    f[29] = (float)chained;
    f[30] = lg2(sp.mat ? (double)sp.a * (double)sp.b : (double)sp.a);
    const double tot = (double)(kc.bytes_read + kc.bytes_written);
    f[31] = tot > 0 ? (float)(kc.bytes_written / tot) : 0.f;
}

}  // namespace kf
