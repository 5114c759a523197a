// api.cpp -- the C ABI: script recording, compilation, binding and launch.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <sstream>

#include <sys/stat.h>

#include "kf_internal.h"

namespace kf {

static thread_local std::string g_err = "no error";

kf_status set_error(kf_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
hipError_t launch_stream(int kind, void* dst, const void* src, size_t bytes, hipStream_t st);
hipError_t launch_quantize_rows(const float* A, long rows, long cols, long lda, int fp8, void* codes, long ldq,
                                float* scales, hipStream_t st);
hipError_t launch_fill_uniform(float* dst, long rows, long cols, long ld, unsigned long long key, float pad,
                               hipStream_t st);

// Loaded kernels, by generated name (a hash of the kernel text). Modules stay
// loaded for the life of the process so plans can share kernels.
struct Registry {
    std::mutex mu;
    std::map<std::string, hipFunction_t> funcs;  // launch name -> loaded function
    std::set<std::string> compiled;               // kernel names compiled in this process
    std::vector<hipModule_t> modules;
    std::map<std::string, hipModule_t> by_ident;  // disk-cache file identity -> module
};
static Registry& registry() {
    static Registry* r = new Registry();  // never destroyed: modules outlive static dtors
    return *r;
}

// Make the launches of kc available (registry lock held): reuse loaded
// functions, else a module already loaded from the same cache file, else
// compile or read the code object and load it.
static kf_status ensure_loaded_locked(Registry& reg, const KernelCode& kc) {
    bool have = true;
    for (const Launch& l : kc.launches)
        if (!reg.funcs.count(l.name)) have = false;
    if (have) return KF_OK;
    hipModule_t mod = nullptr;
    const std::string ident = jit_cache_ident(kc);
    auto it = ident.empty() ? reg.by_ident.end() : reg.by_ident.find(ident);
    if (it != reg.by_ident.end()) {
        mod = it->second;
    } else {
        std::string co, log;
        if (!jit_compile_one(kc, &co, &log)) return set_error(KF_ERR_COMPILE, log);
        reg.compiled.insert(kc.name);
        hipError_t e = hipModuleLoadData(&mod, co.data());
        if (e != hipSuccess) return set_error(KF_ERR_HIP, std::string("hipModuleLoadData: ") + hipGetErrorString(e));
        reg.modules.push_back(mod);
        const std::string id2 = ident.empty() ? jit_cache_ident(kc) : ident;
        if (!id2.empty()) reg.by_ident[id2] = mod;
    }
    for (const Launch& l : kc.launches) {
        hipFunction_t fn = nullptr;
        hipError_t e = hipModuleGetFunction(&fn, mod, l.name.c_str());
        if (e != hipSuccess) return set_error(KF_ERR_HIP, std::string("hipModuleGetFunction: ") + hipGetErrorString(e));
        reg.funcs[l.name] = fn;
    }
    return KF_OK;
}

// Compile the kernels of one plan that are not loaded yet with one compiler
// invocation (its fixed cost is most of a small kernel's compile time): into
// the disk cache when one is configured (each kernel is then loaded from its
// entry), else straight into one module. A failure here is not final: the
// kernels are then compiled one by one, which names the failing kernel.
static void load_together_locked(Registry& reg, const std::vector<const KernelCode*>& ks) {
    std::vector<const KernelCode*> todo;
    for (const KernelCode* k : ks) {
        bool have = true;
        for (const Launch& l : k->launches)
            if (!reg.funcs.count(l.name)) have = false;
        bool dup = false;
        for (const KernelCode* t : todo)
            if (t->name == k->name) dup = true;
        if (!have && !dup) todo.push_back(k);
    }
    if (todo.size() < 2) return;
    std::string co, log;
    if (jit_cache_enabled()) {
        (void)jit_precompile(todo, &log);
        return;
    }
    if (!jit_compile_together(todo, &co, &log)) return;
    hipModule_t mod = nullptr;
    if (hipModuleLoadData(&mod, co.data()) != hipSuccess) return;
    reg.modules.push_back(mod);
    for (const KernelCode* k : todo) {
        for (const Launch& l : k->launches) {
            hipFunction_t fn = nullptr;
            if (hipModuleGetFunction(&fn, mod, l.name.c_str()) != hipSuccess) return;
            reg.funcs[l.name] = fn;
        }
        reg.compiled.insert(k->name);
    }
}

// Compile (through the caches) and load one kernel; fills fns with one
// function per launch.
kf_status load_kernel(const KernelCode& kc, std::vector<void*>* fns) {
    Registry& reg = registry();
    std::lock_guard<std::mutex> lock(reg.mu);
    kf_status st = ensure_loaded_locked(reg, kc);
    if (st != KF_OK) return st;
    fns->clear();
    for (const Launch& l : kc.launches) fns->push_back((void*)reg.funcs[l.name]);
    return KF_OK;
}

}  // namespace kf

using namespace kf;

static const char* kVersion = "kfuse 0.1 gfx950";

#define KF_TRY(...)                                                                   \
    try {                                                                             \
        __VA_ARGS__;                                                                  \
    } catch (const std::bad_alloc&) {                                                 \
        return set_error(KF_ERR_NOMEM, "host allocation failed");                     \
    } catch (const std::exception& ex) {                                              \
        return set_error(KF_ERR_INTERNAL, std::string("internal error: ") + ex.what()); \
    } catch (...) {                                                                   \
        return set_error(KF_ERR_INTERNAL, "internal error");                           \
    }

extern "C" {

const char* kf_last_error(void) { return g_err.c_str(); }
const char* kf_version(void) { return kVersion; }

kf_status kf_script_create(kf_script** out) {
    if (!out) return set_error(KF_ERR_ARG, "null out");
    KF_TRY(*out = new kf_script());
    return KF_OK;
}

void kf_script_destroy(kf_script* s) { delete s; }

static bool valid_value(const kf_script* s, kf_value v) {
    return s && v >= 0 && v < (kf_value)s->s.values.size();
}

static kf_status add_value(kf_script* s, const Value& v, kf_value* out) {
    if (!s || !out) return set_error(KF_ERR_ARG, "null argument");
    KF_TRY(s->s.values.push_back(v));
    *out = (kf_value)s->s.values.size() - 1;
    return KF_OK;
}

kf_status kf_vector(kf_script* s, int64_t n, kf_value* out) {
    if (n < 1) return set_error(KF_ERR_SHAPE, "vector length must be >= 1");
    Value v;
    v.kind = VK::Vec;
    v.n = n;
    return add_value(s, v, out);
}

kf_status kf_matrix(kf_script* s, int64_t rows, int64_t cols, int64_t ld, kf_value* out) {
    if (rows < 1 || cols < 1) return set_error(KF_ERR_SHAPE, "matrix dimensions must be >= 1");
    if (ld == 0) ld = (cols + 3) / 4 * 4;
    if (ld < cols) return set_error(KF_ERR_SHAPE, "ld < cols");
    if (ld % 4) return set_error(KF_ERR_ALIGN, "ld must be a multiple of 4 floats");
    Value v;
    v.kind = VK::Mat;
    v.rows = rows;
    v.cols = cols;
    v.ld = ld;
    return add_value(s, v, out);
}

kf_status kf_matrix_layout(kf_script* s, int64_t rows, int64_t cols, int64_t ld, int32_t layout, kf_value* out) {
    if (layout == KF_ROW_MAJOR) return kf_matrix(s, rows, cols, ld, out);
    if (layout != KF_COL_MAJOR) return set_error(KF_ERR_ARG, "layout must be KF_ROW_MAJOR or KF_COL_MAJOR");
    if (rows < 1 || cols < 1) return set_error(KF_ERR_SHAPE, "matrix dimensions must be >= 1");
    if (ld == 0) ld = (rows + 3) / 4 * 4;
    if (ld < rows) return set_error(KF_ERR_SHAPE, "ld < rows (column-major)");
    if (ld % 4) return set_error(KF_ERR_ALIGN, "ld must be a multiple of 4 floats");
    // column j of the declared matrix is row j of its row-major transpose
    Value v;
    v.kind = VK::Mat;
    v.rows = cols;
    v.cols = rows;
    v.ld = ld;
    v.colmajor = true;
    return add_value(s, v, out);
}

kf_status kf_matrix_q(kf_script* s, int64_t rows, int64_t cols, int64_t ld, int32_t dtype, kf_value scale,
                      kf_value* out) {
    if (dtype == KF_F32) {
        if (scale != KF_NONE) return set_error(KF_ERR_ARG, "FP32 matrices take no scale vector");
        return kf_matrix(s, rows, cols, ld, out);
    }
    if (dtype != KF_BF16 && dtype != KF_FP8_E4M3) return set_error(KF_ERR_DTYPE, "unknown matrix storage format");
    if (rows < 1 || cols < 1) return set_error(KF_ERR_SHAPE, "matrix dimensions must be >= 1");
    const int64_t per16 = 16 / dtype_size(dtype);
    if (ld == 0) ld = (cols + per16 - 1) / per16 * per16;
    if (ld < cols) return set_error(KF_ERR_SHAPE, "ld < cols");
    if (ld % per16) return set_error(KF_ERR_ALIGN, "ld must make every row a multiple of 16 bytes");
    if (!valid_value(s, scale)) return set_error(KF_ERR_ARG, "bad scale vector handle");
    const Value& sv = s->s.values[scale];
    if (sv.kind != VK::Vec || sv.n != rows) return set_error(KF_ERR_SHAPE, "scale vector must have rows entries");
    if (!sv.input) return set_error(KF_ERR_STATE, "scale vector is not marked input");
    Value v;
    v.kind = VK::Mat;
    v.rows = rows;
    v.cols = cols;
    v.ld = ld;
    v.dtype = dtype;
    v.scale = scale;
    return add_value(s, v, out);
}

kf_status kf_const(kf_script* s, float c, kf_value* out) {
    Value v;
    v.kind = VK::Const;
    v.cval = c;
    v.input = true;
    return add_value(s, v, out);
}

kf_status kf_scalar(kf_script* s, kf_value* out) {
    Value v;
    v.kind = VK::DevScalar;
    return add_value(s, v, out);
}

kf_status kf_input(kf_script* s, kf_value v) {
    if (!valid_value(s, v)) return set_error(KF_ERR_ARG, "bad value handle");
    Value& x = s->s.values[v];
    if (x.producer >= 0) return set_error(KF_ERR_STATE, "a computed value cannot be an input");
    x.input = true;
    return KF_OK;
}

kf_status kf_output(kf_script* s, kf_value v) {
    if (!valid_value(s, v)) return set_error(KF_ERR_ARG, "bad value handle");
    Value& x = s->s.values[v];
    if (x.producer < 0) return set_error(KF_ERR_STATE, "only computed values can be outputs");
    x.output = true;
    return KF_OK;
}

// Checks shared by the call recorders.
static kf_status need(const kf_script* s, kf_value v, VK kind, const char* what) {
    if (!valid_value(s, v)) return set_error(KF_ERR_ARG, std::string("bad handle for ") + what);
    const Value& x = s->s.values[v];
    bool ok = x.kind == kind || (kind == VK::Const && x.kind == VK::DevScalar);
    if (!ok) return set_error(KF_ERR_DTYPE, std::string(what) + " has the wrong kind");
    if (x.producer < 0 && !x.input)
        return set_error(KF_ERR_STATE, std::string(what) + " is declared but not marked input");
    return KF_OK;
}

static kf_status record(kf_script* s, const Call& c, const Value& outv, kf_value* out) {
    if (!out) return set_error(KF_ERR_ARG, "null out");
    KF_TRY({
        Value v = outv;
        v.producer = (int)s->s.calls.size();
        s->s.values.push_back(v);
        Call k = c;
        k.out = (int)s->s.values.size() - 1;
        s->s.calls.push_back(k);
        int ci = (int)s->s.calls.size() - 1;
        int ops[5] = {k.alpha, k.beta, k.in[0], k.in[1], k.in[2]};
        for (int o : ops)
            if (o >= 0) s->s.values[o].consumers.push_back(ci);
        if (k.in[0] >= 0 && s->s.values[k.in[0]].scale >= 0) s->s.values[s->s.values[k.in[0]].scale].consumers.push_back(ci);
        *out = k.out;
    });
    return KF_OK;
}

#define CHECK(e)                        \
    do {                                \
        kf_status st__ = (e);           \
        if (st__ != KF_OK) return st__; \
    } while (0)

kf_status kf_scal(kf_script* s, kf_value alpha, kf_value x, kf_value* y) {
    if (!s) return set_error(KF_ERR_ARG, "null script");
    CHECK(need(s, alpha, VK::Const, "alpha"));
    CHECK(need(s, x, VK::Vec, "x"));
    Call c;
    c.op = Op::Scal;
    c.alpha = alpha;
    c.in[0] = x;
    Value o;
    o.kind = VK::Vec;
    o.n = s->s.values[x].n;
    return record(s, c, o, y);
}

kf_status kf_axpy(kf_script* s, kf_value alpha, kf_value x, kf_value y, kf_value* z) {
    if (!s) return set_error(KF_ERR_ARG, "null script");
    CHECK(need(s, alpha, VK::Const, "alpha"));
    CHECK(need(s, x, VK::Vec, "x"));
    CHECK(need(s, y, VK::Vec, "y"));
    if (s->s.values[x].n != s->s.values[y].n) return set_error(KF_ERR_SHAPE, "axpy: x and y lengths differ");
    Call c;
    c.op = Op::Axpy;
    c.alpha = alpha;
    c.in[0] = x;
    c.in[1] = y;
    Value o;
    o.kind = VK::Vec;
    o.n = s->s.values[x].n;
    return record(s, c, o, z);
}

kf_status kf_dot(kf_script* s, kf_value x, kf_value y, kf_value* r) {
    if (!s) return set_error(KF_ERR_ARG, "null script");
    CHECK(need(s, x, VK::Vec, "x"));
    CHECK(need(s, y, VK::Vec, "y"));
    if (s->s.values[x].n != s->s.values[y].n) return set_error(KF_ERR_SHAPE, "dot: x and y lengths differ");
    Call c;
    c.op = Op::Dot;
    c.in[0] = x;
    c.in[1] = y;
    Value o;
    o.kind = VK::DevScalar;
    return record(s, c, o, r);
}

static kf_status rec_gemv(kf_script* s, bool trans, kf_value alpha, kf_value A, kf_value x,
                          kf_value beta, kf_value y0, kf_value* y) {
    if (!s) return set_error(KF_ERR_ARG, "null script");
    CHECK(need(s, alpha, VK::Const, "alpha"));
    CHECK(need(s, A, VK::Mat, "A"));
    CHECK(need(s, x, VK::Vec, "x"));
    const Value& Av = s->s.values[A];
    // A x with A column-major is (storage)^T x, and A^T x is (storage) x
    if (Av.colmajor) trans = !trans;
    int64_t nin = trans ? Av.rows : Av.cols, nout = trans ? Av.cols : Av.rows;
    if (s->s.values[x].n != nin) return set_error(KF_ERR_SHAPE, "gemv: x length does not match A");
    if (y0 != KF_NONE) {
        CHECK(need(s, y0, VK::Vec, "y0"));
        if (s->s.values[y0].n != nout) return set_error(KF_ERR_SHAPE, "gemv: y0 length does not match A");
        if (beta == KF_NONE) return set_error(KF_ERR_ARG, "gemv: y0 given without beta");
        CHECK(need(s, beta, VK::Const, "beta"));
    }
    Call c;
    c.op = trans ? Op::Gemtv : Op::Gemv;
    c.alpha = alpha;
    c.beta = y0 != KF_NONE ? beta : -1;
    c.in[0] = A;
    c.in[1] = x;
    c.in[2] = y0 != KF_NONE ? y0 : -1;
    Value o;
    o.kind = VK::Vec;
    o.n = nout;
    return record(s, c, o, y);
}

kf_status kf_gemv(kf_script* s, kf_value alpha, kf_value A, kf_value x, kf_value beta,
                  kf_value y0, kf_value* y) {
    return rec_gemv(s, false, alpha, A, x, beta, y0, y);
}

kf_status kf_gemtv(kf_script* s, kf_value alpha, kf_value A, kf_value x, kf_value beta,
                   kf_value y0, kf_value* y) {
    return rec_gemv(s, true, alpha, A, x, beta, y0, y);
}

kf_status kf_ger(kf_script* s, kf_value alpha, kf_value A, kf_value u, kf_value v, kf_value* B) {
    if (!s) return set_error(KF_ERR_ARG, "null script");
    CHECK(need(s, alpha, VK::Const, "alpha"));
    CHECK(need(s, A, VK::Mat, "A"));
    CHECK(need(s, u, VK::Vec, "u"));
    CHECK(need(s, v, VK::Vec, "v"));
    const Value& Av = s->s.values[A];
    // on column-major storage S = A^T the update is S + alpha v u^T: u and v swap
    if (Av.colmajor) std::swap(u, v);
    if (s->s.values[u].n != Av.rows || s->s.values[v].n != Av.cols)
        return set_error(KF_ERR_SHAPE, "ger: u/v lengths do not match A");
    Call c;
    c.op = Op::Ger;
    c.alpha = alpha;
    c.in[0] = A;
    c.in[1] = u;
    c.in[2] = v;
    Value o;
    o.kind = VK::Mat;
    o.rows = Av.rows;
    o.cols = Av.cols;
    o.ld = (Av.cols + 3) / 4 * 4;
    o.colmajor = Av.colmajor;   // B keeps A's layout
    return record(s, c, o, B);
}

kf_status kf_value_info(const kf_script* s, kf_value v, int32_t* kind, int64_t* d0, int64_t* d1,
                        int64_t* d2) {
    if (!valid_value(s, v)) return set_error(KF_ERR_ARG, "bad value handle");
    const Value& x = s->s.values[v];
    if (kind) *kind = (int32_t)x.kind;
    if (d0) *d0 = x.kind == VK::Mat ? (x.colmajor ? x.cols : x.rows) : x.n;
    if (d1) *d1 = x.colmajor ? x.rows : x.cols;
    if (d2) *d2 = x.ld;
    return KF_OK;
}

kf_status kf_value_layout(const kf_script* s, kf_value v, int32_t* layout) {
    if (!valid_value(s, v) || !layout) return set_error(KF_ERR_ARG, "bad argument");
    const Value& x = s->s.values[v];
    if (x.kind != VK::Mat) return set_error(KF_ERR_DTYPE, "not a matrix");
    *layout = x.colmajor ? KF_COL_MAJOR : KF_ROW_MAJOR;
    return KF_OK;
}

kf_status kf_script_num_calls(const kf_script* s, int32_t* n) {
    if (!s || !n) return set_error(KF_ERR_ARG, "null argument");
    *n = (int32_t)s->s.calls.size();
    return KF_OK;
}

kf_status kf_script_call(const kf_script* s, int32_t i, int32_t* op, kf_value* alpha, kf_value* beta,
                         kf_value* in3, kf_value* out) {
    if (!s) return set_error(KF_ERR_ARG, "null script");
    if (i < 0 || i >= (int32_t)s->s.calls.size()) return set_error(KF_ERR_ARG, "call index out of range");
    const Call& c = s->s.calls[i];
    if (op) *op = (int32_t)c.op;
    if (alpha) *alpha = c.alpha;
    if (beta) *beta = c.beta;
    if (in3)
        for (int j = 0; j < 3; ++j) in3[j] = c.in[j];
    if (out) *out = c.out;
    return KF_OK;
}

void kf_compile_opts_init(kf_compile_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->mode = KF_MODE_FUSED;
}

kf_status kf_enumerate(const kf_script* s, int32_t max_plans, kf_planset** out) {
    if (!s || !out) return set_error(KF_ERR_ARG, "null argument");
    if (s->s.calls.empty()) return set_error(KF_ERR_STATE, "script has no calls");
    KF_TRY({
        auto* ps = new kf_planset();
        ps->parts = enumerate_partitions(s->s, max_plans);
        *out = ps;
    });
    return KF_OK;
}

void kf_planset_destroy(kf_planset* ps) { delete ps; }

kf_status kf_planset_count(const kf_planset* ps, int32_t* n) {
    if (!ps || !n) return set_error(KF_ERR_ARG, "null argument");
    *n = (int32_t)ps->parts.size();
    return KF_OK;
}

kf_status kf_planset_get(const kf_planset* ps, int32_t i, int32_t* partition, int32_t len) {
    if (!ps || !partition) return set_error(KF_ERR_ARG, "null argument");
    if (i < 0 || i >= (int32_t)ps->parts.size()) return set_error(KF_ERR_ARG, "plan index out of range");
    if (len < (int32_t)ps->parts[i].size()) return set_error(KF_ERR_ARG, "partition buffer too small");
    for (size_t c = 0; c < ps->parts[i].size(); ++c) partition[c] = ps->parts[i][c];
    return KF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// compilation
// ---------------------------------------------------------------------------
static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static size_t value_bytes(const Value& v) {
    switch (v.kind) {
        case VK::Vec: return (size_t)v.n * 4;
        case VK::Mat: return (size_t)v.rows * v.ld * (size_t)dtype_size(v.dtype);
        case VK::DevScalar: return 4;
        default: return 0;
    }
}

static kf_status check_params(const MatParams& mp, const VecParams& vp) {
    if (mp.sched < 0 || mp.sched > 1) return set_error(KF_ERR_ARG, "mat_sched must be 0 or 1");
    if (mp.unit != 0 && mp.unit != 4 && mp.unit != 16) return set_error(KF_ERR_ARG, "mat_unit must be 0, 4 or 16");
    if (mp.k && mp.k != 1 && mp.k != 2 && mp.k != 4) return set_error(KF_ERR_ARG, "mat_k must be 1, 2 or 4");
    if (mp.waves && (mp.waves < 1 || mp.waves > 16)) return set_error(KF_ERR_ARG, "mat_waves must be 1..16");
    if (mp.group && (mp.group & (mp.group - 1) || mp.group > 16)) return set_error(KF_ERR_ARG, "mat_group must be 1, 2, 4, 8 or 16");
    if (mp.rows < 0) return set_error(KF_ERR_ARG, "mat_rows must be >= 0");
    if (vp.unroll && (vp.unroll < 1 || vp.unroll > 8)) return set_error(KF_ERR_ARG, "vec_unroll must be 1..8");
    if (vp.threads && (vp.threads < 64 || vp.threads > 1024 || vp.threads % 64)) return set_error(KF_ERR_ARG, "vec_threads must be a multiple of 64 in 64..1024");
    if (vp.grid < 0) return set_error(KF_ERR_ARG, "vec_grid must be >= 0");
    return KF_OK;
}

kf_status build_plan(const Script& sc, const std::vector<int>& part, const kf_compile_opts& o,
                            kf_plan** out) {
    const int ncall = (int)sc.calls.size();
    if ((int)part.size() != ncall) return set_error(KF_ERR_ARG, "partition length != number of calls");
    int nk = 0;
    for (int k : part) {
        if (k < 0) return set_error(KF_ERR_ARG, "negative kernel id in partition");
        nk = std::max(nk, k + 1);
    }
    std::vector<std::vector<int>> members(nk);
    for (int c = 0; c < ncall; ++c) members[part[c]].push_back(c);
    for (int k = 0; k < nk; ++k) {
        if (members[k].empty()) return set_error(KF_ERR_ARG, "partition kernel ids must be dense");
        std::string why = block_illegal_reason(sc, members[k]);
        if (members[k].size() > 1 && !why.empty())
            return set_error(KF_ERR_UNSUPPORTED, "illegal fusion: " + why);
    }
    if (!partition_acyclic(sc, part, nk)) return set_error(KF_ERR_UNSUPPORTED, "illegal plan: kernels form a cycle");

    auto* p = new kf_plan();
    std::unique_ptr<kf_plan> guard(p);
    p->s = sc;
    p->part = part;
    p->mode = o.mode;
    const size_t nv = sc.values.size();
    p->mp.k = o.mat_k; p->mp.waves = o.mat_waves; p->mp.group = o.mat_group; p->mp.rows = o.mat_rows;
    p->mp.sched = o.mat_sched;
    p->mp.unit = o.mat_unit;
    p->vp.unroll = o.vec_unroll; p->vp.threads = o.vec_threads; p->vp.grid = o.vec_grid;
    p->bind.assign(nv, nullptr);
    p->consts.assign(nv, 0.f);
    p->inter_off.assign(nv, SIZE_MAX);
    p->is_read.assign(nv, 0);
    p->is_written.assign(nv, 0);
    for (size_t v = 0; v < nv; ++v)
        if (sc.values[v].kind == VK::Const) p->consts[v] = sc.values[v].cval;

    MatParams mp0;
    mp0.k = o.mat_k;
    mp0.waves = o.mat_waves;
    mp0.group = o.mat_group;
    mp0.rows = o.mat_rows;
    mp0.sched = o.mat_sched;
    mp0.unit = o.mat_unit;
    if (o.flags & KF_COMPILE_RUNTIME_SHAPE) {
        // every matrix shares one storage shape, and every vector is a row or a
        // column vector of it; runs may then take any smaller shape
        int64_t M = -1, N = -1;
        for (const Value& x : sc.values)
            if (x.kind == VK::Mat) {
                if (M < 0) { M = x.rows; N = x.cols; }
                if (x.rows != M || x.cols != N)
                    return set_error(KF_ERR_UNSUPPORTED, "runtime-shape plans need every matrix of one shape");
            }
        if (M < 0) return set_error(KF_ERR_UNSUPPORTED, "runtime-shape plans need BLAS-2 calls");
        for (const Value& x : sc.values)
            if (x.kind == VK::Vec && x.n != M && x.n != N)
                return set_error(KF_ERR_UNSUPPORTED, "runtime-shape plans need vectors of the matrix's rows or cols");
        for (int c = 0; c < (int)sc.calls.size(); ++c)
            if (!call_space(sc, c).mat) return set_error(KF_ERR_UNSUPPORTED, "runtime-shape plans take BLAS-2 kernels only");
        if (o.mat_sched == 1) return set_error(KF_ERR_UNSUPPORTED, "runtime-shape plans use the strip schedule");
        mp0.dyn = true;
        p->dyn = true;
        p->decl_m = p->rt_m = M;
        p->decl_n = p->rt_n = N;
        p->rt_ld.assign(nv, 0);
        for (size_t v = 0; v < nv; ++v)
            if (sc.values[v].kind == VK::Mat) p->rt_ld[v] = sc.values[v].ld;
    }
    VecParams vp0;
    vp0.unroll = o.vec_unroll;
    vp0.threads = o.vec_threads;
    vp0.grid = o.vec_grid;
    kf_status pst = check_params(mp0, vp0);
    if (pst != KF_OK) return pst;

    auto order = kernels_in_order(sc, part);
    if (o.kernel_params_len < 0 || (o.kernel_params_len > 0 && !o.kernel_params))
        return set_error(KF_ERR_ARG, "kernel_params missing or of negative length");
    if (o.kernel_params_len > (int32_t)order.size())
        return set_error(KF_ERR_ARG, "more kernel_params entries than kernels in the plan");
    for (size_t ki = 0; ki < order.size(); ++ki) {
        const auto& calls = order[ki];
        PlanKernel pk;
        MatParams mp = mp0;
        VecParams vp = vp0;
        if ((int32_t)ki < o.kernel_params_len) {
            const kf_impl_params& e = o.kernel_params[ki];
            if (e.mat_k) mp.k = e.mat_k;
            if (e.mat_waves) mp.waves = e.mat_waves;
            if (e.mat_group) mp.group = e.mat_group;
            if (e.mat_rows) mp.rows = e.mat_rows;
            if (e.mat_sched) mp.sched = e.mat_sched;
            if (e.mat_unit) mp.unit = e.mat_unit;
            if (e.vec_unroll) vp.unroll = e.vec_unroll;
            if (e.vec_threads) vp.threads = e.vec_threads;
            if (e.vec_grid) vp.grid = e.vec_grid;
            pst = check_params(mp, vp);
            if (pst != KF_OK) return pst;
        }
        pk.mp = mp;
        pk.vp = vp;
        Space sp = call_space(sc, calls[0]);
        if (mp0.dyn && (mp.sched == 1 || needs_rowres(sc, calls)))
            return set_error(KF_ERR_UNSUPPORTED, "runtime-shape plans use the strip schedule (this kernel needs whole rows)");
        if (sp.mat && (mp.sched == 1 || needs_rowres(sc, calls))) {
            if (sp.b > 32768) return set_error(KF_ERR_UNSUPPORTED, "row-resident schedule needs cols <= 32768");
            if (kernel_has_quantized(sc, calls))
                return set_error(KF_ERR_UNSUPPORTED, "row-resident schedule reads FP32 matrices only");
            if (mp.sched == 1 && mp.rows && mp.group && mp.rows % mp.group)
                return set_error(KF_ERR_ARG, "mat_rows must be a multiple of mat_group");
            if (mp.sched == 1 && mp.waves && (int64_t)mp.waves * 256 * 8 < sp.b)
                return set_error(KF_ERR_ARG, "row-resident schedule: mat_waves too small for the row length");
            {   // the wave partials of a row group are merged one per lane
                MatParams q = mp;
                if (q.sched != 1) q.waves = q.group = q.rows = 0;   // strip parameters do not carry over
                const RowresGeom g = rowres_geometry(sp.a, sp.b, q);
                if (g.G * g.WP > 64)
                    return set_error(KF_ERR_ARG, "row-resident schedule: mat_group times mat_waves (rounded up to a "
                                                 "power of two) must be <= 64");
            }
        } else if (sp.mat) {
            MatParams q = default_mat_params(sp.a, sp.b, mp, kernel_unit_elems(sc, calls, mp.unit));
            if (q.rows % (q.waves * q.group)) return set_error(KF_ERR_ARG, "mat_rows must be a multiple of mat_waves * mat_group");
        }
        pk.code = generate_kernel(sc, calls, part, mp, vp);
        if (pk.code.lds_bytes > 160 * 1024)
            return set_error(KF_ERR_ARG, "parameters need " + std::to_string(pk.code.lds_bytes) +
                                             " bytes of LDS per workgroup (gfx950 limit 163840)");
        for (const Launch& l : pk.code.launches)
            for (const KArg& a : l.args) {
                if (a.kind == ArgKind::MatIn || a.kind == ArgKind::VecIn || a.kind == ArgKind::DevScalarIn) p->is_read[a.value] = 1;
                if (a.kind == ArgKind::MatOut || a.kind == ArgKind::VecOut || a.kind == ArgKind::DevScalarOut) p->is_written[a.value] = 1;
            }
        p->ks.push_back(std::move(pk));
    }
    // workspace: partial sums, then intermediates kept in HBM
    size_t off = 0;
    for (auto& k : p->ks) { k.ws_off = off; off = align_up(off + k.code.ws_floats * 4, 256); }
    for (size_t v = 0; v < nv; ++v) {
        const Value& x = sc.values[v];
        if (x.producer >= 0 && !x.output && p->is_written[v]) {
            p->inter_off[v] = off;
            off = align_up(off + value_bytes(x), 256);
        }
    }
    p->ws_need = off;

    if (o.flags & KF_COMPILE_CODEGEN_ONLY) {   // plan structure only: features, bytes, predictions
        p->loaded = false;
        *out = guard.release();
        return KF_OK;
    }
    // compile (and load) the kernels not yet known
    Registry& reg = registry();
    std::lock_guard<std::mutex> lock(reg.mu);
    const bool load = !(o.flags & KF_COMPILE_NO_LOAD);
    if (load) {
        std::vector<const KernelCode*> all;
        for (auto& k : p->ks) all.push_back(&k.code);
        load_together_locked(reg, all);
    }
    for (auto& k : p->ks) {
        const std::string& nm = k.code.name;
        if (!load) {
            if (reg.compiled.count(nm) || reg.funcs.count(k.code.launches[0].name)) continue;
            std::string co, log;
            if (!jit_compile_one(k.code, &co, &log)) return set_error(KF_ERR_COMPILE, log);
            reg.compiled.insert(nm);
            continue;
        }
        kf_status st = ensure_loaded_locked(reg, k.code);
        if (st != KF_OK) return st;
    }
    if (load)
        for (auto& k : p->ks)
            for (const Launch& l : k.code.launches) k.fns.push_back((void*)reg.funcs[l.name]);
    p->loaded = load;
    *out = guard.release();
    return KF_OK;
}

kf_status compile_additive(const kf_script* s, const kf_compile_opts& o, kf_plan** out);
namespace kf {
kf_status compile_learned(const kf_script* s, const kf_compile_opts& o, kf_plan** out);
kf_status compile_exhaustive(const kf_script* s, const kf_compile_opts& o, kf_plan** out);
kf_status timed_workspace_bytes(const kf_script* s, const kf_compile_opts& o, size_t* bytes);
}  // namespace kf

extern "C" {

kf_status kf_compile_workspace_bytes(const kf_script* s, const kf_compile_opts* opts, size_t* bytes) {
    if (!s || !bytes) return set_error(KF_ERR_ARG, "null argument");
    if (s->s.calls.empty()) return set_error(KF_ERR_STATE, "script has no calls");
    kf_compile_opts o;
    kf_compile_opts_init(&o);
    if (opts) o = *opts;
    KF_TRY({ return kf::timed_workspace_bytes(s, o, bytes); });
    return KF_OK;
}

kf_status kf_compile(const kf_script* s, const kf_compile_opts* opts, kf_plan** out) {
    if (!s || !out) return set_error(KF_ERR_ARG, "null argument");
    if (s->s.calls.empty()) return set_error(KF_ERR_STATE, "script has no calls");
    kf_compile_opts o;
    kf_compile_opts_init(&o);
    if (opts) o = *opts;
    std::vector<int> part;
    KF_TRY({
        switch (o.mode) {
            case KF_MODE_UNFUSED: part = unfused_partition(s->s); break;
            case KF_MODE_FUSED: part = fused_partition(s->s); break;
            case KF_MODE_PARTITION:
                if (!o.partition || o.partition_len != (int32_t)s->s.calls.size())
                    return set_error(KF_ERR_ARG, "partition missing or of the wrong length");
                part.assign(o.partition, o.partition + o.partition_len);
                break;
            case KF_MODE_ADDITIVE:
                return compile_additive(s, o, out);
            case KF_MODE_LEARNED:
                return kf::compile_learned(s, o, out);
            case KF_MODE_EXHAUSTIVE:
                return kf::compile_exhaustive(s, o, out);
            default: return set_error(KF_ERR_ARG, "unknown mode");
        }
        return build_plan(s->s, part, o, out);
    });
    return KF_OK;
}

void kf_plan_destroy(kf_plan* p) { delete p; }

kf_status kf_plan_workspace_bytes(const kf_plan* p, size_t* bytes) {
    if (!p || !bytes) return set_error(KF_ERR_ARG, "null argument");
    *bytes = p->ws_need;
    return KF_OK;
}

static bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + nb && y < x + na;
}

// Bytes of value v's buffer as the plan will touch it: the declared shape, or
// for runtime-shape plans the current shape (rows x leading dimension for a
// matrix, rows or cols entries for a vector).
static size_t bound_bytes(const kf_plan* p, int v) {
    const Value& x = p->s.values[v];
    if (!p->dyn) return value_bytes(x);
    switch (x.kind) {
        case VK::Vec: return (size_t)(x.n == p->decl_m ? p->rt_m : p->rt_n) * 4;
        case VK::Mat: return (size_t)p->rt_m * (size_t)p->rt_ld[v] * (size_t)dtype_size(x.dtype);
        case VK::DevScalar: return 4;
        default: return 0;
    }
}

static kf_status bind_checked(kf_plan* p, kf_value v, void* ptr) {
    if (!p) return set_error(KF_ERR_ARG, "null plan");
    if (v < 0 || v >= (kf_value)p->s.values.size()) return set_error(KF_ERR_ARG, "bad value handle");
    const Value& x = p->s.values[v];
    if (x.kind == VK::Const) return set_error(KF_ERR_DTYPE, "constants are set with kf_set_const");
    if (x.producer >= 0 && !x.output)
        return set_error(KF_ERR_ARG, "intermediate values live in the plan workspace");
    if (!ptr) return set_error(KF_ERR_ARG, "null device pointer");
    size_t al = x.kind == VK::DevScalar ? 4 : 16;
    if ((uintptr_t)ptr % al) return set_error(KF_ERR_ALIGN, "device pointer misaligned");
    const size_t nb = bound_bytes(p, v);
    // an output must not overlap any other bound value
    for (size_t w = 0; w < p->s.values.size(); ++w) {
        if ((kf_value)w == v || !p->bind[w]) continue;
        const Value& y = p->s.values[w];
        bool vw = x.producer >= 0, ww = y.producer >= 0;
        if ((vw || ww) && overlap(ptr, nb, p->bind[w], bound_bytes(p, (int)w)))
            return set_error(KF_ERR_ALIAS, "an output buffer overlaps another operand");
    }
    p->bind[v] = ptr;
    return KF_OK;
}

kf_status kf_bind(kf_plan* p, kf_value v, void* ptr) { return bind_checked(p, v, ptr); }

kf_status kf_plan_set_shape(kf_plan* p, int64_t rows, int64_t cols) {
    if (!p) return set_error(KF_ERR_ARG, "null plan");
    if (!p->dyn) return set_error(KF_ERR_STATE, "the plan was not compiled with KF_COMPILE_RUNTIME_SHAPE");
    if (rows < 1 || cols < 1 || rows > p->decl_m || cols > p->decl_n)
        return set_error(KF_ERR_SHAPE, "runtime shape outside 1 .. the declared shape");
    if (p->decl_m == p->decl_n && rows != cols)
        return set_error(KF_ERR_SHAPE, "a plan declared square runs square shapes only");
    p->rt_m = rows;
    p->rt_n = cols;
    for (size_t v = 0; v < p->s.values.size(); ++v) {
        if (p->inter_off[v] == SIZE_MAX) p->bind[v] = nullptr;
        if (p->s.values[v].kind == VK::Mat) p->rt_ld[v] = p->s.values[v].ld;
    }
    return KF_OK;
}

kf_status kf_bind_matrix(kf_plan* p, kf_value v, void* ptr, int64_t ld) {
    if (!p) return set_error(KF_ERR_ARG, "null plan");
    if (!p->dyn) return set_error(KF_ERR_STATE, "the plan was not compiled with KF_COMPILE_RUNTIME_SHAPE");
    if (v < 0 || v >= (kf_value)p->s.values.size() || p->s.values[v].kind != VK::Mat)
        return set_error(KF_ERR_DTYPE, "not a matrix value");
    const int es = dtype_size(p->s.values[v].dtype);
    if (ld < p->rt_n || (ld * es) % 16) return set_error(KF_ERR_ALIGN, "ld must be >= the runtime cols and make 16-byte rows");
    const int64_t old = p->rt_ld[v];
    p->rt_ld[v] = ld;
    kf_status st = bind_checked(p, v, ptr);
    if (st != KF_OK) p->rt_ld[v] = old;
    return st;
}

kf_status kf_bind_workspace(kf_plan* p, void* ptr, size_t bytes) {
    if (!p) return set_error(KF_ERR_ARG, "null plan");
    if (bytes < p->ws_need) return set_error(KF_ERR_WORKSPACE, "workspace smaller than kf_plan_workspace_bytes");
    if (p->ws_need && !ptr) return set_error(KF_ERR_ARG, "null workspace");
    if ((uintptr_t)ptr % 256) return set_error(KF_ERR_ALIGN, "workspace must be 256-byte aligned");
    p->ws = ptr;
    p->ws_bound = bytes;
    return KF_OK;
}

kf_status kf_set_const(kf_plan* p, kf_value v, float value) {
    if (!p) return set_error(KF_ERR_ARG, "null plan");
    if (v < 0 || v >= (kf_value)p->s.values.size()) return set_error(KF_ERR_ARG, "bad value handle");
    if (p->s.values[v].kind != VK::Const) return set_error(KF_ERR_DTYPE, "not a constant");
    p->consts[v] = value;
    return KF_OK;
}

// Device address of value v: a bound buffer, or its place in workspace ws.
static void* value_ptr(kf_plan* p, int v, void* ws) {
    if (p->inter_off[v] != SIZE_MAX) return (char*)ws + p->inter_off[v];
    return p->bind[v];
}

// Launches first .. last - 1 of kernel k with workspace ws (the bound one, or
// the static scratch of kf_run_noalloc).
static kf_status launch_kernel(kf_plan* p, PlanKernel& k, hipStream_t stream, void* ws, int first = 0,
                               int last = -1) {
    if (last < 0) last = (int)k.code.launches.size();
    for (size_t li = (size_t)first; li < (size_t)last; ++li) {
        const Launch& l = k.code.launches[li];
        const size_t na = l.args.size();
        uint64_t store[64];
        void* ptrs[64];
        if (na > 64) return set_error(KF_ERR_INTERNAL, "too many kernel arguments");
        int64_t grid = l.grid;
        if (l.dyn_grid) {
            const int64_t S = (p->rt_n + l.dyn_c - 1) / l.dyn_c, NB = (p->rt_m + l.dyn_r - 1) / l.dyn_r;
            const int64_t NP = (p->rt_n + 3) / 4 * 4;
            grid = l.dyn_grid == 1 ? S * NB
                                   : (l.dyn_rpart ? (p->rt_m + l.dyn_fwb - 1) / l.dyn_fwb : 0) +
                                         (l.dyn_cpart ? (NP / 4 + 63) / 64 : 0);
        }
        for (size_t i = 0; i < na; ++i) {
            const KArg& a = l.args[i];
            store[i] = 0;
            switch (a.kind) {
                case ArgKind::ConstScalar: {
                    float f = p->consts[a.value];
                    std::memcpy(&store[i], &f, 4);
                    break;
                }
                case ArgKind::Workspace: store[i] = (uint64_t)(uintptr_t)((char*)ws + k.ws_off); break;
                case ArgKind::ShapeM: store[i] = (uint64_t)p->rt_m; break;
                case ArgKind::ShapeN: store[i] = (uint64_t)p->rt_n; break;
                case ArgKind::MatLd:   // an intermediate in the workspace keeps its declared pitch
                    store[i] = (uint64_t)(p->inter_off[a.value] != SIZE_MAX ? p->s.values[a.value].ld : p->rt_ld[a.value]);
                    break;
                default: {
                    void* q = value_ptr(p, a.value, ws);
                    if (!q) return set_error(KF_ERR_UNBOUND, "value " + std::to_string(a.value) + " is not bound");
                    store[i] = (uint64_t)(uintptr_t)q;
                }
            }
            ptrs[i] = &store[i];
        }
        if (grid <= 0) continue;
        hipError_t e = hipModuleLaunchKernel((hipFunction_t)k.fns[li], (unsigned)grid, 1, 1, (unsigned)l.block, 1, 1, 0,
                                             stream, ptrs, nullptr);
        if (e != hipSuccess) return set_error(KF_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
    }
    return KF_OK;
}

static kf_status check_runnable(const kf_plan* p) {
    if (!p) return set_error(KF_ERR_ARG, "null plan");
    if (!p->loaded) return set_error(KF_ERR_STATE, "plan compiled without loading");
    if (p->ws_need && !p->ws) return set_error(KF_ERR_UNBOUND, "workspace not bound");
    return KF_OK;
}

kf_status kf_run(kf_plan* p, void* stream) {
    CHECK(check_runnable(p));
    for (auto& k : p->ks) CHECK(launch_kernel(p, k, (hipStream_t)stream, p->ws));
    return KF_OK;
}

extern "C++" kf_status kf::plan_loaded(const kf_plan* p) {
    if (!p) return set_error(KF_ERR_ARG, "null plan");
    if (!p->loaded) return set_error(KF_ERR_STATE, "plan compiled without loading");
    return KF_OK;
}

extern "C++" kf_status kf::run_on_workspace(kf_plan* p, void* ws, void* stream) {
    CHECK(plan_loaded(p));
    if (p->ws_need && !ws) return set_error(KF_ERR_ARG, "null workspace");
    if ((uintptr_t)ws % 256) return set_error(KF_ERR_ALIGN, "workspace must be 256-byte aligned");
    for (auto& k : p->ks) CHECK(launch_kernel(p, k, (hipStream_t)stream, ws));
    return KF_OK;
}

kf_status kf_plan_run_many(kf_plan* p, int64_t count, const int64_t* shapes, int32_t nvals, const kf_value* values,
                           void* const* ptrs, const int64_t* lds, void* stream) {
    if (!p || count < 0 || nvals < 0 || (count > 0 && (!shapes || (nvals > 0 && (!values || !ptrs)))))
        return set_error(KF_ERR_ARG, "bad argument");
    CHECK(check_runnable(p));
    for (int64_t i = 0; i < count; ++i) {
        CHECK(kf_plan_set_shape(p, shapes[2 * i], shapes[2 * i + 1]));
        for (int32_t j = 0; j < nvals; ++j) {
            const kf_value v = values[j];
            void* ptr = ptrs[i * nvals + j];
            if (v >= 0 && v < (kf_value)p->s.values.size() && p->s.values[v].kind == VK::Mat)
                CHECK(kf_bind_matrix(p, v, ptr, lds ? lds[i * nvals + j] : p->s.values[v].ld));
            else
                CHECK(bind_checked(p, v, ptr));
        }
        for (auto& k : p->ks) CHECK(launch_kernel(p, k, (hipStream_t)stream, p->ws));
    }
    return KF_OK;
}

kf_status kf_plan_num_launches(const kf_plan* p, int32_t k, int32_t* n) {
    if (!p || !n) return set_error(KF_ERR_ARG, "null argument");
    if (k < 0 || k >= (int32_t)p->ks.size()) return set_error(KF_ERR_ARG, "kernel index out of range");
    *n = (int32_t)p->ks[k].code.launches.size();
    return KF_OK;
}

kf_status kf_run_launch(kf_plan* p, int32_t k, int32_t l, void* stream) {
    CHECK(check_runnable(p));
    if (k < 0 || k >= (int32_t)p->ks.size()) return set_error(KF_ERR_ARG, "kernel index out of range");
    if (l < 0 || l >= (int32_t)p->ks[k].code.launches.size()) return set_error(KF_ERR_ARG, "launch index out of range");
    return launch_kernel(p, p->ks[k], (hipStream_t)stream, p->ws, l, l + 1);
}

kf_status kf_run_kernel(kf_plan* p, int32_t k, void* stream) {
    CHECK(check_runnable(p));
    if (k < 0 || k >= (int32_t)p->ks.size()) return set_error(KF_ERR_ARG, "kernel index out of range");
    return launch_kernel(p, p->ks[k], (hipStream_t)stream, p->ws);
}

kf_status kf_time_plan(kf_plan* p, void* stream, int32_t warmup, int32_t reps, float* median_us) {
    if (!p || !median_us || reps < 1 || warmup < 0) return set_error(KF_ERR_ARG, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < warmup; ++i) CHECK(kf_run(p, stream));
    std::vector<hipEvent_t> ev(2 * reps);
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) return set_error(KF_ERR_HIP, "hipEventCreate");
    kf_status st_out = KF_OK;
    for (int i = 0; i < reps && st_out == KF_OK; ++i) {
        if (hipEventRecord(ev[2 * i], st) != hipSuccess) { st_out = set_error(KF_ERR_HIP, "hipEventRecord"); break; }
        st_out = kf_run(p, stream);
        if (st_out == KF_OK && hipEventRecord(ev[2 * i + 1], st) != hipSuccess) st_out = set_error(KF_ERR_HIP, "hipEventRecord");
    }
    std::vector<float> t;
    if (st_out == KF_OK) {
        if (hipStreamSynchronize(st) != hipSuccess) st_out = set_error(KF_ERR_HIP, "hipStreamSynchronize");
        for (int i = 0; i < reps && st_out == KF_OK; ++i) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) != hipSuccess) st_out = set_error(KF_ERR_HIP, "hipEventElapsedTime");
            t.push_back(ms * 1000.f);
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (st_out != KF_OK) return st_out;
    std::sort(t.begin(), t.end());
    *median_us = t.size() % 2 ? t[t.size() / 2] : 0.5f * (t[t.size() / 2 - 1] + t[t.size() / 2]);
    return KF_OK;
}

kf_status kf_time_plan_kernels(kf_plan* p, void* stream, int32_t warmup, int32_t reps, float* us) {
    if (!p || !us || reps < 1 || warmup < 0) return set_error(KF_ERR_ARG, "bad argument");
    CHECK(check_runnable(p));
    hipStream_t st = (hipStream_t)stream;
    const size_t nk = p->ks.size();
    for (int i = 0; i < warmup; ++i) CHECK(kf_run(p, stream));
    // events[(rep * nk + k) * 2 + {0, 1}] bracket kernel k of run rep
    std::vector<hipEvent_t> ev(2 * nk * (size_t)reps, nullptr);
    kf_status st_out = KF_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            st_out = set_error(KF_ERR_HIP, "hipEventCreate");
            break;
        }
    for (int i = 0; i < reps && st_out == KF_OK; ++i)
        for (size_t k = 0; k < nk && st_out == KF_OK; ++k) {
            const size_t at = ((size_t)i * nk + k) * 2;
            if (hipEventRecord(ev[at], st) != hipSuccess) { st_out = set_error(KF_ERR_HIP, "hipEventRecord"); break; }
            st_out = launch_kernel(p, p->ks[k], st, p->ws);
            if (st_out == KF_OK && hipEventRecord(ev[at + 1], st) != hipSuccess) st_out = set_error(KF_ERR_HIP, "hipEventRecord");
        }
    std::vector<std::vector<float>> t(nk);
    if (st_out == KF_OK) {
        if (hipStreamSynchronize(st) != hipSuccess) st_out = set_error(KF_ERR_HIP, "hipStreamSynchronize");
        for (int i = 0; i < reps && st_out == KF_OK; ++i)
            for (size_t k = 0; k < nk && st_out == KF_OK; ++k) {
                const size_t at = ((size_t)i * nk + k) * 2;
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, ev[at], ev[at + 1]) != hipSuccess) st_out = set_error(KF_ERR_HIP, "hipEventElapsedTime");
                t[k].push_back(ms * 1000.f);
            }
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (st_out != KF_OK) return st_out;
    for (size_t k = 0; k < nk; ++k) {
        auto& v = t[k];
        std::sort(v.begin(), v.end());
        us[k] = v.size() % 2 ? v[v.size() / 2] : 0.5f * (v[v.size() / 2 - 1] + v[v.size() / 2]);
    }
    return KF_OK;
}

kf_status kf_plan_kernel_params(const kf_plan* p, int32_t k, kf_impl_params* out) {
    if (!p || !out) return set_error(KF_ERR_ARG, "null argument");
    if (k < 0 || k >= (int32_t)p->ks.size()) return set_error(KF_ERR_ARG, "kernel index out of range");
    const PlanKernel& pk = p->ks[k];
    const Space sp = call_space(p->s, pk.code.calls[0]);
    kf_impl_params r;
    std::memset(&r, 0, sizeof r);
    if (sp.mat) {
        const bool rowres = pk.mp.sched == 1 || needs_rowres(p->s, pk.code.calls);
        MatParams q = rowres ? pk.mp
                             : default_mat_params(sp.a, sp.b, pk.mp, kernel_unit_elems(p->s, pk.code.calls, pk.mp.unit));
        if (rowres && pk.mp.sched != 1) q.waves = q.group = q.rows = 0;   // strip parameters do not carry over
        r.mat_k = q.k; r.mat_waves = q.waves; r.mat_group = q.group; r.mat_rows = q.rows;
        r.mat_sched = rowres ? 1 : 0;
        r.mat_unit = kernel_has_quantized(p->s, pk.code.calls) ? q.unit : 0;   // FP32 kernels have no load unit
    } else {
        const VecParams q = default_vec_params(sp.a, pk.vp);
        r.vec_unroll = q.unroll; r.vec_threads = q.threads; r.vec_grid = q.grid;
    }
    *out = r;
    return KF_OK;
}

kf_status kf_plan_bytes(const kf_plan* p, uint64_t* rd, uint64_t* wr) {
    if (!p || !rd || !wr) return set_error(KF_ERR_ARG, "null argument");
    uint64_t r = 0, w = 0;
    for (auto& k : p->ks) { r += k.code.bytes_read; w += k.code.bytes_written; }
    *rd = r;
    *wr = w;
    return KF_OK;
}

kf_status kf_plan_num_kernels(const kf_plan* p, int32_t* n) {
    if (!p || !n) return set_error(KF_ERR_ARG, "null argument");
    *n = (int32_t)p->ks.size();
    return KF_OK;
}

static kf_status copy_out(const std::string& s, char* buf, size_t cap, size_t* needed) {
    if (needed) *needed = s.size() + 1;
    if (buf && cap) {
        size_t n = std::min(cap - 1, s.size());
        std::memcpy(buf, s.data(), n);
        buf[n] = '\0';
    }
    return KF_OK;
}

kf_status kf_plan_source(const kf_plan* p, int32_t k, char* buf, size_t cap, size_t* needed) {
    if (!p) return set_error(KF_ERR_ARG, "null plan");
    if (k < 0 || k >= (int32_t)p->ks.size()) return set_error(KF_ERR_ARG, "kernel index out of range");
    return copy_out(p->ks[k].code.source, buf, cap, needed);
}

kf_status kf_plan_kernel_geometry(const kf_plan* p, int32_t k, int32_t* grid, int32_t* block) {
    if (!p) return set_error(KF_ERR_ARG, "null plan");
    if (k < 0 || k >= (int32_t)p->ks.size()) return set_error(KF_ERR_ARG, "kernel index out of range");
    if (grid) *grid = p->ks[k].code.launches[0].grid;
    if (block) *block = p->ks[k].code.launches[0].block;
    return KF_OK;
}

kf_status kf_plan_describe(const kf_plan* p, char* buf, size_t cap, size_t* needed) {
    if (!p) return set_error(KF_ERR_ARG, "null plan");
    std::ostringstream o;
    uint64_t r = 0, w = 0;
    o << "{\"kernels\": [";
    for (size_t i = 0; i < p->ks.size(); ++i) {
        const KernelCode& k = p->ks[i].code;
        o << (i ? ", " : "") << "{\"name\": \"" << k.name << "\", \"class\": \"" << (k.mat ? "blas2" : "blas1")
          << "\", \"calls\": [";
        for (size_t j = 0; j < k.calls.size(); ++j)
            o << (j ? ", " : "") << "{\"index\": " << k.calls[j] << ", \"op\": \"" << op_name(p->s.calls[k.calls[j]].op) << "\"}";
        o << "], \"launches\": [";
        for (size_t j = 0; j < k.launches.size(); ++j)
            o << (j ? ", " : "") << "{\"name\": \"" << k.launches[j].name << "\", \"grid\": " << k.launches[j].grid
              << ", \"block\": " << k.launches[j].block << ", \"bytes_read\": " << k.launches[j].bytes_read
              << ", \"bytes_written\": " << k.launches[j].bytes_written << "}";
        o << "], \"grid\": " << k.launches[0].grid << ", \"block\": " << k.launches[0].block
          << ", \"params\": " << k.params_json << ", \"bytes_read\": " << k.bytes_read
          << ", \"bytes_written\": " << k.bytes_written << ", \"workspace_floats\": " << k.ws_floats
          << ", \"lds_bytes\": " << k.lds_bytes << "}";
        r += k.bytes_read;
        w += k.bytes_written;
    }
    o << "], \"partition\": [";
    for (size_t i = 0; i < p->part.size(); ++i) o << (i ? ", " : "") << p->part[i];
    o << "], \"bytes_read\": " << r << ", \"bytes_written\": " << w << ", \"workspace_bytes\": " << p->ws_need
      << "}";
    return copy_out(o.str(), buf, cap, needed);
}

kf_status kf_jit_release(void) {
    Registry& reg = registry();
    std::lock_guard<std::mutex> lock(reg.mu);
    for (hipModule_t m : reg.modules) (void)hipModuleUnload(m);
    reg.modules.clear();
    reg.funcs.clear();
    reg.compiled.clear();
    reg.by_ident.clear();
    return KF_OK;
}

kf_status kf_jit_set_cache_dir(const char* dir) {
    if (dir && *dir) {
        struct stat st;
        if (::stat(dir, &st) != 0 || !S_ISDIR(st.st_mode)) return set_error(KF_ERR_ARG, std::string("not a directory: ") + dir);
    }
    jit_set_cache_dir(dir ? dir : "", dir == nullptr);
    return KF_OK;
}

kf_status kf_jit_stats(int64_t* modules, int64_t* kernels_compiled) {
    Registry& reg = registry();
    std::lock_guard<std::mutex> lock(reg.mu);
    if (modules) *modules = (int64_t)reg.modules.size();
    if (kernels_compiled) *kernels_compiled = (int64_t)reg.compiled.size();
    return KF_OK;
}

kf_status kf_quantize_rows(const float* A, int64_t rows, int64_t cols, int64_t lda, int32_t dtype, void* codes,
                           int64_t ldq, float* scales, void* stream) {
    if (!A || !codes || !scales) return set_error(KF_ERR_ARG, "null argument");
    if (rows < 1 || cols < 1 || lda < cols || ldq < cols) return set_error(KF_ERR_ARG, "bad sizes");
    if (rows > 0x7fffffff) return set_error(KF_ERR_ARG, "more than 2^31 - 1 rows");
    if (dtype != KF_BF16 && dtype != KF_FP8_E4M3) return set_error(KF_ERR_ARG, "dtype must be KF_BF16 or KF_FP8_E4M3");
    const int es = dtype_size(dtype);
    if ((uintptr_t)codes % 16 || (ldq * es) % 16) return set_error(KF_ERR_ALIGN, "codes need 16-byte aligned rows");
    if ((uintptr_t)A % 4 || (uintptr_t)scales % 4) return set_error(KF_ERR_ALIGN, "A and scales need 4-byte alignment");
    const size_t abytes = (size_t)((rows - 1) * lda + cols) * 4;
    if (overlap(A, abytes, codes, (size_t)(rows * ldq * es)) || overlap(A, abytes, scales, (size_t)rows * 4))
        return set_error(KF_ERR_ALIAS, "codes or scales overlap A");
    hipError_t e = launch_quantize_rows(A, rows, cols, lda, dtype == KF_FP8_E4M3, codes, ldq, scales,
                                        (hipStream_t)stream);
    if (e != hipSuccess) return set_error(KF_ERR_HIP, hipGetErrorString(e));
    return KF_OK;
}

kf_status kf_util_fill_uniform(float* dst, int64_t rows, int64_t cols, int64_t ld, uint64_t key, float pad,
                               void* stream) {
    if (!dst || rows < 0 || cols < 0 || ld < cols) return set_error(KF_ERR_ARG, "bad argument");
    hipError_t e = launch_fill_uniform(dst, rows, cols, ld, key, pad, (hipStream_t)stream);
    if (e != hipSuccess) return set_error(KF_ERR_HIP, hipGetErrorString(e));
    return KF_OK;
}

kf_status kf_util_stream(int32_t kind, void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src || (uintptr_t)dst % 16 || (uintptr_t)src % 16) return set_error(KF_ERR_ARG, "null or unaligned buffer");
    if (kind == 0) {
        if (bytes % 16) return set_error(KF_ERR_ARG, "read reference needs a multiple of 16 bytes");
    } else if (kind == 1) {
        if (bytes % 65536) return set_error(KF_ERR_ARG, "copy reference needs a multiple of 64 KiB");
        if (overlap(dst, bytes, src, bytes)) return set_error(KF_ERR_ALIAS, "copy reference buffers overlap");
    } else {
        return set_error(KF_ERR_ARG, "kind must be 0 (read) or 1 (copy)");
    }
    hipError_t e = launch_stream(kind, dst, src, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return set_error(KF_ERR_HIP, hipGetErrorString(e));
    return KF_OK;
}

kf_status kf_util_copy(void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src || bytes % 16 || (uintptr_t)dst % 16 || (uintptr_t)src % 16)
        return set_error(KF_ERR_ARG, "copy needs 16-byte aligned buffers and size");
    hipError_t e = launch_copy(dst, src, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return set_error(KF_ERR_HIP, hipGetErrorString(e));
    return KF_OK;
}

}  // extern "C"
