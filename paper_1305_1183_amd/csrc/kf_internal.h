// kf_internal.h -- host-side data structures of the fused BLAS sequence engine.
#pragma once
#include <cstdint>
#include <map>
#include <memory>
#include <set>
#include <string>
#include <vector>
#include <cmath>

#include "../../include/kf.h"

namespace kf {

// Kinds of values a script declares or produces (Listing 1 declarations).
enum class VK : int { Vec = 0, Mat = 1, Const = 2, DevScalar = 3 };

struct Value {
    VK kind = VK::Vec;
    int64_t n = 0;                 // vector length
    int64_t rows = 0, cols = 0, ld = 0;
    int dtype = 0;                 // matrices: KF_F32, KF_BF16, KF_FP8_E4M3
    int scale = -1;                // quantised matrices: value id of the row-scale vector
    // Matrices declared column-major: rows/cols/ld describe the storage, the
    // row-major transpose of the declared matrix; calls are recorded on it.
    bool colmajor = false;
    float cval = 0.f;              // kf_const value
    int producer = -1;             // call index, -1 for declared values
    bool input = false, output = false;
    std::vector<int> consumers;    // call indices (one entry per use)
};

// Elementary calls (Section 3.3).
enum class Op : int { Scal = 0, Axpy = 1, Dot = 2, Gemv = 3, Gemtv = 4, Ger = 5 };

const char* op_name(Op op);

struct Call {
    Op op = Op::Scal;
    int alpha = -1, beta = -1;     // scalar values (-1 = none)
    int in[3] = {-1, -1, -1};      // operand values, see kf.h
    int out = -1;
};

struct Script {
    std::vector<Value> values;
    std::vector<Call> calls;
};

// Iteration space of a call: BLAS-1 calls iterate over a vector of length n,
// BLAS-2 calls over an rows x cols matrix (nesting depth 1 vs 2, Section 3.2).
struct Space {
    bool mat = false;
    int64_t a = 0, b = 0;          // n (vec) or rows, cols (mat)
    bool operator==(const Space& o) const { return mat == o.mat && a == o.a && b == o.b; }
    bool operator<(const Space& o) const {
        if (mat != o.mat) return mat < o.mat;
        if (a != o.a) return a < o.a;
        return b < o.b;
    }
};
Space call_space(const Script& s, int c);
bool is_reduction(Op op);

// ---- legality and enumeration (plan.cpp) ----------------------------------
// Reason a call set cannot be one kernel (empty = legal).
std::string block_illegal_reason(const Script& s, const std::vector<int>& calls);
bool partition_acyclic(const Script& s, const std::vector<int>& part, int nk);
// Enumerate legal partitions; part[i] = kernel id of call i (ids numbered in
// order of first call). Fewest kernels first, capped at max_plans.
std::vector<std::vector<int>> enumerate_partitions(const Script& s, int max_plans);
// The legal partition with the fewest kernels (ties: first enumerated).
std::vector<int> fused_partition(const Script& s);
std::vector<int> unfused_partition(const Script& s);
// Kernel ids in a dependency-respecting order; calls of each kernel in
// recording order (a topological order of the SSA script).
std::vector<std::vector<int>> kernels_in_order(const Script& s, const std::vector<int>& part);

// ---- implementation parameters ---------------------------------------------
// sched 1 = row-resident; dyn: rows, cols and leading dimensions are kernel
// arguments (a plan compiled with KF_COMPILE_RUNTIME_SHAPE), not constants
struct MatParams { int k = 0, waves = 0, group = 0, rows = 0, sched = 0, unit = 0; bool dyn = false; };
struct VecParams { int unroll = 0, threads = 0, grid = 0; };
// e_per_unit: matrix elements per 16-byte load unit of the kernel (4 for FP32,
// 8 with a BF16 matrix, 16 with an FP8 matrix).
MatParams default_mat_params(int64_t rows, int64_t cols, const MatParams& req, int e_per_unit = 4);
int dtype_size(int dtype);
// Geometry of a row-resident kernel on a rows x cols matrix after defaults:
// W waves (WP: W rounded up to a power of two), KP float4 per lane per row,
// G rows per group, R rows per workgroup.
struct RowresGeom { int W = 0, WP = 0, KP = 0, G = 0; int64_t R = 0; };
RowresGeom rowres_geometry(int64_t rows, int64_t cols, const MatParams& p);
// Elements per 16-byte unit of the kernel made of `calls` (smallest element size
// of the matrices it loads).
int kernel_unit_elems(const Script& s, const std::vector<int>& calls, int req = 0);
bool kernel_has_quantized(const Script& s, const std::vector<int>& calls);
VecParams default_vec_params(int64_t n, const VecParams& req);

// ---- code generation (codegen.cpp) --------------------------------------------
enum class ArgKind : int {
    MatIn, MatOut, VecIn, VecOut, ConstScalar, DevScalarIn, DevScalarOut, Workspace,
    ShapeM, ShapeN, MatLd      // runtime-shape plans: rows, cols, leading dimension of matrix `value`
};
struct KArg { ArgKind kind; int value; };   // value id (or -1 for the workspace)

// One HIP kernel launch: the main pass of a plan kernel, or the pass that
// finishes its cross-workgroup reductions.
struct Launch {
    std::string name;              // extern "C" symbol
    std::vector<KArg> args;        // launch argument order
    int grid = 0, block = 0;
    uint64_t bytes_read = 0, bytes_written = 0;   // algorithmic HBM bytes of this launch
    // Runtime-shape plans compute the grid from the shape of each run:
    // dyn_grid 1 = strips x row blocks (S NB), 2 = finishing launch (row blocks
    // of rows plus column groups of 64 float4).
    int dyn_grid = 0;
    long dyn_c = 0, dyn_r = 0, dyn_fwb = 0;
    bool dyn_rpart = false, dyn_cpart = false;
};

struct KernelCode {
    std::string name;              // name of the main launch (unique per text)
    std::string source;            // text of every launch (without the building blocks)
    std::vector<Launch> launches;  // main pass, then the finishing pass if any
    size_t ws_floats = 0;          // partial-sum floats this kernel needs
    size_t lds_bytes = 0;          // static LDS per workgroup of the main pass
    uint64_t bytes_read = 0, bytes_written = 0;
    std::string params_json;
    std::vector<int> calls;
    bool mat = false;
    // Row-resident kernels: the generator's estimate of the VGPRs per lane a row
    // group keeps live, and whether it exceeds the register budget (such a
    // kernel likely spills to scratch memory)
    int reg_estimate = 0;
    bool over_budget = false;
};
KernelCode generate_kernel(const Script& s, const std::vector<int>& calls,
                           const std::vector<int>& part, const MatParams& mp,
                           const VecParams& vp);
// Does the call set need the row-resident schedule (a gemv result feeding a
// gemtv of the same kernel)?
bool needs_rowres(const Script& s, const std::vector<int>& calls);
// Single-routine probe kernel (one launch; args: src, dst, sink): strip or
// row-resident geometry (mp.sched), holding extra_kb KiB of LDS besides its own.
KernelCode generate_probe(int routine, int64_t rows, int64_t cols, const MatParams& mp,
                          const VecParams& vp, int extra_kb);
// KF_FEATURE_DIM features of one plan kernel.
void kernel_features(const Script& s, const KernelCode& kc, const std::vector<int>& part,
                     const MatParams& mp, const VecParams& vp, float* f);
// Operand-level byte accounting of one kernel (reads, writes) in HBM.
void kernel_bytes(const Script& s, const std::vector<int>& calls, const std::vector<int>& part,
                  uint64_t* rd, uint64_t* wr);

// ---- JIT (jit.cpp) ------------------------------------------------------------
const std::string& blocks_source();
// Compile one plan kernel (all its launches, one translation unit) to a gfx950
// code object, through the memory/disk cache. Returns false and fills log on
// failure.
bool jit_compile_one(const KernelCode& k, std::string* code_object, std::string* log);
// Identity of the disk-cache file holding kernel k ("" if not cached): kernels
// compiled together share one file, which is then loaded once per process.
std::string jit_cache_ident(const KernelCode& k);

// ---- errors ---------------------------------------------------------------------
kf_status set_error(kf_status st, const std::string& msg);
// Launch every kernel of plan p on stream with ws as its workspace (at least
// kf_plan_workspace_bytes, 256-byte aligned) instead of the bound one.
kf_status run_on_workspace(kf_plan* p, void* ws, void* stream);
// KF_OK if plan p is loaded (its kernels can launch), else the error.
kf_status plan_loaded(const kf_plan* p);

// ---- plans -------------------------------------------------------------------
struct PlanKernel {
    KernelCode code;
    MatParams mp;             // implementation parameters requested for this kernel
    VecParams vp;             // (0 = library default for the shape)
    std::vector<void*> fns;   // hipFunction_t per launch
    size_t ws_off = 0;        // bytes from workspace base to this kernel's partial sums
};
// Compile (through the caches) and load a kernel (needs a GPU).
kf_status load_kernel(const KernelCode& kc, std::vector<void*>* fns);
// Compile several kernels as one translation unit into the disk cache (each
// kernel's cache entry is a link to the shared code object).
bool jit_precompile(const std::vector<const KernelCode*>& ks, std::string* log);
// Compile several kernels (distinct names) as one translation unit, without
// the disk cache; and whether a disk cache directory is configured.
bool jit_compile_together(const std::vector<const KernelCode*>& ks, std::string* code_object, std::string* log);
bool jit_cache_enabled();
// Disk cache directory for later compilations (use_env: back to KF_CACHE_DIR).
void jit_set_cache_dir(const char* dir, bool use_env);

}  // namespace kf

kf_status build_plan(const kf::Script& sc, const std::vector<int>& part, const kf_compile_opts& o,
                     kf_plan** out);

struct kf_plan {
    kf::Script s;
    std::vector<int> part;
    std::vector<kf::PlanKernel> ks;
    std::vector<void*> bind;          // per value (caller buffers)
    std::vector<float> consts;        // per value (kf_const)
    std::vector<size_t> inter_off;    // per value: workspace offset of intermediates, or SIZE_MAX
    std::vector<char> is_read, is_written;
    kf::MatParams mp;                 // plan-wide requested parameters (0 = default per shape);
    kf::VecParams vp;                 // each kernel's own are in ks[k].mp / ks[k].vp
    void* ws = nullptr;
    size_t ws_bound = 0;
    size_t ws_need = 0;
    bool loaded = false;
    int mode = 0;
    // KF_COMPILE_RUNTIME_SHAPE: every matrix has the declared storage shape
    // decl_m x decl_n; runs use rt_m x rt_n (<= declared) and per-matrix rt_ld
    bool dyn = false;
    int64_t decl_m = 0, decl_n = 0, rt_m = 0, rt_n = 0;
    std::vector<int64_t> rt_ld;
};

// Opaque C handles.
struct kf_script { kf::Script s; bool compiled_from = false; };
struct kf_planset {
    std::vector<std::vector<int>> parts;      // partition per entry
    std::vector<kf_compile_opts> params;      // implementation parameters per entry (candidates)
    kf::Script s;                             // copy of the script (candidates)
    bool candidates = false;
};
