/* kf.h -- C ABI of the fused BLAS-1/BLAS-2 sequence engine for MI355X (gfx950).
 *
 * Method: Filipovic, Madzin, Fousek, Matyska, "Optimizing CUDA Code By Kernel
 * Fusion -- Application on BLAS" (arXiv 1305.1183). A caller records a
 * *script* of elementary BLAS-1/BLAS-2 calls over declared vectors, matrices
 * and scalars (Section 4.1, Listing 1), the library builds the data-dependency
 * graph, enumerates the legal fusions (Section 3.2, Section 4.2), picks a plan
 * and compiles each kernel of the plan from gfx950 building blocks (Section
 * 4.3, Algorithms 1 and 2) at run time with hipRTC. The plan then runs on the
 * caller's HIP stream.
 *
 * Conventions
 *  - Every function returns kf_status; KF_OK is 0, errors are negative.
 *    kf_last_error() gives a thread-local message for the last failure.
 *    Out-parameters are written only on KF_OK. No C++ exception crosses the ABI.
 *  - All data is FP32. Matrices are row-major: element (i, j) of an
 *    rows x cols matrix with leading dimension ld lives at ptr[i*ld + j]; a
 *    matrix buffer holds rows*ld floats. ld must be >= cols and a multiple of
 *    4, base pointers 16-byte aligned.
 *    Columns cols..ld-1 are padding and are never read into a result nor
 *    written. Vectors are dense, 16-byte aligned, any length >= 1.
 *  - Values are SSA (Listing 1): each call returns a fresh value; declared
 *    values are inputs and are never written. Outputs must not alias inputs.
 *  - Ownership: the caller owns all device memory (operands, outputs and the
 *    workspace). The library owns host metadata and the loaded code objects.
 *  - A plan runs on one stream at a time; distinct plans are independent.
 */
#ifndef KF_H
#define KF_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t kf_status;
enum {
    KF_OK = 0,
    KF_ERR_ARG = -1,         /* null pointer, bad enum, bad handle          */
    KF_ERR_SHAPE = -2,       /* operand shapes do not match the call        */
    KF_ERR_DTYPE = -3,       /* operand kind (vector/matrix/scalar) wrong    */
    KF_ERR_ALIGN = -4,       /* pointer or leading dimension misaligned     */
    KF_ERR_ALIAS = -5,       /* an output buffer overlaps an input buffer   */
    KF_ERR_STATE = -6,       /* SSA violation, script already compiled, ... */
    KF_ERR_UNBOUND = -7,     /* kf_run with a value or workspace not bound  */
    KF_ERR_WORKSPACE = -8,   /* workspace smaller than kf_plan_workspace_bytes */
    KF_ERR_COMPILE = -9,     /* hipRTC failed; the log is in kf_last_error  */
    KF_ERR_HIP = -10,        /* a HIP runtime call failed                   */
    KF_ERR_NOMEM = -11,      /* host allocation failed                      */
    KF_ERR_UNSUPPORTED = -12,/* legal request the library does not handle  */
    KF_ERR_INTERNAL = -13
};

typedef int32_t kf_value;
#define KF_NONE ((kf_value)-1)

typedef struct kf_script kf_script;
typedef struct kf_plan kf_plan;
typedef struct kf_planset kf_planset;

/* Thread-local description of the last error (never NULL). */
const char* kf_last_error(void);
/* Library version string, e.g. "kfuse 0.1 gfx950". */
const char* kf_version(void);

/* ---- script recording (Section 4.1, Listing 1) ------------------------- */
kf_status kf_script_create(kf_script** out);
void kf_script_destroy(kf_script* s);

/* Storage formats of matrices. FP32 is the default. BF16 (upper half of an
 * IEEE single) and OCP FP8-E4M3 (1 sign, 4 exponent bits with bias 7, 3
 * mantissa bits, largest finite 448, no infinities) hold a row-scaled matrix:
 * element (i, j) stands for scale[i] * decode(q_ij), where scale is an FP32
 * vector of `rows` entries. Quantised matrices are read-only inputs of gemv,
 * gemtv and ger (whose result is FP32); arithmetic stays FP32 (the scale is
 * folded into the row dot, into the gemtv multiplier, or applied before the
 * ger update). Their ld is counted in elements and must make each row a
 * multiple of 16 bytes. */
enum { KF_F32 = 0, KF_BF16 = 1, KF_FP8_E4M3 = 2 };

/* Declarations. A vector has n >= 1 FP32 entries; a matrix is rows x cols
 * row-major with leading dimension ld (0 = cols rounded up to a multiple of 4).
 * kf_const is a host FP32 scalar passed to the kernels by value (rebindable
 * with kf_set_const); kf_scalar is an FP32 scalar in device memory. */
kf_status kf_vector(kf_script* s, int64_t n, kf_value* out);
kf_status kf_matrix(kf_script* s, int64_t rows, int64_t cols, int64_t ld, kf_value* out);
/* A matrix in either layout (Section 3.3: a matrix is a list of rows or a list
 * of columns, and transposed operations are expressed the same way).
 * layout KF_ROW_MAJOR is kf_matrix. KF_COL_MAJOR: element (i, j) at
 * ptr[j * ld + i], ld >= rows and a multiple of 4 (0 = rows rounded up to a
 * multiple of 4); the bound buffer holds cols * ld floats. The column-major
 * rows x cols matrix is the same memory as the row-major cols x rows matrix
 * A^T, so calls are recorded on that storage: gemv on A becomes gemtv on A^T
 * and the reverse, and ger(A, u, v) becomes ger(A^T, v, u) (kf_script_call
 * reports these storage-form calls). A ger result keeps the layout of its
 * input: a column-major B with ld = rows rounded up to a multiple of 4.
 * kf_value_info reports the declared rows and cols. FP32 only; KF_ERR_ARG for
 * an unknown layout, KF_ERR_SHAPE / KF_ERR_ALIGN as kf_matrix. */
enum { KF_ROW_MAJOR = 0, KF_COL_MAJOR = 1 };
kf_status kf_matrix_layout(kf_script* s, int64_t rows, int64_t cols, int64_t ld, int32_t layout,
                           kf_value* out);
/* A quantised matrix (dtype KF_BF16 or KF_FP8_E4M3; KF_F32 is kf_matrix with
 * scale KF_NONE) with its row-scale vector `scale` (an input vector of rows
 * entries). ld 0 = cols rounded up to a 16-byte row. */
kf_status kf_matrix_q(kf_script* s, int64_t rows, int64_t cols, int64_t ld, int32_t dtype,
                      kf_value scale, kf_value* out);
/* Fill the storage of a quantised matrix from FP32 data on the device (a
 * caller that holds an FP32 matrix and wants BF16 or FP8-E4M3 storage for
 * kf_matrix_q). A: rows x cols FP32, element (i, j) at A[i * lda + j]
 * (lda >= cols). codes: rows x ldq elements of 2 bytes (KF_BF16) or 1 byte
 * (KF_FP8_E4M3), ldq >= cols with 16-byte rows; columns cols..ldq-1 are set
 * to code 0. scales: rows floats. Every code is the nearest value, ties to
 * even, of the exact number it stands for:
 *   KF_BF16      scale_i = 1 and the code is a_ij rounded to BF16 (the 16 high
 *                bits of a binary32 value); values beyond the largest BF16
 *                round to infinity and NaN stays a quiet NaN;
 *   KF_FP8_E4M3  scale_i = amax_i / 448 (amax over the row's finite entries,
 *                correctly rounded binary32 division; 1 for a row of zeros),
 *                and the code is the exact quotient a_ij / scale_i rounded to
 *                E4M3, saturating at +-448 (0x7e | sign); NaN gives 0x7f | sign.
 * Element (i, j) of the stored matrix stands for scale_i * decode(code_ij).
 * Asynchronous on `stream`; allocates nothing. KF_ERR_ARG for null pointers,
 * sizes < 1 or an unknown dtype, KF_ERR_ALIGN for unaligned codes or rows,
 * KF_ERR_ALIAS if codes or scales overlap A. */
kf_status kf_quantize_rows(const float* A, int64_t rows, int64_t cols, int64_t lda, int32_t dtype, void* codes,
                           int64_t ldq, float* scales, void* stream);
kf_status kf_const(kf_script* s, float v, kf_value* out);
kf_status kf_scalar(kf_script* s, kf_value* out);
/* Listing 1 `input` and `return`. Declared values must be marked input before
 * they are used; any value may be marked output (results are written to the
 * buffer bound to it). */
kf_status kf_input(kf_script* s, kf_value v);
kf_status kf_output(kf_script* s, kf_value v);

/* Elementary calls (all out-of-place, Section 3.3 and Table 1). alpha and beta
 * are scalar values (kf_const, kf_scalar or a kf_dot result).
 *   kf_scal : y = alpha x                            (BLAS-1 map)
 *   kf_axpy : z = alpha x + y                        (BLAS-1 map)
 *   kf_dot  : r = x^T y          (device scalar)     (map + reduce)
 *   kf_gemv : y = alpha A x + beta y0    (y0 may be KF_NONE; eq. (2))
 *   kf_gemtv: y = alpha A^T x + beta y0  (A viewed as a list of columns)
 *   kf_ger  : B = A + alpha u v^T        (rank-1 update; B gets ld of A's
 *                                         cols rounded up to a multiple of 4) */
kf_status kf_scal(kf_script* s, kf_value alpha, kf_value x, kf_value* y);
kf_status kf_axpy(kf_script* s, kf_value alpha, kf_value x, kf_value y, kf_value* z);
kf_status kf_dot(kf_script* s, kf_value x, kf_value y, kf_value* r);
kf_status kf_gemv(kf_script* s, kf_value alpha, kf_value A, kf_value x, kf_value beta,
                  kf_value y0, kf_value* y);
kf_status kf_gemtv(kf_script* s, kf_value alpha, kf_value A, kf_value x, kf_value beta,
                   kf_value y0, kf_value* y);
kf_status kf_ger(kf_script* s, kf_value alpha, kf_value A, kf_value u, kf_value v,
                 kf_value* B);

/* Shape of a value: kind 0 vector (d0 = n), 1 matrix (d0 = rows, d1 = cols,
 * d2 = ld in elements), 2 const scalar, 3 device scalar. */
kf_status kf_value_info(const kf_script* s, kf_value v, int32_t* kind, int64_t* d0,
                        int64_t* d1, int64_t* d2);
/* Layout of matrix value v (KF_ROW_MAJOR or KF_COL_MAJOR); KF_ERR_DTYPE if v
 * is not a matrix. */
kf_status kf_value_layout(const kf_script* s, kf_value v, int32_t* layout);
kf_status kf_script_num_calls(const kf_script* s, int32_t* n);
/* Call i of the script: op (0 scal, 1 axpy, 2 dot, 3 gemv, 4 gemtv, 5 ger),
 * scalar operands alpha and beta, operands in[0..2] as documented for the
 * recorders (KF_NONE where absent) and the output value. */
kf_status kf_script_call(const kf_script* s, int32_t i, int32_t* op, kf_value* alpha,
                         kf_value* beta, kf_value* in3, kf_value* out);

/* ---- compilation (Section 4.2: fusions, implementations, combinations) -- */
enum {
    KF_MODE_UNFUSED = 0,      /* one kernel per call                           */
    KF_MODE_FUSED = 1,        /* the legal partition with fewest kernels       */
    /* The three ranking modes below cost every kernel of every candidate on
     * its own and combine, per partition, the cheapest implementation of each
     * kernel (the "combination of fusion implementations" of Section 4.2:
     * kernels of one plan may use different parameter points); the partition
     * whose combination costs least wins (ties within 0.1%: fewer kernels). */
    KF_MODE_ADDITIVE = 2,     /* costs from the additive routine predictor      */
    KF_MODE_LEARNED = 3,      /* costs from the learned cost model (opts.model);
                                 with opts.top_k > 1 the top_k candidates by
                                 predicted plan time, and those of the predicted
                                 combination, are timed kernel by kernel (needs
                                 opts.bind_*) and the measured times combined  */
    KF_MODE_EXHAUSTIVE = 4,   /* every candidate timed kernel by kernel on
                                 opts.stream with the buffers of opts.bind_*,
                                 the measured times combined                   */
    KF_MODE_PARTITION = 5     /* the partition given in opts.partition         */
};
enum {
    KF_COMPILE_NO_LOAD = 1,       /* stop after hipRTC (no GPU needed): build checks */
    KF_COMPILE_CODEGEN_ONLY = 2,  /* generate code but do not compile: features, bytes,
                                     additive predictions (kf_run is refused) */
    KF_COMPILE_RUNTIME_SHAPE = 4  /* kernels take rows, cols and each matrix's leading
                                     dimension as arguments (kf_plan_set_shape) */
};
struct kf_routine_entry;
/* Implementation parameters of one plan kernel (fields as in kf_compile_opts;
 * 0 = take the value of the enclosing kf_compile_opts). */
typedef struct kf_impl_params {
    int32_t mat_k, mat_waves, mat_group, mat_rows, mat_sched, mat_unit;
    int32_t vec_unroll, vec_threads, vec_grid;
} kf_impl_params;
typedef struct kf_compile_opts {
    int32_t mode;            /* KF_MODE_*                                         */
    int32_t flags;           /* KF_COMPILE_*                                      */
    /* Implementation parameters; 0 = library default for the shape.
     * mat_k: float4 columns per lane (1, 2, 4); mat_waves: waves per workgroup
     * (1..16); mat_group: rows per wave step (1, 2, 4, 8, 16); mat_rows: rows
     * per workgroup (multiple of mat_waves*mat_group). vec_unroll: float4 per
     * thread per step (1, 2, 4, 8); vec_threads: 64..1024; vec_grid: max
     * workgroups (grid-stride beyond). */
    int32_t mat_k, mat_waves, mat_group, mat_rows;
    int32_t vec_unroll, vec_threads, vec_grid;
    /* BLAS-2 schedule: 0 = column strips x row blocks (mat_k used), 1 = row-
     * resident (a workgroup owns whole rows, mat_waves split the columns,
     * cols <= 32768). Kernels in which a gemv result feeds a gemtv of the same
     * kernel always use the row-resident schedule. */
    int32_t mat_sched;
    /* KF_MODE_PARTITION: partition[i] = kernel id of call i (calls numbered in
     * recording order), ids 0..K-1. */
    const int32_t* partition;
    int32_t partition_len;
    /* Ranking modes: the number of partitions considered (0 = 64) and the
     * implementation-parameter points to cross them with (NULL: every
     * environment present in the routine table for KF_MODE_ADDITIVE, the
     * default grid of kf_candidates for the other two). KF_MODE_ADDITIVE: the
     * routine table. */
    const struct kf_routine_entry* table;
    int32_t table_len;
    int32_t max_partitions;
    const struct kf_compile_opts* grid;
    int32_t grid_len;
    /* Quantised matrices (BF16, FP8): elements per lane and load. 4 = four
     * elements (4 or 8 bytes), laid out like FP32; 16 = one 16-byte load (8
     * BF16 or 16 FP8 elements); 0 = four when the kernel expands the matrix
     * into an FP32 one (ger), else 16. FP32 kernels ignore it. */
    int32_t mat_unit;
    /* KF_MODE_LEARNED: the trained model (not owned, with bound memory).
     * KF_MODE_LEARNED with top_k > 1 and KF_MODE_EXHAUSTIVE time candidates on
     * `stream` with the caller's device buffers: bind_ptrs[i] is bound to
     * script value bind_values[i] (every input and output, as for kf_bind; the
     * inputs are read, the outputs overwritten), and the plans' workspace is
     * opts.workspace (below). */
    struct kf_costmodel* model;
    void* stream;
    const int32_t* bind_values;
    void* const* bind_ptrs;
    int32_t bind_len;
    int32_t top_k;
    /* Per-kernel parameters (modes UNFUSED, FUSED, PARTITION): entry i applies
     * to the i-th kernel of the plan in launch order (the order of
     * kf_plan_describe); kernels past kernel_params_len, and zero fields, use
     * the parameters above (mat_rows is the rows per workgroup in both
     * schedules, so a plan-wide value reaches row-resident kernels too).
     * KF_ERR_ARG if there are more entries than kernels. Not owned; read
     * during the call only. */
    const kf_impl_params* kernel_params;
    int32_t kernel_params_len;
    /* KF_MODE_EXHAUSTIVE and KF_MODE_LEARNED with top_k > 1: once this many
     * milliseconds of wall clock have passed since timing began, no further
     * candidate is timed and those timed so far (at least one) are combined;
     * 0 = no limit. */
    int32_t time_budget_ms;
    /* The timed modes' plan workspace: caller device memory, 256-byte aligned,
     * workspace_bytes long (kf_compile_workspace_bytes gives the size every
     * candidate fits in). A candidate that needs more is not timed;
     * KF_ERR_WORKSPACE if none fits. */
    void* workspace;
    size_t workspace_bytes;
} kf_compile_opts;

/* Fill opts with defaults (mode KF_MODE_FUSED, all parameters 0). */
void kf_compile_opts_init(kf_compile_opts* o);
/* Compile a plan. The plan deep-copies what it needs from the script. */
kf_status kf_compile(const kf_script* s, const kf_compile_opts* opts, kf_plan** out);
/* The largest kf_plan_workspace_bytes among the candidates that the timed
 * modes of kf_compile would time with these opts (partitions and grid as in
 * KF_MODE_EXHAUSTIVE); code generation only, no GPU needed. */
kf_status kf_compile_workspace_bytes(const kf_script* s, const kf_compile_opts* opts, size_t* bytes);
void kf_plan_destroy(kf_plan* p);

/* ---- plan-space enumeration (Section 4.2) ------------------------------- */
/* Enumerate the legal partitions of the script's calls into kernels (rules of
 * Section 3.2: same iteration space, no reduction result consumed in the
 * kernel that computes it, convex and acyclic, fusions must share data),
 * at most max_plans of them, fewest kernels first. */
kf_status kf_enumerate(const kf_script* s, int32_t max_plans, kf_planset** out);
void kf_planset_destroy(kf_planset* ps);
kf_status kf_planset_count(const kf_planset* ps, int32_t* n);
/* partition[call] = kernel id for plan i (len = number of calls). */
kf_status kf_planset_get(const kf_planset* ps, int32_t i, int32_t* partition, int32_t len);

/* Candidate plans (Section 4.2, fusion implementations): the first
 * max_partitions legal partitions crossed with the implementation parameter
 * points grid[0..grid_len) (only their implementation parameters are read, as
 * one point for every kernel of a candidate; kernel_params and the other fields
 * of the entries are ignored; only the fields of the kernel classes present
 * matter, and candidates whose kernels would be identical are listed once). Each candidate uses one point for all its
 * kernels; the ranking modes of kf_compile combine, per partition, kernels of
 * different candidates. grid = NULL takes 32 points: the shape-dependent
 * defaults, six fixed strip shapes and the row-resident schedule, crossed with
 * the defaults and three fixed BLAS-1 shapes. */
kf_status kf_candidates(const kf_script* s, int32_t max_partitions, const kf_compile_opts* grid,
                        int32_t grid_len, kf_planset** out);
/* Parameters of candidate i (mode = KF_MODE_PARTITION, partition pointing into
 * the planset, valid while it lives). */
kf_status kf_planset_params(const kf_planset* ps, int32_t i, kf_compile_opts* out);
/* Compile candidate i with `flags` (KF_COMPILE_*). */
kf_status kf_planset_compile(const kf_planset* ps, int32_t i, int32_t flags, kf_plan** out);
/* Compile the kernels of candidates idx[0..n) as one hipRTC unit into the
 * KF_CACHE_DIR disk cache (no GPU needed); later kf_planset_compile calls in
 * any process find them there. */
kf_status kf_planset_precompile(const kf_planset* ps, const int32_t* idx, int32_t n);
/* Additive predictions (us) of every candidate (no compilation). */
kf_status kf_planset_predict_additive(const kf_planset* ps, const kf_routine_entry* table,
                                      int32_t table_len, float* pred_us);

/* ---- bind and run --------------------------------------------------------- */
/* Bytes of device workspace the plan needs: partial sums of reductions and
 * intermediate values that a later kernel of the plan reads from HBM. */
kf_status kf_plan_workspace_bytes(const kf_plan* p, size_t* bytes);
/* Bind a device buffer to a vector, matrix or device-scalar value. Checks
 * alignment and, for outputs, overlap with every bound input. */
kf_status kf_bind(kf_plan* p, kf_value v, void* dev_ptr);
kf_status kf_bind_workspace(kf_plan* p, void* dev_ptr, size_t bytes);
/* Change a kf_const value without recompiling. */
kf_status kf_set_const(kf_plan* p, kf_value v, float value);

/* Runtime-shape plans (KF_COMPILE_RUNTIME_SHAPE; the same problem at many
 * sizes without recompiling, e.g. one plan per size class of a batch). Every
 * matrix of the script must have one storage shape rows x cols (the
 * declared, largest shape) and every vector rows or cols entries; every call
 * must be a BLAS-2 call, and the kernels use the strip schedule (a kernel that
 * needs whole rows in a workgroup is KF_ERR_UNSUPPORTED). The workspace is
 * sized for the declared shape.
 * kf_plan_set_shape: run at rows x cols (1 .. declared; square if declared
 * square); unbinds every buffer, since their sizes change. Vectors then hold
 * rows or cols entries (as declared), matrices rows x ld elements.
 * kf_bind_matrix: bind a matrix with its own leading dimension ld (in
 * elements, >= cols of the current shape, rows of 16 bytes); kf_bind uses the
 * declared ld. Errors: KF_ERR_STATE for a plan without runtime shape,
 * KF_ERR_SHAPE, KF_ERR_ALIGN, KF_ERR_DTYPE, KF_ERR_ALIAS. */
kf_status kf_plan_set_shape(kf_plan* p, int64_t rows, int64_t cols);
kf_status kf_bind_matrix(kf_plan* p, kf_value v, void* dev_ptr, int64_t ld);
/* Run a runtime-shape plan over `count` instances, one after another on
 * `stream`: instance i has shape shapes[2i] x shapes[2i + 1] and binds
 * values[j] to ptrs[i * nvals + j] (matrices with leading dimension
 * lds[i * nvals + j], or the declared ld when lds is NULL); the workspace
 * bound to the plan serves every instance. Same as kf_plan_set_shape, the
 * binds and kf_run per instance, without host round trips in between.
 * Leaves the last instance's shape and buffers bound. */
kf_status kf_plan_run_many(kf_plan* p, int64_t count, const int64_t* shapes, int32_t nvals, const kf_value* values,
                           void* const* ptrs, const int64_t* lds, void* stream);
/* Launch every kernel of the plan on `stream` (a hipStream_t; NULL = the null
 * stream). Asynchronous; allocates nothing and keeps no state on the device
 * between runs, so repeated runs and graph replays need no preparation. A
 * kernel whose reductions span several workgroups is two launches: the main
 * pass writes partial sums to the workspace, a small second pass adds them
 * in a fixed order (the final reduction "by extra kernel", Section 3.2.2). */
kf_status kf_run(kf_plan* p, void* stream);
/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): run the plan as
 * kf_run does, but with a fixed array of KF_NOALLOC_SCRATCH_BYTES (32 MiB)
 * that the library holds on each GPU it runs on, until the process ends, as
 * the workspace (partial sums of reductions and intermediates). No workspace
 * need be bound; the caller still binds every input and output. Allocates
 * nothing. A plan whose kf_plan_workspace_bytes exceeds the array is refused
 * with KF_ERR_WORKSPACE: every fused plan of the Table 1 sequences on square
 * matrices up to 32768 fits, unfused plans that keep a matrix intermediate do
 * not. Nothing in the array has to start at zero: each run writes every
 * partial before it reads it. All calls on one GPU share that GPU's array and
 * it keeps the last call's contents, so calls that overlap in time on one GPU
 * (two streams, two threads, two plans) race and give wrong results: the
 * caller serialises them. The array used is the current device's, which must
 * be the device the plan was loaded on. Errors: as kf_run, plus
 * KF_ERR_WORKSPACE (too large) and KF_ERR_HIP (the array's address could not
 * be looked up). */
#define KF_NOALLOC_SCRATCH_BYTES (32u << 20)
kf_status kf_run_noalloc(kf_plan* p, void* stream);
/* Launch only kernel k of the plan (in plan order), e.g. to time one kernel.
 * Its inputs must already hold valid data. */
kf_status kf_run_kernel(kf_plan* p, int32_t k, void* stream);
/* Number of HIP launches of kernel k (1, or 2 with a finishing pass), and
 * launch l of kernel k alone (main pass l = 0, finishing pass l = 1). */
kf_status kf_plan_num_launches(const kf_plan* p, int32_t k, int32_t* n);
kf_status kf_run_launch(kf_plan* p, int32_t k, int32_t l, void* stream);
/* Time the plan: `warmup` untimed runs, then `reps` runs each bracketed by HIP
 * events; returns the median in microseconds. Synchronises the stream. */
kf_status kf_time_plan(kf_plan* p, void* stream, int32_t warmup, int32_t reps,
                       float* median_us);
/* Time each kernel inside whole runs of the plan: `warmup` untimed runs, then
 * `reps` runs in which HIP events bracket every kernel (all its launches);
 * us[k] receives the median for plan kernel k (us holds kf_plan_num_kernels
 * floats). Synchronises the stream. */
kf_status kf_time_plan_kernels(kf_plan* p, void* stream, int32_t warmup, int32_t reps, float* us);
/* The implementation parameters kernel k was generated with, after defaults
 * for its shape were applied (mat_* for BLAS-2 kernels, vec_* for BLAS-1;
 * mat_unit as requested, and only for kernels that load a BF16 or FP8
 * matrix). */
kf_status kf_plan_kernel_params(const kf_plan* p, int32_t k, kf_impl_params* out);

/* ---- introspection -------------------------------------------------------- */
/* JSON description (kernels, calls, parameters, grid, bytes). Row-resident
 * kernels also report "register_estimate" (VGPRs per lane a row group keeps
 * live, as the generator estimates it) and "over_register_budget". Writes at
 * most cap bytes (NUL-terminated) and the needed size to *needed. */
kf_status kf_plan_describe(const kf_plan* p, char* buf, size_t cap, size_t* needed);
/* Algorithmic HBM bytes of one run: every operand counted once per kernel
 * that reads or writes it in HBM (the paper's "really transferred" bytes,
 * Section 5.2); workspace traffic is excluded. */
kf_status kf_plan_bytes(const kf_plan* p, uint64_t* read, uint64_t* written);
kf_status kf_plan_num_kernels(const kf_plan* p, int32_t* n);
/* HIP source of kernel k of the plan (for inspection and tests). */
kf_status kf_plan_source(const kf_plan* p, int32_t k, char* buf, size_t cap, size_t* needed);
/* Launch geometry of kernel k: grid (workgroups) and block (threads). */
kf_status kf_plan_kernel_geometry(const kf_plan* p, int32_t k, int32_t* grid, int32_t* block);

/* ---- plan ranking (Section 4.2: performance prediction) ------------------- */
/* Routines of the additive predictor. The paper benchmarks each routine of an
 * elementary function (loads, compute, stores) in a simulated fusion
 * environment and predicts a fusion as max(sum of transfer times, sum of
 * compute times). Here a routine is timed alone by a probe kernel with the
 * workgroup geometry and serial iterations of a real kernel:
 *   LOAD_MAT / STORE_MAT     stream a matrix from / to HBM (per element),
 *   COMPUTE_GEMV/GEMTV/GER   the call's arithmetic on on-chip (LDS) tiles,
 *   LOAD_VEC / STORE_VEC     stream a vector (per entry),
 *   COMPUTE_SCAL/AXPY/DOT    the call's arithmetic on register data,
 *   FINISH                   one finishing launch (per launch).            */
enum {
    KF_ROUTINE_LOAD_MAT = 0, KF_ROUTINE_STORE_MAT = 1, KF_ROUTINE_COMPUTE_GEMV = 2,
    KF_ROUTINE_COMPUTE_GEMTV = 3, KF_ROUTINE_COMPUTE_GER = 4, KF_ROUTINE_LOAD_VEC = 5,
    KF_ROUTINE_STORE_VEC = 6, KF_ROUTINE_COMPUTE_SCAL = 7, KF_ROUTINE_COMPUTE_AXPY = 8,
    KF_ROUTINE_COMPUTE_DOT = 9, KF_ROUTINE_FINISH = 10, KF_NUM_ROUTINES = 11
};
/* One entry of the routine table: the environment and the time per unit in
 * microseconds (per matrix element, per vector entry, or per launch for
 * FINISH). Environments ("simulated fusion environments", Section 4.2):
 *   cls 0  BLAS-1: env = (vec_unroll, vec_threads, vec_grid, 0);
 *   cls 1  BLAS-2 column strips: env = (mat_k, mat_waves, mat_group, mat_rows);
 *   cls 2  BLAS-2 row-resident: env = (mat_waves, mat_group, mat_rows, 0) as
 *          requested (0 = the default for the shape);
 * and lds_kb, the extra LDS the probe workgroup held besides its own (0, 16,
 * 32, 64 KiB): a fused kernel's LDS use lowers how many of its workgroups a CU
 * holds, so a kernel is priced in the environment whose lds_kb is nearest to
 * its own LDS bytes. */
typedef struct kf_routine_entry {
    int32_t cls;          /* 0, 1, 2 as above */
    int32_t env[4];
    int32_t routine;      /* KF_ROUTINE_* */
    int32_t lds_kb;
    float us_per_unit;
} kf_routine_entry;
/* Time routine `routine` alone on a rows x cols matrix (BLAS-2 routines; ld =
 * cols, a multiple of 4) or on a rows-entry vector (BLAS-1 routines; cols
 * ignored) with the implementation parameters of `params` (mode ignored;
 * mat_sched 1 gives the row-resident geometry: whole rows per workgroup, a
 * workgroup barrier per row group for the row dot) while each workgroup holds
 * extra_lds_kb KiB of LDS besides its own (0 .. 96). `buf` is a device buffer
 * of at least rows*cols*4 + 65536 bytes (vector: rows*4 + 65536); its
 * contents are overwritten. Median of `reps` runs. KF_ROUTINE_FINISH is not a
 * probe (time a finishing launch instead). */
kf_status kf_routine_time(int32_t routine, int64_t rows, int64_t cols,
                          const kf_compile_opts* params, int32_t extra_lds_kb, void* buf, size_t buf_bytes,
                          void* stream, int32_t warmup, int32_t reps, float* median_us);
/* Additive prediction of a plan: for each kernel, max(t_t, t_c) with t_t the
 * sum of its transfer routines (every matrix and vector it moves through HBM)
 * and t_c the sum of its compute routines (one per call), plus one FINISH per
 * finishing launch; summed over kernels. Entries are matched on class and
 * environment, then the nearest extra LDS (row-resident kernels use the cls 2
 * entries; a table without any prices them with its first BLAS-2
 * environment); KF_ERR_UNSUPPORTED if a needed entry is missing. A kernel
 * over the generator's register budget ("over_register_budget" in
 * kf_plan_describe) gets 1e9 us added, so that it ranks after every
 * implementation within budget (Section 4.2 prunes implementations that need
 * more on-chip memory than another of the same fusion). */
kf_status kf_predict_additive(const kf_plan* p, const kf_routine_entry* table, int32_t n,
                              float* us);

/* Features of every kernel of a plan for the learned cost model: `rows` x
 * KF_FEATURE_DIM floats, row k for plan kernel k (in plan order). Features:
 *  0 BLAS-2 flag; 1 log2 rows (or n); 2 log2 cols; 3 log2 bytes read;
 *  4 log2 bytes written; 5 log2 bytes saved against one kernel per call;
 *  6..11 number of scal, axpy, dot, gemv, gemtv, ger calls; 12/13 matrices
 *  loaded/stored; 14/15 vectors (and device scalars) loaded/stored; 16 k;
 *  17 waves; 18 log2 group; 19 log2 rows per workgroup; 20 vec unroll;
 *  21 vec threads/256; 22 log2 vec grid; 23 log2 workgroups of the main
 *  launch; 24 log2 threads per workgroup; 25 launches; 26 log2 workspace
 *  floats; 27 LDS bytes/4096; 28 calls; 29 chained y0; 30 log2 elements of
 *  the iteration space; 31 written share of the bytes.
 * *nk receives the number of kernels; KF_ERR_ARG if rows < *nk. */
#define KF_FEATURE_DIM 32
kf_status kf_plan_features(const kf_plan* p, float* out, int32_t rows, int32_t* nk);

/* ---- learned cost model ---------------------------------------------------- */
/* A multilayer perceptron in_dim -> hidden (x layers, ReLU) -> 1 that maps the
 * (normalised) features of one plan kernel to its log run time. Parameters,
 * gradients, Adam moments, inputs and the workspace are caller-owned device
 * buffers of FP32; layer l's weights are a row-major in x out matrix at
 * w_off (kf_mlp_layout) followed by its out biases at b_off. Every product runs
 * on the GPU (16x16x4 FP32 matrix-core instructions); results are
 * bit-reproducible. The stream argument is a hipStream_t. */
typedef struct kf_mlp kf_mlp;
kf_status kf_mlp_create(int32_t in_dim, int32_t hidden, int32_t layers, kf_mlp** out);
void kf_mlp_destroy(kf_mlp* m);
kf_status kf_mlp_param_count(const kf_mlp* m, int64_t* n);
kf_status kf_mlp_layout(const kf_mlp* m, int32_t layer, int64_t* w_off, int64_t* b_off,
                        int64_t* rows, int64_t* cols);
/* He-uniform weights (SplitMix64 stream from `seed`), zero biases, written to
 * a host array of kf_mlp_param_count floats. */
kf_status kf_mlp_init_params(const kf_mlp* m, uint64_t seed, float* host_params);
kf_status kf_mlp_workspace_bytes(const kf_mlp* m, int32_t batch, size_t* bytes);
/* pred[0..n) = network(X) for X of n x in_dim (row-major). */
kf_status kf_mlp_forward(const kf_mlp* m, const float* params, const float* X, int32_t n,
                         float* pred, void* ws, size_t ws_bytes, void* stream);
/* Mean squared error of network(X) against y[0..n) into *loss (device float),
 * and its gradient with respect to every parameter into grads (overwritten). */
kf_status kf_mlp_loss_grad(const kf_mlp* m, const float* params, const float* X, const float* y,
                           int32_t n, float* grads, float* loss, void* ws, size_t ws_bytes,
                           void* stream);
/* One Adam step (Kingma and Ba) with bias correction for step `step` >= 1. */
kf_status kf_mlp_adam(const kf_mlp* m, float* params, const float* grads, float* mstate,
                      float* vstate, int32_t step, float lr, float beta1, float beta2, float eps,
                      void* stream);

/* Cost model for plan ranking: the MLP above over KF_FEATURE_DIM kernel
 * features, predicting the log of a kernel's run time in microseconds; a
 * plan's prediction is the sum over its kernels of exp(prediction) plus
 * launch_us per launch (feature 25 counts launches). The object holds the
 * network's shape, the feature and target standardisation and, until device
 * memory is bound, the parameters on the host; it allocates no device memory.
 * Training and prediction need kf_costmodel_bind. Every kernel runs on the
 * caller's stream. */
typedef struct kf_costmodel kf_costmodel;
kf_status kf_costmodel_create(int32_t hidden, int32_t layers, uint64_t seed, kf_costmodel** out);
void kf_costmodel_destroy(kf_costmodel* cm);
/* Bytes of device memory for a model whose calls take up to `rows` feature
 * rows at a time (the training minibatch; predictions go in chunks of rows):
 * parameters, gradients, Adam moments, the MLP workspace, staging of
 * features, targets and predictions, and the statistics. */
kf_status kf_costmodel_workspace_bytes(const kf_costmodel* cm, int64_t rows, size_t* bytes);
/* Give the model caller-owned device memory: `mem` of at least
 * kf_costmodel_workspace_bytes(rows) bytes, 256-byte aligned, alive while the
 * model uses it. The parameters and statistics are copied into it (on
 * `stream`, which is synchronised) and live there from then on; binding new
 * memory first copies the parameters back from the old one. Errors:
 * KF_ERR_ALIGN, KF_ERR_WORKSPACE (too small), KF_ERR_HIP. */
kf_status kf_costmodel_bind(kf_costmodel* cm, void* mem, size_t bytes, int64_t rows, void* stream);
/* Train on n samples in caller device memory: X is n x KF_FEATURE_DIM floats
 * (row-major), y_log_us the n targets. Features and targets are standardised
 * with the training data's per-column mean and deviation (computed on the GPU
 * and kept in the model); MSE on the standardised log time, Adam (0.9,
 * 0.999, 1e-8) at rate lr, minibatches of `batch` (<= the bound rows) in an
 * order shuffled per epoch from `seed`. loss_per_epoch (optional host array
 * of `epochs` floats) gets the mean minibatch loss of each epoch. The stream
 * is synchronised once per minibatch. KF_ERR_UNBOUND without bound memory. */
kf_status kf_costmodel_train(kf_costmodel* cm, const float* X, const float* y_log_us, int64_t n, int32_t epochs,
                             int32_t batch, float lr, uint64_t seed, void* stream, float* loss_per_epoch);
/* log_us[i] = predicted log microseconds of feature row i; X (n x
 * KF_FEATURE_DIM) and log_us are caller device memory. Asynchronous on
 * `stream`. KF_ERR_UNBOUND without bound memory. */
kf_status kf_costmodel_predict(kf_costmodel* cm, const float* X, int64_t n, float* log_us, void* stream);
/* Predicted run times (us) of nplans plans from host feature rows (as
 * kf_plan_features writes them): plan i owns rows start[i] .. start[i + 1] - 1
 * of feats (rows x KF_FEATURE_DIM), and us[i] = sum over them of
 * exp(prediction) + launch_us * launches. The rows are staged through the
 * bound memory; synchronises `stream`. */
kf_status kf_costmodel_plan_us(kf_costmodel* cm, const float* feats, int64_t rows, const int64_t* start,
                               int32_t nplans, double* us, void* stream);
kf_status kf_costmodel_set_launch_us(kf_costmodel* cm, float us);
/* Host copies of the parameters (kf_costmodel_dims' nparams floats, the
 * kf_mlp layout; read from the bound memory after the device is
 * synchronised), the feature means and deviations (KF_FEATURE_DIM each), the
 * target mean and deviation (two doubles) and the launch term; any pointer
 * may be NULL. kf_costmodel_set installs them (and copies them into bound
 * memory). */
kf_status kf_costmodel_get(const kf_costmodel* cm, float* params, float* mu, float* sd, double* y_mu_sd,
                           float* launch_us);
kf_status kf_costmodel_set(kf_costmodel* cm, const float* params, const float* mu, const float* sd,
                           const double* y_mu_sd, float launch_us);
kf_status kf_costmodel_dims(const kf_costmodel* cm, int32_t* hidden, int32_t* layers, int64_t* nparams);
/* Binary file of the model ("KFCM", version 2, with a checksum); load creates a new model. */
kf_status kf_costmodel_save(const kf_costmodel* cm, const char* path);
kf_status kf_costmodel_load(const char* path, kf_costmodel** out);

/* ---- run-time compilation cache ------------------------------------------ */
/* Each plan kernel is compiled by hipRTC for gfx950 once per process (keyed
 * by a hash of its text); the kernels of a plan that are not loaded yet are
 * compiled together in one hipRTC invocation (and, without a disk cache, one
 * module). If the environment variable KF_CACHE_DIR names a directory, code
 * objects are also read from and written to it, so several processes can
 * share compilations. kf_jit_release unloads every loaded
 * module: all plans must have been destroyed before. kf_jit_stats reports the
 * number of loaded modules and of kernels compiled in this process. */
kf_status kf_jit_release(void);
/* Disk cache directory for later compilations, in place of KF_CACHE_DIR: an
 * existing directory, "" for no disk cache, or NULL to go back to the
 * environment variable. KF_ERR_ARG if dir is not a directory. Process-wide. */
kf_status kf_jit_set_cache_dir(const char* dir);
kf_status kf_jit_stats(int64_t* modules, int64_t* kernels_compiled);

/* ---- batched uneven sizes: one persistent launch --------------------------
 * Many independent BiCGK (q = A p, s = A^T r; Table 1) and GEMVER
 * (B = A + u1 v1^T + u2 v2^T, x = beta B^T y + z, w = alpha B x; Table 1)
 * instances, each square with 1 <= n <= 2048, run as one launch of a fixed
 * grid of workgroups that take work items from a queue: a small instance is
 * one item (for GEMVER the workgroup completes x and then computes w, so the
 * global barrier between the two kernels of the fused plan becomes a
 * workgroup barrier); a larger one is cut into row blocks whose column
 * partials are added in block order by the last block to finish. This is the
 * persistent-threads form of fusion that Section 5 leaves open.
 *
 * Layout: the library places every operand of every instance in one float
 * arena that the caller allocates (kf_batch_arena_elems floats, 256-byte
 * aligned) and fills at the offsets kf_batch_offset reports. Matrices are row
 * major with row pitch ld = round_up(n, 32) (rows start on 128-byte lines);
 * padding columns are never read as
 * data nor written. Operand ids: 0 = A, 1 = B (GEMVER output), then vectors
 * 2 + slot, BiCGK slots p, r, q, s and GEMVER slots u1, v1, u2, v2, y, z,
 * x, w (inputs first, then outputs; each n floats).
 *
 * Tile shape: instances fall into six size buckets (n <= 64, 128, 256, 512,
 * 1024, 2048). opts->tile[kind][bucket] picks the lane tile from the bucket's
 * menu (kf_batch_tile_info): entry 0 is the default, and a whole-row tile
 * lets 2^ltpr lanes share a row with k float4 chunks each, walking
 * 256 / 2^ltpr rows per step and reducing row sums every 2^lg steps; a wide
 * tile (BiCGK above n = 512) lets the four waves split each row, k float4
 * chunks per lane, 2^lg rows per step. opts->rows[kind][bucket] is the number
 * of rows per work item, a multiple of the tile's rows per step (0: the
 * library default rounded up to one); an instance with n <= rows is one item.
 * The project's autotuner chooses both per kind and bucket. opts->grid is the
 * number of persistent workgroups (0: as many as are resident on the device);
 * opts->spin_limit bounds the wait of a dependent item (0: default, about a
 * second); a wait that runs out sets error bit 1 (kf_batch_error) and the
 * item is skipped: that run's outputs are not valid, and its counters stay
 * behind until kf_batch_error (or kf_batch_bind) clears them, so call
 * kf_batch_error after a run before the next one when the results matter.
 *
 * Workspace: kf_batch_workspace_bytes bytes, 256-byte aligned, owned by the
 * caller like the arena. It holds the counters, the column partials of split
 * instances and the instance and item tables; kf_batch_bind uploads the
 * tables and clears the counters, and the launch leaves them cleared, so runs
 * and graph replays need no clearing. The library allocates no device memory.
 * Two runs of one batch must not overlap in time. */
typedef struct kf_batch kf_batch;
enum { KF_BATCH_BICGK = 0, KF_BATCH_GEMVER = 1 };
#define KF_BATCH_BUCKETS 6
typedef struct {
    int32_t rows[2][KF_BATCH_BUCKETS];
    int32_t grid;
    uint32_t spin_limit;
    int32_t tile[2][KF_BATCH_BUCKETS];
} kf_batch_opts;
/* Entry t of the tile menu of (kind, bucket): *count gets the menu's length;
 * when t < count, out[0..4] = wide (0/1), ltpr, k, lg, rows per step. Host
 * only. KF_ERR_ARG for a bad kind, bucket or t. */
kf_status kf_batch_tile_info(int32_t kind, int32_t bucket, int32_t t, int32_t* count, int32_t* out);

/* kind[i] in {KF_BATCH_BICGK, KF_BATCH_GEMVER}, n[i] in [1, 2048];
 * alpha/beta per instance (GEMVER; may be NULL for 1.0). Host only: no GPU
 * call. Errors: KF_ERR_ARG, KF_ERR_UNSUPPORTED (n out of range). */
kf_status kf_batch_create(int64_t count, const int32_t* kind, const int64_t* n, const float* alpha,
                          const float* beta, const kf_batch_opts* opts, kf_batch** out);
void kf_batch_destroy(kf_batch* b);
kf_status kf_batch_arena_elems(const kf_batch* b, int64_t* elems);
kf_status kf_batch_workspace_bytes(const kf_batch* b, size_t* bytes);
/* Arena offset (floats) of one operand of instance i; *ld gets the row pitch
 * of a matrix or n of a vector. KF_ERR_ARG for an operand the kind lacks. */
kf_status kf_batch_offset(const kf_batch* b, int64_t i, int32_t operand, int64_t* offset, int64_t* ld);
/* Algorithmic bytes of the fused plans of all instances (BiCGK: A, p, r read,
 * q, s written; GEMVER: A, six vectors, then B and x read; B, x, w written). */
kf_status kf_batch_bytes(const kf_batch* b, int64_t* read, int64_t* written);
/* JSON summary (instances per bucket, items, split instances, rows, grid). */
kf_status kf_batch_describe(const kf_batch* b, char* buf, size_t len, size_t* needed);
/* Work items, which = 0: queue order of the persistent launch, 1: instance
 * order of the launch loop; arrays of cap entries, *count gets the total. */
kf_status kf_batch_items(const kf_batch* b, int32_t which, int32_t* inst, int32_t* phase, int32_t* blk,
                         int64_t cap, int64_t* count);
/* Device pointers; uploads the instance and item tables into the workspace
 * and clears the counters on `stream`, which it synchronises. Errors:
 * KF_ERR_ALIGN, KF_ERR_ALIAS, KF_ERR_HIP. */
kf_status kf_batch_bind(kf_batch* b, float* arena, void* workspace, void* stream);
/* which = 0: the persistent launch; 1: the baseline loop, one launch per
 * instance (and one more for the w rows of a split GEMVER instance). */
kf_status kf_batch_run(kf_batch* b, int32_t which, void* stream);
/* Record kf_batch_run(which) on `stream` (not the null stream) into a graph
 * kept in the batch; kf_batch_graph_launch replays it. kf_batch_bind drops
 * the graphs. */
kf_status kf_batch_capture(kf_batch* b, int32_t which, void* stream);
kf_status kf_batch_graph_launch(kf_batch* b, int32_t which, void* stream);
/* Median over reps of HIP events around one run (graph != 0: the replay). */
kf_status kf_batch_time(kf_batch* b, int32_t which, int32_t graph, void* stream, int32_t warmup, int32_t reps,
                        float* median_us);
/* Synchronises `stream` and returns the error bits (1: a dependent item's
 * wait ran out) of the runs since the last call. When a bit is set it also
 * clears the counters, flags and error word, so the next run starts clean. */
kf_status kf_batch_error(kf_batch* b, void* stream, uint32_t* bits);

/* ---- measurement helper -------------------------------------------------- */
/* dst[0..bytes) = src[0..bytes) with a plain streaming kernel (128-bit
 * non-temporal loads and stores) on `stream`; bytes and both pointers must be
 * multiples of 16. Used to calibrate memory-traffic counters against a copy of
 * known size. */
kf_status kf_util_copy(void* dst, const void* src, size_t bytes, void* stream);
/* Streaming references for the bandwidth this device attains (no part of any
 * plan), asynchronous on `stream`, 16-byte aligned pointers.
 * kind 0, read: streams src[0..bytes) (bytes a multiple of 16) with 16-byte
 *   non-temporal loads, eight in flight per lane, over 2048 workgroups; dst
 *   receives each workgroup's sum of its floats (2048 floats, 8 KiB).
 * kind 1, copy: dst[0..bytes) = src[0..bytes) (bytes a multiple of 64 KiB, no
 *   overlap) in the layout of the strip kernels: rows of 64 KiB, 2 KiB column
 *   strips, 2048 rows per workgroup of two waves (one workgroup per CU at
 *   1 GiB), so few DRAM streams are open at once.
 * KF_ERR_ARG for other kinds, sizes or alignments; KF_ERR_ALIAS for overlap. */
kf_status kf_util_stream(int32_t kind, void* dst, const void* src, size_t bytes, void* stream);
/* Seeded synthetic inputs on the device: dst[i * ld + j] for i < rows,
 * j < ld is, for j < cols, the SplitMix64 output number i * cols + j + 1 of
 * the stream that starts at `key`, mapped to (h >> 40) 2^-23 - 1 (uniform on
 * [-1, 1), exact in float32), and `pad` for j >= cols. The same values as the
 * project's host-side generator for the same key, so large inputs need not
 * cross PCIe. Asynchronous on `stream`. */
kf_status kf_util_fill_uniform(float* dst, int64_t rows, int64_t cols, int64_t ld, uint64_t key, float pad,
                               void* stream);

#ifdef __cplusplus
}
#endif
#endif /* KF_H */
