"""Thin ctypes binding of the ``kf.h`` C ABI (argument marshalling only).

Every function keeps the C name and raises :class:`KFError` on a negative
status. Device buffers are passed as integer addresses (``tensor.data_ptr()``)
and streams as ``hipStream_t`` integers (``torch.cuda.current_stream().cuda_stream``).

PyTorch's wheel ships its own HIP runtime with the same soname as the system
one; it is imported before the library is loaded so that the process holds a
single HIP runtime.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (load order: one HIP runtime per process)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkf.so")

KF_OK = 0
ERRORS = {
    -1: "KF_ERR_ARG", -2: "KF_ERR_SHAPE", -3: "KF_ERR_DTYPE", -4: "KF_ERR_ALIGN",
    -5: "KF_ERR_ALIAS", -6: "KF_ERR_STATE", -7: "KF_ERR_UNBOUND", -8: "KF_ERR_WORKSPACE",
    -9: "KF_ERR_COMPILE", -10: "KF_ERR_HIP", -11: "KF_ERR_NOMEM", -12: "KF_ERR_UNSUPPORTED",
    -13: "KF_ERR_INTERNAL",
}
globals().update({name: code for code, name in ERRORS.items()})   # KF_ERR_ARG = -1, ...
KF_NONE = -1
MODES = {"unfused": 0, "fused": 1, "additive": 2, "learned": 3, "exhaustive": 4, "partition": 5}
KF_COMPILE_NO_LOAD = 1
KF_COMPILE_CODEGEN_ONLY = 2
KF_COMPILE_RUNTIME_SHAPE = 4

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_sz = ctypes.c_size_t
_f32 = ctypes.c_float
_P = ctypes.POINTER


class KFError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (ERRORS.get(status, str(status)), message))
        self.status = status
        self.name = ERRORS.get(status, str(status))


class kf_routine_entry(ctypes.Structure):
    _fields_ = [("cls", _i32), ("env", _i32 * 4), ("routine", _i32), ("lds_kb", _i32), ("us_per_unit", _f32)]


class kf_compile_opts(ctypes.Structure):
    pass


IMPL_FIELDS = ["mat_k", "mat_waves", "mat_group", "mat_rows", "mat_sched", "mat_unit",
               "vec_unroll", "vec_threads", "vec_grid"]


class kf_impl_params(ctypes.Structure):
    _fields_ = [(f, _i32) for f in IMPL_FIELDS]


kf_compile_opts._fields_ = [("mode", _i32), ("flags", _i32),
                            ("mat_k", _i32), ("mat_waves", _i32), ("mat_group", _i32), ("mat_rows", _i32),
                            ("vec_unroll", _i32), ("vec_threads", _i32), ("vec_grid", _i32),
                            ("mat_sched", _i32),
                            ("partition", _P(_i32)), ("partition_len", _i32),
                            ("table", _P(kf_routine_entry)), ("table_len", _i32), ("max_partitions", _i32),
                            ("grid", _P(kf_compile_opts)), ("grid_len", _i32), ("mat_unit", _i32),
                            ("model", _vp), ("stream", _vp), ("bind_values", _P(_i32)), ("bind_ptrs", _P(_vp)),
                            ("bind_len", _i32), ("top_k", _i32),
                            ("kernel_params", _P(kf_impl_params)), ("kernel_params_len", _i32),
                            ("time_budget_ms", _i32), ("workspace", _vp), ("workspace_bytes", ctypes.c_size_t)]
PARAM_FIELDS = ["mat_k", "mat_waves", "mat_group", "mat_rows", "vec_unroll", "vec_threads", "vec_grid",
                "mat_sched", "mat_unit"]


ROUTINES = ["LOAD_MAT", "STORE_MAT", "COMPUTE_GEMV", "COMPUTE_GEMTV", "COMPUTE_GER", "LOAD_VEC",
            "STORE_VEC", "COMPUTE_SCAL", "COMPUTE_AXPY", "COMPUTE_DOT", "FINISH"]
FEATURE_DIM = 32

_SIGS = {
    "kf_last_error": ([], ctypes.c_char_p),
    "kf_version": ([], ctypes.c_char_p),
    "kf_script_create": ([_P(_vp)], _i32),
    "kf_script_destroy": ([_vp], None),
    "kf_vector": ([_vp, _i64, _P(_i32)], _i32),
    "kf_matrix": ([_vp, _i64, _i64, _i64, _P(_i32)], _i32),
    "kf_matrix_q": ([_vp, _i64, _i64, _i64, _i32, _i32, _P(_i32)], _i32),
    "kf_matrix_layout": ([_vp, _i64, _i64, _i64, _i32, _P(_i32)], _i32),
    "kf_value_layout": ([_vp, _i32, _P(_i32)], _i32),
    "kf_const": ([_vp, _f32, _P(_i32)], _i32),
    "kf_scalar": ([_vp, _P(_i32)], _i32),
    "kf_input": ([_vp, _i32], _i32),
    "kf_output": ([_vp, _i32], _i32),
    "kf_scal": ([_vp, _i32, _i32, _P(_i32)], _i32),
    "kf_axpy": ([_vp, _i32, _i32, _i32, _P(_i32)], _i32),
    "kf_dot": ([_vp, _i32, _i32, _P(_i32)], _i32),
    "kf_gemv": ([_vp, _i32, _i32, _i32, _i32, _i32, _P(_i32)], _i32),
    "kf_gemtv": ([_vp, _i32, _i32, _i32, _i32, _i32, _P(_i32)], _i32),
    "kf_ger": ([_vp, _i32, _i32, _i32, _i32, _P(_i32)], _i32),
    "kf_value_info": ([_vp, _i32, _P(_i32), _P(_i64), _P(_i64), _P(_i64)], _i32),
    "kf_script_num_calls": ([_vp, _P(_i32)], _i32),
    "kf_script_call": ([_vp, _i32, _P(_i32), _P(_i32), _P(_i32), _P(_i32), _P(_i32)], _i32),
    "kf_compile_opts_init": ([_P(kf_compile_opts)], None),
    "kf_compile_workspace_bytes": ([_vp, _P(kf_compile_opts), _P(_sz)], _i32),
    "kf_plan_set_shape": ([_vp, _i64, _i64], _i32),
    "kf_bind_matrix": ([_vp, _i32, _vp, _i64], _i32),
    "kf_plan_run_many": ([_vp, _i64, _P(_i64), _i32, _P(_i32), _P(_vp), _P(_i64), _vp], _i32),
    "kf_compile": ([_vp, _P(kf_compile_opts), _P(_vp)], _i32),
    "kf_plan_destroy": ([_vp], None),
    "kf_enumerate": ([_vp, _i32, _P(_vp)], _i32),
    "kf_planset_destroy": ([_vp], None),
    "kf_planset_count": ([_vp, _P(_i32)], _i32),
    "kf_planset_get": ([_vp, _i32, _P(_i32), _i32], _i32),
    "kf_candidates": ([_vp, _i32, _P(kf_compile_opts), _i32, _P(_vp)], _i32),
    "kf_planset_params": ([_vp, _i32, _P(kf_compile_opts)], _i32),
    "kf_planset_compile": ([_vp, _i32, _i32, _P(_vp)], _i32),
    "kf_planset_precompile": ([_vp, _P(_i32), _i32], _i32),
    "kf_planset_predict_additive": ([_vp, _P(kf_routine_entry), _i32, _P(_f32)], _i32),
    "kf_plan_workspace_bytes": ([_vp, _P(_sz)], _i32),
    "kf_bind": ([_vp, _i32, _vp], _i32),
    "kf_bind_workspace": ([_vp, _vp, _sz], _i32),
    "kf_set_const": ([_vp, _i32, _f32], _i32),
    "kf_run": ([_vp, _vp], _i32),
    "kf_run_noalloc": ([_vp, _vp], _i32),
    "kf_run_kernel": ([_vp, _i32, _vp], _i32),
    "kf_plan_num_launches": ([_vp, _i32, _P(_i32)], _i32),
    "kf_run_launch": ([_vp, _i32, _i32, _vp], _i32),
    "kf_time_plan": ([_vp, _vp, _i32, _i32, _P(_f32)], _i32),
    "kf_time_plan_kernels": ([_vp, _vp, _i32, _i32, _P(_f32)], _i32),
    "kf_plan_kernel_params": ([_vp, _i32, _P(kf_impl_params)], _i32),
    "kf_plan_describe": ([_vp, ctypes.c_char_p, _sz, _P(_sz)], _i32),
    "kf_plan_bytes": ([_vp, _P(_u64), _P(_u64)], _i32),
    "kf_plan_num_kernels": ([_vp, _P(_i32)], _i32),
    "kf_plan_source": ([_vp, _i32, ctypes.c_char_p, _sz, _P(_sz)], _i32),
    "kf_plan_kernel_geometry": ([_vp, _i32, _P(_i32), _P(_i32)], _i32),
    "kf_util_copy": ([_vp, _vp, _sz, _vp], _i32),
    "kf_util_stream": ([_i32, _vp, _vp, _sz, _vp], _i32),
    "kf_jit_set_cache_dir": ([ctypes.c_char_p], _i32),
    "kf_util_fill_uniform": ([_vp, _i64, _i64, _i64, _u64, _f32, _vp], _i32),
    "kf_quantize_rows": ([_vp, _i64, _i64, _i64, _i32, _vp, _i64, _vp, _vp], _i32),
    "kf_jit_release": ([], _i32),
    "kf_routine_time": ([_i32, _i64, _i64, _P(kf_compile_opts), _i32, _vp, _sz, _vp, _i32, _i32, _P(_f32)], _i32),
    "kf_predict_additive": ([_vp, _P(kf_routine_entry), _i32, _P(_f32)], _i32),
    "kf_plan_features": ([_vp, _P(_f32), _i32, _P(_i32)], _i32),
    "kf_mlp_create": ([_i32, _i32, _i32, _P(_vp)], _i32),
    "kf_mlp_destroy": ([_vp], None),
    "kf_mlp_param_count": ([_vp, _P(_i64)], _i32),
    "kf_mlp_layout": ([_vp, _i32, _P(_i64), _P(_i64), _P(_i64), _P(_i64)], _i32),
    "kf_mlp_init_params": ([_vp, _u64, _P(_f32)], _i32),
    "kf_mlp_workspace_bytes": ([_vp, _i32, _P(_sz)], _i32),
    "kf_mlp_forward": ([_vp, _vp, _vp, _i32, _vp, _vp, _sz, _vp], _i32),
    "kf_mlp_loss_grad": ([_vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _sz, _vp], _i32),
    "kf_mlp_adam": ([_vp, _vp, _vp, _vp, _vp, _i32, _f32, _f32, _f32, _f32, _vp], _i32),
    "kf_jit_stats": ([_P(_i64), _P(_i64)], _i32),
    "kf_costmodel_create": ([_i32, _i32, _u64, _P(_vp)], _i32),
    "kf_costmodel_destroy": ([_vp], None),
    "kf_costmodel_workspace_bytes": ([_vp, _i64, _P(_sz)], _i32),
    "kf_costmodel_bind": ([_vp, _vp, _sz, _i64, _vp], _i32),
    "kf_costmodel_train": ([_vp, _vp, _vp, _i64, _i32, _i32, _f32, _u64, _vp, _P(_f32)], _i32),
    "kf_costmodel_predict": ([_vp, _vp, _i64, _vp, _vp], _i32),
    "kf_costmodel_plan_us": ([_vp, _P(_f32), _i64, _P(_i64), _i32, _P(ctypes.c_double), _vp], _i32),
    "kf_costmodel_set_launch_us": ([_vp, _f32], _i32),
    "kf_costmodel_get": ([_vp, _P(_f32), _P(_f32), _P(_f32), _P(ctypes.c_double), _P(_f32)], _i32),
    "kf_costmodel_set": ([_vp, _P(_f32), _P(_f32), _P(_f32), _P(ctypes.c_double), _f32], _i32),
    "kf_costmodel_dims": ([_vp, _P(_i32), _P(_i32), _P(_i64)], _i32),
    "kf_costmodel_save": ([_vp, ctypes.c_char_p], _i32),
    "kf_costmodel_load": ([ctypes.c_char_p, _P(_vp)], _i32),
    "kf_batch_create": ([_i64, _P(_i32), _P(_i64), _P(_f32), _P(_f32), _vp, _P(_vp)], _i32),
    "kf_batch_destroy": ([_vp], None),
    "kf_batch_arena_elems": ([_vp, _P(_i64)], _i32),
    "kf_batch_workspace_bytes": ([_vp, _P(_sz)], _i32),
    "kf_batch_offset": ([_vp, _i64, _i32, _P(_i64), _P(_i64)], _i32),
    "kf_batch_bytes": ([_vp, _P(_i64), _P(_i64)], _i32),
    "kf_batch_describe": ([_vp, ctypes.c_char_p, _sz, _P(_sz)], _i32),
    "kf_batch_items": ([_vp, _i32, _P(_i32), _P(_i32), _P(_i32), _i64, _P(_i64)], _i32),
    "kf_batch_bind": ([_vp, _vp, _vp, _vp], _i32),
    "kf_batch_run": ([_vp, _i32, _vp], _i32),
    "kf_batch_capture": ([_vp, _i32, _vp], _i32),
    "kf_batch_graph_launch": ([_vp, _i32, _vp], _i32),
    "kf_batch_time": ([_vp, _i32, _i32, _vp, _i32, _i32, _P(_f32)], _i32),
    "kf_batch_error": ([_vp, _vp, _P(_u32)], _i32),
    "kf_batch_tile_info": ([_i32, _i32, _i32, _P(_i32), _P(_i32)], _i32),
}
EXPORTED = sorted(_SIGS)

_lib = None


def lib():
    """Load libkf.so; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libkf.so is not built; run paper_1305_1183_amd/build.py "
                               "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _chk(st: int) -> None:
    if st != KF_OK:
        raise KFError(st, lib().kf_last_error().decode())


def kf_last_error() -> str:
    return lib().kf_last_error().decode()


def kf_version() -> str:
    return lib().kf_version().decode()


# ---- script recording --------------------------------------------------------
class Script:
    """Owning handle of a kf_script, passed to the C calls as its pointer. The
    script is destroyed when the last reference to the handle goes (or by
    kf_script_destroy), so an owner that is collected early (a temporary
    sequence object) cannot free a script that a call is still using."""

    def __init__(self, h):
        self._as_parameter_ = h

    def destroy(self) -> None:
        h = self._as_parameter_
        self._as_parameter_ = _vp()
        if h.value:
            lib().kf_script_destroy(h)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def kf_script_create() -> Script:
    h = _vp()
    _chk(lib().kf_script_create(ctypes.byref(h)))
    return Script(h)


def kf_script_destroy(s) -> None:
    """Destroy now (later calls on the handle get a null script: KF_ERR_ARG)."""
    if isinstance(s, Script):
        s.destroy()
    else:
        lib().kf_script_destroy(s)


def _new(fn, *args) -> int:
    out = _i32()
    _chk(fn(*args, ctypes.byref(out)))
    return out.value


def kf_vector(s, n: int) -> int:
    return _new(lib().kf_vector, s, n)


def kf_matrix(s, rows: int, cols: int, ld: int = 0) -> int:
    return _new(lib().kf_matrix, s, rows, cols, ld)


KF_ROW_MAJOR, KF_COL_MAJOR = 0, 1


def kf_matrix_layout(s, rows: int, cols: int, layout: int, ld: int = 0) -> int:
    """Matrix in either layout; KF_COL_MAJOR stores element (i, j) at j * ld + i."""
    return _new(lib().kf_matrix_layout, s, rows, cols, ld, layout)


def kf_value_layout(s, v: int) -> int:
    return _new(lib().kf_value_layout, s, v)


KF_F32, KF_BF16, KF_FP8_E4M3 = 0, 1, 2
DTYPES = {"f32": KF_F32, "bf16": KF_BF16, "fp8": KF_FP8_E4M3}


def kf_matrix_q(s, rows: int, cols: int, dtype, scale: int, ld: int = 0) -> int:
    dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    return _new(lib().kf_matrix_q, s, rows, cols, ld, dt, scale)


def kf_const(s, v: float) -> int:
    return _new(lib().kf_const, s, v)


def kf_scalar(s) -> int:
    return _new(lib().kf_scalar, s)


def kf_input(s, v: int) -> None:
    _chk(lib().kf_input(s, v))


def kf_output(s, v: int) -> None:
    _chk(lib().kf_output(s, v))


def kf_scal(s, alpha: int, x: int) -> int:
    return _new(lib().kf_scal, s, alpha, x)


def kf_axpy(s, alpha: int, x: int, y: int) -> int:
    return _new(lib().kf_axpy, s, alpha, x, y)


def kf_dot(s, x: int, y: int) -> int:
    return _new(lib().kf_dot, s, x, y)


def kf_gemv(s, alpha: int, A: int, x: int, beta: int = KF_NONE, y0: int = KF_NONE) -> int:
    return _new(lib().kf_gemv, s, alpha, A, x, beta, y0)


def kf_gemtv(s, alpha: int, A: int, x: int, beta: int = KF_NONE, y0: int = KF_NONE) -> int:
    return _new(lib().kf_gemtv, s, alpha, A, x, beta, y0)


def kf_ger(s, alpha: int, A: int, u: int, v: int) -> int:
    return _new(lib().kf_ger, s, alpha, A, u, v)


def kf_value_info(s, v: int):
    k, d0, d1, d2 = _i32(), _i64(), _i64(), _i64()
    _chk(lib().kf_value_info(s, v, ctypes.byref(k), ctypes.byref(d0), ctypes.byref(d1),
                             ctypes.byref(d2)))
    return k.value, d0.value, d1.value, d2.value


def kf_script_num_calls(s) -> int:
    n = _i32()
    _chk(lib().kf_script_num_calls(s, ctypes.byref(n)))
    return n.value


OP_NAMES = ["scal", "axpy", "dot", "gemv", "gemtv", "ger"]


def kf_script_call(s, i: int) -> dict:
    op, a, b, o = _i32(), _i32(), _i32(), _i32()
    ins = (_i32 * 3)()
    _chk(lib().kf_script_call(s, i, ctypes.byref(op), ctypes.byref(a), ctypes.byref(b), ins, ctypes.byref(o)))
    return {"op": OP_NAMES[op.value], "alpha": a.value, "beta": b.value, "in": list(ins), "out": o.value}


# ---- compile / enumerate --------------------------------------------------------
def kf_compile_opts_init(mode="fused", flags=0, partition=None, table=None, grid=None, max_partitions=0,
                         model=None, stream=None, bind=None, top_k=0, kernel_params=None, time_budget_ms=0,
                         workspace=None, **params) -> kf_compile_opts:
    """bind: {script value handle: device pointer} of every input and output
    (timing in the learned top-k and exhaustive modes); workspace: (device
    pointer, bytes) of the timed modes' plan workspace; model: a cost-model
    handle with bound memory; kernel_params: one dict of implementation
    parameters per plan kernel, in launch order (missing or zero entries take
    the plan-wide parameters)."""
    o = kf_compile_opts()
    lib().kf_compile_opts_init(ctypes.byref(o))
    o.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    o.flags = flags
    o.max_partitions = max_partitions
    o.top_k = int(top_k)
    o.time_budget_ms = int(time_budget_ms)
    if workspace is not None:
        o.workspace = int(workspace[0])
        o.workspace_bytes = int(workspace[1])
    if model is not None:
        o.model = model
    if stream is not None:
        o.stream = stream
    for k, v in params.items():
        if k not in PARAM_FIELDS:
            raise TypeError("unknown compile option %s" % k)
        setattr(o, k, int(v))
    keep = []
    if table is not None:
        o.table = ctypes.cast(table, _P(kf_routine_entry))
        o.table_len = len(table)
        keep.append(table)
    if grid is not None:
        garr = grid_array(grid)
        o.grid = ctypes.cast(garr, _P(kf_compile_opts))
        o.grid_len = len(garr)
        keep.append(garr)
    if bind:
        vals = (_i32 * len(bind))(*[int(k) for k in bind])
        ptrs = (_vp * len(bind))(*[int(v) for v in bind.values()])
        o.bind_values = ctypes.cast(vals, _P(_i32))
        o.bind_ptrs = ctypes.cast(ptrs, _P(_vp))
        o.bind_len = len(bind)
        keep += [vals, ptrs]
    if kernel_params:
        karr = (kf_impl_params * len(kernel_params))()
        for i, kp in enumerate(kernel_params):
            for k, v in (kp or {}).items():
                if k not in IMPL_FIELDS:
                    raise TypeError("unknown kernel parameter %s" % k)
                setattr(karr[i], k, int(v))
        o.kernel_params = ctypes.cast(karr, _P(kf_impl_params))
        o.kernel_params_len = len(kernel_params)
        keep.append(karr)
    if partition is not None:
        arr = (_i32 * len(partition))(*partition)
        o.partition = ctypes.cast(arr, _P(_i32))
        o.partition_len = len(partition)
        keep.append(arr)
    o._keep = keep  # keep the arrays alive with the struct
    return o


def kf_compile_workspace_bytes(s, opts=None, **kw) -> int:
    if opts is None:
        opts = kf_compile_opts_init(**kw)
    n = _sz()
    _chk(lib().kf_compile_workspace_bytes(s, ctypes.byref(opts), ctypes.byref(n)))
    return n.value


def kf_compile(s, opts=None, **kw):
    if opts is None:
        opts = kf_compile_opts_init(**kw)
    ws = None
    timed = opts.mode == MODES["exhaustive"] or (opts.mode == MODES["learned"] and opts.top_k > 1)
    if timed and not opts.workspace and opts.bind_len > 0:
        # the caller's side of the ownership contract: the timed modes' plan
        # workspace, sized by the library and allocated here by torch
        import torch
        need = kf_compile_workspace_bytes(s, opts)
        if need:
            ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
            opts.workspace = (ws.data_ptr() + 255) // 256 * 256
            opts.workspace_bytes = need
    h = _vp()
    try:
        _chk(lib().kf_compile(s, ctypes.byref(opts), ctypes.byref(h)))
    finally:
        if ws is not None:
            torch.cuda.current_stream().synchronize()
            opts.workspace, opts.workspace_bytes = None, 0
            del ws
    return h


def kf_plan_destroy(p) -> None:
    lib().kf_plan_destroy(p)


def kf_enumerate(s, max_plans: int = 0) -> list:
    """All legal partitions (list of lists: kernel id per call)."""
    h = _vp()
    _chk(lib().kf_enumerate(s, max_plans, ctypes.byref(h)))
    try:
        n = _i32()
        _chk(lib().kf_planset_count(h, ctypes.byref(n)))
        nc = kf_script_num_calls(s)
        out = []
        buf = (_i32 * max(nc, 1))()
        for i in range(n.value):
            _chk(lib().kf_planset_get(h, i, buf, nc))
            out.append(list(buf[:nc]))
        return out
    finally:
        lib().kf_planset_destroy(h)


def grid_array(points) -> ctypes.Array:
    """Array of kf_compile_opts from dicts of implementation parameters."""
    points = list(points)
    arr = (kf_compile_opts * max(1, len(points)))()
    for i, pt in enumerate(points):
        lib().kf_compile_opts_init(ctypes.byref(arr[i]))
        for k, v in pt.items():
            if k not in PARAM_FIELDS:
                raise TypeError("unknown parameter %s" % k)
            setattr(arr[i], k, int(v))
    return arr


class Candidates:
    """Candidate plans of a script (partitions x parameter points)."""

    def __init__(self, script, max_partitions=64, grid=None):
        self.script = script
        h = _vp()
        garr = grid_array(grid) if grid is not None else None
        _chk(lib().kf_candidates(script, max_partitions, garr, len(garr) if garr is not None else 0,
                                 ctypes.byref(h)))
        self.h = h
        n = _i32()
        _chk(lib().kf_planset_count(h, ctypes.byref(n)))
        self.n = n.value
        self.ncalls = kf_script_num_calls(script)

    def __len__(self):
        return self.n

    def __del__(self):
        try:
            lib().kf_planset_destroy(self.h)
        except Exception:
            pass

    def partition(self, i):
        buf = (_i32 * max(1, self.ncalls))()
        _chk(lib().kf_planset_get(self.h, i, buf, self.ncalls))
        return list(buf[:self.ncalls])

    def params(self, i) -> dict:
        o = kf_compile_opts()
        _chk(lib().kf_planset_params(self.h, i, ctypes.byref(o)))
        return {k: getattr(o, k) for k in PARAM_FIELDS}

    def compile(self, i, flags=0):
        p = _vp()
        _chk(lib().kf_planset_compile(self.h, i, flags, ctypes.byref(p)))
        return p

    def precompile(self, idx) -> None:
        idx = list(idx)
        arr = (_i32 * max(1, len(idx)))(*idx)
        _chk(lib().kf_planset_precompile(self.h, arr, len(idx)))

    def predict_additive(self, table):
        import numpy as np
        out = np.zeros(self.n, dtype=np.float32)
        _chk(lib().kf_planset_predict_additive(self.h, table, len(table), out.ctypes.data_as(_P(_f32))))
        return out


# ---- bind / run ------------------------------------------------------------------
def kf_plan_workspace_bytes(p) -> int:
    n = _sz()
    _chk(lib().kf_plan_workspace_bytes(p, ctypes.byref(n)))
    return n.value


def kf_bind(p, v: int, dev_ptr: int) -> None:
    _chk(lib().kf_bind(p, v, _vp(dev_ptr)))


def kf_plan_set_shape(p, rows: int, cols: int) -> None:
    _chk(lib().kf_plan_set_shape(p, rows, cols))


def kf_bind_matrix(p, v: int, dev_ptr: int, ld: int) -> None:
    _chk(lib().kf_bind_matrix(p, v, _vp(dev_ptr), ld))


def kf_plan_run_many(p, shapes, values, ptrs, lds=None, stream: int = 0) -> None:
    """shapes: (count, 2) int64; values: nvals value handles; ptrs: (count,
    nvals) device pointers; lds: (count, nvals) leading dimensions or None."""
    import numpy as np
    shapes = np.ascontiguousarray(shapes, dtype=np.int64)
    vals = np.ascontiguousarray(values, dtype=np.int32)
    ptrs = np.ascontiguousarray(ptrs, dtype=np.uint64)
    count = shapes.shape[0]
    lp = None
    if lds is not None:
        lds = np.ascontiguousarray(lds, dtype=np.int64)
        lp = lds.ctypes.data_as(_P(_i64))
    _chk(lib().kf_plan_run_many(p, count, shapes.ctypes.data_as(_P(_i64)), len(vals), vals.ctypes.data_as(_P(_i32)),
                                ptrs.ctypes.data_as(_P(_vp)), lp, _vp(stream)))


def kf_bind_workspace(p, dev_ptr: int, nbytes: int) -> None:
    _chk(lib().kf_bind_workspace(p, _vp(dev_ptr), nbytes))


def kf_set_const(p, v: int, value: float) -> None:
    _chk(lib().kf_set_const(p, v, value))


def kf_run(p, stream: int = 0) -> None:
    _chk(lib().kf_run(p, _vp(stream)))


# Size of the library's fixed per-device workspace of kf_run_noalloc
# (KF_NOALLOC_SCRATCH_BYTES in kf.h).
KF_NOALLOC_SCRATCH_BYTES = 32 << 20


def kf_run_noalloc(p, stream: int = 0) -> None:
    _chk(lib().kf_run_noalloc(p, _vp(stream)))


def kf_run_kernel(p, k: int, stream: int = 0) -> None:
    _chk(lib().kf_run_kernel(p, k, _vp(stream)))


def kf_plan_num_launches(p, k: int) -> int:
    n = _i32()
    _chk(lib().kf_plan_num_launches(p, k, ctypes.byref(n)))
    return n.value


def kf_run_launch(p, k: int, l: int, stream: int = 0) -> None:
    _chk(lib().kf_run_launch(p, k, l, _vp(stream)))


def kf_time_plan(p, stream: int = 0, warmup: int = 3, reps: int = 20) -> float:
    t = _f32()
    _chk(lib().kf_time_plan(p, _vp(stream), warmup, reps, ctypes.byref(t)))
    return t.value


def kf_time_plan_kernels(p, stream: int = 0, warmup: int = 2, reps: int = 5) -> list:
    """Median time (us) of every plan kernel inside whole runs of the plan."""
    n = kf_plan_num_kernels(p)
    t = (_f32 * n)()
    _chk(lib().kf_time_plan_kernels(p, _vp(stream), warmup, reps, t))
    return [float(x) for x in t]


def kf_plan_kernel_params(p, k: int) -> dict:
    """Implementation parameters of plan kernel k (defaults for its shape applied)."""
    e = kf_impl_params()
    _chk(lib().kf_plan_kernel_params(p, k, ctypes.byref(e)))
    return {f: getattr(e, f) for f in IMPL_FIELDS if getattr(e, f)}


def _text(fn, *args) -> str:
    need = _sz()
    _chk(fn(*args, None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value)
    _chk(fn(*args, buf, need.value, ctypes.byref(need)))
    return buf.value.decode()


def kf_plan_describe(p) -> str:
    return _text(lib().kf_plan_describe, p)


def kf_plan_source(p, k: int) -> str:
    return _text(lib().kf_plan_source, p, k)


def kf_plan_bytes(p):
    r, w = _u64(), _u64()
    _chk(lib().kf_plan_bytes(p, ctypes.byref(r), ctypes.byref(w)))
    return r.value, w.value


def kf_plan_num_kernels(p) -> int:
    n = _i32()
    _chk(lib().kf_plan_num_kernels(p, ctypes.byref(n)))
    return n.value


def kf_plan_kernel_geometry(p, k: int):
    g, b = _i32(), _i32()
    _chk(lib().kf_plan_kernel_geometry(p, k, ctypes.byref(g), ctypes.byref(b)))
    return g.value, b.value


def kf_jit_release() -> None:
    _chk(lib().kf_jit_release())


def kf_jit_set_cache_dir(path) -> None:
    """Disk cache directory for later compilations ("" = none, None = KF_CACHE_DIR)."""
    _chk(lib().kf_jit_set_cache_dir(None if path is None else str(path).encode()))


def kf_jit_stats():
    a, b = _i64(), _i64()
    _chk(lib().kf_jit_stats(ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def kf_util_copy(dst: int, src: int, nbytes: int, stream: int = 0) -> None:
    _chk(lib().kf_util_copy(_vp(dst), _vp(src), nbytes, _vp(stream)))


def kf_util_stream(kind: int, dst: int, src: int, nbytes: int, stream: int = 0) -> None:
    """Streaming reference: kind 0 reads src (dst gets 2048 workgroup sums),
    kind 1 copies src to dst in the strip kernels' layout."""
    _chk(lib().kf_util_stream(int(kind), _vp(dst), _vp(src), nbytes, _vp(stream)))


# ---- batched uneven sizes ------------------------------------------------------------
KF_BATCH_BICGK, KF_BATCH_GEMVER = 0, 1
BATCH_BUCKETS = 6
BATCH_ROWS_PER_STEP = (64, 32, 16, 16, 8, 4)   # of each bucket's default tile (menu entry 0)
BATCH_OPERANDS = {0: ["A", "B_unused", "p", "r", "q", "s"],
                  1: ["A", "B", "u1", "v1", "u2", "v2", "y", "z", "x", "w"]}


class kf_batch_opts(ctypes.Structure):
    _fields_ = [("rows", (_i32 * BATCH_BUCKETS) * 2), ("grid", _i32), ("spin_limit", _u32),
                ("tile", (_i32 * BATCH_BUCKETS) * 2)]


def batch_opts(rows=None, grid: int = 0, spin_limit: int = 0, tiles=None):
    """rows: {kind: [rows per bucket]} (0 = library default); tiles: {kind:
    [tile menu entry per bucket]} (0 = the bucket's default tile)."""
    o = kf_batch_opts()
    for k, lst in (rows or {}).items():
        for j, r in enumerate(lst):
            o.rows[k][j] = int(r)
    for k, lst in (tiles or {}).items():
        for j, t in enumerate(lst):
            o.tile[k][j] = int(t)
    o.grid = int(grid)
    o.spin_limit = int(spin_limit)
    return o


def kf_batch_tile_info(kind: int, bucket: int, t: int):
    """(menu length, entry t as dict or None past the end)."""
    c = _i32()
    out = (_i32 * 5)()
    _chk(lib().kf_batch_tile_info(kind, bucket, t, ctypes.byref(c), out))
    if t >= c.value:
        return c.value, None
    return c.value, dict(wide=out[0], ltpr=out[1], k=out[2], lg=out[3], rows_per_step=out[4])


def kf_batch_create(kinds, ns, alphas=None, betas=None, opts=None):
    import numpy as np
    kinds = np.ascontiguousarray(kinds, dtype=np.int32)
    ns = np.ascontiguousarray(ns, dtype=np.int64)
    cnt = len(kinds)
    al = None if alphas is None else np.ascontiguousarray(alphas, dtype=np.float32)
    be = None if betas is None else np.ascontiguousarray(betas, dtype=np.float32)
    fp = lambda a: None if a is None else a.ctypes.data_as(_P(_f32))
    b = _vp()
    _chk(lib().kf_batch_create(cnt, kinds.ctypes.data_as(_P(_i32)), ns.ctypes.data_as(_P(_i64)), fp(al), fp(be),
                               None if opts is None else ctypes.byref(opts), ctypes.byref(b)))
    return b


def kf_batch_destroy(b) -> None:
    lib().kf_batch_destroy(b)


def kf_batch_arena_elems(b) -> int:
    v = _i64()
    _chk(lib().kf_batch_arena_elems(b, ctypes.byref(v)))
    return v.value


def kf_batch_workspace_bytes(b) -> int:
    v = _sz()
    _chk(lib().kf_batch_workspace_bytes(b, ctypes.byref(v)))
    return v.value


def kf_batch_offset(b, i: int, operand: int):
    off, ld = _i64(), _i64()
    _chk(lib().kf_batch_offset(b, i, operand, ctypes.byref(off), ctypes.byref(ld)))
    return off.value, ld.value


def kf_batch_bytes(b):
    r, w = _i64(), _i64()
    _chk(lib().kf_batch_bytes(b, ctypes.byref(r), ctypes.byref(w)))
    return r.value, w.value


def kf_batch_describe(b) -> str:
    return _text(lib().kf_batch_describe, b)


def kf_batch_items(b, which: int):
    import numpy as np
    cnt = _i64()
    _chk(lib().kf_batch_items(b, which, None, None, None, 0, ctypes.byref(cnt)))
    inst, ph, blk = (np.empty(cnt.value, dtype=np.int32) for _ in range(3))
    P = lambda a: a.ctypes.data_as(_P(_i32))
    _chk(lib().kf_batch_items(b, which, P(inst), P(ph), P(blk), cnt.value, ctypes.byref(cnt)))
    return inst, ph, blk


def kf_batch_bind(b, arena: int, workspace: int, stream: int = 0) -> None:
    _chk(lib().kf_batch_bind(b, _vp(arena), _vp(workspace), _vp(stream)))


def kf_batch_run(b, which: int = 0, stream: int = 0) -> None:
    _chk(lib().kf_batch_run(b, which, _vp(stream)))


def kf_batch_capture(b, which: int, stream: int) -> None:
    _chk(lib().kf_batch_capture(b, which, _vp(stream)))


def kf_batch_graph_launch(b, which: int, stream: int = 0) -> None:
    _chk(lib().kf_batch_graph_launch(b, which, _vp(stream)))


def kf_batch_time(b, which: int = 0, graph: bool = False, stream: int = 0, warmup: int = 2, reps: int = 10) -> float:
    t = _f32()
    _chk(lib().kf_batch_time(b, which, int(graph), _vp(stream), warmup, reps, ctypes.byref(t)))
    return t.value


def kf_batch_error(b, stream: int = 0) -> int:
    v = _u32()
    _chk(lib().kf_batch_error(b, _vp(stream), ctypes.byref(v)))
    return v.value


def kf_util_fill_uniform(dst: int, rows: int, cols: int, ld: int, key: int, pad: float = float("nan"),
                         stream: int = 0) -> None:
    _chk(lib().kf_util_fill_uniform(_vp(dst), rows, cols, ld, key, pad, _vp(stream)))


def kf_quantize_rows(A: int, rows: int, cols: int, lda: int, dtype: int, codes: int, ldq: int, scales: int,
                     stream: int = 0) -> None:
    """Row-scaled BF16 / FP8-E4M3 storage of an FP32 device matrix (device pointers)."""
    _chk(lib().kf_quantize_rows(_vp(A), rows, cols, lda, dtype, _vp(codes), ldq, _vp(scales), _vp(stream)))


# ---- plan ranking ------------------------------------------------------------------
def kf_routine_time(routine: int, rows: int, cols: int, buf: int, buf_bytes: int, stream: int = 0,
                    warmup: int = 2, reps: int = 10, extra_lds_kb: int = 0, **params) -> float:
    o = kf_compile_opts_init(**params)
    t = _f32()
    _chk(lib().kf_routine_time(routine, rows, cols, ctypes.byref(o), extra_lds_kb, _vp(buf), buf_bytes,
                               _vp(stream), warmup, reps, ctypes.byref(t)))
    return t.value


def routine_table(entries) -> ctypes.Array:  # noqa: F811
    """entries: iterable of (cls, (e0, e1, e2, e3), routine, us_per_unit[, lds_kb])."""
    entries = list(entries)
    arr = (kf_routine_entry * max(1, len(entries)))()
    for i, ent in enumerate(entries):
        cls, env, r, us = ent[:4]
        arr[i].cls = cls
        for j in range(4):
            arr[i].env[j] = int(env[j])
        arr[i].routine = r
        arr[i].lds_kb = int(ent[4]) if len(ent) > 4 else 0
        arr[i].us_per_unit = us
    return arr


def kf_predict_additive(p, table) -> float:
    t = _f32()
    _chk(lib().kf_predict_additive(p, table, len(table), ctypes.byref(t)))
    return t.value


def kf_plan_features(p):
    import numpy as np
    nk = _i32()
    _chk(lib().kf_plan_features(p, None, 0, ctypes.byref(nk)))
    out = np.zeros((nk.value, FEATURE_DIM), dtype=np.float32)
    _chk(lib().kf_plan_features(p, out.ctypes.data_as(_P(_f32)), nk.value, ctypes.byref(nk)))
    return out


# ---- learned cost model ----------------------------------------------------------------
def kf_mlp_create(in_dim: int, hidden: int, layers: int):
    h = _vp()
    _chk(lib().kf_mlp_create(in_dim, hidden, layers, ctypes.byref(h)))
    return h


def kf_mlp_destroy(m) -> None:
    lib().kf_mlp_destroy(m)


def kf_mlp_param_count(m) -> int:
    n = _i64()
    _chk(lib().kf_mlp_param_count(m, ctypes.byref(n)))
    return n.value


def kf_mlp_layout(m, layer: int):
    a, b, r, c = _i64(), _i64(), _i64(), _i64()
    _chk(lib().kf_mlp_layout(m, layer, ctypes.byref(a), ctypes.byref(b), ctypes.byref(r), ctypes.byref(c)))
    return a.value, b.value, r.value, c.value


def kf_mlp_init_params(m, seed: int):
    import numpy as np
    out = np.zeros(kf_mlp_param_count(m), dtype=np.float32)
    _chk(lib().kf_mlp_init_params(m, seed, out.ctypes.data_as(_P(_f32))))
    return out


def kf_mlp_workspace_bytes(m, batch: int) -> int:
    n = _sz()
    _chk(lib().kf_mlp_workspace_bytes(m, batch, ctypes.byref(n)))
    return n.value


def kf_mlp_forward(m, params: int, X: int, n: int, pred: int, ws: int, ws_bytes: int, stream: int = 0) -> None:
    _chk(lib().kf_mlp_forward(m, _vp(params), _vp(X), n, _vp(pred), _vp(ws), ws_bytes, _vp(stream)))


def kf_mlp_loss_grad(m, params: int, X: int, y: int, n: int, grads: int, loss: int, ws: int, ws_bytes: int,
                     stream: int = 0) -> None:
    _chk(lib().kf_mlp_loss_grad(m, _vp(params), _vp(X), _vp(y), n, _vp(grads), _vp(loss), _vp(ws), ws_bytes,
                                _vp(stream)))


def kf_mlp_adam(m, params: int, grads: int, mstate: int, vstate: int, step: int, lr: float, beta1: float = 0.9,
                beta2: float = 0.999, eps: float = 1e-8, stream: int = 0) -> None:
    _chk(lib().kf_mlp_adam(m, _vp(params), _vp(grads), _vp(mstate), _vp(vstate), step, lr, beta1, beta2, eps,
                           _vp(stream)))
