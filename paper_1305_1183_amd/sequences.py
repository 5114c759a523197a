"""Scripts of the paper's Table 1 sequences, recorded through the C ABI.

Each builder records the sequence as elementary calls (the paper prints the
script only for BiCGK, Listing 1; the others use the same vocabulary):

* AXPYDOT  z = axpy(-alpha, v, w); r = dot(z, u)            outputs z, r
* WAXPBY   t = scal(beta, y); w = axpy(alpha, x, t)          output w
* BiCGK    q = gemv(1, A, p); s = gemtv(1, A, r)             outputs q, s
* ATAX     t = gemv(1, A, x); y = gemtv(1, A, t)             output y
* GESUMMV  t = gemv(alpha, A, x); y = gemv(beta, B, x, 1, t) output y
* GEMVER   B1 = ger(1, A, u1, v1); B = ger(1, B1, u2, v2);
           x = gemtv(beta, B, y, 1, z); w = gemv(alpha, B, x) outputs B, x, w

A :class:`Sequence` keeps the script and the value handles by name;
:meth:`Sequence.compile` returns a :class:`Program` that binds torch tensors
and launches the plan on the current stream.
"""
from __future__ import annotations

import json
from dataclasses import dataclass, field

import torch

from . import kf


@dataclass
class Sequence:
    name: str
    script: object
    values: dict = field(default_factory=dict)      # name -> kf_value
    inputs: list = field(default_factory=list)       # names of vectors/matrices to bind
    outputs: list = field(default_factory=list)      # names of results
    consts: dict = field(default_factory=dict)       # name -> (kf_value, float)
    shapes: dict = field(default_factory=dict)       # name -> tuple

    # the script handle (kf.Script) destroys the script when its last
    # reference goes, which may outlive this object

    def compile(self, mode="fused", **opts) -> "Program":
        plan = kf.kf_compile(self.script, mode=mode, **opts)
        return Program(self, plan)


class Program:
    """A compiled plan plus the device buffers bound to it."""

    def __init__(self, seq: Sequence, plan):
        self.seq = seq
        self.plan = plan
        self.tensors = {}
        self.workspace = None

    def __del__(self):
        try:
            kf.kf_plan_destroy(self.plan)
        except Exception:
            pass

    @property
    def num_kernels(self) -> int:
        return kf.kf_plan_num_kernels(self.plan)

    def describe(self) -> dict:
        return json.loads(kf.kf_plan_describe(self.plan))

    def bytes(self):
        return kf.kf_plan_bytes(self.plan)

    def bind(self, device="cuda", **tensors):
        """Bind input tensors by name; allocate outputs and the workspace."""
        for name in self.seq.inputs:
            t = tensors[name]
            want = {"bf16": torch.int16, "fp8": torch.uint8}.get(getattr(self.seq, "dtypes", {}).get(name), torch.float32)
            if t.dtype != want or not t.is_contiguous():
                raise ValueError("%s must be a contiguous %s tensor" % (name, want))
            self.tensors[name] = t
            kf.kf_bind(self.plan, self.seq.values[name], t.data_ptr())
        for name in self.seq.outputs:
            if name in tensors:
                t = tensors[name]
            else:
                t = torch.empty(self.seq.shapes[name], dtype=torch.float32, device=device)
            self.tensors[name] = t
            kf.kf_bind(self.plan, self.seq.values[name], t.data_ptr())
        nb = kf.kf_plan_workspace_bytes(self.plan)
        self.workspace = torch.empty(max(nb, 256) // 4 + 64, dtype=torch.float32, device=device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        kf.kf_bind_workspace(self.plan, aligned, nb)
        return self

    def set_const(self, name: str, value: float) -> None:
        kf.kf_set_const(self.plan, self.seq.consts[name][0], value)

    def run(self, stream=None) -> dict:
        st = torch.cuda.current_stream().cuda_stream if stream is None else stream
        kf.kf_run(self.plan, st)
        return {n: self.tensors[n] for n in self.seq.outputs}

    def time(self, warmup=3, reps=20) -> float:
        return kf.kf_time_plan(self.plan, torch.cuda.current_stream().cuda_stream, warmup, reps)

    def time_kernels(self, warmup=2, reps=10) -> list:
        """Median time (us) of each plan kernel inside whole runs."""
        return kf.kf_time_plan_kernels(self.plan, torch.cuda.current_stream().cuda_stream, warmup, reps)


def _seq(name):
    return Sequence(name=name, script=kf.kf_script_create())


def _vec(q, name, n):
    v = kf.kf_vector(q.script, n)
    kf.kf_input(q.script, v)
    q.values[name] = v
    q.inputs.append(name)
    q.shapes[name] = (n,)
    return v


def _mat(q, name, rows, cols, ld=0, layout=kf.KF_ROW_MAJOR):
    """Input matrix; a column-major one is bound as its (cols, ld) storage."""
    v = kf.kf_matrix_layout(q.script, rows, cols, layout, ld)
    kf.kf_input(q.script, v)
    ld = kf.kf_value_info(q.script, v)[3]
    q.values[name] = v
    q.inputs.append(name)
    q.shapes[name] = (cols, ld) if layout == kf.KF_COL_MAJOR else (rows, ld)
    return v


def _dscalar(q, name):
    """Input scalar in device memory (bound like a one-entry vector)."""
    v = kf.kf_scalar(q.script)
    kf.kf_input(q.script, v)
    q.values[name] = v
    q.inputs.append(name)
    q.shapes[name] = (1,)
    return v


def _const(q, name, value):
    v = kf.kf_const(q.script, float(value))
    q.consts[name] = (v, float(value))
    return v


def _out(q, name, v):
    kf.kf_output(q.script, v)
    q.values[name] = v
    q.outputs.append(name)
    kind, d0, d1, d2 = kf.kf_value_info(q.script, v)
    if kind == 1 and kf.kf_value_layout(q.script, v) == kf.KF_COL_MAJOR:
        d0 = d1   # column-major storage: cols x ld
    q.shapes[name] = {0: (d0,), 1: (d0, d2), 3: (1,)}[kind]
    return v


def axpydot(n: int, alpha: float) -> Sequence:
    q = _seq("axpydot")
    w, v, u = _vec(q, "w", n), _vec(q, "v", n), _vec(q, "u", n)
    na = _const(q, "neg_alpha", -alpha)
    z = kf.kf_axpy(q.script, na, v, w)
    r = kf.kf_dot(q.script, z, u)
    _out(q, "z", z)
    _out(q, "r", r)
    return q


def waxpby(n: int, alpha: float, beta: float) -> Sequence:
    q = _seq("waxpby")
    x, y = _vec(q, "x", n), _vec(q, "y", n)
    a, b = _const(q, "alpha", alpha), _const(q, "beta", beta)
    t = kf.kf_scal(q.script, b, y)
    w = kf.kf_axpy(q.script, a, x, t)
    _out(q, "w", w)
    return q


def bicgk(m: int, n: int, ld: int = 0, layout: int = kf.KF_ROW_MAJOR) -> Sequence:
    q = _seq("bicgk")
    A = _mat(q, "A", m, n, ld, layout)
    p, r = _vec(q, "p", n), _vec(q, "r", m)
    one = _const(q, "one", 1.0)
    qq = kf.kf_gemv(q.script, one, A, p)
    ss = kf.kf_gemtv(q.script, one, A, r)
    _out(q, "q", qq)
    _out(q, "s", ss)
    return q


def atax(m: int, n: int, ld: int = 0, layout: int = kf.KF_ROW_MAJOR) -> Sequence:
    q = _seq("atax")
    A = _mat(q, "A", m, n, ld, layout)
    x = _vec(q, "x", n)
    one = _const(q, "one", 1.0)
    t = kf.kf_gemv(q.script, one, A, x)
    y = kf.kf_gemtv(q.script, one, A, t)
    _out(q, "y", y)
    return q


def gesummv(m: int, n: int, alpha: float, beta: float, lda: int = 0, ldb: int = 0,
            layout: int = kf.KF_ROW_MAJOR) -> Sequence:
    q = _seq("gesummv")
    A = _mat(q, "A", m, n, lda, layout)
    B = _mat(q, "B", m, n, ldb, layout)
    x = _vec(q, "x", n)
    a, b, one = _const(q, "alpha", alpha), _const(q, "beta", beta), _const(q, "one", 1.0)
    t = kf.kf_gemv(q.script, a, A, x)
    y = kf.kf_gemv(q.script, b, B, x, one, t)
    _out(q, "y", y)
    return q


def gemver(m: int, n: int, alpha: float, beta: float, ld: int = 0,
           layout: int = kf.KF_ROW_MAJOR) -> Sequence:
    q = _seq("gemver")
    A = _mat(q, "A", m, n, ld, layout)
    u1, v1 = _vec(q, "u1", m), _vec(q, "v1", n)
    u2, v2 = _vec(q, "u2", m), _vec(q, "v2", n)
    y, z = _vec(q, "y", m), _vec(q, "z", n)
    a, b, one = _const(q, "alpha", alpha), _const(q, "beta", beta), _const(q, "one", 1.0)
    B1 = kf.kf_ger(q.script, one, A, u1, v1)
    B = kf.kf_ger(q.script, one, B1, u2, v2)
    x = kf.kf_gemtv(q.script, b, B, y, one, z)
    w = kf.kf_gemv(q.script, a, B, x)
    _out(q, "B", B)
    _out(q, "x", x)
    _out(q, "w", w)
    return q


def gemver_dev(m: int, n: int) -> Sequence:
    """GEMVER with alpha and beta in device memory (inputs "alpha", "beta"), so
    that one plan serves instances with their own scalars."""
    q = _seq("gemver")
    A = _mat(q, "A", m, n)
    u1, v1 = _vec(q, "u1", m), _vec(q, "v1", n)
    u2, v2 = _vec(q, "u2", m), _vec(q, "v2", n)
    y, z = _vec(q, "y", m), _vec(q, "z", n)
    a, b = _dscalar(q, "alpha"), _dscalar(q, "beta")
    one = _const(q, "one", 1.0)
    B1 = kf.kf_ger(q.script, one, A, u1, v1)
    B = kf.kf_ger(q.script, one, B1, u2, v2)
    x = kf.kf_gemtv(q.script, b, B, y, one, z)
    w = kf.kf_gemv(q.script, a, B, x)
    _out(q, "B", B)
    _out(q, "x", x)
    _out(q, "w", w)
    return q


def sgemvt(m: int, n: int, alpha: float, beta: float, ld: int = 0,
           layout: int = kf.KF_ROW_MAJOR) -> Sequence:
    """x = beta A^T y + z; w = alpha A x (the gemv needs all of x: two kernels
    under the strip rules)."""
    q = _seq("sgemvt")
    A = _mat(q, "A", m, n, ld, layout)
    y, z = _vec(q, "y", m), _vec(q, "z", n)
    a, b, one = _const(q, "alpha", alpha), _const(q, "beta", beta), _const(q, "one", 1.0)
    x = kf.kf_gemtv(q.script, b, A, y, one, z)
    w = kf.kf_gemv(q.script, a, A, x)
    _out(q, "x", x)
    _out(q, "w", w)
    return q


def vadd(n: int) -> Sequence:
    """x = w + y + z as two axpy calls with unit scale."""
    q = _seq("vadd")
    w, y, z = _vec(q, "w", n), _vec(q, "y", n), _vec(q, "z", n)
    one = _const(q, "one", 1.0)
    t = kf.kf_axpy(q.script, one, w, y)
    x = kf.kf_axpy(q.script, one, t, z)
    _out(q, "x", x)
    return q


BUILDERS = {"axpydot": axpydot, "waxpby": waxpby, "bicgk": bicgk, "atax": atax,
            "gesummv": gesummv, "gemver": gemver, "sgemvt": sgemvt, "vadd": vadd}


def by_name(name: str, m: int, n: int, scal: dict, ld: int = 0, layout: int = kf.KF_ROW_MAJOR) -> Sequence:
    """Sequence `name` on an m x n matrix (BLAS-2, in `layout`) or n-entry vectors (BLAS-1)."""
    if name == "axpydot":
        return axpydot(n, scal["alpha"])
    if name == "waxpby":
        return waxpby(n, scal["alpha"], scal["beta"])
    if name == "bicgk":
        return bicgk(m, n, ld, layout=layout)
    if name == "atax":
        return atax(m, n, ld, layout=layout)
    if name == "gesummv":
        return gesummv(m, n, scal["alpha"], scal["beta"], ld, ld, layout=layout)
    if name == "sgemvt":
        return sgemvt(m, n, scal["alpha"], scal["beta"], ld, layout=layout)
    if name == "vadd":
        return vadd(n)
    if name == "gemver":
        return gemver(m, n, scal["alpha"], scal["beta"], ld, layout=layout)
    raise KeyError(name)


def _qmat(q, name, rows, cols, fmt):
    """Matrix input in storage format fmt ('f32', 'bf16', 'fp8') with its row scales."""
    if fmt == "f32":
        return _mat(q, name, rows, cols)
    sc = _vec(q, name + "_scale", rows)
    v = kf.kf_matrix_q(q.script, rows, cols, fmt, sc)
    kf.kf_input(q.script, v)
    ld = kf.kf_value_info(q.script, v)[3]
    q.values[name] = v
    q.inputs.append(name)
    q.shapes[name] = (rows, ld)
    q.dtypes = getattr(q, "dtypes", {})
    q.dtypes[name] = fmt
    return v


def bicgk_q(m: int, n: int, fmt: str) -> Sequence:
    """BiCGK with A stored as fmt (row-scaled BF16 / FP8-E4M3, or FP32)."""
    q = _seq("bicgk_" + fmt)
    A = _qmat(q, "A", m, n, fmt)
    p, r = _vec(q, "p", n), _vec(q, "r", m)
    one = _const(q, "one", 1.0)
    _out(q, "q", kf.kf_gemv(q.script, one, A, p))
    _out(q, "s", kf.kf_gemtv(q.script, one, A, r))
    return q


def gemver_q(m: int, n: int, alpha: float, beta: float, fmt: str) -> Sequence:
    """GEMVER with A stored as fmt; B, x, w are FP32."""
    q = _seq("gemver_" + fmt)
    A = _qmat(q, "A", m, n, fmt)
    u1, v1 = _vec(q, "u1", m), _vec(q, "v1", n)
    u2, v2 = _vec(q, "u2", m), _vec(q, "v2", n)
    y, z = _vec(q, "y", m), _vec(q, "z", n)
    a, b, one = _const(q, "alpha", alpha), _const(q, "beta", beta), _const(q, "one", 1.0)
    B1 = kf.kf_ger(q.script, one, A, u1, v1)
    B = kf.kf_ger(q.script, one, B1, u2, v2)
    x = kf.kf_gemtv(q.script, b, B, y, one, z)
    w = kf.kf_gemv(q.script, a, B, x)
    _out(q, "B", B)
    _out(q, "x", x)
    _out(q, "w", w)
    return q


def decode_probe(ncodes: int, fmt: str) -> Sequence:
    """gemtv of a 1 x ncodes matrix in format fmt by x = [1]: returns the decoded row."""
    q = _seq("decode_" + fmt)
    A = _qmat(q, "A", 1, ncodes, fmt)
    x = _vec(q, "x", 1)
    one = _const(q, "one", 1.0)
    _out(q, "y", kf.kf_gemtv(q.script, one, A, x))
    return q
