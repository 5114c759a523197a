"""Seeded synthetic workloads of the Table 1 sequences.

Sizes and distributions: the paper states none, so the single-instance suite
uses n = 16384 (A is 16384 x 16384 row-major FP32, 1 GiB) and 2**26-entry
vectors, all entries uniform on [-1, 1) and scalars uniform on [0.5, 2]; the
small parity case is BiCGK at n = 1024. Tensor ids follow the order in which
the sequence declares its operands; the seed is ``1000 * suite + index``.
"""
from __future__ import annotations

import numpy as np

from . import inputs as I

# operand declaration order of each sequence (tensor ids 0, 1, 2, ...)
OPERANDS = {
    "axpydot": ["w", "v", "u"],
    "waxpby": ["x", "y"],
    "bicgk": ["A", "p", "r"],
    "atax": ["A", "x"],
    "gesummv": ["A", "B", "x"],
    "gemver": ["A", "u1", "v1", "u2", "v2", "y", "z"],
    "sgemvt": ["A", "y", "z"],
    "vadd": ["w", "y", "z"],
}
SCALARS = {"axpydot": ["alpha"], "waxpby": ["alpha", "beta"], "bicgk": [], "atax": [],
           "gesummv": ["alpha", "beta"], "gemver": ["alpha", "beta"], "sgemvt": ["alpha", "beta"],
           "vadd": []}
MATRIX = {"A", "B"}
ORDER = ["axpydot", "waxpby", "bicgk", "atax", "gesummv", "gemver"]
# further Table 1 sequences with more than one call (not in the headline suite)
EXTRA = ["sgemvt", "vadd"]
SEQ_INDEX = {name: i for i, name in enumerate(ORDER + EXTRA)}
BLAS1 = {"axpydot", "waxpby", "vadd"}

SUITE_N = 16384
SUITE_VEC = 1 << 26


def seed_for(suite: int, name: str) -> int:
    return 1000 * suite + SEQ_INDEX[name]


def vector_length(name: str, which: str, m: int, n: int) -> int:
    """Length of vector operand `which` for an m x n matrix (BLAS-2) or n (BLAS-1)."""
    if name in BLAS1:
        return n
    row_indexed = {"bicgk": {"r"}, "atax": set(), "gesummv": set(),
                   "gemver": {"u1", "u2", "y"}, "sgemvt": {"y"}}[name]
    return m if which in row_indexed else n


def make(name: str, m: int, n: int, seed: int, ld: int | None = None, pad_value=np.nan):
    """Operands (float32 numpy) and scalars (python floats) of one instance."""
    arrays = {}
    for tid, op in enumerate(OPERANDS[name]):
        if op in MATRIX:
            arrays[op] = I.matrix(seed, tid, m, n, ld=ld if ld else I.padded_ld(n),
                                  pad_value=pad_value)
        else:
            arrays[op] = I.vector(seed, tid, vector_length(name, op, m, n))
    scal = {}
    for j, sname in enumerate(SCALARS[name]):
        scal[sname] = I.scalar_uniform(seed, 100 + j, 0.5, 2.0)
    return arrays, scal


def reduction_length(name: str, m: int, n: int) -> int:
    """Longest reduction feeding an output (sets the accuracy tolerance)."""
    if name in BLAS1:
        return n
    return max(m, n)


def tolerance(name: str, m: int, n: int) -> float:
    """Relative L2 error bound 1e-5 * log2(n) against the FP64 oracle."""
    return 1e-5 * max(1.0, float(np.log2(reduction_length(name, m, n))))


def rel_l2(got, ref) -> float:
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = float(np.linalg.norm(ref))
    num = float(np.linalg.norm(got - ref))
    return num / den if den > 0 else num


# Implementation parameters the benchmark uses for the suite at n = 16384 and
# 2**26-entry vectors, per plan kind, as chosen by the autotuner
# (``python bench.py --tune``: every grid point timed kernel by kernel inside
# whole runs, median of 10). A "kernel_params" list gives each plan kernel its
# own point (Section 4.2: one implementation per fused kernel), in launch order.
_S1 = dict(mat_k=1, mat_waves=4, mat_group=2, mat_rows=1024)      # strips, 4 waves, 2 rows per step
_R16 = dict(mat_sched=1, mat_waves=16, mat_group=2)                 # row-resident, 16 waves, 2 rows per group
_LONG = dict(mat_k=2, mat_waves=4, mat_group=2, mat_rows=2048)     # 2 KiB strips down 2048 rows
# Row-resident points: a sweep of waves 8/16 x rows per group 1/2/4 x rows per
# workgroup 0-128 put 16 waves, two rows per group first for every
# row-resident kernel of the suite (GEMVER's gemv 154 us, SGEMVT's 153 us,
# GESUMMV 301 us with 32 rows per workgroup).
TUNED = {
    ("bicgk", "fused"): _S1, ("bicgk", "unfused"): dict(kernel_params=[_R16, _S1]),
    ("atax", "fused"): {},   # row-resident (t = A x feeds A^T t in the kernel): library defaults
    ("atax", "unfused"): dict(kernel_params=[_R16, _S1]),
    ("gesummv", "fused"): dict(mat_sched=1, mat_waves=16, mat_group=2, mat_rows=32),
    ("gesummv", "unfused"): _R16,
    # K1 {ger, ger, gemtv} streams A in and B out; K2 {gemv} reads B
    ("gemver", "fused"): dict(kernel_params=[_LONG, _R16]),
    # one point for all four kernels: measured faster than the per-kernel choice
    ("gemver", "unfused"): dict(mat_k=2, mat_waves=8, mat_group=2, mat_rows=1024),
    ("axpydot", "fused"): dict(vec_unroll=4, vec_threads=256, vec_grid=16384),
    ("axpydot", "unfused"): dict(vec_unroll=4, vec_threads=256, vec_grid=16384),
    ("waxpby", "fused"): dict(vec_unroll=4, vec_threads=256, vec_grid=16384),
    ("waxpby", "unfused"): dict(vec_unroll=4, vec_threads=256, vec_grid=16384),
    ("sgemvt", "fused"): dict(kernel_params=[_S1, _R16]),
    ("sgemvt", "unfused"): dict(kernel_params=[_S1, _R16]),
    ("vadd", "fused"): dict(vec_unroll=4, vec_threads=256, vec_grid=16384),
    ("vadd", "unfused"): dict(vec_unroll=4, vec_threads=256, vec_grid=16384),
}


# Fused plans of column-major A at the suite shape. The calls run on the
# row-major storage of A^T with gemv and gemtv swapped. BiCGK keeps its strip
# point, and column-major ATAX takes row-major SGEMVT's two kernels. Column-major
# SGEMVT {gemv, gemtv} and GEMVER {ger, ger, gemv, gemtv} are one row-resident
# kernel each. Their points come from a grid search: waves 8/16, rows per
# reduction 1/2/4, rows per block 0-128 (16 waves and two rows per group first
# for both, 32 rows per block for GEMVER).
LAYOUT_TUNED = {
    "bicgk": _S1,
    "atax": TUNED[("sgemvt", "fused")],
    "sgemvt": _R16,
    "gemver": dict(mat_sched=1, mat_waves=16, mat_group=2, mat_rows=32),
}
LAYOUT_SEQ = ["bicgk", "atax", "sgemvt", "gemver"]


def tuned_params(name: str, m: int, n: int, mode: str = "fused") -> dict:
    """Tuned parameters for the suite shapes; library defaults elsewhere."""
    suite = (m, n) == ((SUITE_VEC, SUITE_VEC) if name in BLAS1 else (SUITE_N, SUITE_N))
    return dict(TUNED.get((name, mode), {})) if suite else {}


def traffic_from_profiles(profile_dir: str, kernel_name: str, batched: bool = False):
    """HBM bytes per launch of `kernel_name` from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE, scaled by the same counters of
    a streaming copy of known size), or None when the summary does not cover
    this exact kernel text (the name is a hash of it)."""
    import json
    import os
    path = os.path.join(profile_dir, "pmc_summary_batched.json" if batched else "pmc_summary.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    ks = d.get("kernels", {})
    k = ks.get(kernel_name)
    if k is None and batched:       # the batched kernel's record carries its full signature
        k = next((v for name, v in ks.items() if kernel_name in name), None)
    if not k:
        return None
    return int(round(k["fetch_bytes_scaled"] + k["write_bytes_scaled"]))


# rocprofv3 --kernel-trace --stats summary of the default benchmark command
SUITE_STATS_FILE = "suite_n16384_fused_kernel_stats.txt"


def kernel_stats_from_profiles(profile_dir: str, fname: str, kernel_name: str):
    """{file, command, calls, avg_us, min_us, max_us} of `kernel_name` in a
    committed rocprofv3 statistics summary, or None when the summary does not
    list this exact kernel (the name is a hash of its text)."""
    import os
    path = os.path.join(profile_dir, fname)
    if not os.path.exists(path):
        return None
    command = ""
    for line in open(path):
        if line.startswith("# command:"):
            command = line.split(":", 1)[1].strip()
        f = line.split()
        if len(f) >= 5 and f[0] == kernel_name:
            return {"file": "profiles/" + fname, "command": command, "calls": int(f[1]),
                    "avg_us": float(f[2]), "min_us": float(f[3]), "max_us": float(f[4])}
    return None


# ---- reduced-precision suite: A ~ N(0, 1) drawn in float64, stored per format
PREC_N = 32768
PREC_FORMATS = ("f32", "bf16", "fp8")
PREC_SEQ = ("bicgk", "gemver")


PREC_PANEL = 512
# tuned fused-plan parameters per (sequence, storage format) at n = 32768: each
# kernel's point varied with the others fixed, timed kernel by kernel inside
# whole runs; GEMVER's K2 reads the FP32 B whatever A's format
PREC_TUNED = {
    ("bicgk", "f32"): dict(mat_k=2, mat_waves=4, mat_group=2, mat_rows=2048),
    ("bicgk", "bf16"): dict(mat_k=2, mat_waves=4, mat_group=2, mat_rows=2048),
    ("bicgk", "fp8"): dict(mat_k=1, mat_waves=4, mat_group=2, mat_rows=1024),
    ("gemver", "f32"): dict(kernel_params=[dict(mat_k=1, mat_waves=8, mat_group=2, mat_rows=1024),
                                           dict(mat_sched=1, mat_waves=16, mat_group=2)]),
    # per-kernel points only: a plan-wide mat_rows would also set the rows per
    # workgroup of the row-resident K2
    ("gemver", "bf16"): dict(kernel_params=[dict(mat_k=1, mat_waves=8, mat_group=4, mat_rows=256),
                                            dict(mat_sched=1, mat_waves=16, mat_group=2, mat_rows=128)]),
    ("gemver", "fp8"): dict(kernel_params=[dict(mat_k=2, mat_waves=8, mat_group=2, mat_rows=1024),
                                           dict(mat_sched=1, mat_waves=16, mat_group=2, mat_rows=128)]),
}


def plan_wide(params: dict) -> dict:
    """One point for every kernel: the plan-wide fields, with the first
    kernel's own point on top (for plans whose kernels differ in number)."""
    out = {k: v for k, v in params.items() if k != "kernel_params"}
    kp = params.get("kernel_params")
    if kp:
        out.update(kp[0] or {})
    return out


def normal_panel(seed: int, n: int, r0: int, panel: int = PREC_PANEL) -> np.ndarray:
    """Rows r0 .. r0 + panel - 1 of the float64 N(0, 1) matrix: numpy PCG64
    seeded per row panel (seed, panel index), so any panel can be redrawn."""
    rng = np.random.Generator(np.random.PCG64([int(seed), int(r0 // panel)]))
    return rng.standard_normal((min(panel, n - r0), n))


def precision_inputs(name: str, n: int, formats, seed: int, panel: int = PREC_PANEL, keep=None):
    """Operands of BiCGK or GEMVER with A (n x n) drawn N(0, 1) in float64
    (row panels, normal_panel) and stored in each of `formats` with row
    scales; vectors uniform [-1, 1). Returns ({fmt: (storage, scales)},
    vectors, scalars). keep = (rows, cols) index arrays: the float64 rows and
    columns of A at those indices are also kept, in keep["A64_rows"] and
    keep["A64_cols"] (a dict passed in), without a second draw."""
    from concurrent.futures import ThreadPoolExecutor
    from . import quant as Q
    out = {}
    if keep is not None:
        krows, kcols = (np.asarray(keep["rows"], np.int64), np.asarray(keep["cols"], np.int64))
        keep["A64_rows"] = np.empty((len(krows), n))
        keep["A64_cols"] = np.empty((n, len(kcols)))

    ld = {"f32": (n + 3) // 4 * 4, "bf16": (n + 7) // 8 * 8, "fp8": (n + 15) // 16 * 16}
    dt = {"f32": np.float32, "bf16": np.uint16, "fp8": np.uint8}
    for f in formats:
        out[f] = (np.zeros((n, ld[f]), dt[f]), np.empty(n, np.float32))

    def do_panel(r0):
        A64 = normal_panel(seed, n, r0, panel)
        if keep is not None:
            mine = np.flatnonzero((krows >= r0) & (krows < r0 + A64.shape[0]))
            keep["A64_rows"][mine] = A64[krows[mine] - r0]
            keep["A64_cols"][r0:r0 + A64.shape[0]] = A64[:, kcols]
        for c0 in range(0, A64.shape[0], 4):          # small row groups stay in cache
            blk = A64[c0:c0 + 4]
            for f in formats:
                st, sc = Q.quantize_rows(blk, f, ld[f])
                out[f][0][r0 + c0:r0 + c0 + blk.shape[0]] = st
                out[f][1][r0 + c0:r0 + c0 + blk.shape[0]] = sc

    with ThreadPoolExecutor(I._threads()) as ex:
        list(ex.map(do_panel, range(0, n, panel)))
    names = ["p", "r"] if name == "bicgk" else ["u1", "v1", "u2", "v2", "y", "z"]
    vecs = {k: I.vector(seed, 1 + i, n) for i, k in enumerate(names)}
    scal = {} if name == "bicgk" else {"alpha": I.scalar_uniform(seed, 100), "beta": I.scalar_uniform(seed, 101)}
    return out, vecs, scal


def precision_arrays(fmt, stored, vecs):
    """Bindable arrays of one format (FP32 matrices take no scale vector)."""
    st, sc = stored[fmt]
    arrays = dict(vecs, A=st)
    if fmt != "f32":
        arrays["A_scale"] = sc
    return arrays


# ---- batched uneven sizes: 4096 BiCGK + 4096 GEMVER, n log-uniform on [32, 2048]
BATCH_COUNTS = (4096, 4096)
BATCH_SEED = 3000
# rows per work item for (BiCGK, GEMVER) x size bucket (n <= 64, 128, 256,
# 512, 1024, 2048) (0 = library default). Alone, every bucket but GEMVER's
# n <= 1024 runs fastest as whole instances (`bench.py --tune-batch`). The
# mixed batch wants otherwise: the coordinate search on the mixed batch itself
# (`bench.py --tune-batch-mix`, profiles/batch_autotune_mix.jsonl) cut GEMVER
# instances above n = 512 into 256-row items (6.05 ms against 6.38 ms from
# halved instances), which spreads the largest instances' work over more
# workgroups and shortens the tail of the launch, and kept every default tile
# (the per-bucket picks made the mix 13% slower).
BATCH_TUNED = {0: [64, 128, 256, 512, 1024, 1024], 1: [64, 128, 256, 512, 256, 256]}


# The per-instance launch loop (the baseline) launches one instance at a time,
# so it wants many small items per instance to fill the GPU: it keeps the
# library's default rows per item.
BATCH_LOOP_ROWS = {0: [0] * 6, 1: [0] * 6}


# Lane tile per kind and bucket (entries of the library's tile menus, 0 = the
# default tile), from the mixed-batch search above; no other tile beat a
# default by more than 0.3% there.
BATCH_TILES = {0: [0] * 6, 1: [0] * 6}


def batch_opts(grid: int = 0, loop: bool = False):
    from . import kf
    if loop:
        return kf.batch_opts(rows=BATCH_LOOP_ROWS, grid=grid)
    return kf.batch_opts(rows=BATCH_TUNED, tiles=BATCH_TILES, grid=grid)
