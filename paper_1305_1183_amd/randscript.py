"""Seeded random scripts of BLAS-1/BLAS-2 calls for the plan-search study.

A script has 8-12 calls drawn from {scal, axpy, dot, gemv, gemtv, ger} over
shared operands, forming a DAG: square matrices of one size n in
{2^10 .. 2^15} (log-uniform), vectors of length n for the BLAS-2 calls and of
one BLAS-1 length in {2^14 .. 2^24}. Operands reuse earlier values with high
probability, so calls share data and fusions exist; outputs are the sinks plus
a random quarter of the other results. The matrices of a script fit in 48 GiB.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import kf

OPS = ["gemv", "gemtv", "ger", "axpy", "scal", "dot"]
WEIGHTS = np.array([0.22, 0.20, 0.12, 0.20, 0.10, 0.16])


@dataclass
class RandomScript:
    seed: int
    script: object
    n_mat: int
    n_vec: int
    inputs: dict = field(default_factory=dict)    # value id -> shape tuple
    outputs: dict = field(default_factory=dict)   # value id -> shape tuple
    calls: list = field(default_factory=list)     # op names in recording order

    def describe(self) -> str:
        return "seed %d n=%d vec=%d calls=%s" % (self.seed, self.n_mat, self.n_vec, ",".join(self.calls))


def random_script(seed: int, mem_cap: int = 48 << 30, min_calls: int = 8, max_calls: int = 12,
                  mat_log2=(10, 15), vec_log2=(14, 24)) -> RandomScript:
    rng = np.random.Generator(np.random.PCG64(seed))
    ncalls = int(rng.integers(min_calls, max_calls + 1))
    nm = 2 ** int(rng.integers(mat_log2[0], mat_log2[1] + 1))
    nv = 2 ** int(rng.integers(vec_log2[0], vec_log2[1] + 1))
    s = kf.kf_script_create()
    rs = RandomScript(seed=seed, script=s, n_mat=nm, n_vec=nv)
    mat_bytes = 4 * nm * nm
    max_mats = max(1, int(mem_cap // (2 * mat_bytes)))
    mats, vm, vv, scal = [], [], [], []
    consumers = {}

    def use(v):
        consumers[v] = consumers.get(v, 0) + 1
        return v

    def new_vec(n):
        v = kf.kf_vector(s, n)
        kf.kf_input(s, v)
        rs.inputs[v] = (n,)
        (vm if n == nm else vv).append(v)
        return v

    def pick_vec(pool, n, p_reuse=0.75, avoid=None):
        cand = [v for v in pool if v != avoid]
        if cand and rng.random() < p_reuse:
            return use(cand[int(rng.integers(len(cand)))])
        return use(new_vec(n))

    def alpha():
        if scal and rng.random() < 0.3:
            return use(scal[int(rng.integers(len(scal)))])
        return kf.kf_const(s, float(np.float32(rng.uniform(0.5, 2.0))))

    for _ in range(ncalls):
        op = OPS[int(rng.choice(len(OPS), p=WEIGHTS))]
        if op in ("gemv", "gemtv", "ger"):
            if mats and (rng.random() < 0.8 or len(mats) >= max_mats):
                A = use(mats[int(rng.integers(len(mats)))])
            else:
                A = kf.kf_matrix(s, nm, nm, 0)
                kf.kf_input(s, A)
                rs.inputs[A] = (nm, kf.kf_value_info(s, A)[3])
                mats.append(A)
                use(A)
            if op == "ger":
                if len(mats) >= max_mats:
                    op = "gemv"
                else:
                    u = pick_vec(vm, nm)
                    v = pick_vec(vm, nm)
                    B = kf.kf_ger(s, alpha(), A, u, v)
                    mats.append(B)
            if op in ("gemv", "gemtv"):
                x = pick_vec(vm, nm)
                fn = kf.kf_gemv if op == "gemv" else kf.kf_gemtv
                if vm and rng.random() < 0.3:
                    y0 = pick_vec(vm, nm, p_reuse=0.9, avoid=x)
                    y = fn(s, alpha(), A, x, kf.kf_const(s, float(np.float32(rng.uniform(0.5, 2.0)))), y0)
                else:
                    y = fn(s, alpha(), A, x)
                vm.append(y)
        else:
            if vm and rng.random() < 0.3:
                pool, n = vm, nm
            else:
                pool, n = vv, nv
            if op == "scal":
                y = kf.kf_scal(s, alpha(), pick_vec(pool, n))
                pool.append(y)
            elif op == "axpy":
                x = pick_vec(pool, n)
                z = kf.kf_axpy(s, alpha(), x, pick_vec(pool, n, avoid=x))
                pool.append(z)
            else:
                x = pick_vec(pool, n)
                r = kf.kf_dot(s, x, pick_vec(pool, n))
                scal.append(r)
        rs.calls.append(op)
    # outputs: every computed value nobody consumes, plus a quarter of the rest
    produced = [v for v in set(mats + vm + vv + scal) if v not in rs.inputs]
    for v in sorted(produced):
        if consumers.get(v, 0) == 0 or rng.random() < 0.25:
            kf.kf_output(s, v)
            kind, d0, d1, d2 = kf.kf_value_info(s, v)
            rs.outputs[v] = {0: (d0,), 1: (d0, d2), 3: (1,)}[kind]
    return rs
