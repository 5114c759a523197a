"""Shared helpers of the GPU parity tests: build, run and compare one sequence
instance against the FP64 oracle."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_1305_1183_amd import sequences as S
from paper_1305_1183_amd import workloads as WL


def build_sequence(name, m, n, scal, ld=0):
    return S.by_name(name, m, n, scal, ld)


def oracle_outputs(name, arrays, scal, n):
    a = arrays
    if name == "axpydot":
        z, r = oracle.axpydot(scal["alpha"], a["w"], a["v"], a["u"])
        return {"z": z, "r": np.array([r])}
    if name == "waxpby":
        return {"w": oracle.waxpby(scal["alpha"], a["x"], scal["beta"], a["y"])}
    if name == "bicgk":
        q, s = oracle.bicgk(a["A"], a["p"], a["r"], cols=n)
        return {"q": q, "s": s}
    if name == "atax":
        return {"y": oracle.atax(a["A"], a["x"], cols=n)}
    if name == "gesummv":
        return {"y": oracle.gesummv(scal["alpha"], a["A"], scal["beta"], a["B"], a["x"], cols=n)}
    if name == "gemver":
        B, x, w = oracle.gemver(scal["alpha"], scal["beta"], a["A"], a["u1"], a["v1"], a["u2"],
                                a["v2"], a["y"], a["z"], cols=n)
        return {"B": B, "x": x, "w": w}
    if name == "sgemvt":
        x, w = oracle.sgemvt(scal["alpha"], scal["beta"], a["A"], a["y"], a["z"], cols=n)
        return {"x": x, "w": w}
    if name == "vadd":
        return {"x": oracle.vadd(a["w"], a["y"], a["z"])}
    raise KeyError(name)


def run_gpu(name, m, n, arrays, scal, mode="fused", ld=0, **params):
    q = build_sequence(name, m, n, scal, ld)
    prog = q.compile(mode=mode, **params)
    dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in arrays.items()}
    prog.bind(**dev)
    outs = prog.run()
    torch.cuda.synchronize()
    host = {k: v.cpu().numpy() for k, v in outs.items()}
    return q, prog, host


def check_against_oracle(name, m, n, host, ref, tol=None):
    tol = WL.tolerance(name, m, n) if tol is None else tol
    errs = {}
    for k, r in ref.items():
        g = host[k]
        if g.ndim == 2:
            g = g[:, :n]
        errs[k] = WL.rel_l2(g, r)
        assert np.all(np.isfinite(g)), (name, k, "non-finite output")
        assert errs[k] <= tol, (name, k, errs[k], tol)
    return errs
