"""Plant plausible mistakes in a copy of the oracle and check the pins catch them.

Each mutant is the oracle source with one textual change (a dropped term, a
flipped sign, a wrong operand or index), compiled to a temporary library on
the CPU. The pins of ``test_oracle_pins`` must reject every mutant; the real
oracle source is never modified.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests.test_oracle_pins import ALL_PINS

SRC = os.path.join(os.path.dirname(oracle.__file__), "kf_oracle.c")

MUTANTS = {
    "scal_add": ("y[i] = alpha * x[i];", "y[i] = alpha + x[i];"),
    "axpy_sign": ("z[i] = alpha * x[i] + y[i];", "z[i] = alpha * x[i] - y[i];"),
    "dot_drop_first": ("s += x[i] * y[i];", "s += (i > 0) ? x[i] * y[i] : 0.0;"),
    "gemv_no_alpha": ("y[i] = alpha * s + (y0 ? beta * y0[i] : 0.0);",
                      "y[i] = s + (y0 ? beta * y0[i] : 0.0);"),
    "gemv_beta_dropped": ("y[i] = alpha * s + (y0 ? beta * y0[i] : 0.0);",
                          "y[i] = alpha * s + (y0 ? y0[i] : 0.0);"),
    "gemtv_alpha_for_beta": ("y[j] = alpha * s + (y0 ? beta * y0[j] : 0.0);",
                             "y[j] = alpha * s + (y0 ? alpha * y0[j] : 0.0);"),
    "gemtv_reversed_x": ("s += a[i * n + j] * x[i];", "s += a[i * n + j] * x[m - 1 - i];"),
    "ger_reversed_v": ("alpha * u[i] * v[j];", "alpha * u[i] * v[n - 1 - j];"),
    "axpydot_sign": ("kfo_axpy(n, -alpha, vd, wd, z);", "kfo_axpy(n, alpha, vd, wd, z);"),
    "waxpby_wrong_scalar": ("kfo_scal(n, beta, yd, t);", "kfo_scal(n, alpha, yd, t);"),
    "bicgk_wrong_vector": ("kfo_gemtv(m, n, 1.0, ad, rd, 0.0, NULL, s);",
                           "kfo_gemtv(m, n, 1.0, ad, pd, 0.0, NULL, s);"),
    "atax_skips_ax": ("kfo_gemtv(m, n, 1.0, ad, t, 0.0, NULL, y);",
                      "kfo_gemtv(m, n, 1.0, ad, xd, 0.0, NULL, y);"),
    "gesummv_drops_a": ("kfo_gemv(m, n, beta, bd, xd, 1.0, t, y);",
                        "kfo_gemv(m, n, beta, bd, xd, 0.0, t, y);"),
    "gemver_drops_u2v2": ("kfo_ger(m, n, 1.0, b1, u2d, v2d, b);",
                          "kfo_ger(m, n, 0.0, b1, u2d, v2d, b);"),
    "gemver_drops_z": ("kfo_gemtv(m, n, beta, b, yd, 1.0, zd, x);",
                       "kfo_gemtv(m, n, beta, b, yd, 0.0, zd, x);"),
    "gemver_w_uses_a": ("kfo_gemv(m, n, alpha, b, x, 0.0, NULL, w);",
                        "kfo_gemv(m, n, alpha, ad, x, 0.0, NULL, w);"),
    "mat_ignores_ld": ("dst[i * n + j] = (double)a[i * ld + j];",
                       "dst[i * n + j] = (double)a[i * n + j];"),
    "rows_ignores_ld": ("const float* row = a + idx[k] * ld;",
                        "const float* row = a + idx[k] * n;"),
    "cols_ignores_ld": ("s += (double)a[i * ld + idx[k]] * x[i];",
                        "s += (double)a[i * n + idx[k]] * x[i];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not unique: %s" % name
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    so = tmp_path / ("libmutant_%s.so" % name)
    hdr_dir = os.path.dirname(SRC)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                           "-I", hdr_dir, "-o", str(so), str(mpath)])
    monkeypatch.setattr(oracle, "_lib", oracle.load(str(so)))
    failures = []
    for pin in ALL_PINS:
        try:
            pin(oracle)
        except AssertionError:
            failures.append(pin.__name__)
    assert failures, "mutant %s passed every pin" % name


def _sgemvt_transposed(alpha, beta, A, y, z, cols=None):
    n = int(cols) if cols is not None else A.shape[1]
    Ad = np.asarray(A)[:, :n].astype(np.float64)
    x = oracle.gemtv(beta, Ad, np.asarray(y, dtype=np.float64), 1.0, np.asarray(z, dtype=np.float64))
    if Ad.shape[0] != Ad.shape[1]:
        return x, oracle.gemv(alpha, Ad, x)
    return x, oracle.gemtv(alpha, Ad, x)          # A^T x where A x is meant


def _sgemvt_swapped_scalars(alpha, beta, A, y, z, cols=None):
    return oracle.sgemvt(beta, alpha, A, y, z, cols)


def _sgemvt_drops_z(alpha, beta, A, y, z, cols=None):
    return oracle.sgemvt(alpha, beta, A, y, np.zeros_like(np.asarray(z)), cols)


def _vadd_drops_z(w, y, z):
    return oracle.axpy(1.0, np.asarray(w, dtype=np.float64), np.asarray(y, dtype=np.float64))


def _vadd_sub(w, y, z):
    return oracle.axpy(-1.0, oracle.axpy(1.0, np.asarray(w, np.float64), np.asarray(y, np.float64)),
                       np.asarray(z, np.float64))


PY_MUTANTS = {"sgemvt_gemv_as_gemtv": ("sgemvt", _sgemvt_transposed),
              "sgemvt_swapped_scalars": ("sgemvt", _sgemvt_swapped_scalars),
              "sgemvt_drops_z": ("sgemvt", _sgemvt_drops_z),
              "vadd_drops_z": ("vadd", _vadd_drops_z),
              "vadd_subtracts": ("vadd", _vadd_sub)}


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_composition_mutant_is_caught(name):
    """Mistakes in the Python-level sequence compositions fail a pin too."""
    import types
    attr, fn = PY_MUTANTS[name]
    O = types.SimpleNamespace(**{k: getattr(oracle, k) for k in dir(oracle) if not k.startswith("__")})
    setattr(O, attr, fn)
    failures = []
    for pin in ALL_PINS:
        try:
            pin(O)
        except AssertionError:
            failures.append(pin.__name__)
    assert failures, "mutant %s passed every pin" % name
