"""The all-core (OpenMP) build of the oracle gives the same bits as the
one-thread build: its threads split rows, entries or (for gemtv) columns, and
each output entry keeps its plain summation order. The benchmark times the
oracle on the host's cores with this build."""
import numpy as np
import pytest

import oracle
from paper_1305_1183_amd import inputs as I
from paper_1305_1183_amd import workloads as WL
from tests import seqcheck as SC


def _outputs(name, arrays, scal, n):
    return SC.oracle_outputs(name, arrays, scal, n)


@pytest.mark.parametrize("name", ["axpydot", "waxpby", "vadd", "bicgk", "atax", "gesummv", "gemver", "sgemvt"])
def test_all_cores_bitwise_equal(name):
    m, n = (100003, 100003) if name in WL.BLAS1 else (1000, 1001)
    arrays, scal = WL.make(name, m, n, seed=WL.seed_for(9, name))
    ref = _outputs(name, arrays, scal, n)
    with oracle.all_cores(4) as threads:
        assert threads == 4
        par = _outputs(name, arrays, scal, n)
    assert oracle.lib().kfo_threads() == 1     # the one-thread build is back in place
    for k in ref:
        assert np.array_equal(ref[k], par[k]), (name, k)


def test_all_cores_elementary_calls():
    m, n = 513, 777
    A = I.matrix(3, 0, m, n, ld=n).astype(np.float64)
    x, y = I.vector(3, 1, n).astype(np.float64), I.vector(3, 2, m).astype(np.float64)
    u, v = I.vector(3, 3, m).astype(np.float64), I.vector(3, 4, n).astype(np.float64)
    calls = lambda: [oracle.gemv(1.5, A, x, 0.5, y), oracle.gemtv(0.75, A, y, 2.0, x),
                     oracle.ger(1.25, A, u, v), oracle.scal(3.0, x), oracle.axpy(-1.5, x, v),
                     np.array([oracle.dot(x, v)])]
    ref = calls()
    with oracle.all_cores(3):
        par = calls()
    for a, b in zip(ref, par):
        assert np.array_equal(a, b)
