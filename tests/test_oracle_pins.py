"""Pins of the FP64 oracle against facts it does not compute itself.

Each check below is a closed form, an exact special case, an invariant or a
library routine -- never the oracle's own formula retyped -- chosen so that a
dropped term, a wrong sign, a wrong index or a transposed operand in any
oracle routine fails at least one of them (``test_oracle_mutants`` plants such
mistakes in a copy of the oracle source and checks that they are caught).
"""
import numpy as np
import pytest

from paper_1305_1183_amd import inputs as I

pytestmark = pytest.mark.filterwarnings("ignore")


def _ints(seed, tid, shape, lo=-4, hi=4):
    n = int(np.prod(shape))
    return I.small_ints(seed, tid, n, lo, hi).reshape(shape)


# --------------------------------------------------------------------- pins
def pin_elementary(O):
    """scal/axpy/dot/gemv/gemtv/ger pins (Section 3.3 definitions)."""
    m, n = 5, 7
    x = _ints(1, 0, (n,)).astype(np.float64)
    y = _ints(1, 1, (n,)).astype(np.float64)
    # scal and axpy with dyadic scalars are exact: compare to hand-known values
    assert np.array_equal(O.scal(2.0, x), x + x)
    assert np.array_equal(O.axpy(-0.5, x, y), y - x / 2)
    # dot: ones.ones = n; integer data -> exact and symmetric
    assert O.dot(np.ones(n), np.ones(n)) == n
    assert O.dot(x, y) == O.dot(y, x) == float(sum(int(a) * int(b) for a, b in zip(x, y)))
    # rank-1 non-square A = a b^T:  A p = a (b.p),  A^T r = b (a.r)  (catches transposes)
    a = _ints(1, 2, (m,)).astype(np.float64)
    b = _ints(1, 3, (n,)).astype(np.float64)
    A = np.outer(a, b)
    p = _ints(1, 4, (n,)).astype(np.float64)
    r = _ints(1, 5, (m,)).astype(np.float64)
    assert np.array_equal(O.gemv(1.0, A, p), a * float(b @ p))
    assert np.array_equal(O.gemtv(1.0, A, r), b * float(a @ r))
    # alpha/beta placement: y = alpha*S + beta*y0 with dyadic alpha, beta
    y0 = _ints(1, 6, (m,)).astype(np.float64)
    assert np.array_equal(O.gemv(2.0, A, p, 0.25, y0), 2 * a * float(b @ p) + y0 / 4)
    y1 = _ints(1, 7, (n,)).astype(np.float64)
    assert np.array_equal(O.gemtv(0.5, A, r, 4.0, y1), b * float(a @ r) / 2 + 4 * y1)
    # identity and diagonal matrices
    d = _ints(1, 8, (n,), 1, 5).astype(np.float64)
    assert np.array_equal(O.gemv(1.0, np.diag(d), p), d * p)
    assert np.array_equal(O.gemtv(1.0, np.eye(n), p), p)
    # adjoint identity r^T (A p) == (A^T r)^T p for a general non-square A
    G = _ints(1, 9, (m, n)).astype(np.float64)
    assert float(r @ O.gemv(1.0, G, p)) == float(O.gemtv(1.0, G, r) @ p)
    # ger: A + alpha u v^T  on A = 0 equals the outer product; entries by hand
    u = _ints(1, 10, (m,)).astype(np.float64)
    v = _ints(1, 11, (n,)).astype(np.float64)
    B = O.ger(2.0, G, u, v)
    for i in (0, m - 1):
        for j in (0, 3, n - 1):
            assert B[i, j] == G[i, j] + 2 * u[i] * v[j]
    assert np.array_equal(O.ger(1.0, np.zeros((m, n)), u, v), np.outer(u, v))


def pin_library(O):
    """Random float data: numpy float64 (BLAS) agrees to 1e-12 relative."""
    m, n = 37, 53
    A = I.matrix(3, 0, m, n).astype(np.float64)
    x = I.vector(3, 1, n).astype(np.float64)
    r = I.vector(3, 2, m).astype(np.float64)
    np.testing.assert_allclose(O.gemv(1.5, A, x), 1.5 * (A @ x), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(O.gemtv(0.75, A, r), 0.75 * (A.T @ r), rtol=1e-12, atol=1e-12)
    assert abs(O.dot(x, x) - float(np.dot(x, x))) <= 1e-12 * float(np.dot(x, x))


def pin_axpydot(O):
    n = 1001
    v = I.vector(4, 0, n)
    u = I.vector(4, 1, n)
    # w = 2 v and alpha = 2 make z identically zero and r = 0 (sign pin)
    z, r = O.axpydot(2.0, 2 * v, v, u)
    assert np.all(z == 0.0) and r == 0.0
    # linearity: r = w.u - alpha v.u with dyadic alpha on integer data (exact)
    w = I.small_ints(4, 2, n, -8, 8)
    vi = I.small_ints(4, 3, n, -8, 8)
    ui = I.small_ints(4, 4, n, -8, 8)
    z, r = O.axpydot(0.5, w, vi, ui)
    wi, vv, uu = (a.astype(np.int64) for a in (w, vi, ui))
    assert r == float((2 * wi - vv) @ uu) / 2
    assert np.array_equal(z, w.astype(np.float64) - vi.astype(np.float64) / 2)


def pin_waxpby(O):
    n = 777
    x = I.vector(5, 0, n)
    y = I.vector(5, 1, n)
    w = O.waxpby(2.0, x, 0.5, y)
    # powers-of-two scalars: one rounding at most, and both terms present
    assert np.array_equal(w, 2.0 * x.astype(np.float64) + 0.5 * y.astype(np.float64))
    assert np.array_equal(O.waxpby(1.0, x, 0.0, y), x.astype(np.float64))
    assert np.array_equal(O.waxpby(0.0, x, 1.0, y), y.astype(np.float64))


def pin_bicgk(O):
    m, n = 6, 9
    a = I.small_ints(6, 0, m, -3, 3)
    b = I.small_ints(6, 1, n, -3, 3)
    A = np.outer(a, b).astype(np.float32)
    p = I.vector(6, 2, n)
    r = I.vector(6, 3, m)
    q, s = O.bicgk(A, p, r)
    # rank-1 A: q = a (b.p), s = b (a.r) with exact float64 inner products
    bp = float(np.dot(b.astype(np.float64), p.astype(np.float64)))
    ar = float(np.dot(a.astype(np.float64), r.astype(np.float64)))
    np.testing.assert_allclose(q, a.astype(np.float64) * bp, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(s, b.astype(np.float64) * ar, rtol=1e-15, atol=1e-15)
    # identity: q = p, s = r (square)
    k = 8
    e = np.eye(k, dtype=np.float32)
    pp = I.vector(6, 4, k)
    rr = I.vector(6, 5, k)
    q, s = O.bicgk(e, pp, rr)
    assert np.array_equal(q, pp.astype(np.float64)) and np.array_equal(s, rr.astype(np.float64))
    # padded leading dimension: NaN padding must never reach the result
    G = I.matrix(6, 6, m, n, ld=12)
    q1, s1 = O.bicgk(G, p, r, cols=n)
    q2, s2 = O.bicgk(np.ascontiguousarray(G[:, :n]), p, r)
    assert np.array_equal(q1, q2) and np.array_equal(s1, s2) and np.all(np.isfinite(q1))


def pin_atax(O):
    # diagonal A: y_i = d_i^2 x_i (dyadic values, exact)
    n = 10
    d = I.small_ints(7, 0, n, -4, 4) / 2
    x = I.small_ints(7, 1, n, -6, 6) / 4
    y = O.atax(np.diag(d).astype(np.float32), x.astype(np.float32))
    assert np.array_equal(y, (d.astype(np.float64) ** 2) * x)
    # rank-1 non-square: A^T A x = b (a.a)(b.x)
    m, n = 4, 7
    a = I.small_ints(7, 2, m, -3, 3)
    b = I.small_ints(7, 3, n, -3, 3)
    xx = I.small_ints(7, 4, n, -3, 3)
    y = O.atax(np.outer(a, b).astype(np.float32), xx)
    expect = b.astype(np.float64) * (float(a @ a) * float(b @ xx))
    assert np.array_equal(y, expect)


def pin_gesummv(O):
    m, n = 11, 13
    A = I.matrix(8, 0, m, n)
    x = I.vector(8, 1, n)
    # B = A:  y = (alpha + beta) A x   (both terms present, same x)
    y = O.gesummv(0.75, A, 1.25, A, x)
    ref = 2.0 * (A.astype(np.float64) @ x.astype(np.float64))
    np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-13)
    # identity A = B:  y = (alpha + beta) x
    e = np.eye(n, dtype=np.float32)
    y = O.gesummv(0.5, e, 0.25, e, x)
    assert np.array_equal(y, 0.75 * x.astype(np.float64))
    # B = -A with alpha = beta cancels exactly
    y = O.gesummv(1.5, A, 1.5, -A, x)
    assert np.all(y == 0.0)


def pin_gemver(O):
    m, n = 5, 8
    A = np.zeros((m, n), dtype=np.float32)
    u1, u2 = I.small_ints(9, 0, m, -3, 3), I.small_ints(9, 1, m, -3, 3)
    v1, v2 = I.small_ints(9, 2, n, -3, 3), I.small_ints(9, 3, n, -3, 3)
    y = I.small_ints(9, 4, m, -3, 3)
    z = I.small_ints(9, 5, n, -3, 3)
    alpha, beta = 0.5, 2.0
    B, x, w = O.gemver(alpha, beta, A, u1, v1, u2, v2, y, z)
    f = lambda a: a.astype(np.float64)
    # A = 0: B = u1 v1^T + u2 v2^T;  x = beta (v1 (u1.y) + v2 (u2.y)) + z;
    # w = alpha (u1 (v1.x) + u2 (v2.x)) -- every stage exact in float64
    assert np.array_equal(B, np.outer(f(u1), f(v1)) + np.outer(f(u2), f(v2)))
    xe = beta * (f(v1) * float(f(u1) @ f(y)) + f(v2) * float(f(u2) @ f(y))) + f(z)
    assert np.array_equal(x, xe)
    we = alpha * (f(u1) * float(f(v1) @ xe) + f(u2) * float(f(v2) @ xe))
    assert np.array_equal(w, we)
    # u = 0 reduces GEMVER to x = beta A^T y + z, w = alpha A x (numpy float64)
    G = I.matrix(9, 6, m, n)
    zero_m = np.zeros(m, np.float32)
    yy = I.vector(9, 7, m)
    zz = I.vector(9, 8, n)
    B, x, w = O.gemver(1.5, 0.75, G, zero_m, v1, zero_m, v2, yy, zz)
    Gd = G.astype(np.float64)
    np.testing.assert_allclose(x, 0.75 * (Gd.T @ f(yy)) + f(zz), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(w, 1.5 * (Gd @ x), rtol=1e-13, atol=1e-13)


def pin_sampled(O):
    m, n = 19, 23
    A = I.matrix(10, 0, m, n, ld=24)
    x = I.vector(10, 1, n).astype(np.float64)
    r = I.vector(10, 2, m).astype(np.float64)
    Ad = A[:, :n].astype(np.float64)
    idx = np.array([0, 5, m - 1])
    np.testing.assert_allclose(O.gemv_rows(A, x, idx, cols=n), (Ad @ x)[idx], rtol=1e-13)
    jdx = np.array([0, 7, n - 1])
    np.testing.assert_allclose(O.gemtv_cols(A, r, jdx, cols=n), (Ad.T @ r)[jdx], rtol=1e-13)


def pin_bruteforce_fraction(O):
    """Tiny sizes: the oracle agrees with exact rational arithmetic to within the
    float64 error bound n * 2**-53 * sum |terms|."""
    from fractions import Fraction as Fr
    m, n = 3, 4
    A = I.matrix(11, 0, m, n)
    p = I.vector(11, 1, n)
    r = I.vector(11, 2, m)
    q, s = O.bicgk(A, p, r)
    for i in range(m):
        terms = [Fr(float(A[i, j])) * Fr(float(p[j])) for j in range(n)]
        bound = n * 2.0 ** -53 * float(sum(abs(t) for t in terms))
        assert abs(float(sum(terms)) - q[i]) <= bound
    for j in range(n):
        terms = [Fr(float(A[i, j])) * Fr(float(r[i])) for i in range(m)]
        bound = m * 2.0 ** -53 * float(sum(abs(t) for t in terms))
        assert abs(float(sum(terms)) - s[j]) <= bound




def pin_sampled_sequences(O):
    """The sampled/panelled compositions equal the whole-output definitions."""
    m, n = 37, 45
    A = I.matrix(12, 0, m, n, ld=48)
    B = I.matrix(12, 1, m, n, ld=48)
    v = {k: I.vector(12, 2 + i, m if k in ("u1", "u2", "y", "r") else n)
         for i, k in enumerate(["u1", "v1", "u2", "v2", "y", "z", "p", "r", "x"])}
    rows, cols = np.array([0, 3, m - 1]), np.array([1, 7, n - 1])
    q, s = O.bicgk(A, v["p"], v["r"], cols=n)
    qs, ss = O.bicgk_sampled(A, v["p"], v["r"], rows, cols, cols=n)
    np.testing.assert_allclose(qs, q[rows], rtol=1e-14)
    np.testing.assert_allclose(ss, s[cols], rtol=1e-14)
    y = O.atax(A, v["x"], cols=n)
    np.testing.assert_allclose(O.atax_sampled(A, v["x"], cols, cols=n), y[cols], rtol=1e-13)
    y = O.gesummv(1.25, A, 0.5, B, v["x"], cols=n)
    np.testing.assert_allclose(O.gesummv_sampled(1.25, A, 0.5, B, v["x"], rows, cols=n), y[rows], rtol=1e-14)
    Bf, x, w = O.gemver(1.5, 0.75, A, v["u1"], v["v1"], v["u2"], v["v2"], v["y"], v["z"], cols=n)
    Br, xs, ws = O.gemver_sampled(1.5, 0.75, A, v["u1"], v["v1"], v["u2"], v["v2"], v["y"], v["z"],
                                  rows, cols=n, panel=8)
    np.testing.assert_array_equal(Br, Bf[rows])
    np.testing.assert_allclose(xs, x, rtol=1e-14)
    np.testing.assert_allclose(ws, w[rows], rtol=1e-13)
    x, w = O.sgemvt(1.5, 0.75, A, v["y"], v["z"], cols=n)
    xs, ws = O.sgemvt_sampled(1.5, 0.75, A, v["y"], v["z"], rows, cols=n, panel=8)
    np.testing.assert_allclose(xs, x, rtol=1e-14)
    np.testing.assert_allclose(ws, w[rows], rtol=1e-13)


def pin_sgemvt(O):
    """Table 1 SGEMVT on a rank-1 A = a b^T of small integers with dyadic
    scalars: x = beta b (a.y) + z and w = alpha a (b.x), exact in float64;
    the identity reduces it to x = beta y + z, w = alpha x."""
    m, n = 6, 9
    a, b = I.small_ints(13, 0, m, -3, 3), I.small_ints(13, 1, n, -3, 3)
    y, z = I.small_ints(13, 2, m, -4, 4), I.small_ints(13, 3, n, -4, 4)
    alpha, beta = 0.75, -1.5
    A = np.outer(a, b).astype(np.float32)
    x, w = O.sgemvt(alpha, beta, A, y, z)
    a64, b64, y64, z64 = (v.astype(np.float64) for v in (a, b, y, z))
    x_ref = beta * b64 * float(np.dot(a64, y64)) + z64
    assert np.array_equal(x, x_ref)
    assert np.array_equal(w, alpha * a64 * float(np.dot(b64, x_ref)))
    # square, non-symmetric rank-1: A x and A^T x differ
    sa, sb = I.small_ints(13, 7, 8, -3, 3), I.small_ints(13, 8, 8, 1, 4)
    sy, sz = I.small_ints(13, 9, 8, -4, 4), I.small_ints(13, 10, 8, -4, 4)
    x, w = O.sgemvt(alpha, beta, np.outer(sa, sb).astype(np.float32), sy, sz)
    sa, sb, sy, sz = (v.astype(np.float64) for v in (sa, sb, sy, sz))
    x_ref = beta * sb * float(np.dot(sa, sy)) + sz
    assert np.array_equal(x, x_ref) and np.array_equal(w, alpha * sa * float(np.dot(sb, x_ref)))
    k = 7
    e = np.eye(k, dtype=np.float32)
    yy, zz = I.small_ints(13, 4, k, -4, 4), I.small_ints(13, 5, k, -4, 4)
    x, w = O.sgemvt(2.0, 0.5, e, yy, zz)
    assert np.array_equal(x, 0.5 * yy.astype(np.float64) + zz) and np.array_equal(w, 2.0 * x)
    # padded leading dimension
    G = I.matrix(13, 6, m, n, ld=12)
    x1, w1 = O.sgemvt(alpha, beta, G, y, z, cols=n)
    x2, w2 = O.sgemvt(alpha, beta, np.ascontiguousarray(G[:, :n]), y, z)
    assert np.array_equal(x1, x2) and np.array_equal(w1, w2) and np.all(np.isfinite(w1))


def pin_vadd(O):
    """Table 1 VADD: integers sum exactly; random floats agree with numpy's
    float64 (w + y) + z bit for bit."""
    n = 1001
    w, y, z = (I.small_ints(14, t, n, -100, 100) for t in range(3))
    assert np.array_equal(O.vadd(w, y, z), w.astype(np.float64) + y + z)
    w, y, z = (I.vector(14, 3 + t, n) for t in range(3))
    ref = (w.astype(np.float64) + y.astype(np.float64)) + z.astype(np.float64)
    assert np.array_equal(O.vadd(w, y, z), ref)


ALL_PINS = [pin_elementary, pin_library, pin_axpydot, pin_waxpby, pin_bicgk, pin_atax,
            pin_gesummv, pin_gemver, pin_sgemvt, pin_vadd, pin_sampled, pin_bruteforce_fraction,
            pin_sampled_sequences]


@pytest.mark.parametrize("pin", ALL_PINS, ids=[p.__name__ for p in ALL_PINS])
def test_oracle_pin(oracle_lib, pin):
    pin(oracle_lib)
