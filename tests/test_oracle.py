"""Pins of the FP64 oracle against closed forms, invariants, exact arithmetic
and library routines (CPU only).  Each test names what it would catch."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import EXPRS, X, Y, W

SMALL_N = [0, 1, 2, 3, 63, 64, 65, 127, 129, 1023, 1025, 4097]


def _xyw(n, seed=1, dtype="f32"):
    return [synth.fill(seed, t, n, dtype) for t in range(3)]


def _f64(a, dtype):
    return synth.bf16_to_f64(a) if dtype == "bf16" else a.astype(np.float64)


# ---- widening of stored values --------------------------------------------

def test_f16_widening_exhaustive():
    """Every one of the 65536 f16 bit patterns widens as numpy's decoder does
    (catches a wrong exponent bias or subnormal scale)."""
    bits = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    v, mu = oracle.evaluate(X, [bits.view(np.float16)], "f16")
    want = bits.view(np.float16).astype(np.float64)
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(v), nan)
    assert np.array_equal(v[~nan], want[~nan]) and not mu.any()


def test_bf16_widening_exhaustive():
    bits = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    v, _ = oracle.evaluate(X, [bits], "bf16")
    want = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(v), nan) and np.array_equal(v[~nan], want[~nan])


# ---- element-wise closed forms ----------------------------------------------

@pytest.mark.parametrize("dtype", ["f32", "f64", "bf16", "f16"])
def test_c1_special_cases(dtype):
    n = 3000
    x, y, w = _xyw(n, 1, dtype)
    zero = np.zeros_like(w)
    # W = 0  =>  Z = X*Y, a single exact-in-FP64 product (catches a wrong term)
    v, _ = oracle.evaluate(EXPRS["c1_z"], [x, y, zero], dtype)
    assert np.array_equal(v, _f64(x, dtype) * _f64(y, dtype))
    # Y = 0  =>  Z = 2W exactly (catches a wrong coefficient)
    v, _ = oracle.evaluate(EXPRS["c1_z"], [x, np.zeros_like(y), w], dtype)
    assert np.array_equal(v, 2.0 * _f64(w, dtype))


def test_c2_special_cases():
    n = 4096
    x, y, w = [a.astype(np.float64) for a in _xyw(n, 2, "f64")]
    e = EXPRS["c2_z"]
    zero, one = np.zeros(n), np.ones(n)
    v, _ = oracle.evaluate(e, [zero, zero, zero], "f64")
    assert not v.any()
    v, _ = oracle.evaluate(e, [one, one, zero], "f64")          # (1+1)*1/(1+1) = 1
    assert np.all(v == 1.0)
    v, _ = oracle.evaluate(e, [x, y, zero], "f64")              # exp(0) = 1
    assert np.array_equal(v, (x + y) / (1.0 + x * x))
    v, _ = oracle.evaluate(e, [zero, one, w], "f64")            # Z = exp(-|W|)
    assert np.all(v <= 1.0) and np.all(v >= math.exp(-1.0))
    assert np.allclose(v, np.exp(-np.abs(w)), rtol=1e-15, atol=0)
    v1, _ = oracle.evaluate(e, [x, y, w], "f64")                # even in W
    v2, _ = oracle.evaluate(e, [x, y, -w], "f64")
    assert np.array_equal(v1, v2)
    v3, _ = oracle.evaluate(e, [-x, -y, w], "f64")              # odd in (X, Y) jointly
    assert np.array_equal(v3, -v1)
    v4, _ = oracle.evaluate(e, [y, x, w], "f64")                # not symmetric in X, Y
    assert not np.array_equal(v4, v1)


def test_u32_special_cases_and_wrap():
    n = 5000
    x, y, w = [synth.fill(1, t, n, "u32", "uint31") for t in range(3)]
    e = EXPRS["u32_z"]
    z, _ = oracle.evaluate_u32(e, [x, x, w])                    # X^X = 0
    assert np.array_equal(z, (3 * w.astype(np.uint64) % 2 ** 32).astype(np.uint32))
    z, _ = oracle.evaluate_u32(e, [x, y, np.zeros_like(w)])     # W = 0
    assert np.array_equal(z, x ^ y)
    # values near 2^32 exercise the modular wrap of + and *
    big = np.array([0xFFFFFFFF, 0x80000000, 0x55555556, 1, 0], np.uint32)
    z, tot = oracle.evaluate_u32(e, [big, big[::-1].copy(), big])
    want = [((int(a) ^ int(b)) + 3 * int(c)) % 2 ** 32 for a, b, c in zip(big, big[::-1], big)]
    assert [int(t) for t in z] == want and tot == sum(want)


# ---- sums against exact arithmetic -----------------------------------------

@pytest.mark.parametrize("n", SMALL_N)
def test_accu_exact_fraction(n):
    """accu(X%Y) against the exact rational sum of the exact products."""
    x, y, _ = _xyw(n, 1)
    s, mu = oracle.evaluate(EXPRS["xy"], [x, y], "f32", reduce="accu")
    exact = sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0))
    assert abs(Fraction(float(s[0])) - exact) <= Fraction(2.0 ** -52) * abs(exact)
    if n == 0:
        assert s[0] == 0.0 and mu[0] == 0.0


def test_accu_matches_fsum_on_hard_cancellation():
    rng = np.random.default_rng(0)
    t = rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000)
    t = np.concatenate([t, -t[::2]])
    s, _ = oracle.evaluate(X, [t], "f64", reduce="accu")
    assert s[0] == math.fsum(t) or abs(s[0] - math.fsum(t)) <= 2 ** -50 * abs(math.fsum(t))


def test_accu_of_constants():
    for n in [0, 1, 1000, 1 << 20]:
        ones = np.ones(n, np.float32)
        s, _ = oracle.evaluate(X, [ones], "f32", reduce="accu")
        assert s[0] == n
    tenth = np.full(100000, 0.1, np.float64)
    s, _ = oracle.evaluate(X, [tenth], "f64", reduce="accu")
    assert s[0] == math.fsum(tenth)
    s, _ = oracle.evaluate(X, [np.ones(7 * 11, np.float32)], "f32", shape=(7, 11), reduce="accu")
    assert s[0] == 77


def test_dot_equals_accu_schur():
    x, y, _ = _xyw(10000, 2)
    s1, _ = oracle.evaluate(EXPRS["xy"], [x, y], "f32", reduce="accu")
    s2, _ = oracle.evaluate(Y % X, [x, y], "f32", reduce="accu")
    assert s1[0] == s2[0]


# ---- column-major dimension sums ----------------------------------------------

@pytest.mark.parametrize("shape", [(1, 7), (7, 1), (3, 5), (17, 33), (64, 64), (65, 63),
                                   (8191, 3), (600, 700)])
def test_dim_sums_layout_and_exactness(shape):
    m, k = shape
    # element (r, c) at linear index r + c*m holds c + 1/(r+2): distinguishes
    # rows from columns, so a transposed layout fails
    r, c = np.meshgrid(np.arange(m), np.arange(k), indexing="ij")
    a = (c + 1.0 / (r + 2.0)).reshape(-1, order="F")
    cs, _ = oracle.evaluate(X, [a], "f64", shape=shape, reduce="colsum")
    rs, _ = oracle.evaluate(X, [a], "f64", shape=shape, reduce="rowsum")
    for j in range(0, k, max(1, k // 5)):
        col = a[j * m:(j + 1) * m]
        assert cs[j] == math.fsum(col)
    for i in range(0, m, max(1, m // 5)):
        row = a[i::m]
        assert rs[i] == math.fsum(row)
    ones = np.ones(m * k, np.float32)
    cs, _ = oracle.evaluate(X, [ones], "f32", shape=shape, reduce="colsum")
    rs, _ = oracle.evaluate(X, [ones], "f32", shape=shape, reduce="rowsum")
    assert np.all(cs == m) and np.all(rs == k)


def test_rowsum_is_colsum_of_transpose():
    m, k = 300, 217
    x, y, w = [synth.fill(2, t, m * k, "f32") for t in range(3)]
    rs, _ = oracle.evaluate(EXPRS["c2_z"], [x, y, w], "f32", shape=(m, k), reduce="rowsum")
    tr = [np.ascontiguousarray(np.asarray(a).reshape((m, k), order="F").T).reshape(-1, order="F")
          for a in (x, y, w)]
    cs, _ = oracle.evaluate(EXPRS["c2_z"], tr, "f32", shape=(k, m), reduce="colsum")
    assert np.allclose(rs, cs, rtol=1e-14, atol=1e-14)


def test_sums_agree():
    m, k = 513, 257
    x, y, w = [synth.fill(2, t, m * k, "f64") for t in range(3)]
    args = dict(shape=(m, k))
    e = EXPRS["c2_z"]
    cs, _ = oracle.evaluate(e, [x, y, w], "f64", reduce="colsum", **args)
    rs, _ = oracle.evaluate(e, [x, y, w], "f64", reduce="rowsum", **args)
    ac, _ = oracle.evaluate(e, [x, y, w], "f64", reduce="accu", **args)
    assert abs(math.fsum(cs) - ac[0]) < 1e-12 and abs(math.fsum(rs) - ac[0]) < 1e-12


# ---- Frobenius norm ------------------------------------------------------

def test_norm_identities():
    m, k = 1000, 300
    x, y, _ = [synth.fill(2, t, m * k, "f32") for t in range(3)]
    d = EXPRS["diff"]
    nrm, _ = oracle.evaluate(d, [x, y], "f32", shape=(m, k), reduce="norm")
    ref = np.linalg.norm((x.astype(np.float64) - y).reshape((m, k), order="F"), "fro")
    assert abs(nrm[0] - ref) <= 1e-14 * ref
    z, mu = oracle.evaluate(d, [x, x], "f32", shape=(m, k), reduce="norm")
    assert z[0] == 0.0
    two, _ = oracle.evaluate(d, [2 * x, 2 * y], "f32", shape=(m, k), reduce="norm")
    assert two[0] == 2 * nrm[0]
    ones = np.ones(8192 * 64, np.float32)
    n1, _ = oracle.evaluate(X, [ones], "f32", shape=(8192, 64), reduce="norm")
    assert n1[0] == math.sqrt(8192 * 64)
    sq, _ = oracle.evaluate(d % d, [x, y], "f32", shape=(m, k), reduce="accu")
    assert abs(nrm[0] ** 2 - sq[0]) <= 1e-13 * sq[0]


# ---- the running error bound -------------------------------------------------

def _f32_one_op_at_a_time(x, y, w):
    """The C2 expression evaluated in FP32 one operator at a time, in numpy."""
    f = np.float32
    t1 = (x + y).astype(f)
    t2 = np.abs(w)
    t3 = -t2
    t4 = np.exp(t3).astype(f)
    t5 = (t1 * t4).astype(f)
    t6 = (x * x).astype(f)
    t7 = (f(1) + t6).astype(f)
    return (t5 / t7).astype(f)


def test_mu_bounds_fp32_evaluation_and_is_tight():
    n = 200000
    x, y, w = _xyw(n, 2)
    v, mu = oracle.evaluate(EXPRS["c2_z"], [x, y, w], "f32")
    z32 = _f32_one_op_at_a_time(x, y, w)
    err = np.abs(z32.astype(np.float64) - v)
    # the first-order bound holds without the factor 4 ...
    assert np.all(err <= oracle.U32 * mu * 1.0001)
    # ... and is not vacuous: it stays within a few units of |v| (the
    # cancellation in X+Y is what makes mu/|v| large, so look at the median)
    assert np.median(mu / np.maximum(np.abs(v), 1e-30)) < 8
    ok, rep = oracle.check(z32, v, mu, "f32")
    assert ok.all(), rep


def test_sum_rule_accepts_pairwise_fp32_sum():
    """numpy's float32 sum is pairwise (error ~ log2(n) u sum|t|): the sum term
    of the bound must admit it, at every size."""
    for n in [100, 4097, 1 << 16, 1 << 20]:
        x, y, _ = _xyw(n, 1)
        s, mu = oracle.evaluate(EXPRS["xy"], [x, y], "f32", reduce="accu")
        pairwise = float(np.sum((x * y).astype(np.float32), dtype=np.float32))
        ok, rep = oracle.check(np.array([pairwise]), s, mu, "f32")
        assert ok.all(), rep


def test_check_rejects_planted_errors():
    n = 1000
    x, y, w = _xyw(n, 1)
    v, mu = oracle.evaluate(EXPRS["c1_z"], [x, y, w], "f32")
    good = v.astype(np.float32)
    assert oracle.check(good, v, mu, "f32")[0].all()
    bad = good.copy()
    bad[17] = np.nextafter(bad[17], np.float32(np.inf))
    for _ in range(40):
        bad[17] = np.nextafter(bad[17], np.float32(np.inf))
    assert not oracle.check(bad, v, mu, "f32")[0][17]
    # a planted dropped term (Z = X%Y, missing 2W) is rejected wholesale
    wrong = (x * y).astype(np.float32)
    assert oracle.check(wrong, v, mu, "f32")[0].mean() < 0.01


def test_half_output_rule():
    x, y, w = _xyw(5000, 3, "f16")
    v, mu = oracle.evaluate(EXPRS["c1_z"], [x, y, w], "f16")
    z = v.astype(np.float32).astype(np.float16)  # FP32 rounding then half RNE
    ok, rep = oracle.check(z.astype(np.float64), v, mu, "f16", out_dtype="f16")
    assert ok.all(), rep
    off = z.copy()
    off[::7] = np.nextafter(off[::7], np.float16(np.inf))
    off[::7] = np.nextafter(off[::7], np.float16(np.inf))
    ok, _ = oracle.check(off.astype(np.float64), v, mu, "f16", out_dtype="f16")
    assert not ok[::7].any()


def test_bad_trees_are_rejected():
    with pytest.raises(ValueError):          # XOR has no floating-point meaning
        oracle.evaluate(X ^ Y, [np.ones(4), np.ones(4)], "f64")
    with pytest.raises(AssertionError):      # a leaf without an input
        oracle.evaluate(X + Y, [np.ones(4)], "f64")


def test_f16_overflow_reading():
    v = np.array([65519.0, 65520.0, -70000.0, 1.0])
    mu = np.zeros(4)
    got = np.array([65504.0, np.inf, -np.inf, 1.0])
    ok, _ = oracle.check(got, v, mu, "f16", out_dtype="f16")
    assert ok.all()
    ok, _ = oracle.check(np.array([65504.0, 65504.0, -65504.0, 1.0]), v, mu, "f16", out_dtype="f16")
    assert list(ok) == [True, False, False, True]


# ---- the paper's benchmark expressions (Sec. 4) -----------------------------

def test_paper_ops_against_libm_and_identities():
    x = np.linspace(-3, 3, 6001)
    P = oracle.paper_expr
    v, _ = oracle.evaluate(oracle.log(X), [np.exp(x)], "f64")
    assert np.allclose(v, x, rtol=0, atol=1e-15)
    v, _ = oracle.evaluate(oracle.tanh(X), [x], "f64")
    assert np.allclose(v, np.tanh(x), rtol=4.5e-16, atol=0) and v[3000] == 0.0
    v, _ = oracle.evaluate(oracle.pow_(X, 2), [x], "f64")
    assert np.allclose(v, x * x, rtol=2.3e-16, atol=0)
    v, _ = oracle.evaluate(P("relu"), [x], "f64")              # X % (X > 0) = max(X, 0)
    assert np.array_equal(v, np.maximum(x, 0))
    v1, _ = oracle.evaluate(P("sigmoid"), [x], "f64")
    v2, _ = oracle.evaluate(P("sigmoid"), [-x], "f64")
    assert np.allclose(v1 + v2, 1.0, rtol=0, atol=6e-16) and v1[3000] == 0.5
    for beta in (0.5, 1.0, 1.75):
        v, _ = oracle.evaluate(P("swish", beta=beta), [x], "f64")
        assert np.allclose(v, x / (1 + np.exp(-beta * x)), rtol=1e-15, atol=0)
    g1, _ = oracle.evaluate(P("gelu"), [x], "f64")              # gelu(x) - gelu(-x) = x
    g2, _ = oracle.evaluate(P("gelu"), [-x], "f64")
    assert np.allclose(g1 - g2, x, rtol=0, atol=1e-15) and g1[3000] == 0.0
    y = synth.fill(1, 1, x.size, "f64")
    v, _ = oracle.evaluate(oracle.conv_to_f32(X), [y], "f64")
    assert np.array_equal(v, y.astype(np.float32).astype(np.float64))


def test_expr3_and_mixed_dtypes():
    n = 5000
    xf = synth.fill(1, 0, n, "f32")
    y64 = synth.fill(1, 1, n, "f64")
    w = synth.fill(1, 2, n, "f32", "uniform12")
    e = oracle.paper_expr("expr3")
    v, mu = oracle.evaluate(e, [xf, y64, w], "f32", input_dtypes=["f32", "f64", "f32"])
    x64 = xf.astype(np.float64)
    want = 1 / (x64 * y64.astype(np.float32) + np.log(np.log(x64 + 2) * w))
    assert np.allclose(v, want, rtol=1e-14, atol=0)
    v0, _ = oracle.evaluate(e, [xf, np.zeros(n), w], "f32", input_dtypes=["f32", "f64", "f32"])
    assert np.allclose(v0, 1 / np.log(np.log(x64 + 2) * w), rtol=1e-14)   # Y = 0


def test_undefined_bound_demands_exact_agreement():
    # X = -1: log(X + 2) = 0, log(0) = -inf and the reciprocal is -0; the
    # running bound meets 0 * inf there and is NaN
    x = np.array([-1.0, 0.5], np.float32)
    y = np.array([0.25, 0.25])
    w = np.array([1.5, 1.5], np.float32)
    v, mu = oracle.evaluate(oracle.paper_expr("expr3"), [x, y, w], "f32",
                            input_dtypes=["f32", "f64", "f32"])
    assert v[0] == 0.0 and np.signbit(v[0]) and np.isnan(mu[0]) and np.isfinite(mu[1])
    assert oracle.check(v.copy(), v, mu, "f32")[0].all()
    bad = v.copy()
    bad[0] = 1e-30
    assert list(oracle.check(bad, v, mu, "f32")[0]) == [False, True]


@pytest.mark.parametrize("k", [1, 2, 3, 7, 16])
def test_addn_is_left_to_right_sum(k):
    xs = [synth.fill(2, t, 3001, "f32") for t in range(k)]
    v, mu = oracle.evaluate(oracle.addn(k), xs, "f32")
    s = xs[0].astype(np.float64)
    for t in xs[1:]:
        s = s + t
    assert np.array_equal(v, s)
    # FP32 left-to-right accumulation passes the rule
    s32 = xs[0].copy()
    for t in xs[1:]:
        s32 = (s32 + t).astype(np.float32)
    assert oracle.check(s32, v, mu, "f32")[0].all()


# ---- strided views: transpose, submatrix, diagonal (Sec. 3, Sec. 4) -----------

def _mat(seed, t, m, n):
    return synth.fill(seed, t, m * n, "f64").reshape(m, n, order="F")


def test_views_match_numpy_indexing():
    m, n = 7, 5
    A = _mat(3, 0, m, n)
    flat = [A.reshape(-1, order="F")]
    v, _ = oracle.evaluate(X.t(), flat, "f64", shape=(n, m))          # transpose
    assert np.array_equal(v, A.T.reshape(-1, order="F"))
    v, _ = oracle.evaluate(X.t().t(), flat, "f64", shape=(m, n))      # double transpose
    assert np.array_equal(v, flat[0])
    v, _ = oracle.evaluate(oracle.submat(0, 2, 1, m), flat, "f64", shape=(3, 2))
    assert np.array_equal(v, A[2:5, 1:3].reshape(-1, order="F"))
    for k in (-2, -1, 0, 1, 3):
        L = oracle.diag_len(m, n, k)
        v, _ = oracle.evaluate(oracle.diag(0, k, m), flat, "f64", shape=(L, 1))
        assert np.array_equal(v, np.diag(A, k)), k
    r0, c0, R, C = oracle.center(10, 8)
    assert (r0, c0, R, C) == (2, 2, 5, 4) and oracle.center(10000, 10000) == (2500, 2500, 5000, 5000)
    with pytest.raises(AssertionError):          # a view outside its input is refused
        oracle.evaluate(oracle.submat(0, 5, 4, m), flat, "f64", shape=(3, 2))


def test_transpose_of_an_expression_moves_to_its_leaves():
    m = 6
    B, C = _mat(4, 1, m, m), _mat(4, 2, m, m)
    ins = [B.reshape(-1, order="F"), C.reshape(-1, order="F")]
    v, _ = oracle.evaluate((X + Y).t(), ins, "f64", shape=(m, m))
    assert np.array_equal(v, (B + C).T.reshape(-1, order="F"))
    v, _ = oracle.evaluate((X.t() - Y).t(), ins, "f64", shape=(m, m))   # (X' - Y)' = X - Y'
    assert np.array_equal(v, (B - C.T).reshape(-1, order="F"))


def test_paper_view_expressions():
    m = 9
    P = oracle.paper_view_expr
    mats = [_mat(5, t, m, m) for t in range(4)]
    ins = [M.reshape(-1, order="F") for M in mats]
    e, shape = P("expr1", m, m)                 # symmetric: Z' = Z exactly
    v, _ = oracle.evaluate(e, ins[:2], "f64", shape=shape)
    Z = v.reshape(m, m, order="F")
    assert np.array_equal(Z, Z.T)
    assert np.allclose(Z, 2 * (mats[0].T + mats[1]) + 2 * (mats[0] + mats[1].T), rtol=1e-15)
    e, shape = P("expr2", m, m, a=0.5)
    v, _ = oracle.evaluate(e, ins, "f64", shape=shape)
    want = 0.5 * mats[0] + (mats[1] + mats[2]).T + np.log(mats[3] ** 2)
    assert np.allclose(v, want.reshape(-1, order="F"), rtol=1e-14)
    for name, k in (("addsub2", 2), ("addsub4", 4)):
        e, shape = P(name, m, m)
        r0, c0, R, C = oracle.center(m, m)
        v, _ = oracle.evaluate(e, ins[:k], "f64", shape=shape)
        sub = sum(M[r0:r0 + R, c0:c0 + C] for M in mats[:k])
        assert shape == (R, C) and np.allclose(v, sub.reshape(-1, order="F"), rtol=1e-15)
    e, shape = P("diagsum", m, m)
    v, _ = oracle.evaluate(e, ins[:2], "f64", shape=shape)
    d = lambda M: np.diag(M, -1) + np.diag(M, 1)
    assert shape == (m - 1, 1) and np.array_equal(v, d(mats[0]) * d(mats[1]))
    v, _ = oracle.evaluate(e, [ins[0], ins[0]], "f64", shape=shape)     # X = Y: a square
    assert np.all(v >= 0)


def test_check_reports_results_that_need_the_running_bound():
    # three results of value 1 with a running bound of 100 units: exact, off by
    # 1e-5 (beyond the 1e-6 relative tolerance, inside 4*u*mu = 2.4e-5) and off
    # by 1e-4 (a failure); only the middle one passes through the mu branch
    v = np.ones(3)
    mu = np.full(3, 100.0)
    ok, rep = oracle.check(np.array([1.0, 1.0 + 1e-5, 1.0 + 1e-4]), v, mu, "f32")
    assert ok.tolist() == [True, True, False]
    assert rep["fail"] == 1 and rep["needed_mu_branch"] == 1
    # a half-format output: its own rounding (u_half |v|) is the relative part
    ok, rep = oracle.check(np.array([1.0 + 2.0 ** -9, 1.0 + 2.0 ** -7]), np.ones(2), np.full(2, 1e5),
                           "f32", out_dtype="bf16")
    assert ok.all() and rep["needed_mu_branch"] == 1
