"""Pins of the oracle's running error bound mu, one operator at a time (CPU).

For a tree of correctly rounded operations and elementary functions with
allowance f, the first-order worst case of evaluating it in precision u is
reached by some choice of signs of the individual rounding errors: each node
k returns its exact result times (1 + s_k e_k), with e_k = u for + - * / sqrt
and conversions and e_k = f u for an elementary function.  Enumerating every
sign vector therefore gives the worst case by brute force, without any
derivative.  For each operator, on a tree whose operand already carries
error, that brute-force worst case must equal u * mu to first order:

  * not above it (mu bounds the error), and
  * not below it (mu is tight: an operator term that over-admits, such as a
    missing 1/|a| in log's term or a wrong derivative, fails here).

The acceptance rule must also admit a real FP32 evaluation one operator at a
time (numpy's correctly rounded float32 arithmetic; elementary functions
rounded once from FP64, well inside their allowance), and reject a result a
hair beyond max(tol |v|, 4 u mu).
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle import E, const, leaf

U = {"f32": 2.0 ** -24, "f64": 2.0 ** -53}
N = 4000

# Functions of the simulation (exact up to the working precision).
FN = {"exp": np.exp, "log": np.log, "tanh": np.tanh, "sqrt": np.sqrt}
ROUNDED = {"add", "sub", "mul", "div", "sqrt", "exp", "log", "tanh", "pow", "tof32"}


def _inputs(dtype, k=4, seed=11):
    return [synth.fill(seed, t, N, dtype) for t in range(k)]


def _pre():
    """X % Y + W: an operand that carries two roundings."""
    return leaf(0) % leaf(1) + leaf(2)


def _pre2():
    return leaf(3) % leaf(2) - leaf(0)


TREES = {
    "add": lambda: _pre() + _pre2(),
    "sub": lambda: _pre() - _pre2(),
    "mul": lambda: _pre() % _pre2(),
    "div": lambda: _pre() / (2.0 + leaf(3) % leaf(2)),
    "div_by_rounded": lambda: _pre2() / (_pre() + 3.0),
    "exp": lambda: oracle.exp(_pre()),
    "log": lambda: oracle.log(_pre() + 2.5),          # argument in [0.5, 4.5]
    "tanh": lambda: oracle.tanh(_pre()),
    "sqrt": lambda: oracle.sqrt(_pre() + 2.5),
    "pow3": lambda: oracle.pow_(_pre(), 3),
    "pow2": lambda: oracle.pow_(_pre() + 2.5, 2),
    "neg": lambda: -_pre(),
    "abs": lambda: oracle.abs_(_pre()),
    "inexact_const": lambda: 0.1 + leaf(0) % leaf(1),
    "tof32": lambda: oracle.conv_to_f32(_pre()) % leaf(3),
}


def _simulate(e, xs, signs, eps, wt, counter):
    """Evaluate tree `e` in working type `wt` with node k's result scaled by
    (1 + signs[k] * eps(node)); counter numbers the rounded nodes."""
    op = e.op
    if op == "leaf":
        return xs[e.leaf]
    if op == "const":
        c = wt(e.cst)
        if e.cst != float(np.float32(e.cst)) and eps("const") > 0:
            k = counter[0]
            counter[0] += 1
            c = c * (wt(1) + wt(signs[k]) * wt(eps("const")))
        return c
    kids = [_simulate(c, xs, signs, eps, wt, counter) for c in e.kids]
    if op == "add":
        v = kids[0] + kids[1]
    elif op == "sub":
        v = kids[0] - kids[1]
    elif op == "mul":
        v = kids[0] * kids[1]
    elif op == "div":
        v = kids[0] / kids[1]
    elif op == "neg":
        v = -kids[0]
    elif op == "abs":
        v = np.abs(kids[0])
    elif op == "pow":
        v = np.power(kids[0], kids[1])
    elif op == "tof32":
        v = kids[0]
    else:
        v = FN[op](kids[0])
    if op in ROUNDED:
        k = counter[0]
        counter[0] += 1
        v = v * (wt(1) + wt(signs[k]) * wt(eps(op)))
    return v


def _rounded_count(e):
    n = 1 if e.op in ROUNDED else 0
    if e.op == "const" and e.cst != float(np.float32(e.cst)):
        n = 1
    return n + sum(_rounded_count(c) for c in e.kids)


def _worst_case(expr, inputs, dtype):
    """Largest |perturbed - exact| over every sign vector, per element."""
    wt = np.float64 if dtype == "f32" else np.longdouble
    u = U[dtype]
    fa = oracle.F_ALLOW[dtype]

    def eps(op):
        if op in ("exp", "log", "tanh", "pow"):
            return fa[op] * u
        if op == "const":
            return u if dtype == "f32" else 0.0
        return u

    xs = [np.asarray(x, np.float64).astype(wt) for x in inputs]
    K = _rounded_count(expr)
    exact = _simulate(expr, xs, [0] * max(K, 1), eps, wt, [0])
    worst = np.zeros(exact.shape, wt)
    for signs in itertools.product((-1, 1), repeat=K):
        v = _simulate(expr, xs, signs, eps, wt, [0])
        worst = np.maximum(worst, np.abs(v - exact))
    return worst.astype(np.float64), K


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("name", sorted(TREES))
def test_mu_equals_brute_force_worst_case(name, dtype):
    if name == "tof32" and dtype == "f64":
        pytest.skip("conversion to FP32 occurs only in FP32-compute expressions")
    expr = TREES[name]()
    xs = _inputs(dtype)
    v, mu = oracle.evaluate(expr, xs, dtype)
    worst, K = _worst_case(expr, xs, dtype)
    assert K >= 1
    bound = U[dtype] * mu
    ratio = worst / bound
    # FP32: the simulation resolves u = 2^-24 to about 2^-29 of itself.  FP64
    # is simulated in x87 extended precision (64-bit significand), which
    # resolves 2^-53 to about 2^-11.  The second-order terms are, relative to
    # the first-order ones, of the order of the relative error itself
    # (u mu / |v|), which cancellation inside the operand can make large.
    rel = bound / np.maximum(np.abs(v), 1e-300)
    tol = (2e-5 if dtype == "f32" else 5e-3) + 8 * rel
    assert np.all(ratio <= 1 + tol), (name, float((ratio - 1 - tol).max()))
    assert np.all(ratio >= 1 - tol), (name, float((1 - tol - ratio).max()))
    assert np.median(np.abs(ratio - 1)) < (1e-5 if dtype == "f32" else 2e-3)


def _fp32_one_op_at_a_time(e, xs):
    op = e.op
    f = np.float32
    if op == "leaf":
        return xs[e.leaf].astype(f)
    if op == "const":
        return f(e.cst)
    k = [_fp32_one_op_at_a_time(c, xs) for c in e.kids]
    if op == "add":
        return (k[0] + k[1]).astype(f)
    if op == "sub":
        return (k[0] - k[1]).astype(f)
    if op == "mul":
        return (k[0] * k[1]).astype(f)
    if op == "div":
        return (k[0] / k[1]).astype(f)
    if op == "neg":
        return -k[0]
    if op == "abs":
        return np.abs(k[0])
    if op == "sqrt":
        return np.sqrt(k[0])
    if op == "tof32":
        return k[0]
    if op == "pow":
        assert float(k[1]) in (2.0, 3.0)
        x2 = (k[0] * k[0]).astype(f)
        return x2 if float(k[1]) == 2.0 else (x2 * k[0]).astype(f)
    # an elementary function rounded once from FP64 (0.5 ulp, inside f)
    return FN[op](k[0].astype(np.float64)).astype(f)


@pytest.mark.parametrize("name", sorted(TREES))
def test_fp32_evaluation_within_first_order_bound(name):
    expr = TREES[name]()
    xs = _inputs("f32")
    v, mu = oracle.evaluate(expr, xs, "f32")
    z = _fp32_one_op_at_a_time(expr, xs).astype(np.float64)
    err = np.abs(z - v)
    assert np.all(err <= U["f32"] * mu * (1 + 1e-6)), name
    ok, rep = oracle.check(z, v, mu, "f32")
    assert ok.all(), rep


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("name", sorted(TREES))
def test_rule_edge_is_where_mu_puts_it(name, dtype):
    if name == "tof32" and dtype == "f64":
        pytest.skip("conversion to FP32 occurs only in FP32-compute expressions")
    expr = TREES[name]()
    xs = _inputs(dtype)
    v, mu = oracle.evaluate(expr, xs, dtype)
    lim = np.maximum(oracle.TOL[dtype] * np.abs(v), 4 * U[dtype] * mu)
    s = np.where(np.arange(v.size) % 2 == 0, 1.0, -1.0)
    inside = v + s * 0.99 * lim
    outside = v + s * 1.01 * lim
    assert oracle.check(inside, v, mu, dtype)[0].all(), name
    assert not oracle.check(outside, v, mu, dtype)[0].any(), name


def test_sqrt_bound_near_zero():
    """sqrt of an operand whose error is as large as the operand itself (a
    product minus its own rounded value): the first-order term mu_a/(2|v|)
    underestimates there, and the bound takes the exact spread of sqrt over
    the operand's error interval.  The brute-force worst case must stay
    inside it."""
    x, y = _inputs("f32", 2, seed=12)
    p = (x * y).astype(np.float32)            # fl(x*y): x*y - p is its rounding error
    expr = oracle.sqrt(oracle.abs_(leaf(0) % leaf(1) - leaf(2)))
    xs = [x, y, p]
    v, mu = oracle.evaluate(expr, xs, "f32")
    worst, _ = _worst_case(expr, xs, "f32")
    ratio = worst / (U["f32"] * mu)
    assert np.all(ratio <= 1 + 1e-6)
    # not vacuous: the sign vectors reach it for most elements (where the
    # error interval straddles 0 the extreme sits inside it, at |a| = 0,
    # which no sign vector visits)
    assert np.median(ratio) > 0.9
    # the operand's error is comparable to the operand for most elements
    a = np.abs(x.astype(np.float64) * y - p)
    assert np.mean(a < 1e-6) > 0.9


def test_planted_operator_mistakes_are_caught():
    """Bounds built with a mistaken operator term, as a buggy oracle would
    compute them, fail the brute-force comparison (so the comparison above
    is able to see such mistakes)."""
    xs = _inputs("f32")
    x, y, w = [a.astype(np.float64) for a in xs[:3]]
    u = U["f32"]
    f = oracle.F_ALLOW["f32"]
    a = x * y + w + 2.5
    mu_a = np.abs(x * y) + np.abs(x * y + w) + np.abs(a)
    worst, _ = _worst_case(TREES["log"](), xs, "f32")
    right = mu_a / np.abs(a) + f["log"] * np.abs(np.log(a))
    dropped = mu_a + f["log"] * np.abs(np.log(a))          # 1/|a| left out
    assert np.allclose(worst, u * right, rtol=2e-5)
    assert not np.allclose(worst, u * dropped, rtol=1e-2)
    t = x * y + w
    mu_t = np.abs(x * y) + np.abs(t)
    worst, _ = _worst_case(TREES["tanh"](), xs, "f32")
    right = (1 - np.tanh(t) ** 2) * mu_t + f["tanh"] * np.abs(np.tanh(t))
    wrong = mu_t + f["tanh"] * np.abs(np.tanh(t))           # derivative taken as 1
    assert np.allclose(worst, u * right, rtol=2e-5)
    assert not np.allclose(worst, u * wrong, rtol=1e-2)
