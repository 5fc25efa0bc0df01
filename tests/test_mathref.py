"""Pins of the sweep that measures the device's elementary functions
(oracle/mathref.c), on the CPU: correctly rounded results measure at most half
an ulp, planted errors are found at the right input, and overflow, underflow,
subnormal and NaN results are judged as documented."""
import math

import numpy as np

import oracle


def _bits(lo: float, n: int) -> int:
    return int(np.array([lo], np.float32).view(np.uint32)[0])


def _inputs(b0, n):
    return np.arange(b0, b0 + n, dtype=np.uint64).astype(np.uint32).view(np.float32)


def _rounded(fn, x):
    with np.errstate(all="ignore"):
        return getattr(np, fn)(x.astype(np.float64)).astype(np.float32)


def test_correctly_rounded_results_measure_half_an_ulp():
    for fn, lo in [("exp", -3.0), ("log", 0.25), ("tanh", -2.0), ("sqrt", 0.5)]:
        b0 = _bits(lo, 0)
        x = _inputs(b0, 1 << 18)
        st = oracle.sweep_f32(fn, b0, _rounded(fn, x), 1.0)
        assert st["n_bad"] == 0 and st["first_bad"] == -1, (fn, st)
        assert st["max_ulp"] <= 0.5 and st["max_rel_u"] <= 1.0, (fn, st)
        assert st["max_ulp"] > 0.49, (fn, st)    # the sweep does see rounding


def test_planted_error_is_found_at_its_input():
    b0 = _bits(0.5, 0)
    x = _inputs(b0, 100000)
    got = _rounded("exp", x)
    got[4321] = np.nextafter(got[4321], np.float32(np.inf))
    got[4321] = np.nextafter(got[4321], np.float32(np.inf))     # 1.5 to 2.5 ulp off
    st = oracle.sweep_f32("exp", b0, got, 2.0)
    assert st["first_bad"] == 4321 and st["n_bad"] == 1 and st["argmax"] == 4321
    assert 1.5 <= st["max_ulp"] <= 2.5
    assert oracle.sweep_f32("exp", b0, got, 6.0)["n_bad"] == 0   # a wider allowance admits it


def test_pow_reference_and_two_roundings():
    b0 = _bits(-3.0, 0)
    x = _inputs(b0, 1 << 18)
    x2 = (x * x).astype(np.float32)
    st = oracle.sweep_f32("pow", b0, (x2 * x).astype(np.float32), 2.0, k=3.0)
    # two roundings: at most u + u of relative error, more than half an ulp
    assert st["n_bad"] == 0 and 1.0 < st["max_rel_u"] <= 2.0 + 1e-6 and st["max_ulp"] > 0.5


def test_overflow_underflow_subnormal_and_nan():
    # exp across its overflow threshold: the rounded results are +inf there
    b0 = _bits(88.5, 0)
    x = _inputs(b0, 60000)
    got = _rounded("exp", x)
    assert np.isinf(got).any() and not np.isinf(got).all()
    assert oracle.sweep_f32("exp", b0, got, 1.0)["n_bad"] == 0
    capped = np.where(np.isinf(got), np.float32(3.4028235e38), got)
    assert oracle.sweep_f32("exp", b0, capped, 1.0)["n_bad"] == int(np.isinf(got).sum())
    # exp into the subnormal range and to zero: judged in subnormal ulps
    b0 = _bits(-104.0, 0) - 200000
    x = _inputs(b0, 400000)
    got = _rounded("exp", x)
    st = oracle.sweep_f32("exp", b0, got, 1.0)
    assert st["n_subnormal"] > 0 and st["n_bad"] == 0 and st["max_sub_ulp"] <= 0.5
    sub = np.flatnonzero((np.abs(got) < 2.0 ** -126) & (got > 0))
    off = got.copy()
    off[sub[10]] = np.nextafter(np.nextafter(off[sub[10]], np.float32(1)), np.float32(1))
    assert oracle.sweep_f32("exp", b0, off, 1.0)["first_bad"] == sub[10]
    # log of negative numbers is NaN; a number there is wrong
    b0 = _bits(-2.0, 0)
    x = _inputs(b0, 1000)
    got = _rounded("log", x)
    assert np.isnan(got).all() and oracle.sweep_f32("log", b0, got, 1.0)["n_bad"] == 0
    assert oracle.sweep_f32("log", b0, np.zeros_like(got), 1.0)["n_bad"] == 1000
    # exact zeros: log(1) must be 0 exactly
    b0 = _bits(1.0, 0)
    got = _rounded("log", _inputs(b0, 3))
    assert got[0] == 0.0 and oracle.sweep_f32("log", b0, got, 1.0)["n_bad"] == 0
    got[0] = np.float32(1e-30)
    assert oracle.sweep_f32("log", b0, got, 1e6)["first_bad"] == 0


def test_f64_reference_resolves_fp64_rounding():
    x = np.linspace(-20.0, 20.0, 200001)
    libm = np.array([math.exp(v) for v in x])
    st = oracle.sweep_f64("exp", x, libm, 2.0)
    # the C library's exp is within about half an ulp; the extended-precision
    # reference resolves that
    assert st["n_bad"] == 0 and 0.45 < st["max_ulp"] < 0.55
    got = libm.copy()
    got[777] = got[777] * (1 + 2.0 ** -50)           # 4 ulp-ish
    st = oracle.sweep_f64("exp", x, got, 2.0)
    assert st["first_bad"] == 777 and st["n_bad"] == 1
    st = oracle.sweep_f64("pow", x, x * x * x, 2.0, k=3.0)
    assert st["n_bad"] == 0 and 1.0 < st["max_rel_u"] <= 2.0 + 1e-6
