"""Sweeps of the device's elementary functions against libm.

The oracle's running error bound gives each elementary function an allowance
f (units of the compute roundoff u, relative to the result): F_ALLOW.  These
tests establish it.  Each function is evaluated by the library's own
one-operator kernel (the same device function the fused expressions inline)

  * over EVERY FP32 bit pattern (2^32 inputs, NaNs and infinities included),
    referenced to the FP64 libm value of the widened input, and
  * over 2^24 FP64 inputs (seeded: uniform over bit patterns, and uniform over
    the function's usual range), referenced to x87 extended precision,

and every result must lie within f u |y| of the reference y (sqrt: within
u |y|, i.e. correctly rounded; results in the subnormal range: within one
ulp; NaN, infinite and zero references must be met exactly).  pow is the
library's pow(x, 3), which the expressions evaluate as (x * x) * x; its
FP32 sweep covers |x| <= 2^42 (x^3 <= 2^126): next to FP32's overflow a
product of two roundings can overflow where the exact cube does not, which
no relative allowance describes.

With FX_SWEEP_REPORT set, each test appends one JSON line with its figures
to that file."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import need_gpu

pytestmark = pytest.mark.gpu

CHUNK = 1 << 26
FUNCS = ["exp", "log", "tanh", "sqrt", "pow3"]
# usual ranges of the FP64 value sample (the bit-pattern sample covers the rest)
RANGE64 = {"exp": (-30.0, 30.0), "log": (0.0, 4.0), "tanh": (-6.0, 6.0), "sqrt": (0.0, 4.0),
           "pow3": (-3.0, 3.0)}


def _allow(dtype, fn):
    if fn == "sqrt":
        return 1.0   # correctly rounded: half an ulp is at most u |y|
    return oracle.F_ALLOW[dtype]["pow" if fn == "pow3" else fn]


def _launch(fx, fn, X, out):
    if fn == "pow3":
        fx.fx_op_scalar("spow", X, 3.0, out)
    else:
        fx.fx_op_unary(fn, X, out)


def _merge(tot, st, base):
    if tot is None:
        tot = dict(st)
        for k in ("argmax", "first_bad"):
            if tot[k] >= 0:
                tot[k] += base
        return tot
    if st["max_rel_u"] > tot["max_rel_u"]:
        tot["max_rel_u"], tot["argmax"] = st["max_rel_u"], st["argmax"] + base
    tot["max_ulp"] = max(tot["max_ulp"], st["max_ulp"])
    if st["first_bad"] >= 0 and tot["first_bad"] < 0:
        tot["first_bad"] = st["first_bad"] + base
    tot["n_bad"] += st["n_bad"]
    tot["n_subnormal"] += st["n_subnormal"]
    tot["max_sub_ulp"] = max(tot["max_sub_ulp"], st["max_sub_ulp"])
    return tot


def _report(rec):
    print(json.dumps(rec), flush=True)
    path = os.environ.get("FX_SWEEP_REPORT")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(rec) + "\n")


@pytest.mark.parametrize("fn", FUNCS)
def test_f32_every_input(fn):
    torch, fx = need_gpu()
    allow = _allow("f32", fn)
    k = 3.0 if fn == "pow3" else 0.0
    name = "pow" if fn == "pow3" else fn
    max_abs_x = 2.0 ** 42 if fn == "pow3" else 0.0
    base = torch.arange(0, CHUNK, dtype=torch.int32, device="cuda")
    out = torch.empty(CHUNK, dtype=torch.float32, device="cuda")
    host = torch.empty(CHUNK, dtype=torch.float32, pin_memory=True)
    tot = None
    for b0 in range(0, 1 << 32, CHUNK):
        # bit patterns b0 .. b0 + CHUNK - 1 as int32 (two's complement); a
        # chunk never crosses the sign bit, so the int32 add cannot overflow
        s0 = b0 - (1 << 32) if b0 >= (1 << 31) else b0
        X = (base + s0).view(torch.float32)
        _launch(fx, fn, X, out)
        host.copy_(out)
        tot = _merge(tot, oracle.sweep_f32(name, b0, host.numpy(), allow, k, max_abs_x), b0)
    rec = dict(tot, dtype="f32", fn=fn, inputs=1 << 32, allow=allow, max_abs_x=max_abs_x)
    rec["argmax_input"] = float(np.array([tot["argmax"]], np.uint32).view(np.float32)[0])
    _report(rec)
    if tot["n_bad"]:
        b = np.array([tot["first_bad"]], np.uint32)
        raise AssertionError("%s: %d FP32 results beyond %.3g u; first input %r (bits 0x%08x)"
                             % (fn, tot["n_bad"], allow, float(b.view(np.float32)[0]),
                                int(b[0])))


@pytest.mark.parametrize("fn", FUNCS)
def test_f64_sample(fn):
    torch, fx = need_gpu()
    allow = _allow("f64", fn)
    k = 3.0 if fn == "pow3" else 0.0
    name = "pow" if fn == "pow3" else fn
    n = 1 << 23
    tid = FUNCS.index(fn)
    by_bits = synth.raw(synth.SEED["mathsweep"], 2 * tid, n).view(np.float64)
    lo, hi = RANGE64[fn]
    u = synth.fill_f64(synth.SEED["mathsweep"], 2 * tid + 1, n)   # U[-1, 1]
    by_value = lo + (u + 1.0) * 0.5 * (hi - lo)
    x = np.concatenate([by_bits, by_value])
    X = torch.from_numpy(x).to("cuda")
    out = torch.empty_like(X)
    _launch(fx, fn, X, out)
    got = out.cpu().numpy()
    st = oracle.sweep_f64(name, x, got, allow, k)
    rec = dict(st, dtype="f64", fn=fn, inputs=int(x.size), allow=allow)
    rec["argmax_input"] = float(x[st["argmax"]]) if st["argmax"] >= 0 else None
    _report(rec)
    if st["n_bad"]:
        i = st["first_bad"]
        raise AssertionError("%s: %d FP64 results beyond %.3g u; first input %r got %r"
                             % (fn, st["n_bad"], allow, float(x[i]), float(got[i])))
