"""GPU parity of the paper's benchmark expressions (Sec. 4) and of the add-N
family against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_close, empty, from_dev, need_gpu, to_dev

pytestmark = pytest.mark.gpu

SCAL = {"swish": (1.0,), "gelu": (0.044715,)}
ARITY = {"add2": 2, "add4": 4, "relu": 1, "sigmoid": 1, "swish": 1, "gelu": 1, "expr3": 3}


def _inputs(name, n, dtype):
    if name == "expr3":  # X ~ U[-1,1], Y ~ U[-1,1] stored as FP64, W ~ U[1,2]: logs stay finite
        return ([synth.fill(7, 0, n, dtype), synth.fill(7, 1, n, "f64"),
                 synth.fill(7, 2, n, dtype, "uniform12")], [dtype, "f64", dtype])
    return [synth.fill(7, t, n, dtype) for t in range(ARITY[name])], [dtype] * ARITY[name]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("name", list(ARITY))
def test_paper_expressions(name, dtype):
    torch, fx = need_gpu()
    shape = (1000, 1001)
    n = shape[0] * shape[1]
    host, dts = _inputs(name, n, dtype)
    dev = [to_dev(h, d) for h, d in zip(host, dts)]
    Z = empty(n, dtype)
    sc = SCAL.get(name, ())
    fx.fx_paper_expr(name, dev, Z, shape, sc, dt=fx.dtype_code(dev[0]))
    torch.cuda.synchronize()
    s = {k: float(np.float32(v)) for k, v in zip(("beta",) if name == "swish" else ("alpha",), sc)}
    e = oracle.paper_expr(name, **s)
    v, mu = oracle.evaluate(e, host, dtype, shape=shape, input_dtypes=dts)
    half = dtype if dtype == "bf16" else None
    assert_close(from_dev(Z, dtype), v, mu, dtype, "paper %s %s" % (name, dtype), out_dtype=half)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("k", list(range(1, 17)))
def test_addn(k, dtype):
    torch, fx = need_gpu()
    n = 123457
    host = [synth.fill(8, t, n, dtype) for t in range(k)]
    Z = empty(n, dtype)
    fx.fx_addn([to_dev(h, dtype) for h in host], Z, (n, 1))
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.addn(k), host, dtype)
    half = dtype if dtype == "bf16" else None
    assert_close(from_dev(Z, dtype), v, mu, dtype, "add%d %s" % (k, dtype), out_dtype=half)


def test_paper_suite_full_size():
    """10k x 10k FP32 (the paper's size) in the benchmark's configuration:
    add16 and gelu, every element against the oracle."""
    torch, fx = need_gpu()
    shape = (10000, 10000)
    n = shape[0] * shape[1]
    host = [synth.fill(9, t, n, "f32") for t in range(16)]
    dev = [to_dev(h, "f32") for h in host]
    Z = empty(n, "f32")
    fx.fx_addn(dev, Z, shape)
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.addn(16), host, "f32", shape=shape)
    assert_close(from_dev(Z, "f32"), v, mu, "f32", "add16 10k")
    del v, mu
    fx.fx_paper_expr("gelu", dev[:1], Z, shape, (0.044715,))
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.paper_expr("gelu", alpha=float(np.float32(0.044715))), host[:1],
                            "f32", shape=shape)
    assert_close(from_dev(Z, "f32"), v, mu, "f32", "gelu 10k")
