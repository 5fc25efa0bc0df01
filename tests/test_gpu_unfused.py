"""GPU tests of the unfused baseline: single operators are bit-exact against
correctly rounded results (for + - * / sqrt in FP32, rounding the exact FP64
result once more is innocuous since 53 >= 2*24 + 2), whole expressions
evaluated one operator at a time pass the same oracle rule as the fused
kernels."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_close, empty, from_dev, inputs, need_gpu, to_dev

pytestmark = pytest.mark.gpu

N = 3 * 65536 + 17


def _host(t, dtype):
    return from_dev(t, dtype)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("op", ["add", "sub", "schur", "div"])
def test_binary_bit_exact(dtype, op):
    torch, fx = need_gpu()
    host, (A, B, _) = inputs(5, N, dtype)
    B = B + 1.5 if op == "div" else B   # keep divisors away from zero
    out = empty(N, dtype)
    fx.fx_op_binary(op, A, B, out)
    torch.cuda.synchronize()
    a, b = _host(A, dtype), _host(B, dtype)
    exact = {"add": a + b, "sub": a - b, "schur": a * b, "div": a / b}[op]
    want = exact.astype(np.float32).astype(np.float64) if dtype == "f32" else exact
    assert np.array_equal(_host(out, dtype), want)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("op", ["neg", "abs", "sqrt", "exp"])
def test_unary(dtype, op):
    torch, fx = need_gpu()
    host, (A, _, _) = inputs(5, N, dtype)
    if op == "sqrt":
        A = A.abs()
    out = empty(N, dtype)
    fx.fx_op_unary(op, A, out)
    torch.cuda.synchronize()
    a = _host(A, dtype)
    got = _host(out, dtype)
    if op == "exp":
        ex = np.exp(a)
        ulp = np.spacing(ex.astype(np.float32)).astype(np.float64) if dtype == "f32" else np.spacing(ex)
        assert np.max(np.abs(got - ex) / ulp) <= 1.0    # within one ulp of the exact value
        return
    exact = {"neg": -a, "abs": np.abs(a), "sqrt": np.sqrt(a)}[op]
    want = exact.astype(np.float32).astype(np.float64) if dtype == "f32" else exact
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("op,k", [("sadd", 1.0), ("smul", 2.0), ("sdiv", 3.0), ("srdiv", 3.0),
                                  ("ssub", 0.5), ("srsub", 0.5)])
def test_scalar_bit_exact(dtype, op, k):
    torch, fx = need_gpu()
    _, (A, _, _) = inputs(6, N, dtype)
    A = A + 2.0 if op == "srdiv" else A
    out = empty(N, dtype)
    fx.fx_op_scalar(op, A, k, out)
    torch.cuda.synchronize()
    a = _host(A, dtype)
    exact = {"sadd": k + a, "smul": k * a, "sdiv": a / k, "srdiv": k / a, "ssub": a - k,
             "srsub": k - a}[op]
    want = exact.astype(np.float32).astype(np.float64) if dtype == "f32" else exact
    assert np.array_equal(_host(out, dtype), want)


@pytest.mark.parametrize("op", ["add", "sub", "schur", "xor"])
def test_u32_binary_bit_exact(op):
    torch, fx = need_gpu()
    host, (A, B, _) = inputs(1, N, "u32")
    out = empty(N, "u32")
    fx.fx_op_binary(op, A, B, out)
    torch.cuda.synchronize()
    a, b = host[0].astype(np.uint64), host[1].astype(np.uint64)
    m = np.uint64(0xFFFFFFFF)
    want = {"add": (a + b) & m, "sub": (a - b) & m, "schur": (a * b) & m, "xor": a ^ b}[op]
    assert np.array_equal(from_dev(out, "u32"), want.astype(np.uint32))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_half_ops_round_once(dtype):
    torch, fx = need_gpu()
    host, (A, B, _) = inputs(5, N, dtype)
    out = empty(N, dtype)
    fx.fx_op_binary("schur", A, B, out)
    torch.cuda.synchronize()
    a, b = from_dev(A, dtype), from_dev(B, dtype)
    if dtype == "bf16":   # the product of two bf16 values is exact in FP32
        want = torch.from_numpy((a * b).astype(np.float32)).to(torch.bfloat16).float().double()
        assert np.array_equal(from_dev(out, dtype), want.numpy())
    else:                 # FP32: the exact (FP64) product rounded once
        want = (a * b).astype(np.float32).astype(np.float64)
        assert np.array_equal(from_dev(out, dtype), want)


EXPRS = [("c1_z", "c1_z", None), ("c2_z", "c2_z", None), ("accu_xy", "xy", "accu"),
         ("norm_diff", "diff", "norm"), ("c2_colsum", "c2_z", "colsum"),
         ("c2_rowsum", "c2_z", "rowsum"), ("colsum_xy", "xy", "colsum")]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("name,oname,red", EXPRS)
def test_unfused_expressions_vs_oracle(dtype, name, oname, red):
    torch, fx = need_gpu()
    shape = (1000, 333)
    n = shape[0] * shape[1]
    host, devs = inputs(2, n, dtype)
    tmp = torch.zeros(fx.fx_unfused_tmp_bytes(name, fx.dtype_code(devs[0]), shape),
                      dtype=torch.uint8, device="cuda")
    kind = {None: None, "accu": fx.R_ACCU, "norm": fx.R_NORM, "colsum": fx.R_COLSUM,
            "rowsum": fx.R_ROWSUM}[red]
    ws = fx.workspace(kind, fx.dtype_code(devs[0]), shape) if kind else None
    acc = "f64" if dtype == "f64" else "f32"
    if red is None:
        out = empty(n, dtype)
    elif red in ("accu", "norm"):
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
    else:
        out = empty(shape[1] if red == "colsum" else shape[0], acc)
    fx.fx_unfused(name, devs, out, shape, tmp, ws)
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.EXPRS[oname], host[:oracle.EXPRS[oname].n_inputs()], dtype,
                            shape=shape, reduce=red)
    got = from_dev(out, dtype if red is None else ("f64" if red in ("accu", "norm") else acc))
    assert_close(got, v, mu, dtype, "unfused %s %s" % (name, dtype))


def test_unfused_u32_c1_bit_exact():
    torch, fx = need_gpu()
    host, devs = inputs(1, N, "u32")
    tmp = torch.zeros(fx.fx_unfused_tmp_bytes("c1_z", fx.U32, (N, 1)), dtype=torch.uint8,
                      device="cuda")
    out = empty(N, "u32")
    fx.fx_unfused("c1_z", devs, out, (N, 1), tmp)
    torch.cuda.synchronize()
    want, _ = oracle.evaluate_u32(oracle.EXPRS["u32_z"], host)
    assert np.array_equal(from_dev(out, "u32"), want)


def test_unfused_axy_expw():
    torch, fx = need_gpu()
    host, devs = inputs(7, N, "f32")
    a = 0.375
    tmp = torch.zeros(fx.fx_unfused_tmp_bytes("axy_expw", fx.F32, (N, 1)), dtype=torch.uint8,
                      device="cuda")
    out = empty(N, "f32")
    fx.fx_unfused("axy_expw", devs, out, (N, 1), tmp, a=a)
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.axy_expw(a), host, "f32")
    assert_close(from_dev(out, "f32"), v, mu, "f32", "unfused axy_expw")
