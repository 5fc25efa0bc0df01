"""GPU tests of the kernels generated as source from expression types and
compiled by the driver at first use: every workload expression in every
storage type against the oracle (ragged shapes, split reductions, empty
shapes), u32 bit-exact, and agreement with the ahead-of-time kernel that the
same expression type instantiates."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_close, empty, from_dev, inputs, need_gpu

pytestmark = pytest.mark.gpu

FP = ["f32", "f64", "bf16", "f16"]
ACC = {"f32": "f32", "bf16": "f32", "f16": "f32", "f64": "f64"}
# expression id -> (oracle expression, reduction, inputs)
EXPRS = {"c1_z": ("c1_z", None, 3), "accu_xy": ("xy", "accu", 2), "c2_z": ("c2_z", None, 3),
         "c2_colsum": ("c2_z", "colsum", 3), "c2_rowsum": ("c2_z", "rowsum", 3),
         "norm_diff": ("diff", "norm", 2), "colsum_xy": ("xy", "colsum", 2)}
KIND = {None: 0, "accu": 1, "colsum": 2, "rowsum": 3, "norm": 4}


def _out(torch, red, shape, dtype):
    n = shape[0] * shape[1]
    if red is None:
        return empty(n, dtype), dtype
    if red in ("accu", "norm"):
        return torch.zeros(1, dtype=torch.float64, device="cuda"), "f64"
    return empty(shape[1] if red == "colsum" else shape[0], ACC[dtype]), ACC[dtype]


@pytest.mark.parametrize("dtype", FP)
@pytest.mark.parametrize("expr", sorted(EXPRS))
@pytest.mark.parametrize("shape", [(1000, 333), (8192, 17), (64, 4099)])
def test_workloads_against_the_oracle(dtype, expr, shape):
    torch, fx = need_gpu()
    oname, red, k = EXPRS[expr]
    n = shape[0] * shape[1]
    host, devs = inputs(12, n, dtype, k=k)
    out, od = _out(torch, red, shape, dtype)
    dcode = fx.dtype_code(devs[0])
    ws = fx.workspace(KIND[red], dcode, shape) if red else None
    for _ in range(2):      # the workspace is left zeroed for the next call
        fx.fx_source_eval(expr, devs, out, shape, ws)
        torch.cuda.synchronize()
        v, mu = oracle.evaluate(oracle.EXPRS[oname], host, dtype, shape=shape, reduce=red)
        assert_close(from_dev(out, od), v, mu, dtype, "source %s %s %s" % (expr, dtype, shape),
                     out_dtype=dtype if red is None and dtype in ("bf16", "f16") else None)


def test_axy_expw_and_u32():
    torch, fx = need_gpu()
    n = (1 << 20) + 12
    host, devs = inputs(13, n, "f32")
    Z = empty(n, "f32")
    a = 0.375
    fx.fx_source_eval("axy_expw", devs, Z, (n, 1), a=a)
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.axy_expw(a), host, "f32")
    assert_close(from_dev(Z, "f32"), v, mu, "f32", "source axy_expw")
    hu, du = inputs(13, n, "u32")
    ZU = empty(n, "u32")
    fx.fx_source_eval("c1_z", du, ZU, (n, 1))
    torch.cuda.synchronize()
    want, _ = oracle.evaluate_u32(oracle.EXPRS["u32_z"], hu)
    assert np.array_equal(from_dev(ZU, "u32"), want)


def test_same_type_as_the_compile_time_kernel():
    """The generated kernel and the ahead-of-time kernel of the same
    expression type both pass the rule on the same inputs (their compilers
    may contract multiply-adds differently, so bits may differ)."""
    torch, fx = need_gpu()
    shape = (4096, 1000)
    n = shape[0] * shape[1]
    host, (X, Y, W) = inputs(14, n, "f32")
    Za, Zs = empty(n, "f32"), empty(n, "f32")
    fx.fx_c2_z(X, Y, W, Za, shape)
    fx.fx_source_eval("c2_z", [X, Y, W], Zs, shape)
    ca, cs = empty(shape[1], "f32"), empty(shape[1], "f32")
    ws = fx.workspace(fx.R_COLSUM, fx.F32, shape)
    fx.fx_c2_colsum(X, Y, W, ca, shape, ws)
    fx.fx_source_eval("c2_colsum", [X, Y, W], cs, shape, ws)
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.EXPRS["c2_z"], host, "f32", shape=shape)
    assert_close(from_dev(Zs, "f32"), v, mu, "f32", "source Z")
    assert_close(from_dev(Za, "f32"), v, mu, "f32", "compiled Z")
    print("identical Z elements: %.4f" % torch.eq(Za, Zs).float().mean().item())
    v, mu = oracle.evaluate(oracle.EXPRS["c2_z"], host, "f32", shape=shape, reduce="colsum")
    assert_close(from_dev(cs, "f32"), v, mu, "f32", "source colsum")
    assert_close(from_dev(ca, "f32"), v, mu, "f32", "compiled colsum")


def test_empty_and_degenerate_shapes():
    torch, fx = need_gpu()
    X = torch.zeros(16, device="cuda")
    out = torch.full((5,), 7.0, device="cuda")
    fx.fx_source_eval("c2_colsum", [X, X, X], out, (0, 5))
    s = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    fx.fx_source_eval("accu_xy", [X, X], s, (0, 1))
    fx.fx_source_eval("c2_z", [X, X, X], out, (0, 0))
    torch.cuda.synchronize()
    assert out.eq(0).all() and s.item() == 0.0
    for shape in [(1, 1), (1, 7), (7, 1), (3, 5)]:
        n = shape[0] * shape[1]
        host, devs = inputs(15, n, "f32")
        c = empty(shape[1], "f32")
        fx.fx_source_eval("c2_colsum", devs, c, shape, fx.workspace(fx.R_COLSUM, fx.F32, shape))
        torch.cuda.synchronize()
        v, mu = oracle.evaluate(oracle.EXPRS["c2_z"], host, "f32", shape=shape, reduce="colsum")
        assert_close(from_dev(c, "f32"), v, mu, "f32", "source colsum %s" % (shape,))
