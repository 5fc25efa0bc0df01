"""GPU parity of the run-time source mode (hipRTC-compiled kernels) against
the FP64 oracle and the compile-time path: every result kind and storage
type, ragged and degenerate shapes, workspace reuse."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_close, empty, from_dev, need_gpu, oracle_expr, tree_inputs
from synth import trees

pytestmark = pytest.mark.gpu

FP = ["f32", "f64", "bf16", "f16"]
ACC = {"f32": "f32", "bf16": "f32", "f16": "f32", "f64": "f64"}


def _code(fx, dtype):
    return {"f32": fx.F32, "f64": fx.F64, "bf16": fx.BF16, "f16": fx.F16}[dtype]


def _run(fx, torch, nodes, k, seed, e, dtype, shape, kind, repeat=1):
    n = shape[0] * shape[1]
    host, dev = tree_inputs(seed, e, k, n, dtype)
    dcode = _code(fx, dtype)
    red = {0: None, fx.R_ACCU: "accu", fx.R_NORM: "norm", fx.R_COLSUM: "colsum",
           fx.R_ROWSUM: "rowsum"}[kind]
    if kind == 0:
        out, od = empty(n, dtype), dtype
    elif kind in (fx.R_ACCU, fx.R_NORM):
        out, od = torch.full((1,), 7.0, dtype=torch.float64, device="cuda"), "f64"
    else:
        out, od = empty(shape[1] if kind == fx.R_COLSUM else shape[0], ACC[dtype]), ACC[dtype]
    ws = fx.workspace(kind, dcode, shape) if kind else None
    r = fx.Rtc(nodes, dcode, kind)
    got = []
    for _ in range(repeat):                    # the finish clears its counters for reuse
        r.eval(dev, out, shape, ws)
        torch.cuda.synchronize()
        got.append(from_dev(out, od).copy())
    for g in got[1:]:
        assert np.array_equal(g, got[0], equal_nan=True), "repeat differs"
    v, mu = oracle.evaluate(oracle_expr(nodes), host, dtype, shape=shape, reduce=red)
    out_half = dtype if (kind == 0 and dtype in ("bf16", "f16")) else None
    return assert_close(got[0], v, mu, dtype,
                        "rtc seed %d tree %d %s kind %d %s" % (seed, e, dtype, kind, shape),
                        out_dtype=out_half)


@pytest.mark.parametrize("dtype", FP)
@pytest.mark.parametrize("e", range(0, 40, 5))
def test_random_trees_elementwise(dtype, e):
    torch, fx = need_gpu()
    nodes, k, _ = trees.random_tree(4, e)
    for n in (1, 3, 1000, 100003):
        _run(fx, torch, nodes, k, 4, e, dtype, (n, 1), 0)


@pytest.mark.parametrize("dtype", FP)
@pytest.mark.parametrize("e", range(1, 40, 6))
def test_random_trees_accu_and_norm(dtype, e):
    torch, fx = need_gpu()
    nodes, k, _ = trees.random_tree(4, e)
    _run(fx, torch, nodes, k, 4, e, dtype, (50000 + e, 1), fx.R_ACCU, repeat=2)
    _run(fx, torch, nodes, k, 4, e, dtype, (250, 201), fx.R_NORM)
    _run(fx, torch, nodes, k, 4, e, dtype, (3, 1), fx.R_ACCU)


@pytest.mark.parametrize("dtype", FP)
@pytest.mark.parametrize("e", range(2, 40, 7))
def test_random_trees_dim_sums(dtype, e):
    torch, fx = need_gpu()
    nodes, k, _ = trees.random_tree(5, e, depth=(2, 8))
    _run(fx, torch, nodes, k, 5, e, dtype, (1024, 77), fx.R_COLSUM, repeat=2)
    _run(fx, torch, nodes, k, 5, e, dtype, (1000, 65), fx.R_ROWSUM, repeat=2)
    _run(fx, torch, nodes, k, 5, e, dtype, (7, 300), fx.R_COLSUM)       # thin columns
    _run(fx, torch, nodes, k, 5, e, dtype, (1001, 33), fx.R_COLSUM)     # rows not whole vectors
    _run(fx, torch, nodes, k, 5, e, dtype, (1001, 33), fx.R_ROWSUM)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_split_reductions(dtype):
    # shapes whose default launch splits the reduction over many blocks:
    # long columns (chunks per column), short wide matrices (column chunks
    # per row block) and a long vector (one partial per block)
    torch, fx = need_gpu()
    nodes, k, _ = trees.random_tree(6, 3)
    for shape, kind in (((1 << 17, 5), fx.R_COLSUM), ((64, 20000), fx.R_ROWSUM),
                        ((1 << 21, 1), fx.R_ACCU)):
        split = fx.fx_resolve_launch(kind, _code(fx, dtype), shape)[3]
        assert split > 1, (shape, split)
        _run(fx, torch, nodes, k, 6, 3, dtype, shape, kind, repeat=3)


def test_degenerate_shapes():
    torch, fx = need_gpu()
    from test_rtc_host import C2
    x = torch.zeros(16, device="cuda")
    # an empty element-wise result is a no-op; accu and norm of nothing are 0;
    # sums over an empty dimension are zeros
    fx.Rtc(C2, fx.F32).eval([x, x, x], x, (0, 1))
    for kind in (fx.R_ACCU, fx.R_NORM):
        out = torch.full((1,), 5.0, dtype=torch.float64, device="cuda")
        fx.Rtc(C2, fx.F32, kind).eval([x, x, x], out, (0, 4))
        torch.cuda.synchronize()
        assert out.item() == 0.0
    cs = torch.full((5,), 3.0, device="cuda")
    fx.Rtc(C2, fx.F32, fx.R_COLSUM).eval([x, x, x], cs, (0, 5))
    rs = torch.full((4,), 3.0, device="cuda")
    fx.Rtc(C2, fx.F32, fx.R_ROWSUM).eval([x, x, x], rs, (4, 0))
    torch.cuda.synchronize()
    assert cs.abs().sum().item() == 0.0 and rs.abs().sum().item() == 0.0


def test_constants_sum_exactly():
    # accu of a constant tree over m*k elements and its column/row sums are
    # exact (every partial is an integer below 2^24)
    torch, fx = need_gpu()
    one = [("const", -1, -1, -1, 1.0)]
    m, k = 4096, 3000
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    shape = (m, k)
    fx.Rtc(one, fx.F32, fx.R_ACCU).eval([], out, shape, fx.workspace(fx.R_ACCU, fx.F32, shape))
    cs = torch.empty(k, device="cuda")
    fx.Rtc(one, fx.F32, fx.R_COLSUM).eval([], cs, shape, fx.workspace(fx.R_COLSUM, fx.F32, shape))
    rs = torch.empty(m, device="cuda")
    fx.Rtc(one, fx.F32, fx.R_ROWSUM).eval([], rs, shape, fx.workspace(fx.R_ROWSUM, fx.F32, shape))
    torch.cuda.synchronize()
    assert out.item() == m * k
    assert bool((cs == m).all()) and bool((rs == k).all())


def test_matches_the_compile_time_kernel():
    torch, fx = need_gpu()
    from test_rtc_host import C2
    import synth
    n = 1 << 20
    host = [synth.fill(2, t, n, "f32") for t in range(3)]
    dev = [torch.from_numpy(h).cuda() for h in host]
    a, b = empty(n, "f32"), empty(n, "f32")
    fx.Rtc(C2, fx.F32).eval(dev, a)
    fx.fx_c2_z(*dev, b, (n, 1))
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.EXPRS["c2_z"], host, "f32")
    assert_close(from_dev(a, "f32"), v, mu, "f32", "rtc c2")
    # same operations in the same order: the results agree to the last bit
    # wherever neither side contracted a product into an FMA differently
    same = np.mean(a.cpu().numpy() == b.cpu().numpy())
    assert same > 0.99, same


def test_column_sums_match_the_compile_time_kernel():
    # the matrix workload's column sums at a reduced size: the generated
    # kernel and the fused one assign elements to threads the same way
    torch, fx = need_gpu()
    from test_rtc_host import C2
    import synth
    shape = (4096, 512)
    n = shape[0] * shape[1]
    host = [synth.fill(2, t, n, "f32") for t in range(3)]
    dev = [torch.from_numpy(h).cuda() for h in host]
    a, b = empty(shape[1], "f32"), empty(shape[1], "f32")
    fx.Rtc(C2, fx.F32, fx.R_COLSUM).eval(dev, a, shape, fx.workspace(fx.R_COLSUM, fx.F32, shape))
    fx.fx_c2_colsum(*dev, b, shape, fx.workspace(fx.R_COLSUM, fx.F32, shape))
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.EXPRS["c2_z"], host, "f32", shape=shape, reduce="colsum")
    assert_close(from_dev(a, "f32"), v, mu, "f32", "rtc c2 colsum")
    assert_close(from_dev(b, "f32"), v, mu, "f32", "fused c2 colsum")


def test_misaligned_arrays_are_refused():
    torch, fx = need_gpu()
    from test_rtc_host import C2
    x = torch.zeros(1027, device="cuda")
    out = torch.empty(1026, device="cuda")
    with pytest.raises(fx.FxError) as e:
        fx.Rtc(C2, fx.F32).eval([x[1:], x[1:], x[1:]], out)
    assert e.value.code == 1


def test_missing_workspace_is_refused():
    torch, fx = need_gpu()
    from test_rtc_host import C2
    shape = (1 << 20, 1)
    x = torch.zeros(shape[0], device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(fx.FxError) as e:
        fx.Rtc(C2, fx.F32, fx.R_ACCU).eval([x, x, x], out, shape)
    assert e.value.code == 4                    # FX_E_WORKSPACE
