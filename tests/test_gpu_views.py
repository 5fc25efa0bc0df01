"""GPU parity of the paper's strided-view expressions (Sec. 4: centre
submatrices, transposes, diagonals) against the FP64 oracle's views."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_close, empty, from_dev, need_gpu, to_dev

pytestmark = pytest.mark.gpu

ARITY = {"addsub2": 2, "addsub4": 4, "expr1": 2, "expr2": 4, "diagsum": 2}
# square sizes: one tile, several tiles with ragged edges, odd rows (the
# scalar kernel: rows not a multiple of the vector width); FP32 squares with
# rows a multiple of 4 span 1, 2, 3, 16 and 17 tiles a side
SIZES = [1, 2, 7, 64, 65, 128, 130, 192, 257, 1000, 1028]


def _inputs(name, m, n, dtype, seed=21):
    k = ARITY[name]
    host = [synth.fill(seed, t, m * n, dtype) for t in range(k)]
    if name == "expr2":   # D away from 0 so log(D^2) stays finite
        host[3] = synth.fill(seed, 3, m * n, dtype, "uniform12")
    return host


def _check(name, m, n, dtype, a=1.5):
    torch, fx = need_gpu()
    host = _inputs(name, m, n, dtype)
    dev = [to_dev(h, dtype) for h in host]
    shape = fx.fx_paper_view_shape(name, (m, n))
    e, oshape = oracle.paper_view_expr(name, m, n, a=float(np.float32(a)) if dtype != "f64" else a)
    assert tuple(shape) == tuple(oshape)
    Z = empty(max(1, shape[0] * shape[1]), dtype)
    fx.fx_paper_view_expr(name, dev, Z, (m, n), (a,))
    torch.cuda.synchronize()
    if shape[0] * shape[1] == 0:
        return
    v, mu = oracle.evaluate(e, host, dtype, shape=oshape)
    half = dtype if dtype == "bf16" else None
    got = from_dev(Z, dtype)[:shape[0] * shape[1]]
    assert_close(got, v, mu, dtype, "%s %dx%d %s" % (name, m, n, dtype), out_dtype=half)


@pytest.mark.parametrize("dtype", ["f32", "f64", "bf16"])
@pytest.mark.parametrize("m", SIZES)
@pytest.mark.parametrize("name", list(ARITY))
def test_view_expressions_square(name, m, dtype):
    _check(name, m, m, dtype)


@pytest.mark.parametrize("shape", [(9, 4), (4, 9), (130, 67), (67, 130), (256, 64)])
@pytest.mark.parametrize("name", ["addsub2", "addsub4", "diagsum"])
def test_view_expressions_rectangular(name, shape):
    _check(name, shape[0], shape[1], "f32")


def test_square_only_expressions_refuse_rectangles():
    torch, fx = need_gpu()
    for name in ("expr1", "expr2"):
        with pytest.raises(fx.FxError) as e:
            fx.fx_paper_view_shape(name, (4, 5))
        assert e.value.code == 2     # FX_E_SHAPE


def _block_expr(name, m, R0, C0, B, a):
    """The oracle's expression for the B x B block of the full result that
    starts at (R0, C0): every leaf is a view into the full inputs."""
    V = lambda q, off, rs, cs: oracle.E("leaf", leaf=q, view=(off, rs, cs))
    plain = lambda q, r0=0, c0=0: V(q, (R0 + r0) + (C0 + c0) * m, 1, m)
    trans = lambda q: V(q, C0 + R0 * m, m, 1)
    if name == "expr1":
        return 2 * (trans(0) + plain(1)) + 2 * (plain(0) + trans(1))
    if name == "expr2":
        return a * plain(0) + (trans(1) + trans(2)) + oracle.log(oracle.pow_(plain(3), 2))
    r0, c0, _, _ = oracle.center(m, m)
    return plain(0, r0, c0) + plain(1, r0, c0) + plain(2, r0, c0) + plain(3, r0, c0)


def test_views_full_size_sampled():
    """10k x 10k FP32, the paper's size and the benchmark's launch: three
    64 x 64 blocks of each result (first, last with its ragged tile, one
    inside) against the oracle evaluating those blocks through views of the
    same full-size inputs."""
    torch, fx = need_gpu()
    m, B, a = 10000, 64, 1.5
    for name in ("expr1", "expr2", "addsub4"):
        host = _inputs(name, m, m, "f32", seed=23)
        dev = [to_dev(h, "f32") for h in host]
        shape = fx.fx_paper_view_shape(name, (m, m))
        Z = empty(shape[0] * shape[1], "f32")
        fx.fx_paper_view_expr(name, dev, Z, (m, m), (a,))
        torch.cuda.synchronize()
        full = Z.view(shape[1], shape[0]).cpu().numpy().T   # rows x cols
        for R0, C0 in ((0, 0), (shape[0] - B, shape[1] - B), (shape[0] // 2 + 1, shape[1] // 3 + 1)):
            e = _block_expr(name, m, R0, C0, B, float(np.float32(a)))
            v, mu = oracle.evaluate(e, host, "f32", shape=(B, B))
            got = full[R0:R0 + B, C0:C0 + B].reshape(-1, order="F").astype(np.float64)
            assert_close(got, v, mu, "f32", "%s block (%d, %d)" % (name, R0, C0))
        del dev, Z
