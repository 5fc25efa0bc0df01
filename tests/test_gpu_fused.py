"""GPU parity of the fused entry points against the FP64 oracle, through the
C ABI.  Sizes span several tiles and ragged tails; configurations cover the
compiled vector widths and EPT values."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_close, empty, from_dev, inputs, need_gpu, to_dev

pytestmark = pytest.mark.gpu

FP = ["f32", "f64", "bf16", "f16"]
NS = [0, 1, 3, 4, 5, 63, 64, 65, 1023, 1025, 4097, 65537, (1 << 20) + 3]
CFGS = [None, (64, 1, 0, 0), (128, 2, 16, 3), (256, 4, 16, 0), (512, 8, 16, 7),
        (256, 8, 0, 1), (192, 4, 4, 0)]


ELEM = {"f32": 4, "f64": 8, "bf16": 2, "f16": 2, "u32": 4}


def _compiled(cfg, dtype):
    """Compiled vector widths: the element size and 16 bytes."""
    return cfg is None or cfg[2] in (0, 16, ELEM[dtype]) or (cfg[2] < ELEM[dtype])


@pytest.mark.parametrize("dtype", FP)
@pytest.mark.parametrize("n", NS)
def test_c1_z(dtype, n):
    torch, fx = need_gpu()
    host, (X, Y, W) = inputs(1, n, dtype)
    Z = empty(n, dtype)
    fx.fx_c1_z(X, Y, W, Z)
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.EXPRS["c1_z"], host, dtype)
    out = dtype if dtype in ("bf16", "f16") else None
    assert_close(from_dev(Z, dtype), v, mu, dtype, "c1_z %s n=%d" % (dtype, n), out_dtype=out)


@pytest.mark.parametrize("cfg", CFGS)
@pytest.mark.parametrize("dtype", FP)
def test_c1_z_configs(dtype, cfg):
    torch, fx = need_gpu()
    n = 3 * 65536 + 11
    host, (X, Y, W) = inputs(1, n, dtype)
    Z = empty(n, dtype)
    if not _compiled(cfg, dtype):
        with pytest.raises(fx.FxError) as ei:
            fx.fx_c1_z(X, Y, W, Z, cfg=cfg)
        assert ei.value.code == 6  # FX_E_UNSUPPORTED, nothing enqueued
        return
    fx.fx_c1_z(X, Y, W, Z, cfg=cfg)
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.EXPRS["c1_z"], host, dtype)
    out = dtype if dtype in ("bf16", "f16") else None
    assert_close(from_dev(Z, dtype), v, mu, dtype, "c1_z cfg %s" % (cfg,), out_dtype=out)


# Outputs just below and just above the 256 MiB last-level cache: the first
# take ordinary stores, the second streaming stores; every element, ragged
# tails included, must match the oracle either way.
@pytest.mark.parametrize("dtype,n", [("f32", (1 << 26) - 59), ("f32", (1 << 26) + 37),
                                     ("bf16", (1 << 27) + 37), ("u32", (1 << 26) + 37)])
def test_store_policy_both_sides(dtype, n):
    torch, fx = need_gpu()
    host, (X, Y, W) = inputs(1, n, dtype)
    Z = empty(n, dtype)
    fx.fx_c1_z(X, Y, W, Z)
    torch.cuda.synchronize()
    if dtype == "u32":
        want, _ = oracle.evaluate_u32(oracle.EXPRS["u32_z"], host)
        assert np.array_equal(from_dev(Z, "u32"), want)
        return
    v, mu = oracle.evaluate(oracle.EXPRS["c1_z"], host, dtype)
    out = dtype if dtype in ("bf16", "f16") else None
    assert_close(from_dev(Z, dtype), v, mu, dtype, "c1_z %s n=%d" % (dtype, n), out_dtype=out)


@pytest.mark.parametrize("n", NS)
def test_c1_z_u32_bit_exact(n):
    torch, fx = need_gpu()
    host, (X, Y, W) = inputs(1, n, "u32")
    Z = empty(n, "u32")
    fx.fx_c1_z(X, Y, W, Z)
    torch.cuda.synchronize()
    want, _ = oracle.evaluate_u32(oracle.EXPRS["u32_z"], host)
    assert np.array_equal(from_dev(Z, "u32"), want)


def test_c1_z_misaligned_and_in_place():
    torch, fx = need_gpu()
    n = 10001
    host, (X, Y, W) = inputs(1, n + 1, "f32")
    # offset views are 4-byte but not 16-byte aligned: the scalar path runs
    Xo, Yo, Wo = X[1:], Y[1:], W[1:]
    Z = empty(n + 1, "f32")[1:]
    fx.fx_c1_z(Xo, Yo, Wo, Z)
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.EXPRS["c1_z"], [h[1:].copy() for h in host], "f32")
    assert_close(from_dev(Z, "f32"), v, mu, "f32", "misaligned")
    # exact aliasing of output and input is allowed
    fx.fx_c1_z(X, Y, W, W)
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.EXPRS["c1_z"], host, "f32")
    assert_close(from_dev(W, "f32"), v, mu, "f32", "in place")


@pytest.mark.parametrize("dtype", FP)
def test_c1_z_closed_forms(dtype):
    torch, fx = need_gpu()
    n = 70001
    host, (X, Y, W) = inputs(1, n, dtype)
    Z = empty(n, dtype)
    zero = torch.zeros_like(W)
    fx.fx_c1_z(X, Y, zero, Z)      # W = 0: Z = round(X*Y)
    torch.cuda.synchronize()
    xy = from_dev(X, dtype) * from_dev(Y, dtype)
    if dtype == "f32":
        assert np.array_equal(from_dev(Z, dtype), xy.astype(np.float32).astype(np.float64))
    if dtype == "f64":
        assert np.array_equal(from_dev(Z, dtype), xy)
    fx.fx_c1_z(X, torch.zeros_like(Y), W, Z)   # Y = 0: Z = 2W exactly
    torch.cuda.synchronize()
    assert np.array_equal(from_dev(Z, dtype), 2 * from_dev(W, dtype))


@pytest.mark.parametrize("dtype", FP)
def test_axy_expw(dtype):
    torch, fx = need_gpu()
    n = 100003
    host, (X, Y, W) = inputs(7, n, dtype)
    a = -1.75
    Z = empty(n, dtype)
    fx.fx_axy_expw(a, X, Y, W, Z)
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.axy_expw(a), host, dtype)
    out = dtype if dtype in ("bf16", "f16") else None
    assert_close(from_dev(Z, dtype), v, mu, dtype, "axy_expw", out_dtype=out)


# ---- full reductions --------------------------------------------------------------

@pytest.mark.parametrize("dtype", FP)
@pytest.mark.parametrize("n", NS)
def test_accu_xy(dtype, n):
    torch, fx = need_gpu()
    host, (X, Y, _) = inputs(1, n, dtype)
    out = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    ws = fx.workspace(fx.R_ACCU, fx.dtype_code(X), (n, 1))
    fx.fx_accu_xy(X, Y, out, ws)
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.EXPRS["xy"], host[:2], dtype, reduce="accu")
    assert_close(out.cpu().numpy(), v, mu, dtype, "accu %s n=%d" % (dtype, n))
    if ws is not None:
        assert int(ws[:4].view(torch.int32).item()) == 0, "ticket counter not reset"


@pytest.mark.parametrize("cfg", CFGS)
def test_accu_configs_and_determinism(cfg):
    torch, fx = need_gpu()
    n = (1 << 18) + 5
    host, (X, Y, _) = inputs(2, n, "f32")
    ws = fx.workspace(fx.R_ACCU, fx.F32, (n, 1), cfg)
    outs = []
    for _ in range(3):
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
        fx.fx_accu_xy(X, Y, out, ws, cfg=cfg)
        torch.cuda.synchronize()
        outs.append(out.item())
    assert outs[0] == outs[1] == outs[2], "not bitwise reproducible: %s" % outs
    v, mu = oracle.evaluate(oracle.EXPRS["xy"], host[:2], "f32", reduce="accu")
    assert_close(np.array(outs[:1]), v, mu, "f32", "accu cfg %s" % (cfg,))
    d = torch.zeros(1, dtype=torch.float64, device="cuda")
    fx.fx_dot(X, Y, d, ws, cfg=cfg)
    torch.cuda.synchronize()
    assert d.item() == outs[0]


def test_accu_u32_exact():
    torch, fx = need_gpu()
    n = (1 << 20) + 3
    host, (X, Y, _) = inputs(1, n, "u32")
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = fx.workspace(fx.R_ACCU, fx.U32, (n, 1))
    fx.fx_accu_xy(X, Y, out, ws)
    torch.cuda.synchronize()
    got = int(out.cpu().numpy().view(np.uint64)[0])
    prod = (host[0].astype(np.uint64) * host[1].astype(np.uint64)) & np.uint64(0xFFFFFFFF)
    assert got == int(prod.sum(dtype=np.uint64))


@pytest.mark.parametrize("n", [1, 1000, (1 << 20) + 1, 1 << 24])
def test_accu_of_ones_exact(n):
    torch, fx = need_gpu()
    ones = torch.ones(n, dtype=torch.float32, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = fx.workspace(fx.R_ACCU, fx.F32, (n, 1))
    fx.fx_accu_xy(ones, ones, out, ws)
    torch.cuda.synchronize()
    assert out.item() == n


def test_kahan_known_answer():
    """[1.0] followed by 2^24 copies of 2^-24 summed by 64 threads in one
    block: thread 0 adds ~2^18 tiny terms to 1.0, which an uncompensated FP32
    sum would drop (1 + 2^-24 rounds to 1).  Exact answer 2.0."""
    torch, fx = need_gpu()
    n = (1 << 24) + 1
    x = torch.full((n,), 2.0 ** -24, dtype=torch.float32, device="cuda")
    x[0] = 1.0
    ones = torch.ones(n, dtype=torch.float32, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    for cfg in [(64, 1, 4, 1), (64, 4, 16, 1), (256, 4, 16, 1)]:
        fx.fx_accu_xy(x, ones, out, None, cfg=cfg)
        torch.cuda.synchronize()
        assert abs(out.item() - 2.0) <= 2.0 ** -23, (cfg, out.item())


@pytest.mark.parametrize("dtype", FP)
@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (7, 1), (3, 5), (17, 33), (64, 64),
                                   (65, 63), (8191, 3), (600, 700), (1024, 1024)])
def test_norm_fro_diff(dtype, shape):
    torch, fx = need_gpu()
    n = shape[0] * shape[1]
    host, (X, Y, _) = inputs(2, n, dtype)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = fx.workspace(fx.R_NORM, fx.dtype_code(X), shape)
    fx.fx_norm_fro_diff(X, Y, out, shape, ws)
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.EXPRS["diff"], host[:2], dtype, shape=shape, reduce="norm")
    assert_close(out.cpu().numpy(), v, mu, dtype, "norm %s %s" % (dtype, shape))


def test_norm_identities():
    torch, fx = need_gpu()
    shape = (1000, 777)
    n = shape[0] * shape[1]
    _, (X, Y, _) = inputs(2, n, "f32")
    ws = fx.workspace(fx.R_NORM, fx.F32, shape)

    def nrm(A, B):
        o = torch.zeros(1, dtype=torch.float64, device="cuda")
        fx.fx_norm_fro_diff(A, B, o, shape, ws)
        torch.cuda.synchronize()
        return o.item()

    assert nrm(X, X) == 0.0
    assert nrm(2 * X, 2 * Y) == 2 * nrm(X, Y)          # exact scaling by 2
    ones = torch.ones(8192 * 512, dtype=torch.float32, device="cuda")
    o = torch.zeros(1, dtype=torch.float64, device="cuda")
    zero = torch.zeros_like(ones)
    fx.fx_norm_fro_diff(ones, zero, o, (8192, 512), fx.workspace(fx.R_NORM, fx.F32, (8192, 512)))
    torch.cuda.synchronize()
    assert o.item() == math.sqrt(8192 * 512)


# ---- the C2 expression and its dimension sums ---------------------------------------

SHAPES = [(1, 1), (1, 7), (7, 1), (3, 5), (17, 33), (33, 17), (64, 64), (65, 63), (8191, 3),
          (3, 8191), (600, 700), (1024, 1024), (4096, 256)]


@pytest.mark.parametrize("dtype", FP)
@pytest.mark.parametrize("shape", SHAPES)
def test_c2_z_and_sums(dtype, shape):
    torch, fx = need_gpu()
    rows, cols = shape
    n = rows * cols
    host, (X, Y, W) = inputs(2, n, dtype)
    e = oracle.EXPRS["c2_z"]
    Z = empty(n, dtype)
    fx.fx_c2_z(X, Y, W, Z, shape)
    acc = "f64" if dtype == "f64" else "f32"
    cs, rs = empty(cols, acc), empty(rows, acc)
    fx.fx_c2_colsum(X, Y, W, cs, shape, fx.workspace(fx.R_COLSUM, fx.dtype_code(X), shape))
    fx.fx_c2_rowsum(X, Y, W, rs, shape, fx.workspace(fx.R_ROWSUM, fx.dtype_code(X), shape))
    torch.cuda.synchronize()
    out = dtype if dtype in ("bf16", "f16") else None
    v, mu = oracle.evaluate(e, host, dtype, shape=shape)
    assert_close(from_dev(Z, dtype), v, mu, dtype, "c2_z", out_dtype=out)
    v, mu = oracle.evaluate(e, host, dtype, shape=shape, reduce="colsum")
    assert_close(from_dev(cs, acc), v, mu, dtype, "c2 colsum %s %s" % (dtype, shape))
    v, mu = oracle.evaluate(e, host, dtype, shape=shape, reduce="rowsum")
    assert_close(from_dev(rs, acc), v, mu, dtype, "c2 rowsum %s %s" % (dtype, shape))


@pytest.mark.parametrize("cfg", [(64, 1, 0, 1), (128, 2, 16, 5), (256, 4, 16, 0),
                                 (512, 8, 16, 2), (256, 2, 4, 64)])
def test_dim_sum_configs(cfg):
    torch, fx = need_gpu()
    shape = (2048 + 8, 515)
    n = shape[0] * shape[1]
    host, (X, Y, W) = inputs(3, n, "f32")
    e = oracle.EXPRS["c2_z"]
    for kind, fn, m in [(fx.R_COLSUM, fx.fx_c2_colsum, shape[1]), (fx.R_ROWSUM, fx.fx_c2_rowsum, shape[0])]:
        ws = fx.workspace(kind, fx.F32, shape, cfg)
        outs = []
        for _ in range(2):
            o = empty(m, "f32")
            fn(X, Y, W, o, shape, ws, cfg=cfg)
            torch.cuda.synchronize()
            outs.append(o.cpu().numpy())
        assert np.array_equal(outs[0], outs[1])
        v, mu = oracle.evaluate(e, host, "f32", shape=shape,
                                reduce="colsum" if kind == fx.R_COLSUM else "rowsum")
        assert_close(outs[0].astype(np.float64), v, mu, "f32", "kind %d cfg %s" % (kind, cfg))


def test_dim_sums_of_ones_exact():
    torch, fx = need_gpu()
    for shape in [(8192, 64), (5, 9000), (3000, 2), (1 << 16, 1)]:
        n = shape[0] * shape[1]
        ones = torch.ones(n, dtype=torch.float32, device="cuda")
        cs, rs = empty(shape[1], "f32"), empty(shape[0], "f32")
        fx.fx_colsum_xy(ones, ones, cs, shape, fx.workspace(fx.R_COLSUM, fx.F32, shape))
        fx.fx_reduce(fx.R_ROWSUM, ones, None, rs, shape, fx.workspace(fx.R_ROWSUM, fx.F32, shape))
        torch.cuda.synchronize()
        assert (cs == shape[0]).all().item() and (rs == shape[1]).all().item(), shape


@pytest.mark.parametrize("dtype", ["bf16", "f16", "f32"])
def test_colsum_xy(dtype):
    torch, fx = need_gpu()
    shape = (1 << 10, 1 << 9)
    n = shape[0] * shape[1]
    host, (X, Y, _) = inputs(3, n, dtype)
    cs = empty(shape[1], "f32")
    fx.fx_colsum_xy(X, Y, cs, shape, fx.workspace(fx.R_COLSUM, fx.dtype_code(X), shape))
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.EXPRS["xy"], host[:2], dtype, shape=shape, reduce="colsum")
    assert_close(from_dev(cs, "f32"), v, mu, dtype, "colsum_xy")


def test_empty_dimension_sums_write_zero():
    torch, fx = need_gpu()
    X = torch.empty(0, dtype=torch.float32, device="cuda")
    cs = torch.full((5,), 7.0, device="cuda")
    fx.fx_c2_colsum(X, X, X, cs, (0, 5), None)
    rs = torch.full((4,), 7.0, device="cuda")
    fx.fx_c2_rowsum(X, X, X, rs, (4, 0), None)
    s = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    fx.fx_accu_xy(X, X, s, None)
    torch.cuda.synchronize()
    assert (cs == 0).all().item() and (rs == 0).all().item() and s.item() == 0.0


# Arguments naming one buffer several times: the kernels read each distinct
# (address, type) once and reuse it for every leaf naming it.
ALIASES = {"x_y_w": (0, 1, 2), "y_is_x": (0, 0, 1), "w_is_x": (0, 1, 0), "w_is_y": (0, 1, 1),
           "all_x": (0, 0, 0)}


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f64"])
@pytest.mark.parametrize("alias", list(ALIASES))
def test_c2_repeated_buffers(dtype, alias):
    torch, fx = need_gpu()
    shape = (257, 129)
    n = shape[0] * shape[1]
    host, dev = inputs(12, n, dtype)
    pick = ALIASES[alias]
    hx, dx = [host[q] for q in pick], [dev[q] for q in pick]
    e = oracle.EXPRS["c2_z"]
    Z = empty(n, dtype)
    fx.fx_c2_z(*dx, Z, shape)
    acc = "f64" if dtype == "f64" else "f32"
    cs = empty(shape[1], acc)
    fx.fx_c2_colsum(*dx, cs, shape, fx.workspace(fx.R_COLSUM, fx.dtype_code(dx[0]), shape))
    nrm = torch.zeros(1, dtype=torch.float64, device="cuda")
    fx.fx_norm_fro_diff(dx[0], dx[1], nrm, shape, fx.workspace(fx.R_NORM, fx.dtype_code(dx[0]), shape))
    torch.cuda.synchronize()
    out = dtype if dtype == "bf16" else None
    v, mu = oracle.evaluate(e, hx, dtype, shape=shape)
    assert_close(from_dev(Z, dtype), v, mu, dtype, "c2_z %s" % alias, out_dtype=out)
    v, mu = oracle.evaluate(e, hx, dtype, shape=shape, reduce="colsum")
    assert_close(from_dev(cs, acc), v, mu, dtype, "c2 colsum %s" % alias)
    v, mu = oracle.evaluate(oracle.EXPRS["diff"], hx[:2], dtype, shape=shape, reduce="norm")
    assert_close(nrm.cpu().numpy(), v, mu, dtype, "norm %s" % alias)
    if pick[0] == pick[1]:
        assert nrm.item() == 0.0   # X - X is exactly zero
