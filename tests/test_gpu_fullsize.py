"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (the library defaults): the matrix workload at 8192 x 8192
(FP32 and FP64, every output compared), and the precision workload at 2^28
elements in BF16 and FP16 storage with uniform and heavy-tailed inputs
(element-wise outputs on sampled windows, sums in full).  Errors against the
FP64 oracle are printed per result."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_close, empty, from_dev, need_gpu, to_dev

pytestmark = pytest.mark.gpu

ROWS = COLS = 8192


def _report(name, rep):
    print("%-34s n=%-9d max_rel=%.3e err/allowed=%.3f needed_mu_branch=%d" % (
        name, rep["n"], rep["max_rel"], rep["max_err_over_allowed"], rep["needed_mu_branch"]),
        flush=True)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_matrix_workload_full(dtype):
    torch, fx = need_gpu()
    n = ROWS * COLS
    shape = (ROWS, COLS)
    host = [synth.fill(2, t, n, dtype) for t in range(3)]
    X, Y, W = [to_dev(h, dtype) for h in host]
    d = fx.dtype_code(X)
    Z = empty(n, dtype)
    cs = empty(COLS, dtype)
    nrm = torch.zeros(1, dtype=torch.float64, device="cuda")
    fx.fx_c2_z(X, Y, W, Z, shape)
    fx.fx_c2_colsum(X, Y, W, cs, shape, fx.workspace(fx.R_COLSUM, d, shape))
    fx.fx_norm_fro_diff(X, Y, nrm, shape, fx.workspace(fx.R_NORM, d, shape))
    torch.cuda.synchronize()
    e = oracle.EXPRS["c2_z"]
    v, mu = oracle.evaluate(e, host, dtype, shape=shape)
    _report("c2 Z %s" % dtype, assert_close(from_dev(Z, dtype), v, mu, dtype, "c2 Z"))
    del v, mu, Z
    v, mu = oracle.evaluate(e, host, dtype, shape=shape, reduce="colsum")
    _report("c2 sum(Z,0) %s" % dtype, assert_close(from_dev(cs, dtype), v, mu, dtype, "colsum"))
    v, mu = oracle.evaluate(oracle.EXPRS["diff"], host[:2], dtype, shape=shape, reduce="norm")
    _report("norm_fro(X-Y) %s" % dtype, assert_close(nrm.cpu().numpy(), v, mu, dtype, "norm"))


def test_matrix_workload_row_sums_full():
    torch, fx = need_gpu()
    n = ROWS * COLS
    shape = (ROWS, COLS)
    host = [synth.fill(2, t, n, "f32") for t in range(3)]
    X, Y, W = [to_dev(h, "f32") for h in host]
    rs = empty(ROWS, "f32")
    fx.fx_c2_rowsum(X, Y, W, rs, shape, fx.workspace(fx.R_ROWSUM, fx.F32, shape))
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.EXPRS["c2_z"], host, "f32", shape=shape, reduce="rowsum")
    _report("c2 sum(Z,1) f32", assert_close(from_dev(rs, "f32"), v, mu, "f32", "rowsum"))


M = 1 << 28
SIDE = 1 << 14
WINDOWS = 24
WIN = 4096


def _windows():
    starts = np.linspace(0, M - WIN, WINDOWS).astype(np.int64)
    starts = np.concatenate([starts, [M - WIN]])
    return [(int(s), int(s) + WIN) for s in starts]


@pytest.mark.parametrize("dist", ["uniform", "lognormal"])
@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_precision_workload_2_28(dtype, dist):
    torch, fx = need_gpu()
    param = 3.0 if dist == "lognormal" else 0.0
    host, sats = [], 0
    for t in range(3):
        h, s = synth.fill(3, t, M, dtype, dist, param, return_saturations=True)
        host.append(h)
        sats += s
    print("inputs %s %s: %d FP16 saturations" % (dtype, dist, sats), flush=True)
    X, Y, W = [to_dev(h, dtype) for h in host]
    d = fx.dtype_code(X)
    Z = empty(M, dtype)
    fx.fx_c1_z(X, Y, W, Z)
    s = torch.zeros(1, dtype=torch.float64, device="cuda")
    fx.fx_accu_xy(X, Y, s, fx.workspace(fx.R_ACCU, d, (M, 1)))
    nrm = torch.zeros(1, dtype=torch.float64, device="cuda")
    fx.fx_norm_fro_diff(X, Y, nrm, (SIDE, SIDE), fx.workspace(fx.R_NORM, d, (SIDE, SIDE)))
    cs = empty(SIDE, "f32")
    fx.fx_colsum_xy(X, Y, cs, (SIDE, SIDE), fx.workspace(fx.R_COLSUM, d, (SIDE, SIDE)))
    torch.cuda.synchronize()
    # element-wise output on sampled windows
    z = Z.cpu()
    got, val, mus = [], [], []
    for a, b in _windows():
        v, mu = oracle.evaluate(oracle.EXPRS["c1_z"], [h[a:b] for h in host], dtype)
        got.append(from_dev(z[a:b], dtype))
        val.append(v)
        mus.append(mu)
    _report("C1 Z %s %s (windows)" % (dtype, dist),
            assert_close(np.concatenate(got), np.concatenate(val), np.concatenate(mus), dtype,
                         "Z windows", out_dtype=dtype))
    v, mu = oracle.evaluate(oracle.EXPRS["xy"], host[:2], dtype, reduce="accu")
    _report("accu(X%%Y) %s %s" % (dtype, dist), assert_close(s.cpu().numpy(), v, mu, dtype, "accu"))
    v, mu = oracle.evaluate(oracle.EXPRS["diff"], host[:2], dtype, shape=(SIDE, SIDE), reduce="norm")
    _report("norm_fro(X-Y) %s %s" % (dtype, dist),
            assert_close(nrm.cpu().numpy(), v, mu, dtype, "norm"))
    v, mu = oracle.evaluate(oracle.EXPRS["xy"], host[:2], dtype, shape=(SIDE, SIDE),
                            reduce="colsum")
    _report("sum(X%%Y,0) %s %s" % (dtype, dist),
            assert_close(from_dev(cs, "f32"), v, mu, dtype, "colsum"))
    if dist == "uniform":
        # error against the unrounded FP64 draws, which adds storage quantisation
        raw = [synth.fill_f64(3, t, M) for t in range(2)]
        exact = float(np.dot(raw[0], raw[1]))
        print("accu(X%%Y) %s vs pre-storage draws: rel %.3e" % (
            dtype, abs(s.item() - exact) / abs(exact)), flush=True)


def test_beyond_2_31_elements():
    """The largest size class: n = 2^31 + 37 FP32 elements (8.6 GB per
    array), past every 32-bit index.  Z = X % Y + 2 W and accu(X % W) with
    X = Y = 1 through the compiled kernels, a tape and a run-time generated
    kernel: Z on windows at the start, the middle and the end (across element
    2^31) against the oracle, the sums against the oracle over all n elements, and accu(X % Y)
    = n exactly."""
    torch, fx = need_gpu()
    n = (1 << 31) + 37
    print("n = %d" % n, flush=True)
    w = synth.fill(7, 2, n, "f32")
    W = torch.from_numpy(w).cuda()
    ones = torch.ones(n, dtype=torch.float32, device="cuda")
    Z = torch.empty(n, dtype=torch.float32, device="cuda")
    ws = fx.workspace(fx.R_ACCU, fx.F32, (n, 1))
    s_ones = torch.zeros(1, dtype=torch.float64, device="cuda")
    fx.fx_accu_xy(ones, ones, s_ones, ws)
    s_w = torch.zeros(1, dtype=torch.float64, device="cuda")
    fx.fx_accu_xy(ones, W, s_w, ws)
    torch.cuda.synchronize()
    assert s_ones.item() == n
    # the first elements, the middle, and the last 4096 (which cross element 2^31)
    wins = [(0, 4096), ((1 << 30) - 2048, (1 << 30) + 2048), (n - 4096, n)]
    assert wins[-1][0] < (1 << 31) < wins[-1][1]

    def check_windows(what):
        torch.cuda.synchronize()
        for a, b in wins:
            one = np.ones(b - a, np.float32)
            v, mu = oracle.evaluate(oracle.EXPRS["c1_z"], [one, one, w[a:b]], "f32")
            assert_close(Z[a:b].cpu().numpy().astype(np.float64), v, mu, "f32",
                         "%s Z[%d:%d]" % (what, a, b))
        Z.fill_(float("nan"))

    fx.fx_c1_z(ones, ones, W, Z)
    check_windows("compiled")
    nodes = [("leaf", -1, -1, 0, 0.0), ("leaf", -1, -1, 1, 0.0), ("mul", 0, 1, -1, 0.0),
             ("leaf", -1, -1, 2, 0.0), ("const", -1, -1, -1, 2.0), ("mul", 4, 3, -1, 0.0),
             ("add", 2, 5, -1, 0.0)]
    fx.fx_tape_eval(fx.Tape(nodes), [ones, ones, W], Z, (n, 1))
    check_windows("tape")
    fx.Rtc(nodes, fx.F32).eval([ones, ones, W], Z, (n, 1))
    check_windows("run-time source")
    xw = [("leaf", -1, -1, 0, 0.0), ("leaf", -1, -1, 1, 0.0), ("mul", 0, 1, -1, 0.0)]
    s_tape = torch.zeros(1, dtype=torch.float64, device="cuda")
    fx.fx_tape_eval(fx.Tape(xw), [ones, W], s_tape, (n, 1), fx.R_ACCU, ws)
    s_rtc = torch.zeros(1, dtype=torch.float64, device="cuda")
    fx.Rtc(xw, fx.F32, fx.R_ACCU).eval([ones, W], s_rtc, (n, 1), ws)
    torch.cuda.synchronize()
    del Z, W, ones
    torch.cuda.empty_cache()
    v, mu = oracle.evaluate(oracle.EXPRS["xy"], [np.ones(n, np.float32), w], "f32", reduce="accu")
    for what, s in (("compiled", s_w), ("tape", s_tape), ("run-time source", s_rtc)):
        _report("accu(1 %% W) n=2^31+37 %s" % what,
                assert_close(s.cpu().numpy(), v, mu, "f32", "%s accu beyond 2^31" % what))
