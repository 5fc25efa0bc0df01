"""The entry point that allocates nothing: fx_tape_eval_static (reductions
take the library's static device scratch instead of a caller workspace)
against fx_tape_eval with a workspace of its own, through the C ABI: the same
kernels and configuration, so the same bits, and within the oracle's rule.
Two calls in a row, the second smaller, for every result kind."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import assert_close, empty, from_dev, inputs, need_gpu

ACC = {"f32": "f32", "bf16": "f32", "f64": "f64"}
RED = {0: None, 1: "accu", 4: "norm", 2: "colsum", 3: "rowsum"}
C2 = [("leaf", -1, -1, 0, 0.0), ("leaf", -1, -1, 1, 0.0), ("add", 0, 1, -1, 0.0),
      ("leaf", -1, -1, 2, 0.0), ("abs", 3, -1, -1, 0.0), ("neg", 4, -1, -1, 0.0),
      ("exp", 5, -1, -1, 0.0), ("mul", 2, 6, -1, 0.0), ("const", -1, -1, -1, 1.0),
      ("mul", 0, 0, -1, 0.0), ("add", 8, 9, -1, 0.0), ("div", 7, 10, -1, 0.0)]


def _out(torch, kind, shape, dtype):
    if kind == 0:
        return empty(shape[0] * shape[1], dtype), dtype
    if kind in (1, 4):
        return torch.zeros(1, dtype=torch.float64, device="cuda"), "f64"
    return empty(shape[1] if kind == 2 else shape[0], ACC[dtype]), ACC[dtype]


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", ["f32", "bf16", "f64"])
@pytest.mark.parametrize("kind", [0, 1, 4, 2, 3])
def test_static_scratch_matches_the_workspace_entry_point(dtype, kind):
    torch, fx = need_gpu()
    tape = fx.Tape(C2)
    for shape in [(4096, 777), (1000, 33)]:          # the second call is smaller
        n = shape[0] * shape[1]
        host, devs = inputs(21, n, dtype)
        dcode = fx.dtype_code(devs[0])
        out_s, od = _out(torch, kind, shape, dtype)
        out_w, _ = _out(torch, kind, shape, dtype)
        ws = fx.workspace(kind, dcode, shape) if kind else None
        fx.fx_tape_eval_static(tape, devs, out_s, shape, kind)
        fx.fx_tape_eval(tape, devs, out_w, shape, kind, ws)
        torch.cuda.synchronize()
        assert torch.equal(out_s, out_w), (dtype, kind, shape)
        v, mu = oracle.evaluate(oracle.EXPRS["c2_z"], host, dtype, shape=shape, reduce=RED[kind])
        assert_close(from_dev(out_s, od), v, mu, dtype, "static %s %s %s" % (dtype, kind, shape),
                     out_dtype=dtype if kind == 0 and dtype == "bf16" else None)


@pytest.mark.gpu
def test_static_scratch_split_reductions_back_to_back():
    """Split reductions reuse the scratch's counters: 200 in a row, alternating
    sizes, each equal to the workspace entry point's result."""
    torch, fx = need_gpu()
    tape = fx.Tape(C2)
    cases = []
    for shape in [(1 << 20, 1), (4096, 7)]:
        n = shape[0] * shape[1]
        _, devs = inputs(22, n, "f32")
        kind = 1 if shape[1] == 1 else 2
        ref, _ = _out(torch, kind, shape, "f32")
        fx.fx_tape_eval(tape, devs, ref, shape, kind, fx.workspace(kind, fx.F32, shape))
        cases.append((devs, shape, kind, ref))
    outs = []
    for i in range(200):
        devs, shape, kind, _ = cases[i % 2]
        o, _ = _out(torch, kind, shape, "f32")
        fx.fx_tape_eval_static(tape, devs, o, shape, kind)
        outs.append(o)
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        assert torch.equal(o, cases[i % 2][3]), i


def test_static_scratch_refuses_oversized_workspaces():
    """Host-side: a reduction whose workspace exceeds the static scratch is
    refused before anything is enqueued."""
    import paper_2604_22242_amd as fx
    L = fx.lib()
    tape = fx.Tape(C2)
    arr = (ctypes.c_void_p * 3)(0x10000, 0x10000, 0x10000)
    shape = fx.Shape(1 << 20, 1024)
    assert fx.fx_workspace_bytes(fx.R_ROWSUM, fx.F32, (1 << 20, 1024)) > 16 << 20
    assert L.fx_tape_eval_static(tape.handle, fx.F32, arr, 3, shape, fx.R_ROWSUM, 0x10000, None,
                                 None) == 4
    assert "static scratch" in fx.fx_last_error()
