"""GPU parity of run-time tapes (random trees) against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import (assert_close, empty, from_dev, need_gpu, oracle_expr, to_dev,
                      tree_inputs)
from synth import trees

pytestmark = pytest.mark.gpu

FP = ["f32", "f64", "bf16", "f16"]
ACC = {"f32": "f32", "bf16": "f32", "f16": "f32", "f64": "f64"}


def _run(fx, torch, nodes, k, seed, e, dtype, shape, kind, cfg=None):
    n = shape[0] * shape[1]
    host, dev = tree_inputs(seed, e, k, n, dtype)
    tape = fx.Tape(nodes)
    dcode = {"f32": fx.F32, "f64": fx.F64, "bf16": fx.BF16, "f16": fx.F16}[dtype]
    red = {0: None, fx.R_ACCU: "accu", fx.R_NORM: "norm", fx.R_COLSUM: "colsum",
           fx.R_ROWSUM: "rowsum"}[kind]
    if kind == 0:
        out, od = empty(n, dtype), dtype
    elif kind in (fx.R_ACCU, fx.R_NORM):
        out, od = torch.zeros(1, dtype=torch.float64, device="cuda"), "f64"
    else:
        out, od = empty(shape[1] if kind == fx.R_COLSUM else shape[0], ACC[dtype]), ACC[dtype]
    ws = fx.workspace(kind, dcode, shape, cfg) if kind else None
    fx.fx_tape_eval(tape, dev, out, shape, kind, ws, cfg=cfg, dt=dcode)
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle_expr(nodes), host, dtype, shape=shape, reduce=red)
    out_half = dtype if (kind == 0 and dtype in ("bf16", "f16")) else None
    return assert_close(from_dev(out, od), v, mu, dtype,
                        "tape seed %d tree %d %s kind %d %s" % (seed, e, dtype, kind, shape),
                        out_dtype=out_half)


@pytest.mark.parametrize("dtype", FP)
@pytest.mark.parametrize("e", range(0, 48, 3))
def test_random_trees_elementwise(dtype, e):
    torch, fx = need_gpu()
    nodes, k, _ = trees.random_tree(4, e)
    _run(fx, torch, nodes, k, 4, e, dtype, (20000 + 7 * e, 1), 0)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f64"])
@pytest.mark.parametrize("e", range(1, 48, 4))
def test_random_trees_accu_and_norm(dtype, e):
    torch, fx = need_gpu()
    nodes, k, _ = trees.random_tree(4, e)
    _run(fx, torch, nodes, k, 4, e, dtype, (50000 + e, 1), fx.R_ACCU)
    _run(fx, torch, nodes, k, 4, e, dtype, (250, 201), fx.R_NORM)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("e", range(2, 40, 5))
def test_random_trees_dim_sums(dtype, e):
    torch, fx = need_gpu()
    nodes, k, _ = trees.random_tree(5, e, depth=(2, 8))
    _run(fx, torch, nodes, k, 5, e, dtype, (1024, 77), fx.R_COLSUM)
    _run(fx, torch, nodes, k, 5, e, dtype, (1000, 65), fx.R_ROWSUM)
    _run(fx, torch, nodes, k, 5, e, dtype, (7, 300), fx.R_COLSUM)   # thin columns


@pytest.mark.parametrize("cfg", [(64, 1, 4, 0), (128, 2, 16, 0), (256, 1, 16, 5),
                                 (512, 2, 16, 0), (256, 1, 2, 0), (256, 4, 16, 0),
                                 (128, 4, 8, 0), (64, 2, 8, 7), (512, 4, 4, 0)])
def test_tape_configs(cfg):
    torch, fx = need_gpu()
    nodes, k, _ = trees.random_tree(5, 11, depth=(6, 8))
    for dtype in ("f32", "bf16"):
        if cfg[2] == 2 and dtype == "f32":
            continue
        if cfg[2] == 4 and dtype == "bf16":
            with pytest.raises(fx.FxError):
                _run(fx, torch, nodes, k, 5, 11, dtype, (3 * 4096 + 5, 1), 0, cfg)
            continue
        _run(fx, torch, nodes, k, 5, 11, dtype, (3 * 4096 + 5, 1), 0, cfg)
        _run(fx, torch, nodes, k, 5, 11, dtype, (3 * 4096 + 5, 1), fx.R_ACCU, cfg)
        if cfg[2] in (8, 16) and cfg[1] == 4:   # the widths only tapes are compiled for
            _run(fx, torch, nodes, k, 5, 11, dtype, (1024, 77), fx.R_COLSUM, cfg[:3] + (0,))
            _run(fx, torch, nodes, k, 5, 11, dtype, (1000, 64), fx.R_ROWSUM, cfg[:3] + (0,))
            _run(fx, torch, nodes, k, 5, 11, dtype, (4096, 20), fx.R_NORM, cfg)


def test_tape_ept_cap():
    # tapes are compiled for EPT 1, 2 and 4; an explicit EPT 8 is refused
    torch, fx = need_gpu()
    nodes, k, _ = trees.random_tree(4, 3)
    with pytest.raises(fx.FxError) as ei:
        _run(fx, torch, nodes, k, 4, 3, "f32", (4096, 1), 0, (256, 8, 16, 0))
    assert ei.value.code == 6


def test_tape_matches_fused_c2():
    """The C2 expression as a tape: same oracle rule, and close to the fused
    kernel (they may differ only by contraction)."""
    torch, fx = need_gpu()
    X, Y, W = 0, 1, 2
    nodes = [("leaf", -1, -1, X, 0), ("leaf", -1, -1, Y, 0), ("add", 0, 1, -1, 0),
             ("leaf", -1, -1, W, 0), ("abs", 3, -1, -1, 0), ("neg", 4, -1, -1, 0),
             ("exp", 5, -1, -1, 0), ("mul", 2, 6, -1, 0), ("const", -1, -1, -1, 1.0),
             ("mul", 0, 0, -1, 0), ("add", 8, 9, -1, 0), ("div", 7, 10, -1, 0)]
    shape = (1024, 300)
    _run(fx, torch, nodes, 3, 2, 0, "f32", shape, 0)
    _run(fx, torch, nodes, 3, 2, 0, "f64", shape, fx.R_COLSUM)


def test_constant_tree():
    torch, fx = need_gpu()
    nodes = [("const", -1, -1, -1, 2.0), ("const", -1, -1, -1, 0.5), ("div", 0, 1, -1, 0)]
    tape = fx.Tape(nodes)
    out = empty(1000, "f32")
    fx.fx_tape_eval(tape, [], out, (1000, 1), 0, dt=fx.F32)
    s = torch.zeros(1, dtype=torch.float64, device="cuda")
    fx.fx_tape_eval(tape, [], s, (1000, 1), fx.R_ACCU, fx.workspace(fx.R_ACCU, fx.F32, (1000, 1)),
                    dt=fx.F32)
    torch.cuda.synchronize()
    assert (out == 4.0).all().item() and s.item() == 4000.0


def _balanced(depth, k=4):
    """A full binary tree over exp(leaf) with the four operators in turn:
    every operand needs code, so the program needs depth + 4 slots."""
    nodes, level = [], []
    for i in range(2 ** depth):
        nodes.append(("leaf", -1, -1, i % k, 0.0))
        nodes.append(("exp", len(nodes) - 1, -1, -1, 0.0))
        level.append(len(nodes) - 1)
    ops, j = ("add", "sub", "mul", "div"), 0
    while len(level) > 1:
        nxt = []
        for a, b in zip(level[::2], level[1::2]):
            nodes.append((ops[j % 4], a, b, -1, 0.0))
            j += 1
            nxt.append(len(nodes) - 1)
        level = nxt
    return nodes


@pytest.mark.parametrize("dtype", ["f32", "f64", "bf16"])
def test_sixteen_slot_programs(dtype):
    """A program needing more than 8 slots runs on the 16-slot file."""
    torch, fx = need_gpu()
    nodes = _balanced(5)
    assert fx.Tape(nodes).info()["n_slots"] > 8
    _run(fx, torch, nodes, 4, 9, 0, dtype, (33333, 1), 0)
    _run(fx, torch, nodes, 4, 9, 0, dtype, (40001, 1), fx.R_ACCU)
    _run(fx, torch, nodes, 4, 9, 0, dtype, (129, 131), fx.R_COLSUM)


@pytest.mark.parametrize("kind", [0, 2])
def test_native_autotune(kind, tmp_path):
    # the exhaustive search returns a configuration of the grid, and the
    # tape run under it matches the oracle
    torch, fx = need_gpu()
    from paper_2604_22242_amd.model import C2_NODES
    shape = (4096, 96)
    n = shape[0] * shape[1]
    host, dev = tree_inputs(7, 1, 3, n, "f32")
    tape = fx.Tape(C2_NODES)
    out = empty(n if kind == 0 else shape[1], "f32")
    ws = torch.zeros(64 << 20, dtype=torch.uint8, device="cuda") if kind else None
    db = tmp_path / "tune.jsonl"
    best, ms = fx.fx_autotune(tape, dev, out, shape, kind, ws, warmup=1, reps=3, db=db)
    grid = fx.fx_tune_grid(kind, fx.F32)
    assert best in grid[:-1] and ms > 0
    # the appended database line names the same argmin, with the tape's
    # features, and the trainer reads it
    import json
    from paper_2604_22242_amd.model import dataset
    from paper_2604_22242_amd.tune import load_db, record_grid
    (rec,) = load_db(str(db)).values()
    assert rec["mode"] == "native" and rec["reduce"] == (None if kind == 0 else "colsum")
    assert rec["shape"] == list(shape) and len(rec["ms"]) == len(grid)
    assert grid[rec["best"]] == best and abs(rec["best_ms"] - ms) <= 1e-6 * ms
    assert rec["ms"][rec["best"]] == min(x for x in rec["ms"][:-1] if x is not None)
    assert rec["features"] == [float("%.4g" % f) for f in
                               fx.fx_tape_features(tape, fx.F32, shape, kind)]
    assert record_grid(rec)[rec["best"]][0] == best
    X, Y = dataset([rec])
    assert X.shape == (1, 25) and Y.shape == (1, 4)
    json.loads(db.read_text().splitlines()[0])
    ws2 = fx.workspace(kind, fx.F32, shape, best) if kind else None
    fx.fx_tape_eval(tape, dev, out, shape, kind, ws2, cfg=best)
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle_expr(C2_NODES), host, "f32", shape=shape,
                            reduce=None if kind == 0 else "colsum")
    assert_close(from_dev(out, "f32"), v, mu, "f32", "autotuned %s" % (best,))


@pytest.mark.parametrize("red", [None, "accu", "colsum", "rowsum", "norm"])
def test_attached_model_chooses_the_launch(red):
    # a tape with the shipped model attached runs, where the caller leaves the
    # launch to the library, exactly the model's pick for each shape (bit for
    # bit the same result as passing that pick), falls back to the defaults
    # when the caller's workspace only covers those, and matches the oracle
    torch, fx = need_gpu()
    import os
    kind = {None: 0, "accu": fx.R_ACCU, "colsum": fx.R_COLSUM, "rowsum": fx.R_ROWSUM,
            "norm": fx.R_NORM}[red]
    nodes, k, _ = trees.random_tree(5, 17, depth=(4, 7))
    model = fx.fx_model_load(os.path.join(os.path.dirname(fx.LIB_PATH), "launch_model.fxm"))
    attached, plain = fx.Tape(nodes), fx.Tape(nodes)
    attached.set_model(model)
    od = "f32" if kind in (0, fx.R_COLSUM, fx.R_ROWSUM) else "f64"
    for shape in [(3000, 257), (1000, 99)]:  # a new shape replaces the cached pick
        n = shape[0] * shape[1]
        host, dev = tree_inputs(5, 17, k, n, "f32")

        def out_buf():
            if kind in (fx.R_ACCU, fx.R_NORM):
                return torch.zeros(1, dtype=torch.float64, device="cuda")
            return empty({0: n, fx.R_COLSUM: shape[1], fx.R_ROWSUM: shape[0]}[kind], "f32")

        pick = model.predict(fx.fx_tape_features(plain, fx.F32, shape, kind), kind, fx.F32)
        ws_pick = fx.workspace(kind, fx.F32, shape, pick) if kind else None
        a, b = out_buf(), out_buf()
        fx.fx_tape_eval(attached, dev, a, shape, kind, ws_pick)
        fx.fx_tape_eval(plain, dev, b, shape, kind, ws_pick, cfg=pick)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (shape, pick)
        v, mu = oracle.evaluate(oracle_expr(nodes), host, "f32", shape=shape, reduce=red)
        assert_close(from_dev(a, od), v, mu, "f32", "model pick %s %s" % (pick, shape))
        if kind:
            need_pick = fx.fx_workspace_bytes(kind, fx.F32, shape, pick)
            need_def = fx.fx_workspace_bytes(kind, fx.F32, shape, None)
            ws_def = fx.workspace(kind, fx.F32, shape, None)
            c, d = out_buf(), out_buf()
            fx.fx_tape_eval(attached, dev, c, shape, kind, ws_def)
            fx.fx_tape_eval(plain, dev, d, shape, kind, ws_def,
                            cfg=pick if need_pick <= need_def else None)
            torch.cuda.synchronize()
            assert torch.equal(c, d), (shape, pick, need_pick, need_def)
    attached.set_model(None)  # detached: the defaults again
    a, b = out_buf(), out_buf()
    ws_def = fx.workspace(kind, fx.F32, shape, None) if kind else None
    fx.fx_tape_eval(attached, dev, a, shape, kind, ws_def)
    fx.fx_tape_eval(plain, dev, b, shape, kind, ws_def)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
