"""GPU tests of the persistent batch: per-expression results equal the
single-tape results (bitwise for element-wise outputs, within the oracle rule
for sums), are independent of the order of the batch, survive HIP-graph
replays, and the full 4096-expression workload matches the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_close, empty, from_dev, need_gpu, oracle_expr, tree_inputs
from synth import trees

pytestmark = pytest.mark.gpu


def _build(fx, torch, tset, dtype, seed):
    """Inputs, outputs and tapes for a list of generated trees."""
    items, host = [], []
    for t in tset:
        h, dev = tree_inputs(seed, t["id"], t["n_inputs"], t["n"], dtype)
        tape = fx.Tape(t["nodes"])
        if t["reduce"]:
            out = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
            kind = fx.R_ACCU
        else:
            out = empty(t["n"], dtype)
            kind = 0
        items.append((tape, dev, out, t["n"], kind))
        host.append(h)
    return items, host


def _single(fx, torch, item, dtype):
    tape, dev, out, n, kind = item
    dc = {"f32": fx.F32, "bf16": fx.BF16, "f64": fx.F64, "f16": fx.F16}[dtype]
    if kind == 0:
        o = torch.empty_like(out)
        fx.fx_tape_eval(tape, dev, o, (n, 1), 0, dt=dc)
    else:
        o = torch.zeros(1, dtype=torch.float64, device="cuda")
        fx.fx_tape_eval(tape, dev, o, (n, 1), fx.R_ACCU, fx.workspace(fx.R_ACCU, dc, (n, 1)), dt=dc)
    return o


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f64"])
def test_batch_matches_single_tapes(dtype):
    torch, fx = need_gpu()
    tset = trees.batch_set(160)
    items, host = _build(fx, torch, tset, dtype, 4)
    dc = {"f32": fx.F32, "bf16": fx.BF16, "f64": fx.F64}[dtype]
    b = fx.Batch(items, dc, tile_elems=4096)
    b.launch()
    torch.cuda.synchronize()
    for t, it, h in zip(tset, items, host):
        single = _single(fx, torch, it, dtype)
        torch.cuda.synchronize()
        if it[4] == 0:
            assert torch.equal(it[2], single), "tree %d differs from its single launch" % t["id"]
            v, mu = oracle.evaluate(oracle_expr(t["nodes"]), h, dtype, shape=(t["n"], 1))
            half = dtype if dtype in ("bf16", "f16") else None
            assert_close(from_dev(it[2], dtype), v, mu, dtype, "batch tree %d" % t["id"], half)
        else:
            v, mu = oracle.evaluate(oracle_expr(t["nodes"]), h, dtype, shape=(t["n"], 1),
                                    reduce="accu")
            assert_close(it[2].cpu().numpy(), v, mu, dtype, "batch accu tree %d" % t["id"])
            assert_close(single.cpu().numpy(), v, mu, dtype, "single accu tree %d" % t["id"])


def test_batch_order_independent():
    torch, fx = need_gpu()
    tset = trees.batch_set(120)
    items, _ = _build(fx, torch, tset, "f32", 4)
    b = fx.Batch(items, fx.F32, tile_elems=2048)
    b.launch()
    torch.cuda.synchronize()
    first = [it[2].clone() for it in items]
    perm = np.random.default_rng(0).permutation(len(items))
    for it in items:
        it[2].fill_(float("nan"))
    b2 = fx.Batch([items[i] for i in perm], fx.F32, tile_elems=2048)
    b2.launch()
    torch.cuda.synchronize()
    for i, it in enumerate(items):
        assert torch.equal(it[2], first[i]), "tree %d changed with the order" % i


def test_batch_graph_replays():
    torch, fx = need_gpu()
    tset = trees.batch_set(96)
    items, host = _build(fx, torch, tset, "f32", 4)
    b = fx.Batch(items, fx.F32)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        b.launch(st)
    st.synchronize()
    ref = [it[2].clone() for it in items]
    for rep in range(4):
        for it in items:                  # eager work between replays
            it[2].fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            b.graph(st)
        st.synchronize()
        for i, it in enumerate(items):
            assert torch.equal(it[2], ref[i]), "replay %d, tree %d" % (rep, i)


def test_batch_edge_items():
    torch, fx = need_gpu()
    const = fx.Tape([("const", -1, -1, -1, 3.0)])
    leaf = fx.Tape([("leaf", -1, -1, 0, 0)])
    x = torch.arange(1, 1001, dtype=torch.float32, device="cuda")
    o1 = empty(1000, "f32")
    o2 = empty(997, "f32")
    s1 = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    s2 = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    s3 = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    z = empty(0, "f32")
    items = [(const, [], o1, 1000, 0), (leaf, [x[3:]], o2, 997, 0), (leaf, [x], s1, 1000, fx.R_ACCU),
             (const, [], s2, 77777, fx.R_ACCU), (leaf, [x], s3, 0, fx.R_ACCU), (leaf, [x], z, 0, 0)]
    b = fx.Batch(items, fx.F32, tile_elems=256)
    assert b.info()["vec_bytes"] == 4     # x[3:] is not 16-byte aligned: element path
    b.launch()
    torch.cuda.synchronize()
    assert (o1 == 3).all().item() and torch.equal(o2, x[3:])
    assert s1.item() == 500500.0 and s2.item() == 3.0 * 77777 and s3.item() == 0.0


def test_batch_full_workload():
    """The 4096-expression workload (sizes 256..2^20, half ending in accu):
    every accu result and every 16th element-wise result against the oracle."""
    torch, fx = need_gpu()
    tset = trees.batch_set(4096)
    items, host = _build(fx, torch, tset, "f32", 4)
    b = fx.Batch(items, fx.F32)
    info = b.info()
    print("batch:", info, trees.summary(tset), flush=True)
    b.graph(torch.cuda.Stream())
    torch.cuda.synchronize()
    worst = 0.0
    for t, it, h in zip(tset, items, host):
        if it[4] == fx.R_ACCU:
            v, mu = oracle.evaluate(oracle_expr(t["nodes"]), h, "f32", shape=(t["n"], 1),
                                    reduce="accu")
            rep = assert_close(it[2].cpu().numpy(), v, mu, "f32", "accu tree %d" % t["id"])
        elif t["id"] % 32 == 0:
            v, mu = oracle.evaluate(oracle_expr(t["nodes"]), h, "f32", shape=(t["n"], 1))
            rep = assert_close(from_dev(it[2], "f32"), v, mu, "f32", "tree %d" % t["id"])
        else:
            continue
        worst = max(worst, rep["max_err_over_allowed"])
    print("batch worst err/allowed %.3f" % worst, flush=True)


def test_batch_with_a_sixteen_slot_program():
    """One item needing more than 8 slots moves the whole batch to the
    16-slot kernel; results still match the single tapes and the oracle."""
    torch, fx = need_gpu()
    from test_gpu_tape import _balanced
    tset = trees.batch_set(24)
    tset.append({"id": 24, "nodes": _balanced(5), "n_inputs": 4, "n": 5000, "reduce": None})
    tset.append({"id": 25, "nodes": _balanced(5), "n_inputs": 4, "n": 7001, "reduce": "accu"})
    items, host = _build(fx, torch, tset, "f32", 6)
    b = fx.Batch(items, fx.F32, tile_elems=2048)
    b.launch()
    torch.cuda.synchronize()
    for t, it, h in zip(tset, items, host):
        red = "accu" if it[4] else None
        v, mu = oracle.evaluate(oracle_expr(t["nodes"]), h, "f32", shape=(t["n"], 1), reduce=red)
        got = it[2].cpu().numpy() if it[4] else from_dev(it[2], "f32")
        assert_close(got, v, mu, "f32", "16-slot batch tree %d" % t["id"])
