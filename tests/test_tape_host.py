"""CPU tests of the run-time tape compiler (no kernels are launched)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import oracle_expr
from synth import trees


@pytest.fixture(scope="module")
def fx():
    import os
    import paper_2604_22242_amd as fx
    if not os.path.exists(fx.LIB_PATH):
        from paper_2604_22242_amd import build
        build.build()
    return fx


def test_compile_simple(fx):
    # X % Y + 2*W : leaves, a constant, three operators
    nodes = [("leaf", -1, -1, 0, 0), ("leaf", -1, -1, 1, 0), ("mul", 0, 1, -1, 0),
             ("const", -1, -1, -1, 2.0), ("leaf", -1, -1, 2, 0), ("mul", 3, 4, -1, 0),
             ("add", 2, 5, -1, 0)]
    t = fx.Tape(nodes)
    info = t.info()
    assert info["n_inputs"] == 3 and info["depth"] == 2
    assert info["op_count"][:4] == [1, 0, 2, 0] and info["n_consts"] == 1
    # X % Y into the accumulator, kept in slot 3 while 2 * W is computed
    # (the constant is an immediate), then the sum
    # (the loads fold into their consumers: ST 3 + LD 2 is one STLD)
    assert t.program() == [("MUL_S|ld", 1, 0, 0.0), ("STLD", 3, 2, 0.0), ("MUL_I", 0, 0, 2.0),
                           ("ADD_S", 3, 0, 0.0)]
    assert info["n_instructions"] == 4 and info["n_slots"] == 4


def test_constant_and_leaf_trees(fx):
    assert fx.Tape([("const", -1, -1, -1, 3.0)]).program() == [("LDI", 0, 0, 3.0)]
    leaf = fx.Tape([("leaf", -1, -1, 0, 0)])
    assert leaf.program() == [("LD", 0, 0, 0.0)] and leaf.info()["n_inputs"] == 1
    two = fx.Tape([("const", -1, -1, -1, 1.0), ("const", -1, -1, -1, 2.0),
                   ("sub", 0, 1, -1, 0)])
    assert two.program() == [("LDI", 0, 0, 1.0), ("SUB_I", 0, 0, 2.0)]
    # an immediate on the left of a slot: the reversed form keeps the order
    rev = fx.Tape([("const", -1, -1, -1, 1.0), ("leaf", -1, -1, 0, 0), ("div", 0, 1, -1, 0)])
    assert rev.program() == [("RDIV_I|ld", 0, 0, 1.0)]


def test_abs_and_neg_fold_into_the_consumer(fx):
    X = ("leaf", -1, -1, 0, 0.0)
    # the generator's guards: sqrt(|x|), exp(0 - |x|), x / (1 + |y|)
    t = fx.Tape([X, ("abs", 0, -1, -1, 0), ("sqrt", 1, -1, -1, 0)])
    assert t.program() == [("SQRT|ld|abs", 0, 0, 0.0)]
    t = fx.Tape([X, ("const", -1, -1, -1, 0.0), ("abs", 0, -1, -1, 0), ("sub", 1, 2, -1, 0),
                 ("exp", 3, -1, -1, 0)])
    assert t.program() == [("RSUB_I|ld|abs", 0, 0, 0.0), ("EXP", 0, 0, 0.0)]
    t = fx.Tape([X, ("leaf", -1, -1, 1, 0.0), ("const", -1, -1, -1, 1.0), ("abs", 1, -1, -1, 0),
                 ("add", 2, 3, -1, 0), ("div", 0, 4, -1, 0)])
    assert t.program() == [("ADD_I|ld|abs", 0, 1, 1.0), ("RDIV_S", 0, 0, 0.0)]
    # compositions: -(-x) vanishes, -|x| keeps both, |-x| is |x|; a root
    # modifier becomes an instruction of its own
    nn = fx.Tape([X, ("neg", 0, -1, -1, 0), ("neg", 1, -1, -1, 0), ("exp", 2, -1, -1, 0)])
    assert nn.program() == [("EXP|ld", 0, 0, 0.0)]
    na = fx.Tape([X, ("abs", 0, -1, -1, 0), ("neg", 1, -1, -1, 0), ("exp", 2, -1, -1, 0)])
    assert na.program() == [("EXP|ld|abs|neg", 0, 0, 0.0)]
    an = fx.Tape([X, ("neg", 0, -1, -1, 0), ("abs", 1, -1, -1, 0), ("exp", 2, -1, -1, 0)])
    assert an.program() == [("EXP|ld|abs", 0, 0, 0.0)]
    root = fx.Tape([X, ("exp", 0, -1, -1, 0), ("abs", 1, -1, -1, 0), ("neg", 2, -1, -1, 0)])
    assert root.program() == [("EXP|ld", 0, 0, 0.0), ("ABS", 0, 0, 0.0), ("NEG", 0, 0, 0.0)]
    # a shared abs node is stored with its modifier applied
    sh = fx.Tape([X, ("exp", 0, -1, -1, 0), ("abs", 1, -1, -1, 0), ("mul", 2, 2, -1, 0)])
    assert sh.program() == [("EXP|ld", 0, 0, 0.0), ("ST|abs", 1, 0, 0.0), ("MUL_S", 1, 0, 0.0)]


def test_dag_shared_node(fx):
    # t = X + Y used twice: (t % t) - t
    nodes = [("leaf", -1, -1, 0, 0), ("leaf", -1, -1, 1, 0), ("add", 0, 1, -1, 0),
             ("mul", 2, 2, -1, 0), ("sub", 3, 2, -1, 0)]
    t = fx.Tape(nodes)
    assert t.info()["op_count"][:3] == [1, 1, 1]
    # t is computed once and kept in a slot for its later uses
    assert t.program() == [("ADD_S|ld", 1, 0, 0.0), ("ST", 2, 0, 0.0), ("MUL_S", 2, 0, 0.0),
                           ("SUB_S", 2, 0, 0.0)]


@pytest.mark.parametrize("bad", [
    [("add", 0, 1, -1, 0)],                                       # operands not earlier
    [("leaf", -1, -1, 0, 0), ("exp", 1, -1, -1, 0)],              # self reference
    [("leaf", -1, -1, 0, 0), (99, 0, -1, -1, 0)],                 # unknown operator
])
def test_malformed_trees(fx, bad):
    with pytest.raises(fx.FxError) as e:
        fx.Tape(bad)
    assert e.value.code == 1


def test_limits(fx):
    with pytest.raises(fx.FxError) as e:     # a fifth input
        fx.Tape([("leaf", -1, -1, 4, 0)])
    assert e.value.code == 6
    # a balanced tree needing more than 16 live slots
    nodes, level = [], []
    for i in range(2 ** 17 // 2 ** 12):
        nodes.append(("leaf", -1, -1, i % 4, 0))
        level.append(len(nodes) - 1)
    while len(level) > 1:
        nxt = []
        for a, b in zip(level[::2], level[1::2]):
            nodes.append(("exp", a, -1, -1, 0))
            nodes.append(("add", len(nodes) - 1, b, -1, 0))
            nxt.append(len(nodes) - 1)
        level = nxt
    info = fx.Tape(nodes).info()                  # 32 leaves: fits
    assert info["n_slots"] <= 16


def test_generated_trees_compile(fx):
    for i in range(300):
        nodes, k, D = trees.random_tree(4, i)
        info = fx.Tape(nodes).info()
        assert info["n_inputs"] == k
        assert info["depth"] == trees.depth_of(nodes) >= D
    for i in range(200):                          # the deeper launch-config set
        nodes, k, D = trees.random_tree(5, i, depth=(2, 8))
        fx.Tape(nodes)


def test_tree_generator_is_deterministic():
    a = trees.random_tree(4, 17)
    b = trees.random_tree(4, 17)
    assert a == b and trees.random_tree(4, 18) != a
    s = trees.batch_set(64)
    assert all(256 <= t["n"] <= 1 << 20 for t in s)
    assert sum(1 for t in s if t["reduce"] == "accu") == 32


def run_program(prog, inputs):
    """Execute an accumulator program in FP64 with numpy (the machine that
    fx_tape_program documents)."""
    slots = [None] * 16
    for q, x in enumerate(inputs):
        slots[q] = x.astype(np.float64)
    acc = None
    for name, s, s2, k in prog:
        op, *mods = name.split("|")
        if "ld" in mods:
            acc = slots[s2].copy()
        if "abs" in mods:
            acc = np.abs(acc)
        if "neg" in mods:
            acc = -acc
        y = slots[s] if op.endswith("_S") or op == "LD" else k
        if op == "LD":
            acc = slots[s].copy()
        elif op == "LDI":
            acc = np.full(inputs[0].shape if inputs else (1,), k)
        elif op == "ST":
            slots[s] = acc.copy()
        elif op == "STLD":
            slots[s] = acc.copy()
            acc = slots[s2].copy()
        elif op.startswith("ADD"):
            acc = acc + y
        elif op.startswith("SUB"):
            acc = acc - y
        elif op.startswith("RSUB"):
            acc = y - acc
        elif op.startswith("MUL"):
            acc = acc * y
        elif op.startswith("DIV"):
            acc = acc / y
        elif op.startswith("RDIV"):
            acc = y / acc
        elif op == "NEG":
            acc = -acc
        elif op == "ABS":
            acc = np.abs(acc)
        elif op == "EXP":
            acc = np.exp(acc)
        else:
            acc = np.sqrt(acc)
    return acc


@pytest.mark.parametrize("which", ["batch", "tuning"])
def test_programs_compute_the_tree(fx, which):
    """Every generated tree's program, run in FP64 on the host, agrees with
    the oracle's node-by-node FP64 evaluation: operand order, reversed forms,
    spills and slot reuse all show up here."""
    n = 257
    for i in range(250):
        if which == "batch":
            nodes, k, _ = trees.random_tree(4, i)
        else:
            nodes = trees.tuning_item(5, i)["nodes"]
            k = max([nd[3] for nd in nodes if nd[0] == "leaf"] + [-1]) + 1
        xs = [synth.fill_f64(11, t, n) for t in range(k)]
        got = run_program(fx.Tape(nodes).program(), xs)
        v, mu = oracle.evaluate(oracle_expr(nodes), xs, "f64") if k else (None, None)
        if k == 0:
            continue
        ok, rep = oracle.check(got, v, mu, "f64")
        assert ok.all(), (which, i, rep)
