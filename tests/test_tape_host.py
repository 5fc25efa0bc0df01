"""CPU tests of the run-time tape compiler (no kernels are launched)."""
import pytest

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
    info = fx.Tape(nodes).info()
    assert info["n_inputs"] == 3 and info["depth"] == 2
    assert info["n_instructions"] == 3          # the constant is an immediate
    assert info["op_count"][:4] == [1, 0, 2, 0] and info["n_consts"] == 1
    assert info["n_slots"] <= 5


def test_constant_and_leaf_trees(fx):
    assert fx.Tape([("const", -1, -1, -1, 3.0)]).info()["n_instructions"] == 1
    leaf = fx.Tape([("leaf", -1, -1, 0, 0)]).info()
    assert leaf["n_instructions"] == 0 and leaf["n_inputs"] == 1
    two = fx.Tape([("const", -1, -1, -1, 1.0), ("const", -1, -1, -1, 2.0),
                   ("add", 0, 1, -1, 0)]).info()
    assert two["n_instructions"] == 2           # one immediate materialised


def test_dag_shared_node(fx):
    # t = X + Y used twice: (t % t) - t
    nodes = [("leaf", -1, -1, 0, 0), ("leaf", -1, -1, 1, 0), ("add", 0, 1, -1, 0),
             ("mul", 2, 2, -1, 0), ("sub", 3, 2, -1, 0)]
    info = fx.Tape(nodes).info()
    assert info["n_instructions"] == 3 and info["op_count"][:3] == [1, 1, 1]


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
