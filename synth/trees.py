"""Seeded random expression trees (the batching and launch-config workloads).

A tree is a list of nodes, children first, root last; each node is a tuple
(op, a, b, input, value):
    op     one of "leaf", "const", "add", "sub", "mul", "div", "exp", "abs",
           "sqrt", "neg"
    a, b   indices of earlier nodes (-1 if unused)
    input  input index for "leaf"
    value  the constant for "const"
This module only draws structure; it evaluates nothing.

Recipe.  Draw a target depth D and an input count k.  Grow one branch to
depth D (the "forced" branch, which picks one operand of every binary node
at random); any other operand of an internal node at depth d < D is itself
internal with probability 1/2 (a leaf at d + 1 == D).  Internal operators
are uniform over {+, -, %, /, exp, abs, sqrt}.  A leaf is a constant from
{0.5, 1, 2, 3} with probability 0.1, else an input drawn uniformly from
[0, k); leaves are then relabelled so that the inputs used are exactly
0..k'-1 (k' <= k).  Guards keep values finite on inputs in [-1, 1]:
sqrt(a) -> sqrt(abs(a)), a/b -> a/(1 + abs(b)), exp(a) -> exp(0 - abs(a));
they are ordinary nodes and count in the final depth.

Randomness is counter-based (SplitMix64 draws of stream 2^20 + index under
the given seed), so tree i of a set is the same whatever else is drawn.
"""
from __future__ import annotations

import math

import numpy as np

from . import raw

OPS = ("add", "sub", "mul", "div", "exp", "abs", "sqrt")
CONSTS = (0.5, 1.0, 2.0, 3.0)
UNARY = ("exp", "abs", "sqrt", "neg")
TREE_STREAM = 1 << 20


class Draws:
    """Uniform draws from one counter-based stream."""

    def __init__(self, seed: int, stream: int, block: int = 256):
        self.seed, self.stream, self.k, self.block = seed, stream, 0, block
        self.buf = raw(seed, stream, block, 0)
        self.i = 0

    def u64(self) -> int:
        if self.i == self.block:
            self.k += self.block
            self.buf = raw(self.seed, self.stream, self.block, self.k)
            self.i = 0
        v = int(self.buf[self.i])
        self.i += 1
        return v

    def uniform(self) -> float:          # [0, 1)
        return (self.u64() >> 11) * 2.0 ** -53

    def integer(self, lo: int, hi: int) -> int:   # inclusive
        return lo + int(self.uniform() * (hi - lo + 1))

    def normal(self) -> float:           # Box-Muller
        u1 = ((self.u64() >> 11) + 1) * 2.0 ** -53
        u2 = self.uniform()
        return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


class _Builder:
    def __init__(self):
        self.nodes: list[tuple] = []

    def add(self, op, a=-1, b=-1, inp=-1, val=0.0) -> int:
        self.nodes.append((op, a, b, inp, val))
        return len(self.nodes) - 1

    def const(self, v):
        return self.add("const", val=float(v))

    def guarded(self, op, a, b=-1) -> int:
        if op == "sqrt":
            return self.add("sqrt", self.add("abs", a))
        if op == "div":
            return self.add("div", a, self.add("add", self.const(1.0), self.add("abs", b)))
        if op == "exp":
            return self.add("exp", self.add("sub", self.const(0.0), self.add("abs", a)))
        if op in UNARY:
            return self.add(op, a)
        return self.add(op, a, b)


def random_tree(seed: int, index: int, depth=(2, 6), inputs=(1, 4), p_const=0.1,
                p_internal=0.5):
    """Tree `index` of the set drawn under `seed`.  Returns
    (nodes, n_inputs, target_depth)."""
    r = Draws(seed, TREE_STREAM + index)
    D = r.integer(*depth)
    k = r.integer(*inputs)
    b = _Builder()

    def leaf():
        if r.uniform() < p_const:
            return b.const(CONSTS[r.integer(0, len(CONSTS) - 1)])
        return b.add("leaf", inp=r.integer(0, k - 1))

    def grow(d: int, forced: bool) -> int:
        if d == D or (not forced and r.uniform() >= p_internal):
            return leaf()
        op = OPS[r.integer(0, len(OPS) - 1)]
        if op in UNARY:
            return b.guarded(op, grow(d + 1, forced))
        force_left = r.uniform() < 0.5
        left = grow(d + 1, forced and force_left)
        right = grow(d + 1, forced and not force_left)
        return b.guarded(op, left, right)

    grow(0, True)
    # relabel inputs to 0..k'-1 in order of first use
    used = {}
    nodes = []
    for (op, a, bb, inp, val) in b.nodes:
        if op == "leaf":
            inp = used.setdefault(inp, len(used))
        nodes.append((op, a, bb, inp, val))
    return nodes, len(used), D


def depth_of(nodes) -> int:
    d = [0] * len(nodes)
    for i, (op, a, b, _, _) in enumerate(nodes):
        if a >= 0:
            d[i] = max(d[a] + 1, d[b] + 1 if b >= 0 else 0)
    return d[-1]


def lognormal_size(seed: int, index: int, lo=256, hi=1 << 20, mu=math.log(2 ** 14),
                   sigma=2 * math.log(2)) -> int:
    """n = round(exp(N(mu, sigma^2))), redrawn until it lies in [lo, hi]."""
    r = Draws(seed, TREE_STREAM * 2 + index)
    while True:
        n = int(round(math.exp(mu + sigma * r.normal())))
        if lo <= n <= hi:
            return n


def batch_set(count: int = 4096, seed: int = 4):
    """The batching workload: `count` trees of depth 2..6 over 1..4 inputs,
    lognormal sizes in [256, 2^20]; even ids element-wise, odd ids end in
    accu.  Returns a list of dicts."""
    out = []
    for e in range(count):
        nodes, k, D = random_tree(seed, e, depth=(2, 6))
        out.append({"id": e, "nodes": nodes, "n_inputs": k, "target_depth": D,
                    "n": lognormal_size(seed, e), "reduce": "accu" if e % 2 else None})
    return out


def input_tensor_id(expr: int, q: int) -> int:
    """Tensor id of input q of expression `expr` in a generated set."""
    return 8 * expr + q


def summary(trees) -> dict:
    sizes = np.array([t["n"] for t in trees])
    return {"count": len(trees), "n_min": int(sizes.min()), "n_median": float(np.median(sizes)),
            "n_mean": float(sizes.mean()), "n_max": int(sizes.max()),
            "nodes_max": max(len(t["nodes"]) for t in trees)}


REDUCTIONS = (None, "accu", "colsum", "rowsum", "norm")
REDUCTION_P = (0.40, 0.15, 0.15, 0.15, 0.15)
TUNE_STREAM = 3 * TREE_STREAM


def tuning_item(seed: int, index: int) -> dict:
    """One launch-configuration workload item: a tree of depth 2..8 over 1..4
    inputs; n = round(2^U(12, 28)) rounded up to a multiple of 64; storage
    FP32 or BF16; reduction none / accu / colsum / rowsum / norm with
    probabilities .40/.15/.15/.15/.15; dimension sums view the data as
    n_rows = 2^ceil(log2(n)/2) rows by ceil(n / n_rows) columns."""
    nodes, k, D = random_tree(seed, index, depth=(2, 8))
    r = Draws(seed, TUNE_STREAM + index)
    n = int(round(2.0 ** (12 + 16 * r.uniform())))
    n = (n + 63) // 64 * 64
    dtype = "f32" if r.uniform() < 0.5 else "bf16"
    u, acc, red = r.uniform(), 0.0, None
    for cand, p in zip(REDUCTIONS, REDUCTION_P):
        acc += p
        if u < acc:
            red = cand
            break
    if red in ("colsum", "rowsum"):
        rows = 2 ** math.ceil(math.log2(n) / 2)
        shape = (rows, -(-n // rows))
    else:
        shape = (n, 1)
    return {"id": index, "seed": seed, "nodes": nodes, "n_inputs": k, "target_depth": D,
            "n": shape[0] * shape[1], "shape": shape, "dtype": dtype, "reduce": red}
