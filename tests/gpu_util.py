"""Helpers shared by the GPU tests: seeded inputs on the device and
comparison against the oracle."""
import numpy as np
import pytest

import oracle
import synth

TORCH_DT = {"f32": "float32", "f64": "float64", "bf16": "bfloat16", "f16": "float16",
            "u32": "uint32"}


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_22242_amd as fx
    fx.lib()  # raises if the HIP library is missing: no fallback
    return torch, fx


def to_dev(a: np.ndarray, dtype: str):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype == "bf16":
        t = t.view(torch.int16).view(torch.bfloat16)
    elif dtype == "u32":
        t = t.view(torch.int32).view(torch.uint32)
    return t.to("cuda")


def from_dev(t, dtype: str) -> np.ndarray:
    import torch
    t = t.detach().cpu()
    if dtype == "bf16":
        return synth.bf16_to_f64(t.view(torch.int16).numpy().view(np.uint16))
    if dtype == "u32":
        return t.view(torch.int32).numpy().view(np.uint32)
    return t.numpy().astype(np.float64)


def empty(n, dtype: str):
    import torch
    return torch.empty(n, dtype=getattr(torch, TORCH_DT[dtype]), device="cuda")


def inputs(seed, n, dtype, k=3, dist=None, param=0.0):
    if dist is None:
        dist = "uint31" if dtype == "u32" else "uniform"
    host = [synth.fill(seed, t, n, dtype, dist, param) for t in range(k)]
    return host, [to_dev(h, dtype) for h in host]


def assert_close(got, value, mu, dtype, what, out_dtype=None):
    ok, rep = oracle.check(got, value, mu, dtype, out_dtype=out_dtype)
    if not ok.all():
        bad = np.flatnonzero(~ok)[:5]
        raise AssertionError("%s: %s; first bad %s got %s want %s" % (
            what, rep, bad.tolist(), np.asarray(got).ravel()[bad].tolist(),
            np.asarray(value).ravel()[bad].tolist()))
    return rep


def oracle_expr(nodes):
    """The oracle's expression for generated tree nodes (children first)."""
    built = []
    for (op, a, b, inp, val) in nodes:
        if op == "leaf":
            e = oracle.leaf(inp)
        elif op == "const":
            e = oracle.const(val)
        elif op == "neg":
            e = -built[a]
        elif op == "abs":
            e = oracle.abs_(built[a])
        elif op == "exp":
            e = oracle.exp(built[a])
        elif op == "sqrt":
            e = oracle.sqrt(built[a])
        else:
            e = oracle.E(op, (built[a], built[b]))
        built.append(e)
    return built[-1]


def tree_inputs(seed, expr, k, n, dtype):
    from synth import trees
    host = [synth.fill(seed, trees.input_tensor_id(expr, q), n, dtype) for q in range(k)]
    return host, [to_dev(h, dtype) for h in host]
