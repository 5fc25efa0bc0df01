"""Known-answer tests of the compensated per-thread sums and stress tests of
the single-pass cross-block finish.

A thread keeps one compensated sum per vector lane: the elements at lane j of
the vectors it visits form chain j, in visiting order (the default launch
configuration fixes which elements a thread visits).  t is half an ulp of 1
in the compute type (2^-24, or 2^-53 for FP64): 1 + t rounds to 1.

Known answer 1 (FP32 compute): the first element each thread visits holds +1
or -1 (alternating over the threads), every other element t.  The exact sum
(#+1 - #-1) + (n - T) t is held exactly by FP64, and every chain reaches its
part exactly only if it keeps what each 1 + t drops; a plain sum, or a
pairwise pre-sum of a tile's values ahead of the compensated add, loses t
per +1.

Known answer 2 (every storage type, FP64 included): the first three elements
of chain 0 of every thread are +-1, +t, -t and all others 0.  Compensated,
each chain ends at exactly +-1 and the FP64 combine of those is exact;
uncompensated, 1 + t - t ends at 1 - t.

Stress: thousands of back-to-back reductions whose blocks (spread over all
eight XCDs) publish partials for the last block to combine must each give
the bits of the first, and leave their counters at zero."""
import numpy as np
import pytest

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu

TINY = {"f32": 2.0 ** -24, "bf16": 2.0 ** -24, "f16": 2.0 ** -24, "f64": 2.0 ** -53}
TORCH = {"f32": "float32", "bf16": "bfloat16", "f16": "float16", "f64": "float64"}


def _dt(fx, dtype):
    return {"f32": fx.F32, "f64": fx.F64, "bf16": fx.BF16, "f16": fx.F16}[dtype]


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("n", [1 << 22, (1 << 24) + 4096])
def test_accu_known_answer_at_every_thread(dtype, n):
    torch, fx = need_gpu()
    block, ept, vec_bytes, split = fx.fx_resolve_launch(fx.R_ACCU, _dt(fx, dtype), (n, 1))
    esize = {"f32": 4, "f64": 8, "bf16": 2, "f16": 2}[dtype]
    N = vec_bytes // esize
    tile = block * ept                       # vectors per block and tile
    assert split * tile * N <= n, "every thread must own a whole first tile"
    t = TINY[dtype]
    x = np.full(n, t)
    first = ((np.arange(split)[:, None] * tile + np.arange(block)[None, :]) * N).ravel()
    signs = np.where(np.arange(first.size) % 2 == 0, 1.0, -1.0)
    x[first] = signs
    want = float(signs.sum()) + (n - first.size) * t
    tt = getattr(torch, TORCH[dtype])
    X = torch.from_numpy(x).to(tt).to("cuda")
    ones = torch.ones(n, dtype=tt, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = fx.workspace(fx.R_ACCU, _dt(fx, dtype), (n, 1))
    fx.fx_accu_xy(X, ones, out, ws)
    torch.cuda.synchronize()
    assert out.item() == want, (dtype, n, (block, ept, vec_bytes, split), out.item(), want)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("shape", [(8192, 64), (20000, 8)])
def test_colsum_known_answer_at_every_thread(dtype, shape):
    """sum(X % ones, 0) with +-1 at the first element of every thread of
    every column chunk."""
    torch, fx = need_gpu()
    rows, cols = shape
    block, ept, vec_bytes, split = fx.fx_resolve_launch(fx.R_COLSUM, _dt(fx, dtype), shape)
    esize = {"f32": 4, "f64": 8, "bf16": 2, "f16": 2}[dtype]
    N = vec_bytes // esize
    assert split >= 1 and rows % N == 0
    rpc = -(-(-(-rows // split)) // N) * N   # rows per chunk, a multiple of N
    t = TINY[dtype]
    x = np.full((rows, cols), t)             # column-major: x[:, c] is column c
    want = np.empty(cols)
    for c in range(cols):
        k = 0
        for s in range(split):
            r0, r1 = s * rpc, min(rows, s * rpc + rpc)
            nv = max(r1 - r0, 0) // N
            for i in range(min(block, nv)):
                x[r0 + i * N, c] = 1.0 if k % 2 == 0 else -1.0
                k += 1
        want[c] = float(k % 2) + (rows - k) * t
    tt = getattr(torch, TORCH[dtype])
    X = torch.from_numpy(np.asfortranarray(x).ravel(order="F").copy()).to(tt).to("cuda")
    ones = torch.ones(rows * cols, dtype=tt, device="cuda")
    acc = torch.float64 if dtype == "f64" else torch.float32
    out = torch.empty(cols, dtype=acc, device="cuda")
    ws = fx.workspace(fx.R_COLSUM, _dt(fx, dtype), shape)
    fx.fx_colsum_xy(X, ones, out, shape, ws)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    assert np.array_equal(got, want), (dtype, shape, (block, ept, vec_bytes, split),
                                       np.flatnonzero(got != want)[:5])


def _chain0(starts, i, block, ept, nv, count=3):
    """The first `count` vectors (indices) on chain 0 of thread i whose tiles
    start at the vector indices in `starts` (in visiting order)."""
    out = []
    for t0 in starts:
        for k in range(ept):
            v = t0 + i + k * block
            if v < nv:
                out.append(v)
                if len(out) == count:
                    return out
    return out


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16", "f64"])
def test_accu_known_answer_chain(dtype):
    torch, fx = need_gpu()
    n = 1 << 22
    block, ept, vec_bytes, split = fx.fx_resolve_launch(fx.R_ACCU, _dt(fx, dtype), (n, 1))
    esize = {"f32": 4, "f64": 8, "bf16": 2, "f16": 2}[dtype]
    N = vec_bytes // esize
    nv = n // N
    tile = block * ept
    t = TINY[dtype]
    x = np.zeros(n)
    want = 0.0
    for b in range(split):
        starts = [tt * tile for tt in range(b, -(-nv // tile), split)]
        for i in range(block):
            ch = _chain0(starts, i, block, ept, nv)
            assert len(ch) == 3
            sign = 1.0 if (b * block + i) % 2 == 0 else -1.0
            x[ch[0] * N], x[ch[1] * N], x[ch[2] * N] = sign, t, -t
            want += sign
    tt = getattr(torch, TORCH[dtype])
    X = torch.from_numpy(x).to(tt).to("cuda")
    ones = torch.ones(n, dtype=tt, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    fx.fx_accu_xy(X, ones, out, fx.workspace(fx.R_ACCU, _dt(fx, dtype), (n, 1)))
    torch.cuda.synchronize()
    assert out.item() == want, (dtype, (block, ept, vec_bytes, split), out.item(), want)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16", "f64"])
def test_colsum_known_answer_chain(dtype):
    torch, fx = need_gpu()
    rows, cols = 8192, 4096    # one chunk per column: every chain gets three elements
    block, ept, vec_bytes, split = fx.fx_resolve_launch(fx.R_COLSUM, _dt(fx, dtype), (rows, cols))
    esize = {"f32": 4, "f64": 8, "bf16": 2, "f16": 2}[dtype]
    N = vec_bytes // esize
    assert split == 1
    nv = rows // N
    tile = block * ept
    t = TINY[dtype]
    col = np.zeros(rows)       # every column gets the same pattern
    want = 0.0
    for i in range(min(block, nv)):
        ch = _chain0(list(range(0, nv, tile)), i, block, ept, nv)
        assert len(ch) == 3
        sign = 1.0 if i % 2 == 0 else -1.0
        for v, val in zip(ch, (sign, t, -t)):
            col[v * N] = val
        want += sign
    tt = getattr(torch, TORCH[dtype])
    X = torch.from_numpy(col).to(tt).to("cuda").repeat(cols)
    ones = torch.ones(rows * cols, dtype=tt, device="cuda")
    acc = torch.float64 if dtype == "f64" else torch.float32
    out = torch.empty(cols, dtype=acc, device="cuda")
    fx.fx_colsum_xy(X, ones, out, (rows, cols), fx.workspace(fx.R_COLSUM, _dt(fx, dtype), (rows, cols)))
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    assert np.all(got == want), (dtype, (block, ept, vec_bytes, split), got[:4], want)


def _counters_zero(torch, ws, nbytes):
    return not torch.any(ws[:nbytes] != 0).item()


def test_finish_stress_accu_split_512():
    """2000 back-to-back full reductions of 2^16 elements over 512 blocks
    (most of them hold no tile and only take a ticket)."""
    torch, fx = need_gpu()
    n = 1 << 16
    g = torch.Generator().manual_seed(5)
    X = torch.rand(n, generator=g, dtype=torch.float32).to("cuda") - 0.5
    Y = torch.rand(n, generator=g, dtype=torch.float32).to("cuda") - 0.5
    cfg = (256, 1, 16, 512)
    ws = fx.workspace(fx.R_ACCU, fx.F32, (n, 1), cfg)
    reps = 2000
    out = torch.zeros(reps, dtype=torch.float64, device="cuda")
    for i in range(reps):
        fx.fx_accu_xy(X, Y, out[i:i + 1], ws, cfg=cfg)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    bad = np.flatnonzero(o != o[0])
    assert bad.size == 0, "run %d gave %r, run 0 gave %r" % (bad[0], o[bad[0]], o[0])
    assert _counters_zero(torch, ws, 256)
    ref = float(np.dot(X.cpu().double().numpy(), Y.cpu().double().numpy()))
    assert abs(o[0] - ref) <= 1e-6 * abs(ref) + 1e-9


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_finish_stress_colsum_split(dtype):
    """2000 back-to-back column sums whose columns are split over 64 blocks
    each: every column's last block combines 64 partials published by blocks
    on other XCDs."""
    torch, fx = need_gpu()
    shape = (1 << 14, 8)
    n = shape[0] * shape[1]
    tt = getattr(torch, TORCH[dtype])
    g = torch.Generator().manual_seed(6)
    X = (torch.rand(n, generator=g) - 0.5).to(tt).to("cuda")
    Y = (torch.rand(n, generator=g) - 0.5).to(tt).to("cuda")
    cfg = (256, 1, 16, 64)
    dt = _dt(fx, dtype)
    ws = fx.workspace(fx.R_COLSUM, dt, shape, cfg)
    reps = 2000
    out = torch.zeros((reps, shape[1]), dtype=torch.float32, device="cuda")
    for i in range(reps):
        fx.fx_colsum_xy(X, Y, out[i], shape, ws, cfg=cfg)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    bad = np.flatnonzero(np.any(o != o[0], axis=1))
    assert bad.size == 0, "run %d differs from run 0" % bad[0]
    assert _counters_zero(torch, ws, 4 * shape[1])


def test_finish_stress_tape_accu():
    """The same protocol through a run-time tape: 1000 back-to-back tape
    reductions over 256 blocks."""
    torch, fx = need_gpu()
    n = 1 << 18
    g = torch.Generator().manual_seed(7)
    X = (torch.rand(n, generator=g) - 0.5).to("cuda")
    Y = (torch.rand(n, generator=g) - 0.5).to("cuda")
    tape = fx.Tape([("leaf", -1, -1, 0, 0.0), ("leaf", -1, -1, 1, 0.0), ("mul", 0, 1, -1, 0.0),
                    ("exp", 2, -1, -1, 0.0)])
    cfg = (256, 1, 16, 256)
    ws = fx.workspace(fx.R_ACCU, fx.F32, (n, 1), cfg)
    reps = 1000
    out = torch.zeros(reps, dtype=torch.float64, device="cuda")
    for i in range(reps):
        fx.fx_tape_eval(tape, [X, Y], out[i:i + 1], (n, 1), fx.R_ACCU, ws, cfg=cfg)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    bad = np.flatnonzero(o != o[0])
    assert bad.size == 0, "run %d differs from run 0" % bad[0]
    assert _counters_zero(torch, ws, 256)
