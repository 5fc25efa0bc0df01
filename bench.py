"""Benchmark of the fused expression path on one MI355X.

A step is one pass of the fused hot path over the matrix workload: FP32
8192 x 8192 column-major X, Y, W ~ U[-1,1] (seeded), computing
    Z = (X + Y) % exp(-abs(W)) / (1 + X % X)      (element-wise)
    sum(Z, 0)                                       (column sums, fused)
    norm_fro(X - Y)                                 (Frobenius norm, fused)
Protocol: W untimed warm-up steps, then K timed steps (the paper's protocol is
2 warm-ups and the mean of 50 runs, Sec. 4).  `value` is algorithmic bytes
(distinct inputs read once + outputs written once) over the wall time of the
timed region, in GB/s.  Alongside: per-kernel HIP-event times, the same
results through the unfused one-kernel-per-operator baseline, the same
workload with BF16 storage, the copy ceiling, and the FP64 CPU oracle timed
on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, vendor figure
ROWS = COLS = 8192


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(dtype, n, seed=2):
    import numpy as np
    import torch

    import synth
    out = []
    for t in range(3):
        h = synth.fill(seed, t, n, dtype)
        tt = torch.from_numpy(h)
        if dtype == "bf16":
            tt = tt.view(torch.int16).view(torch.bfloat16)
        out.append(tt.to("cuda"))
        del h
    return out


class Workload:
    """The three fused results (or their unfused evaluation) on one dtype."""

    def __init__(self, fx, torch, dtype, rows, cols):
        self.fx, self.torch = fx, torch
        self.dtype, self.shape = dtype, (rows, cols)
        n = rows * cols
        self.X, self.Y, self.W = make_inputs(dtype, n)
        tdt = self.X.dtype
        acc = torch.float64 if dtype == "f64" else torch.float32  # column sums' dtype
        self.Z = torch.empty(n, dtype=tdt, device="cuda")
        self.cs = torch.empty(cols, dtype=acc, device="cuda")
        self.nrm = torch.zeros(1, dtype=torch.float64, device="cuda")
        dt = fx.dtype_code(self.X)
        self.ws_c = fx.workspace(fx.R_COLSUM, dt, self.shape)
        self.ws_n = fx.workspace(fx.R_NORM, dt, self.shape)
        esz = self.X.element_size()
        # algorithmic bytes: distinct inputs read once, outputs written once
        self.bytes = {"z": 4 * n * esz, "colsum": 3 * n * esz + cols * self.cs.element_size(),
                      "norm": 2 * n * esz + 8}
        self.tmp = None

    def fused(self, which, stream):
        fx = self.fx
        if which == "z":
            fx.fx_c2_z(self.X, self.Y, self.W, self.Z, self.shape, stream=stream)
        elif which == "colsum":
            fx.fx_c2_colsum(self.X, self.Y, self.W, self.cs, self.shape, self.ws_c, stream=stream)
        else:
            fx.fx_norm_fro_diff(self.X, self.Y, self.nrm, self.shape, self.ws_n, stream=stream)

    def unfused(self, which, stream):
        fx, torch = self.fx, self.torch
        if self.tmp is None:
            nb = fx.fx_unfused_tmp_bytes("c2_colsum", fx.dtype_code(self.X), self.shape)
            self.tmp = torch.empty(nb, dtype=torch.uint8, device="cuda")
        ins = [self.X, self.Y, self.W]
        if which == "z":
            fx.fx_unfused("c2_z", ins, self.Z, self.shape, self.tmp, stream=stream)
        elif which == "colsum":
            fx.fx_unfused("c2_colsum", ins, self.cs, self.shape, self.tmp, self.ws_c, stream=stream)
        else:
            fx.fx_unfused("norm_diff", ins[:2], self.nrm, self.shape, self.tmp, self.ws_n,
                          stream=stream)


RESULTS = ("z", "colsum", "norm")


def time_steps(torch, run, steps, warmup, stream, timed=RESULTS):
    """W warm-up steps, then K timed steps bracketed by synchronisations;
    returns (wall seconds, per-result mean kernel ms from HIP events recorded
    on the launch stream around the results in `timed`).  Each event record
    is a packet in the stream that costs the step a few microseconds, so the
    step whose wall time is the benchmark's value times only the dominant
    kernel (the roofline's), and the per-result times come from a pass of
    their own."""
    for _ in range(warmup):
        for r in RESULTS:
            run(r, stream)
    torch.cuda.synchronize()
    ev = {r: [] for r in timed}
    t0 = time.perf_counter()
    for _ in range(steps):
        for r in RESULTS:
            if r in ev:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                run(r, stream)
                b.record(stream)
                ev[r].append((a, b))
            else:
                run(r, stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = {r: sum(a.elapsed_time(b) for a, b in ev[r]) / steps for r in timed}
    return wall, ms


def spin_up(run, steps=20):
    """Untimed steps before a detail pass: the first milliseconds after a
    workload's inputs are built run several percent slow."""
    for _ in range(steps):
        for r in RESULTS:
            run(r, None)


def copy_ceiling(fx, torch, stream, nbytes=1 << 31, reps=20):
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        fx.fx_bw_copy(src, dst, nbytes, stream=stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fx.fx_bw_copy(src, dst, nbytes, stream=stream)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def read_flush(fx, torch, stream, nbytes=1 << 30):
    """A function that streams `nbytes` (4x the 256 MB last-level cache)
    through our read kernel: afterwards no line of anything else is cached,
    and, unlike a write, it leaves no dirty lines whose write-back would
    slow the next kernel."""
    buf = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    cfg = (256, 2, 16, 1024)
    sink = torch.zeros(cfg[3], dtype=torch.float64, device="cuda")
    return lambda: fx.fx_bw_read(buf, nbytes, sink, cfg=cfg, stream=stream)


def cold_ms(torch, stream, fn, reps, flush):
    """Median HIP-event time of fn() with flush() run before each launch
    (outside the events): no input left in the 256 MB last-level cache."""
    times = []
    for _ in range(reps):
        flush()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    return sorted(times)[len(times) // 2]


def ceilings_detail(fx, torch, stream, reps=5):
    """Bandwidth ceilings of this GPU from our own kernels, each timed cold
    (a 1 GiB read before every launch, median of `reps`) at 2^28 FP32
    elements (1 GiB) per array, best over a small launch sweep: read, write,
    copy (1 read : 1 write) and triad (3 reads : 1 write, the mix of the
    matrix workload's Z).  GB/s over the bytes each moves."""
    n = 1 << 28
    nb = 4 * n
    bufs = [torch.empty(n, dtype=torch.float32, device="cuda").fill_(float(q + 1))
            for q in range(4)]
    # the read kernel writes one double per block: as many as the largest grid
    grid_default = fx.fx_resolve_launch(0, fx.F32, (n, 1))[3]
    sink = torch.zeros(max(grid_default, 4096), dtype=torch.float64, device="cuda")
    flush = read_flush(fx, torch, stream)
    cfgs = [None] + [(blk, ept, 16, grid) for blk in (256, 512) for ept in (1, 2, 4)
                     for grid in (512, 1024, 2048, 4096)]
    kinds = {
        "read": (nb, lambda c, st: fx.fx_bw_read(bufs[0], nb, sink, cfg=c, stream=st)),
        "write": (nb, lambda c, st: fx.fx_bw_write(bufs[3], nb, 7, cfg=c, stream=st)),
        "copy": (2 * nb, lambda c, st: fx.fx_bw_copy(bufs[0], bufs[3], nb, cfg=c, stream=st)),
        "triad": (4 * nb, lambda c, st: fx.fx_bw_triad(bufs[0], bufs[1], bufs[2], bufs[3], nb,
                                                       False, cfg=c, stream=st)),
        "triad_streaming_stores": (4 * nb, lambda c, st: fx.fx_bw_triad(
            bufs[0], bufs[1], bufs[2], bufs[3], nb, True, cfg=c, stream=st)),
    }
    out = {}
    with torch.cuda.stream(stream):
        for name, (moved, fn) in kinds.items():
            best = None
            for c in cfgs:
                if name == "copy" and c is not None and c[3] > 2048:
                    continue
                ms = cold_ms(torch, stream, lambda: fn(c, stream), reps, flush)
                if best is None or ms < best[0]:
                    best = (ms, c)
            out[name] = {"GB/s": round(moved / (best[0] * 1e-3) / 1e9, 1),
                         "ms": round(best[0], 4), "cfg": list(best[1]) if best[1] else "default"}
    del bufs, sink
    torch.cuda.empty_cache()
    return out


_SLEEP_CYCLES_PER_MS = None


def hold_stream(torch, stream, ms):
    """Keep `stream` busy for about `ms` with a GPU-side spin that touches no
    memory, so that work enqueued meanwhile starts back to back."""
    global _SLEEP_CYCLES_PER_MS
    if not hasattr(torch.cuda, "_sleep"):
        return
    with torch.cuda.stream(stream):
        if _SLEEP_CYCLES_PER_MS is None:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            torch.cuda._sleep(1_000_000)
            b.record(stream)
            torch.cuda.synchronize()
            _SLEEP_CYCLES_PER_MS = 1_000_000 / max(a.elapsed_time(b), 1e-3)
        torch.cuda._sleep(int(_SLEEP_CYCLES_PER_MS * ms))


def event_ms(torch, stream, fn, reps, warm_ms=5.0):
    """Mean HIP-event time of fn() over reps launches after a warm-up of at
    least three launches and about warm_ms of GPU time.  Short kernels are
    enqueued behind a GPU-side spin, so that they are timed back to back on
    the GPU rather than at the host's launch rate."""
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()  # a first launch may load the kernel's code
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(2):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    each = max(a.elapsed_time(b) / 2, 1e-3)
    for _ in range(min(200, int(warm_ms / each))):
        fn()
    torch.cuda.synchronize()
    if each < 0.1:
        hold_stream(torch, stream, min(10.0, 0.05 * reps))
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def c1_detail(fx, torch, stream, reps):
    """The small vector workload, n = 2^20 FP32 (16 MiB: it fits the 256 MB
    last-level cache): Z = X%Y + 2W and accu(X%Y), and its u32 form
    Z = (X^Y) + 3W, warm (back-to-back launches) and cold (a 1 GiB read
    between launches, outside the timed events)."""
    import synth
    n = 1 << 20
    X, Y, W = [torch.from_numpy(synth.fill(1, t, n, "f32")).cuda() for t in range(3)]
    U = [torch.from_numpy(synth.fill(1, t, n, "u32", "uint31").view("int32")).cuda()
         for t in range(3)]
    Z = torch.empty(n, device="cuda")
    ZU = torch.empty(n, dtype=torch.int32, device="cuda")
    s = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = fx.workspace(fx.R_ACCU, fx.F32, (n, 1))
    flush = read_flush(fx, torch, stream)
    runs = {"z": (lambda: fx.fx_c1_z(X, Y, W, Z, stream=stream), 16 * n),
            "accu": (lambda: fx.fx_accu_xy(X, Y, s, ws, stream=stream), 8 * n),
            "u32_z": (lambda: fx.fx_c1_z(*U, ZU, stream=stream), 16 * n)}
    out = {}
    with torch.cuda.stream(stream):
        for name, (fn, nbytes) in runs.items():
            warm = event_ms(torch, stream, fn, reps)
            times = []
            for _ in range(reps):
                flush()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                fn()
                b.record(stream)
                torch.cuda.synchronize()
                times.append(a.elapsed_time(b))
            cold = sum(times) / len(times)
            out[name] = {"warm_us": round(warm * 1e3, 2), "warm_GB/s": round(nbytes / warm / 1e6, 1),
                         "cold_us": round(cold * 1e3, 2), "cold_GB/s": round(nbytes / cold / 1e6, 1)}
    return out


def precision_detail(fx, torch, stream, reps):
    """The C1 expressions at 2^28 elements: BF16 and FP16 storage against the
    FP32 storage reference (Z = X%Y + 2W and accu(X%Y)), plus norm_fro(X-Y)
    and sum(X%Y, 0) with the vector read as a 2^14 x 2^14 column-major
    matrix."""
    import synth
    m = 1 << 28
    out = {}
    for dt in ("f32", "bf16", "f16"):
        X, Y, W = [torch.from_numpy(synth.fill(3, t, m, dt)) for t in range(3)]
        if dt == "bf16":
            X, Y, W = [t.view(torch.int16).view(torch.bfloat16) for t in (X, Y, W)]
        X, Y, W = X.cuda(), Y.cuda(), W.cuda()
        Z = torch.empty_like(X)
        s = torch.zeros(1, dtype=torch.float64, device="cuda")
        ws = fx.workspace(fx.R_ACCU, fx.dtype_code(X), (m, 1))
        es = X.element_size()
        side = 1 << 14
        sq = (side, side)
        wn = fx.workspace(fx.R_NORM, fx.dtype_code(X), sq)
        wc = fx.workspace(fx.R_COLSUM, fx.dtype_code(X), sq)
        cs = torch.empty(side, dtype=torch.float32, device="cuda")
        zt = event_ms(torch, stream, lambda: fx.fx_c1_z(X, Y, W, Z, stream=stream), reps)
        at = event_ms(torch, stream, lambda: fx.fx_accu_xy(X, Y, s, ws, stream=stream), reps)
        nt = event_ms(torch, stream, lambda: fx.fx_norm_fro_diff(X, Y, s, sq, wn, stream=stream), reps)
        ct = event_ms(torch, stream, lambda: fx.fx_colsum_xy(X, Y, cs, sq, wc, stream=stream), reps)
        out[dt] = {"z_ms": round(zt, 4), "z_GB/s": round(4 * es * m / zt / 1e6, 1),
                   "accu_ms": round(at, 4), "accu_GB/s": round(2 * es * m / at / 1e6, 1),
                   "norm_ms": round(nt, 4), "norm_GB/s": round(2 * es * m / nt / 1e6, 1),
                   "colsum_ms": round(ct, 4),
                   "colsum_GB/s": round((2 * es * m + 4 * side) / ct / 1e6, 1)}
        del X, Y, W, Z
        torch.cuda.empty_cache()
    for dt in ("bf16", "f16"):
        for r in ("z", "accu", "norm", "colsum"):
            out[dt][r + "_speedup_vs_f32_storage"] = round(out["f32"][r + "_ms"] / out[dt][r + "_ms"], 3)
    return out


def batch_detail(fx, torch, stream, reps):
    """4096 random expressions (sizes 256..2^20, half ending in accu), FP32:
    one persistent launch replayed from a HIP graph against 4096 separate
    launches of the same tapes."""
    import synth
    from synth import trees
    tset = trees.batch_set(4096)
    items = []
    for t in tset:
        ins = [torch.from_numpy(synth.fill(4, trees.input_tensor_id(t["id"], q), t["n"], "f32")).cuda()
               for q in range(t["n_inputs"])]
        out = (torch.zeros(1, dtype=torch.float64, device="cuda") if t["reduce"] else
               torch.empty(t["n"], dtype=torch.float32, device="cuda"))
        items.append((fx.Tape(t["nodes"]), ins, out, t["n"], fx.R_ACCU if t["reduce"] else 0))
    b = fx.Batch(items, fx.F32)
    info = b.info()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        # medians over three interleaved rounds: the first round after the
        # batch is built runs several percent slow
        gs, ones = [], []
        for _ in range(3):
            gs.append(event_ms(torch, st, lambda: b.graph(st), reps))
            ones.append(event_ms(torch, st, lambda: b.launch(st), reps))
        g, one = statistics.median(gs), statistics.median(ones)
        each = event_ms(torch, st, lambda: b.launch_each(st), max(3, reps // 5))
    res = {"expressions": 4096, "tiles": info["n_tiles"], "tile_elems": info["tile_elems"],
           "bytes": info["bytes"], "graph_ms": round(g, 4), "persistent_launch_ms": round(one, 4),
           "separate_launches_ms": round(each, 4), "speedup_vs_separate": round(each / g, 2),
           "graph_GB/s": round(info["bytes"] / g / 1e6, 1)}
    b.destroy()
    return res


def paper_suite_detail(fx, torch, stream, reps):
    """The paper's expressions at its size, 10k x 10k FP32 (Sec. 4), fused;
    and the add-N sweep N = 2..16: fused against one add kernel per operator
    (what toolkits without fusion launch), as effective GB/s over the same
    algorithmic bytes."""
    import synth
    shape, n = (10000, 10000), 10 ** 8
    ins = []
    for t in range(16):
        ins.append(torch.from_numpy(synth.fill(10, t, n, "f32")).cuda())
    Z = torch.empty(n, device="cuda")
    T = torch.empty(n, device="cuda")
    suite = {}
    for name, k, sc in [("add2", 2, ()), ("add4", 4, ()), ("relu", 1, ()), ("sigmoid", 1, ()),
                        ("swish", 1, (1.0,)), ("gelu", 1, (0.044715,))]:
        ms = event_ms(torch, stream, lambda: fx.fx_paper_expr(name, ins[:k], Z, shape, sc,
                                                              stream=stream), reps)
        suite[name] = {"ms": round(ms, 4), "GB/s": round((k + 1) * 4 * n / ms / 1e6, 1)}
    y64 = torch.from_numpy(synth.fill(10, 20, n, "f64")).cuda()
    w = torch.from_numpy(synth.fill(10, 21, n, "f32", "uniform12")).cuda()
    ms = event_ms(torch, stream, lambda: fx.fx_paper_expr("expr3", [ins[0], y64, w], Z, shape,
                                                          stream=stream), reps)
    suite["expr3"] = {"ms": round(ms, 4), "GB/s": round((4 + 8 + 4 + 4) * n / ms / 1e6, 1)}
    del y64, w
    sweep = {}
    for N in range(2, 17):
        f = event_ms(torch, stream, lambda: fx.fx_addn(ins[:N], Z, shape, stream=stream), reps)

        def unfused():
            fx.fx_op_binary("add", ins[0], ins[1], T if N > 2 else Z, stream=stream)
            for q in range(2, N):
                fx.fx_op_binary("add", T, ins[q], T if q < N - 1 else Z, stream=stream)

        u = event_ms(torch, stream, unfused, max(3, reps // 2))
        b = (N + 1) * 4 * n
        sweep[N] = {"fused_GB/s": round(b / f / 1e6, 1), "unfused_GB/s": round(b / u / 1e6, 1),
                    "speedup": round(u / f, 2)}
    return {"expressions_10k": suite, "add_N_sweep_10k": sweep}


def modes_detail(fx, torch, stream, reps):
    """One expression four ways: compile-time template (the fused kernel),
    run-time tape (interpreter; also with the shipped launch model attached),
    run-time source (a tape's node list as text, hipRTC-compiled at first use)
    and source generated at compile time from the template's own expression
    type (hipRTC-compiled at first use).  The matrix
    workload's Z and its column sums over 2^26 FP32 elements, and the
    deepest of the first 200 generated tuning trees (depth <= 8) over 2^26
    elements."""
    import synth
    from synth import trees
    from paper_2604_22242_amd.model import C2_NODES
    n = ROWS * COLS
    ins = [torch.from_numpy(synth.fill(2, t, n, "f32")).cuda() for t in range(4)]
    Z = torch.empty(n, device="cuda")
    out = {}
    model = fx.fx_model_load(os.path.join(ROOT, "paper_2604_22242_amd", "launch_model.fxm"))

    def model_tape(nodes, shape, kind):
        t = fx.Tape(nodes)
        t.set_model(model)
        return t, model.predict(fx.fx_tape_features(t, fx.F32, shape, kind), kind, fx.F32)

    def timed(fns):
        """Median over three interleaved rounds of each variant's event time
        (one round of a variant alone varies by up to 20% here)."""
        got = {k: [] for k in fns}
        for _ in range(3):
            for k, f in fns.items():
                got[k].append(event_ms(torch, stream, f, reps))
        return {k: round(statistics.median(v), 4) for k, v in got.items()}

    r = fx.Rtc(C2_NODES, fx.F32)
    tape = fx.Tape(C2_NODES)
    tm, pick = model_tape(C2_NODES, (n, 1), 0)
    et_compile = fx.fx_source_prepare("c2_z", fx.F32)  # first use: the hipRTC compile
    out["c2_z"] = timed({
        "compile_time_ms": lambda: fx.fx_c2_z(*ins[:3], Z, (ROWS, COLS), stream=stream),
        "tape_ms": lambda: fx.fx_tape_eval(tape, ins[:3], Z, (n, 1), stream=stream),
        "tape_model_ms": lambda: fx.fx_tape_eval(tm, ins[:3], Z, (n, 1), stream=stream),
        "runtime_source_ms": lambda: r.eval(ins[:3], Z, stream=stream),
        "et_source_ms": lambda: fx.fx_source_eval("c2_z", ins[:3], Z, (ROWS, COLS), stream=stream)})
    out["c2_z"].update({"model_pick": list(pick), "hiprtc_compile_ms": round(r.compile_ms(), 1),
                        "et_source_compile_ms": round(et_compile, 1)})
    cs = torch.empty(COLS, device="cuda")
    shape = (ROWS, COLS)
    ws = fx.workspace(fx.R_COLSUM, fx.F32, shape)
    r = fx.Rtc(C2_NODES, fx.F32, fx.R_COLSUM)
    tape = fx.Tape(C2_NODES)
    tm, pick = model_tape(C2_NODES, shape, fx.R_COLSUM)
    wm = fx.workspace(fx.R_COLSUM, fx.F32, shape, pick)
    et_compile = fx.fx_source_prepare("c2_colsum", fx.F32)
    out["c2_colsum"] = timed({
        "compile_time_ms": lambda: fx.fx_c2_colsum(*ins[:3], cs, shape, ws, stream=stream),
        "tape_ms": lambda: fx.fx_tape_eval(tape, ins[:3], cs, shape, fx.R_COLSUM, ws, stream=stream),
        "tape_model_ms": lambda: fx.fx_tape_eval(tm, ins[:3], cs, shape, fx.R_COLSUM, wm,
                                                 stream=stream),
        "runtime_source_ms": lambda: r.eval(ins[:3], cs, shape, ws, stream=stream),
        "et_source_ms": lambda: fx.fx_source_eval("c2_colsum", ins[:3], cs, shape, ws,
                                                  stream=stream)})
    out["c2_colsum"].update({"model_pick": list(pick), "hiprtc_compile_ms": round(r.compile_ms(), 1),
                             "et_source_compile_ms": round(et_compile, 1)})
    best = max((trees.tuning_item(5, i) for i in range(200)),
               key=lambda it: fx.Tape(it["nodes"]).info()["n_instructions"])
    k = best["n_inputs"]
    tape = fx.Tape(best["nodes"])
    r = fx.Rtc(best["nodes"], fx.F32)
    tm, pick = model_tape(best["nodes"], (n, 1), 0)
    out["deep_tree"] = {"tree": best["id"], "nodes": len(best["nodes"]),
                        "tape_instructions": tape.info()["n_instructions"]}
    out["deep_tree"].update(timed({
        "tape_ms": lambda: fx.fx_tape_eval(tape, ins[:k], Z, (n, 1), stream=stream),
        "tape_model_ms": lambda: fx.fx_tape_eval(tm, ins[:k], Z, (n, 1), stream=stream),
        "runtime_source_ms": lambda: r.eval(ins[:k], Z, stream=stream)}))
    out["deep_tree"].update({"model_pick": list(pick), "hiprtc_compile_ms": round(r.compile_ms(), 1)})
    return out


def paper_views_detail(fx, torch, stream, reps):
    """The paper's strided-view expressions at its size, 10k x 10k FP32
    inputs (Sec. 4): centre-submatrix sums, expressions with transposes and
    the diagonal sum; effective GB/s over the algorithmic bytes (each
    distinct input once, plus the output)."""
    import synth
    m = 10000
    n = m * m
    ins = [torch.from_numpy(synth.fill(11, t, n, "f32")).cuda() for t in range(3)]
    ins.append(torch.from_numpy(synth.fill(11, 3, n, "f32", "uniform12")).cuda())
    out = {}
    for name, k in (("addsub2", 2), ("addsub4", 4), ("expr1", 2), ("expr2", 4), ("diagsum", 2)):
        shape = fx.fx_paper_view_shape(name, (m, m))
        nz = shape[0] * shape[1]
        Z = torch.empty(nz, device="cuda")
        ms = event_ms(torch, stream, lambda: fx.fx_paper_view_expr(name, ins[:k], Z, (m, m), (1.5,),
                                                                    stream=stream), reps)
        if name.startswith("addsub"):
            nbytes = (k + 1) * 4 * nz                 # k centre blocks read, Z written
        elif name == "diagsum":
            nbytes = 4 * 4 * (m - 1) + 4 * nz         # four diagonals read, Z written
        else:
            nbytes = (k + 1) * 4 * n                  # each matrix once, Z written
        out[name] = {"ms": round(ms, 4), "GB/s": round(nbytes / ms / 1e6, 1),
                     "out_shape": list(shape)}
        del Z
    return out


PROFILE = os.path.join(ROOT, "profiles", "c2_8192_fused_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2604_22242_amd", "csrc", f)
                  for f in ("fx_core.hpp", "fx_expr.hpp", "fx_kernels.hpp", "fx_fused_c2.hip",
                            "fx_fused_c2sum.hip", "fx_fused_xy.hip")]


def measured_traffic(kernel_tag="k_ew[c2,f32"):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None if there is none or the
    kernel sources have changed since it was taken."""
    import hashlib
    import re
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    h = hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SOURCES)).hexdigest()[:16]
    m = re.search(r"Kernel source hash[^:]*: ([0-9a-f]{16})", text)
    if not m or m.group(1) != h:
        return None
    for line in text.splitlines():
        if line.startswith("| fx::" + kernel_tag):
            cells = [c.strip() for c in line.strip("|").split("|")]
            return int(round((float(cells[5]) + float(cells[6])) * 2 ** 20))
    return None


VALU_PROFILE = os.path.join(ROOT, "profiles", "c2_8192_fused_valu.md")
SIMDS, CLOCK_HZ = 1024, 2.4e9  # MI355X: 256 CUs x 4 SIMDs, peak engine clock


def measured_valu():
    """{dtype: {result: VALU issue quad-cycles per launch}} from the committed
    rocprofv3 SQ_ACTIVE_INST_VALU summary, or None if there is none or the
    kernel sources have changed since it was taken."""
    import hashlib
    import re
    try:
        text = open(VALU_PROFILE).read()
    except OSError:
        return None
    h = hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SOURCES)).hexdigest()[:16]
    m = re.search(r"Kernel source hash[^:]*: ([0-9a-f]{16})", text)
    j = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m or m.group(1) != h or not j:
        return None
    return json.loads(j.group(1))


def valu_roofline(counts, dt, live_ms):
    """VALU-time bound of each result (every SIMD issuing VALU work every
    cycle: 4 cycles per quad-cycle counted) and the live time's fraction of
    it."""
    if not counts or dt not in counts:
        return {}
    out = {}
    for r, q in counts[dt].items():
        bound_ms = q * 4 / (SIMDS * CLOCK_HZ) * 1e3
        out[r] = {"valu_bound_ms": round(bound_ms, 5), "valu_frac": round(bound_ms / live_ms[r], 3)}
    return out


def cpu_baseline(cols_sample=COLS, min_seconds=10.0, threads=None):
    """The FP64 oracle, as it stands, on a bounded sample of the workload: the
    same three results over the first `cols_sample` columns, repeated until
    at least `min_seconds` of CPU work has been timed.  threads: OpenMP
    threads (default: all the host offers)."""
    import oracle
    import synth
    all_threads = oracle.num_threads()
    if threads:
        oracle.set_threads(threads)
    n = ROWS * cols_sample
    host = [synth.fill(2, t, n, "f32") for t in range(3)]
    shape = (ROWS, cols_sample)
    e = oracle.EXPRS["c2_z"]
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.evaluate(e, host, "f32", shape=shape)
        oracle.evaluate(e, host, "f32", shape=shape, reduce="colsum")
        oracle.evaluate(oracle.EXPRS["diff"], host[:2], "f32", shape=shape, reduce="norm")
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    nbytes = reps * (16 * n + 12 * n + 8 * n)
    used = oracle.num_threads()
    oracle.set_threads(all_threads)
    return {"value": round(nbytes / dt / 1e9, 3), "unit": "GB/s", "cores": used,
            "kind": "oracle",
            "sample": "C2 FP32 Z, sum(Z,0), norm_fro(X-Y) over 8192 x %d columns, %d repetitions "
                      "in %.1f s (FP64, explicit temporaries)" % (cols_sample, reps, dt)}


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo; lscpu reads the same)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_oracle_configs(min_seconds=3.0, threads=None):
    """The FP64 oracle on bounded samples of the vector workload (2^20 FP32:
    Z = X%Y + 2W, accu(X%Y), and the u32 Z = (X^Y) + 3W) and of the
    precision workload (BF16 storage: Z = X%Y + 2W, accu(X%Y),
    norm_fro(X-Y) and sum(X%Y, 0) over the first 256 of the 2^14 x 2^14
    matrix's columns), each repeated for at least `min_seconds`; GB/s over
    the same algorithmic bytes as the GPU kernels."""
    import oracle
    import synth
    all_threads = oracle.num_threads()
    if threads:
        oracle.set_threads(threads)

    def timed(fn, nbytes):
        reps, t0 = 0, time.perf_counter()
        while True:
            fn()
            reps += 1
            dt = time.perf_counter() - t0
            if dt >= min_seconds:
                return round(reps * nbytes / dt / 1e9, 3), reps, round(dt, 2)

    out = {}
    n = 1 << 20
    x, y, w = [synth.fill(1, t, n, "f32") for t in range(3)]
    u = [synth.fill(1, t, n, "u32", "uint31") for t in range(3)]

    def c1():
        oracle.evaluate(oracle.EXPRS["c1_z"], [x, y, w], "f32")
        oracle.evaluate(oracle.EXPRS["xy"], [x, y], "f32", reduce="accu")
        oracle.evaluate_u32(oracle.EXPRS["u32_z"], u)

    v, reps, dt = timed(c1, 16 * n + 8 * n + 16 * n)
    out["c1"] = {"GB/s": v, "sample": "2^20 FP32 Z, accu(X%%Y) and u32 Z: %d repetitions in "
                 "%.1f s" % (reps, dt)}
    side, cols = 1 << 14, 256
    m = side * cols
    xb, yb, wb = [synth.fill(3, t, m, "bf16") for t in range(3)]

    def c3():
        oracle.evaluate(oracle.EXPRS["c1_z"], [xb, yb, wb], "bf16")
        oracle.evaluate(oracle.EXPRS["xy"], [xb, yb], "bf16", reduce="accu")
        oracle.evaluate(oracle.EXPRS["diff"], [xb, yb], "bf16", shape=(side, cols), reduce="norm")
        oracle.evaluate(oracle.EXPRS["xy"], [xb, yb], "bf16", shape=(side, cols), reduce="colsum")

    v, reps, dt = timed(c3, (8 + 4 + 4 + 4) * m)
    out["c3_bf16"] = {"GB/s": v, "sample": "BF16 Z, accu, norm_fro, sum(.,0) over 2^14 x 256 "
                      "of the 2^14 x 2^14 matrix: %d repetitions in %.1f s" % (reps, dt)}
    out["threads"] = oracle.num_threads()
    oracle.set_threads(all_threads)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the fused FP32 steps")
    ap.add_argument("--profile", action="store_true",
                    help="fused FP32 steps, then the same steps with BF16 and FP64 storage, "
                         "plus one 1 GiB copy (the known-size kernel that scales hardware "
                         "byte counters); no CPU baseline")
    ap.add_argument("--profile-set", choices=("step", "views", "paper", "batch", "precision", "c1"),
                    default="step",
                    help="with --profile: which kernels to run (the matrix-workload step, the "
                         "paper's strided-view expressions, the paper's expression suite, the "
                         "4096-expression batch, the 2^28 half-storage workload, or the 2^20 "
                         "vector workload with its u32 form), always followed by the 1 GiB copy")
    a = ap.parse_args()
    if a.profile:
        a.no_extra = a.no_cpu = True
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this path has no multi-GPU form "
              "(see the sharding design); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2604_22242_amd as fx
    fx.lib()
    stream = torch.cuda.current_stream()
    if a.profile and a.profile_set != "step":
        run = {"views": paper_views_detail, "paper": paper_suite_detail,
               "batch": batch_detail, "precision": precision_detail,
               "c1": c1_detail}[a.profile_set]
        log("bench: profile set %s, %d repetitions" % (a.profile_set, a.steps))
        res = run(fx, torch, stream, a.steps)
        torch.cuda.empty_cache()
        log("bench: 1 GiB reference copy")
        copy_ceiling(fx, torch, stream, nbytes=1 << 30, reps=1)
        print(json.dumps({"profile_set": a.profile_set, "detail": res}), flush=True)
        return
    log("bench: fused FP32 %dx%d, %d warm-up + %d timed steps" % (ROWS, COLS, a.warmup, a.steps))
    wl = Workload(fx, torch, "f32", ROWS, COLS)
    # per-result kernel times (their own pass, after untimed steps), then
    # the timed steps with events around the dominant kernel only
    if not a.profile:
        spin_up(lambda r, _: wl.fused(r, stream))
    _, ms = time_steps(torch, wl.fused, a.steps, a.warmup, stream)
    dominant = max(RESULTS, key=lambda r: ms[r])
    wall, dms_live = time_steps(torch, wl.fused, a.steps, a.warmup, stream, timed=(dominant,))
    step_bytes = sum(wl.bytes.values())
    value = step_bytes * a.steps / wall / 1e9
    per = {r: {"ms": round(ms[r], 5), "GB/s": round(wl.bytes[r] / (ms[r] * 1e-3) / 1e9, 1)}
           for r in RESULTS}
    detail = {"fp32_fused": per}
    dominant_bytes = wl.bytes[dominant]
    achieved = dominant_bytes / (dms_live[dominant] * 1e-3) / 1e9
    # the same kernels with a 1 GiB read before each launch: the 1 GiB
    # working set of a warm step keeps part of itself in the last-level cache
    # (not in profile runs, whose per-kernel averages must be the steps')
    achieved_cold = None
    if not a.profile:
        flush = read_flush(fx, torch, stream)
        with torch.cuda.stream(stream):
            cold = {r: cold_ms(torch, stream, lambda: wl.fused(r, stream), 11, flush)
                    for r in RESULTS}
        del flush
        torch.cuda.empty_cache()
        for r in RESULTS:
            per[r]["cold_ms"] = round(cold[r], 5)
            per[r]["cold_GB/s"] = round(wl.bytes[r] / (cold[r] * 1e-3) / 1e9, 1)
        achieved_cold = round(dominant_bytes / (cold[dominant] * 1e-3) / 1e9, 1)

    if not a.no_extra:
        log("bench: unfused FP32 baseline")
        spin_up(lambda r, _: wl.unfused(r, stream))
        _, ums = time_steps(torch, wl.unfused, a.steps, a.warmup, stream)
        detail["fp32_unfused_ms"] = {r: round(ums[r], 5) for r in RESULTS}
        detail["speedup_vs_unfused"] = {r: round(ums[r] / ms[r], 3) for r in RESULTS}
        del wl
        torch.cuda.empty_cache()
        log("bench: fused BF16 storage")
        wb = Workload(fx, torch, "bf16", ROWS, COLS)
        spin_up(lambda r, _: wb.fused(r, stream))
        _, bms = time_steps(torch, wb.fused, a.steps, a.warmup, stream)
        spin_up(lambda r, _: wb.unfused(r, stream))
        _, bums = time_steps(torch, wb.unfused, a.steps, a.warmup, stream)
        detail["bf16_fused"] = {r: {"ms": round(bms[r], 5),
                                    "GB/s": round(wb.bytes[r] / (bms[r] * 1e-3) / 1e9, 1),
                                    "hbm_frac": round(wb.bytes[r] / (bms[r] * 1e-3) / 1e9
                                                      / PEAK_HBM_GBS, 3)}
                                for r in RESULTS}
        # BF16 storage halves the bytes but not the arithmetic: the VALU-time
        # bound from the committed instruction counts, against the live time
        for r, v in valu_roofline(measured_valu(), "bf16", bms).items():
            detail["bf16_fused"][r].update(v)
        detail["bf16_speedup_vs_unfused"] = {r: round(bums[r] / bms[r], 3) for r in RESULTS}
        detail["bf16_speedup_vs_fp32_storage"] = {r: round(ms[r] / bms[r], 3) for r in RESULTS}
        del wb
        torch.cuda.empty_cache()
        log("bench: fused FP64 storage")
        wd = Workload(fx, torch, "f64", ROWS, COLS)
        spin_up(lambda r, _: wd.fused(r, stream))
        _, dms = time_steps(torch, wd.fused, a.steps, a.warmup, stream)
        spin_up(lambda r, _: wd.unfused(r, stream))
        _, dums = time_steps(torch, wd.unfused, a.steps, a.warmup, stream)
        detail["fp64_fused"] = {r: {"ms": round(dms[r], 5),
                                    "GB/s": round(wd.bytes[r] / (dms[r] * 1e-3) / 1e9, 1)}
                                for r in RESULTS}
        detail["fp64_speedup_vs_unfused"] = {r: round(dums[r] / dms[r], 3) for r in RESULTS}
        del wd
        torch.cuda.empty_cache()
        log("bench: copy ceiling")
        detail["copy_ceiling_GB/s"] = round(copy_ceiling(fx, torch, stream), 1)
        log("bench: read / write / copy / triad ceilings, cold, 2^28 elements")
        detail["ceilings_cold_2^28"] = ceilings_detail(fx, torch, stream)
        log("bench: precision workload, 2^28 elements")
        detail["precision_2^28"] = precision_detail(fx, torch, stream, 20)
        torch.cuda.empty_cache()
        log("bench: the paper's expressions and add-N sweep, 10k x 10k")
        detail["paper_suite"] = paper_suite_detail(fx, torch, stream, 10)
        torch.cuda.empty_cache()
        log("bench: n = 2^20 vectors, warm and cold")
        detail["c1_2^20"] = c1_detail(fx, torch, stream, 50)
        log("bench: the paper's strided-view expressions, 10k x 10k")
        detail["paper_views"] = paper_views_detail(fx, torch, stream, 10)
        torch.cuda.empty_cache()
        log("bench: compile-time, tape and run-time source modes")
        detail["modes"] = modes_detail(fx, torch, stream, 20)
        torch.cuda.empty_cache()
        log("bench: batch of 4096 expressions")
        detail["batch_4096"] = batch_detail(fx, torch, stream, 20)
        torch.cuda.empty_cache()

    if a.profile:
        del wl
        torch.cuda.empty_cache()
        for dt in ("bf16", "f64"):
            log("bench: fused %s storage steps" % dt.upper())
            wb = Workload(fx, torch, dt, ROWS, COLS)
            time_steps(torch, wb.fused, a.steps, a.warmup, stream)
            del wb
            torch.cuda.empty_cache()
        log("bench: 1 GiB reference copy")
        copy_ceiling(fx, torch, stream, nbytes=1 << 30, reps=1)

    cpu = None
    if not a.no_cpu:
        log("bench: CPU oracle baseline")
        cpu = cpu_baseline()
        cpu["cpu_model"] = cpu_model()
        if not a.no_extra:
            log("bench: CPU oracle on one core")
            one = cpu_baseline(cols_sample=COLS // 16, min_seconds=5.0, threads=1)
            cpu["one_core"] = {"value": one["value"], "unit": one["unit"], "sample": one["sample"]}
            log("bench: CPU oracle, vector and precision workloads")
            cpu["other_configs"] = {"all_cores": cpu_oracle_configs(),
                                    "one_core": cpu_oracle_configs(min_seconds=2.0, threads=1)}

    line = {
        "metric": "fused-expr HBM GB/s (% of peak) + speedup vs unfused, FP32 & BF16 storage",
        "value": round(value, 2),
        "unit": "GB/s",
        "pct_of_peak": round(100 * value / PEAK_HBM_GBS, 2),
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (SplitMix64 seed 2, U[-1,1])",
        "config": {"workload": "C2 matrix expressions: Z=(X+Y)%exp(-abs(W))/(1+X%X), sum(Z,0), "
                               "norm_fro(X-Y); FP32 8192x8192 column-major",
                   "rows": ROWS, "cols": COLS, "bytes_per_step": step_bytes},
        "roofline": {"bound": "hbm", "kernel": "c2_" + dominant,
                     "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic() if dominant == "z" else None,
                     "algorithmic_bytes": dominant_bytes,
                     "achieved_cold": achieved_cold,
                     "frac_cold": round(achieved_cold / PEAK_HBM_GBS, 4) if achieved_cold else None},
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
