"""Train and evaluate the learned launch-configuration model.

Training data are autotuner timing databases (tune.py): each record gives
the model's features and, for every configuration of the grid, its median
time; the label is the class of each knob in the fastest configuration.
Training runs on the GPU (fx_model_train_step: hand-written forward,
backward and Adam kernels); single queries use the host twin
(fx_model_choose).

    python -m paper_2604_22242_amd.model --train a.jsonl b.jsonl \
        --heldout c.jsonl --out profiles/launch_model

A trained model is saved as <out>.bin (flat FP32 parameters) and
<out>.json (dimensions, heads, feature standardisation).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from . import Model, lib
from .tune import BLOCKS, EPTS, FEATURES, HEADS, VECS, load_db, record_grid, split_choices

HIDDEN = 64


def dataset(records):
    X = np.array([r["features"] for r in records], np.float32)
    Y = np.array([record_grid(r)[r["best"]][1] for r in records], np.int32)
    return X, Y


def init_params(F, H, C, seed=0, constant=()):
    """He-uniform first layer, Glorot-uniform second, zero biases (numpy's
    seeded PCG64 generator).  The first-layer weights of the `constant`
    features start at zero: such a feature standardises to 0 on every
    training row, so its weights get no gradient and would keep their random
    start, which a query with another value of that feature (the operator
    count of an operator the training trees never use) would then feed
    through unchanged."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (H, F)) * math.sqrt(6.0 / F)
    W1[:, list(constant)] = 0.0
    W2 = rng.uniform(-1, 1, (C, H)) * math.sqrt(6.0 / (H + C))
    return np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(C)]).astype(np.float32)


def train(records, hidden=HIDDEN, epochs=400, batch=256, lr=2e-3, seed=0, verbose=False):
    import torch
    lib()
    X, Y = dataset(records)
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    constant = np.flatnonzero(std < 1e-6)
    std[constant] = 1.0
    m = Model(X.shape[1], hidden, HEADS)
    m.set(init_params(X.shape[1], hidden, sum(HEADS), seed, constant), mean, std)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.from_numpy(Y).cuda()
    rng = np.random.default_rng(seed + 1)
    n = X.shape[0]
    perm = np.stack([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)
    losses = torch.zeros(max(1, epochs), device="cuda")
    m.train(Xd, Yd, epochs, batch, lr, perm, losses)  # the whole loop in fx_model_train
    losses = losses.cpu().tolist()
    curve = [(ep, losses[ep]) for ep in range(epochs) if ep % 50 == 0 or ep == epochs - 1]
    if verbose:
        for c in curve:
            print("epoch %d loss %.4f" % c, flush=True)
    m.get()  # refresh the host twin
    return m, curve


def write_fxm(path: str, n_features, hidden, heads, mean, std, params):
    """The self-contained model file the C loader reads (fx_model_load):
    "FXM1", int32 n_features, hidden, n_heads, head sizes; float32 means,
    standard deviations; int32 parameter count; float32 parameters."""
    import struct
    with open(path, "wb") as f:
        f.write(b"FXM1" + struct.pack("<3i", n_features, hidden, len(heads)))
        f.write(struct.pack("<%di" % len(heads), *heads))
        f.write(np.asarray(mean, np.float32).tobytes() + np.asarray(std, np.float32).tobytes())
        f.write(struct.pack("<i", len(params)) + np.asarray(params, np.float32).tobytes())


def save(m: Model, path: str):
    params, mean, std = m.get()
    params.tofile(path + ".bin")
    json.dump({"n_features": m.n_features, "hidden": m.hidden, "heads": list(m.heads),
               "features": FEATURES, "mean": mean.tolist(), "std": std.tolist()},
              open(path + ".json", "w"), indent=1)
    write_fxm(path + ".fxm", m.n_features, m.hidden, m.heads, mean, std, params)


def load(path: str) -> Model:
    meta = json.load(open(path + ".json"))
    m = Model(meta["n_features"], meta["hidden"], meta["heads"])
    params = np.fromfile(path + ".bin", np.float32)
    m.set(params, np.array(meta["mean"], np.float32), np.array(meta["std"], np.float32))
    return m


def config_of(choice, reduce, dtype, cus=256):
    """The launch configuration a model choice stands for."""
    bi, ei, vi, si = choice
    elem = 4 if dtype == "f32" else 2
    vb = elem if VECS[vi] == "elem" else max(VECS[vi], elem)
    return (BLOCKS[bi], EPTS[ei], vb, split_choices(reduce, cus)[si])


def evaluate(m: Model, records, cus=256):
    """Predicted configuration against the exhaustive best and the library
    default, measured on the records' own timings."""
    ratios, dratios, lat = [], [], []
    missing = 0
    for r in records:
        t0 = time.perf_counter()
        ch = m.choose(r["features"])
        lat.append(time.perf_counter() - t0)
        cfg = config_of(ch, r["reduce"], r["dtype"], r.get("cus", cus))
        cfgs = [c for c, _ in record_grid(r)]
        t = r["ms"][cfgs.index(cfg)] if cfg in cfgs else None
        if t is None or not (t == t):
            missing += 1
            t = r["default_ms"]
        ratios.append(t / r["best_ms"])
        dratios.append(r["default_ms"] / r["best_ms"])
    ratios, dratios = np.array(ratios), np.array(dratios)
    geo = lambda a: float(np.exp(np.mean(np.log(a))))
    sweep = np.array([r["tune_seconds"] for r in records])
    return {"records": len(records),
            "model_geomean_vs_best": round(geo(ratios), 4),
            "model_within_1.05": round(float(np.mean(ratios <= 1.05)), 4),
            "model_within_1.10": round(float(np.mean(ratios <= 1.10)), 4),
            "default_geomean_vs_best": round(geo(dratios), 4),
            "default_within_1.05": round(float(np.mean(dratios <= 1.05)), 4),
            "default_within_1.10": round(float(np.mean(dratios <= 1.10)), 4),
            "choose_us_median": round(float(np.median(lat)) * 1e6, 2),
            "exhaustive_sweep_s_median": round(float(np.median(sweep)), 4),
            "choose_speedup_vs_sweep": round(float(np.median(sweep) / np.median(lat)), 1),
            "unmeasured_predictions": missing}


# The matrix workload's expression trees (Z = (X+Y) % exp(-abs(W)) / (1 + X%X),
# and X - Y for the norm) as node lists, for the model's features.
C2_NODES = [("leaf", -1, -1, 0, 0.0), ("leaf", -1, -1, 1, 0.0), ("add", 0, 1, -1, 0.0),
            ("leaf", -1, -1, 2, 0.0), ("abs", 3, -1, -1, 0.0), ("neg", 4, -1, -1, 0.0),
            ("exp", 5, -1, -1, 0.0), ("mul", 2, 6, -1, 0.0), ("const", -1, -1, -1, 1.0),
            ("mul", 0, 0, -1, 0.0), ("add", 8, 9, -1, 0.0), ("div", 7, 10, -1, 0.0)]
DIFF_NODES = [("leaf", -1, -1, 0, 0.0), ("leaf", -1, -1, 1, 0.0), ("sub", 0, 1, -1, 0.0)]


def et_check(m: Model, cus: int, rows=8192, cols=8192, reps=5):
    """Transfer check: the model (trained on run-time tapes) picks launch
    configurations for the compile-time kernels of the FP32 matrix workload;
    each result's whole grid is timed to find its own best."""
    import statistics
    import torch
    import synth
    from . import (R_COLSUM, R_NORM, STATUS, FxError, Tape, fx_c2_colsum, fx_c2_z,
                   fx_norm_fro_diff, fx_workspace_bytes, F32)
    unsupported = next(k for k, v in STATUS.items() if v == "FX_E_UNSUPPORTED")
    from .tune import features, grid
    shape, n = (rows, cols), rows * cols
    X, Y, W = [torch.from_numpy(synth.fill(2, t, n, "f32")).cuda() for t in range(3)]
    Z = torch.empty(n, device="cuda")
    cs = torch.empty(cols, device="cuda")
    nrm = torch.zeros(1, dtype=torch.float64, device="cuda")
    runs = {"z": (C2_NODES, None, 0, lambda c, ws: fx_c2_z(X, Y, W, Z, shape, cfg=c)),
            "colsum": (C2_NODES, "colsum", R_COLSUM,
                       lambda c, ws: fx_c2_colsum(X, Y, W, cs, shape, ws, cfg=c)),
            "norm": (DIFF_NODES, "norm", R_NORM,
                     lambda c, ws: fx_norm_fro_diff(X, Y, nrm, shape, ws, cfg=c))}
    out = {}
    for name, (nodes, red, kind, fn) in runs.items():
        cfgs = [c for c, _ in grid(red, "f32", cus)]
        wsb = max(fx_workspace_bytes(kind, F32, shape, c) for c in cfgs) if kind else 0
        ws = torch.zeros(max(wsb, 8), dtype=torch.uint8, device="cuda") if kind else None
        times = []
        for c in cfgs:
            try:  # the compile-time kernels take no 8-byte vectors (tapes do)
                fn(c, ws)
            except FxError as e:
                if e.code != unsupported:
                    raise
                times.append(float("inf"))
                continue
            fn(c, ws)
            ev = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                fn(c, ws)
                b.record()
                ev.append((a, b))
            torch.cuda.synchronize()
            times.append(statistics.median(a.elapsed_time(b) for a, b in ev))
        info = Tape(nodes).info()
        pick = config_of(m.choose(features(info, "f32", shape, red)), red, "f32", cus)
        best = min(times)
        mt = times[cfgs.index(pick)]  # inf: a pick the compile-time kernel is not compiled for
        out[name] = {"best_ms": round(best, 5), "best_config": list(cfgs[times.index(best)]),
                     "model_config": list(pick), "model_ms": None if mt == float("inf") else round(mt, 5),
                     "model_vs_best": None if mt == float("inf") else round(mt / best, 4),
                     "default_ms": round(times[-1], 5),
                     "default_vs_best": round(times[-1] / best, 4)}
    return out


def attached_check(path, start, count, warmup=2, reps=5):
    """End to end: held-out tuning items (seed 6) evaluated by fx_tape_eval
    with the model file at `path` attached to the tape, and without it (the
    interpreter defaults); each the median of `reps` event-timed launches
    after `warmup`.  Returns the geometric-mean speedup and per-kind ones."""
    import statistics
    import torch
    from synth import trees
    from . import Tape, fx_model_load, fx_tape_eval
    from .tune import DTYPE, KIND, Pool
    model = fx_model_load(path)
    pool = Pool()
    stream = torch.cuda.current_stream()

    def timed(tape, ins, shape, kind, dt):
        run = lambda: fx_tape_eval(tape, ins, pool.out, shape, kind, pool.ws if kind else None,
                                   dt=dt, stream=stream)
        for _ in range(warmup):
            run()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            run()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return statistics.median(ts)

    ratios, by_kind = [], {}
    for i in range(start, start + count):
        it = trees.tuning_item(6, i)
        kind, dt = KIND[it["reduce"]], DTYPE[it["dtype"]]
        n = it["shape"][0] * it["shape"][1]
        ins = pool.views(it["dtype"], n, it["n_inputs"])
        plain, attached = Tape(it["nodes"]), Tape(it["nodes"])
        attached.set_model(model)
        if i % 2:  # alternate which runs first
            ta = timed(attached, ins, it["shape"], kind, dt)
            tp = timed(plain, ins, it["shape"], kind, dt)
        else:
            tp = timed(plain, ins, it["shape"], kind, dt)
            ta = timed(attached, ins, it["shape"], kind, dt)
        r = tp / ta
        ratios.append(r)
        by_kind.setdefault("%s/%s" % (it["reduce"], it["dtype"]), []).append(r)
    gm = lambda v: math.exp(sum(math.log(x) for x in v) / len(v))
    return {"items": len(ratios), "speedup_geomean": round(gm(ratios), 4),
            "faster_by_5pct": round(sum(r > 1.05 for r in ratios) / len(ratios), 4),
            "slower_by_5pct": round(sum(r < 1 / 1.05 for r in ratios) / len(ratios), 4),
            "by_kind": {k: {"items": len(v), "speedup_geomean": round(gm(v), 4)}
                        for k, v in sorted(by_kind.items())}}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", nargs="+", default=[])
    ap.add_argument("--model", default=None,
                    help="evaluate this saved model (path without suffix) instead of training")
    ap.add_argument("--heldout", nargs="*", default=[])
    ap.add_argument("--out", default=None)
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--report", default=None)
    ap.add_argument("--attached", type=int, nargs=2, metavar=("START", "COUNT"), default=None,
                    help="with --model: time held-out items through tapes with the model "
                         "attached against the interpreter defaults")
    ap.add_argument("--et-check", action="store_true",
                    help="also apply the model to the compile-time matrix-workload kernels")
    a = ap.parse_args(argv)
    if bool(a.train) == bool(a.model):
        ap.error("give either --train databases or a saved --model")
    tr = [r for p in a.train for r in load_db(p).values()]
    ho = [r for p in a.heldout for r in load_db(p).values()]
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    if a.model:
        m = load(a.model)
        rep = {"model": a.model}
    else:
        t0 = time.time()
        m, curve = train(tr, epochs=a.epochs, verbose=True)
        rep = {"train_records": len(tr), "train_seconds": round(time.time() - t0, 1),
               "loss_curve": curve, "train_fit": evaluate(m, tr, cus)}
    if ho:
        rep["heldout"] = evaluate(m, ho, cus)
    if a.et_check:
        rep["compile_time_kernels"] = et_check(m, cus)
    if a.attached:
        if not a.model:
            ap.error("--attached needs --model")
        rep["attached"] = attached_check(a.model + ".fxm", *a.attached)
    if a.out:
        save(m, a.out)
    print(json.dumps(rep, indent=1), flush=True)
    if a.report:
        json.dump(rep, open(a.report, "w"), indent=1)


if __name__ == "__main__":
    main()
