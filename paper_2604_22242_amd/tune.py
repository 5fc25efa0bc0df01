"""Exhaustive autotuner of launch configurations, and the features the
learned cost model reads.

The timing itself is native (fx_tune_time: HIP events around each launch on
the stream); this module chooses the configuration grid, runs the search
(exhaustive, or successive halving for cheap training labels), and keeps an
append-only JSONL timing database that a re-run resumes (keys already
present are skipped).

    python -m paper_2604_22242_amd.tune --set train --start 0 --count 1000 \
        --db tune_train.jsonl --mode halving
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

from . import (BF16, F32, R_ACCU, R_COLSUM, R_NORM, R_ROWSUM, Tape, fx_tune_time,
               fx_workspace_bytes, lib)

BLOCKS = (64, 128, 256, 512)
EPTS = (1, 2, 4)
VECS = ("elem", 8, 16)
KIND = {None: 0, "accu": R_ACCU, "colsum": R_COLSUM, "rowsum": R_ROWSUM, "norm": R_NORM}
DTYPE = {"f32": F32, "bf16": BF16}
ELEM = {"f32": 4, "bf16": 2}


def split_choices(reduce, cus=256):
    """Four values of the `split` knob per reduction kind (0 = library
    default: one tile per block for element-wise, the heuristics otherwise)."""
    if reduce is None:
        return (0, 2 * cus, 8 * cus, 32 * cus)
    if reduce in ("accu", "norm"):
        return (cus, 2 * cus, 4 * cus, 8 * cus)
    if reduce == "colsum":
        return (0, 1, 4, 16)
    return (0, 16, 64, 256)


DEFAULT = (0, 0, 0, 0)  # the library's own choice (timed for comparison, never a label)


def grid(reduce, dtype, cus=256):
    """All configurations: list of ((block, ept, vec_bytes, split), labels)
    where labels are the class index of each knob; the last entry is the
    library default with labels None."""
    out = []
    for bi, b in enumerate(BLOCKS):
        for ei, e in enumerate(EPTS):
            for vi, v in enumerate(VECS):
                vb = ELEM[dtype] if v == "elem" else max(v, ELEM[dtype])
                for si, s in enumerate(split_choices(reduce, cus)):
                    out.append(((b, e, vb, s), (bi, ei, vi, si)))
    out.append((DEFAULT, None))
    return out


HEADS = (len(BLOCKS), len(EPTS), len(VECS), 4)
FEATURES = ["add", "sub", "mul", "div", "neg", "abs", "exp", "sqrt", "consts", "depth",
            "instructions", "slots", "inputs", "bf16", "log2_n", "log2_rows", "log2_cols",
            "red_none", "red_accu", "red_colsum", "red_rowsum", "red_norm", "bytes_per_elem",
            "transcendental", "log2_bytes"]


def features(info: dict, dtype: str, shape, reduce) -> list:
    """The model's input vector for one (tree, size, dtype, reduction)."""
    oc = info["op_count"]
    rows, cols = shape
    if reduce in (None, "accu", "norm"):
        # element-wise results and full reductions see one flat vector
        rows, cols = rows * cols, 1
    n = max(1, rows * cols)
    bpe = ELEM[dtype] * (info["n_inputs"] + (1 if reduce is None else 0))
    red = [1.0 if reduce == r else 0.0 for r in (None, "accu", "colsum", "rowsum", "norm")]
    return [float(c) for c in oc] + [
        float(info["n_consts"]), float(info["depth"]), float(info["n_instructions"]),
        float(info["n_slots"]), float(info["n_inputs"]), 1.0 if dtype == "bf16" else 0.0,
        math.log2(n), math.log2(max(1, rows)), math.log2(max(1, cols))] + red + [
        float(bpe), float(oc[3] + oc[6] + oc[7]), math.log2(max(1, bpe * n))]


def key_of(item) -> str:
    h = hashlib.sha1(json.dumps(item["nodes"]).encode()).hexdigest()[:16]
    return "%s:%dx%d:%s:%s" % (h, item["shape"][0], item["shape"][1], item["dtype"], item["reduce"])


class Pool:
    """Input, output and workspace buffers reused by every timed item (the
    values are seeded U[-1,1]; timing does not depend on them)."""

    def __init__(self, max_n=(1 << 28) + (1 << 16), dtypes=("f32", "bf16")):
        import torch
        import synth
        self.torch = torch
        self.max_n = max_n
        self.inputs, self.out = {}, None
        for dt in dtypes:
            bufs = []
            for q in range(4):
                h = synth.fill(5, 100 + q, max_n, dt)
                t = torch.from_numpy(h)
                if dt == "bf16":
                    t = t.view(torch.int16).view(torch.bfloat16)
                bufs.append(t.cuda())
                del h
            self.inputs[dt] = bufs
        self.out = torch.empty(max_n * 4 + 4096, dtype=torch.uint8, device="cuda")
        self.ws = torch.zeros(64 << 20, dtype=torch.uint8, device="cuda")

    def views(self, dt, n, k):
        return [b[:n] for b in self.inputs[dt][:k]]


def tune_item(item, pool, mode="exhaustive", warmup=2, reps=5, cus=256):
    """Time every configuration of the grid for one item.  Returns a record
    for the timing database."""
    tape = Tape(item["nodes"])
    info = tape.info()
    dt, red, shape = item["dtype"], item["reduce"], item["shape"]
    n = shape[0] * shape[1]
    kind = KIND[red]
    cfgs = grid(red, dt, cus)
    ins = pool.views(dt, n, item["n_inputs"])
    ws_need = max(fx_workspace_bytes(kind, DTYPE[dt], shape, c) for c, _ in cfgs) if kind else 0
    assert ws_need <= pool.ws.numel(), "workspace pool too small"
    ws = pool.ws if kind else None

    def timed(idx, r):
        t = fx_tune_time(tape, ins, pool.out, shape, kind, [cfgs[i][0] for i in idx], ws=ws,
                         warmup=warmup, reps=r, dt=DTYPE[dt])
        return {i: (statistics.median(v) if not any(math.isnan(x) for x in v) else float("nan"))
                for i, v in zip(idx, t)}

    t0 = time.perf_counter()
    if mode == "exhaustive":
        med = timed(list(range(len(cfgs))), reps)
    else:  # successive halving: 1 rep for all, 3 for the best quarter, 5 for the best 4
        med = timed(list(range(len(cfgs))), 1)
        alive = sorted((i for i in med if not math.isnan(med[i])), key=lambda i: med[i])
        alive = alive[:max(4, len(alive) // 4)]
        med.update(timed(alive, 3))
        alive = sorted(alive, key=lambda i: med[i])[:4]
        med.update(timed(alive, reps))
    if len(cfgs) - 1 not in med:  # the default is always timed fully
        med.update(timed([len(cfgs) - 1], reps))
    ok = [i for i in med if not math.isnan(med[i]) and cfgs[i][1] is not None]
    best = min(ok, key=lambda i: med[i])
    r4 = lambda v: float("%.4g" % v)
    return {"key": key_of(item), "id": item["id"], "seed": item["seed"], "dtype": dt,
            "reduce": red, "shape": list(shape), "info": info, "cus": cus,
            "features": [r4(v) for v in features(info, dt, shape, red)],
            "ms": [r4(med[i]) if i in med else None for i in range(len(cfgs))],
            "best": best, "best_ms": med[best], "default_ms": med[len(cfgs) - 1], "mode": mode,
            "tune_seconds": round(time.perf_counter() - t0, 4)}


def retime_default(rec, pool, warmup=2, reps=5):
    """A copy of a database record whose library-default time is measured
    again (after a change of the library's default heuristics); the grid's
    other timings are kept."""
    from synth import trees
    item = trees.tuning_item(rec["seed"], rec["id"])
    assert key_of(item) == rec["key"], "record does not match its generated item"
    tape = Tape(item["nodes"])
    dt, red, shape = item["dtype"], item["reduce"], item["shape"]
    n = shape[0] * shape[1]
    kind = KIND[red]
    ws = pool.ws if kind else None
    t = fx_tune_time(tape, pool.views(dt, n, item["n_inputs"]), pool.out, shape, kind, [DEFAULT],
                     ws=ws, warmup=warmup, reps=reps, dt=DTYPE[dt])[0]
    out = dict(rec)
    out["default_ms"] = statistics.median(t)
    out["ms"] = list(rec["ms"][:-1]) + [float("%.4g" % out["default_ms"])]
    out["default_retimed"] = True
    return out


def noise_summary(pairs) -> dict:
    """Timing noise from (first, second) measurements of the same cells.
    With independent errors of relative spread c in each, the relative
    difference d = t2/t1 - 1 spreads by about c * sqrt(2); the robust
    estimate uses the median absolute deviation (x 1.4826 for a normal
    spread)."""
    import numpy as np
    t1 = np.array([a for a, _ in pairs], float)
    t2 = np.array([b for _, b in pairs], float)
    ok = np.isfinite(t1) & np.isfinite(t2) & (t1 > 0)
    d = t2[ok] / t1[ok] - 1.0
    if d.size == 0:
        return {"cells": 0}
    mad = float(np.median(np.abs(d - np.median(d))))
    return {"cells": int(d.size),
            "median_ratio": round(float(np.median(d)) + 1.0, 4),
            "cv_estimate": round(1.4826 * mad / math.sqrt(2.0), 4),
            "within_2pct": round(float(np.mean(np.abs(d) <= 0.02)), 4),
            "within_5pct": round(float(np.mean(np.abs(d) <= 0.05)), 4)}


def retime_noise(recs, pool, frac=0.01, seed=0, warmup=2, reps=5, progress=None):
    """Re-time every record's argmin and a random `frac` of its other grid
    cells (seeded), against the times stored at collection.  The argmin is
    the least of many noisy times, so its re-time also shows how much of a
    winning margin is luck."""
    import random
    from synth import trees
    rng = random.Random(seed)
    best_pairs, sample_pairs, still_best = [], [], []
    t0 = time.time()
    for k, rec in enumerate(recs):
        item = trees.tuning_item(rec["seed"], rec["id"])
        assert key_of(item) == rec["key"], "record does not match its generated item"
        cfgs = record_grid(rec)
        cells = [rec["best"]] + [i for i in range(len(cfgs) - 1)
                                 if i != rec["best"] and rec["ms"][i] is not None
                                 and rec["ms"][i] == rec["ms"][i] and rng.random() < frac]
        tape = Tape(item["nodes"])
        dt, red, shape = item["dtype"], item["reduce"], item["shape"]
        kind = KIND[red]
        t = fx_tune_time(tape, pool.views(dt, shape[0] * shape[1], item["n_inputs"]), pool.out,
                         shape, kind, [cfgs[i][0] for i in cells], ws=pool.ws if kind else None,
                         warmup=warmup, reps=reps, dt=DTYPE[dt])
        med = [statistics.median(v) for v in t]
        best_pairs.append((rec["best_ms"], med[0]))
        still_best.append(med[0] <= 1.05 * min(x for x in rec["ms"][:-1]
                                               if x is not None and x == x))
        sample_pairs += [(rec["ms"][i], m) for i, m in zip(cells[1:], med[1:])]
        if progress and k % progress == 0:
            print("noise %d/%d  %.0fs" % (k, len(recs), time.time() - t0), flush=True)
    return {"records": len(recs), "sample_fraction": frac,
            "argmin": noise_summary(best_pairs),
            "argmin_within_1.05_of_stored_best": round(sum(still_best) / max(1, len(still_best)), 4),
            "random_cells": noise_summary(sample_pairs)}


def record_grid(r):
    """The (config, labels) grid a database record's times refer to."""
    return grid(r["reduce"], r["dtype"], r.get("cus", 256))


def load_db(path):
    recs = {}
    if os.path.exists(path):
        for line in open(path):
            line = line.strip()
            if line:
                r = json.loads(line)
                recs[r["key"]] = r
    return recs


def main(argv=None):
    from synth import trees
    ap = argparse.ArgumentParser()
    ap.add_argument("--set", choices=("train", "heldout"), default="train")
    ap.add_argument("--start", type=int, default=0)
    ap.add_argument("--count", type=int, default=100)
    ap.add_argument("--db", required=True)
    ap.add_argument("--mode", choices=("exhaustive", "halving"), default=None)
    ap.add_argument("--max-n", type=int, default=(1 << 28) + (1 << 16))
    ap.add_argument("--retime-default", default=None, metavar="IN_DB",
                    help="re-measure the library-default time of every record of IN_DB "
                         "into --db")
    ap.add_argument("--noise", nargs="+", default=None, metavar="IN_DB",
                    help="re-time every record's argmin and a random --frac of its cells; "
                         "write the noise report to --db")
    ap.add_argument("--frac", type=float, default=0.01)
    a = ap.parse_args(argv)
    if a.noise:
        lib()
        recs = [r for p in a.noise for r in load_db(p).values()]
        rep = retime_noise(recs, Pool(a.max_n), frac=a.frac, progress=200)
        json.dump(rep, open(a.db, "w"), indent=1)
        print(json.dumps(rep, indent=1), flush=True)
        return 0
    if a.retime_default:
        lib()
        recs = list(load_db(a.retime_default).values())
        pool = Pool(a.max_n)
        t0 = time.time()
        with open(a.db, "w") as f:
            for k, r in enumerate(recs):
                f.write(json.dumps(retime_default(r, pool)) + "\n")
                if k % 200 == 0:
                    print("retime %d/%d  %.0fs" % (k, len(recs), time.time() - t0), flush=True)
        print("retime done %d records in %.0fs" % (len(recs), time.time() - t0), flush=True)
        return 0
    seed = 5 if a.set == "train" else 6
    mode = a.mode or ("halving" if a.set == "train" else "exhaustive")
    lib()
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    done = load_db(a.db)
    pool = Pool(a.max_n)
    t0 = time.time()
    with open(a.db, "a") as f:
        for i in range(a.start, a.start + a.count):
            item = trees.tuning_item(seed, i)
            if item["n"] > a.max_n or key_of(item) in done:
                continue
            rec = tune_item(item, pool, mode, cus=cus)
            f.write(json.dumps(rec) + "\n")
            f.flush()
            if (i - a.start) % 100 == 0:
                print("tune %s %d/%d  %.0fs" % (a.set, i - a.start, a.count, time.time() - t0),
                      flush=True)
    print("tune done %d items in %.0fs" % (a.count, time.time() - t0), flush=True)


if __name__ == "__main__":
    sys.exit(main())
