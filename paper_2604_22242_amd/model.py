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


def init_params(F, H, C, seed=0):
    """He-uniform first layer, Glorot-uniform second, zero biases (numpy's
    seeded PCG64 generator)."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (H, F)) * math.sqrt(6.0 / F)
    W2 = rng.uniform(-1, 1, (C, H)) * math.sqrt(6.0 / (H + C))
    return np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(C)]).astype(np.float32)


def train(records, hidden=HIDDEN, epochs=400, batch=256, lr=2e-3, seed=0, verbose=False):
    import torch
    lib()
    X, Y = dataset(records)
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std[std < 1e-6] = 1.0
    m = Model(X.shape[1], hidden, HEADS)
    m.set(init_params(X.shape[1], hidden, sum(HEADS), seed), mean, std)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.from_numpy(Y).cuda()
    loss = torch.zeros(1, device="cuda")
    rng = np.random.default_rng(seed + 1)
    n = X.shape[0]
    curve = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        Xp, Yp = Xd[perm].contiguous(), Yd[perm].contiguous()
        for s in range(0, n, batch):
            m.train_step(Xp[s:s + batch], Yp[s:s + batch], lr, loss)
        if ep % 50 == 0 or ep == epochs - 1:
            torch.cuda.synchronize()
            curve.append((ep, float(loss.item())))
            if verbose:
                print("epoch %d loss %.4f" % curve[-1], flush=True)
    m.get()  # refresh the host twin
    return m, curve


def save(m: Model, path: str):
    params, mean, std = m.get()
    params.tofile(path + ".bin")
    json.dump({"n_features": m.n_features, "hidden": m.hidden, "heads": list(m.heads),
               "features": FEATURES, "mean": mean.tolist(), "std": std.tolist()},
              open(path + ".json", "w"), indent=1)


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
    vb = elem if VECS[vi] == "elem" else VECS[vi]
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


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", nargs="+", required=True)
    ap.add_argument("--heldout", nargs="*", default=[])
    ap.add_argument("--out", default=None)
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--report", default=None)
    a = ap.parse_args(argv)
    tr = [r for p in a.train for r in load_db(p).values()]
    ho = [r for p in a.heldout for r in load_db(p).values()]
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    t0 = time.time()
    m, curve = train(tr, epochs=a.epochs, verbose=True)
    rep = {"train_records": len(tr), "train_seconds": round(time.time() - t0, 1),
           "loss_curve": curve, "train_fit": evaluate(m, tr, cus)}
    if ho:
        rep["heldout"] = evaluate(m, ho, cus)
    if a.out:
        save(m, a.out)
    print(json.dumps(rep, indent=1), flush=True)
    if a.report:
        json.dump(rep, open(a.report, "w"), indent=1)


if __name__ == "__main__":
    main()
