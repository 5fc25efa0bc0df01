"""CPU checks of the committed launch-configuration model: its files are
consistent, and a numpy forward pass over the documented parameter layout
reproduces the choice reported for the matrix workload."""
import json
import os

import numpy as np

from paper_2604_22242_amd import model, tune

HERE = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PATH = os.path.join(HERE, "paper_2604_22242_amd", "launch_model")


def _load():
    meta = json.load(open(PATH + ".json"))
    p = np.fromfile(PATH + ".bin", np.float32)
    F, H, heads = meta["n_features"], meta["hidden"], meta["heads"]
    C = sum(heads)
    assert p.size == H * F + H + C * H + C
    W1 = p[:H * F].reshape(H, F)
    b1 = p[H * F:H * F + H]
    W2 = p[H * F + H:H * F + H + C * H].reshape(C, H)
    b2 = p[H * F + H + C * H:]
    return meta, W1, b1, W2, b2


def choose(x):
    meta, W1, b1, W2, b2 = _load()
    z = (np.asarray(x, np.float32) - np.array(meta["mean"], np.float32)) / np.array(meta["std"], np.float32)
    h = np.maximum(W1 @ z + b1, 0)
    logits = W2 @ h + b2
    out, o = [], 0
    for k in meta["heads"]:
        out.append(int(np.argmax(logits[o:o + k])))
        o += k
    return tuple(out)


def test_model_files():
    meta, *_ = _load()
    assert meta["n_features"] == len(tune.FEATURES) == 25 and meta["hidden"] == 64
    assert tuple(meta["heads"]) == tune.HEADS and meta["features"] == tune.FEATURES
    assert all(s > 0 for s in meta["std"])


def test_choice_for_the_matrix_workload():
    import paper_2604_22242_amd as fx
    info = fx.Tape(model.C2_NODES).info()
    ch = choose(tune.features(info, "f32", (8192, 8192), None))
    # the evaluation report's pick for the fused Z: 64 threads, EPT 1, 16 B,
    # one tile per block
    assert model.config_of(ch, None, "f32") == (64, 1, 16, 0)


def test_unused_features_carry_no_weight():
    # the training trees never hold a neg node (exp(-|a|) is built as
    # 0 - |a|), so that count is 0 on every training row: its first-layer
    # weights start at zero and get no gradient, and a tree that does hold
    # one (the matrix workload's exp(-|W|)) is scored as if it had none
    meta, W1, *_ = _load()
    neg = meta["features"].index("neg")
    assert meta["std"][neg] == 1.0 and meta["mean"][neg] == 0.0
    assert not W1[:, neg].any()
    p = model.init_params(5, 4, 3, seed=1, constant=[2])
    W = p[:20].reshape(4, 5)
    assert not W[:, 2].any() and W[:, [0, 1, 3, 4]].all()
