"""CPU tests of the autotuner's configuration grid and model features."""
import math

import pytest

from synth import trees


def test_grid_shape_and_labels():
    from paper_2604_22242_amd import tune
    for red in (None, "accu", "colsum", "rowsum", "norm"):
        for dt in ("f32", "bf16"):
            g = tune.grid(red, dt)
            assert len(g) == 4 * 3 * 3 * 4 + 1 and g[-1] == (tune.DEFAULT, None)
            g = g[:-1]
            assert len({c for c, _ in g}) == len(g)
            for (b, e, v, s), (bi, ei, vi, si) in g:
                assert tune.BLOCKS[bi] == b and tune.EPTS[ei] == e
                assert v == (tune.ELEM[dt] if tune.VECS[vi] == "elem"
                             else max(tune.VECS[vi], tune.ELEM[dt]))
                assert tune.split_choices(red)[si] == s


def test_features():
    from paper_2604_22242_amd import tune
    info = {"op_count": [1, 0, 2, 1, 0, 1, 1, 0], "n_consts": 2, "depth": 4,
            "n_instructions": 6, "n_slots": 5, "n_inputs": 3}
    f = tune.features(info, "bf16", (4096, 2), "colsum")
    assert len(f) == len(tune.FEATURES)
    d = dict(zip(tune.FEATURES, f))
    assert d["log2_n"] == 13 and d["log2_rows"] == 12 and d["log2_cols"] == 1
    assert d["red_colsum"] == 1 and d["red_none"] == 0 and d["bf16"] == 1
    assert d["bytes_per_elem"] == 6 and d["transcendental"] == 2
    assert math.isclose(d["log2_bytes"], math.log2(6 * 8192))


def test_tuning_items():
    items = [trees.tuning_item(5, i) for i in range(400)]
    assert all(4096 <= it["n"] <= (1 << 28) + (1 << 15) for it in items)
    assert all(it["shape"][0] * it["shape"][1] == it["n"] for it in items)
    assert {it["dtype"] for it in items} == {"f32", "bf16"}
    assert trees.tuning_item(5, 7) == trees.tuning_item(5, 7)
    assert trees.tuning_item(6, 7) != trees.tuning_item(5, 7)


def test_noise_summary_recovers_a_known_spread():
    # two independent measurements per cell, each with 3% lognormal noise:
    # the estimate from their relative differences returns about 3%
    import numpy as np
    from paper_2604_22242_amd.tune import noise_summary
    rng = np.random.default_rng(1)
    true = rng.uniform(0.01, 1.0, 20000)
    a = true * np.exp(rng.normal(0, 0.03, true.size))
    b = true * np.exp(rng.normal(0, 0.03, true.size))
    rep = noise_summary(list(zip(a, b)))
    assert rep["cells"] == true.size
    assert abs(rep["cv_estimate"] - 0.03) < 0.002, rep
    assert abs(rep["median_ratio"] - 1.0) < 0.002
    # identical re-times: no spread; unusable cells are skipped
    rep = noise_summary([(1.0, 1.0), (2.0, 2.0), (float("nan"), 1.0), (0.0, 1.0)])
    assert rep["cells"] == 2 and rep["cv_estimate"] == 0.0 and rep["within_2pct"] == 1.0
    assert noise_summary([])["cells"] == 0


def test_native_grid_matches_the_driver():
    # the C library's grid (fx_autotune's search space) and the Python
    # driver's are the same configurations in the same order; no device:
    # 256 CUs assumed by both
    import os
    import paper_2604_22242_amd as fx
    if not os.path.exists(fx.LIB_PATH):
        from paper_2604_22242_amd import build
        build.build()
    from paper_2604_22242_amd import tune
    kinds = {None: 0, "accu": fx.R_ACCU, "colsum": fx.R_COLSUM, "rowsum": fx.R_ROWSUM,
             "norm": fx.R_NORM}
    for red, kind in kinds.items():
        for dt, code in (("f32", fx.F32), ("bf16", fx.BF16)):
            assert fx.fx_tune_grid(kind, code) == [c for c, _ in tune.grid(red, dt)], (red, dt)


def test_native_features_match_the_driver():
    # fx_tape_features (C, host only) and the driver's features() give the
    # model the same inputs, for generated trees of every kind and both
    # storage types
    import numpy as np
    import paper_2604_22242_amd as fx
    from paper_2604_22242_amd import tune
    codes = {"f32": fx.F32, "bf16": fx.BF16}
    kinds = {None: 0, "accu": fx.R_ACCU, "colsum": fx.R_COLSUM, "rowsum": fx.R_ROWSUM,
             "norm": fx.R_NORM}
    for i in range(40):
        item = trees.tuning_item(5, i)
        tape = fx.Tape(item["nodes"])
        got = fx.fx_tape_features(tape, codes[item["dtype"]], item["shape"], kinds[item["reduce"]])
        want = tune.features(tape.info(), item["dtype"], item["shape"], item["reduce"])
        assert np.array_equal(np.float32(got), np.float32(want)), (i, got, want)
    # element-wise results and full reductions are flat: a matrix shape gives
    # the features of its n x 1 vector (the shape every tuning item of those
    # kinds has), in C and in the driver alike; dimension sums keep the shape
    tape = fx.Tape(trees.tuning_item(5, 0)["nodes"])
    for red in (None, "accu", "colsum", "rowsum", "norm"):
        got = fx.fx_tape_features(tape, fx.F32, (8192, 4096), kinds[red])
        flat = fx.fx_tape_features(tape, fx.F32, (8192 * 4096, 1), kinds[red])
        want = tune.features(tape.info(), "f32", (8192, 4096), red)
        assert np.array_equal(np.float32(got), np.float32(want)), red
        assert np.array_equal(np.float32(got), np.float32(flat)) == (red not in ("colsum", "rowsum"))


def test_model_file_layout(tmp_path):
    # the FXM1 file the C loader reads: header, standardisation, parameters
    import struct
    import numpy as np
    from paper_2604_22242_amd import model
    p = tmp_path / "m.fxm"
    model.write_fxm(str(p), 3, 2, (2, 2), [1, 2, 3], [4, 5, 6], np.arange(16, dtype=np.float32))
    b = p.read_bytes()
    assert b[:4] == b"FXM1" and struct.unpack("<5i", b[4:24]) == (3, 2, 2, 2, 2)
    assert struct.unpack("<6f", b[24:48]) == (1, 2, 3, 4, 5, 6)
    assert struct.unpack("<i", b[48:52]) == (16,) and len(b) == 52 + 64
    # the committed model's file matches its parameter and JSON files
    import json, os
    base = os.path.join(os.path.dirname(model.__file__), "launch_model")
    meta = json.load(open(base + ".json"))
    c = open(base + ".fxm", "rb").read()
    F, H, nh = struct.unpack("<3i", c[4:16])
    assert (F, H, list(struct.unpack("<%di" % nh, c[16:16 + 4 * nh]))) == (
        meta["n_features"], meta["hidden"], meta["heads"])
    params = np.fromfile(base + ".bin", np.float32)
    assert c.endswith(params.tobytes())


def test_count_returning_calls_report_errors_as_negative_status():
    # fx_tune_grid and fx_tape_features return a count, so their errors are
    # negative fx_status values (never a count the caller could use)
    import paper_2604_22242_amd as fx
    L = fx.lib()
    assert L.fx_tune_grid(0, fx.U32, None, 0) == -3        # FX_E_DTYPE
    assert L.fx_tune_grid(99, fx.F32, None, 0) == -1       # FX_E_ARG
    assert L.fx_tune_grid(0, fx.F32, None, 0) == 145
    tape = fx.Tape([("leaf", -1, -1, 0, 0.0), ("exp", 0, -1, -1, 0.0)])
    shape = fx.Shape(100, 1)
    assert L.fx_tape_features(tape.handle, fx.U32, shape, 0, None, 0) == -3
    assert L.fx_tape_features(None, fx.F32, shape, 0, None, 0) == -1
    assert L.fx_tape_features(tape.handle, fx.F32, shape, fx.R_DOT, None, 0) == -1
    assert L.fx_tape_features(tape.handle, fx.F32, shape, 0, None, 0) == 25
    for call in (lambda: fx.fx_tune_grid(0, fx.U32),
                 lambda: fx.fx_tape_features(tape, fx.U32, (100, 1), 0)):
        with pytest.raises(fx.FxError) as ei:
            call()
        assert ei.value.code == 3
