"""GPU tests of the learned cost model's hand-written kernels against CPU
references that share nothing with them: numpy float64 forward, torch CPU
autograd gradients, central finite differences, a numpy Adam step."""
import numpy as np
import pytest

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu

F, H, HEADS = 25, 64, (4, 2, 2, 4)
C = sum(HEADS)


def _params(rng):
    W1 = rng.uniform(-1, 1, (H, F)) / np.sqrt(F)
    b1 = rng.uniform(-0.1, 0.1, H)
    W2 = rng.uniform(-1, 1, (C, H)) / np.sqrt(H)
    b2 = rng.uniform(-0.1, 0.1, C)
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2]).astype(np.float32)


def _unpack(p):
    p = p.astype(np.float64)
    o = 0
    W1 = p[o:o + H * F].reshape(H, F); o += H * F
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + C * H].reshape(C, H); o += C * H
    b2 = p[o:o + C]
    return W1, b1, W2, b2


def _forward64(p, X, mean, std):
    W1, b1, W2, b2 = _unpack(p)
    xn = (X.astype(np.float64) - mean) / std
    h = np.maximum(xn @ W1.T + b1, 0)
    return h @ W2.T + b2


def _loss64(p, X, y, mean, std):
    logits = _forward64(p, X, mean, std)
    L, o = 0.0, 0
    for q, k in enumerate(HEADS):
        z = logits[:, o:o + k]
        m = z.max(axis=1, keepdims=True)
        lse = (m[:, 0] + np.log(np.exp(z - m).sum(axis=1)))
        L += np.mean(lse - z[np.arange(len(y)), y[:, q]])
        o += k
    return L


def _data(rng, B):
    X = rng.normal(size=(B, F)).astype(np.float32) * 3 + 1
    y = np.stack([rng.integers(0, k, B) for k in HEADS], axis=1).astype(np.int32)
    return X, y


def _model(fx, rng):
    m = fx.Model(F, H, HEADS)
    p = _params(rng)
    mean = rng.normal(size=F).astype(np.float32)
    std = rng.uniform(0.5, 2, F).astype(np.float32)
    m.set(p, mean, std)
    return m, p, mean, std


def test_forward_and_choose():
    torch, fx = need_gpu()
    rng = np.random.default_rng(1)
    m, p, mean, std = _model(fx, rng)
    X, _ = _data(rng, 513)
    Xd = torch.from_numpy(X).cuda()
    logits = torch.empty(513, C, device="cuda")
    choice = torch.empty(513, len(HEADS), dtype=torch.int32, device="cuda")
    m.forward(Xd, logits, choice)
    torch.cuda.synchronize()
    ref = _forward64(p, X, mean.astype(np.float64), std.astype(np.float64))
    got = logits.cpu().numpy()
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3)) < 1e-4
    ch = choice.cpu().numpy()
    o = 0
    for q, k in enumerate(HEADS):
        assert np.array_equal(ch[:, q], np.argmax(got[:, o:o + k], axis=1))
        o += k
    for b in range(0, 513, 37):                 # the host twin decides identically
        assert m.choose(X[b]) == list(ch[b])


def test_gradient_matches_autograd_and_differences():
    torch, fx = need_gpu()
    rng = np.random.default_rng(2)
    m, p, mean, std = _model(fx, rng)
    X, y = _data(rng, 300)
    grad = torch.empty(m.n_params, device="cuda")
    loss = torch.empty(1, device="cuda")
    m.grad(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), grad, loss)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    # CPU autograd in float64
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    o = 0
    W1 = pt[o:o + H * F].view(H, F); o += H * F
    b1 = pt[o:o + H]; o += H
    W2 = pt[o:o + C * H].view(C, H); o += C * H
    b2 = pt[o:o + C]
    xn = (torch.tensor(X, dtype=torch.float64) - torch.tensor(mean, dtype=torch.float64)) / \
        torch.tensor(std, dtype=torch.float64)
    logits = torch.relu(xn @ W1.T + b1) @ W2.T + b2
    L, o = 0.0, 0
    yt = torch.tensor(y, dtype=torch.int64)
    for q, k in enumerate(HEADS):
        L = L + torch.nn.functional.cross_entropy(logits[:, o:o + k], yt[:, q])
        o += k
    L.backward()
    ref = pt.grad.numpy()
    assert abs(loss.item() - L.item()) < 1e-5 * max(1, abs(L.item()))
    assert np.max(np.abs(g - ref)) < 1e-5 * max(1.0, np.max(np.abs(ref)))
    # central differences on a few parameters of each block
    m64, s64 = mean.astype(np.float64), std.astype(np.float64)
    for i in [0, 7, H * F - 1, H * F + 3, H * F + H + 11, m.n_params - 1]:
        e = np.zeros(m.n_params)
        e[i] = 1e-4
        fd = (_loss64(p + e, X, y, m64, s64) - _loss64(p - e, X, y, m64, s64)) / 2e-4
        assert abs(fd - g[i]) < 1e-4 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_step_matches_numpy():
    torch, fx = need_gpu()
    rng = np.random.default_rng(3)
    m, p, mean, std = _model(fx, rng)
    X, y = _data(rng, 128)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    grad = torch.empty(m.n_params, device="cuda")
    m.grad(Xd, yd, grad)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    lr = 1e-2
    m.train_step(Xd, yd, lr)
    new = m.get()[0].astype(np.float64)
    mom, v = 0.1 * g, 0.001 * g * g                 # first step from zero moments
    want = p - lr * (mom / 0.1) / (np.sqrt(v / 0.001) + 1e-8)
    assert np.max(np.abs(new - want)) < 1e-5


def test_training_reduces_loss_on_separable_data():
    torch, fx = need_gpu()
    rng = np.random.default_rng(4)
    m = fx.Model(F, H, HEADS)
    m.set(_params(rng), np.zeros(F, np.float32), np.ones(F, np.float32))
    B = 1024
    X = rng.normal(size=(B, F)).astype(np.float32)
    y = np.stack([(X[:, 0] > 0) * 2 + (X[:, 1] > 0), X[:, 2] > 0, X[:, 3] + X[:, 4] > 0,
                  np.digitize(X[:, 5], [-0.7, 0, 0.7])], axis=1).astype(np.int32)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    loss = torch.empty(1, device="cuda")
    m.train_step(Xd, yd, 3e-3, loss)
    torch.cuda.synchronize()
    first = loss.item()
    for _ in range(400):
        m.train_step(Xd, yd, 3e-3, loss)
    torch.cuda.synchronize()
    assert loss.item() < 0.15 * first, (first, loss.item())
    choice = torch.empty(B, 4, dtype=torch.int32, device="cuda")
    m.forward(Xd, None, choice)
    torch.cuda.synchronize()
    assert (choice.cpu().numpy() == y).all(axis=1).mean() > 0.9


def test_committed_model_drives_tapes():
    """The trained model shipped with the package loads, its inference kernel
    and host twin agree on its own weights, and tapes launched with its
    picks (held-out items of the tuning set, shrunk to test sizes) match the
    oracle."""
    torch, fx = need_gpu()
    import os
    import oracle
    from gpu_util import assert_close, empty, from_dev, oracle_expr, tree_inputs
    from paper_2604_22242_amd import model, tune
    from synth import trees
    path = os.path.join(os.path.dirname(fx.LIB_PATH), "launch_model")
    m = model.load(path)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    feats, items = [], []
    for i in range(40):
        it = trees.tuning_item(6, i)
        red = it["reduce"]
        shape = (257, 131) if red in ("colsum", "rowsum") else (33331, 1)
        info = fx.Tape(it["nodes"]).info()
        feats.append(tune.features(info, it["dtype"], it["shape"], red))
        items.append((it, shape, red))
    X = torch.tensor(np.array(feats, np.float32)).cuda()
    choice = torch.empty(len(feats), len(tune.HEADS), dtype=torch.int32, device="cuda")
    m.forward(X, None, choice)
    torch.cuda.synchronize()
    ch = choice.cpu().numpy()
    for (it, shape, red), f, c in zip(items, feats, ch):
        assert m.choose(f) == list(c)
        cfg = model.config_of(tuple(c), red, it["dtype"], cus)
        dt = it["dtype"]
        dcode = fx.F32 if dt == "f32" else fx.BF16
        n = shape[0] * shape[1]
        host, dev = tree_inputs(6, it["id"], it["n_inputs"], n, dt)
        kind = tune.KIND[red]
        if kind == 0:
            out, od = empty(n, dt), dt
        elif red in ("accu", "norm"):
            out, od = torch.zeros(1, dtype=torch.float64, device="cuda"), "f64"
        else:
            out, od = empty(shape[1] if red == "colsum" else shape[0], "f32"), "f32"
        ws = fx.workspace(kind, dcode, shape, cfg) if kind else None
        fx.fx_tape_eval(fx.Tape(it["nodes"]), dev, out, shape, kind, ws, cfg=cfg, dt=dcode)
        torch.cuda.synchronize()
        v, mu = oracle.evaluate(oracle_expr(it["nodes"]), host, dt, shape=shape, reduce=red)
        half = dt if (kind == 0 and dt == "bf16") else None
        assert_close(from_dev(out, od), v, mu, dt, "model-picked %s item %d" % (cfg, it["id"]),
                     out_dtype=half)


def test_native_loader_and_predictor_agree_with_the_driver():
    """fx_model_load reads the committed FXM1 file; fx_tape_features and
    fx_model_predict give, for held-out tuning items of every kind, the same
    launch configuration as the Python driver (JSON + parameter files,
    features() and config_of())."""
    torch, fx = need_gpu()
    import os
    from paper_2604_22242_amd import model, tune
    from synth import trees
    base = os.path.join(os.path.dirname(fx.LIB_PATH), "launch_model")
    native = fx.fx_model_load(base + ".fxm")
    driver = model.load(base)
    assert native.heads == driver.heads and native.n_features == driver.n_features
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    kinds = {None: 0, "accu": fx.R_ACCU, "colsum": fx.R_COLSUM, "rowsum": fx.R_ROWSUM,
             "norm": fx.R_NORM}
    for i in range(60):
        it = trees.tuning_item(6, i)
        tape = fx.Tape(it["nodes"])
        code = fx.F32 if it["dtype"] == "f32" else fx.BF16
        f = fx.fx_tape_features(tape, code, it["shape"], kinds[it["reduce"]])
        got = native.predict(f, kinds[it["reduce"]], code)
        want = model.config_of(tuple(driver.choose(tune.features(tape.info(), it["dtype"], it["shape"],
                                                                 it["reduce"]))),
                               it["reduce"], it["dtype"], cus)
        assert got == tuple(want), (i, got, want)
    with pytest.raises(fx.FxError):
        fx.fx_model_load(base + ".json")          # not a model file


def test_native_training_loop_equals_the_step_by_step_loop():
    # fx_model_train, gathering each mini-batch through the epoch's order,
    # gives the same parameters bit for bit as gathering the rows first and
    # calling fx_model_train_step per mini-batch (ragged last batch included)
    torch, fx = need_gpu()
    rng = np.random.default_rng(11)
    n, batch, epochs, lr = 300, 64, 3, 2e-3
    X, y = _data(rng, n)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    perm = np.stack([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)
    a, p, mean, std = _model(fx, np.random.default_rng(12))
    b = fx.Model(F, H, HEADS)
    b.set(p, mean, std)
    loss = torch.zeros(1, device="cuda")
    last = []
    for e in range(epochs):
        idx = torch.from_numpy(perm[e].astype(np.int64)).cuda()
        Xp, yp = Xd[idx].contiguous(), yd[idx].contiguous()
        for s in range(0, n, batch):
            a.train_step(Xp[s:s + batch], yp[s:s + batch], lr, loss)
        last.append(loss.clone())
    losses = torch.zeros(epochs, device="cuda")
    b.train(Xd, yd, epochs, batch, lr, perm, losses)
    torch.cuda.synchronize()
    pa, pb = a.get()[0], b.get()[0]
    assert not np.array_equal(pa, p)
    assert np.array_equal(pa, pb)
    assert torch.cat(last).cpu().tolist() == losses.cpu().tolist()
    # natural order: the same as perm = arange each epoch
    c = fx.Model(F, H, HEADS)
    c.set(p, mean, std)
    d = fx.Model(F, H, HEADS)
    d.set(p, mean, std)
    c.train(Xd, yd, 2, batch, lr)
    d.train(Xd, yd, 2, batch, lr, np.tile(np.arange(n, dtype=np.int32), (2, 1)))
    torch.cuda.synchronize()
    assert np.array_equal(c.get()[0], d.get()[0])


def test_native_training_rejects_a_bad_order():
    torch, fx = need_gpu()
    rng = np.random.default_rng(13)
    X, y = _data(rng, 10)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    m, p, _, _ = _model(fx, rng)
    bad = np.tile(np.arange(10, dtype=np.int32), (2, 1))
    bad[1, 3] = 4  # a repeated row
    with pytest.raises(fx.FxError):
        m.train(Xd, yd, 2, 4, 1e-3, bad)
    bad[1, 3] = 10  # out of range
    with pytest.raises(fx.FxError):
        m.train(Xd, yd, 2, 4, 1e-3, bad)
    assert np.array_equal(m.get()[0], p)  # nothing ran


def test_set_with_null_params_keeps_trained_parameters():
    """After training, fx_model_set(NULL params, mean, std) must keep the
    trained parameters, and the host twin (choose) must use them without an
    explicit fx_model_get: choose agrees with the inference kernel."""
    torch, fx = need_gpu()
    rng = np.random.default_rng(9)
    m, p, mean, std = _model(fx, rng)
    X, y = _data(rng, 256)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    for _ in range(20):
        m.train_step(Xd, yd, 5e-2)
    torch.cuda.synchronize()
    mean2 = (mean + 0.25).astype(np.float32)
    m.set(None, mean2, std)                         # keep the trained parameters
    trained = m.get()[0]
    assert not np.array_equal(trained, p), "training did not move the parameters"
    choice = torch.empty(256, len(HEADS), dtype=torch.int32, device="cuda")
    logits = torch.empty(256, C, device="cuda")
    m.forward(Xd, logits, choice)
    torch.cuda.synchronize()
    ref = _forward64(trained, X, mean2.astype(np.float64), std.astype(np.float64))
    got = logits.cpu().numpy()
    # FP32 forward against FP64: relative to the size of each row's logits
    scale = np.maximum(np.abs(ref).max(axis=1, keepdims=True), 1.0)
    assert np.max(np.abs(got - ref) / scale) < 1e-5
    # and not the untrained parameters' logits
    old = _forward64(p, X, mean2.astype(np.float64), std.astype(np.float64))
    assert np.max(np.abs(got - old) / scale) > 1e-2
    ch = choice.cpu().numpy()
    m2, _, _, _ = _model(fx, np.random.default_rng(9))
    for _ in range(20):
        m2.train_step(Xd, yd, 5e-2)
    m2.set(None, mean2, std)                        # no get(): the twin refreshes itself
    for b in range(0, 256, 17):
        assert m2.choose(X[b]) == list(ch[b])
