"""GPU parity of the run-time source mode (hipRTC-compiled kernels) against
the FP64 oracle and the compile-time path."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_close, empty, from_dev, need_gpu, oracle_expr, tree_inputs
from synth import trees

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("e", range(0, 40, 5))
def test_random_trees(dtype, e):
    torch, fx = need_gpu()
    nodes, k, _ = trees.random_tree(4, e)
    for n in (1, 3, 1000, 100003):
        host, dev = tree_inputs(4, e, k, n, dtype)
        r = fx.Rtc(nodes, fx.F32 if dtype == "f32" else fx.F64)
        out = empty(n, dtype)
        r.eval(dev, out)
        torch.cuda.synchronize()
        v, mu = oracle.evaluate(oracle_expr(nodes), host, dtype, shape=(n, 1))
        assert_close(from_dev(out, dtype), v, mu, dtype, "rtc tree %d n %d %s" % (e, n, dtype))


def test_matches_the_compile_time_kernel():
    torch, fx = need_gpu()
    from test_rtc_host import C2
    import synth
    n = 1 << 20
    host = [synth.fill(2, t, n, "f32") for t in range(3)]
    dev = [torch.from_numpy(h).cuda() for h in host]
    a, b = empty(n, "f32"), empty(n, "f32")
    fx.Rtc(C2, fx.F32).eval(dev, a)
    fx.fx_c2_z(*dev, b, (n, 1))
    torch.cuda.synchronize()
    v, mu = oracle.evaluate(oracle.EXPRS["c2_z"], host, "f32")
    assert_close(from_dev(a, "f32"), v, mu, "f32", "rtc c2")
    # same operations in the same order: the results agree to the last bit
    # wherever neither side contracted a product into an FMA differently
    same = np.mean(a.cpu().numpy() == b.cpu().numpy())
    assert same > 0.99, same


def test_misaligned_arrays_are_refused():
    torch, fx = need_gpu()
    from test_rtc_host import C2
    x = torch.zeros(1027, device="cuda")
    out = torch.empty(1026, device="cuda")
    with pytest.raises(fx.FxError) as e:
        fx.Rtc(C2, fx.F32).eval([x[1:], x[1:], x[1:]], out)
    assert e.value.code == 1
