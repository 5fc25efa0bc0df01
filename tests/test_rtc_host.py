"""CPU tests of the run-time source mode: the generated source, hipRTC
compilation (which needs no device) and the per-process cache."""
import time

import pytest

from synth import trees


@pytest.fixture(scope="module")
def fx():
    import os
    import paper_2604_22242_amd as fx
    if not os.path.exists(fx.LIB_PATH):
        from paper_2604_22242_amd import build
        build.build()
    return fx


C2 = [("leaf", -1, -1, 0, 0.0), ("leaf", -1, -1, 1, 0.0), ("add", 0, 1, -1, 0.0),
      ("leaf", -1, -1, 2, 0.0), ("abs", 3, -1, -1, 0.0), ("neg", 4, -1, -1, 0.0),
      ("exp", 5, -1, -1, 0.0), ("mul", 2, 6, -1, 0.0), ("const", -1, -1, -1, 1.0),
      ("mul", 0, 0, -1, 0.0), ("add", 8, 9, -1, 0.0), ("div", 7, 10, -1, 0.0)]


def test_source_is_the_expression(fx):
    r = fx.Rtc(C2, fx.F32)
    src = r.source()
    # one SSA value per node, constants as exact hexadecimal literals,
    # 16-byte vectors with a scalar tail
    for line in ("const float t2 = t0 + t1;", "const float t6 = expf(t5);",
                 "const float t8 = 0x1p+0f;", "const float t11 = t7 / t10;",
                 "__builtin_nontemporal_load", "return t11;", "fx_rtc_ew"):
        assert line in src, line
    assert "fabsf(t3)" in src and "-t4" in src
    d = fx.Rtc(C2, fx.F64).source()
    assert "const double t8 = 0x1p+0;" in d and "exp(t5)" in d


def test_compiles_and_caches(fx):
    nodes, _, _ = trees.random_tree(77, 3)
    t0 = time.time()
    a = fx.Rtc(nodes, fx.F32)
    first = a.compile_ms()
    b = fx.Rtc(nodes, fx.F32)                 # same text: found in the cache
    assert b.compile_ms() == 0.0 and b.source() == a.source()
    assert first > 0.0 and time.time() - t0 < 60


def test_generated_trees_compile(fx):
    for i in range(8):
        nodes, _, _ = trees.random_tree(4, i)
        for dt in (fx.F32, fx.F64):
            fx.Rtc(nodes, dt)


KINDS = {0: ["fx_rtc_ew"], 1: ["fx_rtc_full"], 4: ["fx_rtc_full"],
         2: ["fx_rtc_colsum_v", "fx_rtc_colsum_s"], 3: ["fx_rtc_rowsum_v", "fx_rtc_rowsum_s"]}


@pytest.mark.parametrize("kind", sorted(KINDS))
def test_every_kind_and_dtype_compiles(fx, kind):
    assert (fx.R_ACCU, fx.R_COLSUM, fx.R_ROWSUM, fx.R_NORM) == (1, 2, 3, 4)
    types = {fx.F32: ("float", "float"), fx.F64: ("double", "double"),
             fx.BF16: ("__bf16", "float"), fx.F16: ("_Float16", "float")}
    for dt, (st, ct) in types.items():
        src = fx.Rtc(C2, dt, kind).source()
        for name in KINDS[kind]:
            assert 'extern "C" __global__' in src and name in src, (kind, dt, name)
        assert "typedef %s st_t;" % st in src and "typedef %s ct_t;" % ct in src
        # the per-lane vector is one 16-byte load of the storage type
        assert "#define FX_N %d" % (16 // {"float": 4, "double": 8}.get(st, 2)) in src
        if kind:
            assert "#pragma clang fp contract(off)" in src       # the compensated sum
            assert ("(x) * (x)" in src) == (kind == fx.R_NORM)
            assert ("__builtin_sqrt(s)" in src) == (kind == fx.R_NORM)


def test_launch_configuration_is_the_library_default(fx):
    # block size and EPT written into the text are the defaults of the kind
    for kind, dt in ((0, fx.F32), (fx.R_ACCU, fx.F32), (fx.R_COLSUM, fx.F32),
                     (fx.R_COLSUM, fx.BF16), (fx.R_ROWSUM, fx.F32), (fx.R_ROWSUM, fx.BF16)):
        src = fx.Rtc(C2, dt, kind).source()
        c = fx.fx_resolve_launch(kind, dt, (4096, 4096))
        assert "#define FX_BLOCK %d\n" % c[0] in src and "#define FX_EPT %d\n" % c[1] in src


def test_errors(fx):
    with pytest.raises(fx.FxError) as e:
        fx.Rtc(C2, fx.U32)
    assert e.value.code == 3                    # FX_E_DTYPE
    with pytest.raises(fx.FxError) as e:
        fx.Rtc(C2, fx.F32, 5)                   # dot is not a kind of one tree
    assert e.value.code == 1
    with pytest.raises(fx.FxError) as e:
        fx.Rtc([("add", 0, 1, -1, 0.0)], fx.F32)
    assert e.value.code == 1                    # operands not earlier
    with pytest.raises(fx.FxError) as e:
        fx.Rtc([("leaf", -1, -1, 5, 0.0)], fx.F32)
    assert e.value.code == 6                    # a sixth input
