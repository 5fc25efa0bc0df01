"""CPU tests of the kernels generated as source from expression types: the
text is the expression's type written out, it is a compile-time constant of
the library, it compiles through hipRTC (no device needed), and bad calls are
refused on the host."""
import ctypes
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_22242_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")

EXPRS = ["c1_z", "accu_xy", "c2_z", "c2_colsum", "c2_rowsum", "norm_diff", "colsum_xy", "axy_expw"]
KIND = {"c1_z": 0, "accu_xy": 1, "c2_z": 0, "c2_colsum": 2, "c2_rowsum": 3, "norm_diff": 4,
        "colsum_xy": 2, "axy_expw": 0}
# the element rule of each expression type, leaves x<k> in depth-first order
RULE = {
    "c1_z": "return ((x0 * x1) + (k0 * x2));",
    "accu_xy": "return (x0 * x1);",
    "c2_z": "return (((x0 + x1) * %s((-%s(x2)))) / (k0 + (x3 * x4)));",
    "c2_colsum": "return (((x0 + x1) * %s((-%s(x2)))) / (k0 + (x3 * x4)));",
    "c2_rowsum": "return (((x0 + x1) * %s((-%s(x2)))) / (k0 + (x3 * x4)));",
    "norm_diff": "return (x0 - x1);",
    "colsum_xy": "return (x0 * x1);",
    "axy_expw": "return (((k0 * x0) * x1) + %s((-x2)));",
}
LEAVES = {"c1_z": 3, "accu_xy": 2, "c2_z": 5, "c2_colsum": 5, "c2_rowsum": 5, "norm_diff": 2,
          "colsum_xy": 2, "axy_expw": 3}


@pytest.fixture(scope="module")
def fx():
    import paper_2604_22242_amd as fx
    if not os.path.exists(fx.LIB_PATH):
        from paper_2604_22242_amd import build
        build.build()
    return fx


@pytest.mark.parametrize("expr", EXPRS)
def test_text_is_the_expression_type(fx, expr):
    for dt, ct, fns in [(fx.F32, "float", ("expf", "__builtin_fabsf")),
                        (fx.F64, "double", ("exp", "__builtin_fabs")),
                        (fx.BF16, "float", ("expf", "__builtin_fabsf"))]:
        t = fx.fx_source_text(expr, dt)
        rule = RULE[expr]
        if "%s" in rule:
            rule = rule % (fns if rule.count("%s") == 2 else fns[:1])
        assert rule in t, (expr, dt)
        assert "typedef %s ct_t;" % ct in t
        L = LEAVES[expr]
        assert "#define FX_NIN %d\n" % L in t
        assert "const st_t* __restrict__ p%d" % (L - 1) in t
        assert "const st_t* __restrict__ p%d" % L not in t
        # the launch configuration written into the text is the library's default
        kind = KIND[expr]
        esize = {fx.F32: 4, fx.F64: 8, fx.BF16: 2}[dt]
        block, ept, _, _ = fx.fx_resolve_launch(1 if kind == 4 else kind, dt, (1 << 20, 64))
        assert "#define FX_BLOCK %d\n" % block in t and "#define FX_EPT %d\n" % ept in t
        assert "#define FX_N %d\n" % (16 // esize) in t
        assert ("__builtin_sqrt(s)" in t) == (kind == 4)


def test_u32_text_and_dtype_refusals(fx):
    t = fx.fx_source_text("c1_z", fx.U32)
    assert "return ((x0 ^ x1) + (k0 * x2));" in t and "typedef unsigned int ct_t;" in t
    L = fx.lib()
    n = ctypes.c_size_t()
    assert L.fx_source_text(fx.EXPR["accu_xy"], fx.U32, None, 0, ctypes.byref(n)) == 3
    assert L.fx_source_text(99, fx.F32, None, 0, ctypes.byref(n)) == 1


def test_text_is_a_compile_time_constant(fx, tmp_path):
    """A translation unit computes, in a constant expression, a hash of the
    text that the front end generates for the matrix workload's expression
    type, and asserts at compile time that it equals the hash of the text the
    library hands out at run time: the library's text is that constant."""
    text = fx.fx_source_text("c2_z", fx.F32)
    h = 0xcbf29ce484222325
    for b in text.encode():
        h = ((h ^ b) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    src = tmp_path / "const_text.hip"
    src.write_text(
        '#include "fx_source.hpp"\n#include "fx_workloads.hpp"\n'
        "using namespace fx;\n"
        "using E = decltype(c2_expr(Leaf<float>{}, Leaf<float>{}, Leaf<float>{}));\n"
        "constexpr unsigned long long fnv(const char* s, unsigned long n) {\n"
        "  unsigned long long h = 0xcbf29ce484222325ull;\n"
        "  for (unsigned long i = 0; i < n; ++i) h = (h ^ (unsigned char)s[i]) * 0x100000001b3ull;\n"
        "  return h;\n}\n"
        "constexpr auto T = program_text<E, float, 0>();\n"
        "static_assert(T.size == %dul, \"length\");\n"
        "static_assert(fnv(T.data(), T.size) == %dull, \"text\");\n" % (len(text), h))
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    subprocess.check_call([hipcc, "-std=c++17", "-fsyntax-only", "--offload-arch=gfx950",
                           "-I", INCLUDE, "-I", CSRC, str(src)])


def test_texts_compile_through_the_driver(fx):
    ms = fx.fx_source_prepare("c2_colsum", fx.BF16)
    assert ms >= 0.0
    assert fx.fx_source_prepare("c2_colsum", fx.BF16) == ms   # compiled once, kept
    fx.fx_source_prepare("norm_diff", fx.F64)
    fx.fx_source_prepare("c1_z", fx.U32)


FAKE = 0x10000


def test_host_checks_come_first(fx):
    L = fx.lib()
    arr = (ctypes.c_void_p * 3)(FAKE + 4, FAKE, FAKE)     # misaligned X
    assert L.fx_source_eval(fx.EXPR["c2_z"], fx.F32, arr, 0.0, FAKE, fx.Shape(64, 64), None, 0,
                            None) == 1
    assert "16-byte" in fx.fx_last_error()
    arr = (ctypes.c_void_p * 3)(FAKE, FAKE, FAKE)
    assert L.fx_source_eval(fx.EXPR["c2_z"], fx.F32, arr, 0.0, FAKE, fx.Shape(-1, 64), None, 0,
                            None) == 1
    assert L.fx_source_eval(fx.EXPR["c2_colsum"], fx.F32, arr, 0.0, FAKE, fx.Shape(8192, 64), None,
                            0, None) == 4                 # workspace missing
    assert L.fx_source_eval(fx.EXPR["c2_z"], 77, arr, 0.0, FAKE, fx.Shape(4, 4), None, 0,
                            None) == 3
    assert L.fx_source_eval(fx.EXPR["c2_z"], fx.F32, arr, 0.0, None, fx.Shape(4, 4), None, 0,
                            None) == 1
