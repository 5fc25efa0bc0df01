"""CPU checks of the C ABI: the header compiles as C and C++, the built
library exports every declared function, the binding covers them, and the
host-side argument checks return their status before anything is enqueued."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(fx_[a-z_0-9]+)\s*\(",
                                 text, flags=re.M)))


@pytest.fixture(scope="module")
def fx():
    import paper_2604_22242_amd as fx
    if not os.path.exists(fx.LIB_PATH):
        from paper_2604_22242_amd import build
        build.build()
    fx.lib()
    return fx


@pytest.mark.parametrize("lang,cc", [("c", "gcc"), ("c++", "g++")])
def test_header_compiles(lang, cc, tmp_path):
    src = tmp_path / ("t." + ("c" if lang == "c" else "cpp"))
    src.write_text('#include "fx.h"\nint main(void) { fx_launch l = {0, 0, 0, 0}; (void)l; '
                   'return (int)FX_OK; }\n')
    std = ["-std=c99"] if lang == "c" else ["-std=c++17"]
    subprocess.check_call([cc, "-Wall", "-Werror", "-pedantic"] + std +
                          ["-I", os.path.dirname(HEADER), "-fsyntax-only", str(src)])


def test_library_exports_every_declared_function(fx):
    decl = declared_functions()
    assert len(decl) >= 20
    L = ctypes.CDLL(fx.LIB_PATH)
    missing = [f for f in decl if not hasattr(L, f)]
    assert not missing, missing
    assert sorted(fx.exported_symbols()) == decl, "binding and header disagree"


def test_version(fx):
    assert "gfx950" in fx.fx_version()


FAKE = 0x10000  # never dereferenced: every call below fails its host checks


def test_argument_errors_return_before_launch(fx):
    L = fx.lib()
    cfg = ctypes.pointer(fx.Launch(100, 0, 0, 0))
    assert L.fx_c1_z(fx.F32, FAKE, FAKE, FAKE, FAKE, -1, None, None) == 1      # FX_E_ARG
    assert L.fx_c1_z(77, FAKE, FAKE, FAKE, FAKE, 16, None, None) == 3          # FX_E_DTYPE
    assert "dtype" in fx.fx_last_error()
    assert L.fx_c1_z(fx.F32, FAKE, FAKE, FAKE, FAKE, 16, cfg, None) == 7       # FX_E_CONFIG
    assert "block" in fx.fx_last_error()
    assert L.fx_c1_z(fx.F32, None, FAKE, FAKE, FAKE, 16, None, None) == 1      # NULL input
    assert L.fx_c1_z(fx.F32, FAKE, FAKE, FAKE, None, 16, None, None) == 1      # NULL output
    assert L.fx_axy_expw(fx.U32, 1.0, FAKE, FAKE, FAKE, FAKE, 16, None, None) == 3
    assert L.fx_c2_z(fx.F32, FAKE, FAKE, FAKE, FAKE, fx.Shape(-1, 2), None, None) == 1
    assert L.fx_op_unary(99, fx.F32, FAKE, FAKE, 16, None, None) == 1
    assert L.fx_op_binary(fx.OP["div"], fx.U32, FAKE, FAKE, FAKE, 16, None, None) == 1
    assert L.fx_op_scalar(fx.OP["sadd"], fx.U32, FAKE, 0.5, FAKE, 16, None, None) == 1
    assert L.fx_reduce(fx.R_NORM, fx.U32, FAKE, None, fx.Shape(4, 4), FAKE, None, 0, None,
                       None) == 3
    for bad in [(64, 3, 0, 0), (64, 1, 12, 0), (64, 1, 0, -1), (1024, 0, 0, 0)]:
        c = ctypes.pointer(fx.Launch(*bad))
        assert L.fx_c1_z(fx.F32, FAKE, FAKE, FAKE, FAKE, 16, c, None) == 7, bad
    assert L.fx_bw_copy(FAKE + 4, FAKE, 64, None, None) == 1                   # misaligned


def test_workspace_query_and_resolution(fx):
    assert fx.fx_workspace_bytes(99, fx.F32, (10, 10)) == 0
    assert fx.fx_workspace_bytes(fx.R_ACCU, 77, (10, 10)) == 0
    # a single block needs no workspace; several need counter + partials
    assert fx.fx_workspace_bytes(fx.R_ACCU, fx.F32, (1000, 1), (256, 4, 16, 1)) == 0
    assert fx.fx_workspace_bytes(fx.R_ACCU, fx.F32, (1 << 20, 1), (256, 4, 16, 100)) == 256 + 800
    assert fx.fx_resolve_launch(fx.R_ACCU, fx.F32, (1 << 20, 1), (128, 2, 16, 9)) == (128, 2, 16, 9)
    b, e, v, s = fx.fx_resolve_launch(0, fx.F32, (1 << 26, 1))
    assert b % 64 == 0 and e in (1, 2, 4, 8) and v == 16 and s >= 1
    # column sums of short columns use one thread per column (no workspace)
    assert fx.fx_resolve_launch(fx.R_COLSUM, fx.F32, (8, 100000))[3] == 0
    assert fx.fx_workspace_bytes(fx.R_COLSUM, fx.F32, (8, 100000)) == 0


def test_unfused_temporaries(fx):
    assert fx.fx_unfused_tmp_bytes("c2_z", fx.F32, (8192, 8192)) == 2 * 8192 * 8192 * 4
    assert fx.fx_unfused_tmp_bytes("accu_xy", fx.BF16, (1000, 1)) == 2048
    assert fx.fx_unfused_tmp_bytes(99, fx.F32, (10, 1)) == 0


def test_view_expressions_refuse_overlapping_outputs(fx):
    """An output that overlaps an input read through a transposed, offset or
    diagonal view is refused on the host (nothing is enqueued)."""
    L = fx.lib()
    m = n = 64
    nbytes = m * n * 4
    a, b, c, d = FAKE, FAKE + nbytes, FAKE + 2 * nbytes, FAKE + 3 * nbytes
    sc = (ctypes.c_double * 1)(1.5)

    def call(which, ins, z):
        arr = (ctypes.c_void_p * 4)(*ins)
        return L.fx_paper_view_expr(fx.PAPER_VIEW[which], fx.F32, arr, sc, z, fx.Shape(m, n), None)

    assert call("expr1", [a, b, 0, 0], a) == 1                 # Z = X, read transposed
    assert "overlaps input 0" in fx.fx_last_error()
    assert call("expr1", [a, b, 0, 0], b + 4) == 1             # partial overlap with Y
    assert call("expr2", [a, b, c, d], b) == 1                 # Z = B, read transposed
    assert call("expr2", [a, b, c, d], a + 64) == 1            # partial overlap with A
    assert call("addsub2", [a, b, 0, 0], a) == 1               # centre submatrix of X
    assert call("addsub4", [a, b, c, d], d + 16) == 1
    assert call("diagsum", [a, b, 0, 0], b + 8) == 1           # a diagonal of Y
