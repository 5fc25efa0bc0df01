"""FP64 CPU oracle (ctypes front end of ``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg.  It never imports the HIP package and the
HIP package never imports it.

Expressions are written with the small builder below in the paper's notation
(``%`` is the Schur product, Sec. 4; capital letters are matrices, lower case
scalars) and evaluated node by node with one FP64 temporary per node.  The
builder knows nothing of the HIP path's expression templates.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

DTYPE = {"f32": 0, "f64": 1, "bf16": 2, "f16": 3, "u32": 4}
OP = {"leaf": 0, "const": 1, "add": 2, "sub": 3, "mul": 4, "div": 5, "neg": 6,
      "abs": 7, "exp": 8, "sqrt": 9, "xor": 10, "log": 11, "tanh": 12, "pow": 13, "gt": 14,
      "tof32": 15}
REDUCE = {None: 0, "accu": 1, "colsum": 2, "rowsum": 3, "norm": 4}

U32 = 2.0 ** -24   # unit roundoff, FP32 compute (f32, bf16, f16 storage)
U64 = 2.0 ** -53   # unit roundoff, FP64 compute
TOL = {"f32": 1e-6, "bf16": 1e-6, "f16": 1e-6, "f64": 1e-13}
U_HALF = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}
HALF_SUBNORMAL_HALF_SPACING = {"bf16": 2.0 ** -134, "f16": 2.0 ** -25}
F16_OVERFLOW = 65520.0   # nearest-even rounding of |z| >= 65520 to FP16 gives inf

# Allowances of the device elementary functions in the running error bound,
# in units of the compute type's roundoff relative to the result (2 = one
# ulp at most), per compute type.  Each must be at least the largest relative
# error that the sweep of the device functions against libm finds over the
# function's domain of use (every FP32 input; a sample of FP64 inputs).
F_ALLOW = {
    # every FP32 input swept: largest errors exp 1.41, log 3.18, tanh 2.49;
    # pow(x, 3) is two correctly rounded products (at most 2)
    "f32": {"exp": 1.5, "log": 3.25, "tanh": 2.5, "pow": 2.0},
    # 2^24 FP64 inputs sampled: largest errors exp 1.24, log 1.13, tanh 1.35,
    # pow(x, 3) 1.99; a sample can miss the worst input, hence 2
    "f64": {"exp": 2.0, "log": 2.0, "tanh": 2.0, "pow": 2.0},
}
F_ORDER = ("exp", "log", "tanh", "pow")


def build(force: bool = False) -> str:
    srcs = [os.path.join(_HERE, f) for f in ("oracle.c", "mathref.c")]
    newest = max(os.path.getmtime(f) for f in srcs)
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < newest:
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-o", tmp] + srcs + ["-lm"])
        os.replace(tmp, _SO)
    return _SO


class SweepStats(ctypes.Structure):
    """Result of a sweep of a device elementary function (mathref.c)."""
    _fields_ = [("max_rel_u", ctypes.c_double), ("max_ulp", ctypes.c_double),
                ("argmax", ctypes.c_int64), ("first_bad", ctypes.c_int64),
                ("n_bad", ctypes.c_int64), ("n_subnormal", ctypes.c_int64),
                ("max_sub_ulp", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        L.or_eval.restype = ctypes.c_int
        L.or_eval.argtypes = [ctypes.c_int, P, P, P, P, P, ctypes.c_int, P, P,
                              ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                              ctypes.c_double, P, P, P]
        L.or_eval_views.restype = ctypes.c_int
        L.or_eval_views.argtypes = [ctypes.c_int, P, P, P, P, P, ctypes.c_int, P, P,
                                    ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                    ctypes.c_double, P, P, P, P, P, P]
        L.or_eval_u32.restype = ctypes.c_int
        L.or_eval_u32.argtypes = [ctypes.c_int, P, P, P, P, P, ctypes.c_int, P,
                                  ctypes.c_int64, P, P]
        L.mr_sweep_f32.restype = ctypes.c_int
        L.mr_sweep_f32.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_int64, ctypes.c_double,
                                   P, ctypes.c_double, ctypes.c_double, ctypes.POINTER(SweepStats)]
        L.mr_sweep_f64.restype = ctypes.c_int
        L.mr_sweep_f64.argtypes = [ctypes.c_int, P, ctypes.c_int64, ctypes.c_double, P,
                                   ctypes.c_double, ctypes.POINTER(SweepStats)]
        L.or_num_threads.restype = ctypes.c_int
        L.or_set_threads.restype = None
        L.or_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


MATH_FN = {"exp": 0, "log": 1, "tanh": 2, "sqrt": 3, "pow": 4}


def sweep_f32(fn: str, bits0: int, got, f_allow: float, k: float = 0.0,
              max_abs_x: float = 0.0) -> dict:
    """Errors of device FP32 results `got` (float32 array) for the inputs
    whose bit patterns are bits0, bits0 + 1, ...: the largest error relative
    to the libm value in units of 2^-24 (max_rel_u), in ulps (max_ulp), and
    the first index beyond `f_allow` (first_bad, -1 if none).  max_abs_x > 0
    skips inputs beyond it in magnitude."""
    got = np.ascontiguousarray(got, np.float32)
    st = SweepStats()
    if lib().mr_sweep_f32(MATH_FN[fn], int(bits0), got.size, float(k), got.ctypes.data,
                          float(f_allow), float(max_abs_x), ctypes.byref(st)) != 0:
        raise ValueError("bad sweep arguments")
    return st.as_dict()


def sweep_f64(fn: str, x, got, f_allow: float, k: float = 0.0) -> dict:
    """As sweep_f32 for FP64 results `got` at the inputs `x`, referenced to
    extended precision; errors in units of 2^-53."""
    x = np.ascontiguousarray(x, np.float64)
    got = np.ascontiguousarray(got, np.float64)
    assert x.size == got.size
    st = SweepStats()
    if lib().mr_sweep_f64(MATH_FN[fn], x.ctypes.data, x.size, float(k), got.ctypes.data,
                          float(f_allow), ctypes.byref(st)) != 0:
        raise ValueError("bad sweep arguments")
    return st.as_dict()


def num_threads() -> int:
    return lib().or_num_threads()


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's loops (for timing it)."""
    lib().or_set_threads(int(n))


# --------------------------------------------------------------------------
# Expression builder: a tree of nodes, flattened children-first.


class E:
    """A node of an expression tree."""

    __slots__ = ("op", "kids", "leaf", "cst", "view")

    def __init__(self, op, kids=(), leaf=-1, cst=0.0, view=None):
        self.op, self.kids, self.leaf, self.cst = op, tuple(kids), leaf, cst
        # leaves only: None (dense), "T" (transposed dense), or (off, rs, cs):
        # element (r, c) of the view is input[off + r*rs + c*cs]
        self.view = view

    @staticmethod
    def wrap(v):
        return v if isinstance(v, E) else const(v)

    def __add__(self, o): return E("add", (self, E.wrap(o)))
    def __radd__(self, o): return E("add", (E.wrap(o), self))
    def __sub__(self, o): return E("sub", (self, E.wrap(o)))
    def __rsub__(self, o): return E("sub", (E.wrap(o), self))
    def __mod__(self, o): return E("mul", (self, E.wrap(o)))     # Schur product
    def __mul__(self, o):                                         # scalar * matrix only
        assert not isinstance(o, E), "matrix product is not an element-wise operation"
        return E("mul", (self, const(o)))
    def __rmul__(self, o):
        assert not isinstance(o, E)
        return E("mul", (const(o), self))
    def __truediv__(self, o): return E("div", (self, E.wrap(o)))
    def __rtruediv__(self, o): return E("div", (E.wrap(o), self))
    def __neg__(self): return E("neg", (self,))
    def __xor__(self, o): return E("xor", (self, E.wrap(o)))

    def t(self):
        """The transpose (Sec. 3): element (r, c) of E.t() is E(c, r), so every
        leaf's access swaps row and column; a double transpose cancels."""
        memo = {}

        def tr(e):
            if id(e) in memo:
                return memo[id(e)]
            if e.op == "leaf":
                v = e.view
                nv = "T" if v is None else None if v == "T" else (v[0], v[2], v[1])
                r = E("leaf", leaf=e.leaf, view=nv)
            elif e.op == "const":
                r = e
            else:
                r = E(e.op, tuple(tr(k) for k in e.kids), e.leaf, e.cst)
            memo[id(e)] = r
            return r
        return tr(self)

    def nodes(self):
        """Post-order list of distinct nodes (root last)."""
        order, seen = [], {}

        def visit(e):
            if id(e) in seen:
                return
            for k in e.kids:
                visit(k)
            seen[id(e)] = len(order)
            order.append(e)

        visit(self)
        return order, seen

    def arrays(self):
        order, seen = self.nodes()
        n = len(order)
        op = np.array([OP[e.op] for e in order], dtype=np.int32)
        a = np.array([seen[id(e.kids[0])] if len(e.kids) > 0 else -1 for e in order], np.int32)
        b = np.array([seen[id(e.kids[1])] if len(e.kids) > 1 else -1 for e in order], np.int32)
        leaf = np.array([e.leaf for e in order], dtype=np.int32)
        cst = np.array([e.cst for e in order], dtype=np.float64)
        assert n == op.size
        return op, a, b, leaf, cst

    def n_inputs(self):
        order, _ = self.nodes()
        return 1 + max([e.leaf for e in order] + [-1])


def leaf(i: int) -> E:
    return E("leaf", leaf=i)


def submat(i: int, r0: int, c0: int, ld: int) -> E:
    """Input i (column-major, leading dimension ld) from row r0, column c0:
    the submatrix view (its size is the expression's shape)."""
    return E("leaf", leaf=i, view=(r0 + c0 * ld, 1, ld))


def diag(i: int, k: int, ld: int) -> E:
    """Diagonal k of input i (leading dimension ld) as a column vector:
    element j is X(j + max(-k, 0), j + max(k, 0))."""
    return E("leaf", leaf=i, view=(max(-k, 0) + max(k, 0) * ld, ld + 1, 0))


def const(c: float) -> E:
    return E("const", cst=float(c))


def exp(e): return E("exp", (e,))
def abs_(e): return E("abs", (e,))
def sqrt(e): return E("sqrt", (e,))
def log(e): return E("log", (e,))
def tanh(e): return E("tanh", (e,))
def pow_(e, k): return E("pow", (e, const(k)))
def gt(e, k): return E("gt", (e, E.wrap(k)))
def conv_to_f32(e): return E("tof32", (e,))       # conv_to<fmat>::from(e)


X, Y, W = leaf(0), leaf(1), leaf(2)

# The expressions of the workloads, in the paper's API notation.
EXPRS = {
    "c1_z": X % Y + 2 * W,                          # Z = X % Y + 2*W
    "xy": X % Y,                                    # accu(X % Y), dot(X, Y), sum(X % Y, 0)
    "c2_z": (X + Y) % exp(-abs_(W)) / (1 + X % X),  # C++ precedence: ((X+Y)%exp(-|W|)) / (1+X%X)
    "diff": X - Y,                                  # norm_fro(X - Y)
    "u32_z": (X ^ Y) + 3 * W,                       # (X ^ Y) + 3*W mod 2^32
}


def addn(n: int) -> E:
    """A1 + A2 + ... + An, left to right as C++ evaluates it (Sec. 4, add-N)."""
    e = leaf(0)
    for q in range(1, n):
        e = e + leaf(q)
    return e


# The paper's element-wise benchmark expressions (Sec. 4) that need no strided
# views; beta, alpha are the scalars of swish and gelu.
def paper_expr(name: str, beta: float = 1.0, alpha: float = 0.044715) -> E:
    A, B = leaf(0), leaf(1)
    if name == "add2":
        return A + B
    if name == "add4":
        return addn(4)
    if name == "relu":                       # Z = X % (X > 0)
        return A % gt(A, 0.0)
    if name == "sigmoid":                    # Z = 1 / (1 + exp(-X))
        return 1 / (1 + exp(-A))
    if name == "swish":                      # Z = X / (1 + exp(-beta * X))
        return A / (1 + exp(-(beta * A)))
    if name == "gelu":                       # (X/2) % (1 + tanh(sqrt(2/pi) * (X + alpha*pow(X,3))))
        c = float(np.float32(math.sqrt(2 / math.pi)))
        return (A / 2) % (1 + tanh(c * (A + alpha * pow_(A, 3))))
    if name == "expr3":                      # 1 / (X % conv_to<fmat>::from(Y) + log(log(X + 2) % W))
        Wl = leaf(2)
        return 1 / (A % conv_to_f32(B) + log(log(A + 2) % Wl))
    raise KeyError(name)


def center(m: int, n: int):
    """The centre submatrix with half the rows and columns of an m x n
    matrix (Sec. 4): (r0, c0, rows, cols)."""
    R, C = m // 2, n // 2
    return (m - R) // 2, (n - C) // 2, R, C


def diag_len(m: int, n: int, k: int) -> int:
    return max(0, min(m, n - k) if k >= 0 else min(m + k, n))


# The paper's expressions with strided views (Sec. 4) over m x n inputs
# (column-major, leading dimension m).  Returns (expression, result shape).
def paper_view_expr(name: str, m: int, n: int, a: float = 2.0):
    if name in ("addsub2", "addsub4"):
        r0, c0, R, C = center(m, n)
        k = 2 if name == "addsub2" else 4
        e = submat(0, r0, c0, m)
        for q in range(1, k):
            e = e + submat(q, r0, c0, m)
        return e, (R, C)
    if name == "expr1":                      # Z = 2 * (X.t() + Y) + 2 * (X + Y.t())
        assert m == n
        X, Y = leaf(0), leaf(1)
        return 2 * (X.t() + Y) + 2 * (X + Y.t()), (m, n)
    if name == "expr2":                      # Z = a * A + (B + C).t() + log(pow(D, 2))
        assert m == n
        A, B, C, D = leaf(0), leaf(1), leaf(2), leaf(3)
        return a * A + (B + C).t() + log(pow_(D, 2)), (m, n)
    if name == "diagsum":                    # (X.diag(-1) + X.diag(1)) % (Y.diag(-1) + Y.diag(1))
        L = min(diag_len(m, n, -1), diag_len(m, n, 1))
        return ((diag(0, -1, m) + diag(0, 1, m)) % (diag(1, -1, m) + diag(1, 1, m))), (L, 1)
    raise KeyError(name)


def axy_expw(a: float) -> E:
    """Z = a*X % Y + exp(-W) for a run-time scalar a (the scalar is held in
    the compute type by the caller, so pass it already rounded)."""
    return a * X % Y + exp(-W)


# --------------------------------------------------------------------------


def _ptrs(inputs):
    arr = (ctypes.c_void_p * max(1, len(inputs)))()
    for i, x in enumerate(inputs):
        arr[i] = x.ctypes.data
    return arr


def compute_unit(dtype: str) -> float:
    return U64 if dtype == "f64" else U32


def evaluate(expr: E, inputs, dtype: str, shape=None, reduce=None, u_c=None,
             f_allow=None, input_dtypes=None):
    """Evaluate `expr` over stored inputs (numpy arrays of the storage dtype,
    bf16 as uint16 bit patterns).  shape=(n_rows, n_cols), column-major;
    default (n, 1).  input_dtypes: per-input storage dtypes when they differ
    from `dtype` (mixed-dtype leaves).  f_allow: the elementary functions'
    allowances {exp, log, tanh, pow} (default: F_ALLOW of the compute type).
    Returns (value, mu): arrays of FP64 values and running error bounds in
    units of u_c (default: the compute type's roundoff)."""
    inputs = [np.ascontiguousarray(x).reshape(-1, order="F") if x.ndim > 1 else
              np.ascontiguousarray(x) for x in inputs]
    n = inputs[0].size if inputs else 0
    if shape is None:
        shape = (n, 1)
    rows, cols = shape
    assert expr.n_inputs() <= len(inputs)
    order, _ = expr.nodes()
    views = any(e.op == "leaf" and e.view is not None for e in order)
    if views:
        voff, vrs, vcs = _views(order, inputs, rows, cols)
    else:
        assert all(x.size == rows * cols for x in inputs)
    if u_c is None:
        u_c = compute_unit(dtype)
    fa = F_ALLOW["f64" if dtype == "f64" else "f32"]
    if f_allow is not None:
        fa = dict(fa, **f_allow)
    fop = np.array([fa[k] for k in F_ORDER], np.float64)
    op, a, b, lf, cst = expr.arrays()
    red = REDUCE[reduce]
    nout = {0: rows * cols, 1: 1, 2: cols, 3: rows, 4: 1}[red]
    out = np.empty(max(nout, 1), np.float64)
    mu = np.empty(max(nout, 1), np.float64)
    dts = np.array([DTYPE[d] for d in (input_dtypes or [dtype] * len(inputs))] or [0],
                   dtype=np.int32)
    if views:
        rc = lib().or_eval_views(op.size, op.ctypes.data, a.ctypes.data, b.ctypes.data,
                                 lf.ctypes.data, cst.ctypes.data, len(inputs), _ptrs(inputs),
                                 dts.ctypes.data, rows, cols, red, u_c, fop.ctypes.data, voff.ctypes.data,
                                 vrs.ctypes.data, vcs.ctypes.data, out.ctypes.data,
                                 mu.ctypes.data)
    else:
        rc = lib().or_eval(op.size, op.ctypes.data, a.ctypes.data, b.ctypes.data,
                           lf.ctypes.data, cst.ctypes.data, len(inputs), _ptrs(inputs),
                           dts.ctypes.data, rows, cols, red, u_c, fop.ctypes.data, out.ctypes.data,
                           mu.ctypes.data)
    if rc != 0:
        raise ValueError("oracle evaluation failed (%d)" % rc)
    return out[:nout], mu[:nout]


def _views(order, inputs, rows, cols):
    """Per-node (off, rs, cs) arrays for an expression of shape rows x cols;
    every view must stay inside its input."""
    voff = np.zeros(len(order), np.int64)
    vrs = np.ones(len(order), np.int64)
    vcs = np.full(len(order), rows, np.int64)
    for k, e in enumerate(order):
        if e.op != "leaf":
            continue
        v = e.view
        if v is None:
            v = (0, 1, rows)          # dense rows x cols
        elif v == "T":
            v = (0, cols, 1)          # the transpose of a dense cols x rows input
        voff[k], vrs[k], vcs[k] = v
        if rows * cols:
            idx = [v[0] + r * v[1] + c * v[2] for r in (0, rows - 1) for c in (0, cols - 1)]
            assert 0 <= min(idx) and max(idx) < inputs[e.leaf].size, "view outside its input"
    return voff, vrs, vcs


def evaluate_u32(expr: E, inputs):
    """Integer tree over u32 inputs; returns (values u32[n], full u64 sum)."""
    inputs = [np.ascontiguousarray(x, dtype=np.uint32) for x in inputs]
    n = inputs[0].size
    op, a, b, lf, cst = expr.arrays()
    out = np.empty(max(n, 1), np.uint32)
    tot = np.zeros(1, np.uint64)
    rc = lib().or_eval_u32(op.size, op.ctypes.data, a.ctypes.data, b.ctypes.data,
                           lf.ctypes.data, cst.ctypes.data, len(inputs), _ptrs(inputs),
                           n, out.ctypes.data, tot.ctypes.data)
    if rc != 0:
        raise ValueError("oracle evaluation failed (%d)" % rc)
    return out[:n], int(tot[0])


# --------------------------------------------------------------------------
# The acceptance rule for floating-point results.


def allowed_error(value, mu, dtype: str, out_dtype: str | None = None):
    """Largest admissible |result - value| for a result computed in the
    compute type of `dtype`:  max(tol*|value|, 4*u_c*mu).  If the result is
    stored in a half format (`out_dtype` bf16/f16), the final rounding adds
    u_half*(|value| + that) plus half the subnormal spacing."""
    value = np.asarray(value, np.float64)
    mu = np.asarray(mu, np.float64)
    u_c = compute_unit(dtype)
    base = np.maximum(TOL[dtype] * np.abs(value), 4.0 * u_c * mu)
    if out_dtype in U_HALF:
        base = 4.0 * u_c * mu + U_HALF[out_dtype] * (np.abs(value) + 4.0 * u_c * mu) \
            + HALF_SUBNORMAL_HALF_SPACING[out_dtype]
    return base


def check(result, value, mu, dtype: str, out_dtype: str | None = None):
    """Element-wise pass mask plus a small report.  NaN must match NaN,
    infinities must match in sign, and where the running bound is undefined
    (NaN) the result must equal the value exactly."""
    r = np.asarray(result, np.float64)
    v = np.asarray(value, np.float64)
    lim = allowed_error(v, mu, dtype, out_dtype)
    with np.errstate(invalid="ignore", over="ignore"):
        err = np.abs(r - v)
        ok = err <= lim
    nan = np.isnan(v)
    ok = np.where(nan, np.isnan(r), ok)
    # The first-order bound is undefined where it meets 0 * inf (e.g. past a
    # log(0) = -inf that a division turns into a zero): there the result must
    # equal the exact value.
    undefined = ~nan & np.isnan(np.asarray(mu, np.float64))
    ok = np.where(undefined, r == v, ok)
    inf = np.isinf(v)
    ok = np.where(inf, r == v, ok)
    if out_dtype == "f16":
        # values at or beyond the FP16 overflow threshold round to +-inf
        ovf = ~inf & (np.abs(v) >= F16_OVERFLOW)
        ok = np.where(ovf, r == np.copysign(np.inf, v), ok)
    # results that pass only through the running-bound branch: beyond the
    # pure relative bound (the tolerance, or for a half-format output its
    # final rounding, u_half |v|), yet within the allowed error
    rel_tol = U_HALF[out_dtype] if out_dtype in U_HALF else TOL[dtype]
    with np.errstate(invalid="ignore", divide="ignore"):
        rel = np.where(v != 0, err / np.abs(v), err)
        # infinities that match (FP16 overflow) are reported as exact
        rel = np.where(np.isinf(r) & ok, 0.0, rel)
        lim = np.where(np.isinf(r) & ok, 1.0, lim)
        err = np.where(np.isinf(r) & ok, 0.0, err)
    with np.errstate(invalid="ignore", divide="ignore"):
        over = np.where(lim > 0, err / np.where(lim > 0, lim, 1.0), err)
    report = {
        "n": int(r.size),
        "fail": int(r.size - np.count_nonzero(ok)),
        "max_rel": float(np.nanmax(rel)) if r.size else 0.0,
        "max_err_over_allowed": float(np.nanmax(over)) if r.size else 0.0,
        "needed_mu_branch": int(np.count_nonzero(ok & ~np.isinf(r) & (err > rel_tol * np.abs(v)))),
    }
    return ok, report


def ceil_log2(n: int) -> int:
    return 0 if n <= 1 else math.ceil(math.log2(n))
