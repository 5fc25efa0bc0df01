"""Python binding of libfx.so, the fused element-wise expression library for
MI355X (gfx950).

Argument marshalling only: every function forwards to the C entry point of
the same name in ``include/fx.h``.  Tensors are torch tensors on a ROCm
device (their data pointers are passed through); the stream defaults to
torch's current stream.  There is no fallback: if the HIP library is missing
or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfx.so")

F32, F64, BF16, F16, U32 = 0, 1, 2, 3, 4
R_ACCU, R_COLSUM, R_ROWSUM, R_NORM, R_DOT = 1, 2, 3, 4, 5
OP = {"neg": 1, "abs": 2, "exp": 3, "sqrt": 4, "log": 5, "tanh": 6, "add": 10, "sub": 11,
      "schur": 12, "div": 13, "xor": 14, "sadd": 20, "smul": 21, "sdiv": 22, "srdiv": 23,
      "ssub": 24, "srsub": 25, "spow": 26, "leaf": 30, "const": 31}
NODE_OP = dict(OP, mul=OP["schur"])  # tree nodes name the Schur product "mul"
EXPR = {"c1_z": 1, "accu_xy": 2, "c2_z": 3, "c2_colsum": 4, "c2_rowsum": 5, "norm_diff": 6,
        "colsum_xy": 7, "axy_expw": 8}
STATUS = {0: "FX_OK", 1: "FX_E_ARG", 2: "FX_E_SHAPE", 3: "FX_E_DTYPE", 4: "FX_E_WORKSPACE",
          5: "FX_E_HIP", 6: "FX_E_UNSUPPORTED", 7: "FX_E_CONFIG"}


class FxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class Launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("ept", ctypes.c_int32),
                ("vec_bytes", ctypes.c_int32), ("split", ctypes.c_int32)]

    def as_tuple(self):
        return (self.block, self.ept, self.vec_bytes, self.split)


class Shape(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64)]


class Node(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("a", ctypes.c_int32), ("b", ctypes.c_int32),
                ("input", ctypes.c_int32), ("value", ctypes.c_double)]


class TapeInfo(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_inputs", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("n_instructions", ctypes.c_int32),
                ("n_slots", ctypes.c_int32), ("n_consts", ctypes.c_int32),
                ("op_count", ctypes.c_int32 * 8)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "op_count"}
        d["op_count"] = list(self.op_count)
        return d


class BatchItem(ctypes.Structure):
    _fields_ = [("tape", ctypes.c_void_p), ("inputs", ctypes.c_void_p * 4),
                ("out", ctypes.c_void_p), ("n", ctypes.c_int64), ("kind", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("block", ctypes.c_int32), ("ept", ctypes.c_int32),
                ("vec_bytes", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("n_tiles", ctypes.c_int64), ("tile_elems", ctypes.c_int64),
                ("bytes", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_D = ctypes.c_double
_LP = ctypes.POINTER(Launch)

# name -> (restype, argtypes)
_SIGS = {
    "fx_version": (ctypes.c_char_p, []),
    "fx_last_error": (ctypes.c_char_p, []),
    "fx_synchronize": (_I, [_P]),
    "fx_workspace_bytes": (_SZ, [_I, _I, Shape, _LP]),
    "fx_resolve_launch": (_I, [_I, _I, Shape, _LP, _LP]),
    "fx_c1_z": (_I, [_I, _P, _P, _P, _P, _I64, _LP, _P]),
    "fx_axy_expw": (_I, [_I, _D, _P, _P, _P, _P, _I64, _LP, _P]),
    "fx_accu_xy": (_I, [_I, _P, _P, _I64, _P, _P, _SZ, _LP, _P]),
    "fx_dot": (_I, [_I, _P, _P, _I64, _P, _P, _SZ, _LP, _P]),
    "fx_c2_z": (_I, [_I, _P, _P, _P, _P, Shape, _LP, _P]),
    "fx_c2_colsum": (_I, [_I, _P, _P, _P, _P, Shape, _P, _SZ, _LP, _P]),
    "fx_c2_rowsum": (_I, [_I, _P, _P, _P, _P, Shape, _P, _SZ, _LP, _P]),
    "fx_norm_fro_diff": (_I, [_I, _P, _P, Shape, _P, _P, _SZ, _LP, _P]),
    "fx_colsum_xy": (_I, [_I, _P, _P, _P, Shape, _P, _SZ, _LP, _P]),
    "fx_paper_expr": (_I, [_I, _I, ctypes.POINTER(_P), ctypes.POINTER(_D), _P, Shape, _LP, _P]),
    "fx_addn": (_I, [_I, ctypes.POINTER(_P), ctypes.c_int32, _P, Shape, _LP, _P]),
    "fx_paper_view_shape": (_I, [_I, Shape, ctypes.POINTER(Shape)]),
    "fx_paper_view_expr": (_I, [_I, _I, ctypes.POINTER(_P), ctypes.POINTER(_D), _P, Shape, _P]),
    "fx_op_unary": (_I, [_I, _I, _P, _P, _I64, _LP, _P]),
    "fx_op_binary": (_I, [_I, _I, _P, _P, _P, _I64, _LP, _P]),
    "fx_op_scalar": (_I, [_I, _I, _P, _D, _P, _I64, _LP, _P]),
    "fx_reduce": (_I, [_I, _I, _P, _P, Shape, _P, _P, _SZ, _LP, _P]),
    "fx_unfused_tmp_bytes": (_SZ, [_I, _I, Shape]),
    "fx_unfused": (_I, [_I, _I, ctypes.POINTER(_P), _D, _P, Shape, _P, _SZ, _P, _SZ, _LP, _P]),
    "fx_tape_create": (_I, [ctypes.POINTER(Node), ctypes.c_int32, ctypes.POINTER(_P)]),
    "fx_tape_destroy": (None, [_P]),
    "fx_tape_describe": (_I, [_P, ctypes.POINTER(TapeInfo)]),
    "fx_tape_program": (ctypes.c_int32, [_P, _P, _P, _P, _P, ctypes.c_int32]),
    "fx_rtc_create": (_I, [ctypes.POINTER(Node), ctypes.c_int32, _I, _I, ctypes.POINTER(_P)]),
    "fx_rtc_destroy": (None, [_P]),
    "fx_rtc_source": (_I, [_P, ctypes.c_char_p, _SZ, ctypes.POINTER(_SZ)]),
    "fx_rtc_compile_ms": (ctypes.c_double, [_P]),
    "fx_rtc_eval": (_I, [_P, ctypes.POINTER(_P), ctypes.c_int32, Shape, _P, _P, _SZ, _P]),
    "fx_source_eval": (_I, [_I, _I, ctypes.POINTER(_P), _D, _P, Shape, _P, _SZ, _P]),
    "fx_source_text": (_I, [_I, _I, ctypes.c_char_p, _SZ, ctypes.POINTER(_SZ)]),
    "fx_source_prepare": (_I, [_I, _I, ctypes.POINTER(_D)]),
    "fx_tape_eval": (_I, [_P, _I, ctypes.POINTER(_P), ctypes.c_int32, Shape, _I, _P, _P, _SZ,
                          _LP, _P]),
    "fx_tape_eval_static": (_I, [_P, _I, ctypes.POINTER(_P), ctypes.c_int32, Shape, _I, _P, _LP,
                                 _P]),
    "fx_batch_create": (_I, [ctypes.POINTER(BatchItem), ctypes.c_int32, _I, _LP, _I64,
                             ctypes.POINTER(_P)]),
    "fx_batch_launch": (_I, [_P, _P]),
    "fx_batch_graph": (_I, [_P, _P]),
    "fx_batch_launch_each": (_I, [_P, _P]),
    "fx_batch_describe": (_I, [_P, ctypes.POINTER(BatchInfo)]),
    "fx_batch_destroy": (None, [_P]),
    "fx_tune_time": (_I, [_P, _I, ctypes.POINTER(_P), ctypes.c_int32, Shape, _I, _P, _P, _SZ,
                          _LP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                          ctypes.POINTER(ctypes.c_float), _P]),
    "fx_tune_grid": (ctypes.c_int32, [_I, _I, _LP, ctypes.c_int32]),
    "fx_autotune": (_I, [_P, _I, ctypes.POINTER(_P), ctypes.c_int32, Shape, _I, _P, _P, _SZ,
                         ctypes.c_int32, ctypes.c_int32, _LP, ctypes.POINTER(ctypes.c_float),
                         ctypes.c_char_p, _P]),
    "fx_model_create": (_I, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                             ctypes.c_int32, ctypes.POINTER(_P)]),
    "fx_model_num_params": (ctypes.c_int32, [_P]),
    "fx_model_set": (_I, [_P, _P, _P, _P]),
    "fx_model_get": (_I, [_P, _P, _P, _P]),
    "fx_model_train_step": (_I, [_P, _P, _P, ctypes.c_int32, ctypes.c_float, _P, _P]),
    "fx_model_train": (_I, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                            ctypes.c_float, _P, _P, _P]),
    "fx_model_grad": (_I, [_P, _P, _P, ctypes.c_int32, _P, _P, _P]),
    "fx_model_forward": (_I, [_P, _P, ctypes.c_int32, _P, _P, _P]),
    "fx_model_choose": (_I, [_P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int32)]),
    "fx_model_destroy": (None, [_P]),
    "fx_tape_features": (ctypes.c_int32, [_P, _I, Shape, _I, ctypes.POINTER(ctypes.c_float),
                                          ctypes.c_int32]),
    "fx_model_load": (_I, [ctypes.c_char_p, ctypes.POINTER(_P)]),
    "fx_tape_set_model": (_I, [_P, _P]),
    "fx_model_predict": (_I, [_P, ctypes.POINTER(ctypes.c_float), _I, _I, _LP]),
    "fx_bw_copy": (_I, [_P, _P, _SZ, _LP, _P]),
    "fx_bw_read": (_I, [_P, _SZ, _P, _LP, _P]),
    "fx_bw_write": (_I, [_P, _SZ, ctypes.c_uint32, _LP, _P]),
    "fx_bw_triad": (_I, [_P, _P, _P, _P, _SZ, _I, _LP, _P]),
}

_lib = None


def lib():
    """The loaded libfx.so.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime; loading it first lets libfx.so bind
        # to that same runtime (one runtime per process) instead of a second
        # copy from /opt/rocm.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise FxError(-1, "%s is missing: run paper_2604_22242_amd.build first" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return sorted(_SIGS)


# ---- marshalling helpers ----------------------------------------------------


def dtype_code(t) -> int:
    import torch
    m = {torch.float32: F32, torch.float64: F64, torch.bfloat16: BF16, torch.float16: F16,
         torch.uint32: U32, torch.int32: U32}
    try:
        return m[t.dtype]
    except KeyError:
        raise FxError(3, "unsupported tensor dtype %s" % t.dtype) from None


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _cfg(cfg):
    if cfg is None:
        return None
    if isinstance(cfg, Launch):
        return ctypes.pointer(cfg)
    if isinstance(cfg, dict):
        cfg = (cfg.get("block", 0), cfg.get("ept", 0), cfg.get("vec_bytes", 0), cfg.get("split", 0))
    return ctypes.pointer(Launch(*cfg))


def _shape(s):
    if isinstance(s, Shape):
        return s
    return Shape(int(s[0]), int(s[1]))


def check(rc):
    if rc != 0:
        raise FxError(rc, lib().fx_last_error().decode())
    return rc


def _shape_of(t, shape):
    if shape is not None:
        return _shape(shape)
    if t.dim() == 2:  # a column-major matrix is handed over as its transpose's storage
        return Shape(t.shape[0], t.shape[1])
    return Shape(t.numel(), 1)


# ---- library ------------------------------------------------------------------


def fx_version() -> str:
    return lib().fx_version().decode()


def fx_last_error() -> str:
    return lib().fx_last_error().decode()


def fx_synchronize(stream=None):
    return check(lib().fx_synchronize(_stream(stream)))


def fx_workspace_bytes(kind, dt, shape, cfg=None) -> int:
    return lib().fx_workspace_bytes(kind, dt, _shape(shape), _cfg(cfg))


def fx_resolve_launch(kind, dt, shape, cfg=None) -> tuple:
    out = Launch()
    check(lib().fx_resolve_launch(kind, dt, _shape(shape), _cfg(cfg), ctypes.pointer(out)))
    return out.as_tuple()


def workspace(kind, dt, shape, cfg=None, device=None):
    """A zero-filled device workspace for reduction `kind` (None if none is
    needed)."""
    import torch
    nb = fx_workspace_bytes(kind, dt, shape, cfg)
    if nb == 0:
        return None
    return torch.zeros(nb, dtype=torch.uint8, device=device or "cuda")


def _ws(ws):
    if ws is None:
        return None, 0
    return ws.data_ptr(), ws.numel() * ws.element_size()


# ---- fused entry points -----------------------------------------------------------


def fx_c1_z(X, Y, W, Z, cfg=None, stream=None, n=None):
    n = X.numel() if n is None else n
    return check(lib().fx_c1_z(dtype_code(X), _ptr(X), _ptr(Y), _ptr(W), _ptr(Z), n, _cfg(cfg),
                               _stream(stream)))


def fx_axy_expw(a, X, Y, W, Z, cfg=None, stream=None, n=None):
    n = X.numel() if n is None else n
    return check(lib().fx_axy_expw(dtype_code(X), float(a), _ptr(X), _ptr(Y), _ptr(W), _ptr(Z),
                                   n, _cfg(cfg), _stream(stream)))


def fx_accu_xy(X, Y, out, ws=None, cfg=None, stream=None, n=None):
    n = X.numel() if n is None else n
    p, nb = _ws(ws)
    return check(lib().fx_accu_xy(dtype_code(X), _ptr(X), _ptr(Y), n, _ptr(out), p, nb,
                                  _cfg(cfg), _stream(stream)))


def fx_dot(X, Y, out, ws=None, cfg=None, stream=None, n=None):
    n = X.numel() if n is None else n
    p, nb = _ws(ws)
    return check(lib().fx_dot(dtype_code(X), _ptr(X), _ptr(Y), n, _ptr(out), p, nb, _cfg(cfg),
                              _stream(stream)))


def fx_c2_z(X, Y, W, Z, shape, cfg=None, stream=None):
    return check(lib().fx_c2_z(dtype_code(X), _ptr(X), _ptr(Y), _ptr(W), _ptr(Z), _shape(shape),
                               _cfg(cfg), _stream(stream)))


def fx_c2_colsum(X, Y, W, out, shape, ws=None, cfg=None, stream=None):
    p, nb = _ws(ws)
    return check(lib().fx_c2_colsum(dtype_code(X), _ptr(X), _ptr(Y), _ptr(W), _ptr(out),
                                    _shape(shape), p, nb, _cfg(cfg), _stream(stream)))


def fx_c2_rowsum(X, Y, W, out, shape, ws=None, cfg=None, stream=None):
    p, nb = _ws(ws)
    return check(lib().fx_c2_rowsum(dtype_code(X), _ptr(X), _ptr(Y), _ptr(W), _ptr(out),
                                    _shape(shape), p, nb, _cfg(cfg), _stream(stream)))


def fx_norm_fro_diff(X, Y, out, shape, ws=None, cfg=None, stream=None):
    p, nb = _ws(ws)
    return check(lib().fx_norm_fro_diff(dtype_code(X), _ptr(X), _ptr(Y), _shape(shape),
                                        _ptr(out), p, nb, _cfg(cfg), _stream(stream)))


def fx_colsum_xy(X, Y, out, shape, ws=None, cfg=None, stream=None):
    p, nb = _ws(ws)
    return check(lib().fx_colsum_xy(dtype_code(X), _ptr(X), _ptr(Y), _ptr(out), _shape(shape),
                                    p, nb, _cfg(cfg), _stream(stream)))


PAPER = {"add2": 1, "add4": 2, "relu": 3, "sigmoid": 4, "swish": 5, "gelu": 6, "expr3": 7}


def fx_paper_expr(which, inputs, Z, shape, scalars=(), cfg=None, stream=None, dt=None):
    arr = (_P * max(1, len(inputs)))(*[_ptr(t) for t in inputs])
    sc = (_D * max(1, len(scalars)))(*scalars) if scalars else None
    dt = dtype_code(inputs[0]) if dt is None else dt
    return check(lib().fx_paper_expr(PAPER.get(which, which), dt, arr, sc, _ptr(Z), _shape(shape),
                                     _cfg(cfg), _stream(stream)))


PAPER_VIEW = {"addsub2": 16, "addsub4": 17, "expr1": 18, "expr2": 19, "diagsum": 20}


def fx_paper_view_shape(which, shape):
    """(rows, cols) of a view expression's result over inputs of `shape`."""
    out = Shape()
    check(lib().fx_paper_view_shape(PAPER_VIEW.get(which, which), _shape(shape), ctypes.byref(out)))
    return (out.n_rows, out.n_cols)


def fx_paper_view_expr(which, inputs, Z, shape, scalars=(), stream=None, dt=None):
    """One of the paper's strided-view expressions over m x n inputs
    (shape = (m, n)); Z is dense, of fx_paper_view_shape(which, shape)."""
    arr = (_P * max(1, len(inputs)))(*[_ptr(t) for t in inputs])
    sc = (_D * max(1, len(scalars)))(*scalars) if scalars else None
    dt = dtype_code(inputs[0]) if dt is None else dt
    return check(lib().fx_paper_view_expr(PAPER_VIEW.get(which, which), dt, arr, sc, _ptr(Z),
                                          _shape(shape), _stream(stream)))


def fx_addn(inputs, Z, shape, cfg=None, stream=None):
    arr = (_P * max(1, len(inputs)))(*[_ptr(t) for t in inputs])
    return check(lib().fx_addn(dtype_code(inputs[0]), arr, len(inputs), _ptr(Z), _shape(shape),
                               _cfg(cfg), _stream(stream)))


# ---- unfused baseline -----------------------------------------------------------------


def fx_op_unary(op, A, out, cfg=None, stream=None):
    return check(lib().fx_op_unary(OP.get(op, op), dtype_code(A), _ptr(A), _ptr(out), A.numel(),
                                   _cfg(cfg), _stream(stream)))


def fx_op_binary(op, A, B, out, cfg=None, stream=None):
    return check(lib().fx_op_binary(OP.get(op, op), dtype_code(A), _ptr(A), _ptr(B), _ptr(out),
                                    A.numel(), _cfg(cfg), _stream(stream)))


def fx_op_scalar(op, A, k, out, cfg=None, stream=None):
    return check(lib().fx_op_scalar(OP.get(op, op), dtype_code(A), _ptr(A), float(k), _ptr(out),
                                    A.numel(), _cfg(cfg), _stream(stream)))


def fx_reduce(kind, A, B, out, shape, ws=None, cfg=None, stream=None):
    p, nb = _ws(ws)
    return check(lib().fx_reduce(kind, dtype_code(A), _ptr(A), _ptr(B), _shape(shape), _ptr(out),
                                 p, nb, _cfg(cfg), _stream(stream)))


def fx_unfused_tmp_bytes(expr, dt, shape) -> int:
    return lib().fx_unfused_tmp_bytes(EXPR.get(expr, expr), dt, _shape(shape))


def fx_unfused(expr, inputs, out, shape, tmp, ws=None, a=0.0, cfg=None, stream=None):
    arr = (_P * 3)(*[_ptr(t) for t in inputs] + [None] * (3 - len(inputs)))
    p, nb = _ws(ws)
    tp, tb = _ws(tmp)
    return check(lib().fx_unfused(EXPR.get(expr, expr), dtype_code(inputs[0]), arr, float(a),
                                  _ptr(out), _shape(shape), tp, tb, p, nb, _cfg(cfg),
                                  _stream(stream)))


# ---- run-time tapes --------------------------------------------------------------------


def nodes_array(nodes):
    """Tree nodes (op, a, b, input, value), children first, as fx_node[]."""
    arr = (Node * len(nodes))()
    for i, (op, a, b, inp, val) in enumerate(nodes):
        arr[i] = Node(NODE_OP[op] if isinstance(op, str) else op, a, b, inp, val)
    return arr


class Tape:
    """An fx_tape handle (compiled on creation, destroyed with the object)."""

    def __init__(self, nodes):
        self.handle = ctypes.c_void_p()
        arr = nodes_array(nodes)
        check(lib().fx_tape_create(arr, len(nodes), ctypes.byref(self.handle)))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fx_tape_destroy(self.handle)
            self.handle = None

    def info(self) -> dict:
        return fx_tape_describe(self)

    def program(self):
        return fx_tape_program(self)

    def set_model(self, model):
        """fx_tape_set_model: evaluations that leave the launch configuration
        to the library take `model`'s pick (None detaches).  The tape keeps a
        reference, so the model outlives the attachment."""
        check(lib().fx_tape_set_model(self.handle, model.handle if model is not None else None))
        self._model = model


def fx_tape_set_model(tape: Tape, model):
    tape.set_model(model)


def fx_tape_create(nodes) -> Tape:
    return Tape(nodes)


def fx_tape_destroy(tape: Tape):
    if tape.handle:
        lib().fx_tape_destroy(tape.handle)
        tape.handle = None


def fx_tape_describe(tape: Tape) -> dict:
    info = TapeInfo()
    check(lib().fx_tape_describe(tape.handle, ctypes.byref(info)))
    return info.as_dict()


TAPE_OPCODES = ("LD", "LDI", "ST", "ADD_S", "ADD_I", "SUB_S", "SUB_I", "RSUB_S", "RSUB_I",
                "MUL_S", "MUL_I", "DIV_S", "DIV_I", "RDIV_S", "RDIV_I", "NEG", "ABS", "EXP",
                "SQRT", "STLD")
TAPE_ABS_IN, TAPE_NEG_IN, TAPE_LD_IN = 0x100, 0x200, 0x400


def fx_tape_program(tape: Tape):
    """The compiled instructions as a list of (opcode name, slot, slot2,
    immediate); input modifiers are appended to the name in the order they
    apply ("ADD_I|ld|abs": acc = |s[slot2]| + imm)."""
    n = lib().fx_tape_program(tape.handle, None, None, None, None, 0)
    if n < 0:
        check(-n)
    op = (ctypes.c_uint16 * max(1, n))()
    slot = (ctypes.c_uint8 * max(1, n))()
    slot2 = (ctypes.c_uint8 * max(1, n))()
    imm = (ctypes.c_double * max(1, n))()
    lib().fx_tape_program(tape.handle, op, slot, slot2, imm, n)

    def name(code):
        mods = (("|ld" if code & TAPE_LD_IN else "") + ("|abs" if code & TAPE_ABS_IN else "") +
                ("|neg" if code & TAPE_NEG_IN else ""))
        return TAPE_OPCODES[code & 0xFF] + mods
    return [(name(op[i]), slot[i], slot2[i], imm[i]) for i in range(n)]


def fx_tape_eval(tape: Tape, inputs, out, shape, kind=0, ws=None, cfg=None, stream=None,
                 dt=None):
    arr = (_P * max(1, len(inputs)))(*[_ptr(t) for t in inputs])
    if dt is None:
        dt = dtype_code(inputs[0]) if inputs else dtype_code(out)
    p, nb = _ws(ws)
    return check(lib().fx_tape_eval(tape.handle, dt, arr, len(inputs), _shape(shape), kind,
                                    _ptr(out), p, nb, _cfg(cfg), _stream(stream)))


def fx_tape_eval_static(tape: Tape, inputs, out, shape, kind=0, cfg=None, stream=None, dt=None):
    """fx_tape_eval with the library's static device scratch as the
    reductions' workspace: the call allocates nothing."""
    arr = (_P * max(1, len(inputs)))(*[_ptr(t) for t in inputs])
    if dt is None:
        dt = dtype_code(inputs[0]) if inputs else dtype_code(out)
    return check(lib().fx_tape_eval_static(tape.handle, dt, arr, len(inputs), _shape(shape), kind,
                                           _ptr(out), _cfg(cfg), _stream(stream)))


# ---- run-time source mode ----------------------------------------------------------------


class Rtc:
    """An fx_rtc handle: the generated kernel of a tree and result kind
    (0: element-wise, or R_ACCU / R_NORM / R_COLSUM / R_ROWSUM), compiled
    with hipRTC (or found in the per-process cache) on creation."""

    def __init__(self, nodes, dt=F32, kind=0):
        self.handle = ctypes.c_void_p()
        self.kind = kind
        arr = nodes_array(nodes)
        check(lib().fx_rtc_create(arr, len(nodes), dt, kind, ctypes.byref(self.handle)))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fx_rtc_destroy(self.handle)
            self.handle = None

    def source(self) -> str:
        return fx_rtc_source(self)

    def compile_ms(self) -> float:
        return lib().fx_rtc_compile_ms(self.handle)

    def eval(self, inputs, out, shape=None, ws=None, stream=None):
        return fx_rtc_eval(self, inputs, out, shape, ws, stream)


def fx_rtc_create(nodes, dt=F32, kind=0) -> Rtc:
    return Rtc(nodes, dt, kind)


def fx_source_eval(expr, inputs, out, shape, ws=None, a=0.0, stream=None, dt=None):
    """A workload expression (EXPR names or FX_EXPR_* codes) through its kernel
    generated as source from the expression type (compiled at first use)."""
    arr = (_P * 3)(*([_ptr(t) for t in inputs] + [None] * (3 - len(inputs))))
    p, nb = _ws(ws)
    dt = dtype_code(inputs[0]) if dt is None else dt
    return check(lib().fx_source_eval(EXPR.get(expr, expr), dt, arr, float(a), _ptr(out),
                                      _shape(shape), p, nb, _stream(stream)))


def fx_source_text(expr, dt) -> str:
    n = _SZ()
    check(lib().fx_source_text(EXPR.get(expr, expr), dt, None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    check(lib().fx_source_text(EXPR.get(expr, expr), dt, buf, n.value + 1, ctypes.byref(n)))
    return buf.value.decode()


def fx_source_prepare(expr, dt) -> float:
    """Compile (expr, dt)'s generated text if not yet done; returns the
    milliseconds that compilation took."""
    ms = _D()
    check(lib().fx_source_prepare(EXPR.get(expr, expr), dt, ctypes.byref(ms)))
    return ms.value


def fx_rtc_source(r: Rtc) -> str:
    n = _SZ()
    check(lib().fx_rtc_source(r.handle, None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    check(lib().fx_rtc_source(r.handle, buf, n.value + 1, ctypes.byref(n)))
    return buf.value.decode()


def fx_rtc_eval(r: Rtc, inputs, out, shape=None, ws=None, stream=None):
    """shape defaults to (out.numel(), 1) for element-wise kernels."""
    if shape is None:
        if r.kind != 0:
            raise ValueError("a reduction needs the inputs' shape")
        shape = (out.numel(), 1)
    arr = (_P * max(1, len(inputs)))(*[_ptr(t) for t in inputs])
    p, nb = _ws(ws)
    return check(lib().fx_rtc_eval(r.handle, arr, len(inputs), _shape(shape), _ptr(out), p, nb,
                                   _stream(stream)))


# ---- batches ----------------------------------------------------------------------------


class Batch:
    """An fx_batch handle.  items: (tape, [inputs], out, n, kind) tuples; the
    tensors must stay alive while the batch is used (the binding keeps
    references to them)."""

    def __init__(self, items, dt, cfg=None, tile_elems=0):
        arr = (BatchItem * max(1, len(items)))()
        self._keep = []
        for i, (tape, ins, out, n, kind) in enumerate(items):
            bi = BatchItem()
            bi.tape = tape.handle
            for q, t in enumerate(ins):
                bi.inputs[q] = _ptr(t)
            bi.out = _ptr(out)
            bi.n = int(n)
            bi.kind = int(kind)
            arr[i] = bi
            self._keep.append((tape, ins, out))
        self.handle = ctypes.c_void_p()
        check(lib().fx_batch_create(arr, len(items), dt, _cfg(cfg), int(tile_elems),
                                    ctypes.byref(self.handle)))

    def launch(self, stream=None):
        return check(lib().fx_batch_launch(self.handle, _stream(stream)))

    def graph(self, stream=None):
        return check(lib().fx_batch_graph(self.handle, _stream(stream)))

    def launch_each(self, stream=None):
        return check(lib().fx_batch_launch_each(self.handle, _stream(stream)))

    def info(self) -> dict:
        inf = BatchInfo()
        check(lib().fx_batch_describe(self.handle, ctypes.byref(inf)))
        return inf.as_dict()

    def destroy(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fx_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.destroy()


def fx_batch_create(items, dt, cfg=None, tile_elems=0) -> Batch:
    return Batch(items, dt, cfg, tile_elems)


def fx_batch_launch(batch: Batch, stream=None):
    return batch.launch(stream)


def fx_batch_graph(batch: Batch, stream=None):
    return batch.graph(stream)


def fx_batch_launch_each(batch: Batch, stream=None):
    return batch.launch_each(stream)


def fx_batch_describe(batch: Batch) -> dict:
    return batch.info()


def fx_batch_destroy(batch: Batch):
    batch.destroy()


# ---- autotuning ---------------------------------------------------------------------------


def fx_tune_time(tape: Tape, inputs, out, shape, kind, cfgs, ws=None, warmup=2, reps=5,
                 stream=None, dt=None):
    """Times (ms) of `tape` under each configuration: a len(cfgs) x reps list."""
    arr = (_P * max(1, len(inputs)))(*[_ptr(t) for t in inputs])
    if dt is None:
        dt = dtype_code(inputs[0]) if inputs else dtype_code(out)
    carr = (Launch * max(1, len(cfgs)))(*[Launch(*c) for c in cfgs])
    ms = (ctypes.c_float * (max(1, len(cfgs)) * reps))()
    p, nb = _ws(ws)
    check(lib().fx_tune_time(tape.handle, dt, arr, len(inputs), _shape(shape), kind, _ptr(out),
                             p, nb, carr, len(cfgs), warmup, reps, ms, _stream(stream)))
    return [[ms[c * reps + r] for r in range(reps)] for c in range(len(cfgs))]


def fx_tape_features(tape: Tape, dt, shape, kind=0) -> list:
    """The cost model's 25 features of `tape` at this dtype, shape and kind."""
    out = (ctypes.c_float * 25)()
    n = lib().fx_tape_features(tape.handle, dt, _shape(shape), kind, out, 25)
    if n < 0:
        check(-n)
    return [out[i] for i in range(n)]


def fx_tune_grid(kind, dt) -> list:
    """The autotuner's configuration grid (145 tuples, the default last)."""
    n = lib().fx_tune_grid(kind, dt, None, 0)
    if n < 0:
        check(-n)
    arr = (Launch * n)()
    check(-min(0, lib().fx_tune_grid(kind, dt, arr, n)))
    return [arr[i].as_tuple() for i in range(n)]


def fx_autotune(tape: Tape, inputs, out, shape, kind=0, ws=None, warmup=2, reps=5, dt=None,
                db=None, stream=None):
    """Exhaustive search over fx_tune_grid: (best configuration, its median
    ms).  With `db` (a path), the search's record is appended to that JSON
    lines timing database."""
    arr = (_P * max(1, len(inputs)))(*[_ptr(t) for t in inputs])
    if dt is None:
        dt = dtype_code(inputs[0]) if inputs else dtype_code(out)
    best = Launch()
    ms = ctypes.c_float()
    p, nb = _ws(ws)
    check(lib().fx_autotune(tape.handle, dt, arr, len(inputs), _shape(shape), kind, _ptr(out), p,
                            nb, warmup, reps, ctypes.byref(best), ctypes.byref(ms),
                            None if db is None else os.fsencode(db), _stream(stream)))
    return best.as_tuple(), ms.value


# ---- learned cost model -------------------------------------------------------------------


class Model:
    """An fx_model handle (a two-layer perceptron with one softmax head per
    launch knob)."""

    def __init__(self, n_features, hidden, heads):
        self.n_features, self.hidden, self.heads = n_features, hidden, tuple(heads)
        hs = (ctypes.c_int32 * len(heads))(*heads)
        self.handle = ctypes.c_void_p()
        check(lib().fx_model_create(n_features, hidden, hs, len(heads),
                                    ctypes.byref(self.handle)))

    @property
    def n_params(self):
        return lib().fx_model_num_params(self.handle)

    def set(self, params=None, mean=None, std=None):
        import numpy as np
        def p(a):
            return None if a is None else np.ascontiguousarray(a, np.float32)
        params, mean, std = p(params), p(mean), p(std)
        self._hold = (params, mean, std)
        check(lib().fx_model_set(self.handle, *[None if a is None else a.ctypes.data
                                                for a in (params, mean, std)]))

    def get(self):
        import numpy as np
        params = np.empty(self.n_params, np.float32)
        mean = np.empty(self.n_features, np.float32)
        std = np.empty(self.n_features, np.float32)
        check(lib().fx_model_get(self.handle, params.ctypes.data, mean.ctypes.data,
                                 std.ctypes.data))
        return params, mean, std

    def train_step(self, X, labels, lr, loss=None, stream=None):
        return check(lib().fx_model_train_step(self.handle, _ptr(X), _ptr(labels), X.shape[0],
                                               float(lr), _ptr(loss), _stream(stream)))

    def train(self, X, labels, epochs, batch, lr, perm=None, losses=None, stream=None):
        """fx_model_train: `epochs` passes over the device rows X / labels in
        mini-batches, epoch e visiting rows perm[e] (host int32 array of
        shape [epochs, n]; None = natural order).  losses: device FP32
        [epochs] or None."""
        n = X.shape[0]
        p = None
        if perm is not None:
            import numpy as np
            perm = np.ascontiguousarray(perm, dtype=np.int32)
            if perm.shape != (epochs, n):
                raise ValueError("perm must have shape (epochs, n)")
            p = perm.ctypes.data_as(ctypes.c_void_p)
        return check(lib().fx_model_train(self.handle, _ptr(X), _ptr(labels), n, epochs, batch,
                                          lr, p, _ptr(losses) if losses is not None else None,
                                          _stream(stream)))

    def grad(self, X, labels, grad, loss=None, stream=None):
        return check(lib().fx_model_grad(self.handle, _ptr(X), _ptr(labels), X.shape[0],
                                         _ptr(grad), _ptr(loss), _stream(stream)))

    def forward(self, X, logits=None, choice=None, stream=None):
        return check(lib().fx_model_forward(self.handle, _ptr(X), X.shape[0], _ptr(logits),
                                            _ptr(choice), _stream(stream)))

    def choose(self, features):
        x = (ctypes.c_float * self.n_features)(*[float(v) for v in features])
        out = (ctypes.c_int32 * len(self.heads))()
        check(lib().fx_model_choose(self.handle, x, out))
        return list(out)

    def predict(self, features, kind, dt) -> tuple:
        """The launch configuration the model picks (fx_model_predict)."""
        x = (ctypes.c_float * self.n_features)(*[float(v) for v in features])
        out = Launch()
        check(lib().fx_model_predict(self.handle, x, kind, dt, ctypes.byref(out)))
        return out.as_tuple()

    def destroy(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fx_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.destroy()


def fx_model_create(n_features, hidden, heads) -> Model:
    return Model(n_features, hidden, heads)


def fx_model_load(path) -> Model:
    """A model from its FXM1 file (the C loader; the header read here only
    sizes the Python wrapper)."""
    import struct
    with open(path, "rb") as f:
        head = f.read(16)
        if len(head) < 16 or head[:4] != b"FXM1":
            raise FxError(1, "%s is not a model file (FXM1)" % path)
        F, H, nh = struct.unpack("<3i", head[4:16])
        heads = struct.unpack("<%di" % nh, f.read(4 * nh)) if 0 < nh <= 8 else ()
    m = Model.__new__(Model)
    m.n_features, m.hidden, m.heads = F, H, tuple(heads)
    m.handle = ctypes.c_void_p()
    check(lib().fx_model_load(str(path).encode(), ctypes.byref(m.handle)))
    return m


def fx_model_num_params(m: Model) -> int:
    return m.n_params


def fx_model_set(m: Model, params=None, mean=None, std=None):
    return m.set(params, mean, std)


def fx_model_get(m: Model):
    return m.get()


def fx_model_train_step(m: Model, X, labels, lr, loss=None, stream=None):
    return m.train_step(X, labels, lr, loss, stream)


def fx_model_grad(m: Model, X, labels, grad, loss=None, stream=None):
    return m.grad(X, labels, grad, loss, stream)


def fx_model_forward(m: Model, X, logits=None, choice=None, stream=None):
    return m.forward(X, logits, choice, stream)


def fx_model_choose(m: Model, features):
    return m.choose(features)


def fx_model_destroy(m: Model):
    m.destroy()


# ---- measurement kernels ------------------------------------------------------------


def fx_bw_copy(src, dst, nbytes, cfg=None, stream=None):
    return check(lib().fx_bw_copy(_ptr(src), _ptr(dst), nbytes, _cfg(cfg), _stream(stream)))


def fx_bw_read(src, nbytes, sink, cfg=None, stream=None):
    return check(lib().fx_bw_read(_ptr(src), nbytes, _ptr(sink), _cfg(cfg), _stream(stream)))


def fx_bw_write(dst, nbytes, value=0, cfg=None, stream=None):
    return check(lib().fx_bw_write(_ptr(dst), nbytes, value, _cfg(cfg), _stream(stream)))


def fx_bw_triad(a, b, c, dst, nbytes, streaming_stores=False, cfg=None, stream=None):
    return check(lib().fx_bw_triad(_ptr(a), _ptr(b), _ptr(c), _ptr(dst), nbytes,
                                   1 if streaming_stores else 0, _cfg(cfg), _stream(stream)))
