"""Seeded synthetic inputs (SplitMix64, counter-based), shared by the HIP
path's tests and benchmark and by the CPU oracle.

Nothing here computes any part of an expression: it draws numbers, rounds
them to a storage dtype, and (in ``trees``) draws random expression trees.
The draws are made by ``synth.c``; see its header for the exact definition.

Storage dtypes are returned as numpy arrays: f32 -> float32, f64 -> float64,
f16 -> float16, u32 -> uint32, bf16 -> uint16 holding the bf16 bit pattern.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")

DTYPES = {"f32": 0, "f64": 1, "bf16": 2, "f16": 3, "u32": 4}
NP_STORAGE = {"f32": np.float32, "f64": np.float64, "bf16": np.uint16,
              "f16": np.float16, "u32": np.uint32}
DISTS = {"uniform": 0, "lognormal": 1, "uint31": 2, "ones": 3, "uniform12": 4}

# Per-workload seeds and tensor ids (X=0, Y=1, W=2, further inputs 3, 4, ...).
SEED = {"small": 1, "matrix": 2, "precision": 3, "batch": 4,
        "tune_train": 5, "tune_heldout": 6, "mathsweep": 7}
TENSOR = {"X": 0, "Y": 1, "W": 2}


def build(force: bool = False) -> str:
    """Compile libsynth.so with gcc (OpenMP)."""
    src = os.path.join(_HERE, "synth.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        L.synth_fill.restype = ctypes.c_int64
        L.synth_fill.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                                 ctypes.c_int64, ctypes.c_void_p]
        L.synth_fill_f64.restype = ctypes.c_int
        L.synth_fill_f64.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_void_p]
        L.synth_raw.restype = None
        L.synth_raw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                ctypes.c_int64, ctypes.c_void_p]
        L.synth_draw.restype = ctypes.c_uint64
        L.synth_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        _lib = L
    return _lib


def fill(seed: int, tensor: int, n: int, dtype: str = "f32", dist: str = "uniform",
         param: float = 0.0, start: int = 0, out: np.ndarray | None = None,
         return_saturations: bool = False):
    """Elements [start, start+n) of tensor `tensor` under seed `seed`.

    dist: "uniform" (U[-1,1]), "uniform12" (U[1,2)), "lognormal" (magnitude
    exp(param*N(0,1)), random sign; param is sigma), "uint31" (u32 in
    [0,2^31)), "ones" (every element equals param).  FP16 values beyond 65504 saturate."""
    if dist == "lognormal" and param == 0.0:
        param = 3.0
    if out is None:
        out = np.empty(n, dtype=NP_STORAGE[dtype])
    assert out.dtype == NP_STORAGE[dtype] and out.size >= n and out.flags.c_contiguous
    sat = lib().synth_fill(seed, tensor, DISTS[dist], float(param), DTYPES[dtype],
                           start, n, out.ctypes.data)
    if sat < 0:
        raise ValueError("unsupported dtype/dist combination %s/%s" % (dtype, dist))
    return (out, int(sat)) if return_saturations else out


def fill_f64(seed: int, tensor: int, n: int, dist: str = "uniform", param: float = 0.0,
             start: int = 0) -> np.ndarray:
    """The exact FP64 draws before rounding to a storage dtype."""
    if dist == "lognormal" and param == 0.0:
        param = 3.0
    out = np.empty(n, dtype=np.float64)
    lib().synth_fill_f64(seed, tensor, DISTS[dist], float(param), start, n, out.ctypes.data)
    return out


def raw(seed: int, tensor: int, n: int, start: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    lib().synth_raw(seed, tensor, start, n, out.ctypes.data)
    return out


def bf16_to_f64(bits: np.ndarray) -> np.ndarray:
    """Widen bf16 bit patterns (uint16) exactly."""
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)

