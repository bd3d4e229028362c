"""CPU oracle for rectangular binary morphology (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The product library never does, and the two share no code:
the oracle is the plain definition of each operation (brute-force window
min/max on an unpacked byte image, per the paper's section "2D Morphological
Operators for Rectangular Masks", which names the brute-force strategy as the
one for reference and verification), plus an independent summed-area-table
evaluator, packing and run-length coding.  See ``morph_oracle.c`` for the
conventions (origin, borders, bit order, half-open runs).

Structuring elements are passed as ``(w, h, cx, cy)``: a w-wide, h-tall
rectangle whose origin is column cx, row cy of the rectangle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "morph_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        for name in ("oracle_erode", "oracle_dilate"):
            getattr(lib, name).argtypes = [P, P, I, I, I, I, I, I]
        for name in ("oracle_open", "oracle_close"):
            getattr(lib, name).argtypes = [P, P, P, I, I, I, I, I, I]
        lib.oracle_sat_build.argtypes = [P, P, I, I]
        for name in ("oracle_sat_erode", "oracle_sat_dilate"):
            getattr(lib, name).argtypes = [P, P, I, I, I, I, I, I]
        lib.oracle_pack.argtypes = [P, P, I, I, I]
        lib.oracle_unpack.argtypes = [P, P, I, I, I]
        lib.oracle_rle_count.argtypes = [P, P, I, I]
        lib.oracle_rle_count.restype = ctypes.c_int64
        lib.oracle_rle_encode.argtypes = [P, P, P, I, I]
        lib.oracle_rle_decode.argtypes = [P, P, P, I, I]
        lib.oracle_threads.restype = I
        lib.oracle_set_threads.argtypes = [I]
        _lib = lib
    return _lib


def threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_load().oracle_threads())


def set_threads(n: int) -> None:
    """Threads for the OpenMP loops from now on (timing on one thread)."""
    _load().oracle_set_threads(int(n))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _img(img) -> np.ndarray:
    a = np.ascontiguousarray(img, dtype=np.uint8)
    if a.ndim != 2:
        raise ValueError("image must be 2-D (H, W)")
    return a


def _check_se(se):
    w, h, cx, cy = (int(v) for v in se)
    if w < 1 or h < 1 or not (0 <= cx < w) or not (0 <= cy < h):
        raise ValueError("bad structuring element %r" % (se,))
    return w, h, cx, cy


def centred(w: int, h: int):
    """The default origin: (floor(w/2), floor(h/2))."""
    return (w, h, w // 2, h // 2)


def reflect(se):
    """The reflected element B^ = (w, h, w-1-cx, h-1-cy)."""
    w, h, cx, cy = _check_se(se)
    return (w, h, w - 1 - cx, h - 1 - cy)


# ---------------------------------------------------------------- brute force
def erode(img, se) -> np.ndarray:
    a = _img(img)
    H, W = a.shape
    out = np.empty_like(a)
    _load().oracle_erode(_ptr(out), _ptr(a), W, H, *_check_se(se))
    return out


def dilate(img, se) -> np.ndarray:
    a = _img(img)
    H, W = a.shape
    out = np.empty_like(a)
    _load().oracle_dilate(_ptr(out), _ptr(a), W, H, *_check_se(se))
    return out


def open_(img, se) -> np.ndarray:
    a = _img(img)
    H, W = a.shape
    out = np.empty_like(a)
    tmp = np.empty_like(a)
    _load().oracle_open(_ptr(out), _ptr(a), _ptr(tmp), W, H, *_check_se(se))
    return out


def close_(img, se) -> np.ndarray:
    a = _img(img)
    H, W = a.shape
    out = np.empty_like(a)
    tmp = np.empty_like(a)
    _load().oracle_close(_ptr(out), _ptr(a), _ptr(tmp), W, H, *_check_se(se))
    return out


OPS = {"erode": erode, "dilate": dilate, "open": open_, "close": close_}


def apply(op: str, img, se) -> np.ndarray:
    """Brute-force result of ``op`` in {'erode','dilate','open','close'}."""
    return OPS[op](img, se)


# ------------------------------------------------------ summed-area evaluator
def _sat(a: np.ndarray) -> np.ndarray:
    H, W = a.shape
    S = np.empty((H + 1, W + 1), dtype=np.int64)
    _load().oracle_sat_build(_ptr(S), _ptr(a), W, H)
    return S


def sat_erode(img, se) -> np.ndarray:
    a = _img(img)
    H, W = a.shape
    S = _sat(a)
    out = np.empty_like(a)
    _load().oracle_sat_erode(_ptr(out), _ptr(S), W, H, *_check_se(se))
    return out


def sat_dilate(img, se) -> np.ndarray:
    a = _img(img)
    H, W = a.shape
    S = _sat(a)
    out = np.empty_like(a)
    _load().oracle_sat_dilate(_ptr(out), _ptr(S), W, H, *_check_se(se))
    return out


def sat_apply(op: str, img, se) -> np.ndarray:
    """Same results as :func:`apply`, by the summed-area table (O(W*H))."""
    if op == "erode":
        return sat_erode(img, se)
    if op == "dilate":
        return sat_dilate(img, se)
    if op == "open":
        return sat_dilate(sat_erode(img, se), se)
    if op == "close":
        return sat_erode(sat_dilate(img, se), se)
    raise ValueError(op)


# ------------------------------------------------------------------- packing
def pack(img, stride: int | None = None) -> np.ndarray:
    """(H, W) bytes -> (H, stride) uint64 words, LSB-first, pad bits 0."""
    a = _img(img)
    H, W = a.shape
    if stride is None:
        stride = (W + 63) // 64
    if stride < (W + 63) // 64:
        raise ValueError("stride too small")
    out = np.empty((H, stride), dtype=np.uint64)
    _load().oracle_pack(_ptr(out), _ptr(a), W, H, stride)
    return out


def unpack(words, W: int) -> np.ndarray:
    """(H, stride) uint64 words -> (H, W) bytes; pad bits are not read."""
    wd = np.ascontiguousarray(words, dtype=np.uint64)
    H, stride = wd.shape
    if stride < (W + 63) // 64:
        raise ValueError("stride too small")
    out = np.empty((H, W), dtype=np.uint8)
    _load().oracle_unpack(_ptr(out), _ptr(wd), W, H, stride)
    return out


# -------------------------------------------------------- run-length coding
def rle_encode(img):
    """Maximal half-open runs per row: (row_ptr int32[H+1], runs int32[n,2])."""
    a = _img(img)
    H, W = a.shape
    counts = np.empty(H, dtype=np.int32)
    total = int(_load().oracle_rle_count(_ptr(counts), _ptr(a), W, H))
    row_ptr = np.empty(H + 1, dtype=np.int32)
    runs = np.empty((max(total, 1), 2), dtype=np.int32)
    _load().oracle_rle_encode(_ptr(row_ptr), _ptr(runs), _ptr(a), W, H)
    return row_ptr, runs[:total].copy()


def rle_decode(row_ptr, runs, W: int, H: int) -> np.ndarray:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    rr = np.ascontiguousarray(runs, dtype=np.int32).reshape(-1, 2)
    if rp.shape != (H + 1,):
        raise ValueError("row_ptr must have H+1 entries")
    if rr.shape[0] < rp[-1]:
        raise ValueError("runs shorter than row_ptr[H]")
    if rr.shape[0] == 0:
        rr = np.zeros((1, 2), dtype=np.int32)
    out = np.empty((H, W), dtype=np.uint8)
    _load().oracle_rle_decode(_ptr(out), _ptr(rp), _ptr(rr), W, H)
    return out


def rle_apply(op: str, row_ptr, runs, W: int, H: int, se, method: str = "brute"):
    """Expected run-length result of ``op``: encode(op(decode(R)))."""
    img = rle_decode(row_ptr, runs, W, H)
    f = apply if method == "brute" else sat_apply
    return rle_encode(f(op, img, se))
