"""Binary and run-length morphology on MI355X (gfx950): Python binding.

Every function named ``morph_*`` here marshals its arguments and calls the
entry point of the same name in ``libmorph.so`` (declared, with its full
contract, in ``include/morph.h``).  PyTorch only supplies device memory and
streams; all work runs in the library's HIP kernels.  There is no other
implementation behind this module: if the library is missing, importing the
package fails.

Images:

* :class:`Bitmap` -- packed rows of 64-bit words (pixel x of a row is bit
  x & 63 of word x >> 6), held in an int64 torch tensor of shape
  ``(npages * height, stride_words)``.
* :class:`RLE` -- run-length rows in CSR form: ``row_ptr`` (int32,
  ``npages * height + 1``) and ``runs`` (int32, ``(capacity, 2)``) of
  half-open ``[start, end)`` intervals.

Structuring elements are ``(w, h, cx, cy)``: a w-wide, h-tall rectangle
whose origin is column cx, row cy of it (see :func:`se`).
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = [
    "Bitmap", "RLE", "MorphError", "se", "OPS",
    "morph_version", "morph_strerror", "morph_last_hip_error", "morph_copy_async",
    "morph_erode_rect_packed", "morph_dilate_rect_packed", "morph_open_rect_packed",
    "morph_close_rect_packed", "morph_erode_rect_rle", "morph_dilate_rect_rle",
    "morph_open_rect_rle", "morph_close_rect_rle", "morph_pack_to_rle", "morph_pack_to_rle_noalloc",
    "MORPH_NOALLOC_MAX_ROWS", "morph_rle_to_pack",
    "morph_workspace_bytes", "morph_rle_workspace_bytes", "morph_rle_workspace_bytes_compact",
    "morph_pack_to_rle_workspace_bytes",
    "morph_rle_max_runs", "morph_rle_validate", "BatchPlan", "RoutedBatch", "RleRoute", "morph_batch_workspace_bytes", "page_desc",
    "morph_batch_launch", "Trace",
    "morph_popcount_pages", "page_densities",
    "morph_transpose_packed", "morph_transpose_rle", "morph_transpose_rle_workspace_bytes",
    "morph_rect_rlet", "morph_rlet_workspace_bytes",
    "morph_rle_label", "morph_rle_label_workspace_bytes", "morph_rle_component_stats", "morph_component_t",
    "morph_rle_run_histograms", "morph_histogram_percentile", "morph_histogram_percentile_workspace_bytes",
    "morph_mask_t", "morph_mask_packed", "morph_mask_rle", "morph_mask_workspace_bytes",
    "morph_shift_rows_packed", "morph_shift_rows_rle", "morph_shift_rows_rle_workspace_bytes",
    "rect_packed", "rect_rle", "pack_to_rle", "rle_to_pack", "transpose_packed", "transpose_rle", "rect_rlet",
    "label_components", "component_stats", "run_histograms", "histogram_percentile", "layout_boxes",
    "Mask", "mask_packed", "mask_rle",
    "shift_rows", "skew_rows", "skew_cols", "rotate", "rotation_rationals", "line_op",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmorph.so")

OPS = ("erode", "dilate", "open", "close")
MORPH_ERODE, MORPH_DILATE, MORPH_OPEN, MORPH_CLOSE = range(4)
MORPH_PACKED, MORPH_RLE = 0, 1

ERRORS = {
    0: "MORPH_OK", -1: "MORPH_E_INVAL", -2: "MORPH_E_SHAPE", -3: "MORPH_E_ALIAS",
    -4: "MORPH_E_WORKSPACE", -5: "MORPH_E_NONCANONICAL", -6: "MORPH_E_CAPACITY",
    -7: "MORPH_E_HIP", -8: "MORPH_E_UNSUPPORTED",
}


class morph_bitmap_t(ctypes.Structure):
    _fields_ = [("words", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("stride_words", ctypes.c_int32), ("npages", ctypes.c_int32)]


class morph_rle_t(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("npages", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("runs", ctypes.c_void_p), ("capacity", ctypes.c_int64)]


class morph_se_t(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int32), ("h", ctypes.c_int32), ("cx", ctypes.c_int32), ("cy", ctypes.c_int32)]


class morph_component_t(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_int32), ("y0", ctypes.c_int32), ("x1", ctypes.c_int32), ("y1", ctypes.c_int32),
                ("area", ctypes.c_int64), ("sum_x", ctypes.c_int64), ("sum_y", ctypes.c_int64)]


class morph_mask_t(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_void_p), ("w", ctypes.c_int32), ("h", ctypes.c_int32), ("cx", ctypes.c_int32),
                ("cy", ctypes.c_int32)]


class morph_kernel_trace_t(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("bytes", ctypes.c_double)]


MORPH_K_COUNT = 20


class morph_page_desc_t(ctypes.Structure):
    _fields_ = [("dst", morph_bitmap_t), ("src", morph_bitmap_t), ("op", ctypes.c_int32),
                ("se", morph_se_t), ("tile_rows", ctypes.c_int32), ("strip_words", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("%s is not built (run __graft_entry__.build() or "
                          "python paper_0712_0121_amd/_build.py)" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    BM, RL, SE = ctypes.POINTER(morph_bitmap_t), ctypes.POINTER(morph_rle_t), morph_se_t
    sig = {
        "morph_version": (ctypes.c_char_p, []),
        "morph_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "morph_last_hip_error": (ctypes.c_char_p, []),
        "morph_copy_async": (ctypes.c_int, [P, P, SZ, P]),
        "morph_pack_to_rle": (ctypes.c_int, [RL, BM, P, SZ, P]),
        "morph_pack_to_rle_noalloc": (ctypes.c_int, [RL, BM, P]),
        "morph_rle_to_pack": (ctypes.c_int, [BM, RL, P]),
        "morph_workspace_bytes": (SZ, [ctypes.c_int, ctypes.c_int, I32, I32, SE]),
        "morph_rle_workspace_bytes": (SZ, [ctypes.c_int, I32, I32, I32, SE]),
        "morph_rle_workspace_bytes_compact": (SZ, [ctypes.c_int, I32, I32, I32, SE]),
        "morph_pack_to_rle_workspace_bytes": (SZ, [I32, I32]),
        "morph_rle_max_runs": (I64, [I32, I32]),
        "morph_rle_validate": (ctypes.c_int, [RL, P]),
        "morph_batch_plan_create": (ctypes.c_int, [ctypes.POINTER(P), ctypes.POINTER(morph_page_desc_t), I32, P]),
        "morph_batch_run": (ctypes.c_int, [P, I32, P]),
        "morph_batch_tiles": (I64, [P]),
        "morph_batch_plan_destroy": (None, [P]),
        "morph_batch_workspace_bytes": (I64, [ctypes.POINTER(morph_page_desc_t), I32]),
        "morph_batch_launch": (ctypes.c_int, [ctypes.POINTER(morph_page_desc_t), I32, P, SZ, P, SZ, P]),
        "morph_trace_begin": (ctypes.c_int, [P, SZ, P]),
        "morph_trace_end": (ctypes.c_int, [ctypes.POINTER(morph_kernel_trace_t), P]),
        "morph_kernel_name": (ctypes.c_char_p, [ctypes.c_int]),
        "morph_transpose_packed": (ctypes.c_int, [BM, BM, P]),
        "morph_popcount_pages": (ctypes.c_int, [BM, P, P]),
        "morph_transpose_rle": (ctypes.c_int, [RL, RL, P, SZ, P]),
        "morph_transpose_rle_workspace_bytes": (SZ, [I32, I32, I32]),
        "morph_rect_rlet": (ctypes.c_int, [ctypes.c_int, RL, RL, SE, P, SZ, P]),
        "morph_rlet_workspace_bytes": (SZ, [ctypes.c_int, I32, I32, I32, SE]),
        "morph_rle_label": (ctypes.c_int, [RL, I32, P, I64, P, P, SZ, P]),
        "morph_rle_label_workspace_bytes": (SZ, [I32, I64]),
        "morph_rle_component_stats": (ctypes.c_int, [RL, P, I64, P, P, I64, P]),
        "morph_rle_run_histograms": (ctypes.c_int, [RL, P, P, P]),
        "morph_histogram_percentile": (ctypes.c_int, [P, I32, I32, I32, I32, P, P, SZ, P]),
        "morph_histogram_percentile_workspace_bytes": (SZ, [I32]),
        "morph_mask_packed": (ctypes.c_int, [ctypes.c_int, BM, BM, ctypes.POINTER(morph_mask_t), P, SZ, P]),
        "morph_mask_rle": (ctypes.c_int, [ctypes.c_int, RL, RL, ctypes.POINTER(morph_mask_t), P, SZ, P]),
        "morph_mask_workspace_bytes": (SZ, [ctypes.c_int, ctypes.c_int, I32, I32, I32,
                                            ctypes.POINTER(morph_mask_t)]),
        "morph_shift_rows_packed": (ctypes.c_int, [BM, BM, P, I32, P]),
        "morph_shift_rows_rle": (ctypes.c_int, [RL, RL, P, I32, P, SZ, P]),
        "morph_shift_rows_rle_workspace_bytes": (SZ, [I32]),
        "morph_skew_spread": (I64, [I32, I32, I32, I32]),
        "morph_skew_workspace_bytes": (SZ, [ctypes.c_int, ctypes.c_int, I32, I32, I32, I32, I32, I32]),
        "morph_skew_packed": (ctypes.c_int, [ctypes.c_int, BM, BM, I32, I32, I32, I32, P, SZ, P]),
        "morph_skew_rle": (ctypes.c_int, [ctypes.c_int, RL, RL, I32, I32, I32, I32, P, SZ, P]),
        "morph_rotation_rationals": (ctypes.c_int, [ctypes.c_double, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "morph_rotate_dims": (ctypes.c_int, [I32, I32, ctypes.c_double, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "morph_rotate_workspace_bytes": (SZ, [ctypes.c_int, I32, I32, I32, ctypes.c_double]),
        "morph_rotate_packed": (ctypes.c_int, [BM, BM, ctypes.c_double, P, SZ, P]),
        "morph_rotate_rle": (ctypes.c_int, [RL, RL, ctypes.c_double, P, SZ, P]),
        "morph_line_op_workspace_bytes": (SZ, [ctypes.c_int, ctypes.c_int, I32, I32, I32, I32, I32, I32]),
        "morph_line_op_packed": (ctypes.c_int, [ctypes.c_int, BM, BM, I32, I32, I32, P, SZ, P]),
        "morph_line_op_rle": (ctypes.c_int, [ctypes.c_int, RL, RL, I32, I32, I32, P, SZ, P]),
        "morph_layout_rle_workspace_bytes": (SZ, [I32, I32, I32, I64]),
        "morph_layout_rle": (ctypes.c_int, [RL, I32, I32, I32, RL, P, I64, P, P, I64, ctypes.POINTER(I32), P, SZ,
                                             P]),
    }
    for op in OPS:
        sig["morph_%s_rect_packed" % op] = (ctypes.c_int, [BM, BM, SE, P, SZ, P])
        sig["morph_%s_rect_rle" % op] = (ctypes.c_int, [RL, RL, SE, P, SZ, P])
    for name, (res, args) in sig.items():
        f = getattr(lib, name)          # AttributeError here = symbol missing
        f.restype = res
        f.argtypes = args
    return lib, sorted(sig)


_lib, SYMBOLS = _load()


class MorphError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = "%s: %s (%s)" % (where, _lib.morph_strerror(code).decode(), ERRORS.get(code, code))
        if code == -7:
            msg += ": " + _lib.morph_last_hip_error().decode()
        super().__init__(msg)
        self.code = code


def _check(code: int, where: str):
    if code != 0:
        raise MorphError(code, where)


def se(w: int, h: int, cx: int | None = None, cy: int | None = None):
    """A w x h rectangle; the origin defaults to (w // 2, h // 2)."""
    return (int(w), int(h), int(w) // 2 if cx is None else int(cx), int(h) // 2 if cy is None else int(cy))


def _se(s) -> morph_se_t:
    if isinstance(s, morph_se_t):
        return s
    w, h, cx, cy = s
    return morph_se_t(int(w), int(h), int(cx), int(cy))


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ws(ws):
    if ws is None:
        return None, 0
    return ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size()


class Bitmap:
    """Packed image(s) in device memory: words is an int64 tensor of shape
    (npages*height, stride_words); npages equal-size pages are stacked."""

    def __init__(self, words: torch.Tensor, width: int, height: int, npages: int = 1):
        if words.dtype != torch.int64 or words.dim() != 2 or not words.is_contiguous():
            raise ValueError("words must be a contiguous 2-D int64 tensor")
        if words.shape[0] != height * npages:
            raise ValueError("words must have npages*height rows")
        self.words, self.width, self.height, self.npages = words, int(width), int(height), int(npages)

    @property
    def stride(self) -> int:
        return self.words.shape[1]

    @classmethod
    def empty(cls, width, height, npages=1, stride=None, device="cuda"):
        stride = (width + 63) // 64 if stride is None else stride
        return cls(torch.empty((height * npages, stride), dtype=torch.int64, device=device),
                   width, height, npages)

    @classmethod
    def from_words(cls, words_np, width, npages=1, device="cuda"):
        """From a host (rows, stride) uint64 array."""
        import numpy as np
        w = torch.from_numpy(np.ascontiguousarray(words_np).view(np.int64)).to(device)
        return cls(w, width, w.shape[0] // npages, npages)

    def to_numpy(self):
        """Host copy as (rows, stride) uint64."""
        import numpy as np
        return self.words.cpu().numpy().view(np.uint64)

    def struct(self) -> morph_bitmap_t:
        return morph_bitmap_t(self.words.data_ptr(), self.width, self.height, self.stride, self.npages)


class RLE:
    """Run-length image(s) in device memory (CSR over rows)."""

    def __init__(self, row_ptr: torch.Tensor, runs: torch.Tensor, width: int, height: int, npages: int = 1):
        if row_ptr.dtype != torch.int32 or runs.dtype != torch.int32:
            raise ValueError("row_ptr and runs must be int32")
        if row_ptr.numel() != height * npages + 1:
            raise ValueError("row_ptr must have npages*height+1 entries")
        if runs.dim() != 2 or runs.shape[1] != 2 or not runs.is_contiguous():
            raise ValueError("runs must be a contiguous (capacity, 2) tensor")
        self.row_ptr, self.runs = row_ptr, runs
        self.width, self.height, self.npages = int(width), int(height), int(npages)

    @property
    def capacity(self) -> int:
        return self.runs.shape[0]

    @classmethod
    def empty(cls, width, height, npages=1, capacity=None, device="cuda"):
        if capacity is None:
            capacity = morph_rle_max_runs(width, height * npages)
        return cls(torch.empty(height * npages + 1, dtype=torch.int32, device=device),
                   torch.empty((max(int(capacity), 1), 2), dtype=torch.int32, device=device),
                   width, height, npages)

    @classmethod
    def from_host(cls, row_ptr, runs, width, height, npages=1, capacity=None, device="cuda"):
        import numpy as np
        rp = torch.from_numpy(np.ascontiguousarray(row_ptr, dtype=np.int32)).to(device)
        rr = np.ascontiguousarray(runs, dtype=np.int32).reshape(-1, 2)
        cap = max(rr.shape[0], 1) if capacity is None else int(capacity)
        t = torch.zeros((cap, 2), dtype=torch.int32, device=device)
        if rr.shape[0]:
            t[: rr.shape[0]] = torch.from_numpy(rr).to(device)
        return cls(rp, t, width, height, npages)

    def nruns(self) -> int:
        return int(self.row_ptr[-1].item())

    def to_host(self):
        """(row_ptr, runs[:n]) as numpy int32 arrays."""
        rp = self.row_ptr.cpu().numpy()
        n = int(rp[-1])
        return rp, self.runs[:n].cpu().numpy()

    def struct(self) -> morph_rle_t:
        return morph_rle_t(self.width, self.height, self.npages, self.row_ptr.data_ptr(),
                           self.runs.data_ptr(), self.capacity)


# ---------------------------------------------------------------- entry points
def morph_version() -> str:
    return _lib.morph_version().decode()


def morph_strerror(code: int) -> str:
    return _lib.morph_strerror(code).decode()


def morph_last_hip_error() -> str:
    return _lib.morph_last_hip_error().decode()


def _packed_entry(op):
    name = "morph_%s_rect_packed" % op
    f = getattr(_lib, name)

    def call(dst: Bitmap, src: Bitmap, s, ws=None, stream=None):
        d, r = dst.struct(), src.struct()
        p, n = _ws(ws)
        _check(f(ctypes.byref(d), ctypes.byref(r), _se(s), p, n, _stream(stream)), name)
    call.__name__ = name
    call.__doc__ = "Calls %s (include/morph.h)." % name
    return call


def _rle_entry(op):
    name = "morph_%s_rect_rle" % op
    f = getattr(_lib, name)

    def call(dst: RLE, src: RLE, s, ws=None, stream=None):
        d, r = dst.struct(), src.struct()
        p, n = _ws(ws)
        _check(f(ctypes.byref(d), ctypes.byref(r), _se(s), p, n, _stream(stream)), name)
    call.__name__ = name
    call.__doc__ = "Calls %s (include/morph.h)." % name
    return call


morph_erode_rect_packed = _packed_entry("erode")
morph_dilate_rect_packed = _packed_entry("dilate")
morph_open_rect_packed = _packed_entry("open")
morph_close_rect_packed = _packed_entry("close")
morph_erode_rect_rle = _rle_entry("erode")
morph_dilate_rect_rle = _rle_entry("dilate")
morph_open_rect_rle = _rle_entry("open")
morph_close_rect_rle = _rle_entry("close")
PACKED = {op: globals()["morph_%s_rect_packed" % op] for op in OPS}
RLE_OPS = {op: globals()["morph_%s_rect_rle" % op] for op in OPS}


def morph_pack_to_rle(dst: RLE, src: Bitmap, ws=None, stream=None):
    d, r = dst.struct(), src.struct()
    p, n = _ws(ws)
    _check(_lib.morph_pack_to_rle(ctypes.byref(d), ctypes.byref(r), p, n, _stream(stream)),
           "morph_pack_to_rle")


MORPH_NOALLOC_MAX_ROWS = 4000000     # rows per call of morph_pack_to_rle_noalloc (include/morph.h)


def morph_pack_to_rle_noalloc(dst: RLE, src: Bitmap, stream=None):
    """morph_pack_to_rle with the library's fixed device scratch instead of a
    workspace (nothing allocated); calls that overlap on one GPU race."""
    d, r = dst.struct(), src.struct()
    _check(_lib.morph_pack_to_rle_noalloc(ctypes.byref(d), ctypes.byref(r), _stream(stream)),
           "morph_pack_to_rle_noalloc")


def morph_copy_async(dst_ptr: int, src_ptr: int, nbytes: int, stream=None):
    """Asynchronous copy of nbytes between device or pinned host addresses
    (integers, e.g. tensor.data_ptr()) on `stream`."""
    _check(_lib.morph_copy_async(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr), nbytes, _stream(stream)),
           "morph_copy_async")


def morph_rle_to_pack(dst: Bitmap, src: RLE, stream=None):
    d, r = dst.struct(), src.struct()
    _check(_lib.morph_rle_to_pack(ctypes.byref(d), ctypes.byref(r), _stream(stream)), "morph_rle_to_pack")


def morph_workspace_bytes(op, repr_, width, height, s) -> int:
    op = OPS.index(op) if isinstance(op, str) else int(op)
    return int(_lib.morph_workspace_bytes(op, int(repr_), int(width), int(height), _se(s)))


def morph_rle_workspace_bytes(op, width, height, npages, s) -> int:
    op = OPS.index(op) if isinstance(op, str) else int(op)
    return int(_lib.morph_rle_workspace_bytes(op, int(width), int(height), int(npages), _se(s)))


def morph_pack_to_rle_workspace_bytes(width, height) -> int:
    return int(_lib.morph_pack_to_rle_workspace_bytes(int(width), int(height)))


def morph_rle_max_runs(width, height) -> int:
    return int(_lib.morph_rle_max_runs(int(width), int(height)))


def morph_rle_validate(r: RLE, stream=None) -> int:
    s = r.struct()
    return int(_lib.morph_rle_validate(ctypes.byref(s), _stream(stream)))


def morph_transpose_packed(dst: Bitmap, src: Bitmap, stream=None):
    d, r = dst.struct(), src.struct()
    _check(_lib.morph_transpose_packed(ctypes.byref(d), ctypes.byref(r), _stream(stream)),
           "morph_transpose_packed")


def morph_popcount_pages(src: Bitmap, counts: torch.Tensor, stream=None):
    """counts (device int64, npages entries) = black pixels of every page."""
    r = src.struct()
    _check(_lib.morph_popcount_pages(ctypes.byref(r), ctypes.c_void_p(counts.data_ptr()), _stream(stream)),
           "morph_popcount_pages")


def page_densities(bitmaps, stream=None):
    """Black fraction of every page of the given bitmaps (in order, stacked
    pages each), counted on the device; one synchronisation to read them."""
    bitmaps = list(bitmaps)
    if not bitmaps:
        return []
    n = sum(b.npages for b in bitmaps)
    counts = torch.empty(n, dtype=torch.int64, device=bitmaps[0].words.device)
    k = 0
    for b in bitmaps:
        morph_popcount_pages(b, counts[k:k + b.npages], stream)
        k += b.npages
    c = counts.tolist()
    out, k = [], 0
    for b in bitmaps:
        for _ in range(b.npages):
            out.append(c[k] / float(b.width * b.height))
            k += 1
    return out


def morph_transpose_rle_workspace_bytes(width, height, npages=1) -> int:
    return int(_lib.morph_transpose_rle_workspace_bytes(int(width), int(height), int(npages)))


def morph_transpose_rle(dst: RLE, src: RLE, ws=None, stream=None):
    d, r = dst.struct(), src.struct()
    p, n = _ws(ws)
    _check(_lib.morph_transpose_rle(ctypes.byref(d), ctypes.byref(r), p, n, _stream(stream)),
           "morph_transpose_rle")


def morph_rlet_workspace_bytes(op, width, height, npages, s) -> int:
    op = OPS.index(op) if isinstance(op, str) else int(op)
    return int(_lib.morph_rlet_workspace_bytes(op, int(width), int(height), int(npages), _se(s)))


def morph_rect_rlet(op, dst: RLE, src: RLE, s, ws=None, stream=None):
    op = OPS.index(op) if isinstance(op, str) else int(op)
    d, r = dst.struct(), src.struct()
    p, n = _ws(ws)
    _check(_lib.morph_rect_rlet(op, ctypes.byref(d), ctypes.byref(r), _se(s), p, n, _stream(stream)),
           "morph_rect_rlet")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def morph_rle_label_workspace_bytes(rows, max_runs) -> int:
    return int(_lib.morph_rle_label_workspace_bytes(int(rows), int(max_runs)))


def morph_rle_label(src: RLE, connectivity, labels, max_runs, comp_ptr, ws=None, stream=None):
    r = src.struct()
    p, n = _ws(ws)
    _check(_lib.morph_rle_label(ctypes.byref(r), int(connectivity), _ptr(labels), int(max_runs), _ptr(comp_ptr),
                                p, n, _stream(stream)), "morph_rle_label")


def morph_rle_component_stats(src: RLE, labels, max_runs, comp_ptr, stats, max_components, stream=None):
    r = src.struct()
    _check(_lib.morph_rle_component_stats(ctypes.byref(r), _ptr(labels), int(max_runs), _ptr(comp_ptr),
                                          _ptr(stats), int(max_components), _stream(stream)),
           "morph_rle_component_stats")


def morph_rle_run_histograms(src: RLE, black, white, stream=None):
    r = src.struct()
    _check(_lib.morph_rle_run_histograms(ctypes.byref(r), _ptr(black), _ptr(white), _stream(stream)),
           "morph_rle_run_histograms")


def morph_histogram_percentile_workspace_bytes(nbins) -> int:
    return int(_lib.morph_histogram_percentile_workspace_bytes(int(nbins)))


def morph_histogram_percentile(hist, nrows, nbins, num, den, out, ws=None, stream=None):
    p, n = _ws(ws)
    _check(_lib.morph_histogram_percentile(_ptr(hist), int(nrows), int(nbins), int(num), int(den), _ptr(out),
                                           p, n, _stream(stream)), "morph_histogram_percentile")


class Mask:
    """An arbitrary structuring element: an (h, w) array of 0/1 (host) and its
    origin (cx, cy), column and row within the array."""

    def __init__(self, bits, cx: int, cy: int):
        import numpy as np
        self.bits = np.ascontiguousarray(bits, dtype=np.uint8)
        if self.bits.ndim != 2:
            raise ValueError("mask must be 2-D (h, w)")
        self.cx, self.cy = int(cx), int(cy)

    def struct(self) -> morph_mask_t:
        h, w = self.bits.shape
        return morph_mask_t(self.bits.ctypes.data, w, h, self.cx, self.cy)


def morph_mask_workspace_bytes(op, repr_, width, height, npages, mask: Mask) -> int:
    op = OPS.index(op) if isinstance(op, str) else int(op)
    m = mask.struct()
    return int(_lib.morph_mask_workspace_bytes(op, int(repr_), int(width), int(height), int(npages), ctypes.byref(m)))


def morph_mask_packed(op, dst: Bitmap, src: Bitmap, mask: Mask, ws=None, stream=None):
    op = OPS.index(op) if isinstance(op, str) else int(op)
    d, r, m = dst.struct(), src.struct(), mask.struct()
    p, n = _ws(ws)
    _check(_lib.morph_mask_packed(op, ctypes.byref(d), ctypes.byref(r), ctypes.byref(m), p, n, _stream(stream)),
           "morph_mask_packed")


def morph_mask_rle(op, dst: RLE, src: RLE, mask: Mask, ws=None, stream=None):
    op = OPS.index(op) if isinstance(op, str) else int(op)
    d, r, m = dst.struct(), src.struct(), mask.struct()
    p, n = _ws(ws)
    _check(_lib.morph_mask_rle(op, ctypes.byref(d), ctypes.byref(r), ctypes.byref(m), p, n, _stream(stream)),
           "morph_mask_rle")


def morph_shift_rows_packed(dst: Bitmap, src: Bitmap, shifts, fill: int, stream=None):
    d, r = dst.struct(), src.struct()
    _check(_lib.morph_shift_rows_packed(ctypes.byref(d), ctypes.byref(r), _ptr(shifts), int(fill), _stream(stream)),
           "morph_shift_rows_packed")


def morph_shift_rows_rle_workspace_bytes(rows) -> int:
    return int(_lib.morph_shift_rows_rle_workspace_bytes(int(rows)))


def morph_shift_rows_rle(dst: RLE, src: RLE, shifts, fill: int, ws=None, stream=None):
    d, r = dst.struct(), src.struct()
    p, n = _ws(ws)
    _check(_lib.morph_shift_rows_rle(ctypes.byref(d), ctypes.byref(r), _ptr(shifts), int(fill), p, n,
                                     _stream(stream)), "morph_shift_rows_rle")


class BatchPlan:
    """Many packed pages, each with its own operation and element, run as one
    persistent launch (morph_batch_plan_create / morph_batch_run)."""

    def __init__(self, items, stream=None):
        """items: iterable of (dst Bitmap, src Bitmap, op, se[, tile_rows, strip_words])."""
        items = list(items)
        arr = (morph_page_desc_t * max(1, len(items)))()
        self._keep = []
        for i, it in enumerate(items):
            dst, src, op, s = it[:4]
            tr, sw = (it[4], it[5]) if len(it) >= 6 else (0, 0)
            arr[i] = morph_page_desc_t(dst.struct(), src.struct(), OPS.index(op) if isinstance(op, str) else op,
                                       _se(s), int(tr), int(sw))
            self._keep.append((dst, src))
        h = ctypes.c_void_p()
        _check(_lib.morph_batch_plan_create(ctypes.byref(h), arr, len(items), _stream(stream)),
               "morph_batch_plan_create")
        self._h = h

    @property
    def tiles(self) -> int:
        return int(_lib.morph_batch_tiles(self._h))

    def run(self, use_graph: bool = True, stream=None):
        _check(_lib.morph_batch_run(self._h, 1 if use_graph else 0, _stream(stream)), "morph_batch_run")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.morph_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RleRoute:
    """Pages sent down the run-length path one at a time: bitmap -> runs ->
    operation -> bitmap (the paper's runtime choice counts the conversions
    as part of that path).  The run-length images and workspaces are shared
    by every page and grow to the largest page seen; the pages run one after
    another on a stream, so one set serves them all."""

    def __init__(self, device):
        self.device = torch.device(device)
        self.W = self.H = 0
        self.rp = self.runs = self.rp2 = self.runs2 = None
        self.ws_p2r = self.ws_op = None
        self.ws_op_bytes = 0

    def _fit(self, W, H, op, s, stream):
        cap = morph_rle_max_runs(W, H)
        with torch.cuda.stream(stream) if isinstance(stream, torch.cuda.Stream) else _nullctx():
            if self.rp is None or self.rp.numel() < H + 1 or self.runs.shape[0] < cap:
                rows = max(H, self.H) + 1
                n = max(cap, self.runs.shape[0] if self.runs is not None else 0)
                self.rp = torch.empty(rows, dtype=torch.int32, device=self.device)
                self.rp2 = torch.empty(rows, dtype=torch.int32, device=self.device)
                self.runs = torch.empty((n, 2), dtype=torch.int32, device=self.device)
                self.runs2 = torch.empty((n, 2), dtype=torch.int32, device=self.device)
                self.H = max(H, self.H)
            need = morph_pack_to_rle_workspace_bytes(W, H)
            if self.ws_p2r is None or self.ws_p2r.numel() < need:
                self.ws_p2r = torch.empty(need, dtype=torch.uint8, device=self.device)
            need = morph_rle_workspace_bytes(op, W, H, 1, s)
            if need > self.ws_op_bytes:
                self.ws_op = torch.empty(need, dtype=torch.uint8, device=self.device)
                self.ws_op_bytes = need

    def run(self, dst: Bitmap, src: Bitmap, op, s, stream=None):
        if src.npages != 1 or dst.npages != 1:
            raise ValueError("RleRoute runs single pages")
        W, H = src.width, src.height
        self._fit(W, H, op, s, stream)
        r_in = RLE(self.rp[:H + 1], self.runs, W, H)
        r_out = RLE(self.rp2[:H + 1], self.runs2, W, H)
        morph_pack_to_rle(r_in, src, self.ws_p2r, stream)
        RLE_OPS[op](r_out, r_in, s, self.ws_op, stream)
        morph_rle_to_pack(dst, r_out, stream)


class _nullctx:
    def __enter__(self):
        return self

    def __exit__(self, *exc):
        return False


class RoutedBatch:
    """A batch whose pages each go down the packed or the run-length path, as
    the tuner chooses from the page's black density, its operation and its
    element size (section "Experiments", subsection "2D Rectangular Masks":
    the representation is picked at run time, conversion costs included).
    The packed pages run as one persistent launch (BatchPlan); each
    run-length page as bitmap -> runs -> operation -> bitmap (RleRoute).

    items: (dst, src, op, se[, tile_rows, strip_words]) with single-page
    bitmaps.  routes: a list of 'packed' / 'rle' to force the choice;
    otherwise tuner.choose_repr(density, op, se) picks it (every page
    'packed' without a tuner), the densities counted on the device by
    morph_popcount_pages unless given."""

    def __init__(self, items, tuner=None, routes=None, densities=None, stream=None):
        items = list(items)
        if routes is None:
            if tuner is None:
                routes = ["packed"] * len(items)
            else:
                if densities is None:
                    densities = page_densities([it[1] for it in items], stream)
                routes = [tuner.choose_repr(d, it[2], tuple(it[3])) for d, it in zip(densities, items)]
        routes = list(routes)
        if len(routes) != len(items) or any(r not in ("packed", "rle") for r in routes):
            raise ValueError("one route, 'packed' or 'rle', per page")
        self.routes = routes
        self.densities = densities
        pk = [it for it, r in zip(items, routes) if r == "packed"]
        self.rle_items = [tuple(it[:4]) for it, r in zip(items, routes) if r == "rle"]
        self.plan = BatchPlan(pk, stream) if pk else None
        self.rle = RleRoute(self.rle_items[0][1].words.device) if self.rle_items else None

    @property
    def tiles(self) -> int:
        return self.plan.tiles if self.plan is not None else 0

    def route_counts(self):
        return {"packed": self.routes.count("packed"), "rle": self.routes.count("rle")}

    def run(self, use_graph: bool = True, stream=None):
        if self.plan is not None:
            self.plan.run(use_graph, stream)
        for dst, src, op, s in self.rle_items:
            self.rle.run(dst, src, op, s, stream)

    def close(self):
        if self.plan is not None:
            self.plan.close()


def _descs(items):
    items = list(items)
    arr = (morph_page_desc_t * max(1, len(items)))()
    for i, it in enumerate(items):
        dst, src, op, s = it[:4]
        tr, sw = (it[4], it[5]) if len(it) >= 6 else (0, 0)
        arr[i] = morph_page_desc_t(dst.struct(), src.struct(), OPS.index(op) if isinstance(op, str) else op,
                                   _se(s), int(tr), int(sw))
    return arr, len(items)


def morph_batch_workspace_bytes(items) -> int:
    """Bytes of device workspace (and pinned staging) morph_batch_launch
    needs for these (dst, src, op, se[, tile_rows, strip_words]) items; -1 if
    the batch kernel cannot take one of them."""
    arr, n = _descs(items)
    return int(_lib.morph_batch_workspace_bytes(arr, n))


def page_desc(dst: "Bitmap", src: "Bitmap", op, s, tile_rows=0, strip_words=0) -> morph_page_desc_t:
    """One batch descriptor, built once and reusable while dst and src live."""
    return morph_page_desc_t(dst.struct(), src.struct(), OPS.index(op) if isinstance(op, str) else op,
                             _se(s), int(tile_rows), int(strip_words))


def morph_batch_launch(items, ws, staging=None, stream=None):
    """One persistent launch over the items (see morph_batch_launch in
    include/morph.h); ws: device uint8 tensor; staging: pinned host uint8
    tensor or None.  items: (dst, src, op, se[, tile_rows, strip_words])
    tuples, or prebuilt page_desc() descriptors."""
    items = list(items)
    if items and isinstance(items[0], morph_page_desc_t):
        arr, n = (morph_page_desc_t * len(items))(*items), len(items)
    else:
        arr, n = _descs(items)
    p, nb = _ws(ws)
    if staging is not None:
        sp, sn = ctypes.c_void_p(staging.data_ptr()), staging.numel()
    else:
        sp, sn = None, 0
    _check(_lib.morph_batch_launch(arr, n, p, nb, sp, sn, _stream(stream)), "morph_batch_launch")


class Trace:
    """Context manager around morph_trace_begin / morph_trace_end: collects,
    per library kernel, launches, event-measured milliseconds and
    algorithmic bytes of everything queued on `stream` inside it."""

    def __init__(self, stream=None):
        self.stream = stream
        self.result = {}

    def __enter__(self):
        nbytes = MORPH_K_COUNT * 2 * 256 * 128
        self.buf = torch.empty(nbytes // 8 + 16, dtype=torch.int64, device="cuda")
        base = (self.buf.data_ptr() + 127) // 128 * 128
        _check(_lib.morph_trace_begin(ctypes.c_void_p(base), nbytes, _stream(self.stream)),
               "morph_trace_begin")
        return self

    def __exit__(self, *exc):
        arr = (morph_kernel_trace_t * MORPH_K_COUNT)()
        _check(_lib.morph_trace_end(arr, _stream(self.stream)), "morph_trace_end")
        self.result = {_lib.morph_kernel_name(k).decode(): {"launches": int(arr[k].launches), "ms": float(arr[k].ms),
                                                             "bytes": float(arr[k].bytes)}
                       for k in range(MORPH_K_COUNT) if arr[k].launches}
        return False


# ------------------------------------------------------------- conveniences
def _alloc_ws(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device) if nbytes else None


def rect_packed(op: str, src: Bitmap, s, dst: Bitmap | None = None, stream=None) -> Bitmap:
    """op in OPS on a packed image; allocates dst and workspace with torch."""
    if dst is None:
        dst = Bitmap.empty(src.width, src.height, src.npages, device=src.words.device)
    ws = _alloc_ws(morph_workspace_bytes(op, MORPH_PACKED, src.width, src.height * src.npages, s),
                   src.words.device)
    PACKED[op](dst, src, s, ws, stream)
    return dst


def morph_rle_workspace_bytes_compact(op, width, height, npages, s) -> int:
    op = OPS.index(op) if isinstance(op, str) else int(op)
    return int(_lib.morph_rle_workspace_bytes_compact(op, int(width), int(height), int(npages), _se(s)))


def rect_rle(op: str, src: RLE, s, dst: RLE | None = None, stream=None, compact: bool = False) -> RLE:
    """op in OPS on a run-length image; allocates dst and workspace with torch
    (compact: the band form's small workspace instead of the slot form's).
    Without dst the result array starts at twice the input's runs plus one
    per row (the input count is read back: a synchronisation) and, if the
    result has more runs than that, is sized from the reported total and the
    operation runs again."""
    size = morph_rle_workspace_bytes_compact if compact else morph_rle_workspace_bytes
    ws = _alloc_ws(size(op, src.width, src.height, src.npages, s), src.row_ptr.device)
    if dst is not None:
        RLE_OPS[op](dst, src, s, ws, stream)
        return dst
    rows = src.height * src.npages
    cap = min(2 * src.nruns() + rows + 16, morph_rle_max_runs(src.width, rows))
    dst = RLE.empty(src.width, src.height, src.npages, capacity=cap, device=src.row_ptr.device)
    RLE_OPS[op](dst, src, s, ws, stream)
    total = dst.nruns()
    if total > cap:
        dst = RLE.empty(src.width, src.height, src.npages, capacity=total, device=src.row_ptr.device)
        RLE_OPS[op](dst, src, s, ws, stream)
    return dst


def pack_to_rle(src: Bitmap, capacity=None, stream=None) -> RLE:
    dst = RLE.empty(src.width, src.height, src.npages, capacity=capacity, device=src.words.device)
    ws = _alloc_ws(morph_pack_to_rle_workspace_bytes(src.width, src.height * src.npages), src.words.device)
    morph_pack_to_rle(dst, src, ws, stream)
    return dst


def rle_to_pack(src: RLE, stride=None, stream=None) -> Bitmap:
    dst = Bitmap.empty(src.width, src.height, src.npages, stride=stride, device=src.row_ptr.device)
    morph_rle_to_pack(dst, src, stream)
    return dst


def transpose_packed(src: Bitmap, stream=None) -> Bitmap:
    dst = Bitmap.empty(src.height, src.width, src.npages, device=src.words.device)
    morph_transpose_packed(dst, src, stream)
    return dst


def transpose_rle(src: RLE, stream=None) -> RLE:
    dst = RLE.empty(src.height, src.width, src.npages, device=src.row_ptr.device)
    ws = _alloc_ws(morph_transpose_rle_workspace_bytes(src.width, src.height, src.npages), src.row_ptr.device)
    morph_transpose_rle(dst, src, ws, stream)
    return dst


def rect_rlet(op: str, src: RLE, s, dst: RLE | None = None, stream=None) -> RLE:
    """op in OPS on a run-length image by within-line operations and
    transposition; same result as rect_rle."""
    if dst is None:
        dst = RLE.empty(src.width, src.height, src.npages, device=src.row_ptr.device)
    ws = _alloc_ws(morph_rlet_workspace_bytes(op, src.width, src.height, src.npages, s), src.row_ptr.device)
    morph_rect_rlet(op, dst, src, s, ws, stream)
    return dst


def label_components(src: RLE, connectivity: int = 8, stream=None):
    """Component number of every run (int32, one per run, numbered per page)
    and comp_ptr (int32, npages + 1).  Reads the run count first (a
    synchronisation) to size the label array."""
    dev = src.row_ptr.device
    n = src.nruns()
    labels = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    comp_ptr = torch.empty(src.npages + 1, dtype=torch.int32, device=dev)
    ws = _alloc_ws(morph_rle_label_workspace_bytes(src.height * src.npages, n), dev)
    morph_rle_label(src, connectivity, labels, n, comp_ptr, ws, stream)
    return labels[:n], comp_ptr


def component_stats(src: RLE, labels, comp_ptr, stream=None):
    """Per component over all pages: (boxes int32 (n, 4) as x0, y0, x1, y1;
    sums int64 (n, 3) as area, sum_x, sum_y).  Reads the component count
    first (a synchronisation)."""
    total = int(comp_ptr[-1].item())
    if total < 0:
        raise MorphError(-6, "component_stats: labelling ran out of room")
    raw = torch.empty((max(total, 1), 10), dtype=torch.int32, device=labels.device)
    morph_rle_component_stats(src, labels, labels.numel(), comp_ptr, raw, total, stream)
    return raw[:total, :4], raw[:total, 4:].contiguous().view(torch.int64)


def run_histograms(src: RLE, stream=None):
    """(black, white) int32 histograms, shape (npages, width + 1)."""
    dev = src.row_ptr.device
    black = torch.empty((src.npages, src.width + 1), dtype=torch.int32, device=dev)
    white = torch.empty_like(black)
    morph_rle_run_histograms(src, black, white, stream)
    return black, white


def histogram_percentile(hist, num: int, den: int, stream=None):
    """Device int32 tensor [1]: the percentile num/den of the summed rows of hist."""
    out = torch.empty(1, dtype=torch.int32, device=hist.device)
    ws = _alloc_ws(morph_histogram_percentile_workspace_bytes(hist.shape[1]), hist.device)
    morph_histogram_percentile(hist, hist.shape[0], hist.shape[1], num, den, out, ws, stream)
    return out


def layout_boxes(src: RLE, num: int = 1, den: int = 3, connectivity: int = 8, stream=None):
    """Layout analysis on runs (morph_layout_rle): gx, gy = percentile num/den
    of the horizontal and vertical white runs between black ones over the
    whole stack; the pages dilated by the centred (gx + 1) x (gy + 1)
    rectangle; the connected components of the result and their boxes.
    Returns (gx, gy, boxes, sums, comp_ptr).  The library waits for the
    stream once, to read the spacings; the label array starts at twice the
    input's runs plus one per row and is enlarged once if the smeared image
    has more runs."""
    dev = src.row_ptr.device
    smeared = RLE.empty(src.width, src.height, src.npages, device=dev)
    comp_ptr = torch.empty(src.npages + 1, dtype=torch.int32, device=dev)
    spacing = (ctypes.c_int32 * 2)()
    max_runs = min(2 * src.nruns() + src.height * src.npages, 2 ** 31 - 2)
    for attempt in range(2):
        labels = torch.empty(max(max_runs, 1), dtype=torch.int32, device=dev)
        stats = torch.empty((max(max_runs, 1), 10), dtype=torch.int32, device=dev)
        ws = _alloc_ws(_lib.morph_layout_rle_workspace_bytes(src.width, src.height, src.npages, max_runs), dev)
        p, nb = _ws(ws)
        _check(_lib.morph_layout_rle(ctypes.byref(src.struct()), num, den, connectivity, ctypes.byref(smeared.struct()),
                                     ctypes.c_void_p(labels.data_ptr()), max_runs,
                                     ctypes.c_void_p(comp_ptr.data_ptr()), ctypes.c_void_p(stats.data_ptr()),
                                     max_runs, spacing, p, nb, _stream(stream)), "morph_layout_rle")
        total = int(comp_ptr[-1].item())
        if total >= 0:
            break
        max_runs = smeared.nruns()              # the labels ran out of room: once more, sized exactly
    if total < 0:
        raise MorphError(-6, "layout_boxes: labelling ran out of room")
    raw = stats[:total]
    return spacing[0], spacing[1], raw[:, :4], raw[:, 4:].contiguous().view(torch.int64), comp_ptr


def mask_packed(op: str, src: Bitmap, mask: Mask, dst: Bitmap | None = None, stream=None) -> Bitmap:
    if dst is None:
        dst = Bitmap.empty(src.width, src.height, src.npages, device=src.words.device)
    ws = _alloc_ws(morph_mask_workspace_bytes(op, MORPH_PACKED, src.width, src.height, src.npages, mask),
                   src.words.device)
    morph_mask_packed(op, dst, src, mask, ws, stream)
    return dst


def mask_rle(op: str, src: RLE, mask: Mask, dst: RLE | None = None, stream=None) -> RLE:
    if dst is None:
        dst = RLE.empty(src.width, src.height, src.npages, device=src.row_ptr.device)
    ws = _alloc_ws(morph_mask_workspace_bytes(op, MORPH_RLE, src.width, src.height, src.npages, mask),
                   src.row_ptr.device)
    morph_mask_rle(op, dst, src, mask, ws, stream)
    return dst


# ------------------------------------------------- skews, rotation, lines
# The image work of these compositions runs in the library (line shifts,
# transposes, rectangle operations); the host only computes the integer
# shift of each line, as it computes an element or a launch.
def shift_rows(src, shifts, width: int, fill: int = 0, stream=None):
    """Every line moves right by its shift (device int32, one per line of all
    pages): dst(x, y) = src(x - shift, y) inside the source, fill elsewhere."""
    if isinstance(src, Bitmap):
        dst = Bitmap.empty(width, src.height, src.npages, device=src.words.device)
        morph_shift_rows_packed(dst, src, shifts, fill, stream)
        return dst
    dst = RLE.empty(width, src.height, src.npages, device=src.row_ptr.device)
    ws = _alloc_ws(morph_shift_rows_rle_workspace_bytes(src.height * src.npages), src.row_ptr.device)
    morph_shift_rows_rle(dst, src, shifts, fill, ws, stream)
    return dst


def _dev(img):
    return img.words.device if isinstance(img, Bitmap) else img.row_ptr.device


def _transpose(img, stream=None):
    return transpose_packed(img, stream) if isinstance(img, Bitmap) else transpose_rle(img, stream)


def _empty_like_repr(img, width, height):
    if isinstance(img, Bitmap):
        return Bitmap.empty(width, height, img.npages, device=img.words.device)
    return RLE.empty(width, height, img.npages, device=img.row_ptr.device)


def _skew(axis, src, num, den, origin, fill, stream):
    if den <= 0:
        raise ValueError("den must be positive")
    repr_ = MORPH_PACKED if isinstance(src, Bitmap) else MORPH_RLE
    lines = src.height if axis == 0 else src.width
    spread = int(_lib.morph_skew_spread(lines, num, den, origin))
    W, H = (src.width + spread, src.height) if axis == 0 else (src.width, src.height + spread)
    dst = _empty_like_repr(src, W, H)
    n = _lib.morph_skew_workspace_bytes(repr_, axis, src.width, src.height, src.npages, num, den, origin)
    if n == 0:
        raise MorphError(-8, "morph_skew: sizes out of range")
    ws = torch.empty(n, dtype=torch.uint8, device=_dev(src))
    p, nb = _ws(ws)
    f = _lib.morph_skew_packed if repr_ == MORPH_PACKED else _lib.morph_skew_rle
    _check(f(axis, ctypes.byref(dst.struct()), ctypes.byref(src.struct()), num, den, origin, fill, p, nb,
             _stream(stream)), "morph_skew")
    # along the lines the workspace starts with the library's shift table:
    # the shifts of the lines of the first page
    v = ws[: 4 * lines].view(torch.int32).cpu().numpy().astype("int64") if axis == 0 else None
    return dst, v


def skew_rows(src, num: int, den: int, origin: int, fill: int = 0, stream=None):
    """Lossless skew along the lines (morph_skew_packed / morph_skew_rle, axis
    0): line y moves by floor(num (y - origin) / den), less the smallest such
    shift; the frame widens by their spread.  Returns (image, the shifts of
    the lines of one page, read back from the library's table)."""
    return _skew(0, src, num, den, origin, fill, stream)


def skew_cols(src, num: int, den: int, origin: int, fill: int = 0, stream=None):
    """Lossless skew across the lines (axis 1: column x moves down by
    floor(num (x - origin) / den) less the smallest).  Returns (image, None)."""
    return _skew(1, src, num, den, origin, fill, stream)


def rotation_rationals(angle: float, den: int = 1 << 16):
    """(tan_num, sin_num, den): tan(angle / 2) and sin(angle) as the nearest
    rationals over den (morph_rotation_rationals)."""
    t, sn = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.morph_rotation_rationals(float(angle), int(den), ctypes.byref(t), ctypes.byref(sn)),
           "morph_rotation_rationals")
    return t.value, sn.value, den


def rotate(src, angle: float, stream=None):
    """Rotation by angle radians (|angle| <= pi/2) as three lossless skews
    about the frame centre (morph_rotate_packed / morph_rotate_rle); the frame
    grows to hold every pixel."""
    ow, oh = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.morph_rotate_dims(src.width, src.height, float(angle), ctypes.byref(ow), ctypes.byref(oh)),
           "morph_rotate_dims")
    repr_ = MORPH_PACKED if isinstance(src, Bitmap) else MORPH_RLE
    dst = _empty_like_repr(src, ow.value, oh.value)
    n = _lib.morph_rotate_workspace_bytes(repr_, src.width, src.height, src.npages, float(angle))
    ws = torch.empty(max(n, 1), dtype=torch.uint8, device=_dev(src))
    p, nb = _ws(ws)
    f = _lib.morph_rotate_packed if repr_ == MORPH_PACKED else _lib.morph_rotate_rle
    _check(f(ctypes.byref(dst.struct()), ctypes.byref(src.struct()), float(angle), p, nb, _stream(stream)),
           "morph_rotate")
    return dst


def line_op(op: str, src, length: int, num: int, den: int, stream=None):
    """Erosion or dilation by a centred line of `length` pixels along the
    slope num/den, |num| <= den (morph_line_op_packed / morph_line_op_rle)."""
    if op not in ("erode", "dilate"):
        raise ValueError("line_op: erode or dilate")
    if den <= 0 or abs(num) > den:
        raise ValueError("line_op: |slope| must be at most 1 (transpose for steeper lines)")
    repr_ = MORPH_PACKED if isinstance(src, Bitmap) else MORPH_RLE
    k = OPS.index(op)
    dst = _empty_like_repr(src, src.width, src.height)
    n = _lib.morph_line_op_workspace_bytes(repr_, k, src.width, src.height, src.npages, length, num, den)
    if n == 0:
        raise MorphError(-8, "morph_line_op: sizes out of range")
    ws = torch.empty(n, dtype=torch.uint8, device=_dev(src))
    p, nb = _ws(ws)
    f = _lib.morph_line_op_packed if repr_ == MORPH_PACKED else _lib.morph_line_op_rle
    _check(f(k, ctypes.byref(dst.struct()), ctypes.byref(src.struct()), length, num, den, p, nb, _stream(stream)),
           "morph_line_op")
    return dst
