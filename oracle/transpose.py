"""Transposition of run-length images and the transpose-based rectangle
operations, in plain Python (test infrastructure only).

* ``rle_transpose`` is the plain definition: decode the run-length image to
  pixels, swap the axes, re-encode (the "decompress and recode" method the
  section "Efficient Transpose" starts from).
* ``transpose_lines`` works on run lists, one output line at a time: output
  line k collects the ranges of consecutive input lines whose runs cover
  pixel k.  It shares nothing with ``rle_transpose`` and pins it.
* ``rect_rlet`` composes a rectangle operation from within-line operations
  and transposition (section "Run Length Image Coding", the erode2d
  composition; section "2D Morphological Operators for Rectangular Masks",
  second strategy): the line operation along the rows, transpose, the line
  operation along the former columns, transpose back.  Opening and closing
  are an erosion and a dilation composed that way in turn.

Lines are lists of half-open runs ``(start, end)``, ascending and separated
by at least one white pixel, as in ``oracle.rle_lines``.
"""
from __future__ import annotations

import numpy as np

from . import rle_decode, rle_encode
from .rle_lines import dilate1d, erode1d


def rle_transpose(row_ptr, runs, W: int, H: int):
    """Transpose of an H x W run-length image: a W x H run-length image whose
    row x holds the runs of column x.  Returns (row_ptr int32[W+1],
    runs int32[n, 2])."""
    img = rle_decode(row_ptr, runs, W, H)
    return rle_encode(np.ascontiguousarray(img.T))


def transpose_lines(lines, W: int):
    """Transposition of a list of H lines of width W into W lines of width
    H, one output line at a time: output line k lists the maximal ranges of
    consecutive input lines whose runs cover pixel k (a binary search over
    each input line's run starts)."""
    import bisect
    H = len(lines)
    starts = [[s for s, _ in line] for line in lines]
    out = []
    for k in range(W):
        runs, first = [], None
        for i, line in enumerate(lines):
            j = bisect.bisect_right(starts[i], k) - 1
            covered = j >= 0 and k < line[j][1]
            if covered and first is None:
                first = i
            elif not covered and first is not None:
                runs.append((first, i))
                first = None
        if first is not None:
            runs.append((first, H))
        out.append(runs)
    return out


def _line_op(lines, n, origin, length, erode):
    f = erode1d if erode else dilate1d
    return [f(l, n, origin, length) for l in lines]


def _rlet_erode_dilate(lines, se, W: int, erode: bool):
    w, h, cx, cy = se
    H = len(lines)
    rows = _line_op(lines, w, cx, W, erode)            # along the rows
    cols = transpose_lines(rows, W)                     # W lines of length H
    cols = _line_op(cols, h, cy, H, erode)              # along the former columns
    return transpose_lines(cols, H)                     # back: H lines of length W


def rect_rlet(lines, op: str, se, W: int):
    """A w x h rectangle operation on H lines of width W by within-line
    operations and transposition."""
    if op == "erode":
        return _rlet_erode_dilate(lines, se, W, True)
    if op == "dilate":
        return _rlet_erode_dilate(lines, se, W, False)
    if op == "open":
        return _rlet_erode_dilate(_rlet_erode_dilate(lines, se, W, True), se, W, False)
    if op == "close":
        return _rlet_erode_dilate(_rlet_erode_dilate(lines, se, W, False), se, W, True)
    raise ValueError(op)


def to_lines(row_ptr, runs):
    rp = np.asarray(row_ptr)
    rr = np.asarray(runs).reshape(-1, 2)
    return [[(int(rr[k, 0]), int(rr[k, 1])) for k in range(rp[y], rp[y + 1])]
            for y in range(len(rp) - 1)]


def from_lines(lines):
    row_ptr = np.zeros(len(lines) + 1, dtype=np.int32)
    flat = []
    for y, l in enumerate(lines):
        flat.extend(l)
        row_ptr[y + 1] = len(flat)
    runs = np.array(flat, dtype=np.int32).reshape(-1, 2)
    return row_ptr, runs


def rlet_apply(op: str, row_ptr, runs, W: int, se):
    """``rect_rlet`` on CSR arrays: returns (row_ptr, runs)."""
    return from_lines(rect_rlet(to_lines(row_ptr, runs), op, se, W))
