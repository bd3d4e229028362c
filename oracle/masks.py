"""Erosion, dilation, opening and closing by arbitrary masks (test
infrastructure only; section "Morphology with Arbitrary Masks").

A mask is an h x w array of 0/1 with an origin (cx, cy) inside its frame:
    erode(x, y)  = AND of A(x + i - cx, y + j - cy) over the mask's pixels (i, j)
    dilate(x, y) = OR  of A(x - i + cx, y - j + cy) over the mask's pixels
with outside pixels 1 for erosion and 0 for dilation, as for rectangles
(dilation uses the reflected mask, i.e. it is the union of the mask placed
at every black pixel).  open = dilate(erode), close = erode(dilate).

* ``apply`` is that definition written out: one shifted AND (OR) of the
  whole image per mask pixel.
* ``runs_of`` lists the mask's horizontal runs.
* ``erode_lines_by_runs`` is the section's run-length method: for every run
  of the mask, erode each line of a copy of the image by the run's length
  (shifted by the run's offset) and intersect it into an accumulator.
* ``erode_rows_by_doubling`` is the section's bit-blit method: horizontal
  erosions by 1, 2, 4, ... pixels are built up once, and each mask run takes
  the largest one not longer than itself, twice, at the run's two ends.

An empty mask erodes to all 1s and dilates to all 0s.
"""
from __future__ import annotations

import numpy as np

from .rle_lines import line_and


def disc(r: int):
    """The disc of radius r: (2r+1) x (2r+1), pixel (i, j) set when
    (i - r)^2 + (j - r)^2 <= r^2, origin (r, r)."""
    j, i = np.mgrid[0:2 * r + 1, 0:2 * r + 1]
    return ((i - r) ** 2 + (j - r) ** 2 <= r * r).astype(np.uint8), r, r


def reflect(mask, cx, cy):
    h, w = mask.shape
    return np.ascontiguousarray(mask[::-1, ::-1]), w - 1 - cx, h - 1 - cy


def _shifted(img, dx, dy, outside):
    """S(x, y) = img(x + dx, y + dy), outside pixels = outside."""
    H, W = img.shape
    out = np.full((H, W), outside, dtype=np.uint8)
    x0, x1 = max(0, -dx), min(W, W - dx)
    y0, y1 = max(0, -dy), min(H, H - dy)
    if x0 < x1 and y0 < y1:
        out[y0:y1, x0:x1] = img[y0 + dy:y1 + dy, x0 + dx:x1 + dx]
    return out


def erode(img, mask, cx, cy):
    a = np.ascontiguousarray(img, dtype=np.uint8)
    out = np.ones_like(a)
    for j, i in zip(*np.nonzero(mask)):
        out &= _shifted(a, int(i) - cx, int(j) - cy, 1)
    return out


def dilate(img, mask, cx, cy):
    a = np.ascontiguousarray(img, dtype=np.uint8)
    out = np.zeros_like(a)
    for j, i in zip(*np.nonzero(mask)):
        out |= _shifted(a, cx - int(i), cy - int(j), 0)
    return out


def apply(op: str, img, mask, cx: int, cy: int):
    if op == "erode":
        return erode(img, mask, cx, cy)
    if op == "dilate":
        return dilate(img, mask, cx, cy)
    if op == "open":
        return dilate(erode(img, mask, cx, cy), mask, cx, cy)
    if op == "close":
        return erode(dilate(img, mask, cx, cy), mask, cx, cy)
    raise ValueError(op)


def runs_of(mask, cx: int, cy: int):
    """Horizontal runs of the mask as (dx, dy, length): the run covers mask
    pixels (cx + dx .. cx + dx + length - 1, cy + dy)."""
    out = []
    for j, row in enumerate(np.asarray(mask)):
        i = 0
        w = len(row)
        while i < w:
            if row[i]:
                k = i
                while k < w and row[k]:
                    k += 1
                out.append((i - cx, j - cy, k - i))
                i = k
            else:
                i += 1
    return out


def _erode_line_by_run(line, dx, length, W):
    """out(x) = AND of A(x + dx .. x + dx + length - 1) on a line of width W
    (outside = 1): each maximal run, extended to infinity where it touches a
    border, keeps the x whose window lies inside it."""
    ext = []
    BIG = 1 << 40
    for s, e in line:
        ext.append([-BIG if s == 0 else s, BIG if e == W else e])
    if not ext or ext[0][0] != -BIG:
        ext.insert(0, [-BIG, 0])
    if ext[-1][1] != BIG:
        ext.append([W, BIG])
    out = []
    for s, e in ext:
        a, b = max(0, s - dx), min(W, e - dx - length + 1)
        if a < b:
            out.append((a, b))
    return out


def erode_lines_by_runs(lines, mask, cx, cy, W):
    """Erosion of a run-length image (H lines of width W) run by run of the
    mask: a copy of the image is eroded line by line by the run and shifted
    down by the run's row offset; the results are intersected."""
    H = len(lines)
    acc = [[(0, W)] if W > 0 else [] for _ in range(H)]
    for dx, dy, length in runs_of(mask, cx, cy):
        for y in range(H):
            src = y + dy
            if 0 <= src < H:
                t = _erode_line_by_run(lines[src], dx, length, W)
            else:
                t = [(0, W)]                    # a whole line outside the image
            acc[y] = line_and(acc[y], t)
    return acc


def erode_rows_by_doubling(img, mask, cx, cy):
    """Erosion of a bit image by the doubling accumulation: each row held as
    a Python integer (bit x = pixel x), padded with 1s, E[k] the horizontal
    erosion by 2^k computed once; a run of length n uses E[k] for the
    largest 2^k <= n at its start and at its end."""
    a = np.asarray(img, dtype=np.uint8)
    H, W = a.shape
    runs = runs_of(mask, cx, cy)
    if not runs:
        return np.ones_like(a)
    pad = max([max(0, -dx) for dx, _, _ in runs] + [0])
    padr = max([max(0, dx + n) for dx, _, n in runs] + [0])
    width = pad + W + padr
    ones = (1 << width) - 1
    rows = []
    for y in range(H):
        v = ones
        for x in range(W):
            if not a[y, x]:
                v &= ~(1 << (pad + x))
        rows.append(v)
    maxlen = max(n for _, _, n in runs)
    E = [rows]
    k = 1
    while 2 * k <= maxlen:
        prev = E[-1]
        E.append([(v & ((v >> k) | (ones ^ (ones >> k)))) for v in prev])
        k *= 2
    out = np.ones((H, W), dtype=np.uint8)
    for dx, dy, n in runs:
        lvl = n.bit_length() - 1
        m = 1 << lvl
        for y in range(H):
            src = y + dy
            if not 0 <= src < H:
                continue                        # a whole row outside: all 1s
            v = E[lvl][src]
            t = (v >> (pad + dx)) & (v >> (pad + dx + n - m))
            for x in range(W):
                if not (t >> x) & 1:
                    out[y, x] = 0
    return out
