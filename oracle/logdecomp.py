"""The paper's logarithmic decomposition on bit rows (test infrastructure only).

Plain-Python rendering, for small images, of the bit-blit strategy of the
paper's sections "Efficient Binary Decompositions" and "2D Morphological
Operators for Rectangular Masks": a rectangle operation is a row pass and a
column pass (separability), and each pass covers a line of n pixels with
shifted ANDs (ORs) whose shift doubles, plus one last shift of n - m where m
is the largest power of two not above n, plus a shift that puts the origin in
place.  Rows are Python integers, pixel x = bit x, so shifts are exact.

This is not the oracle; tests use it to show that the decomposition reaches
exactly the brute-force result (the equivalence the paper relies on).
"""
from __future__ import annotations


def _row_int(row):
    v = 0
    for x, p in enumerate(row):
        if p:
            v |= 1 << x
    return v


def _int_row(v, W):
    return [(v >> x) & 1 for x in range(W)]


def line_pass(v, W, n, origin, erode):
    """One line: out(x) = AND (OR) of a(x - origin .. x - origin + n - 1) for
    erosion, with pixels outside [0, W) = 1; for dilation the window is
    reflected, x - (n-1-origin) .. x + origin, outside = 0.  Written as a
    window that starts at offset lo: E_n(x) = op over a(x .. x+n-1), then
    out(x) = E_n(x + lo)."""
    pad = n + 2                          # room for every shift below
    full = (1 << (W + 2 * pad)) - 1
    inside = ((1 << W) - 1) << pad
    a = v << pad
    if erode:
        a |= full & ~inside              # outside = 1
        lo = -origin
    else:
        lo = -(n - 1 - origin)           # outside = 0
    E = a
    m = 1
    while 2 * m <= n:
        E = (E & (E >> m)) if erode else (E | (E >> m))
        m *= 2
    if m < n:
        s = n - m
        E = (E & (E >> s)) if erode else (E | (E >> s))
    # origin shift: out(x) = E(x + lo)
    if lo < 0:
        E = E << (-lo)
    else:
        E = E >> lo
    return (E >> pad) & ((1 << W) - 1)


def transpose(rows, W):
    H = len(rows)
    return [[rows[y][x] for y in range(H)] for x in range(W)]


def rect_op(img, op, se):
    """Rectangle operation on a list-of-lists 0/1 image by row pass then
    column pass, each log-decomposed; open/close composed."""
    w, h, cx, cy = se
    H = len(img)
    W = len(img[0]) if H else 0
    if op in ("erode", "dilate"):
        er = op == "erode"
        rows = [_int_row(line_pass(_row_int(r), W, w, cx, er), W) for r in img]
        cols = transpose(rows, W)
        cols = [_int_row(line_pass(_row_int(c), H, h, cy, er), H) for c in cols]
        return transpose(cols, H)
    if op == "open":
        return rect_op(rect_op(img, "erode", se), "dilate", se)
    if op == "close":
        return rect_op(rect_op(img, "dilate", se), "erode", se)
    raise ValueError(op)


def blit_count(n):
    """Number of shifted ANDs the doubling loop spends on a line of n pixels
    (excluding the origin shift): one per doubling step plus the last one."""
    m, c = 1, 0
    while 2 * m <= n:
        m *= 2
        c += 1
    if m < n:
        c += 1
    return c
