"""The paper's run-list operations, in plain Python (test infrastructure only).

These follow the paper's run-length algorithms step by step for small cases,
so that tests can check the brute-force oracle against the paper's own
description of what each step computes:

* within-line operations (section "Within-Line Morphological Operations"):
  complement, one-dimensional opening/closing as deletion of short runs/gaps,
  one-dimensional erosion as shrinking runs and dilation by complementation;
* between-line boolean operations (section "Between Line Boolean
  Operations"): the combined value of two lines at every run boundary of
  either, fed in ascending order to a sink that reassembles intervals;
* the logarithmic decomposition of a line structuring element applied
  between lines (section "Efficient Binary Decompositions").

A line is a list of half-open runs ``(start, end)`` of 1s, ascending, with
``end_j < start_{j+1}``.  The paper writes closed intervals but its
complement step only makes sense for half-open ones; this module uses
half-open intervals throughout.  Border handling is the one fixed for the
whole project: outside the line, pixels count as 1 for erosion and 0 for
dilation.
"""
from __future__ import annotations

# ------------------------------------------------------------ within a line
def complement(runs, W):
    """Gaps of the line within [0, W) become runs and runs become gaps."""
    out = []
    last = 0
    for s, e in runs:
        if s > last:
            out.append((last, s))
        last = e
    if last < W:
        out.append((last, W))
    return out


def open1d_interior(runs, u):
    """Delete every run narrower than u (the paper's one-dimensional
    opening).  Equal to dilation(erosion) by a 1 x u element only for runs
    that do not touch the ends of the line."""
    return [(s, e) for s, e in runs if e - s >= u]


def close1d_interior(runs, u, W):
    """Fill every gap narrower than u: complement, open, complement."""
    return complement(open1d_interior(complement(runs, W), u), W)


def erode1d(runs, w, cx, W):
    """Erosion of one line by a 1 x w element with origin cx.

    Each run loses cx pixels on its left and w-1-cx on its right; a run
    that vanishes is dropped.  For odd w centred (cx = w//2) this is the
    paper's shrink by floor(w/2) on each side.  A run end lying on the line
    border does not move, because outside pixels count as 1."""
    out = []
    for s, e in runs:
        ns = 0 if s == 0 else s + cx
        ne = W if e == W else e - (w - 1 - cx)
        if ns < ne:
            out.append((ns, ne))
    return out


def dilate1d(runs, w, cx, W):
    """Dilation of one line by a 1 x w element with origin cx, as the
    complement of the erosion of the complement by the reflected element
    (the paper's second formulation).  Outside pixels count as 0, so the
    complement is taken on [0, W) and eroded with outside = 1."""
    return complement(erode1d(complement(runs, W), w, w - 1 - cx, W), W)


def dilate1d_direct(runs, w, cx, W):
    """The direct form: grow each run by cx on the left and w-1-cx on the
    right, clip to [0, W) and merge runs that overlap or touch."""
    out = []
    for s, e in runs:
        ns, ne = max(0, s - cx), min(W, e + (w - 1 - cx))
        if out and ns <= out[-1][1]:
            out[-1] = (out[-1][0], max(out[-1][1], ne))
        else:
            out.append((ns, ne))
    return out


# ------------------------------------------------------- between two lines
class TransitionSink:
    """Accepts (coordinate, value) pairs in ascending coordinate order and
    re-assembles the intervals where the value is true.  Empty intervals are
    dropped and intervals that touch are joined, so the output is the
    canonical run list."""

    def __init__(self):
        self.runs = []
        self._open = None

    def append(self, x, v):
        if v and self._open is None:
            if self.runs and self.runs[-1][1] == x:     # touching: reopen
                self._open = self.runs.pop()[0]
            else:
                self._open = x
        elif not v and self._open is not None:
            if x > self._open:
                self.runs.append((self._open, x))
            self._open = None


def _covers(line, x):
    """Whether pixel x lies in one of the line's runs."""
    return any(s <= x < e for s, e in line)


def line_merge(l1, l2, combine, offset2=0):
    """A boolean combination of two lines (the second shifted by offset2),
    from the definition: the combined line can only change value where one
    of the two lines does, so it is constant between consecutive run
    boundaries of either line.  At every boundary coordinate x (in
    ascending order) the sink receives combine(pixel x in line 1, pixel x
    in line 2), and it turns these values into the canonical runs."""
    a = list(l1)
    b = [(s + offset2, e + offset2) for s, e in l2]
    cuts = sorted({x for s, e in a + b for x in (s, e)})
    sink = TransitionSink()
    for x in cuts:
        sink.append(x, combine(_covers(a, x), _covers(b, x)))
    return sink.runs


def line_and(l1, l2):
    return line_merge(l1, l2, lambda a, b: a and b)


def line_or(l1, l2):
    return line_merge(l1, l2, lambda a, b: a or b)


# ---------------------------------------------- between lines, log-decomposed
def column_op(lines, h, cy, W, erode=True):
    """Erosion (erode=True) or dilation of a run-length image by an h x 1
    element with origin row cy, by logarithmic decomposition between lines:
    E_1 = the lines; E_2k[y] = E_k[y] op E_k[y+k]; after doubling up to the
    largest power of two m <= h, one more step with offset h-m gives the AND
    (OR) over h consecutive lines; the origin then selects which run of h
    lines each output line takes.  Lines outside the image are full (erosion)
    or empty (dilation)."""
    H = len(lines)
    if erode:
        op, outside, top = line_and, [(0, W)] if W > 0 else [], cy
    else:
        op, outside, top = line_or, [], h - 1 - cy
    # extended index range: row r of E holds image row r - top
    n = H + h - 1
    E = [lines[r - top] if 0 <= r - top < H else outside for r in range(n)]
    k = 1
    while 2 * k <= h:
        E = [op(E[r], E[r + k]) if r + k < len(E) else None for r in range(len(E) - k)]
        k *= 2
    if k < h:
        s = h - k
        E = [op(E[r], E[r + s]) for r in range(len(E) - s)]
    return [E[y] for y in range(H)]


def rect_op(lines, op, se, W):
    """A w x h rectangle operation on a run-length image: the within-line
    pass first, then the between-line pass (the paper's fastest strategy),
    with opening and closing composed from erosion and dilation."""
    w, h, cx, cy = se
    if op == "erode":
        rows = [erode1d(l, w, cx, W) for l in lines]
        return column_op(rows, h, cy, W, erode=True)
    if op == "dilate":
        rows = [dilate1d(l, w, cx, W) for l in lines]
        return column_op(rows, h, cy, W, erode=False)
    if op == "open":
        return rect_op(rect_op(lines, "erode", se, W), "dilate", se, W)
    if op == "close":
        return rect_op(rect_op(lines, "dilate", se, W), "erode", se, W)
    raise ValueError(op)
