"""Connected components, statistics and run-length statistics on run-length
images, in plain Python (test infrastructure only).

* ``run_histograms``: the lengths of the black runs of every row, and of the
  white runs between two black runs of a row (section "Other Operations":
  run-length statistics in linear time over the runs; vertical ones by
  transposing first).
* ``histogram_percentile``: the smallest length at which a histogram's
  cumulative count reaches a given fraction of its total.
* ``label_runs``: section "Connected Component Extraction and Statistics":
  one union-find set per run; line by line, each run is merged with every
  run of the line above that touches it; finally every run takes its set's
  canonical representative.  Here the representative is numbered by the
  component's first run in raster order, so the numbering is unique.
  Runs touch when their pixel intervals overlap (4-connectivity) or overlap
  after widening by one pixel (8-connectivity).
* ``component_stats``: bounding box, area and coordinate sums (for
  centroids) per component, accumulated over the runs by label.
* ``layout_boxes``: the layout experiment of section "Document Analysis
  Performance" as this project reads it: spacing estimates from horizontal
  and vertical white-run statistics, a rectangular dilation that merges
  characters and lines into blocks, then the bounding boxes of the
  connected components.

Lines are lists of half-open runs ``(start, end)`` per row, as in
``oracle.rle_lines``; a page is a list of H lines of width W.
"""
from __future__ import annotations

import numpy as np

from . import apply as rect_apply, rle_decode, rle_encode
from .transpose import from_lines, rle_transpose, to_lines


def run_histograms(lines, W: int):
    """(black, white): int64 arrays of W + 1 bins; bin n counts the black
    runs of length n, resp. the white runs of length n that have a black run
    on both sides in the same row."""
    black = np.zeros(W + 1, dtype=np.int64)
    white = np.zeros(W + 1, dtype=np.int64)
    for line in lines:
        for k, (s, e) in enumerate(line):
            black[e - s] += 1
            if k > 0:
                white[s - line[k - 1][1]] += 1
    return black, white


def histogram_percentile(hist, num: int, den: int) -> int:
    """Smallest n with (count of lengths <= n) * den >= total * num, for
    0 < num <= den; 0 for an empty histogram."""
    total = int(sum(int(c) for c in hist))
    if total == 0:
        return 0
    acc = 0
    for n, c in enumerate(hist):
        acc += int(c)
        if acc * den >= total * num:
            return n
    return len(hist) - 1


class _UnionFind:
    def __init__(self, n):
        self.parent = list(range(n))

    def find(self, a):
        root = a
        while self.parent[root] != root:
            root = self.parent[root]
        while self.parent[a] != root:      # path compression
            self.parent[a], a = root, self.parent[a]
        return root

    def union(self, a, b):
        ra, rb = self.find(a), self.find(b)
        if ra != rb:
            self.parent[max(ra, rb)] = min(ra, rb)


def label_runs(lines, connectivity: int = 8):
    """Component label of every run (a list per line), numbered 0, 1, ... in
    the raster order of each component's first run, and the number of
    components."""
    if connectivity not in (4, 8):
        raise ValueError("connectivity is 4 or 8")
    c = 1 if connectivity == 8 else 0
    index = []                             # run -> running number over the image
    n = 0
    for line in lines:
        index.append(list(range(n, n + len(line))))
        n += len(line)
    uf = _UnionFind(n)
    for y in range(1, len(lines)):
        above = lines[y - 1]
        for k, (s, e) in enumerate(lines[y]):
            for m, (sa, ea) in enumerate(above):
                if sa < e + c and s < ea + c:      # the runs touch
                    uf.union(index[y][k], index[y - 1][m])
    number = {}
    labels = []
    for y, line in enumerate(lines):
        row = []
        for k in range(len(line)):
            root = uf.find(index[y][k])
            if root not in number:
                number[root] = len(number)
            row.append(number[root])
        labels.append(row)
    return labels, len(number)


def component_stats(lines, labels, ncomp: int):
    """Per component: [x0, y0, x1, y1, area, sum_x, sum_y] with the box
    half-open ([x0, x1) x [y0, y1)) and the sums over its pixels."""
    st = [[None, None, None, None, 0, 0, 0] for _ in range(ncomp)]
    for y, line in enumerate(lines):
        for (s, e), lab in zip(line, labels[y]):
            r = st[lab]
            r[0] = s if r[0] is None else min(r[0], s)
            r[1] = y if r[1] is None else min(r[1], y)
            r[2] = e if r[2] is None else max(r[2], e)
            r[3] = y + 1 if r[3] is None else max(r[3], y + 1)
            r[4] += e - s
            r[5] += sum(range(s, e))
            r[6] += y * (e - s)
    return np.array(st, dtype=np.int64).reshape(-1, 7)


def label_image(lines, labels, W: int) -> np.ndarray:
    """Pixel image of component numbers + 1 (0 = background)."""
    img = np.zeros((len(lines), W), dtype=np.int64)
    for y, line in enumerate(lines):
        for (s, e), lab in zip(line, labels[y]):
            img[y, s:e] = lab + 1
    return img


def layout_boxes(pages, W: int, num: int, den: int, connectivity: int = 8):
    """Layout analysis of a stack of equal pages (each a list of lines):
    gx = percentile num/den of the horizontal interior white runs of the
    whole stack, gy the same of the vertical ones (by transposition); the
    pages are dilated by the centred (gx + 1) x (gy + 1) rectangle, which
    closes every gap of at most gx pixels across and gy down; then the
    connected components of each dilated page and their statistics.
    Returns (gx, gy, [stats array per page])."""
    H = len(pages[0])
    hb = np.zeros(W + 1, dtype=np.int64)
    vb = np.zeros(H + 1, dtype=np.int64)
    for lines in pages:
        hb += run_histograms(lines, W)[1]
        vb += run_histograms(to_lines(*rle_transpose(*from_lines(lines), W, H)), H)[1]
    gx = histogram_percentile(hb, num, den)
    gy = histogram_percentile(vb, num, den)
    se = (gx + 1, gy + 1, (gx + 1) // 2, (gy + 1) // 2)
    out = []
    for lines in pages:
        rp, runs = from_lines(lines)
        img = rle_decode(rp, runs, W, H)
        smeared = to_lines(*rle_encode(rect_apply("dilate", img, se)))
        labels, n = label_runs(smeared, connectivity)
        out.append(component_stats(smeared, labels, n))
    return gx, gy, out
