"""Seeded synthetic binary document pages (shared by tests, oracle and bench).

This module holds no morphology: it only draws pages, packs them into the
word layout, and draws request streams.  The pages stand in for the paper's
scanned journal pages (300 dpi letter-size, binarized), which are not
available here; nothing of that collection is reproduced.  Every generator
takes an integer seed and uses ``numpy.random.Generator(PCG64(seed))``.

Workloads (image sizes are W x H; structuring elements are written h x w,
so "1x31" is a horizontal line 31 pixels wide):

* ``small_page``   512 x 512, ~8% black: filled rectangles 3-12 px along text
                   lines, then salt noise (each pixel toggled with p=0.001).
* ``text_page``    letter page 2550 x 3300 (or any size): ~35 lines of
                   glyph-like connected strokes 20-40 px tall, 5-10% black,
                   2-3 ruled lines, speckle (pixels set with p=0.0005).
* ``mixed_batch``  256 pages of sizes 1275x1650, 2480x3508, 2550x3300 and
                   5100x6600, each with a random rectangle (w, h in [1,63])
                   and a random operation.
* ``density_page`` 2550 x 3300 at 1%, 10% or 40% black from rectangles plus
                   Bernoulli (XOR) noise tuned to ~2, ~20, ~60 runs per row.
* ``poisson_trace`` arrival times of a fixed-rate request stream.
"""
from __future__ import annotations

import dataclasses

import numpy as np

OPS = ("erode", "dilate", "open", "close")
PAGE_SIZES = ((1275, 1650), (2480, 3508), (2550, 3300), (5100, 6600))
PAGE_SCALE = {(1275, 1650): 0.5, (2480, 3508): 1.0, (2550, 3300): 1.0, (5100, 6600): 2.0}
# serving chain: close 1x41 -> open 3x3 -> dilate 15x5 -> erode 15x5 (h x w)
SERVE_CHAIN = (("close", 41, 1), ("open", 3, 3), ("dilate", 5, 15), ("erode", 5, 15))


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def words_per_row(W: int) -> int:
    return (W + 63) // 64


def to_words(img: np.ndarray, stride: int | None = None) -> np.ndarray:
    """Byte image (H, W) of 0/1 -> (H, stride) uint64, pixel x at bit x & 63
    of word x >> 6, pad bits 0 (numpy.packbits, little bit order)."""
    H, W = img.shape
    if stride is None:
        stride = words_per_row(W)
    b = np.packbits(img.astype(np.uint8, copy=False), axis=1, bitorder="little")
    out = np.zeros((H, stride * 8), dtype=np.uint8)
    out[:, : b.shape[1]] = b
    return out.view("<u8")


@dataclasses.dataclass
class Page:
    img: np.ndarray            # (H, W) uint8, 0/1
    seed: int

    @property
    def H(self) -> int:
        return self.img.shape[0]

    @property
    def W(self) -> int:
        return self.img.shape[1]

    def words(self, stride: int | None = None) -> np.ndarray:
        return to_words(self.img, stride)

    @property
    def density(self) -> float:
        return float(self.img.mean())

    def runs_per_row(self) -> float:
        a = self.img.astype(np.int8)
        starts = (a[:, 1:] > a[:, :-1]).sum() + a[:, 0].sum()
        return float(starts) / self.H


# ------------------------------------------------------------------ drawing
def _salt(img, r, p):
    """Toggle each pixel independently with probability p."""
    n = r.binomial(img.size, p)
    idx = r.integers(0, img.size, n)
    flat = img.reshape(-1)
    np.bitwise_xor.at(flat, idx, 1)


def _speckle(img, r, p):
    """Set each pixel independently with probability p."""
    n = r.binomial(img.size, p)
    idx = r.integers(0, img.size, n)
    img.reshape(-1)[idx] = 1


def small_page(seed: int, W: int = 512, H: int = 512) -> Page:
    """Filled rectangles with sides in [3,12] along text lines (pitch ~24 px)
    until 8% +- 0.5% black, then salt noise p = 0.001."""
    r = rng(seed)
    img = np.zeros((H, W), dtype=np.uint8)
    pitch = 24
    lines = list(range(8, H - 12, pitch))
    target = 0.08
    black = 0
    while black < (target - 0.004) * W * H:
        y0 = lines[r.integers(len(lines))] + int(r.integers(0, 6))
        x0 = int(r.integers(0, W - 3))
        w, h = (int(v) for v in r.integers(3, 13, 2))
        img[y0:y0 + h, x0:x0 + w] = 1
        black = int(img.sum())
    _salt(img, r, 0.001)
    return Page(img, seed)


def _glyph(img, r, x0, y0, gw, gh, t):
    """A glyph-like component: 1-4 stroke rectangles of thickness t that all
    touch a first vertical stem, so the glyph is connected."""
    H, W = img.shape
    img[y0:y0 + gh, x0:x0 + t] = 1                                 # stem
    for _ in range(int(r.integers(0, 4))):
        kind = int(r.integers(0, 4))
        if kind == 0:
            img[y0:y0 + t, x0:x0 + gw] = 1                         # top bar
        elif kind == 1:
            img[y0 + gh - t:y0 + gh, x0:x0 + gw] = 1               # foot
        elif kind == 2:
            ym = y0 + int(r.integers(0, max(1, gh - t)))
            img[ym:ym + t, x0:x0 + gw] = 1                         # cross bar
        else:
            yb = y0 + int(r.integers(0, max(1, gh // 2)))
            img[yb:y0 + gh, x0 + gw - t:x0 + gw] = 1               # second stem
            img[yb:yb + t, x0:x0 + gw] = 1                         # joined on top


def text_page(seed: int, W: int = 2550, H: int = 3300, scale: float | None = None) -> Page:
    """A text-like page: about 35 lines of glyphs 20-40 px tall (x scale),
    words of 3-8 glyphs, 5-10% black, 2-3 ruled lines 2-4 px thick and
    60-100% of the width, speckle p = 0.0005.  Redrawn with another stroke
    weight until the density is in [5%, 10%]."""
    if scale is None:
        scale = PAGE_SCALE.get((W, H), W / 2550.0)
    r = rng(seed)
    weight = 1.0
    for _attempt in range(8):
        img = np.zeros((H, W), dtype=np.uint8)
        mx = int(r.integers(150, 301) * scale)
        my = int(r.integers(150, 301) * scale)
        nlines = 35
        pitch = (H - 2 * my) / nlines
        for li in range(nlines):
            yl = int(my + li * pitch)
            x = mx
            in_word = int(r.integers(3, 9))
            while True:
                gh = int(r.integers(20, 41) * scale)
                gw = int(r.integers(8, 31) * scale)
                if x + gw >= W - mx:
                    break
                t = max(1, int(round(r.integers(2, 6) * scale * weight)))
                t = min(t, gw, gh)
                y0 = yl + int(r.integers(0, max(1, int(pitch) - gh)))
                y0 = min(y0, H - gh)
                _glyph(img, r, x, y0, gw, gh, t)
                x += gw + int(r.integers(2, 7) * scale)
                in_word -= 1
                if in_word == 0:
                    x += int(r.integers(12, 26) * scale)
                    in_word = int(r.integers(3, 9))
        for _ in range(int(r.integers(2, 4))):
            th = int(r.integers(2, 5) * scale)
            ln = int(W * r.uniform(0.6, 1.0))
            x0 = int(r.integers(0, W - ln + 1))
            y0 = int(r.integers(0, H - th))
            img[y0:y0 + th, x0:x0 + ln] = 1
        _speckle(img, r, 0.0005)
        d = img.mean()
        if 0.05 <= d <= 0.10:
            break
        weight *= (0.075 / max(d, 1e-3)) ** 0.8
    return Page(img, seed)


def letter_page(seed: int) -> Page:
    return text_page(seed, 2550, 3300, 1.0)


@dataclasses.dataclass
class BatchItem:
    page: Page
    op: str
    se: tuple            # (w, h, cx, cy)


def mixed_batch(n: int = 256, seed: int = 3000, pool_per_size: int = 4,
                max_se: int = 63) -> list:
    """n pages with sizes uniform over PAGE_SIZES, each with a random
    rectangle (w, h uniform in [1, max_se], centred origin) and a random
    operation.  Page content comes from a pool of pool_per_size distinct
    pages per size (the batch still gets its own buffer per page)."""
    r = rng(seed)
    pool = {}
    items = []
    for i in range(n):
        size = PAGE_SIZES[int(r.integers(len(PAGE_SIZES)))]
        k = int(r.integers(pool_per_size))
        key = (size, k)
        if key not in pool:
            pool[key] = text_page(seed * 1000 + PAGE_SIZES.index(size) * 100 + k, *size)
        w, h = (int(v) for v in r.integers(1, max_se + 1, 2))
        op = OPS[int(r.integers(4))]
        items.append(BatchItem(pool[key], op, (w, h, w // 2, h // 2)))
    return items


def density_page(density: float, seed: int, W: int = 2550, H: int = 3300) -> Page:
    """Axis-aligned filled rectangles up to about the target density, then
    XOR noise with q tuned (a few seeded bisection steps) so the mean number
    of runs per row is near 2 (1%), 20 (10%) or 60 (40%)."""
    targets = {0.01: 2.0, 0.10: 20.0, 0.40: 60.0}
    want_runs = targets.get(round(density, 2), 2.0 + 145.0 * density)
    r = rng(seed)
    base = np.zeros((H, W), dtype=np.uint8)
    # rectangles: widths chosen so that rectangles alone give fewer runs than wanted
    while base.mean() < density:
        bw = int(r.integers(8, 200)) if density < 0.2 else int(r.integers(40, 400))
        bh = int(r.integers(4, 120))
        x0 = int(r.integers(0, W - bw))
        y0 = int(r.integers(0, H - bh))
        base[y0:y0 + bh, x0:x0 + bw] = 1
    page = Page(base, seed)
    if page.runs_per_row() >= want_runs:
        return page
    lo, hi = 0.0, 0.05
    best = base
    for _ in range(12):
        q = 0.5 * (lo + hi)
        img = base.copy()
        _salt(img, rng(seed + 1), q)
        p = Page(img, seed)
        if p.runs_per_row() < want_runs:
            lo = q
        else:
            hi = q
        best = img
    return Page(best, seed)


def poisson_trace(qps: float, duration_s: float, seed: int = 5000):
    """Arrival times (seconds from start) of a Poisson stream."""
    r = rng(seed)
    t, out = 0.0, []
    while True:
        t += float(r.exponential(1.0 / qps))
        if t >= duration_s:
            return np.array(out)
        out.append(t)
