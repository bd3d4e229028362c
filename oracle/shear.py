"""Line shifts, skews, rotation by skews and line operations at arbitrary
angles (test infrastructure only; sections "Scaling, Skewing, and Rotation"
and "Morphology with Lines at Arbitrary Orientations").

* ``shift_rows``: the within-line skew primitive: every line moves right by
  its own shift, pixels arriving from outside the source take a fill value,
  pixels leaving the destination frame are dropped.
* ``skew_shifts``: the shifts of a skew with a rational slope, as integers:
  line y moves by floor(num * (y - origin) / den) + offset.
* ``skew_rows`` / ``skew_cols``: lossless skews (the frame grows by the
  spread of the shifts); a column skew is a transpose, a line skew and a
  transpose back.
* ``rotate``: rotation as three skews (along the lines, across them, along
  them again), each lossless, with tan(angle / 2) and sin(angle) as given
  rationals.
* ``line_op``: erosion or dilation by a line at a slope num/den (|slope| <= 1):
  skew the columns so that the line becomes horizontal (the new pixels
  outside the image taking the border value of the operation), the
  horizontal operation, then the inverse skew back into the original frame.
"""
from __future__ import annotations

import numpy as np

from . import apply as rect_apply


def shift_rows(img, shifts, width: int, fill: int):
    """dst(x, y) = img(x - shifts[y], y) where that lies in the source, else
    fill; dst has the given width."""
    a = np.asarray(img, dtype=np.uint8)
    H, W = a.shape
    out = np.full((H, width), fill, dtype=np.uint8)
    for y in range(H):
        s = int(shifts[y])
        x0, x1 = max(0, s), min(width, W + s)
        if x0 < x1:
            out[y, x0:x1] = a[y, x0 - s:x1 - s]
    return out


def skew_shifts(n: int, num: int, den: int, origin: int, offset: int = 0):
    """floor(num * (y - origin) / den) + offset for y = 0 .. n-1 (den > 0)."""
    return np.array([(num * (y - origin)) // den + offset for y in range(n)], dtype=np.int64)


def skew_rows(img, num: int, den: int, origin: int, fill: int = 0):
    """Lossless line skew: returns (image, shifts) with the frame widened by
    the spread of the shifts and the smallest shift 0."""
    H, W = np.asarray(img).shape
    s = skew_shifts(H, num, den, origin)
    s = s - s.min()
    return shift_rows(img, s, W + int(s.max()), fill), s


def skew_cols(img, num: int, den: int, origin: int, fill: int = 0):
    t, s = skew_rows(np.ascontiguousarray(np.asarray(img).T), num, den, origin, fill)
    return np.ascontiguousarray(t.T), s


def rotate(img, tan_num: int, sin_num: int, den: int):
    """Rotation by three lossless skews about the frame centre: lines move by
    -tan(a/2) (y - cy), columns by sin(a) (x - cx), lines by -tan(a/2) again,
    with tan(a/2) = tan_num / den and sin(a) = sin_num / den."""
    a = np.asarray(img, dtype=np.uint8)
    a, _ = skew_rows(a, -tan_num, den, a.shape[0] // 2)
    a, _ = skew_cols(a, sin_num, den, a.shape[1] // 2)
    a, _ = skew_rows(a, -tan_num, den, a.shape[0] // 2)
    return a


def line_op(op: str, img, length: int, num: int, den: int):
    """Erosion or dilation by a centred line of `length` pixels along the
    slope num/den (|num| <= den): columns skewed by -floor(num x / den) so the
    line becomes horizontal, the horizontal operation (length x 1, origin
    length // 2), and the columns skewed back into the original frame.  The
    pixels the skew brings in from outside take the operation's border value
    (1 for erosion, 0 for dilation)."""
    a = np.asarray(img, dtype=np.uint8)
    H, W = a.shape
    fill = 1 if op == "erode" else 0
    v = np.array([-((num * x) // den) for x in range(W)], dtype=np.int64)
    off = -int(v.min())
    Ht = H + int(v.max()) + off
    at = np.ascontiguousarray(a.T)                      # W lines of length H
    sk = shift_rows(at, v + off, Ht, fill)              # column x moved down by v(x) + off
    res = rect_apply(op, np.ascontiguousarray(sk.T), (length, 1, length // 2, 0))
    back = shift_rows(np.ascontiguousarray(res.T), -(v + off), H, 0)
    return np.ascontiguousarray(back.T)
