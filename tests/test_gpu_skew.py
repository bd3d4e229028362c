"""GPU parity of line shifts, skews, rotation by skews and line operations at
a slope against the oracle, on packed images (words, pad bits 0) and
run-length images (row_ptr and runs exactly)."""
import math

import numpy as np
import pytest
import torch

import oracle
import pagegen
from gpu_util import blobs_img, garbage_pad, require_gpu, rnd_img
from oracle import shear as osh

pytestmark = pytest.mark.gpu

M = None


@pytest.fixture(scope="module", autouse=True)
def lib():
    require_gpu()
    global M
    import paper_0712_0121_amd as m
    M = m
    return m


def both(img, npages=1):
    rows, W = img.shape
    words = garbage_pad(oracle.pack(img, (W + 63) // 64 + 1), W, 9)
    b = M.Bitmap.from_words(words, W, npages=npages)
    return b, M.pack_to_rle(b)


def assert_img(got, want, what=""):
    if isinstance(got, M.Bitmap):
        torch.cuda.synchronize()
        assert (got.height * got.npages, got.width) == want.shape, what
        np.testing.assert_array_equal(got.to_numpy(), oracle.pack(want), err_msg="packed " + what)
    else:
        rp, runs = got.to_host()
        wrp, wruns = oracle.rle_encode(want)
        np.testing.assert_array_equal(rp, wrp, err_msg="runs row_ptr " + what)
        np.testing.assert_array_equal(runs, wruns, err_msg="runs " + what)


@pytest.mark.parametrize("W", [1, 63, 64, 65, 200])
def test_shift_rows_match_oracle(W):
    H = 41
    r = np.random.default_rng(W)
    img = blobs_img(W + 5, H, W, 0.5) if W > 1 else rnd_img(3, H, W, 0.5)
    img[0] = 1                                      # a full line: border runs on both sides
    shifts = r.integers(-W - 20, W + 20, H)
    shifts[:5] = [0, -W, W, 1, -1]
    pk, rl = both(img)
    for width in sorted({W, W + 37, max(1, W - 10), 1, 130}):
        for fill in (0, 1):
            d = torch.from_numpy(shifts.astype(np.int32)).cuda()
            want = osh.shift_rows(img, shifts, width, fill)
            assert_img(M.shift_rows(pk, d, width, fill), want, "W=%d to %d fill %d" % (W, width, fill))
            assert_img(M.shift_rows(rl, d, width, fill), want, "W=%d to %d fill %d" % (W, width, fill))


def test_shift_rows_stacked_pages_and_huge_shifts():
    P, H, W = 3, 30, 150
    img = np.concatenate([blobs_img(40 + k, H, W, 0.5) for k in range(P)])
    shifts = np.random.default_rng(2).integers(-200, 200, P * H)
    shifts[7] = 2 ** 31 - 1
    shifts[8] = -2 ** 31
    d = torch.from_numpy(shifts.astype(np.int32)).cuda()
    pk, rl = both(img, P)
    for fill in (0, 1):
        want = osh.shift_rows(img, np.clip(shifts, -2 ** 30, 2 ** 30), 170, fill)
        assert_img(M.shift_rows(pk, d, 170, fill), want, "fill %d" % fill)
        assert_img(M.shift_rows(rl, d, 170, fill), want, "fill %d" % fill)


@pytest.mark.parametrize("slope", [(0, 1), (1, 1), (-1, 1), (3, 7), (-5, 2)], ids=lambda s: "%d_%d" % s)
def test_skews_match_oracle(slope):
    num, den = slope
    img = blobs_img(num + 50, 60, 130, 0.4)
    pk, rl = both(img)
    want_r, v = osh.skew_rows(img, num, den, 20)
    want_c, _ = osh.skew_cols(img, num, den, 33)
    for src in (pk, rl):
        got, gv = M.skew_rows(src, num, den, 20)
        np.testing.assert_array_equal(gv, v)
        assert_img(got, want_r, "rows %d/%d" % slope)
        got, _ = M.skew_cols(src, num, den, 33)
        assert_img(got, want_c, "cols %d/%d" % slope)


@pytest.mark.parametrize("angle", [0.0, 0.1, -0.35, 0.7, np.pi / 2], ids=lambda a: "%.2f" % a)
def test_rotation_matches_oracle(angle):
    img = blobs_img(7, 80, 120, 0.4)
    # tan(a/2) and sin(a) over 2^16, computed here and not by the binding
    den = 1 << 16
    tn, sn = int(round(math.tan(angle / 2) * den)), int(round(math.sin(angle) * den))
    assert M.rotation_rationals(angle) == (tn, sn, den)
    want = osh.rotate(img, tn, sn, den)
    pk, rl = both(img)
    assert_img(M.rotate(pk, angle), want, "packed %.2f" % angle)
    assert_img(M.rotate(rl, angle), want, "runs %.2f" % angle)


@pytest.mark.parametrize("op", ["erode", "dilate"])
@pytest.mark.parametrize("slope", [(0, 1), (1, 1), (-1, 1), (1, 3), (-2, 5), (7, 8)], ids=lambda s: "%d_%d" % s)
def test_line_ops_match_oracle(op, slope):
    num, den = slope
    img = blobs_img(abs(num) * 3 + den + 10, 70, 150, 0.5)
    pk, rl = both(img)
    for length in (3, 8, 15):
        want = osh.line_op(op, img, length, num, den)
        assert_img(M.line_op(op, pk, length, num, den), want, "packed %s %d/%d len %d" % (op, num, den, length))
        assert_img(M.line_op(op, rl, length, num, den), want, "runs %s %d/%d len %d" % (op, num, den, length))


def test_line_op_letter_page():
    img = pagegen.letter_page(2000).img
    pk, rl = both(img)
    for op in ("erode", "dilate"):
        want = osh.line_op(op, img, 21, 1, 2)
        assert_img(M.line_op(op, pk, 21, 1, 2), want, "packed " + op)
        assert_img(M.line_op(op, rl, 21, 1, 2), want, "runs " + op)


def test_compositions_on_stacked_pages():
    """Skews, rotation and a line operation over three stacked pages: every
    page on its own, as the oracle does it page by page."""
    P, H, W = 3, 50, 90
    pages = [blobs_img(60 + k, H, W, 0.4) for k in range(P)]
    pk, rl = both(np.concatenate(pages), P)
    den = 1 << 16
    tn, sn = int(round(math.tan(0.3) * den)), int(round(math.sin(0.6) * den))
    for src in (pk, rl):
        got, _ = M.skew_cols(src, -3, 5, 40)
        assert_img(got, np.concatenate([osh.skew_cols(p, -3, 5, 40)[0] for p in pages]), "skew cols")
        assert_img(M.rotate(src, 0.6), np.concatenate([osh.rotate(p, tn, sn, den) for p in pages]), "rotate")
        assert_img(M.line_op("dilate", src, 9, 2, 3),
                   np.concatenate([osh.line_op("dilate", p, 9, 2, 3) for p in pages]), "line")
