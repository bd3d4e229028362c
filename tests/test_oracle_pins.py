"""Pins for the CPU oracle: each test checks it against something other than
itself -- a library routine, a closed form, an algebraic law of morphology,
brute-force enumeration, or a value the paper states for a worked example.

The conventions being pinned: B(w,h,cx,cy) is a w x h rectangle with origin
(cx,cy); erosion counts outside pixels as 1, dilation as 0 and uses the
reflected window (Minkowski dilation); opening = dilation(erosion),
closing = erosion(dilation).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage as ndi

import oracle
from oracle import logdecomp, rle_lines

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")


def rnd_img(seed, H, W, p=0.5):
    r = np.random.default_rng(seed)
    return (r.random((H, W)) < p).astype(np.uint8)


def all_ses(maxw, maxh):
    for w in range(1, maxw + 1):
        for h in range(1, maxh + 1):
            for cx in range(w):
                for cy in range(h):
                    yield (w, h, cx, cy)


# -------------------------------------------------------------- library pin
def scipy_op(op, img, se):
    """scipy.ndimage with origin = c - size//2 per axis; erosion border 1,
    dilation border 0 (scipy's dilation reflects the element)."""
    w, h, cx, cy = se
    st = np.ones((h, w), bool)
    org = (cy - h // 2, cx - w // 2)
    ero = lambda a: ndi.binary_erosion(a, st, origin=org, border_value=1)
    dil = lambda a: ndi.binary_dilation(a, st, origin=org, border_value=0)
    a = img.astype(bool)
    r = {"erode": lambda: ero(a), "dilate": lambda: dil(a),
         "open": lambda: dil(ero(a)), "close": lambda: ero(dil(a))}[op]()
    return r.astype(np.uint8)


@pytest.mark.parametrize("op", oracle.OPS)
def test_matches_scipy_all_small_elements(op):
    img = rnd_img(1, 9, 11, 0.55)
    for se in all_ses(4, 4):
        np.testing.assert_array_equal(oracle.apply(op, img, se), scipy_op(op, img, se), err_msg=str(se))


@pytest.mark.parametrize("op", oracle.OPS)
def test_matches_scipy_random_larger(op):
    r = np.random.default_rng(7)
    for t in range(12):
        H, W = int(r.integers(1, 70)), int(r.integers(1, 140))
        img = rnd_img(100 + t, H, W, float(r.uniform(0.1, 0.9)))
        w, h = int(r.integers(1, 20)), int(r.integers(1, 20))
        se = (w, h, int(r.integers(w)), int(r.integers(h)))
        np.testing.assert_array_equal(oracle.apply(op, img, se), scipy_op(op, img, se), err_msg=str((H, W, se)))


# ----------------------------------------------------- brute-force enumeration
def test_exhaustive_1d_rows():
    """Every row of up to 8 pixels, every 1 x w element (w <= 5), every origin,
    against the set definition evaluated by enumeration of the window."""
    for W in range(1, 9):
        for bits in range(1 << W):
            row = np.array([[(bits >> x) & 1 for x in range(W)]], np.uint8)
            for w in range(1, 6):
                for cx in range(w):
                    se = (w, 1, cx, 0)
                    e = oracle.erode(row, se)[0]
                    d = oracle.dilate(row, se)[0]
                    for x in range(W):
                        win_e = [row[0, xx] if 0 <= xx < W else 1 for xx in range(x - cx, x + w - cx)]
                        win_d = [row[0, xx] if 0 <= xx < W else 0 for xx in range(x - (w - 1 - cx), x + cx + 1)]
                        assert e[x] == min(win_e)
                        assert d[x] == max(win_d)


def test_exhaustive_3x3_images():
    """Every 3x3 image, every element up to 3x3 with every origin: dilation is
    the union of the element placed at each black pixel; erosion is the set
    of positions where the element, placed there, lies inside A u outside."""
    for bits in range(1 << 9):
        img = np.array([(bits >> i) & 1 for i in range(9)], np.uint8).reshape(3, 3)
        for se in all_ses(3, 3):
            w, h, cx, cy = se
            want_d = np.zeros((3, 3), np.uint8)
            for py, px in zip(*np.nonzero(img)):
                for dy in range(-cy, h - cy):
                    for dx in range(-cx, w - cx):
                        y, x = py + dy, px + dx
                        if 0 <= y < 3 and 0 <= x < 3:
                            want_d[y, x] = 1
            want_e = np.zeros((3, 3), np.uint8)
            for y in range(3):
                for x in range(3):
                    ok = True
                    for dy in range(-cy, h - cy):
                        for dx in range(-cx, w - cx):
                            yy, xx = y + dy, x + dx
                            if 0 <= yy < 3 and 0 <= xx < 3 and not img[yy, xx]:
                                ok = False
                    want_e[y, x] = ok
            assert (oracle.dilate(img, se) == want_d).all(), (bits, se)
            assert (oracle.erode(img, se) == want_e).all(), (bits, se)


# --------------------------------------------------------------- closed forms
def test_single_pixel_dilation_is_the_element():
    W, H = 40, 30
    for se in [(1, 1, 0, 0), (5, 3, 2, 1), (6, 4, 0, 3), (7, 2, 6, 0), (31, 1, 15, 0), (1, 21, 0, 10)]:
        w, h, cx, cy = se
        for px, py in [(0, 0), (20, 15), (39, 29), (3, 27)]:
            img = np.zeros((H, W), np.uint8)
            img[py, px] = 1
            want = np.zeros_like(img)
            want[max(0, py - cy):min(H, py + h - cy), max(0, px - cx):min(W, px + w - cx)] = 1
            np.testing.assert_array_equal(oracle.dilate(img, se), want)


def test_rectangle_erosion_shrinks_sides():
    """An interior rectangle [x0,x1] x [y0,y1] erodes to
    [x0+cx, x1-(w-1-cx)] x [y0+cy, y1-(h-1-cy)]; a side on the image border
    does not move (outside counts as 1)."""
    W, H = 60, 50
    for se in [(5, 3, 2, 1), (4, 6, 1, 2), (7, 7, 3, 3), (2, 9, 1, 0)]:
        w, h, cx, cy = se
        img = np.zeros((H, W), np.uint8)
        img[10:40, 12:50] = 1                           # x 12..49, y 10..39
        want = np.zeros_like(img)
        want[10 + cy:40 - (h - 1 - cy), 12 + cx:50 - (w - 1 - cx)] = 1
        np.testing.assert_array_equal(oracle.erode(img, se), want)
        img = np.zeros((H, W), np.uint8)
        img[0:20, 30:W] = 1                             # touches top and right
        want = np.zeros_like(img)
        want[0:20 - (h - 1 - cy), 30 + cx:W] = 1
        np.testing.assert_array_equal(oracle.erode(img, se), want)


def test_empty_and_full():
    for se in [(3, 3, 1, 1), (8, 2, 0, 1), (1, 9, 0, 4)]:
        z = np.zeros((17, 23), np.uint8)
        o = np.ones((17, 23), np.uint8)
        for op in oracle.OPS:
            assert (oracle.apply(op, z, se) == 0).all()
            assert (oracle.apply(op, o, se) == 1).all()


def test_identity_element():
    img = rnd_img(3, 20, 33)
    for op in oracle.OPS:
        np.testing.assert_array_equal(oracle.apply(op, img, (1, 1, 0, 0)), img)


# ------------------------------------------------------------ algebraic laws
CASES = [(5, 3, 2, 1), (4, 4, 0, 3), (6, 2, 5, 0), (3, 7, 1, 6), (9, 1, 4, 0), (1, 8, 0, 4), (2, 2, 1, 1)]


@pytest.mark.parametrize("se", CASES)
def test_separability(se):
    """Rectangle = column element after row element, in either order
    (paper, sections 'Morphological Operations' and '2D Morphological
    Operators for Rectangular Masks')."""
    w, h, cx, cy = se
    img = rnd_img(11, 37, 53, 0.7)
    row, col = (w, 1, cx, 0), (1, h, 0, cy)
    for f in (oracle.erode, oracle.dilate):
        np.testing.assert_array_equal(f(img, se), f(f(img, row), col))
        np.testing.assert_array_equal(f(img, se), f(f(img, col), row))


@pytest.mark.parametrize("se", CASES)
def test_duality_with_reflected_element(se):
    """erode_B(A) = not dilate_B^(not A) and open_B(A) = not close_B^(not A)
    (dilation as complement of erosion of the complement)."""
    img = rnd_img(12, 29, 41, 0.4)
    ref = oracle.reflect(se)
    np.testing.assert_array_equal(oracle.erode(img, se), 1 - oracle.dilate(1 - img, ref))
    np.testing.assert_array_equal(oracle.dilate(img, se), 1 - oracle.erode(1 - img, ref))
    np.testing.assert_array_equal(oracle.open_(img, se), 1 - oracle.close_(1 - img, ref))


def test_composition_law():
    """Applying B1 then B2 equals applying B1 (+) B2 =
    (w1+w2-1, h1+h2-1, cx1+cx2, cy1+cy2): the basis of the doubling."""
    img = rnd_img(13, 31, 47, 0.6)
    r = np.random.default_rng(5)
    for _ in range(20):
        w1, h1, w2, h2 = (int(v) for v in r.integers(1, 7, 4))
        b1 = (w1, h1, int(r.integers(w1)), int(r.integers(h1)))
        b2 = (w2, h2, int(r.integers(w2)), int(r.integers(h2)))
        b12 = (w1 + w2 - 1, h1 + h2 - 1, b1[2] + b2[2], b1[3] + b2[3])
        for f in (oracle.erode, oracle.dilate):
            np.testing.assert_array_equal(f(f(img, b1), b2), f(img, b12))


@pytest.mark.parametrize("se", CASES)
def test_order_properties(se):
    """erode(A) <= A <= dilate(A); open(A) <= A <= close(A); opening and
    closing are idempotent; all four are increasing."""
    img = rnd_img(14, 33, 45, 0.5)
    sub = img & rnd_img(15, 33, 45, 0.8)
    e, d = oracle.erode(img, se), oracle.dilate(img, se)
    o, c = oracle.open_(img, se), oracle.close_(img, se)
    assert (e <= img).all() and (img <= d).all()
    assert (o <= img).all() and (img <= c).all()
    np.testing.assert_array_equal(oracle.open_(o, se), o)
    np.testing.assert_array_equal(oracle.close_(c, se), c)
    for op in oracle.OPS:
        assert (oracle.apply(op, sub, se) <= oracle.apply(op, img, se)).all()


# --------------------------------------------------- the independent evaluator
@pytest.mark.parametrize("op", oracle.OPS)
def test_sat_equals_brute_force(op):
    r = np.random.default_rng(21)
    for t in range(8):
        H, W = int(r.integers(1, 90)), int(r.integers(1, 200))
        img = rnd_img(200 + t, H, W, float(r.uniform(0.05, 0.95)))
        w, h = int(r.integers(1, 40)), int(r.integers(1, 40))
        se = (w, h, int(r.integers(w)), int(r.integers(h)))
        np.testing.assert_array_equal(oracle.sat_apply(op, img, se), oracle.apply(op, img, se), err_msg=str(se))


def test_sat_equals_brute_force_on_page():
    import pagegen
    img = pagegen.small_page(1000).img
    for se in [(3, 3, 1, 1), (1, 9, 0, 4), (9, 1, 4, 0), (21, 21, 10, 10)]:
        for op in oracle.OPS:
            np.testing.assert_array_equal(oracle.sat_apply(op, img, se), oracle.apply(op, img, se))


# --------------------------------------------------------------------- packing
def test_pack_matches_numpy_packbits():
    for W in (1, 63, 64, 65, 127, 128, 200, 511):
        img = rnd_img(W, 7, W)
        stride = (W + 63) // 64 + (W % 3)
        words = oracle.pack(img, stride)
        b = np.packbits(img, axis=1, bitorder="little")
        want = np.zeros((7, stride * 8), np.uint8)
        want[:, :b.shape[1]] = b
        np.testing.assert_array_equal(words, want.view("<u8"))
        np.testing.assert_array_equal(oracle.unpack(words, W), img)


def test_unpack_ignores_pad_bits():
    W = 70
    img = rnd_img(5, 4, W)
    words = oracle.pack(img, 3)
    junk = words.copy()
    junk[:, 1] |= np.uint64(0xFFFFFFFFFFFFFFC0)      # bits 70..127
    junk[:, 2] = np.uint64(0xDEADBEEFCAFEF00D)
    np.testing.assert_array_equal(oracle.unpack(junk, W), img)


# ------------------------------------------------------------ run-length form
def test_rle_round_trip_and_canonical():
    for (H, W, p) in [(1, 1, 0.5), (5, 64, 0.5), (9, 130, 0.3), (40, 77, 0.9), (3, 5, 0.0), (3, 5, 1.0)]:
        img = rnd_img(H * W, H, W, p)
        rp, runs = oracle.rle_encode(img)
        assert rp[0] == 0 and (np.diff(rp) >= 0).all()
        for y in range(H):
            rr = runs[rp[y]:rp[y + 1]]
            assert ((rr[:, 0] >= 0) & (rr[:, 0] < rr[:, 1]) & (rr[:, 1] <= W)).all()
            assert (rr[1:, 0] > rr[:-1, 1]).all()          # maximal: a gap between runs
        np.testing.assert_array_equal(oracle.rle_decode(rp, runs, W, H), img)


def test_rle_run_count_is_rising_edges():
    img = rnd_img(9, 50, 301, 0.35)
    rp, _ = oracle.rle_encode(img)
    padded = np.pad(img.astype(np.int8), ((0, 0), (1, 0)))
    rising = (np.diff(padded, axis=1) == 1).sum(axis=1)
    np.testing.assert_array_equal(np.diff(rp), rising)


def test_rle_decode_encode_identity_on_canonical():
    runs = np.array([[0, 3], [5, 6], [9, 20], [2, 4], [30, 31]], np.int32)
    rp = np.array([0, 3, 3, 5], np.int32)
    img = oracle.rle_decode(rp, runs, 31, 3)
    rp2, runs2 = oracle.rle_encode(img)
    np.testing.assert_array_equal(rp2, rp)
    np.testing.assert_array_equal(runs2, runs)


# -------------------------------------------------- values the paper states
@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_golden_transition_sink(golden):
    g = golden["transition_sink"]
    coord = {f"x{i}": 10 * (i + 1) for i in range(5)}
    sink = rle_lines.TransitionSink()
    for name, v in g["events"]:
        sink.append(coord[name], v)
    assert sink.runs == [(coord[a], coord[b]) for a, b in g["runs"]]


def test_golden_blit_count(golden):
    g = golden["blit_count_19"]
    assert logdecomp.blit_count(g["r"]) == g["blits"]
    for r in range(1, 300):
        assert logdecomp.blit_count(r) == math.ceil(math.log2(r))


def test_golden_worst_case_size(golden):
    """Alternating pixels give ceil(W/2) runs per row; two coordinates of b
    bits each per run against W bits packed and W bytes unpacked."""
    g = golden["worst_case_rle_size"]
    for W in (64, 640, 2550):
        img = np.tile(np.arange(W) % 2 == 0, (3, 1)).astype(np.uint8)
        rp, _ = oracle.rle_encode(img)
        n = int(np.diff(rp)[0])
        assert n == (W + 1) // 2
        if W % 2 == 0:
            rle_bits = n * 2 * g["bits_per_coordinate"]
            assert rle_bits == g["vs_packed"] * W
            assert rle_bits == g["vs_bytes"] * 8 * W


def test_golden_resolution_scaling(golden):
    """Scaling a page by f in both directions multiplies its rows by f while
    each row keeps its run count, so runs grow by f and packed pixels by f^2."""
    import pagegen
    g = golden["resolution_scaling"]
    f = g["factor"]
    img = pagegen.small_page(1001).img[:128, :128]
    big = np.kron(img, np.ones((f, f), np.uint8))
    rp1, _ = oracle.rle_encode(img)
    rp2, _ = oracle.rle_encode(big)
    assert rp2[-1] == g["rle_growth"] * rp1[-1]
    assert big.size == g["packed_growth"] * img.size


def _row(W, runs):
    return oracle.rle_decode(np.array([0, len(runs)], np.int32), np.array(runs, np.int32).reshape(-1, 2), W, 1)


def _runs(img):
    rp, runs = oracle.rle_encode(img)
    return [tuple(map(int, r)) for r in runs[rp[0]:rp[1]]]


def test_golden_open_close_erode_1d(golden):
    g = golden["open1d"]
    u = g["u"]
    se = (u, 1, u // 2, 0)
    assert _runs(oracle.open_(_row(g["W"], g["runs"]), se)) == [tuple(r) for r in g["open"]]
    assert rle_lines.open1d_interior([tuple(r) for r in g["runs"]], u) == [tuple(r) for r in g["open"]]
    g = golden["close1d"]
    u = g["u"]
    se = (u, 1, u // 2, 0)
    assert _runs(oracle.close_(_row(g["W"], g["runs"]), se)) == [tuple(r) for r in g["close"]]
    g = golden["erode1d_odd"]
    u = g["u"]
    se = (u, 1, u // 2, 0)
    assert _runs(oracle.erode(_row(g["W"], g["runs"]), se)) == [tuple(r) for r in g["erode"]]


# ---------------------------------- the paper's run-list algorithms vs oracle
def _all_rows(W):
    for bits in range(1 << W):
        row = np.array([[(bits >> x) & 1 for x in range(W)]], np.uint8)
        yield row, _runs(row)


def test_within_line_ops_match_oracle_exhaustively():
    for W in range(1, 9):
        for row, runs in _all_rows(W):
            for w in range(1, 6):
                for cx in range(w):
                    se = (w, 1, cx, 0)
                    assert rle_lines.erode1d(runs, w, cx, W) == _runs(oracle.erode(row, se))
                    d = _runs(oracle.dilate(row, se))
                    assert rle_lines.dilate1d(runs, w, cx, W) == d
                    assert rle_lines.dilate1d_direct(runs, w, cx, W) == d


def test_open_close_1d_delete_short_runs_away_from_border():
    """The delete-short-runs form equals the true 1-D opening (closing) when
    no run (gap) touches an end of the line."""
    for W in range(3, 10):
        for row, runs in _all_rows(W):
            for u in range(1, 6):
                se = (u, 1, u // 2, 0)
                if not (row[0, 0] or row[0, -1]):
                    assert rle_lines.open1d_interior(runs, u) == _runs(oracle.open_(row, se))
                if row[0, 0] and row[0, -1]:
                    assert rle_lines.close1d_interior(runs, u, W) == _runs(oracle.close_(row, se))


def test_line_and_or_match_pixelwise():
    r = np.random.default_rng(3)
    for _ in range(300):
        W = int(r.integers(1, 40))
        a = (r.random((1, W)) < 0.5).astype(np.uint8)
        b = (r.random((1, W)) < 0.5).astype(np.uint8)
        assert rle_lines.line_and(_runs(a), _runs(b)) == _runs(a & b)
        assert rle_lines.line_or(_runs(a), _runs(b)) == _runs(a | b)


@pytest.mark.parametrize("op", oracle.OPS)
def test_run_length_strategy_matches_oracle(op):
    """Within-line pass then log-decomposed between-line pass (the paper's
    'rle' strategy) reaches exactly the brute-force result."""
    r = np.random.default_rng(31)
    for t in range(6):
        H, W = int(r.integers(1, 25)), int(r.integers(1, 60))
        img = rnd_img(300 + t, H, W, float(r.uniform(0.2, 0.8)))
        w, h = int(r.integers(1, 12)), int(r.integers(1, 12))
        se = (w, h, int(r.integers(w)), int(r.integers(h)))
        rp, runs = oracle.rle_encode(img)
        lines = [[tuple(map(int, x)) for x in runs[rp[y]:rp[y + 1]]] for y in range(H)]
        got = rle_lines.rect_op(lines, op, se, W)
        want = oracle.apply(op, img, se)
        for y in range(H):
            assert got[y] == _runs(want[y:y + 1]), (se, y)


@pytest.mark.parametrize("op", oracle.OPS)
def test_bitblit_log_decomposition_matches_oracle(op):
    """Row pass then column pass, each by shifted AND/OR with doubling
    shifts, reaches exactly the brute-force result."""
    r = np.random.default_rng(41)
    for t in range(6):
        H, W = int(r.integers(1, 30)), int(r.integers(1, 90))
        img = rnd_img(400 + t, H, W, float(r.uniform(0.2, 0.8)))
        w, h = int(r.integers(1, 25)), int(r.integers(1, 25))
        se = (w, h, int(r.integers(w)), int(r.integers(h)))
        got = np.array(logdecomp.rect_op(img.tolist(), op, se), np.uint8).reshape(H, W)
        np.testing.assert_array_equal(got, oracle.apply(op, img, se), err_msg=str(se))


# ------------------------------------------------------------- generator pins
def test_generators_deterministic_and_in_band():
    import pagegen
    a, b = pagegen.small_page(1000), pagegen.small_page(1000)
    assert (a.img == b.img).all()
    assert 0.075 <= a.density <= 0.085
    p = pagegen.letter_page(2000)
    assert p.img.shape == (3300, 2550)
    assert 0.05 <= p.density <= 0.10
    words = p.words()
    assert words.shape == (3300, 40)
    np.testing.assert_array_equal(oracle.unpack(words, 2550), p.img)
    np.testing.assert_array_equal(oracle.pack(p.img, 40), words)


# ------------------------------------------------------------ transposition
from oracle import transpose as otr  # noqa: E402


def test_transpose_hand_example():
    """A 3 x 5 image and its 5 x 3 transpose, written out by hand."""
    rows = ["11001",
            "01101",
            "00111"]
    img = np.array([[int(c) for c in r] for r in rows], dtype=np.uint8)
    want_rows = ["100",
                 "110",
                 "011",
                 "001",
                 "111"]
    want = np.array([[int(c) for c in r] for r in want_rows], dtype=np.uint8)
    rp, runs = oracle.rle_encode(img)
    trp, truns = otr.rle_transpose(rp, runs, 5, 3)
    np.testing.assert_array_equal(oracle.rle_decode(trp, truns, 3, 5), want)
    # the runs of column 4 (row 4 of the transpose): one run over all 3 rows
    assert [tuple(r) for r in truns[trp[4]:trp[5]]] == [(0, 3)]
    assert [tuple(r) for r in truns[trp[1]:trp[2]]] == [(0, 2)]


@pytest.mark.parametrize("seed", range(6))
def test_simple_transpose_matches_decode_recode(seed):
    r = np.random.default_rng(seed)
    H, W = int(r.integers(1, 40)), int(r.integers(1, 70))
    img = rnd_img(100 + seed, H, W, float(r.choice([0.05, 0.5, 0.95])))
    rp, runs = oracle.rle_encode(img)
    want = otr.rle_transpose(rp, runs, W, H)
    got = otr.from_lines(otr.transpose_lines(otr.to_lines(rp, runs), W))
    np.testing.assert_array_equal(got[0], want[0])
    np.testing.assert_array_equal(got[1].reshape(-1, 2), want[1].reshape(-1, 2))


def test_transpose_twice_is_identity_and_degenerate_shapes():
    for H, W, p in [(1, 1, 1.0), (1, 1, 0.0), (1, 67, 0.5), (67, 1, 0.5), (64, 64, 0.5),
                    (65, 130, 0.3), (5, 5, 0.0), (5, 5, 1.0)]:
        img = rnd_img(H * 1000 + W, H, W, p)
        rp, runs = oracle.rle_encode(img)
        trp, truns = otr.rle_transpose(rp, runs, W, H)
        np.testing.assert_array_equal(oracle.rle_decode(trp, truns, H, W), img.T)
        brp, bruns = otr.rle_transpose(trp, truns, H, W)
        np.testing.assert_array_equal(brp, rp)
        np.testing.assert_array_equal(bruns.reshape(-1, 2), runs.reshape(-1, 2))


@pytest.mark.parametrize("op", oracle.OPS)
def test_transpose_composition_matches_oracle(op):
    """Within-line operations plus transposition give the rectangle
    operation (separability), including the borders."""
    r = np.random.default_rng(7)
    for k in range(12):
        H, W = int(r.integers(1, 30)), int(r.integers(1, 50))
        img = rnd_img(200 + k, H, W, float(r.choice([0.3, 0.6, 0.85])))
        w, h = int(r.integers(1, 9)), int(r.integers(1, 9))
        se = (w, h, int(r.integers(0, w)), int(r.integers(0, h)))
        rp, runs = oracle.rle_encode(img)
        grp, gruns = otr.rlet_apply(op, rp, runs, W, se)
        np.testing.assert_array_equal(oracle.rle_decode(grp, gruns, W, H), oracle.apply(op, img, se),
                                      err_msg="%s %s %dx%d" % (op, se, H, W))


# ------------------------------------------------ components and statistics
from oracle import components as occ  # noqa: E402


def _lines(img):
    return otr.to_lines(*oracle.rle_encode(img))


@pytest.mark.parametrize("conn", [4, 8])
def test_labels_match_scipy(conn):
    st = ndi.generate_binary_structure(2, 1 if conn == 4 else 2)
    for k in range(8):
        r = np.random.default_rng(300 + k)
        H, W = int(r.integers(1, 40)), int(r.integers(1, 60))
        img = rnd_img(400 + k, H, W, float(r.choice([0.2, 0.45, 0.6])))
        lines = _lines(img)
        labels, n = occ.label_runs(lines, conn)
        want, nw = ndi.label(img, structure=st)
        assert n == nw
        # scipy numbers components in raster order of their first pixel, as the oracle does
        np.testing.assert_array_equal(occ.label_image(lines, labels, W), want)


def test_connectivity_hand_example():
    """Two diagonal pixels are one component under 8-connectivity and two
    under 4; a U shape is one component either way."""
    img = np.array([[1, 0, 0, 1, 0, 1],
                    [0, 1, 0, 1, 0, 1],
                    [0, 0, 0, 1, 1, 1]], dtype=np.uint8)
    lines = _lines(img)
    assert occ.label_runs(lines, 8)[1] == 2
    assert occ.label_runs(lines, 4)[1] == 3
    labels, _ = occ.label_runs(lines, 4)
    assert labels == [[0, 1, 1], [2, 1, 1], [1]]


def test_component_stats_match_scipy():
    img = rnd_img(5, 37, 53, 0.4)
    lines = _lines(img)
    labels, n = occ.label_runs(lines, 8)
    st = occ.component_stats(lines, labels, n)
    lab, nw = ndi.label(img, structure=np.ones((3, 3)))
    assert n == nw
    for c, sl in enumerate(ndi.find_objects(lab)):
        ys, xs = np.nonzero(lab == c + 1)
        assert list(st[c, :4]) == [sl[1].start, sl[0].start, sl[1].stop, sl[0].stop]
        assert st[c, 4] == len(xs) and st[c, 5] == xs.sum() and st[c, 6] == ys.sum()


def test_run_histograms_brute_force():
    img = rnd_img(9, 30, 70, 0.5)
    img[3] = 0
    img[4] = 1
    black, white = occ.run_histograms(_lines(img), 70)
    wb, ww = np.zeros(71, np.int64), np.zeros(71, np.int64)
    for row in img:
        s = "".join(map(str, row))
        for m in __import__("re").finditer("1+", s):
            wb[len(m.group())] += 1
        for m in __import__("re").finditer("(?<=1)0+(?=1)", s):
            ww[len(m.group())] += 1
    np.testing.assert_array_equal(black, wb)
    np.testing.assert_array_equal(white, ww)
    assert black.sum() == oracle.rle_encode(img)[0][-1]


def test_histogram_percentile_against_sorted_lengths():
    r = np.random.default_rng(3)
    for _ in range(20):
        h = r.integers(0, 5, 40)
        lengths = np.repeat(np.arange(40), h)
        for num, den in [(1, 2), (9, 10), (1, 1), (1, 100)]:
            if len(lengths) == 0:
                assert occ.histogram_percentile(h, num, den) == 0
                continue
            k = -(-len(lengths) * num // den)          # ceil: the k-th smallest length
            assert occ.histogram_percentile(h, num, den) == np.sort(lengths)[k - 1]


def test_layout_boxes_two_blocks():
    """Two text blocks of 'words' (3 x 2 rectangles two pixels apart, rows of
    words five rows apart) far from each other: with the 90th percentile the
    gaps inside the blocks close and each block is one box."""
    W, H = 120, 60
    img = np.zeros((H, W), np.uint8)
    for (x0, y0) in [(5, 5), (70, 30)]:
        for row in range(3):
            for word in range(5):
                x, y = x0 + 5 * word, y0 + 5 * row
                img[y:y + 2, x:x + 3] = 1
    gx, gy, st = occ.layout_boxes([_lines(img)], W, 9, 10)
    assert gx == 2 and gy == 3
    boxes = sorted(tuple(b[:4]) for b in st[0])
    # dilating by 3 x 4 with origin (1, 2) covers [x - 1, x + 1] x [y - 1, y + 2] around each
    # pixel: a block [5, 28) x [5, 17) becomes [4, 29) x [3, 18)
    assert boxes == [(4, 3, 29, 18), (69, 28, 94, 43)]


# ----------------------------------------------------------- arbitrary masks
from oracle import masks as omask  # noqa: E402


def rnd_mask(seed, h, w, p=0.6):
    r = np.random.default_rng(seed)
    m = (r.random((h, w)) < p).astype(np.uint8)
    return m, int(r.integers(0, w)), int(r.integers(0, h))


@pytest.mark.parametrize("op", oracle.OPS)
def test_mask_ops_match_scipy(op):
    for k in range(10):
        r = np.random.default_rng(500 + k)
        img = rnd_img(600 + k, int(r.integers(1, 30)), int(r.integers(1, 40)), float(r.choice([0.3, 0.6, 0.85])))
        m, cx, cy = rnd_mask(700 + k, int(r.integers(1, 7)), int(r.integers(1, 7)))
        if not m.any():
            m[cy, cx] = 1
        h, w = m.shape
        org = (cy - h // 2, cx - w // 2)
        st = m.astype(bool)
        ero = lambda a: ndi.binary_erosion(a, st, origin=org, border_value=1)
        dil = lambda a: ndi.binary_dilation(a, st, origin=org, border_value=0)
        a = img.astype(bool)
        want = {"erode": lambda: ero(a), "dilate": lambda: dil(a),
                "open": lambda: dil(ero(a)), "close": lambda: ero(dil(a))}[op]().astype(np.uint8)
        np.testing.assert_array_equal(omask.apply(op, img, m, cx, cy), want, err_msg="%d %s" % (k, op))


def test_full_mask_is_the_rectangle_and_disc_shape():
    img = rnd_img(3, 25, 33, 0.6)
    for se in [(3, 3, 1, 1), (5, 2, 0, 1), (1, 4, 0, 3)]:
        w, h, cx, cy = se
        for op in oracle.OPS:
            np.testing.assert_array_equal(omask.apply(op, img, np.ones((h, w), np.uint8), cx, cy),
                                          oracle.apply(op, img, se))
    d, cx, cy = omask.disc(2)
    assert d.tolist() == [[0, 0, 1, 0, 0], [0, 1, 1, 1, 0], [1, 1, 1, 1, 1], [0, 1, 1, 1, 0], [0, 0, 1, 0, 0]]
    assert omask.runs_of(d, cx, cy) == [(0, -2, 1), (-1, -1, 3), (-2, 0, 5), (-1, 1, 3), (0, 2, 1)]


def test_mask_hand_example():
    """A plus sign (origin in its centre) on a 4 x 5 image, worked by hand:
    a pixel survives erosion when it and its four neighbours are black
    (outside counts black); dilation paints a plus around every black pixel."""
    plus = np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]], np.uint8)
    img = np.array([[1, 1, 1, 0, 0],
                    [1, 1, 1, 0, 0],
                    [0, 1, 1, 1, 0],
                    [0, 0, 0, 0, 0]], np.uint8)
    want_e = np.array([[1, 1, 0, 0, 0],
                       [0, 1, 0, 0, 0],
                       [0, 0, 0, 0, 0],
                       [0, 0, 0, 0, 0]], np.uint8)
    want_d = np.array([[1, 1, 1, 1, 0],
                       [1, 1, 1, 1, 0],
                       [1, 1, 1, 1, 1],
                       [0, 1, 1, 1, 0]], np.uint8)
    np.testing.assert_array_equal(omask.erode(img, plus, 1, 1), want_e)
    np.testing.assert_array_equal(omask.dilate(img, plus, 1, 1), want_d)
    empty = np.zeros((2, 2), np.uint8)
    assert omask.erode(img, empty, 0, 0).all() and not omask.dilate(img, empty, 0, 0).any()


def test_run_and_doubling_methods_match_definition():
    for k in range(12):
        r = np.random.default_rng(900 + k)
        H, W = int(r.integers(1, 25)), int(r.integers(1, 80))
        img = rnd_img(950 + k, H, W, float(r.choice([0.4, 0.7, 0.9])))
        if k < 4:
            m, cx, cy = omask.disc(int(r.integers(1, 5)))
        else:
            m, cx, cy = rnd_mask(960 + k, int(r.integers(1, 8)), int(r.integers(1, 40)))
        want = omask.erode(img, m, cx, cy)
        lines = otr.to_lines(*oracle.rle_encode(img))
        got = omask.erode_lines_by_runs(lines, m, cx, cy, W)
        np.testing.assert_array_equal(oracle.rle_decode(*otr.from_lines(got), W, H), want, err_msg=str(k))
        np.testing.assert_array_equal(omask.erode_rows_by_doubling(img, m, cx, cy), want, err_msg=str(k))


# ---------------------------------------------------------- skews, rotation
from oracle import shear as osh  # noqa: E402


def _crop(a):
    ys, xs = np.nonzero(a)
    return a[ys.min():ys.max() + 1, xs.min():xs.max() + 1]


def test_shift_rows_against_slicing_and_inverse():
    img = rnd_img(21, 17, 40, 0.5)
    for s, fill in [(0, 0), (5, 0), (-7, 1), (39, 1), (-40, 0), (60, 0)]:
        got = osh.shift_rows(img, [s] * 17, 40, fill)
        want = np.full_like(img, fill)
        if s >= 0:
            want[:, s:] = img[:, :40 - s] if s < 40 else want[:, s:]
        else:
            want[:, :40 + s] = img[:, -s:]
        np.testing.assert_array_equal(got, want, err_msg=str(s))
    sk, s = osh.skew_rows(img, 3, 7, 5)
    assert sk.shape == (17, 40 + int(s.max()))
    np.testing.assert_array_equal(osh.shift_rows(sk, -s, 40, 0), img)
    assert list(osh.skew_shifts(4, -3, 2, 1)) == [1, 0, -2, -3]        # floor division


def test_rotation_by_ninety_degrees_and_zero():
    img = np.zeros((21, 30), np.uint8)
    img[3:8, 4:20] = 1
    img[10:18, 22:25] = 1
    img[15, 2] = 1
    rot = osh.rotate(img, 1 << 16, 1 << 16, 1 << 16)   # tan 45 = 1, sin 90 = 1: exact skews
    np.testing.assert_array_equal(_crop(rot), _crop(np.rot90(img, -1)))
    np.testing.assert_array_equal(osh.rotate(img, 0, 0, 1 << 16), img)
    assert rot.sum() == img.sum()


def test_line_op_horizontal_is_the_rectangle_and_diagonal_by_hand():
    img = rnd_img(4, 25, 31, 0.7)
    for op in ("erode", "dilate"):
        np.testing.assert_array_equal(osh.line_op(op, img, 5, 0, 1), oracle.apply(op, img, (5, 1, 2, 0)))
    diag = np.zeros((9, 9), np.uint8)
    for k in range(1, 8):
        diag[k, k] = 1
    # a 3-pixel line at slope 1 (down-right): the diagonal keeps its inner pixels
    er = osh.line_op("erode", diag, 3, 1, 1)
    assert [(y, x) for y, x in zip(*np.nonzero(er))] == [(k, k) for k in range(2, 7)]
    single = np.zeros((9, 9), np.uint8)
    single[4, 4] = 1
    di = osh.line_op("dilate", single, 3, 1, 1)
    assert [(y, x) for y, x in zip(*np.nonzero(di))] == [(3, 3), (4, 4), (5, 5)]


def _rational(v, den):
    return int(round(v * den))


@pytest.mark.parametrize("angle", [0.1, -0.35, 0.7, 1.2, -1.0])
def test_rotation_general_angles_keep_pixels_and_rotate_displacements(angle):
    """Three lossless skews move every pixel within its line, so the pixel
    count is kept; and the composition of the shears x -= t y, y += s x,
    x -= t y with t = tan(a/2), s = sin(a) is the rotation by a, so the
    displacement between two single pixels turns by a.  Each skew floors
    once: a position is off by at most 1 after the first skew, 1 + |s| after
    the second and 2 + |t| (1 + |s|) after the third, twice that for a
    displacement."""
    den = 1 << 16
    tn, sn = _rational(math.tan(angle / 2), den), _rational(math.sin(angle), den)
    img = rnd_img(31, 40, 57, 0.3)
    rot = osh.rotate(img, tn, sn, den)
    assert rot.sum() == img.sum()
    t, s = tn / den, sn / den
    bx, by = 2 * (2 + abs(t) * (1 + abs(s))), 2 * (1 + abs(s))
    H, W = 40, 57
    rng = np.random.default_rng(5)

    def where(y, x):
        one = np.zeros((H, W), np.uint8)
        one[y, x] = 1
        r = osh.rotate(one, tn, sn, den)
        assert r.shape == rot.shape and r.sum() == 1
        ys, xs = np.nonzero(r)
        return int(ys[0]), int(xs[0])
    for _ in range(12):
        (y0, x0), (y1, x1) = [(int(rng.integers(H)), int(rng.integers(W))) for _ in range(2)]
        p0, p1 = where(y0, x0), where(y1, x1)
        dx, dy = x1 - x0, y1 - y0
        ex = math.cos(angle) * dx - math.sin(angle) * dy
        ey = math.sin(angle) * dx + math.cos(angle) * dy
        assert abs((p1[1] - p0[1]) - ex) <= bx and abs((p1[0] - p0[0]) - ey) <= by, \
            (angle, (y0, x0), (y1, x1), p0, p1, ex, ey)


def test_rotation_inverse_angle_returns_the_image():
    """Rotating by a and then by -a undoes the rotation up to the frame: the
    pixel count is kept and the shape comes back after cropping, for exact
    (a = 90 degrees) skews."""
    den = 1 << 16
    img = np.zeros((15, 22), np.uint8)
    img[2:6, 3:17] = 1
    img[9:13, 18:20] = 1
    fwd = osh.rotate(img, den, den, den)
    back = osh.rotate(fwd, -den, -den, den)
    np.testing.assert_array_equal(_crop(back), _crop(img))


def test_line_op_slope_half_by_hand():
    """A 3-pixel line at slope 1/2 (columns x move by -floor(x / 2)): the
    digital line through (x=3, y=2) covers (2, 2), (3, 2) and (4, 3), so a
    single pixel dilates to those three, and eroding those three keeps only
    the centre (worked through the skew, the horizontal operation with
    origin 1 and the skew back)."""
    single = np.zeros((6, 8), np.uint8)
    single[2, 3] = 1
    di = osh.line_op("dilate", single, 3, 1, 2)
    assert sorted((int(x), int(y)) for y, x in zip(*np.nonzero(di))) == [(2, 2), (3, 2), (4, 3)]
    er = osh.line_op("erode", di, 3, 1, 2)
    assert [(int(x), int(y)) for y, x in zip(*np.nonzero(er))] == [(3, 2)]
