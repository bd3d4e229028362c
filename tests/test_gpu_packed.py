"""GPU parity of the packed path (C-ABI entry points via the binding) against
the CPU oracle: bit-exact on every word of every row, including pad bits
(which must come out 0) and words past the row (which must be untouched)."""
import numpy as np
import pytest
import torch

import oracle
import pagegen
from gpu_util import blobs_img, expected_words, garbage_pad, require_gpu, rnd_img

pytestmark = pytest.mark.gpu

M = None


@pytest.fixture(scope="module", autouse=True)
def lib():
    require_gpu()
    global M
    import paper_0712_0121_amd as m
    M = m
    return m


def run_packed(op, img, se, stride=None, seed=0, npages=1):
    """img: (npages*H, W) bytes.  Returns the output words (rows, stride)."""
    rows, W = img.shape
    nw = (W + 63) // 64
    stride = nw if stride is None else stride
    words = garbage_pad(oracle.pack(img, stride), W, seed)
    src = M.Bitmap.from_words(words, W, npages=npages)
    sentinel = np.full((rows, stride), 0x5A5A5A5A5A5A5A5A, np.uint64)
    dst = M.Bitmap.from_words(sentinel, W, npages=npages)
    ws_n = M.morph_workspace_bytes(op, 0, W, rows, se)
    ws = torch.empty(max(ws_n, 1), dtype=torch.uint8, device="cuda") if ws_n else None
    M.PACKED[op](dst, src, se, ws)
    torch.cuda.synchronize()
    out = dst.to_numpy()
    if stride > nw:
        assert (out[:, nw:] == np.uint64(0x5A5A5A5A5A5A5A5A)).all(), "words past the row were written"
    return out[:, :nw]


def check(op, img, se, stride=None, seed=0, method="brute"):
    got = run_packed(op, img, se, stride, seed)
    want = expected_words(op, img, se, method=method)
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        y, j = bad[0]
        raise AssertionError("%s se=%s shape=%s: %d words differ, first at row %d word %d: got %x want %x"
                             % (op, se, img.shape, len(bad), y, j, got[y, j], want[y, j]))


# ------------------------------------------------------------- small page
SMALL_SES = [(3, 3, 1, 1), (1, 9, 0, 4), (9, 1, 4, 0)]


@pytest.mark.parametrize("op", pagegen.OPS)
@pytest.mark.parametrize("se", SMALL_SES)
def test_small_page(op, se):
    """512 x 512 page, ~8% black: dilate/erode (and open/close) by 3x3, 9x1
    and 1x9, centred origin."""
    img = pagegen.small_page(1000).img
    check(op, img, se)


# ------------------------------------------------------------------- fuzz
def fuzz_cases(n, seed):
    r = np.random.default_rng(seed)
    for i in range(n):
        W = int(r.choice([1, 2, 63, 64, 65, 127, 128, 129, 191, 200, 256, 320, 449, 512, 640, 700,
                          int(r.integers(1, 701))]))
        H = int(r.integers(1, 301))
        w = int(r.choice([1, 2, 3, 31, 32, 33, 63, 64, 65, 127, 128, 129, int(r.integers(1, 131))]))
        h = int(r.choice([1, 2, 3, 16, 17, 33, 64, int(r.integers(1, 131))]))
        cx = int(r.integers(w)) if r.random() < 0.7 else w // 2
        cy = int(r.integers(h)) if r.random() < 0.7 else h // 2
        op = pagegen.OPS[i % 4]
        stride = (W + 63) // 64 + int(r.integers(0, 3))
        yield i, W, H, (w, h, cx, cy), op, stride


@pytest.mark.parametrize("case", list(fuzz_cases(48, 77)), ids=lambda c: "c%d" % c[0])
def test_fuzz_against_oracle(case):
    i, W, H, se, op, stride = case
    img = blobs_img(1000 + i, H, W, density=float(np.random.default_rng(i).uniform(0.05, 0.6)))
    check(op, img, se, stride=stride, seed=i, method="sat")


@pytest.mark.parametrize("W", [64, 65, 127, 128, 129, 4097])
def test_word_boundaries(W):
    img = rnd_img(W, 37, W, 0.6)
    for op in pagegen.OPS:
        for se in [(1, 1, 0, 0), (2, 1, 1, 0), (65, 1, 0, 0), (65, 1, 64, 0), (129, 3, 64, 1), (64, 2, 63, 0)]:
            check(op, img, se, method="sat")


def test_degenerate_images():
    for (H, W) in [(1, 1), (1, 70), (70, 1), (2, 2)]:
        for p in (0.0, 1.0, 0.5):
            img = rnd_img(H * W, H, W, p)
            for op in pagegen.OPS:
                for se in [(1, 1, 0, 0), (3, 3, 1, 1), (5, 2, 0, 1), (40, 40, 20, 20)]:
                    check(op, img, se)


def test_large_elements_decomposed():
    """Elements beyond one launch's reach (origin more than 64 px from a
    side, or taller than one tile) run as several launches through the
    workspace; the composition law keeps the result exact."""
    img = blobs_img(5, 260, 900, 0.4)
    for op in pagegen.OPS:
        for se in [(200, 3, 100, 1), (140, 1, 0, 0), (130, 1, 129, 0), (1, 300, 0, 150), (301, 301, 10, 290)]:
            check(op, img, se, method="sat")


def test_stacked_pages_have_own_borders():
    H, W, P = 57, 300, 3
    imgs = [blobs_img(40 + k, H, W, 0.5) for k in range(P)]
    img = np.concatenate(imgs, axis=0)
    for op in pagegen.OPS:
        for se in [(5, 7, 2, 3), (33, 21, 30, 1)]:
            got = run_packed(op, img, se, npages=P)
            want = np.concatenate([expected_words(op, im, se) for im in imgs], axis=0)
            np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("H", [1, 3, 7, 30, 80])
def test_stacked_short_pages_fused_or_split(H):
    """Openings and closings on stacks of short pages, with the workspace
    sized from the stack's total rows as the binding does: whether the two
    stages share a tile must not depend on the page height (pages under 8
    rows, a 21 x 21 element whose 40 halo rows exceed 30-row pages, a
    51 x 51 element split into two launches on any page)."""
    W, P = 150, 6
    imgs = [rnd_img(700 + 10 * H + k, H, W, 0.4) for k in range(P)]
    img = np.concatenate(imgs, axis=0)
    for op in ("open", "close"):
        for se in [(3, 3, 1, 1), (21, 21, 10, 10), (51, 51, 25, 25), (2, 9, 1, 8)]:
            got = run_packed(op, img, se, npages=P)
            want = np.concatenate([expected_words(op, im, se) for im in imgs], axis=0)
            np.testing.assert_array_equal(got, want, err_msg="%s %s H=%d" % (op, se, H))
            src = M.Bitmap.from_words(oracle.pack(img), W, npages=P)
            out = M.rect_packed(op, src, se)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out.to_numpy(), want, err_msg="binding %s %s H=%d" % (op, se, H))


# ------------------------------------------------------------ full letter page
LETTER_SES = [(31, 1, 15, 0), (1, 31, 0, 15), (3, 3, 1, 1), (21, 21, 10, 10), (51, 51, 25, 25)]


@pytest.fixture(scope="module")
def letter():
    return pagegen.letter_page(2000).img


@pytest.mark.parametrize("op", pagegen.OPS)
@pytest.mark.parametrize("se", LETTER_SES, ids=["1x31", "31x1", "3x3", "21x21", "51x51"])
def test_letter_page(letter, op, se):
    """2550 x 3300 letter page (40 words per row), every element of the
    letter-page workload, against the summed-area evaluator (itself pinned to
    brute force)."""
    check(op, letter, se, method="sat")


def test_letter_page_sampled_brute_force(letter):
    """At full size, erosion and dilation by 51x51 on sampled pixels against
    the brute-force definition evaluated one pixel at a time."""
    se = (51, 51, 25, 25)
    r = np.random.default_rng(9)
    ys = r.integers(0, letter.shape[0], 400)
    xs = r.integers(0, letter.shape[1], 400)
    ys = np.concatenate([ys, [0, 3299, 0, 3299, 17]])
    xs = np.concatenate([xs, [0, 0, 2549, 2549, 2549]])
    for op in ("erode", "dilate"):
        got = oracle.unpack(run_packed(op, letter, se), letter.shape[1])
        for y, x in zip(ys, xs):
            if op == "erode":
                win = letter[max(0, y - 25):y + 26, max(0, x - 25):x + 26]
                want = int(win.min()) if win.size else 1
            else:
                win = letter[max(0, y - 25):y + 26, max(0, x - 25):x + 26]
                want = int(win.max())
            assert got[y, x] == want, (op, y, x)


def test_repeatable_and_tiling_independent(letter):
    """Same result on repeated runs (no races in LDS)."""
    se = (21, 21, 10, 10)
    a = run_packed("open", letter, se)
    for _ in range(3):
        np.testing.assert_array_equal(run_packed("open", letter, se), a)


@pytest.mark.parametrize("H", [199, 220, 221, 232, 240, 241, 461])
def test_tile_row_boundaries(H):
    """Letter-width pages whose heights fall just under, on and over the
    rows of one tile (220 output rows for a two-stage 3 x 3 tile, 240 for
    a one-stage one, halo rows included or not): every band edge and the
    last, shorter band meet the oracle."""
    img = blobs_img(8000 + H, H, 2550, 0.3)
    for op in pagegen.OPS:
        for se in [(3, 3, 1, 1), (21, 21, 10, 10), (1, 31, 0, 15), (51, 51, 25, 25)]:
            check(op, img, se, method="sat")
