"""GPU parity of transposition and of the transpose-based rectangle
operations ("rlet") against the oracle: transposed words must equal the
packed transpose of the image bit for bit, and run-length results must equal
the oracle's canonical encoding exactly."""
import numpy as np
import pytest
import torch

import oracle
import pagegen
from gpu_util import blobs_img, garbage_pad, require_gpu, rnd_img
from oracle import transpose as otr

pytestmark = pytest.mark.gpu

M = None


@pytest.fixture(scope="module", autouse=True)
def lib():
    require_gpu()
    global M
    import paper_0712_0121_amd as m
    M = m
    return m


SIZES = [(1, 1), (1, 130), (130, 1), (63, 64), (64, 64), (65, 65), (127, 129), (200, 77), (64, 4097)]


def bitmap_gpu(img, npages=1, extra_stride=1, seed=0):
    rows, W = img.shape
    words = garbage_pad(oracle.pack(img, (W + 63) // 64 + extra_stride), W, seed)
    return M.Bitmap.from_words(words, W, npages=npages)


def rle_gpu(img, npages=1):
    return M.pack_to_rle(bitmap_gpu(img, npages))


def assert_rle(got, want_rp, want_runs, what=""):
    rp, runs = got.to_host()
    if not np.array_equal(rp, want_rp):
        y = int(np.argmax(rp != want_rp))
        raise AssertionError("%s: row_ptr differs first at %d: %d vs %d" % (what, y, rp[y], want_rp[y]))
    np.testing.assert_array_equal(runs.reshape(-1, 2), np.asarray(want_runs).reshape(-1, 2), err_msg=what)


# ------------------------------------------------------------------ packed
@pytest.mark.parametrize("hw", SIZES, ids=lambda s: "%dx%d" % s)
def test_transpose_packed(hw):
    H, W = hw
    for p in (0.0, 0.5, 1.0):
        img = rnd_img(H * 7 + W + int(p * 10), H, W, p)
        got = M.transpose_packed(bitmap_gpu(img, seed=W))
        torch.cuda.synchronize()
        assert (got.width, got.height) == (H, W)
        np.testing.assert_array_equal(got.to_numpy(), oracle.pack(np.ascontiguousarray(img.T)),
                                      err_msg="%dx%d p=%g" % (H, W, p))


def test_transpose_packed_stacked_pages_and_letter_page():
    H, W, P = 70, 90, 3
    imgs = [blobs_img(30 + k, H, W, 0.4) for k in range(P)]
    got = M.transpose_packed(bitmap_gpu(np.concatenate(imgs), npages=P)).to_numpy()
    want = np.concatenate([oracle.pack(np.ascontiguousarray(im.T)) for im in imgs])
    np.testing.assert_array_equal(got, want)
    img = pagegen.letter_page(2000).img
    src = bitmap_gpu(img, extra_stride=0)
    t = M.transpose_packed(src)
    back = M.transpose_packed(t)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(t.to_numpy(), oracle.pack(np.ascontiguousarray(img.T)))
    np.testing.assert_array_equal(back.to_numpy(), oracle.pack(img))


# -------------------------------------------------------------- run-length
# and for the runs: columns of several 512-row tiles (a multiple of 64 tall,
# so that a column black to the bottom ends past the last block), rows of
# more than 128 words (decoded straight into the transposed bitmap)
RLE_SIZES = SIZES + [(1024, 70), (1100, 600), (513, 3), (20, 9000)]


@pytest.mark.parametrize("hw", RLE_SIZES, ids=lambda s: "%dx%d" % s)
def test_transpose_rle(hw):
    H, W = hw
    for p in (0.0, 0.3, 0.9, 1.0):
        img = blobs_img(H + 3 * W + int(p * 10), H, W, p) if 0 < p < 1 else rnd_img(1, H, W, p)
        rp, runs = oracle.rle_encode(img)
        got = M.transpose_rle(rle_gpu(img))
        torch.cuda.synchronize()
        assert (got.width, got.height) == (H, W)
        wrp, wruns = otr.rle_transpose(rp, runs, W, H)
        assert_rle(got, wrp, wruns, "%dx%d p=%g" % (H, W, p))


def test_transpose_rle_stacked_and_letter():
    H, W, P = 45, 300, 4
    imgs = [blobs_img(90 + k, H, W, 0.5) for k in range(P)]
    got = M.transpose_rle(rle_gpu(np.concatenate(imgs), npages=P))
    want = np.concatenate([np.ascontiguousarray(im.T) for im in imgs])
    wrp, wruns = oracle.rle_encode(want)
    assert_rle(got, wrp, wruns, "stacked")
    img = pagegen.letter_page(2001).img
    r = rle_gpu(img)
    t = M.transpose_rle(r)
    back = M.transpose_rle(t)
    rp, runs = oracle.rle_encode(img)
    wrp, wruns = otr.rle_transpose(rp, runs, img.shape[1], img.shape[0])
    assert_rle(t, wrp, wruns, "letter")
    assert_rle(back, rp, runs, "letter twice")


# --------------------------------------------------------------- rlet ops
def rlet(op, img, se, npages=1):
    out = M.rect_rlet(op, rle_gpu(img, npages), se)
    torch.cuda.synchronize()
    return out


def assert_img(got, img, what=""):
    wrp, wruns = oracle.rle_encode(img)
    assert_rle(got, wrp, wruns, what)


@pytest.mark.parametrize("op", pagegen.OPS)
@pytest.mark.parametrize("se", [(3, 3, 1, 1), (1, 9, 0, 4), (9, 1, 4, 0), (4, 6, 0, 5), (2, 2, 1, 0),
                                (1, 1, 0, 0)])
def test_rlet_small_page(op, se):
    img = pagegen.small_page(1000).img
    assert_img(rlet(op, img, se), oracle.apply(op, img, se), "%s %s" % (op, se))


def rlet_fuzz(n, seed):
    r = np.random.default_rng(seed)
    for i in range(n):
        W = int(r.choice([1, 2, 64, 65, 200, int(r.integers(1, 500))]))
        H = int(r.integers(1, 150))
        w, h = int(r.integers(1, 90)), int(r.integers(1, 90))
        yield i, W, H, (w, h, int(r.integers(w)), int(r.integers(h))), pagegen.OPS[i % 4]


@pytest.mark.parametrize("case", list(rlet_fuzz(40, 17)), ids=lambda c: "c%d" % c[0])
def test_rlet_fuzz(case):
    i, W, H, se, op = case
    img = blobs_img(700 + i, H, W, float(np.random.default_rng(i).uniform(0.05, 0.8)))
    assert_img(rlet(op, img, se), oracle.sat_apply(op, img, se), str(case))


@pytest.mark.parametrize("op", pagegen.OPS)
def test_rlet_letter_page(op):
    img = pagegen.letter_page(2000).img
    for se in [(31, 1, 15, 0), (1, 31, 0, 15), (3, 3, 1, 1), (21, 21, 10, 10), (51, 51, 25, 25)]:
        assert_img(rlet(op, img, se), oracle.sat_apply(op, img, se), "%s %s" % (op, se))


def test_rlet_stacked_empty_full_and_alternating():
    H, W, P = 40, 333, 4
    imgs = [blobs_img(170 + k, H, W, 0.45) for k in range(P)]
    for op in pagegen.OPS:
        se = (7, 9, 3, 2)
        want = np.concatenate([oracle.apply(op, im, se) for im in imgs])
        assert_img(rlet(op, np.concatenate(imgs), se, npages=P), want, "stacked " + op)
    for p in (0.0, 1.0):
        img = rnd_img(1, 30, 130, p)
        for op in pagegen.OPS:
            assert_img(rlet(op, img, (5, 5, 2, 2)), oracle.apply(op, img, (5, 5, 2, 2)), "%s p=%g" % (op, p))
    W, H = 700, 24
    img = np.tile((np.arange(W) % 2 == 0).astype(np.uint8), (H, 1))
    img[::3] ^= 1
    for op in pagegen.OPS:
        for se in [(2, 2, 0, 1), (1, 5, 0, 2), (3, 1, 1, 0)]:
            assert_img(rlet(op, img, se), oracle.apply(op, img, se), "alternating %s %s" % (op, se))


def test_rlet_matches_paper_composition_exactly():
    """The GPU composition (two transpositions for opening and closing) against
    the oracle's step-by-step composition (four), on a small page."""
    img = blobs_img(5, 37, 91, 0.5)
    rp, runs = oracle.rle_encode(img)
    for op in pagegen.OPS:
        se = (6, 5, 4, 1)
        wrp, wruns = otr.rlet_apply(op, rp, runs, 91, se)
        assert_rle(rlet(op, img, se), wrp, wruns, op)


def test_trace_names_the_transpose_kernels():
    img = blobs_img(9, 100, 300, 0.4)
    src = rle_gpu(img)
    torch.cuda.synchronize()
    with M.Trace() as tr:
        M.rect_rlet("erode", src, (3, 3, 1, 1))
        M.transpose_packed(bitmap_gpu(img))
    res = tr.result
    assert res["decode_transpose_kernel"]["launches"] == 2
    # rows of up to 128 words are decoded in their own orientation, and the
    # transpose of that bitmap comes with its rows' run counts, from which the
    # runs are encoded: one traced conversion each way (the traced bit-block
    # transpose is the direct call)
    assert res["transpose_kernel"]["launches"] == 1
    assert res["transpose_to_rle"]["launches"] == 2
    assert "pack_to_rle_kernel" not in res
    n = int(src.nruns())
    # algorithmic bytes of the first decode: the runs and row counts read,
    # the page's words written (5 words x 100 rows)
    assert res["decode_transpose_kernel"]["bytes"] >= 8 * n + 8 * 5 * 100


@pytest.mark.parametrize("op", pagegen.OPS)
def test_rlet_letter_batch_as_timed(op):
    """The benchmark's batch: 256 stacked 2550 x 3300 letter pages (16
    distinct, replicated), one call per operation, as the benchmark times
    it.  The 16 distinct pages are checked whole against the oracle's
    summed-area evaluator, every replica's row counts against its original;
    the packed and run-length transposes of the batch are checked by
    transposing back."""
    B, D = 256, 16
    pool = [pagegen.letter_page(2000 + i) for i in range(D)]
    W, H = 2550, 3300
    host = np.concatenate([pool[i % D].words() for i in range(B)])
    src = M.Bitmap.from_words(host, W, npages=B)
    del host
    r_in = M.pack_to_rle(src)
    se = (21, 21, 10, 10) if op in ("erode", "open") else (1, 31, 0, 15)
    out = M.rect_rlet(op, r_in, se)
    back = M.rle_to_pack(out).to_numpy().reshape(B, H, -1)
    torch.cuda.synchronize()
    for i in range(D):
        want = oracle.pack(oracle.sat_apply(op, pool[i].img, se))
        np.testing.assert_array_equal(back[i], want, err_msg="%s %s page %d" % (op, se, i))
    counts = np.diff(out.row_ptr.cpu().numpy()).reshape(B, H)
    for i in range(D, B):
        np.testing.assert_array_equal(counts[i], counts[i % D], err_msg="replica %d" % i)
    del back, out
    if op == "erode":
        t = M.transpose_packed(src)
        tb = M.transpose_packed(t)
        torch.cuda.synchronize()
        assert torch.equal(tb.words, M.rle_to_pack(r_in).words)
        np.testing.assert_array_equal(t.to_numpy()[:W], oracle.pack(np.ascontiguousarray(pool[0].img.T)))
        del t, tb
        rt = M.transpose_rle(r_in)
        rb = M.transpose_rle(rt)
        torch.cuda.synchronize()
        assert torch.equal(rb.row_ptr, r_in.row_ptr)
        n = int(r_in.row_ptr[-1].item())
        assert torch.equal(rb.runs[:n], r_in.runs[:n])


def test_strategy_tuner_times_both_and_both_agree(tmp_path):
    """The autotuner's choice between the two strategies on runs: it times
    both on a run-length stack and records the faster per (op, width
    bucket, height bucket); both strategies give the same runs."""
    from paper_0712_0121_amd.tune import Tuner, strategy_key
    pages = [pagegen.letter_page(2000 + i).img for i in range(4)]
    img = np.concatenate(pages)
    W, H = 2550, 3300
    src = M.pack_to_rle(M.Bitmap.from_words(oracle.pack(img), W, npages=4))
    cases = [("close", (1, 31, 0, 15)), ("erode", (31, 1, 15, 0))]
    t = Tuner(cache_path=str(tmp_path / "t.json"))
    tab = t.tune_strategy(src, cases)
    for op, se in cases:
        v = tab[strategy_key(op, se)]
        assert v["lines_ms"] > 0 and v["transpose_ms"] > 0 and v["best"] in ("lines", "transpose")
        a = M.rect_rle(op, src, se)
        b = M.rect_rlet(op, src, se)
        torch.cuda.synchronize()
        ra, ua = a.to_host()
        rb, ub = b.to_host()
        np.testing.assert_array_equal(ra, rb)
        np.testing.assert_array_equal(ua, ub)
