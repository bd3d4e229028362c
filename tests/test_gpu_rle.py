"""GPU parity of conversion and of the run-length path against the oracle:
row_ptr and runs must equal the oracle's canonical encoding exactly."""
import numpy as np
import pytest
import torch

import oracle
import pagegen
from gpu_util import blobs_img, garbage_pad, require_gpu, rnd_img

pytestmark = pytest.mark.gpu

M = None


@pytest.fixture(scope="module", autouse=True)
def lib():
    require_gpu()
    global M
    import paper_0712_0121_amd as m
    M = m
    return m


def to_rle_gpu(img, npages=1, stride=None, seed=0, capacity=None):
    rows, W = img.shape
    words = garbage_pad(oracle.pack(img, stride), W, seed)
    src = M.Bitmap.from_words(words, W, npages=npages)
    return M.pack_to_rle(src, capacity=capacity)


def assert_rle_equal(got: "M.RLE", img, what=""):
    rp, runs = got.to_host()
    wrp, wruns = oracle.rle_encode(img)
    if not np.array_equal(rp, wrp):
        y = int(np.argmax(rp != wrp))
        raise AssertionError("%s: row_ptr differs first at %d: %d vs %d" % (what, y, rp[y], wrp[y]))
    np.testing.assert_array_equal(runs, wruns, err_msg=what)


# --------------------------------------------------------------- conversion
@pytest.mark.parametrize("W", [1, 5, 63, 64, 65, 128, 129, 2550, 4096, 4097, 5100, 8192, 8193, 10000])
def test_pack_to_rle_matches_oracle(W):
    """Rows of up to 128 words take one 16-lane group each, wider rows a
    wave each: widths on both sides of 8192 pixels."""
    H = 23
    for p in (0.0, 0.02, 0.5, 0.97, 1.0):
        img = rnd_img(int(W * 10 + p * 100), H, W, p)
        stride = (W + 63) // 64 + 1
        assert_rle_equal(to_rle_gpu(img, stride=stride, seed=W), img, "W=%d p=%g" % (W, p))


@pytest.mark.parametrize("H", [2047, 2048, 2049, 8191, 8192, 8193])
def test_row_offsets_around_scan_limits(H):
    """row_ptr is the prefix sum of the row counts: up to 8192 rows it is
    computed by one workgroup in blocks of 2048, beyond that by three
    launches; row counts on both sides of both limits."""
    img = rnd_img(H, H, 70, 0.3)
    assert_rle_equal(to_rle_gpu(img), img, "H=%d" % H)


def test_alternating_pixels_worst_case():
    W, H = 2550, 9
    img = np.tile((np.arange(W) % 2 == 0).astype(np.uint8), (H, 1))
    r = to_rle_gpu(img)
    assert r.nruns() == H * ((W + 1) // 2) == M.morph_rle_max_runs(W, H)
    assert_rle_equal(r, img)


def test_pack_to_rle_capacity_overflow_reports_total():
    img = rnd_img(3, 40, 300, 0.5)
    wrp, wruns = oracle.rle_encode(img)
    cap = int(wrp[-1]) // 2
    r = to_rle_gpu(img, capacity=cap)
    rp = r.row_ptr.cpu().numpy()
    np.testing.assert_array_equal(rp, wrp)                     # true counts
    np.testing.assert_array_equal(r.runs[:cap].cpu().numpy(), wruns[:cap])


@pytest.mark.parametrize("W", [1, 64, 65, 700, 2550, 5100, 8192, 8193, 10000])
def test_rle_to_pack_round_trip(W):
    img = blobs_img(W, 31, W, 0.4)
    r = to_rle_gpu(img)
    b = M.rle_to_pack(r, stride=(W + 63) // 64 + 2)
    torch.cuda.synchronize()
    words = b.to_numpy()[:, : (W + 63) // 64]
    np.testing.assert_array_equal(words, oracle.pack(img))


def test_density_pages_round_trip():
    for d in (0.01, 0.10, 0.40):
        pg = pagegen.density_page(d, 4000)
        r = to_rle_gpu(pg.img)
        assert_rle_equal(r, pg.img, "density %g" % d)
        b = M.rle_to_pack(r)
        np.testing.assert_array_equal(b.to_numpy(), oracle.pack(pg.img))


def test_validate():
    img = blobs_img(8, 20, 100, 0.5)
    r = to_rle_gpu(img)
    assert M.morph_rle_validate(r) == 0
    rp, runs = oracle.rle_encode(img)
    bad = runs.copy()
    k = int(np.argmax(np.diff(rp) >= 2))
    j = int(rp[k])
    bad[j + 1, 0] = bad[j, 1]            # touching runs: not canonical
    rb = M.RLE.from_host(rp, bad, 100, 20)
    assert M.morph_rle_validate(rb) == -5


# ----------------------------------------------------------- run-length ops
def rle_op(op, img, se, npages=1):
    src = to_rle_gpu(img, npages=npages)
    out = M.rect_rle(op, src, se)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("op", pagegen.OPS)
@pytest.mark.parametrize("se", [(3, 3, 1, 1), (1, 9, 0, 4), (9, 1, 4, 0), (4, 6, 0, 5), (2, 2, 1, 0)])
def test_rle_small_page(op, se):
    img = pagegen.small_page(1000).img
    assert_rle_equal(rle_op(op, img, se), oracle.apply(op, img, se), "%s %s" % (op, se))


def rle_fuzz(n, seed):
    r = np.random.default_rng(seed)
    for i in range(n):
        W = int(r.choice([1, 2, 64, 65, 200, int(r.integers(1, 500))]))
        H = int(r.integers(1, 120))
        w, h = int(r.integers(1, 70)), int(r.integers(1, 70))
        yield i, W, H, (w, h, int(r.integers(w)), int(r.integers(h))), pagegen.OPS[i % 4]


@pytest.mark.parametrize("case", list(rle_fuzz(40, 5)), ids=lambda c: "c%d" % c[0])
def test_rle_fuzz(case):
    i, W, H, se, op = case
    img = blobs_img(500 + i, H, W, float(np.random.default_rng(i).uniform(0.05, 0.7)))
    assert_rle_equal(rle_op(op, img, se), oracle.sat_apply(op, img, se), str(case))


@pytest.mark.parametrize("density", [0.01, 0.10, 0.40])
@pytest.mark.parametrize("op", ["erode", "dilate"])
@pytest.mark.parametrize("se", [(41, 1, 20, 0), (1, 41, 0, 20)], ids=["1x41", "41x1"])
def test_rle_density_sweep(density, op, se):
    """2550 x 3300 pages at 1%, 10%, 40% black, horizontal 1x41 and vertical
    41x1 erosion and dilation on runs, compared with the oracle and with the
    packed path on the same page."""
    img = pagegen.density_page(density, 4000).img
    want = oracle.sat_apply(op, img, se)
    out = rle_op(op, img, se)
    assert_rle_equal(out, want, "%s %s %g" % (op, se, density))
    # RLE result == pack_to_rle(packed result), through rle_to_pack as well
    b = M.rle_to_pack(out)
    src = M.Bitmap.from_words(oracle.pack(img), img.shape[1])
    pk = M.rect_packed(op, src, se)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(b.to_numpy(), pk.to_numpy())


@pytest.mark.parametrize("op", pagegen.OPS)
def test_rle_letter_page(op):
    img = pagegen.letter_page(2000).img
    for se in [(31, 1, 15, 0), (1, 31, 0, 15), (3, 3, 1, 1), (21, 21, 10, 10), (51, 51, 25, 25)]:
        assert_rle_equal(rle_op(op, img, se), oracle.sat_apply(op, img, se), "%s %s" % (op, se))


def test_rle_stacked_pages():
    H, W, P = 40, 333, 4
    imgs = [blobs_img(70 + k, H, W, 0.45) for k in range(P)]
    img = np.concatenate(imgs)
    for op in pagegen.OPS:
        se = (7, 9, 3, 2)
        out = rle_op(op, img, se, npages=P)
        want = np.concatenate([oracle.apply(op, im, se) for im in imgs])
        assert_rle_equal(out, want, op)


def test_rle_empty_and_full():
    for p in (0.0, 1.0):
        img = rnd_img(1, 30, 130, p)
        for op in pagegen.OPS:
            assert_rle_equal(rle_op(op, img, (5, 5, 2, 2)), oracle.apply(op, img, (5, 5, 2, 2)))


def test_trace_counts_launches_and_bytes():
    """Tracing: rect_kernel bytes are one read and one write of the page;
    pack_to_rle counts exactly the runs it wrote."""
    img = pagegen.small_page(1001).img
    W, H = img.shape[1], img.shape[0]
    src = M.Bitmap.from_words(oracle.pack(img), W)
    with M.Trace() as tr:
        M.rect_packed("erode", src, (3, 3, 1, 1))
        r = M.pack_to_rle(src)
        M.rect_rle("dilate", r, (5, 5, 2, 2))
    res = tr.result
    assert res["rect_kernel"]["launches"] == 1
    assert res["rect_kernel"]["bytes"] == 16 * 8 * H
    assert res["rect_kernel"]["ms"] > 0
    n = int(oracle.rle_encode(img)[0][-1])
    assert res["pack_to_rle_kernel"]["bytes"] == 8 * 8 * H + 4 * (H + 1) + 8 * n
    # offsets 1, 2, then 1; the within-line pass runs inside the first of them
    assert res["col_and_kernel"]["launches"] == 3
    assert res.get("row_erode_kernel", {"launches": 0})["launches"] == 0
    assert res["pack_rows_kernel"]["launches"] == 1
    with M.Trace() as tr:
        M.rect_rle("erode", r, (7, 1, 3, 0))                 # one row: the within-line pass alone
    assert tr.result["row_erode_kernel"]["launches"] == 1
    assert tr.result.get("col_and_kernel", {"launches": 0})["launches"] == 0


@pytest.mark.parametrize("op", pagegen.OPS)
def test_letter_batch_as_timed(op):
    """The timed letter workload itself: 256 stacked 2550 x 3300 pages (16
    distinct, replicated) in one launch per operation, on both paths, with
    one vertical and one square element.  The 16 distinct pages are checked
    whole against the oracle's summed-area evaluator, the replicas against
    them, and bitmap -> runs -> bitmap must give back the packed result."""
    B, D = 256, 16
    pool = [pagegen.letter_page(2000 + i) for i in range(D)]
    W, H = 2550, 3300
    host = np.concatenate([pool[i % D].words() for i in range(B)])
    src = M.Bitmap.from_words(host, W, npages=B)
    del host
    r_in = M.pack_to_rle(src)
    for se in [(1, 31, 0, 15), (21, 21, 10, 10)]:
        pk = M.rect_packed(op, src, se).to_numpy().reshape(B, H, -1)
        r_out = M.rect_rle(op, r_in, se)
        back = M.rle_to_pack(r_out).to_numpy().reshape(B, H, -1)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(back, pk, err_msg="%s %s: runs vs packed" % (op, se))
        for i in range(D):
            want = oracle.pack(oracle.sat_apply(op, pool[i].img, se))
            np.testing.assert_array_equal(pk[i], want, err_msg="%s %s page %d" % (op, se, i))
        for i in range(D, B):
            np.testing.assert_array_equal(pk[i], pk[i % D], err_msg="%s %s replica %d" % (op, se, i))
        counts = np.diff(r_out.row_ptr.cpu().numpy()).reshape(B, H)
        for i in range(D, B):
            np.testing.assert_array_equal(counts[i], counts[i % D])
        del pk, back, r_out


@pytest.mark.parametrize("op", pagegen.OPS)
@pytest.mark.parametrize("se", [(3, 5, 1, 2), (1, 9, 0, 4), (6, 4, 5, 0), (3, 11, 1, 5), (2, 17, 0, 16)])
def test_rle_long_rows(op, se):
    """Rows of several hundred runs (more than a group keeps in registers or
    LDS), so the within-line pass, every column step (the first one with
    the within-line erosion applied as rows are read) and the final packing
    take their global-memory paths (for tall elements, the block scans keep
    their running rows in global memory); one page mixes long rows with
    short."""
    W, H = 1500, 60
    r = np.random.default_rng(11)
    img = (r.random((H, W)) < 0.5).astype(np.uint8)
    img[40:45] = 0                                 # short rows beside the long ones
    img[40:45, 100:400] = 1
    img[42, 900:1000] = 1
    n = np.diff(oracle.rle_encode(img)[0])
    assert n.max() > 300 and n.min() < 128
    assert_rle_equal(rle_op(op, img, se), oracle.apply(op, img, se), "%s %s" % (op, se))


def test_rle_alternating_rows_all_ops():
    """The worst case for run counts, ceil(W/2) runs in every row."""
    W, H = 700, 24
    img = np.tile((np.arange(W) % 2 == 0).astype(np.uint8), (H, 1))
    img[::3] ^= 1
    for op in pagegen.OPS:
        for se in [(2, 2, 0, 1), (1, 5, 0, 2), (3, 1, 1, 0), (2, 10, 1, 3)]:
            assert_rle_equal(rle_op(op, img, se), oracle.apply(op, img, se), "%s %s" % (op, se))


@pytest.mark.parametrize("op", pagegen.OPS)
def test_rle_block_scans_on_large_stacks(op):
    """Stacks of at least 32768 rows take the block-scan between-line pass
    for elements of 9 or more rows and 2 or more columns: 560 copies of a
    page whose rows hold several hundred runs (the scans' running rows then
    live in global memory), and 12 letter pages."""
    W, H, P = 1500, 60, 560
    r = np.random.default_rng(13)
    img = (r.random((H, W)) < 0.5).astype(np.uint8)
    img[40:45] = 0
    img[40:45, 100:400] = 1
    for se in [(3, 11, 1, 5), (2, 17, 0, 16)]:
        want = oracle.apply(op, img, se)
        out = rle_op(op, np.tile(img, (P, 1)), se, npages=P)
        rp, runs = out.to_host()
        wrp, wruns = oracle.rle_encode(want)
        n1 = int(wrp[-1])
        assert int(rp[-1]) == P * n1, "%s %s" % (op, se)
        counts = np.diff(rp).reshape(P, H)
        np.testing.assert_array_equal(counts, np.tile(np.diff(wrp), (P, 1)), err_msg="%s %s" % (op, se))
        np.testing.assert_array_equal(runs.reshape(P, n1, 2), np.tile(wruns.reshape(1, n1, 2), (P, 1, 1)),
                                      err_msg="%s %s" % (op, se))
    pages = [pagegen.letter_page(2100 + i).img for i in range(12)]
    stack = np.concatenate(pages)
    for se in [(21, 21, 10, 10), (9, 51, 4, 25)]:
        out = rle_op(op, stack, se, npages=12)
        assert_rle_equal(out, np.concatenate([oracle.sat_apply(op, p, se) for p in pages]), "%s %s" % (op, se))
