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
def rle_op(op, img, se, npages=1, form="slot"):
    """The operation on runs in the slot form (the library's default
    workspace) or the band form (the compact workspace)."""
    src = to_rle_gpu(img, npages=npages)
    out = M.rect_rle(op, src, se, compact=(form == "band"))
    torch.cuda.synchronize()
    return out


FORMS = pytest.mark.parametrize("form", ["slot", "band"])


@pytest.mark.parametrize("op", pagegen.OPS)
@pytest.mark.parametrize("se", [(3, 3, 1, 1), (1, 9, 0, 4), (9, 1, 4, 0), (4, 6, 0, 5), (2, 2, 1, 0)])
@FORMS
def test_rle_small_page(op, se, form):
    img = pagegen.small_page(1000).img
    assert_rle_equal(rle_op(op, img, se, form=form), oracle.apply(op, img, se), "%s %s" % (op, se))


def rle_fuzz(n, seed):
    r = np.random.default_rng(seed)
    for i in range(n):
        W = int(r.choice([1, 2, 64, 65, 200, int(r.integers(1, 500))]))
        H = int(r.integers(1, 120))
        w, h = int(r.integers(1, 70)), int(r.integers(1, 70))
        yield i, W, H, (w, h, int(r.integers(w)), int(r.integers(h))), pagegen.OPS[i % 4]


@pytest.mark.parametrize("case", list(rle_fuzz(40, 5)), ids=lambda c: "c%d" % c[0])
@FORMS
def test_rle_fuzz(case, form):
    i, W, H, se, op = case
    img = blobs_img(500 + i, H, W, float(np.random.default_rng(i).uniform(0.05, 0.7)))
    assert_rle_equal(rle_op(op, img, se, form=form), oracle.sat_apply(op, img, se), str(case))


def row_fuzz(n, seed):
    # one-row elements, every origin, widths from 1 to past the row: the
    # opening and closing take their one-pass form there
    r = np.random.default_rng(seed)
    for i in range(n):
        W = int(r.choice([1, 3, 63, 64, 65, 130, int(r.integers(1, 400))]))
        H = int(r.integers(1, 40))
        w = int(r.choice([1, 2, 3, int(r.integers(1, 40)), W, W + 3]))
        yield i, W, H, (w, 1, int(r.integers(w)), 0), ("open", "close")[i % 2]


@pytest.mark.parametrize("case", list(row_fuzz(40, 11)), ids=lambda c: "c%d" % c[0])
def test_rle_one_row_open_close(case):
    """Opening and closing by a one-row element (one pass: runs, or gaps,
    kept whole when their erosion is not empty) against the oracle's
    dilation of the erosion, border runs and gaps included."""
    i, W, H, se, op = case
    r = np.random.default_rng(900 + i)
    img = (r.random((H, W)) < r.uniform(0.2, 0.8)).astype(np.uint8)
    img[:, :1] = r.integers(0, 2, (H, 1))         # runs and gaps on both borders
    assert_rle_equal(rle_op(op, img, se), oracle.apply(op, img, se), str(case))


@pytest.mark.parametrize("density", [0.01, 0.10, 0.40])
@pytest.mark.parametrize("op", ["erode", "dilate"])
@pytest.mark.parametrize("se", [(41, 1, 20, 0), (1, 41, 0, 20)], ids=["1x41", "41x1"])
@FORMS
def test_rle_density_sweep(density, op, se, form):
    """2550 x 3300 pages at 1%, 10%, 40% black, horizontal 1x41 and vertical
    41x1 erosion and dilation on runs, compared with the oracle and with the
    packed path on the same page."""
    img = pagegen.density_page(density, 4000).img
    want = oracle.sat_apply(op, img, se)
    out = rle_op(op, img, se, form=form)
    assert_rle_equal(out, want, "%s %s %g" % (op, se, density))
    # RLE result == pack_to_rle(packed result), through rle_to_pack as well
    b = M.rle_to_pack(out)
    src = M.Bitmap.from_words(oracle.pack(img), img.shape[1])
    pk = M.rect_packed(op, src, se)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(b.to_numpy(), pk.to_numpy())


@pytest.mark.parametrize("op", pagegen.OPS)
@FORMS
def test_rle_letter_page(op, form):
    img = pagegen.letter_page(2000).img
    for se in [(31, 1, 15, 0), (1, 31, 0, 15), (3, 3, 1, 1), (21, 21, 10, 10), (51, 51, 25, 25)]:
        assert_rle_equal(rle_op(op, img, se, form=form), oracle.sat_apply(op, img, se), "%s %s" % (op, se))


@FORMS
def test_rle_stacked_pages(form):
    H, W, P = 40, 333, 4
    imgs = [blobs_img(70 + k, H, W, 0.45) for k in range(P)]
    img = np.concatenate(imgs)
    for op in pagegen.OPS:
        se = (7, 9, 3, 2)
        out = rle_op(op, img, se, npages=P, form=form)
        want = np.concatenate([oracle.apply(op, im, se) for im in imgs])
        assert_rle_equal(out, want, op)


@FORMS
def test_rle_empty_and_full(form):
    for p in (0.0, 1.0):
        img = rnd_img(1, 30, 130, p)
        for op in pagegen.OPS:
            assert_rle_equal(rle_op(op, img, (5, 5, 2, 2), form=form), oracle.apply(op, img, (5, 5, 2, 2)))


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
    # the slot form: offsets 1, 2, then 1; the within-line pass runs inside
    # the first of them; then the packing into CSR
    assert res["col_and_kernel"]["launches"] == 3
    assert res.get("row_erode_kernel", {"launches": 0})["launches"] == 0
    assert res["pack_rows_kernel"]["launches"] == 1
    with M.Trace() as tr:
        M.rect_rle("erode", r, (7, 1, 3, 0))                 # one row: the within-line pass alone
    assert tr.result["row_erode_kernel"]["launches"] == 1
    assert tr.result.get("col_and_kernel", {"launches": 0})["launches"] == 0
    # the band form: one count launch and one emit launch; the emit launch's
    # bytes are 8 per run read and written plus the row offsets read and written
    with M.Trace() as tr:
        d = M.rect_rle("dilate", r, (5, 5, 2, 2), compact=True)
    torch.cuda.synchronize()
    n_out = d.nruns()
    res = tr.result
    assert res["rle_band_count_kernel"]["launches"] == 1
    assert res["rle_band_kernel"]["launches"] == 1
    assert res["rle_band_kernel"]["bytes"] == 8 * (H + 1) + 8 * (n + n_out)
    for k in ("col_and_kernel", "row_erode_kernel", "pack_rows_kernel"):
        assert k not in res


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
@FORMS
def test_rle_long_rows(op, se, form):
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
    assert_rle_equal(rle_op(op, img, se, form=form), oracle.apply(op, img, se), "%s %s" % (op, se))


@FORMS
def test_rle_alternating_rows_all_ops(form):
    """The worst case for run counts, ceil(W/2) runs in every row."""
    W, H = 700, 24
    img = np.tile((np.arange(W) % 2 == 0).astype(np.uint8), (H, 1))
    img[::3] ^= 1
    for op in pagegen.OPS:
        for se in [(2, 2, 0, 1), (1, 5, 0, 2), (3, 1, 1, 0), (2, 10, 1, 3)]:
            assert_rle_equal(rle_op(op, img, se, form=form), oracle.apply(op, img, se), "%s %s" % (op, se))


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


@pytest.mark.parametrize("op", pagegen.OPS)
def test_rle_slot_form_tall_elements_and_wide_rows(op):
    """The slot form, which takes elements taller than a band holds (more
    than 383 rows of halo: h - 1, or 2 (h - 1) for opening and closing) and
    rows of 65536 pixels or more: tall elements on one page and on a stack
    large enough for the block scans (40000 rows), and a 70000-pixel row."""
    img = blobs_img(21, 500, 260, 0.5)
    for se in [(3, 400, 1, 200), (1, 390, 0, 100), (5, 250, 2, 124)]:
        assert_rle_equal(rle_op(op, img, se), oracle.apply(op, img, se), "%s %s" % (op, se))
    P, H, W = 100, 400, 120
    page = blobs_img(22, H, W, 0.6)
    se = (3, 390, 1, 195)
    want = oracle.apply(op, page, se)
    out = rle_op(op, np.tile(page, (P, 1)), se, npages=P)
    rp, runs = out.to_host()
    wrp, wruns = oracle.rle_encode(want)
    np.testing.assert_array_equal(np.diff(rp).reshape(P, H), np.tile(np.diff(wrp), (P, 1)), err_msg="%s stack" % op)
    np.testing.assert_array_equal(runs.reshape(P, -1, 2), np.tile(wruns.reshape(1, -1, 2), (P, 1, 1)))
    wide = blobs_img(23, 6, 70000, 0.4)
    for se in [(5, 3, 2, 1), (41, 1, 20, 0)]:
        assert_rle_equal(rle_op(op, wide, se), oracle.apply(op, wide, se), "%s wide %s" % (op, se))


def test_rle_small_capacity_reports_true_total():
    """Any output capacity is accepted: the true run count lands in
    row_ptr[rows], the runs that fit are written in place, none past it."""
    img = pagegen.small_page(1002).img
    W, H = img.shape[1], img.shape[0]
    src = M.pack_to_rle(M.Bitmap.from_words(oracle.pack(img), W))
    want_rp, want_runs = oracle.rle_encode(oracle.apply("dilate", img, (3, 3, 1, 1)))
    total = int(want_rp[-1])
    for cap in (1, total // 3, total - 1, total):
        dst = M.RLE.empty(W, H, capacity=cap + 8)
        dst.runs.fill_(-7)
        view = M.RLE(dst.row_ptr, dst.runs[:cap], W, H)
        ws = torch.empty(M.morph_rle_workspace_bytes("dilate", W, H, 1, (3, 3, 1, 1)), dtype=torch.uint8,
                         device="cuda")
        M.morph_dilate_rect_rle(view, src, (3, 3, 1, 1), ws)
        torch.cuda.synchronize()
        rp = dst.row_ptr.cpu().numpy()
        runs = dst.runs.cpu().numpy()
        np.testing.assert_array_equal(rp, want_rp)
        np.testing.assert_array_equal(runs[:cap], want_runs[:cap])
        assert (runs[cap:] == -7).all()


def test_rect_rle_binding_retries_when_the_first_guess_overflows():
    """The binding's first result array holds twice the input's runs plus one
    per row.  One row of 100 dots dilated by a tall column repeats the dots
    in every row below: 40 rows of 100 runs, more than the guess, so the
    binding sizes the array from the reported total and runs again."""
    H, W = 40, 400
    img = np.zeros((H, W), np.uint8)
    img[0, ::4] = 1                                # 100 dots, all in row 0
    src = M.pack_to_rle(M.Bitmap.from_words(oracle.pack(img), W))
    se = (1, 80, 0, 0)                             # every row below gets the 100 dots
    out = M.rect_rle("dilate", src, se)
    assert out.capacity >= out.nruns() > 2 * 100 + H + 16
    assert_rle_equal(out, oracle.apply("dilate", img, se))


def test_rle_1024_letter_pages_in_one_call():
    """1024 stacked letter pages (16 distinct, replicated): more than the slot
    form can take (its worst case passes 2^31 runs), so the library's
    workspace size is the band form's and one call does the whole stack.
    The 16 distinct pages are checked against the oracle's summed-area
    evaluator, every replica against them."""
    B, D = 1024, 16
    pool = [pagegen.letter_page(2000 + i) for i in range(D)]
    W, H = 2550, 3300
    se = (3, 3, 1, 1)
    assert M.morph_rle_max_runs(W, H * B) >= 2 ** 31
    need = M.morph_rle_workspace_bytes("close", W, H, B, se)
    assert need == M.morph_rle_workspace_bytes_compact("close", W, H, B, se) > 0
    host = np.concatenate([pool[i % D].words() for i in range(B)])
    src = M.Bitmap.from_words(host, W, npages=B)
    del host
    r_in = M.pack_to_rle(src, capacity=150 * H * B)
    out = M.rect_rle("close", r_in, se)
    rp = out.row_ptr.cpu().numpy()
    runs = out.runs[: int(rp[-1])].cpu().numpy()
    counts = np.diff(rp).reshape(B, H)
    starts = rp[:-1].reshape(B, H)[:, 0]
    for i in range(D):
        wrp, wruns = oracle.rle_encode(oracle.sat_apply("close", pool[i].img, se))
        np.testing.assert_array_equal(counts[i], np.diff(wrp), err_msg="page %d" % i)
        np.testing.assert_array_equal(runs[starts[i]: starts[i] + int(wrp[-1])], wruns, err_msg="page %d" % i)
    for i in range(D, B):
        np.testing.assert_array_equal(counts[i], counts[i % D], err_msg="replica %d" % i)
