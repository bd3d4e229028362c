"""GPU parity of connected components, component statistics, run-length
histograms and the layout composition against the oracle: labels,
statistics and histograms must be equal exactly."""
import numpy as np
import pytest
import torch
from scipy import ndimage as ndi

import oracle
import pagegen
from gpu_util import blobs_img, garbage_pad, require_gpu, rnd_img
from oracle import components as occ
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


def rle_gpu(img, npages=1):
    rows, W = img.shape
    words = garbage_pad(oracle.pack(img, (W + 63) // 64 + 1), W, 3)
    return M.pack_to_rle(M.Bitmap.from_words(words, W, npages=npages))


def pages_of(img, P):
    H = img.shape[0] // P
    return [otr.to_lines(*oracle.rle_encode(img[p * H:(p + 1) * H])) for p in range(P)]


def expected_labels(img, P, conn):
    flat, counts = [], []
    for lines in pages_of(img, P):
        labels, n = occ.label_runs(lines, conn)
        flat.extend(l for row in labels for l in row)
        counts.append(n)
    return np.array(flat, dtype=np.int32), np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)


CASES = [(1, 1, 1.0), (1, 70, 0.5), (70, 1, 0.5), (33, 64, 0.45), (64, 65, 0.6), (120, 200, 0.35),
         (50, 300, 0.7), (20, 20, 0.0), (20, 20, 1.0)]


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "%dx%d_p%g" % c)
def test_labels_match_oracle(conn, case):
    H, W, p = case
    img = blobs_img(H * 31 + W, H, W, p) if 0 < p < 1 else rnd_img(1, H, W, p)
    labels, comp_ptr = M.label_components(rle_gpu(img), conn)
    want, wptr = expected_labels(img, 1, conn)
    np.testing.assert_array_equal(comp_ptr.cpu().numpy(), wptr)
    np.testing.assert_array_equal(labels.cpu().numpy(), want)


@pytest.mark.parametrize("conn", [4, 8])
def test_labels_stacked_pages(conn):
    P, H, W = 5, 40, 150
    imgs = [blobs_img(900 + k, H, W, 0.5) for k in range(P)]
    imgs[2][:] = 0                                   # a page with no runs
    imgs[3][-1, :] = 1                               # runs on the last row must not join the next page
    imgs[4][0, :] = 1
    img = np.concatenate(imgs)
    labels, comp_ptr = M.label_components(rle_gpu(img, P), conn)
    want, wptr = expected_labels(img, P, conn)
    np.testing.assert_array_equal(comp_ptr.cpu().numpy(), wptr)
    np.testing.assert_array_equal(labels.cpu().numpy(), want)


def label_image(r, labels, W, H):
    rp, runs = r.to_host()
    lab = labels.cpu().numpy()
    out = np.zeros((H, W), dtype=np.int64)
    for y in range(H):
        for k in range(rp[y], rp[y + 1]):
            out[y, runs[k, 0]:runs[k, 1]] = lab[k] + 1
    return out


@pytest.mark.parametrize("conn", [4, 8])
def test_labels_letter_page_match_scipy(conn):
    img = pagegen.letter_page(2000).img
    H, W = img.shape
    r = rle_gpu(img)
    labels, comp_ptr = M.label_components(r, conn)
    want, n = ndi.label(img, structure=ndi.generate_binary_structure(2, 1 if conn == 4 else 2))
    assert int(comp_ptr[-1]) == n
    np.testing.assert_array_equal(label_image(r, labels, W, H), want)


def test_long_vertical_chains_and_spirals():
    """Components whose union-find trees get deep: a full-height bar, a
    staircase, comb teeth joined at the bottom, and a spiral."""
    H, W = 300, 260
    img = np.zeros((H, W), np.uint8)
    img[:, 3] = 1
    for y in range(H):
        img[y, 10 + y // 2] = 1
    img[:280, 200:250:2] = 1
    img[280, 200:250] = 1
    sp = np.zeros((41, 41), np.uint8)
    x0, y0, x1, y1 = 0, 0, 40, 40
    while x0 < x1 and y0 < y1:
        sp[y0, x0:x1 + 1] = 1
        sp[y0:y1 + 1, x1] = 1
        sp[y1, x0:x1 + 1] = 1
        sp[y0 + 2:y1 + 1, x0] = 1
        x0, y0, x1, y1 = x0 + 2, y0 + 2, x1 - 2, y1 - 2
        sp[y0 - 1, x0 - 2] = 1
    img[250:291, 100:141] = sp
    for conn in (4, 8):
        labels, comp_ptr = M.label_components(rle_gpu(img), conn)
        want, wptr = expected_labels(img, 1, conn)
        np.testing.assert_array_equal(comp_ptr.cpu().numpy(), wptr)
        np.testing.assert_array_equal(labels.cpu().numpy(), want)


def test_component_stats_match_oracle():
    P, H, W = 3, 60, 210
    imgs = [blobs_img(40 + k, H, W, 0.4) for k in range(P)]
    img = np.concatenate(imgs)
    r = rle_gpu(img, P)
    labels, comp_ptr = M.label_components(r, 8)
    boxes, sums = M.component_stats(r, labels, comp_ptr)
    got = np.concatenate([boxes.cpu().numpy().astype(np.int64), sums.cpu().numpy()], axis=1)
    want = []
    for lines in pages_of(img, P):
        lab, n = occ.label_runs(lines, 8)
        want.append(occ.component_stats(lines, lab, n))
    np.testing.assert_array_equal(got, np.concatenate(want))


def test_run_histograms_match_oracle():
    P, H, W = 4, 50, 333
    imgs = [blobs_img(60 + k, H, W, 0.3 + 0.1 * k) for k in range(P)]
    img = np.concatenate(imgs)
    black, white = M.run_histograms(rle_gpu(img, P))
    for p, lines in enumerate(pages_of(img, P)):
        wb, ww = occ.run_histograms(lines, W)
        np.testing.assert_array_equal(black[p].cpu().numpy(), wb)
        np.testing.assert_array_equal(white[p].cpu().numpy(), ww)
    # a width beyond the LDS histograms (global counters)
    img = blobs_img(7, 20, 9000, 0.3)
    black, white = M.run_histograms(rle_gpu(img))
    wb, ww = occ.run_histograms(pages_of(img, 1)[0], 9000)
    np.testing.assert_array_equal(black[0].cpu().numpy(), wb)
    np.testing.assert_array_equal(white[0].cpu().numpy(), ww)


def test_histogram_percentile_matches_oracle():
    r = np.random.default_rng(4)
    for k in range(12):
        rows, bins = int(r.integers(1, 6)), int(r.integers(1, 700))
        h = (r.random((rows, bins)) < 0.3) * r.integers(0, 50, (rows, bins))
        if k == 0:
            h[:] = 0
        d = torch.from_numpy(h.astype(np.int32)).cuda()
        for num, den in [(1, 2), (9, 10), (1, 1), (1, 1000), (999, 1000)]:
            got = int(M.histogram_percentile(d, num, den).item())
            assert got == occ.histogram_percentile(h.sum(axis=0), num, den), (k, num, den)


def test_layout_small_stack_matches_oracle():
    P, H, W = 3, 120, 240
    imgs = []
    for k in range(P):
        im = np.zeros((H, W), np.uint8)
        rr = np.random.default_rng(k)
        for (x0, y0) in [(8, 10), (130, 60)]:
            for row in range(4):
                x = x0
                while x < x0 + 90:
                    w = int(rr.integers(2, 6))
                    im[y0 + 7 * row:y0 + 7 * row + 4, x:x + w] = 1
                    x += w + int(rr.integers(1, 4))
        imgs.append(im)
    img = np.concatenate(imgs)
    gx, gy, boxes, sums, comp_ptr = M.layout_boxes(rle_gpu(img, P), 9, 10)
    wgx, wgy, wst = occ.layout_boxes(pages_of(img, P), W, 9, 10)
    assert (gx, gy) == (wgx, wgy)
    got = np.concatenate([boxes.cpu().numpy().astype(np.int64), sums.cpu().numpy()], axis=1)
    np.testing.assert_array_equal(got, np.concatenate(wst))
    np.testing.assert_array_equal(np.diff(comp_ptr.cpu().numpy()), [len(s) for s in wst])


def test_layout_letter_page_matches_oracle():
    img = pagegen.letter_page(2003).img
    W = img.shape[1]
    gx, gy, boxes, sums, comp_ptr = M.layout_boxes(rle_gpu(img, 1), 1, 3)
    # the oracle's steps on the CPU with the brute-force dilation
    wgx, wgy, wst = occ.layout_boxes(pages_of(img, 1), W, 1, 3)
    assert (gx, gy) == (wgx, wgy)
    got = np.concatenate([boxes.cpu().numpy().astype(np.int64), sums.cpu().numpy()], axis=1)
    np.testing.assert_array_equal(got, np.concatenate(wst))


def test_label_overflow_is_reported():
    img = blobs_img(3, 40, 200, 0.5)
    r = rle_gpu(img)
    n = r.nruns()
    labels = torch.empty(n, dtype=torch.int32, device="cuda")
    comp_ptr = torch.empty(2, dtype=torch.int32, device="cuda")
    ws = torch.empty(M.morph_rle_label_workspace_bytes(40, n - 5), dtype=torch.uint8, device="cuda")
    M.morph_rle_label(r, 8, labels, n - 5, comp_ptr, ws)
    torch.cuda.synchronize()
    assert int(comp_ptr[-1]) == -1
    ws = torch.empty(M.morph_rle_label_workspace_bytes(40, n), dtype=torch.uint8, device="cuda")
    M.morph_rle_label(r, 8, labels, n, comp_ptr, ws)
    torch.cuda.synchronize()
    assert int(comp_ptr[-1]) == expected_labels(img, 1, 8)[1][-1]


def test_components_letter_batch_as_timed():
    """The benchmark's batch: 256 stacked letter pages (16 distinct,
    replicated): component counts of the 16 distinct pages against scipy's
    labelling (whole label images for two of them), every replica's labels
    and statistics against its original."""
    B, D = 256, 16
    pool = [pagegen.letter_page(2000 + i) for i in range(D)]
    W, H = 2550, 3300
    host = np.concatenate([pool[i % D].words() for i in range(B)])
    src = M.Bitmap.from_words(host, W, npages=B)
    del host
    r = M.pack_to_rle(src)
    labels, comp_ptr = M.label_components(r, 8)
    boxes, sums = M.component_stats(r, labels, comp_ptr)
    cp = comp_ptr.cpu().numpy()
    counts = np.diff(cp)
    rp = r.row_ptr.cpu().numpy()
    lab = labels.cpu().numpy()
    st8 = ndi.generate_binary_structure(2, 2)
    for i in range(D):
        want, n = ndi.label(pool[i].img, structure=st8)
        assert counts[i] == n
        if i < 2:                                   # whole label images for two pages
            runs = r.runs[rp[i * H]:rp[(i + 1) * H]].cpu().numpy()
            prp = rp[i * H:(i + 1) * H + 1] - rp[i * H]
            img = np.zeros((H, W), np.int64)
            for y in range(H):
                for k in range(prp[y], prp[y + 1]):
                    img[y, runs[k, 0]:runs[k, 1]] = lab[rp[i * H] + k] + 1
            np.testing.assert_array_equal(img, want)
    bx, sm = boxes.cpu().numpy(), sums.cpu().numpy()
    for i in range(D, B):
        j = i % D
        assert counts[i] == counts[j]
        np.testing.assert_array_equal(lab[rp[i * H]:rp[(i + 1) * H]], lab[rp[j * H]:rp[(j + 1) * H]])
        np.testing.assert_array_equal(bx[cp[i]:cp[i + 1]], bx[cp[j]:cp[j + 1]])
        np.testing.assert_array_equal(sm[cp[i]:cp[i + 1]], sm[cp[j]:cp[j + 1]])
