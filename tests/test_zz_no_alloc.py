"""The allocation-free conversion (morph_pack_to_rle_noalloc, scratch in the
library's fixed device array) against morph_pack_to_rle with a caller
workspace, through the C-ABI: row offsets and runs identical, on calls in a
row whose inputs shrink (the array keeps the previous call's contents), and
against the oracle's encoding."""
import numpy as np
import pytest
import torch

import oracle
import pagegen
from gpu_util import blobs_img, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    require_gpu()
    import paper_0712_0121_amd as m
    return m


def _both(M, img, npages, W):
    print("noalloc case: %d rows x %d px, %d page(s)" % (img.shape[0], W, npages), flush=True)
    src = M.Bitmap.from_words(oracle.pack(img), W, npages=npages)
    H = img.shape[0] // npages
    cap = int(M.morph_rle_max_runs(W, H * npages))
    ref = M.RLE.empty(W, H, npages, capacity=cap)
    got = M.RLE.empty(W, H, npages, capacity=cap)
    got.row_ptr.fill_(-7)
    M.morph_pack_to_rle(ref, src, M._alloc_ws(M.morph_pack_to_rle_workspace_bytes(W, H * npages), "cuda"))
    M.morph_pack_to_rle_noalloc(got, src)
    torch.cuda.synchronize()
    return ref, got


def _check(ref, got, img):
    rrp, rruns = ref.to_host()
    grp, gruns = got.to_host()
    np.testing.assert_array_equal(grp, rrp)
    np.testing.assert_array_equal(gruns, rruns)
    wrp, wruns = oracle.rle_encode(img)
    np.testing.assert_array_equal(grp, wrp)
    np.testing.assert_array_equal(gruns, wruns)


def test_noalloc_matches_workspace_entry_on_shrinking_calls(M):
    pages = [pagegen.letter_page(2000 + k).img for k in range(6)]
    big = np.concatenate(pages)                                   # 19800 rows: multi-block scan
    small = blobs_img(3, 37, 200, 0.4)                            # 37 rows: single-block scan
    for img, npages, W in [(big, 6, 2550), (small, 1, 200), (big[:3300 * 2], 2, 2550)]:
        ref, got = _both(M, img, npages, W)
        _check(ref, got, img)


def test_noalloc_at_the_row_limit(M):
    rows = M.MORPH_NOALLOC_MAX_ROWS
    r = np.random.default_rng(11)
    img = (r.random((rows, 64)) < 0.05).astype(np.uint8)
    ref, got = _both(M, img, 1, 64)
    rrp, rruns = ref.to_host()
    grp, gruns = got.to_host()
    np.testing.assert_array_equal(grp, rrp)
    np.testing.assert_array_equal(gruns, rruns)
    # then a much smaller call reuses the same scratch
    small = blobs_img(8, 100, 130, 0.5)
    ref, got = _both(M, small, 1, 130)
    _check(ref, got, small)
