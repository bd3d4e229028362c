"""The letter workload (bitmap -> runs, the letter cases on runs, runs ->
bitmap, and the same cases on the bitmap), on one page and on a stack of 12
pages, captured once into a HIP graph and replayed: every replay, with the
program's own eager work and synchronisations between replays, gives every
output exactly as the eager calls do.  None of these entry points
allocates, copies to the host, synchronises or records a memset, so all of
their launches can be captured.  The stack (39 600 rows) takes the
multi-block scans and, for the tall elements, the block scans along the
columns, which a single page does not reach."""
import numpy as np
import pytest
import torch

import pagegen
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu

SES = [(31, 1, 15, 0), (1, 31, 0, 15), (3, 3, 1, 1), (21, 21, 10, 10), (51, 51, 25, 25)]


@pytest.fixture(scope="module", autouse=True)
def lib():
    require_gpu()


@pytest.mark.parametrize("npages", [1, 12])
def test_workload_graph_replays_match_eager(npages):
    import paper_0712_0121_amd as M
    pages = [pagegen.letter_page(2000 + i) for i in range(npages)]
    W, H = pages[0].W, pages[0].H
    src = M.Bitmap.from_words(np.concatenate([p.words() for p in pages]), W, npages=npages)
    jobs = [(op, se) for se in SES for op in pagegen.OPS]
    pk_out = [M.Bitmap.empty(W, H, npages) for _ in jobs]
    rl_out = [M.RLE.empty(W, H, npages) for _ in jobs]
    r_in = M.RLE.empty(W, H, npages)
    back = M.Bitmap.empty(W, H, npages)
    ws_p = torch.empty(max([1] + [M.morph_workspace_bytes(op, 0, W, H * npages, se) for op, se in jobs]),
                       dtype=torch.uint8, device="cuda")
    ws_r = torch.empty(max(M.morph_rle_workspace_bytes(op, W, H, npages, se) for op, se in jobs),
                       dtype=torch.uint8, device="cuda")
    ws_c = torch.empty(M.morph_pack_to_rle_workspace_bytes(W, H * npages), dtype=torch.uint8, device="cuda")

    def workload():
        M.morph_pack_to_rle(r_in, src, ws_c)
        for (op, se), r in zip(jobs, rl_out):
            M.RLE_OPS[op](r, r_in, se, ws_r)
        M.morph_rle_to_pack(back, rl_out[-1])
        for (op, se), b in zip(jobs, pk_out):
            M.PACKED[op](b, src, se, ws_p)

    def snapshot():
        torch.cuda.synchronize()
        runs = []
        for r in rl_out:
            rp = r.row_ptr.cpu().numpy()
            runs.append((rp, r.runs[: int(rp[-1])].cpu().numpy()))
        return [b.to_numpy() for b in pk_out], runs, back.to_numpy()

    def poison():
        for b in pk_out + [back]:
            b.words.fill_(0x5A5A)
        for r in rl_out:
            r.row_ptr.fill_(-1)
            r.runs.fill_(-7)
        torch.cuda.synchronize()

    with M.Trace() as tr:
        workload()
    want = snapshot()
    scans = tr.result.get("col_scan_kernel", {"launches": 0})["launches"]
    assert (scans > 0) == (npages > 1), "block scans along the columns: %d launches" % scans
    poison()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        workload()
    other = M.Bitmap.empty(W, H, npages)
    for rep in range(3):
        poison()
        g.replay()
        got = snapshot()
        for i, (a, b) in enumerate(zip(got[0], want[0])):
            np.testing.assert_array_equal(a, b, err_msg="replay %d packed job %d" % (rep, i))
        for i, ((rp, rr), (wrp, wrr)) in enumerate(zip(got[1], want[1])):
            np.testing.assert_array_equal(rp, wrp, err_msg="replay %d runs job %d row_ptr" % (rep, i))
            np.testing.assert_array_equal(rr, wrr, err_msg="replay %d runs job %d" % (rep, i))
        np.testing.assert_array_equal(got[2], want[2], err_msg="replay %d rle_to_pack" % rep)
        # the program's own eager work between replays
        M.PACKED["close"](other, src, (5, 5, 2, 2), ws_p)
        torch.cuda.synchronize()
