"""The served form on the GPU: every request's result is the same whether it
is served alone or in a mix with others (arriving while others run, sharing
launches), equals the plain per-page path, and equals the oracle."""
import numpy as np
import pytest
import torch

import oracle
import pagegen
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def lib():
    require_gpu()


def make_requests(n, seed=5):
    from paper_0712_0121_amd.serve import Request, SERVE_CHAIN, chain_ses
    sizes = [(300, 211), (640, 97), (1275, 1650), (130, 40), (2550, 3300)]
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        W, H = sizes[i % len(sizes)]
        if W >= 1275:
            img = pagegen.text_page(7000 + i, W, H).img
        else:
            img = (rng.random((H, W)) < 0.25).astype(np.uint8)
        words = torch.from_numpy(oracle.pack(img).view(np.int64)).pin_memory()
        out.append(Request(i, W, H, words, chain_ses(SERVE_CHAIN)))
    return out


def clone(reqs):
    from paper_0712_0121_amd.serve import Request
    return [Request(r.rid, r.W, r.H, r.words, r.chain) for r in reqs]


def expected(r):
    img = oracle.unpack(r.words.numpy().view(np.uint64), r.W)
    for op, se in r.chain:
        img = oracle.sat_apply(op, img, se)
    return oracle.pack(img)


def served(reqs, arrivals, budget=64 << 30, ex=None):
    from paper_0712_0121_amd.serve import GpuExecutor, Server, run_trace_served
    s = Server(GpuExecutor() if ex is None else ex, budget_bytes=budget)
    run_trace_served(s, reqs, arrivals, timeout=60)
    assert not s.failed, [r.error for r in s.failed]
    return s


def test_mix_equals_alone_equals_plain_equals_oracle():
    from paper_0712_0121_amd.serve import GpuExecutor, PlainRunner
    N = 100
    reqs = make_requests(N)
    # staggered arrivals (some while others run), and every third request
    # arriving together with the one before it, so launches must be shared
    gaps = np.random.default_rng(1).exponential(0.0005, len(reqs))
    gaps[2::3] = 0.0
    arrivals = np.cumsum(gaps)
    s = served(reqs, arrivals)
    assert len(s.completed) == len(reqs)
    assert s.launches < 4 * len(reqs)           # operations shared launches
    mix = {r.rid: r.result.copy() for r in reqs}
    alone_ex = GpuExecutor()
    for r in clone(reqs):
        s1 = served([r], np.zeros(1), ex=alone_ex)
        np.testing.assert_array_equal(r.result, mix[r.rid], err_msg="request %d alone vs mix" % r.rid)
    plain = PlainRunner()
    for r in clone(reqs)[:6]:
        np.testing.assert_array_equal(plain.run_one(r), mix[r.rid])
    for r in reqs:
        np.testing.assert_array_equal(mix[r.rid], expected(r), err_msg="request %d vs oracle" % r.rid)


def test_small_budget_serves_everything():
    reqs = make_requests(8)
    fp = max(2 * r.H * ((r.W + 63) // 64) * 8 for r in reqs)
    s = served(reqs, np.zeros(len(reqs)), budget=fp + 1)
    assert s.peak_used <= fp + 1
    for r in reqs:
        np.testing.assert_array_equal(r.result, expected(r))


def test_pooled_buffers_across_traces():
    """One executor serving three traces with its device buffer pairs and
    pinned result buffers recycled (the benchmark's configuration, results
    not kept), its pools dropped before the third: every result, taken as
    it completes, equals the oracle's."""
    from paper_0712_0121_amd.serve import GpuExecutor, Server, run_trace_served

    class Capturing(GpuExecutor):
        def __init__(self):
            super().__init__(recycle_outputs=True)
            self.got = {}

        def finish(self, r):
            res = super().finish(r)
            self.got[r.rid] = res.copy()
            return res

    ex = Capturing()
    for trace in range(3):
        if trace == 2:
            ex.trim()
            assert not ex.buf_pool and not ex.out_pool
        reqs = make_requests(15, seed=40 + trace)
        for r in reqs:
            r.rid += 100 * trace
        arrivals = np.cumsum(np.random.default_rng(trace).exponential(0.0003, len(reqs)))
        s = Server(ex, 64 << 30, keep_results=False)
        run_trace_served(s, reqs, arrivals, timeout=60)
        assert not s.failed, [r.error for r in s.failed]
        assert len(s.completed) == len(reqs)
        for r in reqs:
            np.testing.assert_array_equal(ex.got[r.rid], expected(r), err_msg="trace %d request %d" % (trace, r.rid))
        assert sum(len(v) for v in ex.buf_pool.values()) >= 1


def test_served_with_run_length_routes(tmp_path):
    """Serving with a tuner that sends the chain's opening 3x3 and erosion
    15x5 on sparse pages (black density up to 3 %) to the run-length path:
    those operations of the sparse requests run as bitmap -> runs ->
    operation -> bitmap between the batched launches, and every result still
    equals the oracle and the all-packed server's."""
    from paper_0712_0121_amd.serve import GpuExecutor, Request, SERVE_CHAIN, chain_ses
    from paper_0712_0121_amd.tune import Tuner, repr_key
    chain = chain_ses(SERVE_CHAIN)
    tuner = Tuner(cache_path=str(tmp_path / "forced.json"))
    tuner.table = {"shape": {}, "repr": {repr_key(0.01, op, se): {"best": "rle"}
                                         for op, se in chain if op in ("open", "erode")}}
    rng = np.random.default_rng(9)
    reqs = []
    for i in range(12):
        W, H = [(640, 97), (300, 211), (1275, 1650)][i % 3]
        p = 0.01 if i % 2 else 0.3
        img = (rng.random((H, W)) < p).astype(np.uint8)
        words = torch.from_numpy(oracle.pack(img).view(np.int64)).pin_memory()
        reqs.append(Request(i, W, H, words, chain))
    arrivals = np.cumsum(rng.exponential(0.0004, len(reqs)))
    ex = GpuExecutor(tuner=tuner)
    s = served(reqs, arrivals, ex=ex)
    assert ex.rle_ops == 2 * 6                    # two operations of each of the six sparse requests
    plain = served(clone(reqs), arrivals)
    for r, q in zip(sorted(s.completed, key=lambda r: r.rid), sorted(plain.completed, key=lambda r: r.rid)):
        np.testing.assert_array_equal(r.result, q.result, err_msg="request %d routed vs packed" % r.rid)
        np.testing.assert_array_equal(r.result, expected(r), err_msg="request %d vs oracle" % r.rid)
