"""The serving scheduler on the CPU, with a mock executor that runs each
operation with the oracle and finishes work only after a few polls (so
requests overlap as they would on the device)."""
import numpy as np
import pytest

import oracle
import pagegen
from paper_0712_0121_amd.serve import Request, Server, SERVE_CHAIN, chain_ses


class Token:
    def __init__(self, polls, err=None):
        self.left = polls
        self.err = err

    def poll(self):
        self.left -= 1
        return self.left <= 0


class MockExecutor:
    def __init__(self, latency_polls=3, fail_on_launch=None, word_bytes=8):
        self.polls = latency_polls
        self.fail_on_launch = fail_on_launch      # launch index that reports an error
        self.launch_count = 0
        self.batch_sizes = []
        self.mixed_positions = 0

    def footprint(self, r):
        return 2 * r.H * ((r.W + 63) // 64) * 8

    def begin(self, r):
        r.state = {"img": oracle.unpack(np.asarray(r.words), r.W), "nxt": None}

    def launch(self, reqs):
        self.launch_count += 1
        self.batch_sizes.append(len(reqs))
        if len({r.pos for r in reqs}) > 1:
            self.mixed_positions += 1
        err = "injected failure" if self.launch_count == self.fail_on_launch else None
        tok = Token(self.polls, err)
        for r in reqs:
            op, se = r.chain[r.pos]
            r.state["nxt"] = oracle.sat_apply(op, r.state["img"], se)
            r.state["last"] = tok
        return tok

    def done(self, t):
        return t.poll()

    def error(self, t):
        return t.err

    def advance(self, r):
        r.state["img"], r.state["nxt"] = r.state["nxt"], None

    def begin_download(self, r):
        r.state["dl"] = Token(2)

    def downloaded(self, r):
        # a download finishes only after the request's last launch
        return r.state["dl"].poll() and r.state["last"].left <= 0

    def finish(self, r):
        return oracle.pack(r.state["img"])

    def release(self, r):
        r.state = {}


def make_requests(n, seed=0, sizes=((130, 40), (300, 77), (64, 9))):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        W, H = sizes[i % len(sizes)]
        img = (rng.random((H, W)) < 0.3).astype(np.uint8)
        out.append(Request(i, W, H, oracle.pack(img), chain_ses(SERVE_CHAIN)))
    return out


def expected(r):
    img = oracle.unpack(r.words, r.W)
    for op, se in r.chain:
        img = oracle.sat_apply(op, img, se)
    return oracle.pack(img)


def run(server, reqs, every=1):
    """Submits one request per `every` steps, then drains."""
    k = 0
    steps = 0
    while k < len(reqs) or not server.idle():
        if k < len(reqs) and steps % every == 0:
            server.submit(reqs[k])
            k += 1
        server.step()
        steps += 1
        assert steps < 100000


def test_all_requests_complete_with_oracle_results():
    ex = MockExecutor()
    s = Server(ex, budget_bytes=1 << 30)
    reqs = make_requests(12)
    run(s, reqs, every=2)
    assert len(s.completed) == 12 and not s.failed
    for r in reqs:
        np.testing.assert_array_equal(r.result, expected(r))
    # continuous batching: later arrivals shared launches with earlier ones
    assert ex.mixed_positions > 0
    assert max(ex.batch_sizes) > 1


def test_budget_is_never_exceeded_and_admission_is_fifo():
    reqs = make_requests(10)
    fp = max(MockExecutor().footprint(r) for r in reqs)
    ex = MockExecutor()
    s = Server(ex, budget_bytes=2 * fp)
    run(s, reqs, every=1)
    assert s.peak_used <= 2 * fp
    admits = [r.t_admit for r in sorted(reqs, key=lambda r: r.rid)]
    assert admits == sorted(admits)
    assert len(s.completed) == 10


def test_request_larger_than_budget_is_rejected():
    reqs = make_requests(3)
    big = Request(99, 4096, 4096, np.zeros((4096, 64), np.uint64), chain_ses(SERVE_CHAIN))
    s = Server(MockExecutor(), budget_bytes=1 << 20)
    s.submit(big)
    run(s, reqs)
    assert big.error and big in s.failed
    assert len(s.completed) == 3


def test_injected_failure_fails_only_its_batch_and_frees_budget():
    reqs = make_requests(9)
    ex = MockExecutor(fail_on_launch=2)
    s = Server(ex, budget_bytes=1 << 30)
    run(s, reqs, every=1)
    assert s.failed and all(r.error == "injected failure" for r in s.failed)
    assert len(s.failed) + len(s.completed) == 9
    assert s.used == 0
    for r in s.completed:
        np.testing.assert_array_equal(r.result, expected(r))


def test_chain_is_the_serving_workload():
    assert [op for op, _ in SERVE_CHAIN] == ["close", "open", "dilate", "erode"]
    assert chain_ses(SERVE_CHAIN)[0] == ("close", (41, 1, 20, 0))
    assert chain_ses(SERVE_CHAIN)[2] == ("dilate", (5, 15, 2, 7))


def test_tuner_rle_possible_and_choice(tmp_path):
    """The representation lookups: a (density bucket, op, size class) entry
    marked 'rle' routes only pages of that bucket, operation and class to
    runs, and rle_possible sees it for any density."""
    from paper_0712_0121_amd.tune import Tuner, repr_key
    t = Tuner(cache_path=str(tmp_path / "t.json"))
    t.table = {"shape": {}, "repr": {repr_key(0.01, "dilate", (9, 1, 4, 0)): {"best": "rle"},
                                     repr_key(0.3, "erode", (3, 3, 1, 1)): {"best": "packed"}}}
    assert t.choose_repr(0.02, "dilate", (15, 5, 7, 2)) == "rle"       # same bucket and class
    assert t.choose_repr(0.05, "dilate", (15, 5, 7, 2)) == "packed"    # denser bucket
    assert t.choose_repr(0.02, "dilate", (41, 1, 20, 0)) == "packed"   # larger class
    assert t.choose_repr(0.02, "erode", (9, 1, 4, 0)) == "packed"      # other operation
    assert t.rle_possible("dilate", (3, 11, 1, 5))
    assert not t.rle_possible("erode", (3, 3, 1, 1))
    assert not t.rle_possible("dilate", (3, 3, 1, 1))


def test_strategy_lookup_defaults_to_lines(tmp_path):
    from paper_0712_0121_amd.tune import Tuner, strategy_key
    t = Tuner(cache_path=str(tmp_path / "s.json"))
    assert t.choose_strategy("close", (1, 31, 0, 15)) == "lines"
    t.table["strategy"] = {strategy_key("close", (1, 31, 0, 15)): {"best": "transpose"}}
    assert t.choose_strategy("close", (1, 25, 0, 12)) == "transpose"     # same width and height buckets
    assert t.choose_strategy("close", (31, 1, 15, 0)) == "lines"
    assert t.choose_strategy("open", (1, 31, 0, 15)) == "lines"


def test_strategy_takes_transposition_only_by_a_margin(tmp_path):
    """Timed alone, the transposition route must beat the between-line route
    by the tuner's margin before it is chosen: near ties stay on runs."""
    from paper_0712_0121_amd.tune import Tuner, strategy_key
    t = Tuner(cache_path=str(tmp_path / "t.json"))
    k = strategy_key("dilate", (21, 21, 10, 10))
    t.table["strategy"] = {k: {"best": "transpose", "lines_ms": 1.00, "transpose_ms": 0.95}}
    assert t.choose_strategy("dilate", (21, 21, 10, 10)) == "lines"
    t.table["strategy"][k]["transpose_ms"] = 1.00 / t.STRATEGY_MARGIN - 0.01
    assert t.choose_strategy("dilate", (21, 21, 10, 10)) == "transpose"
