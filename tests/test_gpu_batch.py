"""GPU parity of the batched form: many pages of uneven sizes, each with its
own operation and element, in one persistent launch (optionally replayed
from a HIP graph), against the oracle and against per-page launches."""
import numpy as np
import pytest
import torch

import oracle
import pagegen
from gpu_util import blobs_img, garbage_pad, require_gpu

pytestmark = pytest.mark.gpu

M = None


@pytest.fixture(scope="module", autouse=True)
def lib():
    require_gpu()
    global M
    import paper_0712_0121_amd as m
    M = m
    return m


def make_batch(n, seed, sizes=((70, 40), (300, 211), (640, 97), (1000, 123)), max_se=63):
    r = np.random.default_rng(seed)
    items = []
    for i in range(n):
        W, H = sizes[int(r.integers(len(sizes)))]
        img = blobs_img(seed * 1000 + i, H, W, float(r.uniform(0.05, 0.6)))
        w, h = (int(v) for v in r.integers(1, max_se + 1, 2))
        se = (w, h, int(r.integers(w)), int(r.integers(h)))
        op = pagegen.OPS[int(r.integers(4))]
        items.append((img, op, se))
    return items


def upload(items):
    srcs, dsts = [], []
    for k, (img, op, se) in enumerate(items):
        W = img.shape[1]
        stride = (W + 63) // 64 + (k % 2)
        srcs.append(M.Bitmap.from_words(garbage_pad(oracle.pack(img, stride), W, k), W))
        dsts.append(M.Bitmap.empty(W, img.shape[0]))
    return srcs, dsts


def test_batch_matches_oracle():
    items = make_batch(40, 1)
    srcs, dsts = upload(items)
    plan = M.BatchPlan([(d, s, op, se) for d, s, (img, op, se) in zip(dsts, srcs, items)])
    assert plan.tiles >= len(items)
    plan.run(use_graph=False)
    torch.cuda.synchronize()
    for (img, op, se), d in zip(items, dsts):
        np.testing.assert_array_equal(d.to_numpy(), oracle.pack(oracle.sat_apply(op, img, se)),
                                      err_msg="%s %s %s" % (op, se, img.shape))


def test_graph_replays_match_eager():
    items = make_batch(24, 2)
    srcs, dsts = upload(items)
    plan = M.BatchPlan([(d, s, op, se) for d, s, (img, op, se) in zip(dsts, srcs, items)])
    plan.run(use_graph=False)
    torch.cuda.synchronize()
    eager = [d.to_numpy().copy() for d in dsts]
    for rep in range(4):
        for d in dsts:
            d.words.fill_(0x1234)          # eager work between replays
        torch.cuda.synchronize()
        plan.run(use_graph=True)
        torch.cuda.synchronize()
        for e, d in zip(eager, dsts):
            np.testing.assert_array_equal(d.to_numpy(), e, err_msg="replay %d" % rep)


def test_batch_equals_per_page_launches():
    """Mixed letter-size and half-size pages with elements up to 63 x 63."""
    items = []
    r = np.random.default_rng(3)
    for i in range(12):
        W, H = [(1275, 1650), (2550, 3300)][i % 2]
        img = pagegen.text_page(3000 + i, W, H).img
        w, h = (int(v) for v in r.integers(1, 64, 2))
        items.append((img, pagegen.OPS[i % 4], (w, h, w // 2, h // 2)))
    srcs, dsts = upload(items)
    plan = M.BatchPlan([(d, s, op, se) for d, s, (img, op, se) in zip(dsts, srcs, items)])
    plan.run(use_graph=True)
    torch.cuda.synchronize()
    for (img, op, se), s, d in zip(items, srcs, dsts):
        single = M.rect_packed(op, s, se)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(d.to_numpy(), single.to_numpy(), err_msg="%s %s" % (op, se))
    # two pages fully against the oracle
    for k in (0, 1):
        img, op, se = items[k]
        np.testing.assert_array_equal(dsts[k].to_numpy(), oracle.pack(oracle.sat_apply(op, img, se)))


def test_full_mixed_batch_as_timed(tmp_path):
    """The timed batched workload itself: 256 pages of 1275x1650, 2480x3508,
    2550x3300 and 5100x6600 with random elements up to 63 x 63, as one
    persistent launch replayed from a graph, with library-default and with
    autotuned tiles.  Every fourth page is checked whole against the oracle's
    summed-area evaluator; every page against its own per-page launch."""
    from paper_0712_0121_amd.tune import Tuner
    items = pagegen.mixed_batch(256, seed=3000, pool_per_size=4)
    words = {}
    srcs, dsts, dsts_t = [], [], []
    for it in items:
        if id(it.page) not in words:
            words[id(it.page)] = it.page.words()
        srcs.append(M.Bitmap.from_words(words[id(it.page)], it.page.W))
        dsts.append(M.Bitmap.empty(it.page.W, it.page.H))
        dsts_t.append(M.Bitmap.empty(it.page.W, it.page.H))
    plan = M.BatchPlan([(d, s, it.op, it.se) for it, s, d in zip(items, srcs, dsts)])
    tuner = Tuner(cache_path=str(tmp_path / "tune.json"))
    widths = {}
    for it in items:
        widths.setdefault(it.page.W, (it.page.H, words[id(it.page)]))
    tuner.tune_shapes(widths, ops=("erode", "open"), h_values=(5, 40), batch=8)
    plan_t = M.BatchPlan([(d, s, it.op, it.se) + tuner.params(it.page.W, it.page.H, it.op, it.se)
                          for it, s, d in zip(items, srcs, dsts_t)])
    for _ in range(2):                      # two replays, the second over the first's output
        plan.run(use_graph=True)
        plan_t.run(use_graph=True)
    torch.cuda.synchronize()
    sizes = set()
    for k, (it, s, d, dt) in enumerate(zip(items, srcs, dsts, dsts_t)):
        got = d.to_numpy()
        np.testing.assert_array_equal(dt.to_numpy(), got, err_msg="tuned tiles, page %d" % k)
        if k % 4 == 0:
            sizes.add((it.page.W, it.page.H))
            want = oracle.pack(oracle.sat_apply(it.op, it.page.img, it.se))
            np.testing.assert_array_equal(got, want, err_msg="page %d %s %s %s" % (k, it.op, it.se, got.shape))
        single = M.rect_packed(it.op, s, it.se)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(single.to_numpy(), got, err_msg="per-page launch, page %d" % k)
    assert sizes == set(pagegen.PAGE_SIZES)


class _ForcedTuner:
    """A tuner whose table sends the given (density bucket, op, size class)
    keys to runs; everything else stays packed (Tuner's own lookups)."""

    def __new__(cls, tmp_path, rle_keys):
        from paper_0712_0121_amd.tune import Tuner
        t = Tuner(cache_path=str(tmp_path / "forced.json"))
        t.table = {"shape": {}, "repr": {k: {"best": "rle"} for k in rle_keys}}
        return t


def test_routed_batch_forced_routes_match_oracle_and_packed():
    """Pages sent down the run-length path (bitmap -> runs -> operation ->
    bitmap) give the same bits as the packed path and the oracle: every
    other page routed to runs, with uneven sizes, strides and elements."""
    items = make_batch(16, 5, max_se=40)
    srcs, dsts = upload(items)
    _, dsts_pk = upload(items)
    routes = ["rle" if k % 2 else "packed" for k in range(len(items))]
    rb = M.RoutedBatch([(d, s, op, se) for d, s, (img, op, se) in zip(dsts, srcs, items)], routes=routes)
    assert rb.route_counts() == {"packed": 8, "rle": 8}
    plan = M.BatchPlan([(d, s, op, se) for d, s, (img, op, se) in zip(dsts_pk, srcs, items)])
    for rep in range(2):
        for d in dsts:
            d.words.fill_(-1)
        rb.run(use_graph=rep > 0)
        plan.run(use_graph=False)
        torch.cuda.synchronize()
        for k, ((img, op, se), d, dp) in enumerate(zip(items, dsts, dsts_pk)):
            got = d.to_numpy()
            np.testing.assert_array_equal(got, dp.to_numpy(), err_msg="page %d (%s) vs packed" % (k, routes[k]))
            np.testing.assert_array_equal(got, oracle.pack(oracle.sat_apply(op, img, se)),
                                          err_msg="page %d %s %s %s" % (k, routes[k], op, se))


def test_routed_batch_tuner_routes_by_density(tmp_path):
    """The tuner's choice routes by the density the library counts on the
    device: sparse pages (1 % black) of an operation the table sends to runs
    take the run-length path, dense ones (40 %) stay packed, and both match
    the oracle."""
    from paper_0712_0121_amd.tune import repr_key
    se = (9, 1, 4, 0)
    tuner = _ForcedTuner(tmp_path, [repr_key(0.01, "dilate", se)])
    items = []
    for k, d in enumerate((0.01, 0.40, 0.01, 0.40)):
        img = pagegen.density_page(d, 4100 + k).img[:400, :700].copy()
        items.append((img, "dilate", se))
    srcs, dsts = upload(items)
    dens = M.page_densities(srcs)
    for (img, _, _), got in zip(items, dens):
        assert abs(got - img.mean()) < 1e-12
    rb = M.RoutedBatch([(d, s, op, se_) for d, s, (img, op, se_) in zip(dsts, srcs, items)], tuner=tuner)
    assert rb.routes == ["rle", "packed", "rle", "packed"]
    rb.run()
    torch.cuda.synchronize()
    for (img, op, se_), d in zip(items, dsts):
        np.testing.assert_array_equal(d.to_numpy(), oracle.pack(oracle.apply(op, img, se_)))
