"""Serving loop: continuous batching of page requests with chains of
rectangle operations on one GPU.

Requests arrive with a packed page (host memory) and a chain of operations,
e.g. close 1x41 -> open 3x3 -> dilate 15x5 -> erode 15x5.  The server

* admits requests first come first served while the device bytes they need
  (two resident page buffers each) fit in an HBM budget; a request larger
  than the whole budget is rejected, others wait;
* uploads admitted pages on one copy stream and downloads results on
  another, so uploads, downloads (the two PCIe directions) and kernels
  overlap;
* every scheduling step runs the next operation of every admitted request
  that is not already on the device as ONE persistent batched launch
  (morph_batch_launch), so requests at different points of their chains,
  and requests that arrived while others were running, share launches;
  the page stays resident between its operations (two buffers, swapped);
* downloads finished pages and frees their budget.

The scheduler only talks to an executor object, so its logic can be tested
without a GPU.  GpuExecutor is the product executor; PlainRunner is the
comparison: one page at a time, upload, each elementary operation as its own
launch, download.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

# chain of the serving workload: (op, (w, h)) with h x w element strings
# close 1x41, open 3x3, dilate 15x5, erode 15x5
SERVE_CHAIN = (("close", (41, 1)), ("open", (3, 3)), ("dilate", (5, 15)), ("erode", (5, 15)))


def centred(w, h):
    return (w, h, w // 2, h // 2)


def chain_ses(chain):
    return [(op, centred(*wh)) if len(wh) == 2 else (op, tuple(wh)) for op, wh in chain]


@dataclasses.dataclass(eq=False, slots=True)
class Request:
    rid: int
    W: int
    H: int
    words: object                  # host (rows, stride) words: numpy uint64 or pinned torch int64
    chain: list                    # [(op, (w, h, cx, cy)), ...]
    arrival: float = 0.0           # seconds on the server clock
    pos: int = 0                   # operations queued
    alone: bool = False            # admitted while the server had nothing else
    t_admit: float = -1.0
    t_done: float = -1.0
    result: object = None
    error: str | None = None
    state: dict = dataclasses.field(default_factory=dict)   # executor-private

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class Server:
    """Admission under a byte budget plus continuous batching (see module
    docstring).  Call submit() as requests arrive and step() in a loop."""

    def __init__(self, executor, budget_bytes: int, max_inflight_batches: int = 4,
                 clock=time.perf_counter, keep_results: bool = True, min_batch: int = 8):
        self.ex = executor
        # with two launches queued, the next one waits until min_batch
        # requests are ready (with fewer queued it goes at once, so a lone
        # request still has its chain queued behind the device's work):
        # each launch costs the host about as much as several pages'
        # bookkeeping, and at high load tiny launches cap the pages per second
        self.min_batch = max(1, int(min_batch))
        self.keep_results = keep_results
        self.budget = int(budget_bytes)
        self.max_batches = max_inflight_batches
        self.clock = clock
        self.t0 = clock()
        self.used = 0
        self.pending = collections.deque()
        self.active = []
        self.batches = collections.deque()     # (token, [requests])
        self.downloading = collections.deque()
        self.completed = []
        self.failed = []
        self.launches = 0
        self.peak_used = 0

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request, arrival: float | None = None):
        req.arrival = self.now() if arrival is None else arrival
        if self.ex.footprint(req) > self.budget:
            req.error = "request needs %d bytes, budget is %d" % (self.ex.footprint(req), self.budget)
            req.t_done = self.now()
            self.failed.append(req)
            return
        self.pending.append(req)

    def _fail(self, reqs, msg):
        for r in reqs:
            if r.error is not None or r in self.completed:
                continue
            r.error = msg
            r.t_done = self.now()
            if r in self.active:
                self.active.remove(r)
            if r in self.downloading:
                self.downloading.remove(r)
            self.used -= self.ex.footprint(r)
            self.ex.release(r)
            self.failed.append(r)

    def step(self) -> bool:
        """One scheduling step; returns True if anything happened.

        Operations of one request are queued in order on one device stream,
        so the next operation of a request is queued as soon as the previous
        one has been queued, without waiting for it (within the same step
        while launch slots are free); a request's download is queued behind
        its last operation.  At most max_batches launches are outstanding at
        a time."""
        moved = False
        while self.batches and self.ex.done(self.batches[0][0]):
            token, reqs = self.batches.popleft()
            err = self.ex.error(token)
            if err:
                self._fail(reqs, err)
            moved = True
        # downloads finish in the order they were queued when the executor
        # says so (one copy stream): then polling stops at the first one
        # still in flight
        # (a deque taken from the front: a step costs the same however many
        # downloads are queued, which keeps a queue from slowing the loop
        # that has to drain it)
        in_order = getattr(self.ex, "downloads_in_order", False)
        if in_order:
            q = self.downloading
            while q:
                r = q[0]
                if r.error is None and not self.ex.downloaded(r):
                    break
                q.popleft()
                if r.error is None:
                    self._complete(r)
                    moved = True
        else:
            still = collections.deque()
            for r in self.downloading:
                if r.error is not None:
                    continue
                if self.ex.downloaded(r):
                    self._complete(r)
                    moved = True
                else:
                    still.append(r)
            self.downloading = still
        # admission, first come first served
        while self.pending and self.used + self.ex.footprint(self.pending[0]) <= self.budget:
            r = self.pending.popleft()
            self.used += self.ex.footprint(r)
            self.peak_used = max(self.peak_used, self.used)
            r.t_admit = self.now()
            # nothing else on the device and nothing else waiting: the
            # executor may keep this request's copies on its compute stream
            r.alone = not (self.active or self.batches or self.downloading or self.pending)
            self.ex.begin(r)
            self.active.append(r)
            moved = True
        # the next operation of every admitted request, as one launch; while
        # launch slots are free, the operation after it too (stream order
        # keeps each request's operations in sequence), so a request that is
        # alone has its whole chain queued at once and later arrivals join
        # the next launch at their own position
        while self.active and len(self.batches) < self.max_batches:
            if len(self.batches) >= 2 and len(self.active) < self.min_batch:
                break
            ready = list(self.active)
            try:
                token = self.ex.launch(ready)
            except Exception as e:          # the launch could not be queued
                self._fail(ready, "launch failed: %s" % e)
                return True
            self.batches.append((token, ready))
            self.launches += 1
            done_chain = False
            for r in ready:
                self.ex.advance(r)
                r.pos += 1
                if r.pos == len(r.chain):
                    done_chain = True
                    self.ex.begin_download(r)
                    self.downloading.append(r)
            if done_chain:
                self.active = [r for r in self.active if r.pos < len(r.chain)]
            moved = True
        return moved

    def _complete(self, r: Request):
        res = self.ex.finish(r)
        r.result = res if self.keep_results else None
        r.t_done = self.now()
        self.ex.release(r)
        self.used -= self.ex.footprint(r)
        self.completed.append(r)

    def idle(self) -> bool:
        return not (self.pending or self.active or self.batches or self.downloading)

    def drain(self, timeout: float = 60.0):
        end = self.clock() + timeout
        while not self.idle():
            self.step()
            if self.clock() > end:
                raise TimeoutError("server did not drain")


class GpuExecutor:
    """Runs the server's work on the GPU through the C ABI.  A step with at
    most `direct_max` pages launches each page's operation directly (no page
    table to build and copy, which dominates for one or two pages); larger
    steps use one persistent batched launch."""

    # downloads complete in the order they were queued: they run on the
    # download stream, except a lone request's, which is admitted only when
    # no download is pending and whose copy precedes, on the compute stream,
    # every launch a later download waits for
    downloads_in_order = True

    def __init__(self, device="cuda:0", ws_bytes=64 << 20, staging_slots=4, direct_max=2,
                 recycle_outputs=False, tuner=None):
        import torch
        import paper_0712_0121_amd as M
        self.M, self.torch = M, torch
        # representation choice per operation (section "Experiments",
        # runtime selection with conversion costs): with a tuner, an
        # operation whose (density, op, element) entry says 'rle' runs as
        # bitmap -> runs -> operation -> bitmap instead of in the batch
        self.tuner = tuner
        self._rle_possible = {}
        self.rle = None
        self.rle_ops = 0
        self.device = torch.device(device)
        self.compute = torch.cuda.Stream(device=self.device)
        self.copy = torch.cuda.Stream(device=self.device)        # uploads
        self.down = torch.cuda.Stream(device=self.device)        # downloads (the other PCIe direction)
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)
        self.staging = [torch.empty(ws_bytes, dtype=torch.uint8, pin_memory=True) for _ in range(staging_slots)]
        self.staging_ev = [None] * staging_slots
        self.slot = 0
        self.direct_max = direct_max
        # with recycle_outputs the pinned result buffers go back to a pool per
        # page shape on release: only for a server that does not keep results
        # (Server(keep_results=False)), since a kept result is a view of one
        self.recycle = recycle_outputs
        self.out_pool = collections.defaultdict(list)
        # events are reused: a new one costs about 80 us of host time at its
        # first record, a recorded one about 5.  Each goes back once: an
        # upload's after the compute stream's wait on it is queued (a wait
        # binds to the record at that moment), a launch's once it has been
        # seen complete, a download's at release
        self.ev_pool = []
        # device buffer pairs per page shape, each with its batch descriptors
        # per chain; a pair goes back on release once the request's download
        # has completed (every upload, launch and copy on it is then done), so
        # the buffers need no per-stream use records, whose bookkeeping on
        # every allocation and free costs more host time than the page's
        # launches
        self.buf_pool = collections.defaultdict(list)

    def footprint(self, r: Request) -> int:
        return 2 * r.H * ((r.W + 63) // 64) * 8

    def _event(self):
        return self.ev_pool.pop() if self.ev_pool else self.torch.cuda.Event()

    def trim(self):
        """Drops the pooled device buffer pairs and pinned result buffers,
        for a server that has seen many page shapes.  Only idle buffers are
        pooled, so this is safe at any time between steps."""
        self.buf_pool.clear()
        self.out_pool.clear()

    def begin(self, r: Request):
        torch, M = self.torch, self.M
        host = r.words
        if not isinstance(host, torch.Tensor):
            host = torch.from_numpy(np.ascontiguousarray(host).view(np.int64))
        pool = self.buf_pool[(r.W, r.H)]
        if pool:
            a, b, cache = pool.pop()
        else:
            a = M.Bitmap.empty(r.W, r.H, device=self.device)
            b = M.Bitmap.empty(r.W, r.H, device=self.device)
            cache = {}
        # a request alone on the device has nothing to overlap with: its
        # copies go on the compute stream, which saves two cross-stream waits
        up = self.compute if r.alone else self.copy
        if host.is_pinned() and host.is_contiguous() and host.shape[1] == a.stride:
            # pooled buffers and a pinned page that lives as long as the
            # request: the library's plain copy, without the framework's
            # per-copy bookkeeping
            M.morph_copy_async(a.words.data_ptr(), host.data_ptr(), a.words.numel() * 8, up)
        else:
            with torch.cuda.stream(up):
                a.words.copy_(host[:, : a.stride], non_blocking=True)
        ev = None
        if up is not self.compute:
            ev = self._event()
            ev.record(up)
        # the chain's batch descriptors, built once: operation k reads the
        # buffer written by operation k-1
        key = tuple(r.chain)
        descs = cache.get(key)
        if descs is None:
            bufs = (a, b)
            descs = [M.page_desc(bufs[(k + 1) % 2], bufs[k % 2], op, se) for k, (op, se) in enumerate(r.chain)]
            cache[key] = descs
        r.state = {"cur": a, "nxt": b, "pair": (a, b, cache), "up": ev, "host": host, "descs": descs,
                   "routes": self._routes(r, host)}

    def _routes(self, r: Request, host):
        """The path of each operation of the chain, or None when every one is
        packed.  The page's black density is counted on the host copy, and
        only for chains the tuner could send to runs."""
        if self.tuner is None:
            return None
        key = tuple(r.chain)
        poss = self._rle_possible.get(key)
        if poss is None:
            poss = any(self.tuner.rle_possible(op, se) for op, se in r.chain)
            self._rle_possible[key] = poss
        if not poss:
            return None
        nw = (r.W + 63) // 64
        words = host.numpy().view(np.uint64)[:, :nw] if hasattr(host, "numpy") else np.asarray(host)[:, :nw]
        black = int(np.bitwise_count(words[:, :nw - 1]).sum())
        tail = (1 << (r.W - 64 * (nw - 1))) - 1 if r.W % 64 else (1 << 64) - 1
        black += int(np.bitwise_count(words[:, nw - 1] & np.uint64(tail)).sum())
        density = black / float(r.W * r.H)
        routes = [self.tuner.choose_repr(density, op, se) for op, se in r.chain]
        return routes if "rle" in routes else None

    def launch(self, reqs):
        torch, M = self.torch, self.M
        items, packed, rle = [], [], []
        for r in reqs:
            st = r.state
            if st.get("up") is not None:
                self.compute.wait_event(st["up"])
                self.ev_pool.append(st["up"])
                st["up"] = None
            rt = st.get("routes")
            if rt is not None and rt[r.pos] == "rle":
                rle.append(r)
            else:
                items.append(st["descs"][r.pos])
                packed.append(r)
        if rle:
            # run-length operations go one page at a time on the compute
            # stream, ahead of the batched launch of the packed ones
            if self.rle is None:
                self.rle = M.RleRoute(self.device)
            for r in rle:
                op, se = r.chain[r.pos]
                self.rle.run(r.state["nxt"], r.state["cur"], op, se, self.compute)
            self.rle_ops += len(rle)
            reqs = packed
        if not items:
            ev = self._event()
            ev.record(self.compute)
            for r in rle:
                r.state["ev"] = ev
            return ev
        if len(items) <= self.direct_max:
            with torch.cuda.stream(self.compute):
                for r in reqs:
                    op, se = r.chain[r.pos]
                    M.PACKED[op](r.state["nxt"], r.state["cur"], se, self.ws)
                ev = self._event()
                ev.record(self.compute)
            for r in reqs + rle:
                r.state["ev"] = ev
            return ev
        k = self.slot
        self.slot = (k + 1) % len(self.staging)
        if self.staging_ev[k] is not None:
            self.staging_ev[k].synchronize()       # its copy has been consumed
        M.morph_batch_launch(items, self.ws, self.staging[k], stream=self.compute)
        ev = self._event()
        ev.record(self.compute)
        self.staging_ev[k] = ev
        for r in reqs + rle:
            r.state["ev"] = ev
        return ev

    def done(self, token) -> bool:
        if not token.query():
            return False
        # complete: its staging copy has been consumed too
        for i, e in enumerate(self.staging_ev):
            if e is token:
                self.staging_ev[i] = None
        self.ev_pool.append(token)
        return True

    def error(self, token):
        return None

    def advance(self, r: Request):
        st = r.state
        st["cur"], st["nxt"] = st["nxt"], st["cur"]

    def begin_download(self, r: Request):
        torch = self.torch
        st = r.state
        shape = (r.H, st["cur"].stride)
        pool = self.out_pool[shape] if self.recycle else None
        out = pool.pop() if pool else torch.empty(shape, dtype=torch.int64, pin_memory=True)
        down = self.compute if r.alone else self.down
        if down is not self.compute:
            down.wait_event(st["ev"])
        # out is pinned and pooled, the device pair too: neither is freed
        # before this copy's event has been seen complete
        self.M.morph_copy_async(out.data_ptr(), st["cur"].words.data_ptr(), out.numel() * 8, down)
        ev = self._event()
        ev.record(down)
        st["out"], st["down"] = out, ev

    def downloaded(self, r: Request) -> bool:
        return r.state["down"].query()

    def finish(self, r: Request):
        return r.state["out"].numpy().view(np.uint64)

    def release(self, r: Request):
        st = r.state
        out, down, pair = st.get("out"), st.get("down"), st.get("pair")
        finished = down is not None and down.query()
        if down is not None and not finished:
            # a failed request's result copy may still be in flight, and the
            # framework does not know of it: wait before its pinned buffer
            # can be freed and handed out again
            down.synchronize()
        if self.recycle and out is not None and finished:
            self.out_pool[tuple(out.shape)].append(out)
        if down is not None:
            self.ev_pool.append(down)
        if pair is not None:
            if finished:
                self.buf_pool[(r.W, r.H)].append(pair)
            else:
                # a failed request may still have work queued on the side
                # streams: the allocator must not hand the buffers out again
                # before that work is done
                for t in (pair[0].words, pair[1].words):
                    t.record_stream(self.copy)
                    t.record_stream(self.compute)
                    t.record_stream(self.down)
        r.state = {}


class PlainRunner:
    """The comparison path: one page at a time, upload, each elementary
    operation (opening and closing split into erosion and dilation) as its
    own launch, download, then the next page."""

    def __init__(self, device="cuda:0"):
        import torch
        import paper_0712_0121_amd as M
        self.M, self.torch = M, torch
        self.device = torch.device(device)
        # with timing set, run_one also records the device time of the
        # chain's launches alone (no copies) into device_ms
        self.timing = False
        self.device_ms = []

    @staticmethod
    def elementary(chain):
        out = []
        for op, se in chain:
            if op == "open":
                out += [("erode", se), ("dilate", se)]
            elif op == "close":
                out += [("dilate", se), ("erode", se)]
            else:
                out.append((op, se))
        return out

    def run_one(self, r: Request):
        torch, M = self.torch, self.M
        host = r.words
        if not isinstance(host, torch.Tensor):
            host = torch.from_numpy(np.ascontiguousarray(host).view(np.int64))
        a = M.Bitmap.empty(r.W, r.H, device=self.device)
        b = M.Bitmap.empty(r.W, r.H, device=self.device)
        a.words.copy_(host[:, : a.stride], non_blocking=True)
        if self.timing:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
        for op, se in self.elementary(r.chain):
            n = M.morph_workspace_bytes(op, 0, r.W, r.H, se)     # 0 unless the element is split
            ws = torch.empty(n, dtype=torch.uint8, device=self.device) if n else None
            M.PACKED[op](b, a, se, ws)
            a, b = b, a
        if self.timing:
            e1.record()
        out = torch.empty((r.H, a.stride), dtype=torch.int64, pin_memory=True)
        out.copy_(a.words, non_blocking=True)
        torch.cuda.current_stream().synchronize()
        if self.timing:
            self.device_ms.append(e0.elapsed_time(e1))
        return out.numpy().view(np.uint64)


def run_trace_served(server: Server, requests, arrivals, timeout=120.0):
    """Submits requests[i] at arrivals[i] seconds (server clock) and runs the
    scheduler until all are done."""
    order = np.argsort(arrivals, kind="stable")
    i = 0
    end = server.clock() + timeout
    while i < len(order) or not server.idle():
        now = server.now()
        while i < len(order) and arrivals[order[i]] <= now:
            server.submit(requests[order[i]], arrival=float(arrivals[order[i]]))
            i += 1
        server.step()
        if server.clock() > end:
            raise TimeoutError("trace did not finish")
    return server.completed


def run_trace_plain(runner: PlainRunner, requests, arrivals, clock=time.perf_counter, keep_results=True):
    """Serves the same trace with the plain path: requests in arrival order,
    each started when it has arrived and the previous one is done."""
    t0 = clock()
    order = np.argsort(arrivals, kind="stable")
    for k in order:
        r = requests[k]
        r.arrival = float(arrivals[k])
        while clock() - t0 < r.arrival:
            time.sleep(10e-6)
        res = runner.run_one(r)
        r.result = res if keep_results else None
        r.t_done = clock() - t0
    return [requests[k] for k in order]


def latency_stats(done, t_first=None):
    lat = np.array([r.latency for r in done])
    if len(lat) == 0:
        return {"n": 0}
    t_first = min(r.arrival for r in done) if t_first is None else t_first
    span = max(r.t_done for r in done) - t_first
    return {"n": int(len(lat)), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "pages_per_s": float(len(lat) / span) if span > 0 else None}
