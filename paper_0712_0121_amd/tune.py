"""Autotuner: tile shapes for the batched launch and the packed-vs-run-length
choice, measured on the device and cached as JSON.

* Tile shape.  Every page of a batch gets (tile_rows, strip_words) from the
  bucket of its row width in words, the height of its element and whether
  its operation has one or two stages (erode/dilate vs open/close).  For each
  bucket the tuner times a small batch of synthetic pages of that shape with
  a few candidate shapes (the library default, shorter tiles, narrower
  strips) and keeps the fastest.
* Representation.  The paper picks between bit-blit and run-length code at
  run time from the mask size and resolution, or from the output complexity
  (section "Experiments", runtime selection including conversion costs).
  Here the tuner times, on batches of pages of a given black density, the
  packed operation against bitmap -> runs -> operation -> bitmap, and
  records the faster one per (density bucket, operation, element size
  class); RoutedBatch and the serving executor route each page by it.

The cache key includes the device name; MORPH_TUNE_CACHE overrides the path.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "morph_tune.json")
H_BUCKETS = (1, 8, 24, 48, 96)             # element heights up to each bound
STRIDE_BUCKETS = (24, 48, 96, 1 << 30)     # words per row up to each bound
DENSITY_BUCKETS = (0.03, 0.2, 1.0)         # black density up to each bound
SIZE_CLASSES = (5, 16, 64, 1 << 30)        # max(w, h) up to each bound
# the elements timed for each size class (the largest class is left to the
# packed path: no entry, so choose_repr answers 'packed')
REPR_SES = (((3, 3, 1, 1),), ((9, 9, 4, 4), (15, 5, 7, 2)),
            ((41, 1, 20, 0), (1, 41, 0, 20), (31, 31, 15, 15)))


def bucket(v, bounds):
    for i, b in enumerate(bounds):
        if v <= b:
            return i
    return len(bounds) - 1


def shape_key(W, H, op, se):
    w, h = se[0], se[1]
    nst = 2 if op in ("open", "close") else 1
    return "s%d_h%d_n%d" % (bucket((W + 63) // 64, STRIDE_BUCKETS), bucket(h, H_BUCKETS), nst)


W_BUCKETS = (1, 4, 16, 64, 1 << 30)        # element widths up to each bound


def strategy_key(op, se):
    return "%s_w%d_h%d" % (op, bucket(se[0], W_BUCKETS), bucket(se[1], H_BUCKETS))


def repr_key(density, op, se):
    return "d%d_%s_k%d" % (bucket(density, DENSITY_BUCKETS), op, bucket(max(se[0], se[1]), SIZE_CLASSES))


class Tuner:
    def __init__(self, cache_path: str | None = None, device="cuda:0"):
        self.path = cache_path or os.environ.get("MORPH_TUNE_CACHE", DEFAULT_CACHE)
        self.device = device
        self.table = {"shape": {}, "repr": {}, "strategy": {}}
        self.arch = None
        self.load()

    # ------------------------------------------------------------ cache
    def _arch(self):
        if self.arch is None:
            import torch
            p = torch.cuda.get_device_properties(self.device)
            self.arch = "%s/%s" % (p.name, getattr(p, "gcnArchName", "gfx"))
        return self.arch

    def load(self):
        try:
            with open(self.path) as f:
                data = json.load(f)
            self.table = data.get(self._arch(), self.table) if data else self.table
            self.table.setdefault("strategy", {})
        except (OSError, ValueError, RuntimeError, AssertionError):
            pass

    def save(self):
        try:
            data = {}
            if os.path.exists(self.path):
                with open(self.path) as f:
                    data = json.load(f)
        except (OSError, ValueError):
            data = {}
        data[self._arch()] = self.table
        os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
        tmp = self.path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    # ------------------------------------------------------------ lookups
    def params(self, W, H, op, se):
        """(tile_rows, strip_words) for a page of the batch; (0, 0) means the
        library default."""
        v = self.table["shape"].get(shape_key(W, H, op, se))
        return tuple(v["best"]) if v else (0, 0)

    # The transposition route moves several bitmap-sized passes per operation
    # where the between-line route moves runs: timed alone it may win by a
    # hair and still cost more when operations share the device.  It is taken
    # only when it is faster by this factor (on the letter batch a near tie
    # taken the other way cost 1 ms of a 15 ms step run on three streams).
    STRATEGY_MARGIN = 1.1

    def choose_strategy(self, op, se):
        """'lines' (within-line passes, then between-line intersections) or
        'transpose' (within-line passes along the rows and, after a
        transposition, along the columns) for an operation on runs."""
        v = self.table.get("strategy", {}).get(strategy_key(op, se))
        if not v:
            return "lines"
        if "lines_ms" in v and "transpose_ms" in v:
            return "transpose" if v["transpose_ms"] * self.STRATEGY_MARGIN < v["lines_ms"] else "lines"
        return v["best"]

    def choose_repr(self, density, op, se):
        """'packed' or 'rle' for a page held packed, conversions included."""
        v = self.table["repr"].get(repr_key(density, op, se))
        return v["best"] if v else "packed"

    # ------------------------------------------------------------ tuning
    def _time(self, fn, reps=5):
        import torch
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            fn()
            e.record()
            torch.cuda.synchronize()
            best = min(best, s.elapsed_time(e))
        return best

    def tune_shapes(self, pages_by_width, ops=("erode", "open"), h_values=(5, 16, 40, 63),
                    batch=32, verbose=False):
        """pages_by_width: {W: (H, host words (rows, stride) uint64)}: a page per
        width class to replicate into a batch of `batch` pages."""
        import torch
        import paper_0712_0121_amd as M
        dev = torch.device(self.device)
        for W, (H, words) in pages_by_width.items():
            src = [M.Bitmap.from_words(words, W, device=dev) for _ in range(batch)]
            dst = [M.Bitmap.empty(W, H, device=dev) for _ in range(batch)]
            nw = (W + 63) // 64
            for op in ops:
                for h in h_values:
                    se = (h, h, h // 2, h // 2)
                    key = shape_key(W, H, op, se)
                    cands = [(0, 0)]
                    for tr in (256, 128, 64, 32):
                        for sw in (0, 40, 20):
                            if sw and sw >= nw:
                                continue
                            cands.append((tr, sw))
                    best, best_t, rows = None, float("inf"), []
                    for c in cands:
                        try:
                            plan = M.BatchPlan([(d, s, op, se, c[0], c[1]) for d, s in zip(dst, src)])
                        except M.MorphError:
                            continue
                        t = self._time(lambda: plan.run(use_graph=False))
                        rows.append((c, t))
                        if t < best_t:
                            best, best_t = c, t
                        plan.close()
                    self.table["shape"][key] = {"best": list(best), "ms": best_t,
                                                "candidates": [[list(c), t] for c, t in rows]}
                    if verbose:
                        print("shape", key, best, "%.3f ms" % best_t)
        return self.table["shape"]

    def tune_repr(self, pages_by_density, ops=("erode", "dilate", "open", "close"), ses_by_class=None,
                  batch=16, verbose=False):
        """pages_by_density: {density: (W, H, host words)}.  For every density,
        operation and element size class, times the representative elements
        of the class on a batch of `batch` stacked copies of the page (a
        batch, not one page that would stay in cache) along both paths: the
        packed operation, and bitmap -> runs -> operation -> bitmap.  The
        path with the smaller summed time wins the (density bucket,
        operation, size class) entry."""
        import torch
        import paper_0712_0121_amd as M
        if ses_by_class is None:
            ses_by_class = REPR_SES
        dev = torch.device(self.device)
        for dens, (W, H, words) in pages_by_density.items():
            host = np.concatenate([words] * batch)
            src = M.Bitmap.from_words(host, W, npages=batch, device=dev)
            del host
            dst = M.Bitmap.empty(W, H, batch, device=dev)
            back = M.Bitmap.empty(W, H, batch, device=dev)
            r_in = M.RLE.empty(W, H, batch, device=dev)
            r_out = M.RLE.empty(W, H, batch, device=dev)
            w_p2r = torch.empty(M.morph_pack_to_rle_workspace_bytes(W, H * batch), dtype=torch.uint8, device=dev)
            for op in ops:
                for ses in ses_by_class:
                    t_pk = t_rle = 0.0
                    for se in ses:
                        w_rle = torch.empty(max(M.morph_rle_workspace_bytes(op, W, H, batch, se), 1),
                                            dtype=torch.uint8, device=dev)
                        n_pk = M.morph_workspace_bytes(op, 0, W, H * batch, se)
                        w_pk = torch.empty(n_pk, dtype=torch.uint8, device=dev) if n_pk else None
                        t_pk += self._time(lambda: M.PACKED[op](dst, src, se, w_pk), 3)

                        def rle_path():
                            M.morph_pack_to_rle(r_in, src, w_p2r)
                            M.RLE_OPS[op](r_out, r_in, se, w_rle)
                            M.morph_rle_to_pack(back, r_out)
                        t_rle += self._time(rle_path, 3)
                        del w_rle, w_pk
                    key = repr_key(dens, op, ses[0])
                    self.table["repr"][key] = {"best": "packed" if t_pk <= t_rle else "rle",
                                               "packed_ms": t_pk, "rle_ms": t_rle, "pages": batch,
                                               "elements": [list(se) for se in ses]}
                    if verbose:
                        print("repr", key, self.table["repr"][key])
            del src, dst, back, r_in, r_out, w_p2r
            torch.cuda.empty_cache()
        return self.table["repr"]

    def tune_strategy(self, src, cases, verbose=False):
        """The paper's two strategies for rectangles on run-length images
        (section "2D Morphological Operators for Rectangular Masks"): within
        lines, then between lines; or within lines along the rows and, after
        a transposition, along the columns.  Times both for every (op,
        element) of `cases` on the run-length batch `src` and records the
        faster per (op, width bucket, height bucket)."""
        import torch
        import paper_0712_0121_amd as M
        dev = src.row_ptr.device
        W, H, P = src.width, src.height, src.npages
        dst = M.RLE.empty(W, H, P, device=dev)
        per_key = {}
        for op, se in cases:
            w_l = torch.empty(max(M.morph_rle_workspace_bytes(op, W, H, P, se), 1), dtype=torch.uint8, device=dev)
            t_l = self._time(lambda: M.RLE_OPS[op](dst, src, se, w_l), 3)
            del w_l
            w_t = torch.empty(max(M.morph_rlet_workspace_bytes(op, W, H, P, se), 1), dtype=torch.uint8, device=dev)
            t_t = self._time(lambda: M.morph_rect_rlet(op, dst, src, se, w_t), 3)
            del w_t
            k = strategy_key(op, se)
            a, b = per_key.get(k, (0.0, 0.0))
            per_key[k] = (a + t_l, b + t_t)
        for k, (t_l, t_t) in per_key.items():
            self.table.setdefault("strategy", {})[k] = {"best": "transpose" if t_t * self.STRATEGY_MARGIN < t_l
                                                        else "lines",
                                                        "lines_ms": t_l, "transpose_ms": t_t, "pages": P}
            if verbose:
                print("strategy", k, self.table["strategy"][k])
        del dst
        torch.cuda.empty_cache()
        return self.table["strategy"]

    def rle_possible(self, op, se):
        """Whether any density bucket sends (op, element size class) to runs:
        callers skip measuring a page's density when none does."""
        k = bucket(max(se[0], se[1]), SIZE_CLASSES)
        suffix = "_%s_k%d" % (op, k)
        return any(key.endswith(suffix) and v.get("best") == "rle" for key, v in self.table["repr"].items())
