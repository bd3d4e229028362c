#!/usr/bin/env python3
"""Benchmark: rectangle morphology of letter pages on one MI355X.

One step runs the whole letter-page workload on a batch of pages that are
already resident in HBM:

* packed path: erode, dilate, open, close with the elements 1x31, 31x1, 3x3,
  21x21 and 51x51 (h x w), each one launch over the whole stacked batch;
* run-length path: bitmap -> runs, the same 20 operations on runs, runs ->
  bitmap of the last result.

It prints one JSON line: Gpixel/s over the step (pixels counted once per
operation and path), the roofline of the dominant kernel measured with HIP
events inside the timed region, and the CPU oracle timed on a sample of the
same work.  Pages are synthetic (seeded), standing in for scanned 300 dpi
letter pages.  Extras beside the step (outside `value`): the mixed batch in
one persistent launch, the representation choice, the serving loop,
transposition and the transpose-based operations, connected components
with the layout composition, and operations by disc-shaped masks.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
LETTER_W, LETTER_H = 2550, 3300
LETTER_SES = [("1x31", (31, 1, 15, 0)), ("31x1", (1, 31, 0, 15)), ("3x3", (3, 3, 1, 1)),
              ("21x21", (21, 21, 10, 10)), ("51x51", (51, 51, 25, 25))]
OPS = ("erode", "dilate", "open", "close")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--pages", type=int, default=256, help="letter pages per batch")
    ap.add_argument("--distinct", type=int, default=16, help="distinct seeded pages in the batch")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="minimum CPU oracle sample time")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--latency-reps", type=int, default=30)
    ap.add_argument("--only", choices=["all", "packed", "rle", "transpose", "components", "masks", "serve"],
                    default="all",
                    help="restrict the step (for profiling); the JSON value needs 'all'; 'transpose', "
                         "'components', 'masks' and 'serve' print only those measurements")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the mixed batch, serving and representation measurements")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--sequential", action="store_true",
                    help="run the packed and the run-length operations of a timed step on one stream")
    ap.add_argument("--rle-lanes", type=int, default=2, choices=(1, 2, 3),
                    help="streams the run-length operations of a timed step are spread over")
    g = ap.add_argument_group("profile summary (no GPU): rocprofv3 CSV output -> markdown")
    g.add_argument("--summarize-profile", action="store_true")
    g.add_argument("--trace-dir", help="rocprofv3 --kernel-trace --stats output directory")
    g.add_argument("--fetch-dir", help="rocprofv3 --pmc FETCH_SIZE output directory")
    g.add_argument("--write-dir", help="rocprofv3 --pmc WRITE_SIZE output directory")
    g.add_argument("--calib-bytes", type=int, default=256 * LETTER_H * 40 * 8,
                   help="bytes the calibration copy reads and writes")
    g.add_argument("--title", default="Kernel time and HBM traffic: letter-page workload, 256 pages")
    g.add_argument("--cmd", action="append", help="profiling command to list in the summary")
    g.add_argument("--out", help="markdown file to write")
    g.add_argument("--summarize-sq", action="store_true",
                   help="SQ counters per kernel (and per packed case with --cases packed) from one --pmc run "
                        "and one --kernel-trace run of the same command")
    g.add_argument("--sq-dir", help="rocprofv3 --pmc output directory with SQ_* counters")
    g.add_argument("--cases", choices=["none", "packed"], default="none",
                   help="also list the last step's packed letter cases, one row per launch")
    return ap.parse_args()


def gen_batch(n, distinct):
    import pagegen
    pool = [pagegen.letter_page(2000 + i) for i in range(distinct)]
    return pool, [pool[i % distinct] for i in range(n)]


def percentile(v, q):
    return float(np.percentile(np.asarray(v), q))


def cpu_model():
    """The host CPU's model name (lscpu's "Model name"), from /proc/cpuinfo."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.lower().startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_workload(img, method):
    """The step's 40 operations on one page by the oracle: the 20 packed
    results (brute force or the summed-area evaluator), the 20 run-length
    results as encode(op(decode(runs))), and the conversions."""
    import oracle
    f = oracle.apply if method == "brute" else oracle.sat_apply
    for _, se in LETTER_SES:
        for op in OPS:
            f(op, img, se)
    rp, runs = oracle.rle_encode(img)
    for _, se in LETTER_SES:
        for op in OPS:
            oracle.rle_apply(op, rp, runs, img.shape[1], img.shape[0], se, method=method)
    last = oracle.rle_encode(f("close", img, LETTER_SES[-1][1]))
    oracle.rle_decode(*last, img.shape[1], img.shape[0])
    return 2 * len(LETTER_SES) * len(OPS) * img.size


def _time_oracle(images, method, min_seconds):
    px, n = 0, 0
    t0 = time.perf_counter()
    while True:
        px += _oracle_workload(images[n % len(images)], method)
        n += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    dt = time.perf_counter() - t0
    return px / dt / 1e9, n, dt


def cpu_baseline(pool, min_seconds):
    """The oracle as it is, timed on the host on bounded samples of the
    step's workload: brute force on all threads (the reported value), brute
    force on one thread (over bands of 128 rows of a page), and the
    summed-area evaluator on all threads and on one, in Gpixel/s."""
    import oracle
    nthreads = oracle.threads()
    v, pages, dt = _time_oracle([p.img for p in pool], "brute", min_seconds)
    band = [p.img[:128].copy() for p in pool[:2]]
    oracle.set_threads(1)
    try:
        v1, n1, dt1 = _time_oracle(band, "brute", min_seconds / 2)
        s1, sn1, sdt1 = _time_oracle([p.img for p in pool], "sat", min_seconds / 4)
    finally:
        oracle.set_threads(nthreads)
    sv, sn, sdt = _time_oracle([p.img for p in pool], "sat", min_seconds / 4)
    return {"value": v, "unit": "Gpixel/s", "cores": nthreads, "kind": "oracle",
            "sample": "%d letter page(s) 2550x3300 through the full workload (20 ops brute force on "
                      "bytes + 20 ops as encode(brute(decode(runs))) + conversions), %.1f s" % (pages, dt),
            "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "one_thread": {"value": v1, "unit": "Gpixel/s", "cores": 1,
                           "sample": "%d band(s) of 2550x128 through the same workload, %.1f s" % (n1, dt1)},
            "sat": {"value": sv, "unit": "Gpixel/s", "cores": nthreads,
                    "sample": "%d letter page(s), the same workload by the summed-area evaluator, %.1f s"
                              % (sn, sdt)},
            "sat_one_thread": {"value": s1, "unit": "Gpixel/s", "cores": 1,
                               "sample": "%d letter page(s), summed-area evaluator, %.1f s" % (sn1, sdt1)}}


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None if there is none or the kernel's source has changed
    since the counters were taken."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "letter_workload_kernels.md")
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    for ln in lines:
        f = ln.split()
        if len(f) >= 5 and f[0] == "traffic" and f[1] == kernel:
            kv = dict(x.split("=", 1) for x in f[2:])
            src = os.path.join(root, kv["source"])
            try:
                cur = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
            except OSError:
                return None
            return float(kv["bytes_per_launch"]) if cur == kv["sha256_16"] else None
    return None


# Kernels whose HBM traffic bench.py reports, with the source file that
# builds each (the traffic figure is used only while that file is unchanged).
TRAFFIC_SOURCES = {
    "rect_kernel": "paper_0712_0121_amd/csrc/packed.hip",
    "col_and_kernel": "paper_0712_0121_amd/csrc/rle.hip",
    "row_erode_kernel": "paper_0712_0121_amd/csrc/rle.hip",
    "pack_rows_kernel": "paper_0712_0121_amd/csrc/rle.hip",
    "col_scan_kernel": "paper_0712_0121_amd/csrc/rle.hip",
    "pack_to_rle_group_kernel": "paper_0712_0121_amd/csrc/rle.hip",
    "rle_to_pack_group_kernel": "paper_0712_0121_amd/csrc/rle.hip",
    "transpose_kernel": "paper_0712_0121_amd/csrc/packed.hip",
    "decode_transpose_kernel": "paper_0712_0121_amd/csrc/rle.hip",
    "rle_band_kernel": "paper_0712_0121_amd/csrc/rle_band.hip",
}
# Trace ids whose events bracket exactly one kernel launch.
SINGLE_LAUNCH = {"rect_kernel", "rect_batch_kernel", "rle_to_pack_kernel", "row_erode_kernel", "col_and_kernel",
                 "transpose_kernel", "decode_transpose_kernel", "col_scan_kernel", "mask_kernel",
                 "mask_and_kernel", "shift_rows_kernel"}
# The calibration kernel: torch's elementwise bitwise_or of the batch with 0
# (a plain copy of known size), picked by the functor in its full name so
# that no other elementwise kernel (clones, compares) enters the scale.
CALIB_TAG = "BitwiseOrFunctor"


def short_kernel_name(name):
    """'void morph::(anonymous namespace)::col_and_kernel<false>(RowsIn, ...)'
    -> 'col_and_kernel'; other names lose their template arguments and
    parameter list."""
    n = name.strip().replace("(anonymous namespace)", "anon")
    if n.startswith("void "):
        n = n[5:]
    depth, out = 0, []
    for ch in n:
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            break
        elif depth == 0:
            out.append(ch)
    n = "".join(out).strip()
    return n.split("::")[-1] if n.startswith("morph::") else n.replace("anon::", "")


def _csv_rows(directory, suffix):
    import csv
    import glob
    rows = []
    for path in sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True)):
        with open(path, newline="") as f:
            rows.extend(csv.DictReader(f))
    if not rows:
        raise SystemExit("no *%s under %s" % (suffix, directory))
    return rows


def _per_dispatch(rows, counter):
    """{dispatch id: (kernel name, summed counter value)} for one counter."""
    out = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        d = r["Dispatch_Id"]
        name, v = out.get(d, (r["Kernel_Name"], 0.0))
        out[d] = (name, v + float(r["Counter_Value"]))
    return out


def summarize_profile(args):
    """Writes the markdown kernel-time and HBM-traffic summary from the CSV
    output of one rocprofv3 --kernel-trace --stats run and one --pmc run each
    for FETCH_SIZE and WRITE_SIZE (KiB per dispatch).  Counter values are
    scaled to bytes by what the same counters read for the calibration copy
    (CALIB_TAG dispatches, calib_bytes read and written each)."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    lines = ["# %s" % args.title, "", "Commands (from the repository root, on one MI355X):", "", "```",
             "export TMPDIR=/tmp"] + list(args.cmd or []) + [
             "python3 bench.py --summarize-profile --trace-dir %s --fetch-dir %s --write-dir %s "
             "--calib-bytes %d --out %s" % (args.trace_dir, args.fetch_dir, args.write_dir, args.calib_bytes,
                                             args.out), "```", ""]
    if args.trace_dir:
        stats = _csv_rows(args.trace_dir, "_kernel_stats.csv")
        tot = sum(float(r["TotalDurationNs"]) for r in stats)
        lines += ["## rocprofv3 --kernel-trace --stats", "", "| kernel | calls | total ms | average us | % |",
                  "|---|---|---|---|---|"]
        grouped = {}
        for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
            name = r["Name"] if len(r["Name"]) <= 100 else r["Name"][:100] + "..."
            lines.append("| %s | %s | %.2f | %.1f | %.1f |" % (name.replace("|", "/"), r["Calls"],
                                                                 float(r["TotalDurationNs"]) / 1e6,
                                                                 float(r["AverageNs"]) / 1e3,
                                                                 100.0 * float(r["TotalDurationNs"]) / tot))
            k = short_kernel_name(r["Name"])
            c, t = grouped.get(k, (0, 0.0))
            grouped[k] = (c + int(r["Calls"]), t + float(r["TotalDurationNs"]))
        lines += ["", "Per kernel, all template instances together (calls, average us): " +
                  "; ".join("%s %d, %.1f" % (k, c, t / c / 1e3) for k, (c, t) in
                            sorted(grouped.items(), key=lambda kv: -kv[1][1]) if k in TRAFFIC_SOURCES), ""]
    fetch = _per_dispatch(_csv_rows(args.fetch_dir, "_counter_collection.csv"), "FETCH_SIZE")
    write = _per_dispatch(_csv_rows(args.write_dir, "_counter_collection.csv"), "WRITE_SIZE")
    cal_f = [v for n, v in fetch.values() if CALIB_TAG in n]
    cal_w = [v for n, v in write.values() if CALIB_TAG in n]
    if not cal_f or not cal_w:
        raise SystemExit("no %s dispatch in the counter runs" % CALIB_TAG)
    kib_f, kib_w = sum(cal_f) / len(cal_f), sum(cal_w) / len(cal_w)
    sf, sw = args.calib_bytes / (kib_f * 1024.0), args.calib_bytes / (kib_w * 1024.0)

    def by_kernel(d):
        g = {}
        for n, v in d.values():
            g.setdefault(short_kernel_name(n), []).append(v)
        return g
    gf, gw = by_kernel(fetch), by_kernel(write)
    lines += ["## HBM traffic per launch (FETCH_SIZE, WRITE_SIZE; per-dispatch means)", "",
              "Scaling: the calibration copy (%d dispatch(es) whose name contains `%s`, %d bytes read and "
              "written each) reads FETCH_SIZE %.0f KiB and WRITE_SIZE %.0f KiB, so FETCH_SIZE x %.3f and "
              "WRITE_SIZE x %.3f give bytes." % (len(cal_f), CALIB_TAG, args.calib_bytes, kib_f, kib_w, sf, sw),
              "", "| kernel | launches | read MB / launch | written MB / launch |", "|---|---|---|---|"]
    traffic = {}
    for k in sorted(set(gf) | set(gw), key=lambda k: -(sum(gf.get(k, [0])) + sum(gw.get(k, [0])))):
        f = gf.get(k, [0.0])
        w = gw.get(k, [0.0])
        rb = sum(f) / len(f) * 1024.0 * sf
        wb = sum(w) / len(w) * 1024.0 * sw
        lines.append("| %s | %d | %.1f | %.1f |" % (k, max(len(f), len(w)), rb / 1e6, wb / 1e6))
        traffic[k] = rb + wb
    lines += ["", "Machine-read lines (bench.py reports `traffic` from these while the kernel source is "
              "unchanged):", ""]
    for k, src in TRAFFIC_SOURCES.items():
        if k in traffic:
            h = hashlib.sha256(open(os.path.join(root, src), "rb").read()).hexdigest()[:16]
            lines.append("traffic %s bytes_per_launch=%.0f source=%s sha256_16=%s" % (k, traffic[k], src, h))
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", args.out)


VALU_ISSUE_PER_S = 256 * 2.4e9      # CU-cycles per second (256 CUs at 2.4 GHz)


def summarize_sq(args):
    """Writes the markdown SQ-counter summary: per library kernel, the SQ
    counters of the --pmc run summed over its dispatches and divided by its
    waves, with the average duration from the --kernel-trace run of the same
    command and the VALU instructions per CU-cycle of that time.
    With --cases packed, also one row per launch of the last step's packed
    letter cases (the last rect_kernel dispatches of both runs, in order)."""
    pmc = _csv_rows(args.sq_dir, "_counter_collection.csv")
    trace = sorted(_csv_rows(args.trace_dir, "_kernel_trace.csv"), key=lambda r: int(r["Start_Timestamp"]))
    disp = {}
    for r in pmc:
        e = disp.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"]})
        e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    counters = sorted({r["Counter_Name"] for r in pmc if r["Counter_Name"].startswith("SQ_")} - {"SQ_WAVES"})
    dur = {}
    for r in trace:
        dur.setdefault(r["Kernel_Name"], []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines = ["# %s" % args.title, "", "Commands (from the repository root, on one MI355X):", "", "```",
             "export TMPDIR=/tmp"] + list(args.cmd or []) + [
             "python3 bench.py --summarize-sq --sq-dir %s --trace-dir %s --cases %s --out %s"
             % (args.sq_dir, args.trace_dir, args.cases, args.out), "```", "",
             "Per kernel: counters summed over its dispatches and divided by its waves; average duration from "
             "the kernel trace. VALU / CU-cycle = VALU instructions per dispatch / (256 CUs x 2.4 GHz x "
             "duration): 1.0 would be one wave64 VALU instruction per CU per cycle. It is an index of how much "
             "of a kernel's time its VALU instructions account for, not a bound: a kernel here reaches more "
             "than 1.0, so part of the mix issues faster than that.", ""]
    head = "| kernel | dispatches | waves / dispatch | " + " | ".join(
        c.replace("SQ_", "").replace("INSTS_", "") + " / wave" for c in counters) + " | average us | VALU / CU-cycle |"
    lines += [head, "|" + "---|" * (len(counters) + 5)]
    groups = {}
    for e in disp.values():
        if "morph::" in e["name"]:          # the library's kernels, not torch's helpers
            groups.setdefault(e["name"], []).append(e)
    for name, es in sorted(groups.items(), key=lambda kv: -sum(x.get("SQ_INSTS_VALU", 0.0) for x in kv[1])):
        waves = sum(x.get("SQ_WAVES", 0.0) for x in es)
        if waves <= 0 or name not in dur:
            continue
        us = sum(dur[name]) / len(dur[name])
        valu = sum(x.get("SQ_INSTS_VALU", 0.0) for x in es) / len(es)
        cells = ["%.1f" % (sum(x.get(c, 0.0) for x in es) / waves) for c in counters]
        lines.append("| %s | %d | %.0f | %s | %.1f | %.2f |" % (
            short_kernel_name(name).replace("anon::", "") + ("<%s>" % name.split("<")[1].split(">")[0]
                                                              if "<" in name else ""),
            len(es), waves / len(es), " | ".join(cells), us, valu / VALU_ISSUE_PER_S / (us * 1e-6)))
    if args.cases == "packed":
        import paper_0712_0121_amd as M
        labels = []
        for name, se in LETTER_SES:
            for op in OPS:
                split = M.morph_workspace_bytes(op, M.MORPH_PACKED, LETTER_W, LETTER_H * args.pages, se) > 0
                labels += ["%s %s (%d/2)" % (op, name, i + 1) for i in range(2)] if split else ["%s %s" % (op, name)]
        rk = [k for k in sorted(disp) if "rect_kernel" in disp[k]["name"]][-len(labels):]
        rt = [r for r in trace if "rect_kernel" in r["Kernel_Name"]][-len(labels):]
        lines += ["", "The last step's packed letter cases, one row per launch:", "",
                  "| case | threads | us | VALU / wave | SALU / wave | LDS / wave | LDS bank conflict / wave "
                  "| VALU / CU-cycle |", "|---|---|---|---|---|---|---|---|"]
        for lab, k, t in zip(labels, rk, rt):
            e = disp[k]
            w = e.get("SQ_WAVES", 1.0)
            us = (int(t["End_Timestamp"]) - int(t["Start_Timestamp"])) / 1e3
            lines.append("| %s | %s | %.1f | %.0f | %.0f | %.0f | %.0f | %.2f |" % (
                lab, t["Kernel_Name"].split("<")[1].split(">")[0], us, e.get("SQ_INSTS_VALU", 0.0) / w,
                e.get("SQ_INSTS_SALU", 0.0) / w, e.get("SQ_INSTS_LDS", 0.0) / w,
                e.get("SQ_LDS_BANK_CONFLICT", 0.0) / w,
                e.get("SQ_INSTS_VALU", 0.0) / VALU_ISSUE_PER_S / (us * 1e-6)))
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", args.out)


def time_ms(fn, reps=5):
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def bench_batched(M, dev, tuner, n=256):
    """Mixed batch: n pages sized 1275x1650, 2480x3508, 2550x3300 or 5100x6600,
    each with its own random element (w, h in [1, 63], centred) and operation:
    per-page launches vs one persistent launch (graph replay), library default
    tiles and autotuned tiles."""
    import pagegen
    items = pagegen.mixed_batch(n, seed=3000, pool_per_size=4)
    cache = {}
    srcs, dsts = [], []
    for it in items:
        key = id(it.page)
        if key not in cache:
            cache[key] = it.page.words()
        srcs.append(M.Bitmap.from_words(cache[key], it.page.W, device=dev))
        dsts.append(M.Bitmap.empty(it.page.W, it.page.H, device=dev))
    px = sum(it.page.W * it.page.H for it in items)
    alg = sum(2 * 8 * ((it.page.W + 63) // 64) * it.page.H for it in items)

    import torch
    ws_n = max([1] + [M.morph_workspace_bytes(it.op, 0, it.page.W, it.page.H, it.se) for it in items])
    ws_pp = torch.empty(ws_n, dtype=torch.uint8, device=dev)      # one page's split operations at a time

    def per_page():
        for it, s_, d_ in zip(items, srcs, dsts):
            M.PACKED[it.op](d_, s_, it.se, ws_pp)
    t_pp = time_ms(per_page, 3)
    plan = M.BatchPlan([(d_, s_, it.op, it.se) for it, s_, d_ in zip(items, srcs, dsts)])
    t_b = time_ms(lambda: plan.run(use_graph=True))
    widths = {}
    for it in items:
        widths.setdefault(it.page.W, (it.page.H, cache[id(it.page)]))
    t0 = time.perf_counter()
    tuner.tune_shapes(widths, ops=("erode", "open"), h_values=(5, 16, 40, 63), batch=16)
    tune_s = time.perf_counter() - t0
    tuned = []
    for it, s_, d_ in zip(items, srcs, dsts):
        tr, sw = tuner.params(it.page.W, it.page.H, it.op, it.se)
        tuned.append((d_, s_, it.op, it.se, tr, sw))
    plan_t = M.BatchPlan(tuned)
    t_t = time_ms(lambda: plan_t.run(use_graph=True))
    # the representation choice per page (density counted on the device,
    # the tuner's packed-vs-runs table), then the routed batch timed
    routed = M.RoutedBatch(tuned, tuner=tuner)
    t_r = time_ms(lambda: routed.run(use_graph=True))
    dens = routed.densities
    ex = lambda ms: {"ms": ms, "gpixel_s": px / (ms / 1e3) / 1e9, "hbm_gbs": alg / (ms / 1e3) / 1e9,
                     "hbm_frac": alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}
    return {"pages": n, "gpixel": px / 1e9, "alg_bytes": alg, "per_page_launches": ex(t_pp),
            "persistent_graph": ex(t_b), "persistent_graph_tuned": ex(t_t),
            "routed": dict(ex(t_r), routes=routed.route_counts(),
                           density_min=min(dens), density_max=max(dens)),
            "tiles": plan.tiles,
            "tiles_tuned": plan_t.tiles, "tune_seconds": tune_s}


class _frozen_requests:
    """A trace's requests are all built before it starts and kept until its
    statistics are taken, which a server does not do (it drops a request
    once answered).  For the trace they are moved out of the collector's
    reach, with everything else alive, so that its full passes walk only what
    the serving loop allocates; otherwise one pass over some 200k objects
    (mostly torch's own) stalls the scheduler for ~100 ms, which the p99 of
    a 5 s trace then reports."""

    def __enter__(self):
        import gc
        gc.collect()
        gc.freeze()

    def __exit__(self, *exc):
        import gc
        gc.unfreeze()


def bench_serving(M, dev, seconds, tuner=None):
    """Serving: Poisson arrivals of pages sized as in the mixed batch, each with
    the chain close 1x41 -> open 3x3 -> dilate 15x5 -> erode 15x5, under a 64 GB
    HBM budget; served (continuous batching) vs plain per-page path on the
    same trace.  Plain saturation: a burst of requests at time 0 (it serves
    one page at a time); served saturation: the highest Poisson arrival rate
    it keeps up with, by bisection."""
    import torch
    import pagegen
    from paper_0712_0121_amd import serve
    pool = []
    for (W, H) in pagegen.PAGE_SIZES:
        for k in range(4):
            p = pagegen.text_page(5000 + 10 * len(pool) + k, W, H)
            pool.append((W, H, torch.from_numpy(p.words().view(np.int64)).pin_memory()))
    chain = serve.chain_ses(serve.SERVE_CHAIN)
    rng = np.random.default_rng(5000)

    def reqs(n):
        out = []
        for i in range(n):
            W, H, w = pool[int(rng.integers(len(pool)))]
            out.append(serve.Request(i, W, H, w, chain))
        return out

    budget = 64 << 30
    runner = serve.PlainRunner(dev)
    ex = serve.GpuExecutor(dev, recycle_outputs=True, tuner=tuner)     # results are not kept
    # warm both paths (first launches, allocator pools), then measure
    # saturation with bursts of requests all arriving at time 0
    serve.run_trace_plain(runner, reqs(64), np.zeros(64), keep_results=False)
    serve.run_trace_served(serve.Server(ex, budget, keep_results=False), reqs(128),
                           np.zeros(128))
    # each burst runs twice and the second is timed: the first sizes the
    # pinned result pools and the allocators for that many pages in flight
    for rep in range(2):
        burst = reqs(512)
        with _frozen_requests():
            t = time.perf_counter()
            serve.run_trace_plain(runner, burst, np.zeros(len(burst)), keep_results=False)
            p0 = len(burst) / (time.perf_counter() - t)
    for rep in range(2):
        burst = reqs(1024)
        with _frozen_requests():
            srv = serve.Server(ex, budget, keep_results=False)
            t = time.perf_counter()
            serve.run_trace_served(srv, burst, np.zeros(len(burst)))
            p1_burst = len(burst) / (time.perf_counter() - t)
    # served saturation: the highest Poisson arrival rate the served path
    # keeps up with (p99 under 20 ms over a 1.5 s trace), by bisection
    # between the plain saturation and 1.5x the larger of it and the burst
    # rate (the burst rate alone varies too much to bound the search).  The
    # completion rate under overload overstates it: an overloaded server
    # forms larger batches than arrivals at 90 % of capacity do
    def sustained(rate, seed):
        arrivals = pagegen.poisson_trace(rate, 1.5, seed=seed)
        rq = reqs(len(arrivals))
        with _frozen_requests():
            srv = serve.Server(ex, budget, keep_results=False)
            serve.run_trace_served(srv, rq, arrivals, timeout=120)
        st = serve.latency_stats(srv.completed, 0.0)
        return st["p99_ms"] < 20.0, st["p99_ms"]
    lo, hi = p0, 1.5 * max(p0, p1_burst)
    probes = []
    for k in range(5):
        mid = 0.5 * (lo + hi)
        ok, p99 = sustained(mid, 5002 + k)
        probes.append({"qps": mid, "p99_ms": p99, "kept_up": ok})
        if ok:
            lo = mid
        else:
            hi = mid
    p1 = lo
    print("serving: saturation plain %.0f, served %.0f pages/s" % (p0, p1), file=sys.stderr, flush=True)
    points = []
    # the fourth point holds the device to a budget of about four of the
    # largest pages' buffer pairs, so that admission waits for memory
    small = 4 * 2 * 6600 * 80 * 8
    for name, qps, bud in (("0.5x plain saturation", 0.5 * p0, budget), ("0.9x plain saturation", 0.9 * p0, budget),
                           ("0.9x served saturation", 0.9 * p1, budget),
                           ("0.9x served saturation, %.0f MB budget" % (small / 1e6), 0.9 * p1, small)):
        arrivals = pagegen.poisson_trace(qps, seconds, seed=5001)
        served = reqs(len(arrivals))
        with _frozen_requests():
            srv = serve.Server(ex, bud, keep_results=False)
            serve.run_trace_served(srv, served, arrivals, timeout=seconds * 20 + 60)
        plain = None
        if bud == budget:               # the plain path keeps one page on the device: no budget
            plain = reqs(len(arrivals))
            with _frozen_requests():
                serve.run_trace_plain(runner, plain, arrivals, keep_results=False)
        print("serving: %s, %d requests done" % (name, len(arrivals)), file=sys.stderr, flush=True)
        points.append({"load": name, "qps": qps, "requests": len(arrivals), "budget_gb": bud / 2**30,
                       "served": serve.latency_stats(srv.completed, 0.0),
                       "plain": serve.latency_stats(plain, 0.0) if plain is not None else None,
                       "served_launches": srv.launches, "served_peak_hbm_gb": srv.peak_used / 2**30})
    # device-only latency: the chain's launches on one resident page, no
    # copies and no queueing, page by page (the plain path is warm by now)
    runner.timing = True
    for r in reqs(200):
        runner.run_one(r)
    runner.timing = False
    dev_ms = np.array(runner.device_ms)
    return {"chain": "close 1x41 -> open 3x3 -> dilate 15x5 -> erode 15x5", "budget_gb": 64,
            "operations_routed_to_runs": ex.rle_ops,
            "seconds_per_trace": seconds,
            "device_only_ms": {"n": int(len(dev_ms)), "p50": float(np.percentile(dev_ms, 50)),
                               "p99": float(np.percentile(dev_ms, 99)), "max": float(dev_ms.max())},
            "saturation_pages_s": {"plain": p0, "served": p1, "served_burst": p1_burst},
            # false when every probe held: "served" is then only a lower bound
            "served_saturation_bounded": any(not q["kept_up"] for q in probes),
            "served_saturation_probes": probes,
            "load_points": points}


def bench_transpose(M, dev, src, rle_ms_per_op):
    """Transposition and the transpose-based ("rlet") rectangle operations on
    the letter batch: the packed transpose, the run-length transpose, and the
    20 operations on runs by within-line passes plus transposition, beside
    the run-length path's own times for the same operations."""
    import torch
    W, H, B = src.width, src.height, src.npages
    nw, nk = (W + 63) // 64, (H + 63) // 64
    tdst = M.Bitmap.empty(H, W, B, device=dev)
    t_pk = time_ms(lambda: M.morph_transpose_packed(tdst, src), 5)
    alg_pk = 8 * B * (nw * H + nk * W)
    del tdst
    r_in = M.RLE.empty(W, H, B, device=dev)
    ws_p2r = torch.empty(M.morph_pack_to_rle_workspace_bytes(W, H * B), dtype=torch.uint8, device=dev)
    M.morph_pack_to_rle(r_in, src, ws_p2r)
    del ws_p2r
    r_t = M.RLE.empty(H, W, B, device=dev)
    ws_t = torch.empty(M.morph_transpose_rle_workspace_bytes(W, H, B), dtype=torch.uint8, device=dev)
    t_rt = time_ms(lambda: M.morph_transpose_rle(r_t, r_in, ws_t), 3)
    with M.Trace() as tr:
        M.morph_transpose_rle(r_t, r_in, ws_t)
    runs_in, runs_t = int(r_in.row_ptr[-1].item()), int(r_t.row_ptr[-1].item())
    del r_t, ws_t
    torch.cuda.empty_cache()
    r_out = M.RLE.empty(W, H, B, device=dev)
    ws_n = max(M.morph_rlet_workspace_bytes(op, W, H, B, se) for op in OPS for _, se in LETTER_SES)
    ws = torch.empty(ws_n, dtype=torch.uint8, device=dev)
    per = {}
    for name, se in LETTER_SES:
        for op in OPS:
            per["%s %s" % (op, name)] = round(time_ms(lambda: M.morph_rect_rlet(op, r_out, r_in, se, ws), 2), 4)
    with M.Trace() as tr2:
        for name, se in LETTER_SES:
            for op in OPS:
                M.morph_rect_rlet(op, r_out, r_in, se, ws)
    del r_out, ws, r_in
    torch.cuda.empty_cache()
    kern = lambda res: {k: {"launches": v["launches"], "ms": round(v["ms"], 4),
                            "gbs": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1) if v["ms"] else None}
                        for k, v in res.items()}
    px = W * H * B
    rlet_ms = sum(per.values())
    out = {"pages": B,
           "packed_transpose": {"ms": t_pk, "alg_bytes": alg_pk, "gbs": alg_pk / (t_pk / 1e3) / 1e9,
                                "hbm_frac": alg_pk / (t_pk / 1e3) / 1e9 / HBM_PEAK_GBS},
           "rle_transpose": {"ms": t_rt, "gpixel_s": px / (t_rt / 1e3) / 1e9, "runs_in": runs_in,
                             "runs_out": runs_t, "kernels": kern(tr.result)},
           "rlet": {"ms_ops": rlet_ms, "gpixel_s": len(per) * px / (rlet_ms / 1e3) / 1e9, "ms_per_op": per,
                    "kernels": kern(tr2.result)}}
    if rle_ms_per_op:
        out["rlet"]["rle_ms_per_op"] = rle_ms_per_op
        out["rlet"]["rle_ms_ops"] = sum(rle_ms_per_op.values())
    return out


def bench_components(M, dev, src):
    """Connected components (8-connectivity), component statistics and
    run-length histograms of the letter batch on runs, and the layout
    composition (spacing estimate, dilation, components, boxes) end to end.
    Algorithmic bytes: labelling reads 8 B per run and 4 B per row count and
    writes 4 B per label; statistics read 8 + 4 B per run and write 40 B per
    component; histograms read 8 B per run."""
    import torch
    W, H, B = src.width, src.height, src.npages
    r = M.RLE.empty(W, H, B, device=dev)
    ws_p2r = torch.empty(M.morph_pack_to_rle_workspace_bytes(W, H * B), dtype=torch.uint8, device=dev)
    M.morph_pack_to_rle(r, src, ws_p2r)
    del ws_p2r
    n = r.nruns()
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    comp_ptr = torch.empty(B + 1, dtype=torch.int32, device=dev)
    ws = torch.empty(M.morph_rle_label_workspace_bytes(H * B, n), dtype=torch.uint8, device=dev)
    t_lab = time_ms(lambda: M.morph_rle_label(r, 8, labels, n, comp_ptr, ws), 5)
    nc = int(comp_ptr[-1].item())
    st = torch.empty((max(nc, 1), 10), dtype=torch.int32, device=dev)
    t_st = time_ms(lambda: M.morph_rle_component_stats(r, labels, n, comp_ptr, st, nc), 5)
    bl = torch.empty((B, W + 1), dtype=torch.int32, device=dev)
    wh = torch.empty_like(bl)
    t_h = time_ms(lambda: M.morph_rle_run_histograms(r, bl, wh), 5)
    del ws, st, bl, wh
    torch.cuda.empty_cache()
    M.layout_boxes(r)                           # warm-up (allocations)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        gx, gy, boxes, sums, cp = M.layout_boxes(r)
    torch.cuda.synchronize()
    t_lay = (time.perf_counter() - t0) * 1e3 / reps
    with M.Trace() as tr:
        M.layout_boxes(r)
    px = W * H * B
    gbs = lambda b, ms: b / (ms / 1e3) / 1e9
    b_lab = 12.0 * n + 4.0 * (H * B + 1)
    b_st = 12.0 * n + 40.0 * nc
    out = {"pages": B, "runs": n, "components": nc,
           "label": {"ms": t_lab, "gpixel_s": px / (t_lab / 1e3) / 1e9, "alg_bytes": b_lab,
                     "gbs": gbs(b_lab, t_lab), "hbm_frac": gbs(b_lab, t_lab) / HBM_PEAK_GBS},
           "stats": {"ms": t_st, "alg_bytes": b_st, "gbs": gbs(b_st, t_st)},
           "histograms": {"ms": t_h, "gbs": gbs(8.0 * n, t_h)},
           "layout": {"ms_wall": t_lay, "pages_s": B / (t_lay / 1e3), "gx": gx, "gy": gy,
                      "blocks": int(cp[-1].item()),
                      "kernels": {k: {"launches": v["launches"], "ms": round(v["ms"], 4)}
                                  for k, v in tr.result.items()}}}
    del r, labels, comp_ptr
    torch.cuda.empty_cache()
    return out


MASK_RADII = (3, 10)


def bench_masks(M, dev, src):
    """Erosion, dilation, opening and closing of the letter batch by discs of
    radius 3 and 10 (7 x 7 and 21 x 21 masks), on both paths: Gpixel/s, and
    for the packed kernel the algorithmic bytes (one read and one write of
    the batch per operation) against the HBM peak."""
    import torch
    W, H, B = src.width, src.height, src.npages
    nw = (W + 63) // 64
    r_in = M.RLE.empty(W, H, B, device=dev)
    ws_p2r = torch.empty(M.morph_pack_to_rle_workspace_bytes(W, H * B), dtype=torch.uint8, device=dev)
    M.morph_pack_to_rle(r_in, src, ws_p2r)
    del ws_p2r
    dst = M.Bitmap.empty(W, H, B, device=dev)
    r_out = M.RLE.empty(W, H, B, device=dev)
    px = W * H * B
    alg = 16.0 * nw * H * B
    out = {"pages": B}
    for rad in MASK_RADII:
        j, i = np.mgrid[0:2 * rad + 1, 0:2 * rad + 1]
        mk = M.Mask(((i - rad) ** 2 + (j - rad) ** 2 <= rad * rad).astype(np.uint8), rad, rad)
        ws_pk = torch.empty(max(M.morph_mask_workspace_bytes("open", 0, W, H, B, mk), 256), dtype=torch.uint8,
                            device=dev)
        ws_rl = torch.empty(M.morph_mask_workspace_bytes("open", 1, W, H, B, mk), dtype=torch.uint8, device=dev)
        res = {}
        for op in OPS:
            tp = time_ms(lambda: M.morph_mask_packed(op, dst, src, mk, ws_pk), 3)
            tr = time_ms(lambda: M.morph_mask_rle(op, r_out, r_in, mk, ws_rl), 2)
            launches = 2 if op in ("open", "close") else 1
            res[op] = {"packed_ms": round(tp, 4), "rle_ms": round(tr, 4),
                       "packed_gpixel_s": px / (tp / 1e3) / 1e9, "rle_gpixel_s": px / (tr / 1e3) / 1e9,
                       "packed_hbm_frac": launches * alg / (tp / 1e3) / 1e9 / HBM_PEAK_GBS}
        out["disc%d" % rad] = res
        del ws_pk, ws_rl
        torch.cuda.empty_cache()
    del r_in, r_out, dst
    torch.cuda.empty_cache()
    return out


def bench_density(M, dev, pages=64, distinct=4):
    """Run-length density sweep: batches of 64 letter-size pages at 1 %, 10 %
    and 40 % black (rectangles plus XOR noise, about 2, 20 and 60 runs per
    row), erosion and dilation by 1x41 (horizontal) and 41x1 (vertical):
    runs resident, bitmap -> runs -> operation -> bitmap end to end, and the
    packed path on the same pages, plus the conversions alone.  %HBM is on
    the algorithmic bytes: 8 B per run in and out and 4 B per row offset of
    each for runs, one read and one write of the words for packed."""
    import torch
    import pagegen
    W, H, P = LETTER_W, LETTER_H, pages
    nw = (W + 63) // 64
    ses = (("1x41", (41, 1, 20, 0)), ("41x1", (1, 41, 0, 20)))
    out = {}
    for d in (0.01, 0.10, 0.40):
        pool = [pagegen.density_page(d, 4000 + i).words() for i in range(distinct)]
        host = np.concatenate([pool[i % distinct] for i in range(P)])
        src = M.Bitmap.from_words(host, W, npages=P, device=dev)
        del host, pool
        dst = M.Bitmap.empty(W, H, P, device=dev)
        ws_c = torch.empty(max(M.morph_pack_to_rle_workspace_bytes(W, H * P), 1), dtype=torch.uint8, device=dev)
        r_in = M.RLE.empty(W, H, P, device=dev)
        r_out = M.RLE.empty(W, H, P, device=dev)
        M.morph_pack_to_rle(r_in, src, ws_c)
        n_in = int(r_in.row_ptr[-1].item())
        px = W * H * P
        img_b = 2.0 * nw * 8 * H * P
        t_p2r = time_ms(lambda: M.morph_pack_to_rle(r_in, src, ws_c))
        t_r2p = time_ms(lambda: M.morph_rle_to_pack(dst, r_in))
        row = {"runs_per_row": n_in / (H * P), "black": float(d),
               "pack_to_rle_ms": t_p2r, "rle_to_pack_ms": t_r2p, "ops": {}}
        for name, se in ses:
            for op in ("erode", "dilate"):
                ws_r = torch.empty(max(M.morph_rle_workspace_bytes(op, W, H, P, se), 1), dtype=torch.uint8, device=dev)
                wsp_n = M.morph_workspace_bytes(op, 0, W, H * P, se)
                ws_p = torch.empty(wsp_n, dtype=torch.uint8, device=dev) if wsp_n else None
                t_rle = time_ms(lambda: M.RLE_OPS[op](r_out, r_in, se, ws_r))
                n_out = int(r_out.row_ptr[-1].item())
                b_rle = 8.0 * (n_in + n_out) + 8.0 * (H * P + 1)

                def e2e():
                    M.morph_pack_to_rle(r_in, src, ws_c)
                    M.RLE_OPS[op](r_out, r_in, se, ws_r)
                    M.morph_rle_to_pack(dst, r_out)
                t_e2e = time_ms(e2e)
                t_pk = time_ms(lambda: M.PACKED[op](dst, src, se, ws_p))
                row["ops"]["%s %s" % (op, name)] = {
                    "rle_ms": t_rle, "rle_gpixel_s": px / (t_rle / 1e3) / 1e9,
                    "rle_hbm_frac": b_rle / (t_rle / 1e3) / 1e9 / HBM_PEAK_GBS, "runs_out": n_out,
                    "end_to_end_ms": t_e2e, "end_to_end_gpixel_s": px / (t_e2e / 1e3) / 1e9,
                    "packed_ms": t_pk, "packed_gpixel_s": px / (t_pk / 1e3) / 1e9,
                    "packed_hbm_frac": img_b / (t_pk / 1e3) / 1e9 / HBM_PEAK_GBS,
                    "faster": "rle" if t_rle < t_pk else "packed"}
                del ws_r, ws_p
        out["%d%%" % round(100 * d)] = row
        del src, dst, r_in, r_out, ws_c
        torch.cuda.empty_cache()
    return {"pages": P, "distinct": distinct, "densities": out}


def bench_small(M, dev, reps=50):
    """One 512x512 image (8 words per row; rectangles of 3-12 px along text
    lines, 8 % black, salt noise): single-image latency of erosion and
    dilation by 3x3, 9x1 (nine rows) and 1x9 on both paths, in microseconds
    and Gpixel/s.  A page this small stays in cache: these are latencies."""
    import torch
    import pagegen
    p = pagegen.small_page(1000)
    src = M.Bitmap.from_words(p.words(), p.W, device=dev)
    dst = M.Bitmap.empty(p.W, p.H, device=dev)
    r_in = M.pack_to_rle(src)
    r_out = M.RLE.empty(p.W, p.H, device=dev)
    out = {}
    for name, se in (("3x3", (3, 3, 1, 1)), ("9x1", (1, 9, 0, 4)), ("1x9", (9, 1, 4, 0))):
        for op in ("erode", "dilate"):
            wsp_n = M.morph_workspace_bytes(op, 0, p.W, p.H, se)
            ws_p = torch.empty(wsp_n, dtype=torch.uint8, device=dev) if wsp_n else None
            ws_r = torch.empty(max(M.morph_rle_workspace_bytes(op, p.W, p.H, 1, se), 1), dtype=torch.uint8, device=dev)
            t_pk = time_ms(lambda: M.PACKED[op](dst, src, se, ws_p), reps)
            t_rl = time_ms(lambda: M.RLE_OPS[op](r_out, r_in, se, ws_r), reps)
            out["%s %s" % (op, name)] = {"packed_us": t_pk * 1e3, "rle_us": t_rl * 1e3,
                                         "packed_gpixel_s": p.W * p.H / (t_pk / 1e3) / 1e9,
                                         "rle_gpixel_s": p.W * p.H / (t_rl / 1e3) / 1e9}
    return {"image": "512x512, %.1f%% black" % (100.0 * p.img.mean()), "ops": out}


def bench_repr(M, dev, tuner):
    """Bitmap vs run-length choice on batches of 16 2550x3300 pages at 1%,
    10%, 40% black (conversions included), as the autotuner records it; the
    mixed batch routes its pages by this table."""
    import pagegen
    pages = {}
    for d in (0.01, 0.10, 0.40):
        p = pagegen.density_page(d, 4000)
        pages[d] = (p.W, p.H, p.words())
    tab = tuner.tune_repr(pages)
    return {k: v for k, v in sorted(tab.items())}


def main():
    args = parse()
    if args.summarize_profile:
        summarize_profile(args)
        return
    if args.summarize_sq:
        summarize_sq(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported (run --gpus 1)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_0712_0121_amd as M

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    B = args.pages
    pool, batch = gen_batch(B, args.distinct)
    W, H = LETTER_W, LETTER_H
    nw = (W + 63) // 64
    words_pool = [torch.from_numpy(p.words().view(np.int64)) for p in pool]
    host = torch.cat([words_pool[i % len(pool)] for i in range(B)], dim=0)
    src = M.Bitmap(host.to(dev), W, H, B)
    if args.only == "serve":
        # the serving workload alone (traces of --serve-seconds each)
        from paper_0712_0121_amd.tune import Tuner
        res = bench_serving(M, dev, args.serve_seconds, Tuner(device="cuda:0"))
        print(json.dumps({"serving": res}), flush=True)
        return
    if args.only in ("transpose", "components", "masks"):
        del host
        res = {"transpose": lambda: bench_transpose(M, dev, src, None), "components": lambda: bench_components(M, dev, src),
               "masks": lambda: bench_masks(M, dev, src)}[args.only]()
        # the elementwise copy whose HBM counters calibrate the profiles
        cal = torch.empty_like(src.words)
        torch.bitwise_or(src.words, 0, out=cal)
        torch.cuda.synchronize()
        print(json.dumps({args.only: res}), flush=True)
        return
    dst = M.Bitmap.empty(W, H, B, device=dev)
    back = M.Bitmap.empty(W, H, B, device=dev)
    del host
    max_runs = M.morph_rle_max_runs(W, H * B)
    rle_src = M.RLE.empty(W, H, B, capacity=max_runs, device=dev)
    rle_dst = M.RLE.empty(W, H, B, capacity=max_runs, device=dev)
    ws_rle_n = max(M.morph_rle_workspace_bytes(op, W, H, B, se) for op in OPS for _, se in LETTER_SES)
    ws_rle = torch.empty(ws_rle_n, dtype=torch.uint8, device=dev)
    ws_p2r = torch.empty(M.morph_pack_to_rle_workspace_bytes(W, H * B), dtype=torch.uint8, device=dev)
    ws_pk_n = max(M.morph_workspace_bytes(op, 0, W, H * B, se) for op in OPS for _, se in LETTER_SES)
    ws_pk = torch.empty(max(ws_pk_n, 1), dtype=torch.uint8, device=dev) if ws_pk_n else None
    stream = torch.cuda.current_stream()

    packed_jobs = [(op, name, se) for name, se in LETTER_SES for op in OPS]
    do_packed = args.only in ("all", "packed")
    do_rle = args.only in ("all", "rle")
    # the strategy of each operation on runs, picked by the autotuner from
    # timings on this batch (untimed): within lines then between lines, or
    # within lines along the rows and the columns around a transposition
    from paper_0712_0121_amd.tune import Tuner
    tuner = Tuner(device="cuda:0")
    strategy = {}
    ws_rlet = None
    if do_rle:
        M.morph_pack_to_rle(rle_src, src, ws_p2r)
        tuner.tune_strategy(rle_src, [(op, se) for op, _, se in packed_jobs])
        strategy = {(op, name): tuner.choose_strategy(op, se) for op, name, se in packed_jobs}
        n_t = max([0] + [M.morph_rlet_workspace_bytes(op, W, H, B, se) for op, name, se in packed_jobs
                         if strategy[(op, name)] == "transpose"])
        ws_rlet = torch.empty(n_t, dtype=torch.uint8, device=dev) if n_t else None

    side = torch.cuda.Stream(device=dev)       # default priority

    def rle_call(op, name, se, d, w_l, w_t):
        if strategy[(op, name)] == "transpose":
            M.morph_rect_rlet(op, d, rle_src, se, w_t)
        else:
            M.RLE_OPS[op](d, rle_src, se, w_l)

    # The run-length operations of a step are independent of one another
    # (one input, results not reused): with their own output and workspaces,
    # further lanes run part of them on streams of their own.  Each operation
    # is timed once here and the lanes are filled longest first.
    lanes = args.rle_lanes if (do_rle and not args.sequential) else 1
    lane_of = {}
    lane_bufs = [(rle_dst, ws_rle, ws_rlet)]
    lane_streams = []
    if do_rle and lanes > 1:
        for _ in range(lanes - 1):
            lane_bufs.append((M.RLE.empty(W, H, B, capacity=max_runs, device=dev),
                              torch.empty(ws_rle_n, dtype=torch.uint8, device=dev),
                              torch.empty(ws_rlet.numel(), dtype=torch.uint8, device=dev)
                              if ws_rlet is not None else None))
            lane_streams.append(torch.cuda.Stream(device=dev))     # default priority
        est = {}
        for op, name, se in packed_jobs:
            rle_call(op, name, se, rle_dst, ws_rle, ws_rlet)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rle_call(op, name, se, rle_dst, ws_rle, ws_rlet)
            torch.cuda.synchronize()
            est[(op, name)] = time.perf_counter() - t0
        load = [0.0] * lanes
        for key in sorted(est, key=lambda k: -est[k]):
            ln = min(range(lanes), key=lambda i: load[i])
            lane_of[key] = ln
            load[ln] += est[key]

    def step(ev=None, conc=False):
        # conc: the packed operations run on a second stream beside the
        # run-length chain (independent inputs and outputs), joined at the end
        cur = torch.cuda.current_stream()
        conc = conc and do_packed and do_rle and ev is None
        if conc:
            side.wait_stream(cur)
            with torch.cuda.stream(side):
                for op, _, se in packed_jobs:
                    M.PACKED[op](dst, src, se, ws_pk)
        elif do_packed:
            for k, (op, _, se) in enumerate(packed_jobs):
                if ev is not None:
                    ev["pk"][k][0].record(stream)
                M.PACKED[op](dst, src, se, ws_pk)
                if ev is not None:
                    ev["pk"][k][1].record(stream)
        if do_rle:
            if ev is not None:
                ev["p2r"][0].record(stream)
            M.morph_pack_to_rle(rle_src, src, ws_p2r)
            if ev is not None:
                ev["p2r"][1].record(stream)
            multi = conc and lanes > 1
            if multi:
                for ln, st in enumerate(lane_streams, start=1):
                    st.wait_stream(cur)
                    d, w_l, w_t = lane_bufs[ln]
                    with torch.cuda.stream(st):
                        for op, name, se in packed_jobs:
                            if lane_of[(op, name)] == ln:
                                rle_call(op, name, se, d, w_l, w_t)
            for k, (op, name, se) in enumerate(packed_jobs):
                if multi and lane_of[(op, name)] != 0:
                    continue
                if ev is not None:
                    ev["rle"][k][0].record(stream)
                rle_call(op, name, se, rle_dst, ws_rle, ws_rlet)
                if ev is not None:
                    ev["rle"][k][1].record(stream)
            if ev is not None:
                ev["r2p"][0].record(stream)
            M.morph_rle_to_pack(back, rle_dst)
            if ev is not None:
                ev["r2p"][1].record(stream)
            if multi:
                for st in lane_streams:
                    cur.wait_stream(st)
        if conc:
            cur.wait_stream(side)

    def new_events():
        E = lambda: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        return {"pk": [E() for _ in packed_jobs], "rle": [E() for _ in packed_jobs], "p2r": E(), "r2p": E()}

    conc = not args.sequential
    for _ in range(args.warmup):
        step(conc=conc)
    torch.cuda.synchronize()
    # the timed steps: nothing but the library calls on the stream(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(conc=conc)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same step captured once into a HIP graph and replayed (no entry
    # point allocates, synchronises or records a memset); its outputs must
    # equal the eager step's byte for byte
    graph_check = {}
    outs = lambda: (dst.words, back.words, rle_src.row_ptr, rle_src.runs) + tuple(
        t for d, _, _ in lane_bufs for t in (d.row_ptr, d.runs))
    eager_out = [t.clone() for t in outs()]
    g_step = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_step):
        step(conc=conc)
    for _ in range(args.warmup):
        g_step.replay()
    torch.cuda.synchronize()
    tg = time.perf_counter()
    for s in range(args.steps):
        g_step.replay()
    torch.cuda.synchronize()
    dt_graph = time.perf_counter() - tg
    graph_check["identical"] = all(bool(torch.equal(a, b)) for a, b in zip(eager_out, outs()))
    del g_step, eager_out
    # the same steps with both paths on one stream, for comparison
    dt_seq = None
    if conc and do_packed and do_rle:
        torch.cuda.synchronize()
        tq = time.perf_counter()
        for s in range(args.steps):
            step(conc=False)
        torch.cuda.synchronize()
        dt_seq = time.perf_counter() - tq
    # the same steps again, with HIP events around every operation and the
    # library's launch tracing, for the per-operation and per-kernel figures
    evs = [new_events() for _ in range(args.steps)]
    torch.cuda.synchronize()
    with M.Trace(stream) as trace:             # HIP events around every library launch
        t1 = time.perf_counter()
        for s in range(args.steps):
            step(evs[s])
        torch.cuda.synchronize()
        dt_traced = time.perf_counter() - t1
    ms_step = dt * 1e3 / args.steps

    def avg(getter):
        return float(np.mean([getter(e)[0].elapsed_time(getter(e)[1]) for e in evs]))

    # device copy of the same batch: a measured bandwidth ceiling, and the
    # reference kernel for scaling the HBM byte counters
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    copy_ms = []
    for _ in range(3):
        c0.record(stream)
        dst.words.copy_(src.words)
        c1.record(stream)
        torch.cuda.synchronize()
        copy_ms.append(c0.elapsed_time(c1))
    copy_gbs = 2 * src.words.numel() * 8 / (min(copy_ms) / 1e3) / 1e9
    # a plain elementwise copy of the same bytes (torch's bitwise_or with 0):
    # the reference kernel whose HBM counters calibrate the profiles
    torch.bitwise_or(src.words, 0, out=dst.words)
    torch.cuda.synchronize()

    page_px = W * H
    n_ops = len(packed_jobs)
    px_step = (n_ops * B * page_px if do_packed else 0) + (n_ops * B * page_px if do_rle else 0)
    out = {
        "metric": "Gpixel/s rect erode/dilate (packed & RLE), % HBM peak; p50/p99 page latency",
        "value": px_step / (dt / args.steps) / 1e9,
        "unit": "Gpixel/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "ms_per_step_graph": dt_graph * 1e3 / args.steps, "graph_outputs_identical": graph_check["identical"],
        "paths_on_two_streams": conc and do_packed and do_rle,
        "rle_lanes": lanes if (conc and do_packed and do_rle) else 1,
        "ms_per_step_one_stream": dt_seq * 1e3 / args.steps if dt_seq is not None else None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64+i32",
        "data": "synthetic (seeded letter pages, %d distinct, resident in HBM)" % args.distinct,
        "config": {"workload": "letter page 2550x3300 (40 words/row), batch of %d pages; erode, dilate, "
                               "open, close x SE {1x31, 31x1, 3x3, 21x21, 51x51}; packed path and "
                               "RLE path (bitmap->RLE, 20 ops on runs, RLE->bitmap)" % B,
                   "pages": B, "width": W, "height": H, "only": args.only},
    }
    alg_bytes_pk = B * 2 * 8 * nw * H           # one read + one write of the batch
    kernels = trace.result
    out["kernels"] = {k: dict(v, gbs=v["bytes"] / (v["ms"] / 1e3) / 1e9 if v["ms"] else None,
                             ms_per_step=v["ms"] / args.steps) for k, v in kernels.items()}
    # the dominant kernel among the trace ids that bracket one launch each (the
    # others bracket a count launch, a scan and an emit launch, or a whole
    # conversion, and have no single kernel for rocprofv3 to agree with)
    single = [k for k in kernels if k in SINGLE_LAUNCH] or list(kernels)
    dom = max(single, key=lambda k: kernels[k]["ms"])
    dv = kernels[dom]
    out["roofline"] = {"bound": "hbm", "kernel": dom,
                       "achieved": dv["bytes"] / (dv["ms"] / 1e3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": dv["bytes"] / (dv["ms"] / 1e3) / 1e9 / HBM_PEAK_GBS,
                       "traffic": profiled_traffic(dom),
                       "bytes_per_launch": dv["bytes"] / dv["launches"],
                       "avg_launch_ms": dv["ms"] / dv["launches"], "launches": dv["launches"],
                       "share_of_step": dv["ms"] / (dt_traced * 1e3),
                       "timing": "HIP events around every launch, in %d steps run after the timed ones "
                                 "(the timed steps carry no events)" % args.steps}
    breakdown = {}
    if do_packed:
        pk_ms = [float(np.mean([e["pk"][k][0].elapsed_time(e["pk"][k][1]) for e in evs]))
                 for k in range(n_ops)]
        per = {"%s %s" % (op, name): round(m, 4) for (op, name, _), m in zip(packed_jobs, pk_ms)}
        mean_ms = float(np.mean(pk_ms))
        breakdown["packed"] = {"ms": sum(pk_ms), "gpixel_s": n_ops * B * page_px / (sum(pk_ms) / 1e3) / 1e9,
                               "ms_per_op": per}
        out["roofline_packed"] = {"bound": "hbm", "kernel": "rect_kernel",
                                  "achieved": alg_bytes_pk / (mean_ms / 1e3) / 1e9, "peak": HBM_PEAK_GBS,
                                  "unit": "GB/s", "frac": alg_bytes_pk / (mean_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                                  "bytes_per_launch": alg_bytes_pk, "avg_launch_ms": mean_ms}
    if do_rle:
        rle_ms = [float(np.mean([e["rle"][k][0].elapsed_time(e["rle"][k][1]) for e in evs]))
                  for k in range(n_ops)]
        p2r = avg(lambda e: e["p2r"])
        r2p = avg(lambda e: e["r2p"])
        breakdown["rle"] = {"ms_ops": sum(rle_ms), "ms_pack_to_rle": p2r, "ms_rle_to_pack": r2p,
                            "gpixel_s": n_ops * B * page_px / ((sum(rle_ms) + p2r + r2p) / 1e3) / 1e9,
                            "ms_per_op": {"%s %s" % (op, name): round(m, 4)
                                          for (op, name, _), m in zip(packed_jobs, rle_ms)},
                            "strategy": {"%s %s" % k: v for k, v in strategy.items()},
                            "runs_in": int(rle_src.row_ptr[-1].item())}
    out["breakdown"] = breakdown
    out["copy_ceiling_gbs"] = copy_gbs

    # single-page latency of the whole page workload (one page resident)
    if args.only == "all" and args.latency_reps > 0:
        one = M.Bitmap(src.words[:H], W, H, 1)
        od = M.Bitmap.empty(W, H, 1, device=dev)
        ob = M.Bitmap.empty(W, H, 1, device=dev)
        r1 = M.RLE.empty(W, H, 1, device=dev)
        r2 = M.RLE.empty(W, H, 1, device=dev)
        w1 = torch.empty(max(M.morph_rle_workspace_bytes(op, W, H, 1, se) for op in OPS for _, se in LETTER_SES),
                         dtype=torch.uint8, device=dev)
        w2 = torch.empty(M.morph_pack_to_rle_workspace_bytes(W, H), dtype=torch.uint8, device=dev)
        w0 = torch.empty(max([1] + [M.morph_workspace_bytes(op, 0, W, H, se) for op, _, se in packed_jobs]),
                         dtype=torch.uint8, device=dev)
        lat_pk, lat_all = [], []
        for rep in range(args.latency_reps + 3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            for op, _, se in packed_jobs:
                M.PACKED[op](od, one, se, w0)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            M.morph_pack_to_rle(r1, one, w2)
            for op, _, se in packed_jobs:
                M.RLE_OPS[op](r2, r1, se, w1)
            M.morph_rle_to_pack(ob, r2)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if rep >= 3:
                lat_pk.append((t1 - t) * 1e6)
                lat_all.append((t2 - t) * 1e6)
        # the same page workload captured once into a HIP graph and replayed
        # (no entry point on it allocates, synchronises or records a memset)
        def page_all():
            for op, _, se in packed_jobs:
                M.PACKED[op](od, one, se, w0)
            M.morph_pack_to_rle(r1, one, w2)
            for op, _, se in packed_jobs:
                M.RLE_OPS[op](r2, r1, se, w1)
            M.morph_rle_to_pack(ob, r2)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            page_all()
        lat_g = []
        for rep in range(args.latency_reps + 3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            g.replay()
            torch.cuda.synchronize()
            if rep >= 3:
                lat_g.append((time.perf_counter() - t) * 1e6)
        del g
        out["page_latency_us"] = {"packed_20_ops": {"p50": percentile(lat_pk, 50), "p99": percentile(lat_pk, 99)},
                                  "packed_and_rle_40_ops": {"p50": percentile(lat_all, 50),
                                                            "p99": percentile(lat_all, 99)},
                                  "packed_and_rle_40_ops_graph": {"p50": percentile(lat_g, 50),
                                                                  "p99": percentile(lat_g, 99)},
                                  "reps": args.latency_reps}
    if args.only == "all" and not args.no_extras:
        del rle_src, rle_dst, ws_rle, ws_rlet
        torch.cuda.empty_cache()
        # the representation table first (the batch and the serving executor
        # route pages by it), then serving, whose latencies depend on the
        # host's state (pinned pools, allocator caches), which the other
        # extras leave loaded
        out["repr_choice"] = bench_repr(M, dev, tuner)
        out["serving"] = bench_serving(M, dev, args.serve_seconds, tuner)
        out["batched"] = bench_batched(M, dev, tuner)
        out["density_sweep"] = bench_density(M, dev)
        out["small_image"] = bench_small(M, dev)
        out["transpose"] = bench_transpose(M, dev, src, breakdown.get("rle", {}).get("ms_per_op"))
        out["components"] = bench_components(M, dev, src)
        out["masks"] = bench_masks(M, dev, src)
        try:
            tuner.save()
        except OSError:
            pass
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(pool, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
