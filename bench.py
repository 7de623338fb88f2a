"""Benchmark: aligned reads/s for 2 x 100 bp pairs (<= 4 diffs) on one MI355X.

Workload: 100 Mbp synthetic genome (41% GC, 40% repeat copies from 500
families) and 1M read pairs 2 x 100 bp (fragment ~ N(300, 30), 1%
substitutions, 0.1% indel events), seeded.  One step = the whole path over
the batch: align end 1 (1M reads), align end 2 (1M reads), then locate and
pair, with reads and index resident in HBM before the timed region.

Prints one JSON line.  The roofline entry is for the dominant kernel (the
first-pass search), timed with HIP events on the launch stream inside the
library; its algorithmic bytes per launch are the oracle's index-line
touches per read (same traversal order) x line size x reads per launch.  The
CPU baseline is the oracle itself on a bounded sample of the same pairs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "aligned reads/s (2x100bp, <=4 diffs) on 1 MI355X, batched vs plain; p99 ms"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--pairs", type=int, default=1_000_000)
    ap.add_argument("--genome", type=int, default=100_000_000)
    ap.add_argument("--cpu-pairs", type=int, default=3000, help="pairs in the oracle's timed sample")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--line-bytes", type=int, default=128)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the path would shard "
              "read pairs across GPUs with a replicated index, which is not built here)", file=sys.stderr)
        sys.exit(2)

    import torch

    import gen  # noqa: F401
    import paper_1505_07855_amd as bw
    from gen import configs

    torch.cuda.set_device(0)
    t0 = time.time()
    g = configs.c2_genome(args.genome)
    pairs = configs.c2_pairs(g, args.pairs)
    log(f"inputs drawn in {time.time() - t0:.1f}s")

    ox_box = {}
    want_cpu = not args.no_cpu

    def build_oracle():
        import oracle
        ox_box["ox"] = oracle.Index(g.seq)

    th = threading.Thread(target=build_oracle)
    if want_cpu:
        th.start()
    t0 = time.time()
    ix = bw.Index(g.seq, line_bytes=args.line_bytes, sa_sample=32).upload()
    log(f"library index built and uploaded in {time.time() - t0:.1f}s ({ix.info()['device_bytes'] / 1e6:.1f} MB)")

    params = bw.Params(**configs.PARAMS["C2"])
    w = configs.PAIR_WINDOW
    ends = []
    for end in (pairs.end1, pairs.end2):
        b = torch.from_numpy(end.bases).cuda()
        o = torch.from_numpy(end.offsets.view(np.int64)).cuda()
        ends.append((b, o))
    stream = torch.cuda.current_stream()
    res = [None, None]
    pair_out = None

    def step():
        nonlocal pair_out
        for e in range(2):
            res[e] = bw.align_batch(ix, ends[e][0], ends[e][1], params, max_len=100, out=res[e],
                                    hit_capacity=4 * args.pairs, stream=stream)
        pair_out = bw.pair_reads(ix, res[0], res[1], w["lo"], w["hi"], w["mu"], configs.MAX_OCC, stream=stream,
                                 out=pair_out)

    for i in range(args.warmup):
        step()
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    bw.timing_enable(True)
    bw.timing_reset()
    times = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        log(f"step {i + 1}/{args.steps}: {times[-1] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    bw.timing_enable(False)
    kernel_ms = {}
    for name in ("align_fast", "align_slow", "compact", "locate_rows", "sort", "pair"):
        ms, n = bw.timing_get(name)
        if n:
            kernel_ms[name] = {"avg_ms": ms / n, "launches": n}

    st = [r.status.cpu().numpy() for r in res]
    aligned = int(sum(((s & bw.ST_HIT) != 0).sum() for s in st))
    n_reads = 2 * args.pairs
    flags = bw.pairs_numpy(pair_out)["flags"]
    ms_step = total / args.steps * 1e3
    value = aligned / (ms_step / 1e3)
    research = int(sum(((s & bw.ST_RESEARCH) != 0).sum() for s in st))

    roofline = None
    cpu = None
    if want_cpu:
        th.join()
        import oracle
        ox = ox_box["ox"]
        op = oracle.Params(**configs.PARAMS["C2"], bases_per_line=ix.info()["bases_per_line"])
        nthreads = args.cpu_threads or min(os.cpu_count() or 1, 16)
        ns = min(args.cpu_pairs, args.pairs)
        sb = [(e.bases[:int(e.offsets[ns])], e.offsets[:ns + 1]) for e in (pairs.end1, pairs.end2)]
        t0 = time.perf_counter()
        ores = [oracle.align(ox, b, o, op, threads=nthreads) for b, o in sb]
        locs = [oracle.locate(ox, r.hits, configs.MAX_OCC) for r in ores]
        oracle.pair(ores[0], locs[0][0], locs[0][1], ores[1], locs[1][0], locs[1][1], w["lo"], w["hi"], w["mu"])
        cpu_s = time.perf_counter() - t0
        cpu_aligned = int(sum(((r.status & oracle.ST_HIT) != 0).sum() for r in ores))
        cpu = {"value": cpu_aligned / cpu_s, "unit": "aligned reads/s", "cores": nthreads, "kind": "oracle",
               "sample": f"first {ns} pairs of the same batch ({2 * ns} reads): align both ends, locate, pair; "
                         f"{cpu_s:.1f} s"}
        # algorithmic bytes of the first-pass search kernel: rank lines the
        # method touches per read (D-array scans + search), same order as the kernel
        touches = np.concatenate([r.counts["touch_s"] + r.counts["touch_d"] for r in ores]).astype(np.float64)
        bytes_per_read = float(touches.mean()) * ix.info()["line_bytes"]
        kf = kernel_ms.get("align_fast")
        if kf:
            per_launch = bytes_per_read * args.pairs
            achieved = per_launch / (kf["avg_ms"] / 1e3) / 1e9
            roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "kernel": "k_align_fast", "bytes_per_read": bytes_per_read,
                        "reads_per_launch": args.pairs, "avg_launch_ms": kf["avg_ms"]}

    out = {
        "metric": METRIC, "value": value, "unit": "aligned reads/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"C2 mid: {args.genome / 1e6:.0f} Mbp synthetic genome (GC 41%, 40% repeats), "
                               f"{args.pairs} pairs 2x100 bp, <=4 diffs, 1 gap open, seed 32/<=2",
                   "pairs": args.pairs, "reads": n_reads, "form": "plain", "line_bytes": args.line_bytes,
                   "parallelism": "1 GPU"},
        "p50_ms": float(np.percentile(np.array(times) * 1e3, 50)),
        "p99_ms": float(np.percentile(np.array(times) * 1e3, 99)),
        "reads_per_s": n_reads / (ms_step / 1e3), "pairs_per_s": args.pairs / (ms_step / 1e3),
        "aligned_fraction": aligned / n_reads, "paired_fraction": float((flags & bw.PF_PAIRED).astype(bool).mean()),
        "research_reads": research, "kernel_ms": kernel_ms,
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
