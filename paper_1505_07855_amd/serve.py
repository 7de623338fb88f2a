"""Serving driver: replay a seeded Poisson stream of paired-end requests
against a bwfm server and report request latency and throughput.

    python -m paper_1505_07855_amd.serve [--rates 0.3 0.6 0.9] [--requests 300]

Requests follow the serving workload's shape: sizes log-uniform in
[min_pairs, max_pairs] pairs, per-pair read length uniform in 76..150, 1%
substitutions and 0.1% indel events.  Arrival rates are fractions rho of the
server's capacity, measured first by submitting a saturating burst.
"""
from __future__ import annotations

import argparse
import json
import sys
import threading
import time

import numpy as np


def make_requests(genome, n: int, seed: int, min_pairs: int, max_pairs: int):
    from gen import configs
    sizes = configs.c4_request_sizes(seed, n, min_pairs, max_pairs)
    reqs = []
    for i, s in enumerate(sizes):
        p = configs.c4_request(genome, int(s), seed * 100003 + i)
        reqs.append((p.end1.bases, p.end1.offsets, p.end2.bases, p.end2.offsets, int(s)))
    return reqs


def replay(server, reqs, rate_per_s: float, seed: int):
    """Submit reqs at Poisson arrival times; return per-request latencies (ms)
    and the wall time from first arrival to last completion."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, len(reqs)) if rate_per_s > 0 else np.zeros(len(reqs))
    tickets = [None] * len(reqs)
    lat = [None] * len(reqs)
    done = threading.Event()

    def waiter():
        for i in range(len(reqs)):
            while tickets[i] is None:
                time.sleep(0.0002)
            t = server.wait(tickets[i], reqs[i][4], extras=server.rescue_mapq)[-1]
            lat[i] = t
        done.set()

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter()
    due = t0
    for i, r in enumerate(reqs):
        due += gaps[i]
        d = due - time.perf_counter()
        if d > 0:
            time.sleep(d)
        tickets[i] = server.submit(r[0], r[1], r[2], r[3])
    done.wait()
    th.join()
    wall = time.perf_counter() - t0
    return lat, wall


def summarize(lat, wall, reqs):
    ms = np.array([x["latency_ms"] for x in lat])
    pairs = sum(r[4] for r in reqs)
    return {"requests": len(reqs), "pairs": pairs, "wall_s": wall, "reads_per_s": 2 * pairs / wall,
            "p50_ms": float(np.percentile(ms, 50)), "p99_ms": float(np.percentile(ms, 99)),
            "mean_queued_ms": float(np.mean([x["queued_ms"] for x in lat]))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--genome", type=int, default=100_000_000)
    ap.add_argument("--rates", type=float, nargs="+", default=[0.3, 0.6, 0.9])
    ap.add_argument("--requests", type=int, default=300)
    ap.add_argument("--min-pairs", type=int, default=1000)
    ap.add_argument("--max-pairs", type=int, default=200_000)
    ap.add_argument("--step-pairs", type=int, default=131072)
    ap.add_argument("--arena-mib", type=int, default=2048)
    ap.add_argument("--device-index", action="store_true", help="build the index on the GPU (for 3.1 Gbp)")
    ap.add_argument("--rescue-mapq", action="store_true", help="also rescue mates and assign MAPQ in every step")
    args = ap.parse_args()

    import paper_1505_07855_amd as bw
    from gen import configs
    t0 = time.perf_counter()
    g = configs.c2_genome(args.genome)
    ix = (bw.Index.build_device(g.seq, **configs.LAYOUT["C3"]) if args.device_index
          else bw.Index(g.seq, **configs.LAYOUT["C3"]).upload())
    print(f"[serve] {args.genome} bp genome and index in {time.perf_counter() - t0:.0f}s", file=sys.stderr, flush=True)
    w = configs.PAIR_WINDOW
    params = bw.Params(**configs.PARAMS["C3"])
    srv = bw.Server(ix, params, w["lo"], w["hi"], w["mu"], configs.MAX_OCC, arena_bytes=args.arena_mib << 20,
                    step_pairs=args.step_pairs, max_len=150, budget_rule=True, rescue_mapq=args.rescue_mapq)
    print("[serve] server up", file=sys.stderr, flush=True)
    # capacity: a saturating burst
    burst = make_requests(g, 20, 4001, 50_000, 50_000)
    lat, wall = replay(srv, burst, 0.0, 1)
    cap_pairs = sum(r[4] for r in burst) / wall
    mean_size = (args.max_pairs - args.min_pairs) / np.log(args.max_pairs / args.min_pairs)
    out = {"genome": args.genome, "rescue_mapq": args.rescue_mapq, "capacity_pairs_per_s": cap_pairs, "mean_request_pairs": mean_size, "rates": []}
    print(f"[serve] capacity {cap_pairs:.0f} pairs/s", file=sys.stderr, flush=True)
    for k, rho in enumerate(args.rates):
        reqs = make_requests(g, args.requests, 5000 + k, args.min_pairs, args.max_pairs)
        lam = rho * cap_pairs / mean_size
        lat, wall = replay(srv, reqs, lam, 77 + k)
        s = summarize(lat, wall, reqs)
        s.update({"rho": rho, "arrivals_per_s": lam})
        out["rates"].append(s)
        print(f"[serve] rho {rho}: p50 {s['p50_ms']:.1f} ms p99 {s['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
    out["server"] = srv.stats()
    srv.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
