"""Measurement probes for the library's roofline figures.

    python -m paper_1505_07855_amd.probes copy   [MiB]   # one device copy of known size
    python -m paper_1505_07855_amd.probes gather [MiB]   # random-line rates
    python -m paper_1505_07855_amd.probes gather_occupancy [MiB]   # the same against resident waves
    python -m paper_1505_07855_amd.probes work                     # the search loop's counters, per layout

`copy` gives the reference against which hardware byte counters
(FETCH_SIZE, WRITE_SIZE under rocprofv3 --pmc) are scaled: a plain copy of
N bytes reads N and writes N bytes.  `gather` reports the achievable rate of
dependent random 64- and 128-byte line fetches over a buffer of the given
size (cache-resident when small, HBM when large).
"""
from __future__ import annotations

import json
import sys


def copy(mib: int = 1024) -> dict:
    import torch
    n = mib << 20
    x = torch.empty(n, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    return {"probe": "copy", "bytes": n}


def gather(mib: int = 2048) -> dict:
    import torch

    import paper_1505_07855_amd as bw
    buf = torch.zeros(mib << 20, dtype=torch.uint8, device="cuda")
    out = {"probe": "gather", "buffer_mib": mib}
    for lb in (64, 128):
        bw.probe_gather(buf, lb, iters=16)  # warm
        lps = bw.probe_gather(buf, lb)
        out[f"lines_per_s_{lb}"] = lps
        out[f"gbs_{lb}"] = lps * lb / 1e9
    return out


def gather_occupancy(mib: int = 64) -> dict:
    """The gather rate of 64-byte lines against the number of resident
    waves per SIMD (1 to 16 over 256 CUs x 4 SIMDs): whether dependent random
    line fetches are bound by latency (the rate grows with waves) or by the
    memory system's throughput (it does not)."""
    import torch

    import paper_1505_07855_amd as bw
    buf = torch.zeros(mib << 20, dtype=torch.uint8, device="cuda")
    out = {"probe": "gather_occupancy", "buffer_mib": mib, "line_bytes": 64, "lines_per_s": {}}
    for w in (1, 2, 4, 8, 16):
        lanes = 256 * 4 * 64 * w
        bw.probe_gather(buf, 64, lanes=lanes, iters=16)  # warm
        out["lines_per_s"][w] = max(bw.probe_gather(buf, 64, lanes=lanes) for _ in range(3))
    return out


def work(genome: int = 100_000_000) -> dict:
    """The batched search's loop counters on the benchmark batch (100 Mbp
    genome, 1M pairs 2 x 100 bp, both ends in one launch), once per
    rank-line layout: wave-iterations, busy lane-iterations, lane-iterations
    that issued a rank query, and states expanded (bwfm_align_batch_counted)."""
    import numpy as np
    import torch

    import paper_1505_07855_amd as bw
    from gen import configs
    g = configs.c2_genome(genome)
    pairs = configs.c2_pairs(g)
    e1, e2 = pairs.end1, pairs.end2
    b = torch.from_numpy(np.concatenate([e1.bases, e2.bases])).cuda()
    o = torch.from_numpy(np.concatenate([e1.offsets[:-1], e1.offsets[-1] + e2.offsets]).view(np.int64)).cuda()
    p = bw.Params(**configs.PARAMS["C2"])
    out = {"probe": "work", "reads": 2 * pairs.end1.n, "layouts": {}}
    for lb, fmt in ((128, bw.RANK_SUB128), (64, bw.RANK_PLANES), (64, bw.RANK_SUBCOUNTS)):
        ix = bw.Index.build_device(g.seq, line_bytes=lb, rank_format=fmt)
        r = bw.align_batch(ix, b, o, p, max_len=100, hit_capacity=8 * pairs.end1.n, counted=True)
        torch.cuda.synchronize()
        w = r.work.cpu().numpy().tolist()
        out["layouts"][f"{lb}B format {fmt}"] = {
            "wave_iterations": w[0], "lane_iterations_busy": w[1], "lane_iterations_query": w[2],
            "expansions": int(r.expand.cpu().numpy().view(np.uint32).astype(np.int64).sum())}
        ix.close()
    return out


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "gather"
    default = {"copy": 1024, "gather": 2048, "gather_occupancy": 64, "work": 100_000_000}[what]
    size = int(sys.argv[2]) if len(sys.argv) > 2 else default
    fn = {"copy": copy, "gather": gather, "gather_occupancy": gather_occupancy, "work": work}[what]
    print(json.dumps(fn(size)), flush=True)
