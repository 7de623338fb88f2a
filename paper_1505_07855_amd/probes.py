"""Measurement probes for the library's roofline figures.

    python -m paper_1505_07855_amd.probes copy   [MiB]   # one device copy of known size
    python -m paper_1505_07855_amd.probes gather [MiB]   # random-line rates

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


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "gather"
    size = int(sys.argv[2]) if len(sys.argv) > 2 else (1024 if what == "copy" else 2048)
    print(json.dumps(copy(size) if what == "copy" else gather(size)), flush=True)
