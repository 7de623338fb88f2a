"""Autotuner for the batched form.

The batched form's speed depends on knobs that do not change its results:
the rank-line format of the index (64-byte planar lines of 192 rows,
64-byte sub-counted lines of 160 rows, 128-byte sub-counted lines of 384
rows: bytes per rank query against bit counting per query), the kernel
build and how many waves stay resident per SIMD (a build held to 128
registers keeps 4 waves per SIMD; the compiler's own budget keeps 3; fewer
resident waves mean fewer lanes in the grid and more reads per lane).
`tune_batched` times every candidate on the caller's own batch (the median
of `repeats` timed calls after one untimed call), checks that every
candidate returns the same bytes, and returns the fastest with the whole
table.  Candidates within `tie` (2%) of the fastest median are treated as
equally fast -- the three layouts' medians on the C2 batch have come out
in either order by up to 1.5% from one GPU to another -- and among them the
one with the longest rank lines wins: each rank-line access fills a
128-byte L2 line whatever the line size, so shorter lines leave part of
every fill unused and move more bytes for the same work.
"""
from __future__ import annotations

import time

import numpy as np

from . import FORM_BATCHED, Index, Params, align_batch, lib

FORMAT_NAMES = {0: "planes", 1: "sub-counted", 2: "sub-counted"}


def _digest(res):
    ho, hits, c1, c2, st = res.to_numpy()
    return (ho.tobytes(), hits.tobytes(), c1.tobytes(), c2.tobytes(), (st & 7).tobytes())


def index_label(ix: Index) -> str:
    i = ix.info()
    return f"{i['line_bytes']}B {FORMAT_NAMES.get(i['rank_format'], '?')} x{i['bases_per_line']}"


def tune_batched(indexes, bases, offsets, params: Params, max_len: int, max_diff=None, waves=(0, 3, 2),
                 repeats: int = 3, hit_capacity: int | None = None, log=None, tie: float = 0.02):
    """Time the batched form for every (index layout, waves per SIMD)
    candidate.  `indexes`: one uploaded index, or several of the same
    reference in different layouts (a list or a dict of any keys).  Returns
    (best, table): best is the fastest table row (index label, line bytes,
    rank format, rows per line, waves per SIMD, median ms, every timing) plus
    `key`, the position (list) or key (dict) of its index."""
    import torch

    lib()
    if isinstance(indexes, Index):
        indexes = [indexes]
    items = list(indexes.items()) if isinstance(indexes, dict) else list(enumerate(indexes))
    table = []
    ref = None
    for key, ix in items:
        info = ix.info()
        for w in waves:
            p = Params(**{**params.__dict__, "form": FORM_BATCHED, "waves_per_simd": w})
            res = align_batch(ix, bases, offsets, p, max_diff=max_diff, max_len=max_len, hit_capacity=hit_capacity)
            torch.cuda.synchronize()
            d = _digest(res)
            if ref is None:
                ref = d
            elif d != ref:
                raise RuntimeError(f"batched form differs for {index_label(ix)}, waves_per_simd={w}")
            ts = []
            for _ in range(repeats):
                t0 = time.perf_counter()
                res = align_batch(ix, bases, offsets, p, max_diff=max_diff, max_len=max_len, out=res)
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t0) * 1e3)
            row = {"index": index_label(ix), "key": key, "line_bytes": info["line_bytes"],
                   "rank_format": info["rank_format"], "bases_per_line": info["bases_per_line"],
                   "waves_per_simd": w, "ms": float(np.median(ts)), "ms_all": [float(t) for t in ts]}
            table.append(row)
            if log:
                log(f"tune: {row['index']} waves_per_simd {w}: {row['ms']:.1f} ms (median of {repeats})")
    return dict(pick(table, tie)), table


def pick(table, tie: float = 0.02):
    """The row the tuner returns: among the rows within `tie` of the fastest
    median, the one with the longest rank lines, then the fastest."""
    fastest = min(r["ms"] for r in table)
    tied = [r for r in table if r["ms"] <= fastest * (1 + tie)]
    return min(tied, key=lambda r: (-r["line_bytes"], r["ms"]))
