"""Autotuner for the batched form.

The batched form's speed depends on launch knobs that do not change its
results: the kernel build and how many waves stay resident per SIMD (a
build held to 128 registers keeps 4 waves per SIMD for latency hiding; the
compiler's own budget keeps 3 with fewer instructions; fewer resident lanes
also means more reads per lane) and the rank-line size of the index (64- or
128-byte lines: bytes per rank query against popcount work per query).
`tune_batched` times one batched call per candidate on the caller's own
batch, checks that every candidate returns the same bytes, and returns the
fastest.
"""
from __future__ import annotations

import time

import numpy as np

from . import FORM_BATCHED, Index, Params, align_batch, lib


def _digest(res):
    ho, hits, c1, c2, st = res.to_numpy()
    return (ho.tobytes(), hits.tobytes(), c1.tobytes(), c2.tobytes(), (st & 7).tobytes())


def tune_batched(indexes: dict[int, Index] | Index, bases, offsets, params: Params, max_len: int, max_diff=None,
                 waves=(0, 3), repeats: int = 1, hit_capacity: int | None = None, log=None):
    """Time the batched form for every (rank-line size, waves per SIMD)
    candidate.  `indexes` maps line bytes to an uploaded index of the same
    reference (or is a single index).  Returns (best, table): best is a dict
    with line_bytes, waves_per_simd and ms; table lists every candidate."""
    import torch

    lib()
    if isinstance(indexes, Index):
        indexes = {indexes.info()["line_bytes"]: indexes}
    table = []
    ref = None
    for lb, ix in sorted(indexes.items()):
        for w in waves:
            p = Params(**{**params.__dict__, "form": FORM_BATCHED, "waves_per_simd": w})
            res = align_batch(ix, bases, offsets, p, max_diff=max_diff, max_len=max_len, hit_capacity=hit_capacity)
            torch.cuda.synchronize()
            d = _digest(res)
            if ref is None:
                ref = d
            elif d != ref:
                raise RuntimeError(f"batched form differs at line_bytes={lb}, waves_per_simd={w}")
            ts = []
            for _ in range(repeats):
                t0 = time.perf_counter()
                res = align_batch(ix, bases, offsets, p, max_diff=max_diff, max_len=max_len, out=res)
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t0) * 1e3)
            row = {"line_bytes": lb, "waves_per_simd": w, "ms": float(np.median(ts))}
            table.append(row)
            if log:
                log(f"tune: line_bytes {lb} waves_per_simd {w}: {row['ms']:.1f} ms")
    best = min(table, key=lambda r: r["ms"])
    return dict(best), table
