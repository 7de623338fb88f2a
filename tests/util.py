"""Helpers shared by the tests: read-truth transcripts, canonical forms and
the tier rule restated as a filter (used to compare sets, never as an
expected value source for the GPU path)."""
from __future__ import annotations

import numpy as np

import oracle


def revcomp(x: np.ndarray) -> np.ndarray:
    return (3 - np.asarray(x, np.uint8)[::-1]).astype(np.uint8)


def positions_set(ix: oracle.Index, res: oracle.AlnResult, r: int) -> set:
    """{(strand, pos, len, score, diffs, n_gapo, n_mm)} for read r's hits."""
    h = res.read_hits(r)
    po, pos = oracle.locate(ix, h, max_occ=1 << 30)
    out = set()
    for i, x in enumerate(h):
        d = int(x["n_mm"]) + int(x["n_gapo"]) + int(x["n_gape"])
        for p in pos[po[i]:po[i + 1]]:
            out.add((int(x["strand"]), int(p), int(x["len"]), int(x["score"]), d, int(x["n_gapo"]), int(x["n_mm"])))
    return out


def brute_set(recs: np.ndarray) -> set:
    return {(int(r["strand"]), int(r["pos"]), int(r["len"]), int(r["score"]),
             int(r["n_mm"]) + int(r["n_gapo"]) + int(r["n_gape"]), int(r["n_gapo"]), int(r["n_mm"])) for r in recs}


def truth_transcript(types, idx, n_ed: int, m: int):
    """Op string of the generator's edit script in read coordinates (5'->3'):
    'M' copy, 'S' substitution, 'I' inserted read base, 'D' deleted reference
    base."""
    subs, ins = set(), set()
    dels = {}
    for t, e in zip(types[:n_ed], idx[:n_ed]):
        if t == 0:
            subs.add(int(e))
        elif t == 1:
            ins.add(int(e))
        else:
            dels[int(e)] = dels.get(int(e), 0) + 1
    ops = []
    pos = []  # read index (or boundary for D) of each op
    for b in range(m + 1):
        for _ in range(dels.get(b, 0)):
            ops.append("D")
            pos.append(b)
        if b < m:
            ops.append("I" if b in ins else ("S" if b in subs else "M"))
            pos.append(b)
    return ops, pos


def transcript_stats(ops, pos, m: int, p: oracle.Params):
    """(valid, score, diffs, n_gapo, n_mm) of an op string under the rules."""
    n_mm = ops.count("S")
    gapo = gape = 0
    prev = None
    for o in ops:
        if o in "ID":
            if o == prev:
                gape += 1
            else:
                gapo += 1
        prev = o
    diffs = n_mm + gapo + gape
    s = p.indel_end_skip
    s1 = max(s, 1)
    sl = min(p.seed_len, m) if p.seed_len > 0 else 0
    seed = 0
    ok = diffs <= p.max_diff and gapo <= p.max_gapo and (p.max_gape < 0 or gape <= p.max_gape)
    for o, e in zip(ops, pos):
        if o == "I" and not (s <= e < m - s):
            ok = False
        if o == "D" and not (s1 <= e <= m - s1):
            ok = False
        if o in "SI" and e < sl:
            seed += 1
        if o == "D" and 0 < e < sl:
            seed += 1
    if p.seed_len > 0 and seed > p.seed_diff:
        ok = False
    score = p.s_mm * n_mm + p.s_gapo * gapo + p.s_gape * gape
    return ok, score, diffs, gapo, n_mm


def tier_filter(all_hits: np.ndarray, p: oracle.Params):
    """Restate the BEST tier rule over an ALL hit list: returns (reported
    hits sorted by (score, strand, k, len), c1, c2, overflow)."""
    if len(all_hits) == 0:
        return all_hits, 0, 0, False
    smin = int(all_hits["score"].min())
    w = all_hits["l"].astype(np.int64) - all_hits["k"].astype(np.int64) + 1
    t1 = all_hits["score"] == smin
    t2 = (all_hits["score"] > smin) & (all_hits["score"] <= smin + p.s_mm)
    c1, c2 = int(w[t1].sum()), int(w[t2].sum())
    cand = t1 | t2
    if cand.sum() > p.max_hits:
        return all_hits[:0], 0xFFFFFFFF, 0xFFFFFFFF, True
    keep = t1 | (t2 if c1 <= p.max_best else np.zeros_like(t2))
    rep = all_hits[keep]
    order = np.lexsort((rep["len"], rep["k"], rep["strand"], rep["score"]))
    return rep[order], min(c1, 0xFFFFFFFF), min(c2, 0xFFFFFFFF), False


def assert_index_equals_oracle(ix, ox: oracle.Index, rows_per_dir: int = 200, seed: int = 0, name: str = ""):
    """A library index (host- or device-built) against the oracle's index of
    the same text: per direction the whole BWT, the $ row, C, every SA sample
    (SA[r] for r a multiple of the sample interval) and Occ of all four bases
    at random rows plus both ends; and the packed reference."""
    info = ix.info()
    sas = info["sa_sample"]
    n = ox.n
    rng = np.random.default_rng(seed)
    for which in (0, 1):
        sa, bwt, C, prim = ox.get(which)
        assert np.array_equal(ix.bwt(which), bwt), (name, which, "bwt")
        assert info["primary"][which] == prim, (name, which, "primary")
        assert info["C"][which] == C.tolist(), (name, which, "C")
        assert np.array_equal(ix.sa_samples(which), sa[::sas]), (name, which, "sa samples")
        rows = np.unique(np.concatenate([rng.integers(0, n + 2, rows_per_dir), [0, 1, n, n + 1]]))
        for i in rows:
            assert ix.occ(int(i), which).tolist() == ox.occ4(int(i), which).tolist(), (name, which, int(i))
    assert np.array_equal(ix.ref(), ox.text), (name, "reference")
