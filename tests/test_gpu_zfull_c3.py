"""The uneven-length workload at full size: a 3.1 Gbp reference built like
the 100 Mbp one (indexed on the device), 10M pairs with lengths from {36,
51, 76, 100, 150} and per-read budgets from the length rule, both ends in
one batched launch as in the benchmark.

The oracle cannot index 3.1 Gbp within a test, so a sample of reads is
checked against properties that hold at any size:

* soundness: the first position of every sampled reported hit holds an
  occurrence whose smallest valid transcript -- found by enumerating every
  transcript against a window of the reference -- has exactly the hit's
  score, mismatches, gap opens and extensions;
* the best score: a read whose generated edit script is valid has
  S* <= that script's score, and when the scores are equal its origin is
  among the reported hits' positions (unless the read overflowed max_hits);
* the tier rule: every reported hit scores at most S* + s_mm; tier-2 hits
  only when c1 <= max_best; c1 and c2 are the summed widths of the tiers;
* report order (score, strand, k, len) without repeated (strand, k, len).
"""
from __future__ import annotations

import os
import time

import numpy as np
import pytest

import oracle
import paper_1505_07855_amd as bw
from gen import configs
from util import revcomp, transcript_stats, truth_transcript

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GENOME = int(os.environ.get("BWFM_C3_GENOME", 3_100_000_000))
PAIRS = int(os.environ.get("BWFM_C3_PAIRS", 10_000_000))
SAMPLE = 600


def _log(msg):
    print(f"[c3-full] {msg}", flush=True)


@pytest.mark.timeout(1100)
def test_c3_full_size_properties():
    t0 = time.time()
    g = configs.c2_genome(GENOME, seed=1003)
    _log(f"genome {GENOME} in {time.time() - t0:.0f}s")
    t0 = time.time()
    ix = bw.Index.build_device(g.seq, **configs.LAYOUT["C3"])
    _log(f"device index in {time.time() - t0:.0f}s, {ix.info()['device_bytes'] / 1e9:.2f} GB")
    t0 = time.time()
    pairs = configs.c3_pairs(g, PAIRS)
    _log(f"{PAIRS} pairs in {time.time() - t0:.0f}s")
    e1, e2 = pairs.end1, pairs.end2
    n = PAIRS
    L = np.concatenate([np.diff(e1.offsets), np.diff(e2.offsets)]).astype(np.int64)
    rule = np.array([bw.max_diff_rule(x) for x in range(513)], np.uint8)
    md = rule[L]
    bases = torch.from_numpy(np.concatenate([e1.bases, e2.bases])).cuda()
    offs = torch.from_numpy(np.concatenate([e1.offsets[:-1], e1.offsets[-1] + e2.offsets]).view(np.int64)).cuda()
    p = bw.Params(**configs.PARAMS["C3"])
    t0 = time.time()
    res = bw.align_batch(ix, bases, offs, p, max_diff=torch.from_numpy(md).cuda(), max_len=150,
                         hit_capacity=16 * n)
    torch.cuda.synchronize()
    _log(f"aligned {2 * n} reads in {time.time() - t0:.1f}s")
    del bases
    rng = np.random.default_rng(1003)
    rows = np.sort(rng.choice(2 * n, SAMPLE, replace=False))
    ho = res.hit_offsets.cpu().numpy().view(np.uint64)
    c1 = res.c1.cpu().numpy().view(np.uint32)
    c2 = res.c2.cpu().numpy().view(np.uint32)
    st = res.status.cpu().numpy()
    hits_all = res.hits
    op = oracle.Params(**configs.PARAMS["C3"])
    gs = g.seq
    n_checked = n_truth = 0
    for r in rows:
        e, j = (e1, r) if r < n else (e2, r - n)
        w = e.read(j)
        m = len(w)
        op.max_diff = int(md[r])
        a, b = int(ho[r]), int(ho[r + 1])
        h = hits_all[a:b].contiguous().cpu().numpy().view(bw.HIT_DTYPE).reshape(-1) if b > a else \
            np.zeros(0, bw.HIT_DTYPE)
        # order and uniqueness
        keys = [(int(x["score"]), int(x["strand"]), int(x["k"]), int(x["len"])) for x in h]
        assert keys == sorted(keys) and len({k[1:] for k in keys}) == len(keys), r
        if st[r] & bw.ST_OVERFLOW:
            assert len(h) == 0 and c1[r] == c2[r] == 0xFFFFFFFF
            continue
        # tiers
        if len(h):
            s_best = int(h["score"].min())
            assert all(int(x["score"]) <= s_best + op.s_mm for x in h)
            w1 = sum(int(x["l"]) - int(x["k"]) + 1 for x in h if int(x["score"]) == s_best)
            w2 = sum(int(x["l"]) - int(x["k"]) + 1 for x in h if int(x["score"]) > s_best)
            assert c1[r] == w1 and (w2 == 0 or (c1[r] <= op.max_best and c2[r] == w2)), r
        # soundness: one position per hit, checked by transcript enumeration
        pos_off, pos = bw.locate(ix, res.window(int(r), int(r) + 1), 1 << 30)
        pos = pos.cpu().numpy().view(np.uint32)
        po = pos_off.cpu().numpy().view(np.uint64)
        located = set()
        for i, x in enumerate(h):
            ps = pos[po[i] - po[0]:po[i + 1] - po[0]]
            for q in ps:
                located.add((int(x["strand"]), int(q), int(x["len"])))
            q0 = int(ps[0])
            lo = max(0, q0 - 8)
            win = gs[lo:q0 + int(x["len"]) + 8]
            recs = oracle.brute_align(win, w, op)
            match = [y for y in recs if (int(y["strand"]), int(y["pos"]) + lo, int(y["len"])) ==
                     (int(x["strand"]), q0, int(x["len"]))]
            assert match, (r, i)
            y = match[0]
            assert (int(y["score"]), int(y["n_mm"]), int(y["n_gapo"]), int(y["n_gape"])) == \
                (int(x["score"]), int(x["n_mm"]), int(x["n_gapo"]), int(x["n_gape"])), (r, i)
            n_checked += 1
        # the best score against the generated edit script
        t = e.truth
        ops, opos = truth_transcript(t.e_type[j], t.e_idx[j], int(t.n_edits[j]), m)
        ok, score, diffs, gapo, nmm = transcript_stats(ops, opos, m, op)
        if ok:
            n_truth += 1
            assert len(h) and int(h["score"].min()) <= score, r
            if int(h["score"].min()) == score:
                assert (int(t.strand[j]), int(t.pos[j]), int(t.ref_len[j])) in located, r
    _log(f"checked {n_checked} hits, {n_truth} reads with valid scripts")
    assert n_checked > SAMPLE // 2 and n_truth > SAMPLE // 2
