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
* report order (score, strand, k, len) without repeated (strand, k, len);
* completeness of exact placements: for every sampled read whose best score
  is 0, the positions of its score-0 hits are exactly the occurrences of the
  read and of its reverse complement found by a plain scan of the whole
  text, and c1 is their number.

The device-built index itself is checked where the oracle cannot go: Occ at
row n + 1 equals the base counts of the text in both directions, and LF
walks from random sampled rows retrace the text backwards and meet the SA
samples they pass.

Then the whole batch is paired, its mates rescued and MAPQ assigned, and
checked by properties: rescue only where no proper pair exists, inserts
within the window, scores within bounds, the reported span of a sample of
rescued mates holding a local alignment of exactly the reported score, most
rescued mates at their generated origin; MAPQ equal on both ends of a proper
pair, 0 for ends left unplaced, a rescued mate's equal to its anchor's.
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
    info = ix.info()
    sas = info["sa_sample"]
    cnt = sum(np.bincount(g.seq[i:i + (1 << 27)], minlength=4) for i in range(0, GENOME, 1 << 27))
    irng = np.random.default_rng(31)
    for which in (0, 1):
        assert ix.occ(GENOME + 1, which).tolist() == cnt.tolist()
        C, prim = info["C"][which], info["primary"][which]
        samp = ix.sa_samples(which)
        for j in irng.choice(len(samp), 100, replace=False):
            row, pos = int(j) * sas, int(samp[j])
            for _ in range(3 * sas):
                if row % sas == 0:
                    assert int(samp[row // sas]) == pos, (which, row)
                if pos == 0:
                    assert row == prim
                    break
                o0, o1 = ix.occ(row, which), ix.occ(row + 1, which)
                a = int(np.flatnonzero(o1 - o0)[0])  # BWT[row]
                assert a == int(g.seq[pos - 1] if which == 0 else g.seq[GENOME - pos]), (which, row)
                row, pos = C[a] + int(o0[a]), pos - 1
    del samp
    _log(f"index: Occ totals and 200 LF walks checked in {time.time() - t0:.0f}s")
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
    exact = []  # (row, read, positions of its score-0 hits by strand, c1)
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
        if len(h) and int(h["score"].min()) == 0:
            zero = {(int(x["strand"]), int(q)) for i, x in enumerate(h) if int(x["score"]) == 0
                    for q in pos[po[i] - po[0]:po[i + 1] - po[0]]}
            exact.append((int(r), w, zero, int(c1[r])))
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
    # exact placements against a scan of the whole text
    t0 = time.time()
    pats = [x for _, w, _, _ in exact for x in (w, revcomp(w))]
    poff = np.zeros(len(pats) + 1, np.uint64)
    poff[1:] = np.cumsum([len(x) for x in pats])
    occ_off, occ = oracle.brute_exact_many(gs, np.concatenate(pats), poff, threads=16)
    for j, (r, w, zero, c1r) in enumerate(exact):
        fw = occ[occ_off[2 * j]:occ_off[2 * j + 1]]
        rc = occ[occ_off[2 * j + 1]:occ_off[2 * j + 2]]
        assert zero == {(0, int(q)) for q in fw} | {(1, int(q)) for q in rc}, r
        assert c1r == len(fw) + len(rc), r
    _log(f"{len(exact)} sampled reads with exact placements complete against a text scan "
         f"({time.time() - t0:.0f}s)")
    assert len(exact) > SAMPLE // 10

    # pairing, mate rescue and MAPQ over the whole batch
    w = configs.PAIR_WINDOW
    t0 = time.time()
    r1, r2 = res.window(0, n), res.window(n, 2 * n)
    prs = bw.pair_reads(ix, r1, r2, w["lo"], w["hi"], w["mu"], configs.MAX_OCC)
    ends = [(torch.from_numpy(e.bases).cuda(), torch.from_numpy(e.offsets.view(np.int64)).cuda()) for e in (e1, e2)]
    resc = bw.rescue_mates(ix, ends[0], ends[1], prs, w["lo"], w["hi"], max_len=150)
    again = bw.rescue_mates(ix, ends[0], ends[1], prs, w["lo"], w["hi"], max_len=150)
    mdd = torch.from_numpy(md).cuda()
    mq = bw.mapq(r1, r2, prs, rescue=resc, budgets1=mdd[:n], budgets2=mdd[n:]).cpu().numpy()[:n]
    torch.cuda.synchronize()
    _log(f"paired, rescued and MAPQ in {time.time() - t0:.1f}s")
    pr = bw.pairs_numpy(prs)[:n]
    rs = bw.rescue_numpy(resc)[:n]
    assert np.array_equal(rs.view(np.uint8), bw.rescue_numpy(again)[:n].view(np.uint8))
    f = pr["flags"]
    m1, m2 = (f & bw.PF_MAPPED1) != 0, (f & bw.PF_MAPPED2) != 0
    cand = ((f & bw.PF_PAIRED) == 0) & (m1 | m2)
    got = rs["end"] != 0
    assert not (got & ~cand).any()
    a1 = m1 & (~m2 | (pr["score1"] <= pr["score2"]))
    assert (rs["end"][got] == np.where(a1, 2, 1)[got]).all()
    assert (rs["insert"][got] >= w["lo"]).all() and (rs["insert"][got] <= w["hi"]).all()
    mlen = np.where(rs["end"] == 1, np.diff(e1.offsets), np.diff(e2.offsets)).astype(np.int64)
    assert (rs["score"][got] >= 20).all() and (rs["score"][got] <= mlen[got]).all()
    anchor_strand = np.where(a1, pr["strand1"], pr["strand2"])
    assert (rs["strand"][got] == 1 - anchor_strand[got]).all()
    _log(f"{int(cand.sum())} pairs without a proper pair, {int(got.sum())} mates rescued")
    assert got.sum() > 0.5 * cand.sum()
    # rescued mates at their generated origin (local ends may clip a few bases)
    idx = np.flatnonzero(got)
    tpos = np.where(rs["end"][idx] == 1, e1.truth.pos[idx], e2.truth.pos[idx]).astype(np.int64)
    near = np.abs(rs["pos"][idx].astype(np.int64) - tpos) <= 8
    _log(f"rescued mates within 8 bases of their origin: {near.mean():.3f}")
    assert near.mean() > 0.8
    # a sample's reported span holds a local alignment of exactly that score
    for i in rng.choice(idx, min(200, len(idx)), replace=False):
        rec = rs[i]
        e = e1 if rec["end"] == 1 else e2
        mate = e.read(int(i))
        q = revcomp(mate) if rec["strand"] == 1 else mate
        span = gs[int(rec["pos"]):int(rec["pos"]) + int(rec["len"])]
        sc, _, _ = oracle.local_best(q, span, -1)
        assert sc == int(rec["score"]), i
    # MAPQ
    paired = (f & bw.PF_PAIRED) != 0
    assert (mq <= 60).all() and (mq[paired, 0] == mq[paired, 1]).all()
    un1 = (pr["pos1"] == 0xFFFFFFFF) & (rs["end"] != 1)
    un2 = (pr["pos2"] == 0xFFFFFFFF) & (rs["end"] != 2)
    assert (mq[un1, 0] == 0).all() and (mq[un2, 1] == 0).all()
    r_2, r_1 = rs["end"] == 2, rs["end"] == 1
    assert (mq[r_2, 1] == mq[r_2, 0]).all() and (mq[r_1, 0] == mq[r_1, 1]).all()
    assert (mq[~paired] <= 37).all()
    _log(f"MAPQ 60 on {np.mean(mq == 60):.3f} of ends")
