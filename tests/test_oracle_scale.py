"""The oracle pinned at the workloads' own sizes, against brute force that
uses no index:

* C1 in full (1 Mbp, 10,000 reads of 36 bp, at most 2 mismatches, no gaps):
  the oracle's ALL set of every read equals a Hamming scan of every
  position on both strands;
* gapped ALL sets on 10 Mbp genomes built like the 100 Mbp one (C2-shaped
  reads with the seed rule and one gap; C5-shaped 250 bp reads with 6
  differences): equal to an edit-distance filter over the whole text
  followed by transcript enumeration at every surviving end position
  (``brute_edit_many``; a hit of d differences is an alignment of unit edit
  cost d, so the filter drops none);
* and the batched brute-force routines themselves against the one-read
  routines they restate (``brute_hamming``, ``brute_align``) and against a
  plain substring search.
"""
from __future__ import annotations

import numpy as np
import pytest

import gen
import oracle
from gen import configs

KEY = [("read", "<u8"), ("strand", "u1"), ("pos", "<u4"), ("len", "<u2"), ("score", "<u2"), ("diffs", "u1"),
       ("n_gapo", "u1"), ("n_mm", "u1")]


def _oracle_keys(ix, res):
    """Every (read, strand, position, length, score, diffs, gap opens,
    mismatches) of an ALL result, located in full, sorted."""
    po, pos = oracle.locate(ix, res.hits, max_occ=1 << 30)
    per_hit = np.diff(po).astype(np.int64)
    reads = np.repeat(np.arange(len(res.hit_off) - 1), np.diff(res.hit_off).astype(np.int64))
    h = np.repeat(res.hits, per_hit)
    out = np.zeros(len(pos), KEY)
    out["read"] = np.repeat(reads, per_hit)
    out["pos"] = pos
    for f in ("strand", "len", "score", "n_gapo", "n_mm"):
        out[f] = h[f]
    out["diffs"] = h["n_mm"] + h["n_gapo"] + h["n_gape"]
    return np.sort(out)


def _brute_keys(off, recs):
    out = np.zeros(len(recs), KEY)
    out["read"] = np.repeat(np.arange(len(off) - 1), np.diff(off).astype(np.int64))
    for f in ("strand", "pos", "len", "score", "n_gapo", "n_mm"):
        out[f] = recs[f]
    out["diffs"] = recs["n_mm"] + recs["n_gapo"] + recs["n_gape"]
    return np.sort(out)


def _assert_same(a, b):
    if not np.array_equal(a, b):
        sa, sb = set(a.tolist()), set(b.tolist())
        raise AssertionError(f"oracle-only {sorted(sa - sb)[:4]}, brute-only {sorted(sb - sa)[:4]}")


def test_c1_in_full_equals_hamming_scan():
    g = configs.c1_genome()
    reads = configs.c1_reads(g)
    assert len(g.seq) == 1_000_000 and reads.n == 10_000 and (np.diff(reads.offsets) == 36).all()
    ix = oracle.Index(g.seq)
    p = oracle.Params(**configs.PARAMS["C1"], mode=oracle.MODE_ALL, max_hits=1 << 30)
    res = oracle.align(ix, reads.bases, reads.offsets, p, threads=8)
    off, recs = oracle.brute_hamming_many(g.seq, reads.bases, reads.offsets, p, threads=8)
    got, exp = _oracle_keys(ix, res), _brute_keys(off, recs)
    _assert_same(got, exp)
    # most reads of 2% substitutions fit within 2 mismatches
    assert len(np.unique(exp["read"])) > 0.9 * reads.n


@pytest.mark.parametrize("shape", ["C2", "C5"])
def test_gapped_all_sets_at_10_mbp_equal_edit_filter_and_enumeration(shape):
    g = configs.c2_genome(10_000_000, seed=71)
    ix = oracle.Index(g.seq)
    if shape == "C2":
        reads = configs.c2_pairs(g, 300, seed=72).end1
    else:
        reads = configs.c5_reads(g, 60, seed=73)
    p = oracle.Params(**configs.PARAMS[shape], mode=oracle.MODE_ALL, max_hits=1 << 30)
    res = oracle.align(ix, reads.bases, reads.offsets, p, threads=8)
    off, recs, ends = oracle.brute_edit_many(g.seq, reads.bases, reads.offsets, p, threads=8)
    got, exp = _oracle_keys(ix, res), _brute_keys(off, recs)
    _assert_same(got, exp)
    # the sets hold gapped hits, and the filter let through only near-hits
    assert (exp["n_gapo"] > 0).any() and (exp["read"].size > 0)
    assert ends.sum() < 200 * reads.n


def test_batched_brute_routines_equal_their_one_read_forms():
    rng = np.random.default_rng(0)
    g = gen.genome_iid(5, 20_000)
    reads = gen.reads_se(6, g, 60, 70, ps=0.03)
    b = reads.bases.copy()
    b[rng.integers(0, len(b), 10)] = 4  # N in reads
    for kw in (dict(max_diff=2, max_gapo=0, seed_len=0), dict(max_diff=4, max_gapo=0, seed_len=20, seed_diff=1)):
        p = oracle.Params(**kw)
        off, recs = oracle.brute_hamming_many(g.seq, b, reads.offsets, p, threads=4)
        for r in range(reads.n):
            w = b[reads.offsets[r]:reads.offsets[r + 1]]
            one = np.sort(oracle.brute_hamming(g.seq, w, p), order=["strand", "pos"])
            assert np.array_equal(one, recs[off[r]:off[r + 1]]), r
    cfgs = [dict(max_diff=3, max_gapo=1, seed_len=0),
            dict(max_diff=4, max_gapo=2, max_gape=1, seed_len=10, seed_diff=1, indel_end_skip=2),
            dict(max_diff=2, max_gapo=0),
            dict(max_diff=5, max_gapo=1, indel_end_skip=0, s_gapo=5, s_gape=2)]
    for seed, kw in enumerate(cfgs):
        g = configs.c2_genome(3000, seed=seed + 10)
        reads = gen.reads_se(seed + 20, g, 30, 26, ps=0.05, indel_ratio=0.3, rep_frac=0.3)
        p = oracle.Params(**kw)
        off, recs, _ = oracle.brute_edit_many(g.seq, reads.bases, reads.offsets, p, threads=4)
        for r in range(reads.n):
            one = oracle.brute_align(g.seq, reads.read(r), p)
            assert np.array_equal(one, recs[off[r]:off[r + 1]]), (seed, r)
    g = configs.c2_genome(200_000, seed=3)
    pats = [g.seq[i:i + L].copy() for i, L in zip(rng.integers(0, 199_000, 50), rng.integers(16, 120, 50))]
    pats.append(rng.integers(0, 4, 40).astype(np.uint8))
    pats.append(g.seq[:16].copy())  # shortest allowed, at the text's start
    pats.append(g.seq[-30:].copy())  # at the text's end
    pb = np.concatenate(pats)
    po = np.zeros(len(pats) + 1, np.uint64)
    po[1:] = np.cumsum([len(x) for x in pats])
    off, pos = oracle.brute_exact_many(g.seq, pb, po, threads=4)
    s = g.seq.tobytes()
    for k, x in enumerate(pats):
        xb, naive = x.tobytes(), []
        i = s.find(xb)
        while i >= 0:
            naive.append(i)
            i = s.find(xb, i + 1)
        assert pos[off[k]:off[k + 1]].tolist() == naive, k
