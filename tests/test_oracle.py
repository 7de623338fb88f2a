"""Pins of the CPU oracle against things other than itself: a hand-worked
example, naive suffix sorting, naive occurrence counting, brute-force
transcript enumeration at every text position, BWT invariants, the
generator's own truth, closed forms and library routines."""
from __future__ import annotations

import os

import numpy as np
import pytest

import gen
import oracle
from gen import configs
from tests.util import brute_set, positions_set, revcomp, tier_filter, transcript_stats, truth_transcript

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CODE = {"A": 0, "C": 1, "G": 2, "T": 3, "$": 4}


def _golden(name):
    kv = {}
    queries = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        k, v = [x.strip() for x in line.split("=", 1)]
        if k == "query":
            q, a, b = v.split()
            queries.append((q, int(a), int(b)))
        else:
            kv[k] = v
    return kv, queries


def _codes(s):
    return np.array([CODE[c] for c in s], np.uint8)


def test_golden_fm_example():
    kv, queries = _golden("fm_acaacg.txt")
    ix = oracle.Index(_codes(kv["text"]))
    sa, bwt, C, prim = ix.get(0)
    assert sa.tolist() == [int(x) for x in kv["sa"].split()]
    assert bwt.tolist() == [CODE[c] for c in kv["bwt"].split()]
    assert C.tolist() == [int(x) for x in kv["C"].split()]
    assert prim == int(kv["primary"])
    rsa, rbwt, _, rprim = ix.get(1)
    assert rsa.tolist() == [int(x) for x in kv["rev_sa"].split()]
    assert rbwt.tolist() == [CODE[c] for c in kv["rev_bwt"].split()]
    assert rprim == int(kv["rev_primary"])
    for q, k, l in queries:
        ok, kk, ll, _ = ix.exact(_codes(q))
        assert (kk, ll) == (k, l) and ok == (k <= l)


@pytest.mark.parametrize("kind", ["random", "allA", "period3", "period7", "two"])
def test_sa_matches_naive_sort(kind, rng):
    for n in [1, 2, 3, 17, 64, 65, 200, 1500]:
        if kind == "random":
            t = rng.integers(0, 4, n).astype(np.uint8)
        elif kind == "allA":
            t = np.zeros(n, np.uint8)
        elif kind == "period3":
            t = np.resize(np.array([0, 1, 2], np.uint8), n)
        elif kind == "period7":
            t = np.resize(np.array([3, 1, 2, 3, 0, 0, 1], np.uint8), n)
        else:
            t = rng.integers(0, 2, n).astype(np.uint8)
        ix = oracle.Index(t)
        for which, tt in ((0, t), (1, t[::-1].copy())):
            sa, bwt, C, prim = ix.get(which)
            assert np.array_equal(sa, oracle.brute_sa(tt)), (kind, n, which)


def test_bwt_invariants(rng):
    for n in [5, 100, 4099]:
        t = rng.integers(0, 4, n).astype(np.uint8)
        ix = oracle.Index(t)
        sa, bwt, C, prim = ix.get(0)
        cnt = np.bincount(t, minlength=4)
        # Occ(a, n + 1) equals the symbol counts, and they sum to n
        tot = ix.occ4(n + 1)
        assert tot.tolist() == cnt.tolist() and tot.sum() == n
        # C[a + 1] - C[a] = count(a), C[0] = 1 (the sentinel row)
        assert C[0] == 1 and np.array_equal(np.diff(C), cnt[:3])
        # BWT is T$ rotated by SA; the sentinel sits at the primary row
        assert bwt[prim] == 4 and sa[prim] == 0
        # LF walk from row 0 reproduces T backwards (LF round trip)
        j, out = 0, []
        for _ in range(n):
            a = int(bwt[j])
            out.append(a)
            j = int(C[a] + ix.occ4(j)[a])
        assert np.array_equal(np.array(out[::-1], np.uint8), t)
        # rank checkpoints agree with a direct count at random rows
        for i in rng.integers(0, n + 2, 50):
            assert ix.occ4(int(i)).tolist() == [int((bwt[:i] == a).sum()) for a in range(4)]


def test_interval_width_is_occurrence_count(rng):
    t = rng.integers(0, 4, 3000).astype(np.uint8)
    t[1000:1040] = t[2000:2040]  # a repeat
    ix = oracle.Index(t)
    tb = t.tobytes()
    for L in [1, 2, 3, 5, 8, 12, 20, 40]:
        for _ in range(40):
            if rng.random() < 0.5:
                s = int(rng.integers(0, len(t) - L))
                x = t[s:s + L]
            else:
                x = rng.integers(0, 4, L).astype(np.uint8)
            xb = x.tobytes()
            occ = sum(1 for i in range(len(t) - L + 1) if tb[i:i + L] == xb)
            ok, k, l, steps = ix.exact(x)
            assert ok == (occ > 0)
            if ok:
                assert l - k + 1 == occ
                assert steps == L  # every base is processed, no shortcut
                sa = ix.get(0)[0]
                assert sorted(sa[k:l + 1].tolist()) == [i for i in range(len(t) - L + 1) if tb[i:i + L] == xb]
            # the reverse index finds reverse(x) with the same count
            ok2, k2, l2, _ = ix.exact(x[::-1].copy(), which=1)
            assert ok2 == ok and (not ok or l2 - k2 == l - k)


def _tiny_genome(seed, n=2500):
    g = gen.genome_repeats(seed, n, gc=0.45, repeat_frac=0.3, n_fam=2, min_len=60, max_len=150, div_lo=0.0,
                           div_hi=0.05)
    return g


def _check_all_vs_brute(ix, t, reads, p, brute_fn):
    res = oracle.align(ix, reads.bases, reads.offsets, p)
    for r in range(reads.n):
        w = reads.read(r)
        exp = brute_set(brute_fn(t, w, p))
        got = positions_set(ix, res, r)
        assert got == exp, (r, sorted(got ^ exp)[:5])
        if exp:
            assert res.status[r] & oracle.ST_HIT


@pytest.mark.parametrize("seed_len", [0, 12])
def test_all_mismatch_only_vs_hamming_scan(seed_len):
    g = _tiny_genome(7, 4000)
    ix = oracle.Index(g.seq)
    reads = gen.reads_se(31, g, 60, 30, ps=0.06)
    p = oracle.Params(max_diff=3, max_gapo=0, seed_len=seed_len, seed_diff=1, mode=oracle.MODE_ALL,
                      max_hits=1 << 20)
    _check_all_vs_brute(ix, g.seq, reads, p, oracle.brute_hamming)


@pytest.mark.parametrize("cfg", [
    dict(max_diff=2, max_gapo=1, seed_len=0, indel_end_skip=5),
    dict(max_diff=3, max_gapo=1, seed_len=10, seed_diff=1, indel_end_skip=3),
    dict(max_diff=3, max_gapo=2, max_gape=1, seed_len=0, indel_end_skip=2),
    dict(max_diff=2, max_gapo=1, seed_len=0, indel_end_skip=0, s_mm=4, s_gapo=5, s_gape=2),
])
def test_all_gapped_vs_transcript_enumeration(cfg):
    g = _tiny_genome(11, 1500)
    ix = oracle.Index(g.seq)
    reads = gen.reads_se(41, g, 16, 26, ps=0.05, indel_ratio=0.6)
    p = oracle.Params(mode=oracle.MODE_ALL, max_hits=1 << 20, **cfg)
    _check_all_vs_brute(ix, g.seq, reads, p, oracle.brute_align)


def test_read_with_N_mismatches_everything():
    g = _tiny_genome(13, 1500)
    ix = oracle.Index(g.seq)
    reads = gen.reads_se(43, g, 10, 24, ps=0.02)
    b = reads.bases.copy()
    b[reads.offsets[:-1].astype(np.int64) + 7] = 4
    reads = gen.Reads(b, reads.offsets)
    p = oracle.Params(max_diff=2, max_gapo=1, indel_end_skip=4, mode=oracle.MODE_ALL, max_hits=1 << 20)
    _check_all_vs_brute(ix, g.seq, reads, p, oracle.brute_align)


def test_d_array_is_a_lower_bound_and_pruning_is_exact():
    g = _tiny_genome(17, 3000)
    ix = oracle.Index(g.seq)
    reads = gen.reads_se(47, g, 40, 32, ps=0.05, indel_ratio=0.3)
    p = oracle.Params(max_diff=3, max_gapo=1, seed_len=0, mode=oracle.MODE_ALL, max_hits=1 << 20)
    a = oracle.align(ix, reads.bases, reads.offsets, p)
    p0 = oracle.Params(**{**p.__dict__, "use_d": 0})
    b = oracle.align(ix, reads.bases, reads.offsets, p0)
    assert np.array_equal(a.hit_off, b.hit_off) and np.array_equal(a.hits, b.hits)
    assert a.counts["expand"].sum() <= b.counts["expand"].sum()
    # D[i] never exceeds the smallest unit edit distance of w[0..i] against
    # any substring of T (mismatches and gap bases, the differences a
    # transcript counts), and the fewest mismatches bound that from above
    t = g.seq.astype(np.int16)
    col = np.arange(len(t) + 1)
    for r in range(8):
        w = reads.read(r)
        D = ix.darray(w, which=0)  # pattern w searched on the index of T
        row = np.zeros(len(t) + 1, np.int64)  # no read base consumed: free start in T
        for i in range(len(w)):
            cur = np.empty_like(row)
            cur[0] = i + 1
            cur[1:] = np.minimum(row[:-1] + ((t != w[i]) | (w[i] > 3)), row[1:] + 1)
            cur = np.minimum.accumulate(cur - col) + col  # skipped reference bases
            row = cur
            ed = int(row.min())
            if i in (3, 10, 20, 31):
                mm = min(int((g.seq[q:q + i + 1] != w[:i + 1]).sum()) for q in range(len(g.seq) - i))
                assert ed <= mm
            assert D[i] <= ed, (r, i)
        assert np.all(np.diff(D.astype(int)) >= 0)


def test_best_is_the_tier_filter_of_all():
    g = _tiny_genome(19, 3000)
    ix = oracle.Index(g.seq)
    reads = gen.reads_se(53, g, 80, 30, ps=0.05, indel_ratio=0.3)
    for mb in [30, 1]:
        pa = oracle.Params(max_diff=3, max_gapo=1, mode=oracle.MODE_ALL, max_hits=1 << 20, max_best=mb)
        pb = oracle.Params(max_diff=3, max_gapo=1, mode=oracle.MODE_BEST, max_hits=1 << 20, max_best=mb)
        a = oracle.align(ix, reads.bases, reads.offsets, pa)
        b = oracle.align(ix, reads.bases, reads.offsets, pb)
        assert b.counts["expand"].sum() <= a.counts["expand"].sum()
        for r in range(reads.n):
            rep, c1, c2, over = tier_filter(a.read_hits(r), pb)
            assert np.array_equal(b.read_hits(r), rep)
            assert (b.c1[r], b.c2[r]) == (c1, c2)
            assert bool(b.status[r] & oracle.ST_OVERFLOW) == over


def test_max_hits_overflow_flag(rng):
    # the read once exactly, and 48 distinct single-substitution variants of
    # it, each between random spacers: 1 tier-1 hit and 48 tier-2 hits
    w = rng.integers(0, 4, 24).astype(np.uint8)
    parts = [rng.integers(0, 4, 40).astype(np.uint8), w]
    for j in range(4, 20):
        for d in (1, 2, 3):
            v = w.copy()
            v[j] = (v[j] + d) % 4
            parts += [rng.integers(0, 4, 40).astype(np.uint8), v]
    t = np.concatenate(parts + [rng.integers(0, 4, 40).astype(np.uint8)])
    ix = oracle.Index(t)
    off = np.array([0, len(w)], np.uint64)
    p = oracle.Params(max_diff=1, max_gapo=0, mode=oracle.MODE_BEST, max_hits=4)
    r = oracle.align(ix, w, off, p)
    assert r.status[0] == oracle.ST_OVERFLOW and r.hit_off[1] == 0 and r.c1[0] == 0xFFFFFFFF
    p.max_hits = 1000
    r = oracle.align(ix, w, off, p)
    assert r.status[0] == oracle.ST_HIT and (r.c1[0], r.c2[0]) == (1, 48) and r.hit_off[1] == 49
    p.max_best = 0  # c1 = 1 > 0: tier 2 is dropped
    r = oracle.align(ix, w, off, p)
    assert r.hit_off[1] == 1 and (r.c1[0], r.c2[0]) == (1, 48)


def test_strand_symmetry_without_seed():
    g = _tiny_genome(23, 3000)
    ix = oracle.Index(g.seq)
    reads = gen.reads_se(59, g, 40, 30, ps=0.04, indel_ratio=0.3)
    rc = np.concatenate([revcomp(reads.read(r)) for r in range(reads.n)])
    p = oracle.Params(max_diff=3, max_gapo=1, mode=oracle.MODE_ALL, max_hits=1 << 20)
    a = oracle.align(ix, reads.bases, reads.offsets, p)
    b = oracle.align(ix, rc, reads.offsets, p)
    for r in range(reads.n):
        sa = positions_set(ix, a, r)
        sb = {(1 - x[0],) + tuple(x[1:]) for x in positions_set(ix, b, r)}
        assert sa == sb


@pytest.mark.parametrize("which", ["C1", "C2"])
def test_truth_recall_and_error_free_reads(which):
    if which == "C1":
        g = gen.genome_iid(1001, 200_000)
        reads = gen.reads_se(61, g, 400, 36, ps=0.02)
    else:
        g = configs.c2_genome(300_000, seed=77)
        reads = gen.reads_pe(63, g, 200, 100, ps=0.01, indel_ratio=0.3).end1
    p = oracle.Params(**configs.PARAMS[which], mode=oracle.MODE_ALL, max_hits=1 << 20)
    ix = oracle.Index(g.seq)
    res = oracle.align(ix, reads.bases, reads.offsets, p)
    pb = oracle.Params(**configs.PARAMS[which])
    best = oracle.align(ix, reads.bases, reads.offsets, pb)
    t = reads.truth
    n_valid = 0
    for r in range(reads.n):
        m = int(reads.offsets[r + 1] - reads.offsets[r])
        ops, pos = truth_transcript(t.e_type[r], t.e_idx[r], int(t.n_edits[r]), m)
        ok, score, diffs, gapo, nmm = transcript_stats(ops, pos, m, p)
        if not ok:
            continue
        n_valid += 1
        hits = {x[:3]: x[3:] for x in positions_set(ix, res, r)}
        key = (int(t.strand[r]), int(t.pos[r]), int(t.ref_len[r]))
        assert key in hits, (r, key)
        assert hits[key] <= (score, diffs, gapo, nmm)
        if t.n_edits[r] == 0:
            # error-free read: its origin is a tier-1 hit of score 0
            bh = positions_set(ix, best, r)
            assert any(x[:3] == key and x[3] == 0 for x in bh)
            ok_, k, l, steps = ix.exact(reads.read(r) if t.strand[r] == 0 else revcomp(reads.read(r)))
            assert ok_ and steps == m
    assert n_valid > reads.n // 2


def test_locate_matches_naive_occurrences(rng):
    g = _tiny_genome(29, 4000)
    ix = oracle.Index(g.seq)
    tb = g.seq.tobytes()
    reads = gen.reads_se(67, g, 50, 20, ps=0.03)
    p = oracle.Params(max_diff=1, max_gapo=0, mode=oracle.MODE_ALL, max_hits=1 << 20)
    res = oracle.align(ix, reads.bases, reads.offsets, p)
    po, pos = oracle.locate(ix, res.hits, max_occ=1 << 30)
    sa_f = ix.get(0)[0]
    for i, h in enumerate(res.hits):
        L = int(h["len"])
        p0 = int(pos[po[i]])
        x = tb[p0:p0 + L]
        naive = [q for q in range(len(tb) - L + 1) if tb[q:q + L] == x]
        assert pos[po[i]:po[i + 1]].tolist() == naive
        assert int(h["l"]) - int(h["k"]) + 1 == len(naive)
    # max_occ cuts hits wider than it
    po2, pos2 = oracle.locate(ix, res.hits, max_occ=1)
    widths = res.hits["l"].astype(int) - res.hits["k"].astype(int) + 1
    assert np.array_equal(np.diff(po2.astype(int)), np.where(widths <= 1, widths, 0))
    del sa_f


def _hits(*rows):
    a = np.zeros(len(rows), oracle.HIT_DTYPE)
    for i, (strand, ln, score) in enumerate(rows):
        a[i]["k"], a[i]["l"], a[i]["len"], a[i]["score"], a[i]["strand"] = i, i, ln, score, strand
        a[i]["n_mm"] = score // 3
    return a


def _pair_case(h1, p1, h2, p2, lo, hi, mu):
    """h*: hit rows (strand, len, score); p*: positions per hit."""
    r1 = oracle.AlnResult(np.array([0, len(h1)], np.uint64), _hits(*h1), np.zeros(1, np.uint32),
                          np.zeros(1, np.uint32), np.ones(1, np.uint8), np.zeros(1, oracle.COUNT_DTYPE))
    r2 = oracle.AlnResult(np.array([0, len(h2)], np.uint64), _hits(*h2), np.zeros(1, np.uint32),
                          np.zeros(1, np.uint32), np.ones(1, np.uint8), np.zeros(1, oracle.COUNT_DTYPE))
    po1 = np.array([0] + list(np.cumsum([len(x) for x in p1])), np.uint64)
    po2 = np.array([0] + list(np.cumsum([len(x) for x in p2])), np.uint64)
    pos1 = np.array([q for x in p1 for q in x], np.uint32)
    pos2 = np.array([q for x in p2 for q in x], np.uint32)
    return oracle.pair(r1, po1, pos1, r2, po2, pos2, lo, hi, mu)[0]


def test_pairing_hand_cases():
    # end 1 repeats (three + placements), end 2 unique on -: only the
    # placement within the window pairs (section 2's use of the other end)
    o = _pair_case([(0, 100, 0)], [[1000, 5000, 9000]], [(1, 100, 3)], [[5200]], 180, 420, 300)
    assert o["flags"] & oracle.PF_PAIRED and (o["pos1"], o["pos2"], o["insert"]) == (5000, 5200, 300)
    # equal score and equal |insert - mu| (350 and 250): the smaller pf wins
    o = _pair_case([(0, 100, 0)], [[1000, 1100]], [(1, 100, 0)], [[1250]], 180, 420, 300)
    assert (o["pos1"], o["insert"]) == (1000, 350)
    # equal score: the insert closer to mu wins (|350 - 300| < |230 - 300|)
    o = _pair_case([(0, 100, 0)], [[1000, 1120]], [(1, 100, 0)], [[1250]], 180, 420, 300)
    assert (o["pos1"], o["insert"]) == (1000, 350)
    o = _pair_case([(0, 100, 0)], [[1000, 1080]], [(1, 100, 0)], [[1250]], 180, 420, 300)
    assert (o["pos1"], o["insert"]) == (1080, 270)
    # lower total score beats a better insert
    o = _pair_case([(0, 100, 3), (0, 100, 0)], [[1000], [1100]], [(1, 100, 0)], [[1300]], 180, 420, 300)
    assert (o["pos1"], o["score1"]) == (1100, 0)
    # same strand, wrong order or outside the window: unpaired, each end its primary
    o = _pair_case([(0, 100, 0)], [[1000]], [(0, 100, 0)], [[1200]], 180, 420, 300)
    assert not o["flags"] & oracle.PF_PAIRED and o["flags"] & oracle.PF_MAPPED1 and o["flags"] & oracle.PF_MAPPED2
    o = _pair_case([(1, 100, 0)], [[1000]], [(0, 100, 0)], [[1200]], 180, 420, 300)
    assert not o["flags"] & oracle.PF_PAIRED
    o = _pair_case([(0, 100, 0)], [[1000]], [(1, 100, 0)], [[1500]], 180, 420, 300)
    assert not o["flags"] & oracle.PF_PAIRED and (o["pos1"], o["pos2"]) == (1000, 1500)
    # end 1 on -, end 2 on +: the + end gives pf
    o = _pair_case([(1, 100, 0)], [[1200]], [(0, 100, 0)], [[1000]], 180, 420, 300)
    assert o["flags"] & oracle.PF_PAIRED and o["insert"] == 300
    # nothing located: unmapped
    o = _pair_case([], [], [(0, 100, 0)], [[10]], 180, 420, 300)
    assert o["flags"] == oracle.PF_MAPPED2 and o["pos1"] == 0xFFFFFFFF


def test_pairing_mirrors_under_end_swap(rng):
    for _ in range(200):
        n1, n2 = int(rng.integers(1, 4)), int(rng.integers(1, 4))
        h1 = [(int(rng.integers(0, 2)), 100, int(rng.integers(0, 3)) * 3) for _ in range(n1)]
        h2 = [(int(rng.integers(0, 2)), 100, int(rng.integers(0, 3)) * 3) for _ in range(n2)]
        p1 = [sorted(rng.choice(2000, int(rng.integers(1, 4)), replace=False).tolist()) for _ in range(n1)]
        p2 = [sorted(rng.choice(2000, int(rng.integers(1, 4)), replace=False).tolist()) for _ in range(n2)]
        a = _pair_case(h1, p1, h2, p2, 100, 400, 250)
        b = _pair_case(h2, p2, h1, p1, 100, 400, 250)
        assert bool(a["flags"] & 1) == bool(b["flags"] & 1)
        if a["flags"] & 1:
            # same fragment chosen: same total score, |insert - mu| and pf
            assert int(a["score1"]) + int(a["score2"]) == int(b["score1"]) + int(b["score2"])
            assert a["insert"] == b["insert"]
            pf_a = a["pos1"] if a["strand1"] == 0 else a["pos2"]
            pf_b = b["pos1"] if b["strand1"] == 0 else b["pos2"]
            assert pf_a == pf_b


def test_estimate_insert_closed_form():
    # 100 inserts: 300 x 40, 310 x 30, 290 x 30 -> quartiles 290 / 310,
    # IQR 20, keep [250, 350] (all); mean 300, population sd sqrt(60) = 7.746
    ins = np.array([300] * 40 + [310] * 30 + [290] * 30, np.int32)
    lo, hi, mu = oracle.estimate_insert(ins)
    sd = np.sqrt((30 * 100 + 30 * 100) / 100.0)
    assert (lo, hi, mu) == (int(np.floor(300 - 4 * sd)), int(np.ceil(300 + 4 * sd)), 300)
    # an outlier beyond p75 + 2 IQR is dropped before the mean
    ins2 = np.concatenate([ins, np.array([5000], np.int32)])
    assert oracle.estimate_insert(ins2) == (lo, hi, mu)
    # fewer than 100 inserts: the fixed fallback window
    assert oracle.estimate_insert(ins[:50]) == (0, 500, 250)


def test_max_diff_rule_against_poisson_tail():
    from scipy.stats import poisson
    table = {36: 2, 51: 3, 76: 4, 100: 5, 150: 6}
    for L, k in table.items():
        assert oracle.max_diff_rule(L) == k
    for L in range(10, 513, 7):
        k = oracle.max_diff_rule(L)
        assert poisson.sf(k, 0.02 * L) < 0.04 and (k == 0 or poisson.sf(k - 1, 0.02 * L) >= 0.04)


def test_invalid_and_empty_reads():
    g = _tiny_genome(31, 2000)
    ix = oracle.Index(g.seq)
    bases = np.concatenate([np.zeros(600, np.uint8), g.seq[100:130]])
    off = np.array([0, 0, 600, 630], np.uint64)
    r = oracle.align(ix, bases, off, oracle.Params(max_diff=2))
    assert r.status.tolist()[:2] == [0, oracle.ST_INVALID] and r.status[2] == oracle.ST_HIT
    md = np.array([2, 2, 16], np.uint8)
    r = oracle.align(ix, bases, off, oracle.Params(max_diff=2), max_diff=md)
    assert r.status[2] == oracle.ST_INVALID
    with pytest.raises(ValueError):
        oracle.Index(np.array([0, 1, 4], np.uint8))


def test_threads_do_not_change_results():
    g = _tiny_genome(37, 20000)
    ix = oracle.Index(g.seq)
    reads = gen.reads_se(71, g, 300, 40, ps=0.03, indel_ratio=0.2)
    p = oracle.Params(max_diff=3)
    a = oracle.align(ix, reads.bases, reads.offsets, p, threads=1)
    b = oracle.align(ix, reads.bases, reads.offsets, p, threads=7)
    for f in ("hit_off", "hits", "c1", "c2", "status", "counts"):
        assert np.array_equal(getattr(a, f), getattr(b, f))


# ------------------------------------------------------------------ mate rescue

def _global_affine(q, r, a, b, o, e):
    """Best score aligning all of q with all of r: match +a, mismatch -b, a
    gap of g bases -(o + e g).  Textbook three-state recursion (ends in a
    match/mismatch, in a gap along r, in a gap along q), written out
    independently of the oracle's local routine."""
    NEG = -10 ** 9
    m, w = len(q), len(r)
    M = [[NEG] * (w + 1) for _ in range(m + 1)]
    X = [[NEG] * (w + 1) for _ in range(m + 1)]  # last op consumes r only
    Y = [[NEG] * (w + 1) for _ in range(m + 1)]  # last op consumes q only
    M[0][0] = 0
    for i in range(m + 1):
        for j in range(w + 1):
            if i and j:
                s = a if (q[i - 1] < 4 and q[i - 1] == r[j - 1]) else -b
                M[i][j] = max(M[i - 1][j - 1], X[i - 1][j - 1], Y[i - 1][j - 1]) + s
            if j:
                X[i][j] = max(max(M[i][j - 1], Y[i][j - 1]) - (o + e), X[i][j - 1] - e)
            if i:
                Y[i][j] = max(max(M[i - 1][j], X[i - 1][j]) - (o + e), Y[i - 1][j] - e)
    return max(M[m][w], X[m][w], Y[m][w])


def _brute_local(q, r, e_min, a=1, b=4, o=6, e=1):
    """(best, smallest end column reaching it) over every pair of non-empty
    substrings q[i0:i1], r[j0:j1] with j1 - 1 >= e_min."""
    best, bend = 0, -1
    for j1 in range(1, len(r) + 1):
        if j1 - 1 < e_min:
            continue
        for j0 in range(j1):
            for i0 in range(len(q)):
                for i1 in range(i0 + 1, len(q) + 1):
                    s = _global_affine(q[i0:i1], r[j0:j1], a, b, o, e)
                    if s > best:
                        best, bend = s, j1 - 1
    return best, bend


def test_local_alignment_against_substring_enumeration(rng):
    for t in range(60):
        m, w = int(rng.integers(1, 6)), int(rng.integers(1, 9))
        q = rng.integers(0, 5 if t % 5 == 0 else 4, m).astype(np.uint8)  # some reads carry N
        r = rng.integers(0, 4, w).astype(np.uint8)
        if t % 3 == 0 and w >= m:  # plant q (with a change) so that gaps and mismatches matter
            p = int(rng.integers(0, w - m + 1))
            r[p:p + m] = np.where(q < 4, q, 0)
            if m > 2:
                r[p + m // 2] = (r[p + m // 2] + 1) % 4
        e_min = int(rng.integers(-1, w))
        for sc in (dict(a=1, b=4, o=6, e=1), dict(a=2, b=1, o=1, e=1)):
            got, jend, jstart = oracle.local_best(q, r, e_min, sc["a"], sc["b"], sc["o"], sc["e"])
            want, wend = _brute_local(q, r, e_min, **sc)
            assert got == want, (q, r, e_min, sc)
            if want > 0:
                assert jend == wend and 0 <= jstart <= jend
                # the reported reference span holds an alignment of that score
                assert max(_global_affine(q[i0:i1], r[jstart:jend + 1], sc["a"], sc["b"], sc["o"], sc["e"])
                           for i0 in range(m) for i1 in range(i0 + 1, m + 1)) == want


def test_local_alignment_closed_cases():
    q = np.array([0, 1, 2, 3, 3, 2, 1, 0, 0, 2, 1, 3, 3, 0, 1, 2, 2, 1, 0, 3], np.uint8)
    r = np.concatenate([np.full(5, 1, np.uint8), q, np.full(6, 2, np.uint8)])
    assert oracle.local_best(q, r, 0) == (20, 24, 5)  # exact: score m, span 5..24
    r2 = r.copy()
    r2[15] = (r2[15] + 1) % 4  # one mismatch mid-read: 20 - 1 - 4 beats either side (10, 9)
    assert oracle.local_best(q, r2, 0) == (15, 24, 5)
    assert oracle.local_best(q, r, 25)[0] < 20  # end forced past the exact copy
    assert oracle.local_best(np.array([4, 4], np.uint8), r, 0) == (0, -1, -1)  # N matches nothing


def _pair_rec(pos1, len1, s1, score1, pos2, len2, s2, score2, flags):
    p = np.zeros(1, oracle.PAIR_DTYPE)
    p["pos1"], p["len1"], p["strand1"], p["score1"] = pos1, len1, s1, score1
    p["pos2"], p["len2"], p["strand2"], p["score2"] = pos2, len2, s2, score2
    p["flags"] = flags
    return p


def test_rescue_finds_planted_mates(rng):
    g = rng.integers(0, 4, 20000).astype(np.uint8)
    lo, hi = 180, 420
    L = 60
    for anchor_strand in (0, 1):
        for ins in (200, 300, 419):
            if anchor_strand == 0:
                pf = 5000
                pr = pf + ins - L
                mate = gen.revcomp(g[pr:pr + L]).copy()  # end 2 on -: its revcomp is g[pr:pr+L]
                mate[10] = (mate[10] + 1) % 4
                rec = _pair_rec(pf, L, 0, 0, 0xFFFFFFFF, 0, 0, 0, 2)  # end 1 mapped, end 2 not
                want = (pr, L, 1, ins)
            else:
                pr = 9000
                pf = pr + L - ins
                mate = g[pf:pf + L].copy()  # end 2 on +
                mate[30] = (mate[30] + 1) % 4
                rec = _pair_rec(pr, L, 1, 0, 0xFFFFFFFF, 0, 0, 0, 2)
                want = (pf, L, 0, ins)
            e1 = (np.zeros(L, np.uint8), np.array([0, L], np.uint64))
            e2 = (mate, np.array([0, L], np.uint64))
            out = oracle.rescue(g, e1, e2, rec, lo, hi)
            assert out[0]["end"] == 2, (anchor_strand, ins)
            assert (int(out[0]["pos"]), int(out[0]["len"]), int(out[0]["strand"]), int(out[0]["insert"])) == want
            assert out[0]["score"] == L - 1 - 4
    # a pair already proper, or with no primary, is left alone
    rec = _pair_rec(5000, L, 0, 0, 5200, L, 1, 0, 1 | 2 | 4)
    e = (np.zeros(L, np.uint8), np.array([0, L], np.uint64))
    assert oracle.rescue(g, e, e, rec, lo, hi)[0]["end"] == 0
    rec = _pair_rec(0xFFFFFFFF, 0, 0, 0, 0xFFFFFFFF, 0, 0, 0, 0)
    assert oracle.rescue(g, e, e, rec, lo, hi)[0]["end"] == 0
    # below min_score nothing is rescued: a random mate
    rec = _pair_rec(5000, L, 0, 0, 0xFFFFFFFF, 0, 0, 0, 2)
    rnd = (rng.integers(0, 4, L).astype(np.uint8), np.array([0, L], np.uint64))
    assert oracle.rescue(g, e, rnd, rec, lo, hi)[0]["end"] == 0


def test_rescue_anchor_choice_and_insert_bounds(rng):
    g = rng.integers(0, 4, 20000).astype(np.uint8)
    lo, hi, L = 180, 420, 60
    e_rand = (rng.integers(0, 4, L).astype(np.uint8), np.array([0, L], np.uint64))
    # both ends mapped, not paired: the end of lower penalty anchors; here end 2
    # (on + at 7000) anchors and end 1 is rescued on - at 7000 + 250 - L
    pr = 7000 + 250 - L
    e1 = (gen.revcomp(g[pr:pr + L]).copy(), np.array([0, L], np.uint64))
    e2 = (g[7000:7000 + L].copy(), np.array([0, L], np.uint64))
    rec = _pair_rec(100, L, 0, 3, 7000, L, 0, 1, 2 | 4)
    out = oracle.rescue(g, e1, e2, rec, lo, hi)[0]
    assert (out["end"], out["pos"], out["strand"], out["insert"], out["score"]) == (1, pr, 1, 250, L)
    # equal penalties: end 1 anchors (at 100, nothing there for end 2's copy)
    rec = _pair_rec(100, L, 0, 1, 7000, L, 0, 1, 2 | 4)
    assert oracle.rescue(g, e1, e2, rec, lo, hi)[0]["end"] != 1
    # the copy lies at insert 150 < lo: no rescue at that place
    pf = 5000
    pr = pf + 150 - L
    e2 = (gen.revcomp(g[pr:pr + L]).copy(), np.array([0, L], np.uint64))
    rec = _pair_rec(pf, L, 0, 0, 0xFFFFFFFF, 0, 0, 0, 2)
    out = oracle.rescue(g, e_rand, e2, rec, lo, hi)[0]
    assert out["end"] == 0 or (out["score"] < L and out["insert"] >= lo)
    assert oracle.rescue(g, e_rand, e2, rec, 150, hi)[0]["insert"] == 150  # allowed once lo admits it
    # the window is clipped at both reference ends
    rec = _pair_rec(len(g) - 2 * L, L, 0, 0, 0xFFFFFFFF, 0, 0, 0, 2)
    tail = gen.revcomp(g[len(g) - L:]).copy()
    out = oracle.rescue(g, e_rand, (tail, np.array([0, L], np.uint64)), rec, 100, hi)[0]
    assert (out["end"], out["pos"], out["insert"]) == (2, len(g) - L, 2 * L)
    rec = _pair_rec(10, L, 1, 0, 0xFFFFFFFF, 0, 0, 0, 2)
    head = g[0:L].copy()
    out = oracle.rescue(g, e_rand, (head, np.array([0, L], np.uint64)), rec, 60, hi)[0]
    assert (out["end"], out["pos"], out["strand"], out["insert"]) == (2, 0, 0, 10 + L)


# ------------------------------------------------------------------ mapping quality

def _one_read_result(c1, c2, hits, status=oracle.ST_HIT):
    """An AlnResult of one read with the given tiers and hit list
    [(score, n_mm, n_gapo, n_gape), ...] (ordered by score)."""
    h = np.zeros(len(hits), oracle.HIT_DTYPE)
    for i, (sc, mm, go, ge) in enumerate(hits):
        h[i]["score"], h[i]["n_mm"], h[i]["n_gapo"], h[i]["n_gape"] = sc, mm, go, ge
        h[i]["k"], h[i]["l"], h[i]["len"] = 10 + i, 10 + i, 50
    return oracle.AlnResult(np.array([0, len(hits)], np.uint64), h, np.array([c1], np.uint32),
                            np.array([c2], np.uint32), np.array([status], np.uint8), np.zeros(1, oracle.COUNT_DTYPE))


def _se_q(c1, c2, hits, pair_score=None, max_diff=4, placed=True, status=oracle.ST_HIT):
    r = _one_read_result(c1, c2, hits, status)
    pr = _pair_rec(1000 if placed else 0xFFFFFFFF, 50, 0, hits[0][0] if pair_score is None else pair_score,
                   0xFFFFFFFF, 0, 0, 0, 2 if placed else 0)
    return int(oracle.mapq(r, None, pr, max_diff=max_diff)[0, 0])


def test_mapq_closed_forms():
    # unique best placement, nothing in tier 2: P = 1, the single-end cap
    assert _se_q(1, 0, [(3, 1, 0, 0)]) == 37
    # one tier-2 placement: 1 - P = r / (1 + r), Q = 10 log10(1 + 10^2.2) = 22.03
    assert _se_q(1, 1, [(0, 0, 0, 0), (3, 1, 0, 0)]) == 22
    # ten of them: 1 - P = 10 r / (1 + 10 r), Q = 10 log10(1 + 10^1.2) = 12.27
    assert _se_q(1, 10, [(0, 0, 0, 0), (3, 1, 0, 0)]) == 12
    # two equal best placements: P = 1/2, Q = 10 log10 2 = 3.01; three: 10 log10 1.5 = 1.76
    assert _se_q(2, 0, [(0, 0, 0, 0), (0, 0, 0, 0)]) == 3
    assert _se_q(3, 0, [(0, 0, 0, 0)] * 3) == 2
    # the chosen placement itself in tier 2 (say, the one that pairs): P = r / (1 + r),
    # 1 - P = 1 / (1 + r), Q = 10 log10(1 + 10^-2.2) = 0.027
    assert _se_q(1, 1, [(0, 0, 0, 0), (3, 1, 0, 0)], pair_score=3) == 0
    # every best hit spends the whole budget: at most 25; one hit under it lifts the cap
    assert _se_q(1, 0, [(12, 4, 0, 0)]) == 25
    assert _se_q(1, 0, [(12, 2, 1, 1)]) == 25  # diffs = mismatches + gap opens + extensions
    assert _se_q(2, 0, [(12, 4, 0, 0), (12, 3, 0, 0)]) == 3
    assert _se_q(1, 0, [(12, 4, 0, 0)], max_diff=5) == 37
    # not placed, or an overflowed candidate set: 0
    assert _se_q(1, 0, [(0, 0, 0, 0)], placed=False) == 0
    assert _se_q(0xFFFFFFFF, 0xFFFFFFFF, [(0, 0, 0, 0)], status=oracle.ST_OVERFLOW) == 0


def test_mapq_pairs_and_rescue():
    a = _one_read_result(1, 0, [(0, 0, 0, 0)])              # Q_se 37
    b = _one_read_result(2, 0, [(0, 0, 0, 0), (0, 0, 0, 0)])  # Q_se 3
    # a proper pair: both ends get min(60, q1 + q2)
    pr = _pair_rec(1000, 50, 0, 0, 1200, 50, 1, 0, 1 | 2 | 4)
    assert oracle.mapq(a, a, pr).tolist() == [[60, 60]]
    assert oracle.mapq(b, a, pr).tolist() == [[40, 40]]
    assert oracle.mapq(b, b, pr).tolist() == [[6, 6]]
    # not paired: each end its own
    pr = _pair_rec(1000, 50, 0, 0, 9000, 50, 1, 0, 2 | 4)
    assert oracle.mapq(a, b, pr).tolist() == [[37, 3]]
    # a rescued mate takes its anchor's single-end quality
    pr = _pair_rec(1000, 50, 0, 0, 0xFFFFFFFF, 0, 0, 0, 2)
    resc = np.zeros(1, oracle.RESCUE_DTYPE)
    resc["end"] = 2
    assert oracle.mapq(b, a, pr, rescue=resc).tolist() == [[3, 3]]
    assert oracle.mapq(b, a, pr).tolist() == [[3, 0]]
    # per-read budgets replace the uniform one
    c = _one_read_result(1, 0, [(6, 2, 0, 0)])
    pr = _pair_rec(1000, 50, 0, 6, 0xFFFFFFFF, 0, 0, 0, 2)
    assert oracle.mapq(c, None, pr, budgets1=np.array([2], np.uint8)).tolist() == [[25, 0]]
    assert oracle.mapq(c, None, pr, budgets1=np.array([3], np.uint8)).tolist() == [[37, 0]]


def test_mapq_monotone_in_competition():
    """More competing placements never raise the quality."""
    qs = [[_se_q(c1, c2, [(0, 0, 0, 0), (3, 1, 0, 0)]) for c2 in range(0, 40)] for c1 in (1, 2, 5)]
    for row in qs:
        assert all(x >= y for x, y in zip(row, row[1:]))
    for a_, b_ in zip(qs, qs[1:]):
        assert all(x >= y for x, y in zip(a_, b_))
