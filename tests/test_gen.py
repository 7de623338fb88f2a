"""The seeded input generator: determinism and truth consistency."""
import numpy as np

import gen
from gen import configs
from tests.util import revcomp


def test_deterministic_by_seed():
    a = gen.genome_repeats(5, 200_000)
    b = gen.genome_repeats(5, 200_000)
    c = gen.genome_repeats(6, 200_000)
    assert np.array_equal(a.seq, b.seq) and np.array_equal(a.spans, b.spans)
    assert not np.array_equal(a.seq, c.seq)
    ra = gen.reads_pe(9, a, 500, [36, 100], ps=0.02, indel_ratio=0.2)
    rb = gen.reads_pe(9, b, 500, [36, 100], ps=0.02, indel_ratio=0.2)
    assert np.array_equal(ra.end1.bases, rb.end1.bases) and np.array_equal(ra.end2.bases, rb.end2.bases)
    assert np.array_equal(ra.end1.offsets, rb.end1.offsets)


def test_composition_and_repeat_fraction():
    g = configs.c2_genome(2_000_000, seed=3)
    f = np.bincount(g.seq, minlength=4) / len(g.seq)
    assert abs(f[1] + f[2] - 0.41) < 0.01
    cov = int((g.spans[:, 1] - g.spans[:, 0]).sum())
    assert 0.40 * len(g.seq) <= cov <= 0.40 * len(g.seq) + 6000 * 1.2
    assert np.all(g.spans[1:, 0] >= g.spans[:-1, 1])


def test_truth_rebuilds_substitution_only_reads():
    g = gen.genome_iid(4, 100_000)
    r = gen.reads_se(8, g, 300, 50, ps=0.05)
    t = r.truth
    for i in range(r.n):
        ref = g.seq[t.pos[i]:t.pos[i] + t.ref_len[i]]
        assert t.ref_len[i] == 50
        w = r.read(i) if t.strand[i] == 0 else revcomp(r.read(i))
        diff = np.nonzero(w != ref)[0]
        subs = sorted(int(e) for ty, e in zip(t.e_type[i][:t.n_edits[i]], t.e_idx[i][:t.n_edits[i]]) if ty == 0)
        exp = subs if t.strand[i] == 0 else sorted(49 - e for e in subs)
        assert diff.tolist() == exp


def test_pairs_are_forward_reverse_within_fragment():
    g = configs.c2_genome(1_000_000, seed=4)
    p = configs.c2_pairs(g, 2000, seed=4)
    f = p.frag
    t1, t2 = p.end1.truth, p.end2.truth
    assert np.all(t1.strand != t2.strand)
    assert np.all(t1.strand == f[:, 2])
    lo = np.minimum(t1.pos, t2.pos)
    hi = np.maximum(t1.pos + t1.ref_len, t2.pos + t2.ref_len)
    assert np.array_equal(lo, f[:, 0]) and np.array_equal(hi - lo, f[:, 1])
    assert abs(float(f[:, 1].mean()) - 300) < 3 and abs(float(f[:, 1].std()) - 30) < 3
    assert np.all(np.diff(p.end1.offsets) == 100)
