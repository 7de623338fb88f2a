"""The short-string interval table: every entry of every level against the
oracle's exact backward search (section 2's search of an exact string), on
both directions and several rank-line formats; the search with and without
the table on the same reads; the entry points' argument errors."""
from __future__ import annotations

import numpy as np
import pytest

import gen
import oracle
import paper_1505_07855_amd as bw

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _padded(b: int) -> int:
    return (b + 255) // 256 * 256


def _codes_to_strings(level: int) -> np.ndarray:
    """Row c holds the string of code c: base j is digit j of c in base 4
    (the base consumed last by backward search is the least significant)."""
    c = np.arange(4 ** level, dtype=np.int64)
    return np.stack([(c >> (2 * j)) & 3 for j in range(level)], axis=1).astype(np.uint8)


@pytest.mark.parametrize("layout", [(64, 192, bw.RANK_PLANES), (128, 0, bw.RANK_PLANES), (32, 0, bw.RANK_PLANES),
                                    (64, 0, bw.RANK_SUBCOUNTS), (128, 0, bw.RANK_SUB128)])
def test_table_entries_match_exact_search(layout):
    lb, bpl, fmt = layout
    g = gen.genome_repeats(71, 30_000, repeat_frac=0.4, n_fam=10, min_len=50, max_len=800, div_lo=0.0,
                           div_hi=0.1)
    K = 6
    ix = bw.Index(g.seq, line_bytes=lb, bases_per_line=bpl, sa_sample=16, rank_format=fmt).upload(kmer_levels=K)
    info = ix.info()
    assert info["kmer_levels"] == K
    assert info["kmer_bytes"] == 2 * _padded(8 * (4 + (4 ** (K + 1) - 4) // 3))
    ox = oracle.Index(g.seq)
    for which in (0, 1):
        root = ix.kmer_entries(which, 0)
        assert root.tolist() == [[0, len(g.seq)]]
        for level in range(1, K + 1):
            e = ix.kmer_entries(which, level).astype(np.int64)
            strings = _codes_to_strings(level)
            for c in range(4 ** level):
                ok, k, l, _ = ox.exact(strings[c], which)
                if ok:
                    assert (e[c, 0], e[c, 1]) == (k, l), (which, level, c)
                else:
                    assert e[c, 0] > e[c, 1], (which, level, c)
            # occurring strings partition the rows of their parent: counts add up
            occ = np.where(e[:, 0] <= e[:, 1], e[:, 1] - e[:, 0] + 1, 0)
            assert occ.sum() == len(g.seq) - level + 1, (which, level)
    # a sampled range read back equals the same slice of the whole level
    whole = ix.kmer_entries(1, 5)
    assert np.array_equal(ix.kmer_entries(1, 5, 100, 37), whole[100:137])


def test_auto_levels_and_rebuild():
    g = gen.genome_iid(72, 5000, 0.5)
    ix = bw.Index(g.seq, line_bytes=64).upload()
    assert ix.info()["kmer_levels"] == 0 and ix.info()["kmer_bytes"] == 0  # opt-in
    ix.kmer_table(-1)
    assert ix.info()["kmer_levels"] == 7  # the least d with 4^d >= 5000
    before = ix.info()["device_bytes"]
    ix.kmer_table(3)
    info = ix.info()
    assert info["kmer_levels"] == 3
    assert info["device_bytes"] == before - 2 * _padded(8 * (4 + (4 ** 8 - 4) // 3)) + 2 * _padded(
        8 * (4 + (4 ** 4 - 4) // 3))
    ix.kmer_table(0)
    assert ix.info()["kmer_levels"] == 0 and ix.info()["kmer_bytes"] == 0


@pytest.mark.parametrize("form", [bw.FORM_BATCHED, bw.FORM_PLAIN])
def test_search_with_and_without_table(form):
    """Results are byte-identical for no table, a shallow one, the automatic
    one and one deeper than some reads are long; all equal the oracle's."""
    g = gen.genome_repeats(73, 200_000, repeat_frac=0.4, n_fam=30, min_len=100, max_len=2000, div_lo=0.0,
                           div_hi=0.1)
    lengths = np.random.default_rng(73).integers(4, 120, 3000).astype(np.int32)
    reads = gen.reads_se(73, g, 3000, lengths, ps=0.02, indel_ratio=0.2)
    kw = dict(max_diff=3, max_gapo=1, seed_len=16, seed_diff=2)
    ix = bw.Index(g.seq, line_bytes=64, bases_per_line=192).upload(kmer_levels=0)
    bt = torch.from_numpy(reads.bases).cuda()
    ot = torch.from_numpy(reads.offsets.view(np.int64)).cuda()
    p = bw.Params(**kw, form=form)
    outs = []
    for K in (0, 2, -1, 12):
        ix.kmer_table(K)
        res = bw.align_batch(ix, bt, ot, p, max_len=int(lengths.max()))
        torch.cuda.synchronize()
        outs.append([a.copy() for a in res.to_numpy()])
    ores = oracle.align(oracle.Index(g.seq), reads.bases, reads.offsets, oracle.Params(**kw), threads=8)
    for o in outs:
        ho, hits, c1, c2, st = o
        assert np.array_equal(ho, ores.hit_off)
        assert np.array_equal(hits.view(np.uint8), ores.hits.view(np.uint8))
        assert np.array_equal(c1, ores.c1) and np.array_equal(c2, ores.c2)
        assert np.array_equal(st & 7, ores.status)


def test_errors():
    g = gen.genome_iid(74, 3000, 0.5)
    ix = bw.Index(g.seq, line_bytes=64)
    with pytest.raises(bw.BwfmError):
        ix.kmer_table(3)  # not uploaded
    ix.upload(kmer_levels=0)
    for bad in (-2, 16):
        with pytest.raises(bw.BwfmError):
            ix.kmer_table(bad)
    with pytest.raises(bw.BwfmError):
        ix.kmer_entries(0, 1)  # no table
    ix.kmer_table(4)
    with pytest.raises(bw.BwfmError):
        ix.kmer_entries(0, 5)  # above its levels
    with pytest.raises(bw.BwfmError):
        ix.kmer_entries(0, 2, 10, 7)  # beyond 4^2 codes
    with pytest.raises(bw.BwfmError):
        ix.kmer_entries(2, 1)
