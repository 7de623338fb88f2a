"""Randomised parity sweep: many small configurations drawn from a seed --
genome size and composition, read lengths from 1 to 300 bases, budgets,
gaps, seeds, search mode, index layout and rank-line format, execution
form, short-string table depth -- each aligned, located and paired on the GPU and by the oracle, and
compared bit for bit, with mate rescue and MAPQ on the same records.
Complements the workload-shaped tests with
combinations none of them reaches (tiny references with few rank lines,
reads longer than the reference, budget 0, every layout with every form)."""
from __future__ import annotations

import numpy as np
import pytest

import gen
import oracle
import paper_1505_07855_amd as bw

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LAYOUTS = [(32, 0, 1, bw.RANK_PLANES), (64, 0, 32, bw.RANK_PLANES), (64, 96, 8, bw.RANK_PLANES),
           (128, 0, 32, bw.RANK_PLANES), (128, 224, 64, bw.RANK_PLANES), (64, 0, 16, bw.RANK_SUBCOUNTS),
           (128, 0, 32, bw.RANK_SUB128), (128, 384, 8, bw.RANK_SUB128)]


def _config(seed: int):
    rng = np.random.default_rng(seed)
    n = int(rng.choice([300, 2000, 20000, 150000]))
    if rng.random() < 0.5:
        g = gen.genome_iid(seed, n, float(rng.uniform(0.3, 0.6)))
    else:
        g = gen.genome_repeats(seed, n, repeat_frac=0.5, n_fam=20, min_len=30, max_len=min(600, n // 4),
                               div_lo=0.0, div_hi=0.05)
    n_reads = int(rng.integers(1, 600))
    lengths = rng.integers(1, 301, n_reads) if rng.random() < 0.3 else \
        np.full(n_reads, int(rng.choice([20, 36, 75, 100, 150])), np.int64)
    lengths = np.maximum(1, np.minimum(lengths, (n - 18) // 8))  # the generator keeps 4 read lengths of margin
    reads = gen.reads_se(seed, g, n_reads, lengths.astype(np.int32), ps=float(rng.uniform(0, 0.05)),
                         indel_ratio=float(rng.uniform(0, 0.3)))
    kw = dict(max_diff=int(rng.integers(0, 7)), max_gapo=int(rng.integers(0, 2)),
              seed_len=int(rng.choice([0, 0, 16, 32])), seed_diff=int(rng.integers(0, 3)),
              mode=int(rng.choice([bw.MODE_ALL, bw.MODE_BEST])), max_hits=int(rng.choice([8, 256])))
    if kw["mode"] == bw.MODE_ALL and kw["max_diff"] > 4:
        kw["max_diff"] = 4  # keep the oracle's ALL enumeration small
    # every layout meets both forms as the seed runs through 2 x len(LAYOUTS) values
    layout = LAYOUTS[seed % len(LAYOUTS)]
    form = (bw.FORM_BATCHED, bw.FORM_PLAIN)[(seed // len(LAYOUTS)) % 2]
    # and every short-string table depth (automatic, none, shallow, deeper
    # than many reads) meets both
    kmer = (-1, 0, 2, 9)[(seed // (2 * len(LAYOUTS))) % 4]
    return g, reads, kw, layout, form, kmer


@pytest.mark.parametrize("seed", range(120))
def test_random_configuration(seed):
    g, reads, kw, layout, form, kmer = _config(5000 + seed)
    lb, bpl, sas, fmt = layout
    ix = bw.Index(g.seq, line_bytes=lb, bases_per_line=bpl, sa_sample=sas, rank_format=fmt).upload(kmer_levels=kmer)
    ox = oracle.Index(g.seq)
    p = bw.Params(**kw, form=form)
    op = oracle.Params(**kw)
    max_len = int(np.diff(reads.offsets).max())
    res = bw.align_batch(ix, torch.from_numpy(reads.bases).cuda(),
                         torch.from_numpy(reads.offsets.view(np.int64)).cuda(), p, max_len=max_len)
    torch.cuda.synchronize()
    ores = oracle.align(ox, reads.bases, reads.offsets, op, threads=8)
    ho, hits, c1, c2, st = res.to_numpy()
    ctx = (seed, kw, layout, form, kmer)
    assert np.array_equal(ho, ores.hit_off), ctx
    assert np.array_equal(hits.view(np.uint8), ores.hits.view(np.uint8)), ctx
    assert np.array_equal(c1, ores.c1) and np.array_equal(c2, ores.c2), ctx
    assert np.array_equal(st & 7, ores.status), ctx
    # locate every hit, and pair the reads with themselves shifted by one as mates
    po, pos = bw.locate(ix, res, 1 << 30)
    opo, opos = oracle.locate(ox, ores.hits, 1 << 30)
    assert np.array_equal(po.cpu().numpy().view(np.uint64), opo), ctx
    assert np.array_equal(pos.cpu().numpy().view(np.uint32), opos), ctx
    k = len(ores.c1) // 2
    if k:
        r1, r2 = res.window(0, k), res.window(k, 2 * k)
        gp = bw.pairs_numpy(bw.pair_reads(ix, r1, r2, 0, 500, 250, 1 << 30))
        o1 = oracle.AlnResult(ores.hit_off[:k + 1], ores.hits, ores.c1[:k], ores.c2[:k], ores.status[:k],
                              ores.counts[:k])
        o2 = oracle.AlnResult(ores.hit_off[k:2 * k + 1], ores.hits, ores.c1[k:2 * k], ores.c2[k:2 * k],
                              ores.status[k:2 * k], ores.counts[k:2 * k])
        l1 = oracle.locate(ox, o1.hits[o1.hit_off[0]:o1.hit_off[-1]], 1 << 30)
        l2 = oracle.locate(ox, o2.hits[o2.hit_off[0]:o2.hit_off[-1]], 1 << 30)
        o1r = oracle.AlnResult(o1.hit_off - o1.hit_off[0], o1.hits[o1.hit_off[0]:o1.hit_off[-1]], o1.c1, o1.c2,
                               o1.status, o1.counts)
        o2r = oracle.AlnResult(o2.hit_off - o2.hit_off[0], o2.hits[o2.hit_off[0]:o2.hit_off[-1]], o2.c1, o2.c2,
                               o2.status, o2.counts)
        op_ = oracle.pair(o1r, l1[0], l1[1], o2r, l2[0], l2[1], 0, 500, 250)
        assert np.array_equal(gp[:k].view(np.uint8), op_.view(np.uint8)), ctx
        # mate rescue and MAPQ on the same records
        bt = torch.from_numpy(reads.bases).cuda()
        ends = [(bt, torch.from_numpy(reads.offsets[a:b].view(np.int64)).cuda()) for a, b in ((0, k + 1),
                                                                                          (k, 2 * k + 1))]
        gpd = torch.from_numpy(op_.view(np.uint8).reshape(k, -1)).cuda()
        gr = bw.rescue_mates(ix, ends[0], ends[1], gpd, 0, 500, max_len=max_len)
        orr = oracle.rescue(g.seq, (reads.bases, reads.offsets[:k + 1]), (reads.bases, reads.offsets[k:2 * k + 1]),
                            op_, 0, 500)
        assert np.array_equal(bw.rescue_numpy(gr)[:k].view(np.uint8), orr.view(np.uint8)), ctx
        gq = bw.mapq(r1, r2, gpd, rescue=gr, max_diff=kw["max_diff"]).cpu().numpy()[:k]
        assert np.array_equal(gq, oracle.mapq(o1r, o2r, op_, rescue=orr, max_diff=kw["max_diff"])), ctx
