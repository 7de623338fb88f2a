"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for
bit (hit lists, c1/c2, statuses, positions, pair records), on seeded inputs
of the workloads' shapes, including the edge cases and both index layouts."""
from __future__ import annotations

import threading

import numpy as np
import pytest

import gen
import oracle
import paper_1505_07855_amd as bw
from gen import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def _gpu_align(ix, reads, params, max_diff=None, counted=False):
    bases = _dev(reads.bases)
    offs = _dev(reads.offsets.view(np.int64))
    md = _dev(max_diff) if max_diff is not None else None
    max_len = int(np.diff(reads.offsets).max()) if reads.n else 0
    res = bw.align_batch(ix, bases, offs, params, max_diff=md, max_len=max(max_len, 1), counted=counted)
    torch.cuda.synchronize()
    return res


def _compare_align(res, ores, rows=None):
    ho, hits, c1, c2, st = res.to_numpy()
    if rows is None:
        assert np.array_equal(ho, ores.hit_off), "hit offsets differ"
        assert np.array_equal(hits.view(np.uint8), ores.hits.view(np.uint8)), "hits differ"
        assert np.array_equal(c1, ores.c1) and np.array_equal(c2, ores.c2)
        assert np.array_equal(st & 7, ores.status)
    else:
        for j, r in enumerate(rows):
            g = hits[ho[r]:ho[r + 1]]
            o = ores.read_hits(j)
            assert np.array_equal(g.view(np.uint8), o.view(np.uint8)), f"read {r}"
            assert (c1[r], c2[r], st[r] & 7) == (ores.c1[j], ores.c2[j], ores.status[j])


def _params_pair(form=None, **kw):
    p = bw.Params(**kw)
    if form is not None:
        p.form = form
    return p, oracle.Params(**kw)


@pytest.fixture(scope="module")
def c1_small():
    g = gen.genome_iid(1001, 200_000)
    reads = gen.reads_se(2001, g, 3000, 36, ps=0.02)
    return g, reads, oracle.Index(g.seq)


FORMS = [bw.FORM_BATCHED, bw.FORM_PLAIN]
# the forms, and the batched one with a split budget so small that nearly
# every read's search is split into task rounds
FORMS_SPLIT = [(bw.FORM_BATCHED, 0), (bw.FORM_BATCHED, 32), (bw.FORM_PLAIN, 0)]
FORMS_SPLIT_IDS = ["batched", "batched-split32", "plain"]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("layout", [(64, 128), (128, 448), (64, 160, bw.RANK_SUBCOUNTS), (128, 384, bw.RANK_SUB128)])
@pytest.mark.parametrize("mode", [bw.MODE_BEST, bw.MODE_ALL])
def test_c1_shape_parity(c1_small, layout, mode, form):
    g, reads, ox = c1_small
    ix = bw.Index(g.seq, line_bytes=layout[0], bases_per_line=layout[1], sa_sample=32,
                  rank_format=layout[2] if len(layout) > 2 else bw.RANK_PLANES).upload()
    p, op = _params_pair(**configs.PARAMS["C1"], mode=mode)
    p.form = form
    res = _gpu_align(ix, reads, p, counted=True)
    ores = oracle.align(ox, reads.bases, reads.offsets, op, threads=8)
    _compare_align(res, ores)
    # same traversal order: the work counters agree for reads done in one pass
    st = res.status.cpu().numpy()
    exp = res.expand.cpu().numpy().view(np.uint32)
    # (reads whose tree was split across lanes or tasks traverse in another order)
    one = (st & (bw.ST_RESEARCH | bw.ST_SHARED | bw.ST_SPLIT)) == 0
    assert np.array_equal(exp[one], ores.counts["expand"][one].astype(np.uint32))


@pytest.fixture(scope="module")
def c1_full():
    g = configs.c1_genome()
    reads = configs.c1_reads(g)
    assert len(g.seq) == 1_000_000 and reads.n == 10_000
    return g, reads, oracle.Index(g.seq)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("mode", [bw.MODE_BEST, bw.MODE_ALL])
def test_c1_full_size_parity(c1_full, mode, form):
    """C1 at its stated size: 1 Mbp, 10,000 reads of 36 bp, at most 2
    mismatches, no gaps, in its own layout (checkpoints every 128 rows, SA
    samples every 32); hits, counts, status and located positions."""
    g, reads, ox = c1_full
    ix = bw.Index(g.seq, **configs.LAYOUT["C1"]).upload()
    p, op = _params_pair(form=form, **configs.PARAMS["C1"], mode=mode)
    res = _gpu_align(ix, reads, p)
    ores = oracle.align(ox, reads.bases, reads.offsets, op, threads=8)
    _compare_align(res, ores)
    assert (ores.status & oracle.ST_HIT).mean() > 0.9
    po, pos = bw.locate(ix, res, configs.MAX_OCC)
    opo, opos = oracle.locate(ox, ores.hits, configs.MAX_OCC)
    assert np.array_equal(po.cpu().numpy().view(np.uint64), opo)
    assert np.array_equal(pos.cpu().numpy().view(np.uint32), opos)


@pytest.fixture(scope="module")
def c2_small():
    g = configs.c2_genome(2_000_000, seed=77)
    pairs = configs.c2_pairs(g, 3000, seed=78)
    return g, pairs, oracle.Index(g.seq)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("layout", [(128, 448, 32), (64, 192, 16), (32, 64, 32), (64, 160, 32, bw.RANK_SUBCOUNTS),
                                    (128, 384, 32, bw.RANK_SUB128)])
def test_c2_shape_parity_align_locate_pair(c2_small, layout, form):
    g, pairs, ox = c2_small
    ix = bw.Index(g.seq, line_bytes=layout[0], bases_per_line=layout[1], sa_sample=layout[2],
                  rank_format=layout[3] if len(layout) > 3 else bw.RANK_PLANES).upload()
    p, op = _params_pair(form=form, **configs.PARAMS["C2"])
    r = []
    for end in (pairs.end1, pairs.end2):
        res = _gpu_align(ix, end, p, counted=True)
        ores = oracle.align(ox, end.bases, end.offsets, op, threads=8)
        _compare_align(res, ores)
        st = res.status.cpu().numpy()
        one = (st & (bw.ST_RESEARCH | bw.ST_SHARED | bw.ST_SPLIT)) == 0
        assert np.array_equal(res.expand.cpu().numpy().view(np.uint32)[one],
                              ores.counts["expand"][one].astype(np.uint32))
        r.append((res, ores))
    # locate
    for res, ores in r:
        for max_occ in (100000, 1):
            po, pos = bw.locate(ix, res, max_occ)
            opo, opos = oracle.locate(ox, ores.hits, max_occ)
            assert np.array_equal(po.cpu().numpy().view(np.uint64), opo)
            assert np.array_equal(pos.cpu().numpy().view(np.uint32), opos)
    # pairing, paired and single-end
    w = configs.PAIR_WINDOW
    gp = bw.pairs_numpy(bw.pair_reads(ix, r[0][0], r[1][0], w["lo"], w["hi"], w["mu"], configs.MAX_OCC))
    po1, pos1 = oracle.locate(ox, r[0][1].hits, configs.MAX_OCC)
    po2, pos2 = oracle.locate(ox, r[1][1].hits, configs.MAX_OCC)
    op_ = oracle.pair(r[0][1], po1, pos1, r[1][1], po2, pos2, w["lo"], w["hi"], w["mu"])
    assert np.array_equal(gp.view(np.uint8), op_.view(np.uint8))
    assert (gp["flags"] & bw.PF_PAIRED).mean() > 0.8
    gs = bw.pairs_numpy(bw.pair_reads(ix, r[0][0], None, w["lo"], w["hi"], w["mu"], configs.MAX_OCC))
    os_ = oracle.pair(r[0][1], po1, pos1, None, None, None, w["lo"], w["hi"], w["mu"])
    assert np.array_equal(gs.view(np.uint8), os_.view(np.uint8))


def test_both_ends_in_one_batch(c2_small):
    """The batched form aligns both ends in one launch; windows of the one
    result feed pairing."""
    g, pairs, ox = c2_small
    ix = bw.Index(g.seq).upload()
    p, op = _params_pair(**configs.PARAMS["C2"])
    n = pairs.end1.n
    both = gen.Reads(np.concatenate([pairs.end1.bases, pairs.end2.bases]),
                     np.concatenate([pairs.end1.offsets[:-1], pairs.end1.offsets[-1] + pairs.end2.offsets]))
    res = _gpu_align(ix, both, p)
    o1 = oracle.align(ox, pairs.end1.bases, pairs.end1.offsets, op, threads=8)
    o2 = oracle.align(ox, pairs.end2.bases, pairs.end2.offsets, op, threads=8)
    w1, w2 = res.window(0, n), res.window(n, 2 * n)
    _compare_align(w1, o1)
    _compare_align(w2, o2)
    po, pos = bw.locate(ix, w2, configs.MAX_OCC)
    opo, opos = oracle.locate(ox, o2.hits, configs.MAX_OCC)
    assert np.array_equal(po.cpu().numpy().view(np.uint64), opo)
    assert np.array_equal(pos.cpu().numpy().view(np.uint32), opos)
    w = configs.PAIR_WINDOW
    gp = bw.pairs_numpy(bw.pair_reads(ix, w1, w2, w["lo"], w["hi"], w["mu"], configs.MAX_OCC))
    po1, pos1 = oracle.locate(ox, o1.hits, configs.MAX_OCC)
    opr = oracle.pair(o1, po1, pos1, o2, opo, opos, w["lo"], w["hi"], w["mu"])
    assert np.array_equal(gp.view(np.uint8), opr.view(np.uint8))


@pytest.mark.parametrize("form,split", FORMS_SPLIT, ids=FORMS_SPLIT_IDS)
def test_second_pass_and_overflow_parity(form, split):
    # a repeat-rich genome and ALL mode: many reads exceed the first pass's
    # 128 hit slots (or, in the plain form, its stack) and are searched
    # again (three repeat families over 800 kbp: about a hundred reads have
    # more than 128 distinct hits within 3 differences)
    g = gen.genome_repeats(91, 800_000, gc=0.41, repeat_frac=0.7, n_fam=3, min_len=300, max_len=800, div_lo=0.0,
                           div_hi=0.03)
    reads = gen.reads_se(92, g, 1500, 40, ps=0.03, indel_ratio=0.2, rep_frac=0.9)
    ox = oracle.Index(g.seq)
    ix = bw.Index(g.seq).upload()
    researched = overflowed = 0
    for kw in (dict(max_diff=3, max_gapo=1, mode=bw.MODE_ALL, max_hits=200),
               dict(max_diff=3, max_gapo=1, mode=bw.MODE_BEST, max_hits=5),
               dict(max_diff=2, max_gapo=0, mode=bw.MODE_ALL, max_hits=1000)):
        p, op = _params_pair(form=form, **kw)
        p.split_budget = split
        res = _gpu_align(ix, reads, p)
        ores = oracle.align(ox, reads.bases, reads.offsets, op, threads=8)
        _compare_align(res, ores)
        st = res.status.cpu().numpy()
        if split:
            assert (st & bw.ST_SPLIT).any() or (st & bw.ST_RESEARCH).any()
        researched += int((st & bw.ST_RESEARCH).astype(bool).sum())
        overflowed += int((st & bw.ST_OVERFLOW).astype(bool).sum())
    assert researched > 0, "the second pass was not exercised"
    assert overflowed > 0, "the max_hits rule was not exercised"


@pytest.mark.parametrize("form,split", FORMS_SPLIT, ids=FORMS_SPLIT_IDS)
def test_edge_cases_parity(form, split):
    g = configs.c2_genome(300_000, seed=5)
    ox = oracle.Index(g.seq)
    ix = bw.Index(g.seq).upload()
    rng = np.random.default_rng(3)
    pieces = [np.zeros(0, np.uint8),                     # empty read
              g.seq[1000:1001].copy(),                   # one base
              g.seq[5000:5512].copy(),                   # the longest read
              rng.integers(0, 4, 100).astype(np.uint8),  # random: no hit
              g.seq[7000:7100].copy(),                   # exact
              np.full(60, 4, np.uint8)]                  # all N
    x = g.seq[9000:9100].copy()
    x[[10, 50, 90]] = 4                                  # with N
    pieces.append(x)
    y = (3 - g.seq[20000:20150][::-1]).astype(np.uint8)  # reverse strand, 150 bp
    pieces.append(y)
    bases = np.concatenate(pieces)
    offs = np.zeros(len(pieces) + 1, np.uint64)
    offs[1:] = np.cumsum([len(p) for p in pieces])
    reads = gen.Reads(bases, offs)
    md = np.array([4, 2, 6, 4, 0, 4, 5, 15], np.uint8)
    p, op = _params_pair(form=form, **configs.PARAMS["C2"])
    p.split_budget = split
    res = _gpu_align(ix, reads, p, max_diff=md)
    ores = oracle.align(ox, reads.bases, reads.offsets, op, max_diff=md, threads=1)
    _compare_align(res, ores)
    st = res.status.cpu().numpy()
    assert st[0] == 0 and st[4] & bw.ST_HIT and st[7] & bw.ST_HIT
    # invalid: a read longer than max_len, a budget above 15
    md2 = md.copy()
    md2[4] = 16
    bases_t, offs_t = _dev(bases), _dev(offs.view(np.int64))
    res2 = bw.align_batch(ix, bases_t, offs_t, p, max_diff=_dev(md2), max_len=200)
    st2 = res2.status.cpu().numpy()
    assert st2[2] == bw.ST_INVALID and st2[4] == bw.ST_INVALID and st2[3] & 7 == ores.status[3]
    # an empty batch
    res3 = bw.align_batch(ix, _dev(np.zeros(1, np.uint8)), _dev(np.zeros(1, np.int64)), p, max_len=1)
    assert res3.n_hits == 0


@pytest.mark.parametrize("form,split", FORMS_SPLIT, ids=FORMS_SPLIT_IDS)
def test_c3_shape_per_read_budgets_parity(form, split):
    g = configs.c2_genome(1_000_000, seed=33)
    pairs = configs.c3_pairs(g, 1500, seed=34)
    ox = oracle.Index(g.seq)
    ix = bw.Index(g.seq).upload()
    p, op = _params_pair(form=form, **configs.PARAMS["C3"])
    p.split_budget = split
    for end in (pairs.end1, pairs.end2):
        L = np.diff(end.offsets).astype(int)
        md_lib = np.array([bw.max_diff_rule(int(x)) for x in L], np.uint8)
        md_orc = np.array([oracle.max_diff_rule(int(x)) for x in L], np.uint8)
        assert np.array_equal(md_lib, md_orc)
        res = _gpu_align(ix, end, p, max_diff=md_lib)
        ores = oracle.align(ox, end.bases, end.offsets, op, max_diff=md_orc, threads=8)
        _compare_align(res, ores)
        if split:
            assert (res.status.cpu().numpy() & bw.ST_SPLIT).any(), "no search was split"


@pytest.mark.parametrize("form,wps,fmt,split", [(bw.FORM_BATCHED, 0, bw.RANK_PLANES, 4096),
                                                (bw.FORM_BATCHED, 3, bw.RANK_PLANES, 4096),
                                                (bw.FORM_PLAIN, 0, bw.RANK_PLANES, 0),
                                                (bw.FORM_BATCHED, 0, bw.RANK_SUBCOUNTS, 4096),
                                                (bw.FORM_BATCHED, 0, bw.RANK_SUB128, 4096),
                                                (bw.FORM_PLAIN, 0, bw.RANK_SUB128, 0),
                                                (bw.FORM_BATCHED, 0, bw.RANK_SUB128, 0),
                                                (bw.FORM_BATCHED, 0, bw.RANK_SUB128, -1),
                                                (bw.FORM_BATCHED, 3, bw.RANK_PLANES, -1),
                                                (bw.FORM_BATCHED, 0, bw.RANK_SUB128, 64),
                                                (bw.FORM_BATCHED, 0, bw.RANK_SUB128, 1024)])
def test_c5_shape_stress_parity(form, wps, fmt, split):
    """250 bp reads, 6 differences with gaps, a tenth from repeat copies: a few
    reads expand hundreds of thousands of states.  In the batched form the
    lanes of a wave share the reads in flight once the batch runs dry, and a
    lane's part past the split budget is handed to tasks for the whole grid
    (0: the library's default, at which this small batch may split nothing;
    64: so small that slots and task room run out at this batch size and
    parts go on alone; -1: no splitting)."""
    g = configs.c2_genome(2_000_000, seed=55)
    reads = configs.c5_reads(g, 2000, seed=56)
    ox = oracle.Index(g.seq)
    ix = bw.Index(g.seq, **configs.FORMAT_LAYOUT[fmt]).upload()
    p, op = _params_pair(form=form, **configs.PARAMS["C5"])
    p.waves_per_simd = wps  # every build of the batched kernel
    p.split_budget = split
    op.bases_per_line = ix.info()["bases_per_line"]
    res = _gpu_align(ix, reads, p, counted=True)
    ores = oracle.align(ox, reads.bases, reads.offsets, op, threads=8)
    _compare_align(res, ores)
    st = res.status.cpu().numpy()
    work = res.work.cpu().numpy()
    if form == bw.FORM_BATCHED and split >= 0:
        n_split = int((st & bw.ST_SPLIT).astype(bool).sum())
        assert n_split > 0 or split == 0, "no search was split"
        # reads split = slots taken (those sent on to the second pass carry
        # the second pass's status instead)
        assert int(work[3]) == n_split + int(work[5]) and int(work[4]) > 0
        print(f"[c5-split {split}] {n_split} split reads, {int(work[4])} tasks, {int(work[5])} to the second pass, "
              f"per generation {work[6:14].tolist()}", flush=True)
    elif form == bw.FORM_BATCHED:
        assert int((st & bw.ST_SHARED).astype(bool).sum()) > 0, "no search tree was shared"
        assert not (st & bw.ST_SPLIT).any()
    else:
        assert not (st & (bw.ST_SHARED | bw.ST_SPLIT)).any()
    one = (st & (bw.ST_RESEARCH | bw.ST_SHARED | bw.ST_SPLIT)) == 0
    exp = res.expand.cpu().numpy().view(np.uint32)
    assert np.array_equal(exp[one], ores.counts["expand"][one].astype(np.uint32))


def test_split_budget_is_checked():
    g = gen.genome_iid(7, 100_000)
    reads = gen.reads_se(8, g, 50, 30, ps=0.0)
    ix = bw.Index(g.seq).upload()
    for b in (8, 15, (1 << 24) + 1, -2):
        with pytest.raises(bw.BwfmError) as e:
            _gpu_align(ix, reads, bw.Params(max_diff=1, split_budget=b))
        assert e.value.code == bw.E_INVAL


def test_hit_capacity_error_reports_need():
    g = gen.genome_iid(7, 100_000)
    reads = gen.reads_se(8, g, 200, 30, ps=0.0)
    ix = bw.Index(g.seq).upload()
    p = bw.Params(max_diff=1, max_gapo=0, mode=bw.MODE_ALL)
    bases, offs = _dev(reads.bases), _dev(reads.offsets.view(np.int64))
    res = bw.align_batch(ix, bases, offs, p, max_len=30, hit_capacity=1)  # grows and retries
    need = res.n_hits
    assert need > 1 and res.hits.shape[0] >= need
    with pytest.raises(bw.BwfmError) as e:
        out = bw.AlignResult(torch.empty(201, dtype=torch.int64, device="cuda"),
                             torch.empty((1, 4), dtype=torch.int32, device="cuda"),
                             torch.empty(200, dtype=torch.int32, device="cuda"),
                             torch.empty(200, dtype=torch.int32, device="cuda"),
                             torch.empty(200, dtype=torch.uint8, device="cuda"), 200)
        r = out._c()
        import ctypes
        rd = bw._reads_struct(bases, offs, None, 30)
        pc = p._c()
        bw._check(bw.lib().bwfm_align_batch(ix.handle, ctypes.byref(rd), ctypes.byref(pc), ctypes.byref(r),
                                            bw._stream_ptr(None)))
    assert e.value.code == bw.E_CAPACITY
    assert int(out.hit_offsets[200].item()) == need


@pytest.fixture(scope="module")
def c2_full():
    """The benchmark's workload at full size: 100 Mbp genome, 1M pairs, and
    the benchmark's index layout (64-byte lines of 192 rows, SA/32)."""
    g = configs.c2_genome()
    box = {}

    def build_oracle():
        box["ox"] = oracle.Index(g.seq)

    t = threading.Thread(target=build_oracle)
    t.start()
    ix = bw.Index(g.seq, **configs.LAYOUT["C2"]).upload()
    t.join()
    pairs = configs.c2_pairs(g)
    return g, pairs, ix, box["ox"]


@pytest.mark.timeout(600)
def test_c2_full_size_sampled_parity(c2_full):
    """Full batch through the GPU in the benchmark's launch configuration;
    a seeded sample of reads, and their pairs, checked against the oracle."""
    g, pairs, ix, ox = c2_full
    p, op = _params_pair(**configs.PARAMS["C2"])
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(pairs.end1.n, 200_000, replace=False))
    n = pairs.end1.n
    both = gen.Reads(np.concatenate([pairs.end1.bases, pairs.end2.bases]),
                     np.concatenate([pairs.end1.offsets[:-1], pairs.end1.offsets[-1] + pairs.end2.offsets]))
    full = _gpu_align(ix, both, p)
    res_e = []
    for e, end in enumerate((pairs.end1, pairs.end2)):
        res = full.window(e * n, (e + 1) * n)
        offs = end.offsets
        sb = np.concatenate([end.bases[offs[r]:offs[r + 1]] for r in sample])
        so = np.zeros(len(sample) + 1, np.uint64)
        so[1:] = np.cumsum(np.diff(offs)[sample])
        ores = oracle.align(ox, sb, so, op, threads=16)
        _compare_align(res, ores, rows=sample)
        res_e.append((res, ores, (sb, so)))
    # pairs of the sampled reads
    w = configs.PAIR_WINDOW
    gpd = bw.pair_reads(ix, res_e[0][0], res_e[1][0], w["lo"], w["hi"], w["mu"], configs.MAX_OCC)
    gp = bw.pairs_numpy(gpd)
    po1, pos1 = oracle.locate(ox, res_e[0][1].hits, configs.MAX_OCC)
    po2, pos2 = oracle.locate(ox, res_e[1][1].hits, configs.MAX_OCC)
    op_ = oracle.pair(res_e[0][1], po1, pos1, res_e[1][1], po2, pos2, w["lo"], w["hi"], w["mu"])
    assert np.array_equal(gp[sample].view(np.uint8), op_.view(np.uint8))
    # whole-batch properties: every pair got a record, most pair properly
    assert (gp["flags"] & bw.PF_PAIRED).mean() > 0.8
    # mate rescue over the whole batch; the sampled pairs against the oracle's
    # rescue of its own pair records
    ends = [(_dev(e.bases), _dev(e.offsets.view(np.int64))) for e in (pairs.end1, pairs.end2)]
    gr = bw.rescue_numpy(bw.rescue_mates(ix, ends[0], ends[1], gpd, w["lo"], w["hi"], max_len=100))
    orr = oracle.rescue(g.seq, res_e[0][2], res_e[1][2], op_, w["lo"], w["hi"])
    assert np.array_equal(gr[sample].view(np.uint8), orr.view(np.uint8))
    unpaired = (gp["flags"] & bw.PF_PAIRED) == 0
    assert (gr["end"][~unpaired] == 0).all() and (gr["end"][unpaired] != 0).sum() > 0


def _sample_reads(reads, rows):
    offs = reads.offsets
    sb = np.concatenate([reads.bases[offs[r]:offs[r + 1]] for r in rows])
    so = np.zeros(len(rows) + 1, np.uint64)
    so[1:] = np.cumsum(np.diff(offs)[rows])
    return sb, so


@pytest.mark.timeout(900)
def test_c5_full_size_sampled_parity(c2_full):
    """C5 at its stated size: the 100 Mbp genome, 2M single-end reads of
    250 bp (3% substitutions, 0.3% indel events, a tenth from repeat
    copies), at most 6 differences with a gap, no seed, all in one batched
    launch; 40,000 sampled reads against the oracle (hits, counts, status,
    located positions), at the default split budget and at 512 (the whole
    batch byte-identical between the two), and whole-batch properties."""
    g, _, ix, ox = c2_full
    reads = configs.c5_reads(g)
    assert reads.n == 2_000_000 and (np.diff(reads.offsets) == 250).all()
    p, op = _params_pair(**configs.PARAMS["C5"])
    print(f"[c5-full] aligning {reads.n} reads", flush=True)
    res = _gpu_align(ix, reads, p)
    rng = np.random.default_rng(1005)
    rows = np.sort(rng.choice(reads.n, 40_000, replace=False))
    sb, so = _sample_reads(reads, rows)
    ores = oracle.align(ox, sb, so, op, threads=16)
    _compare_align(res, ores, rows=rows)
    # positions of the sampled reads' hits
    ho = res.hit_offsets.cpu().numpy().view(np.uint64)
    po, pos = bw.locate(ix, res, configs.MAX_OCC)
    po, pos = po.cpu().numpy().view(np.uint64), pos.cpu().numpy().view(np.uint32)
    opo, opos = oracle.locate(ox, ores.hits, configs.MAX_OCC)
    for j, r in enumerate(rows[:5000]):
        a, b = int(ho[r]), int(ho[r + 1])
        oa, ob = int(ores.hit_off[j]), int(ores.hit_off[j + 1])
        assert b - a == ob - oa
        got = [pos[po[h]:po[h + 1]].tolist() for h in range(a, b)]
        exp = [opos[opo[h]:opo[h + 1]].tolist() for h in range(oa, ob)]
        assert got == exp, r
    # the split budget the C5 bench picks on this batch: the sample against
    # the oracle again, and the whole batch byte-identical to the default's
    p512, _ = _params_pair(**configs.PARAMS["C5"])
    p512.split_budget = 512
    print("[c5-full] aligning again at split budget 512", flush=True)
    res512 = _gpu_align(ix, reads, p512)
    _compare_align(res512, ores, rows=rows)
    a0, a1 = res.to_numpy(), res512.to_numpy()
    for x, y in zip(a0[:4], a1[:4]):
        assert x.tobytes() == y.tobytes()
    assert np.array_equal(a0[4] & 7, a1[4] & 7)
    st = res.status.cpu().numpy()
    ost = ores.status
    print(f"[c5-full] sample: {np.mean(ost & oracle.ST_HIT != 0):.3f} aligned, "
          f"{int((ost & oracle.ST_OVERFLOW).astype(bool).sum())} over max_hits; whole batch: "
          f"{np.mean(st & bw.ST_HIT != 0):.3f} aligned, {int((st & bw.ST_SHARED).astype(bool).sum())} shared trees",
          flush=True)
    assert not (st & bw.ST_INVALID).any()
