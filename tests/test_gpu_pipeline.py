"""The captured step (align both ends, locate, pair as one hipGraph) against
the oracle: eager and replayed runs, replays separated by other device work
and synchronisations, a smaller batch after a larger one (counts are read on
the device), and the capacity errors it reports instead of failing."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_1505_07855_amd as bw
from gen import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _both(pairs, n):
    e1, e2 = pairs.end1, pairs.end2
    b = np.concatenate([e1.bases[:int(e1.offsets[n])], e2.bases[:int(e2.offsets[n])]])
    o = np.concatenate([e1.offsets[:n], e1.offsets[n] + e2.offsets[:n + 1]]).astype(np.uint64)
    return b, o


@pytest.fixture(scope="module")
def setup():
    g = configs.c2_genome(2_000_000, seed=71)
    pairs = configs.c2_pairs(g, 2500, seed=72)
    ox = oracle.Index(g.seq)
    ix = bw.Index(g.seq, **configs.LAYOUT["C2"]).upload()
    return g, pairs, ox, ix


def _expected(ox, pairs, n, op, w):
    res, locs = [], []
    for e in (pairs.end1, pairs.end2):
        b, o = e.bases[:int(e.offsets[n])], e.offsets[:n + 1]
        r = oracle.align(ox, b, o, op, threads=8)
        res.append(r)
        locs.append(oracle.locate(ox, r.hits, configs.MAX_OCC))
    pr = oracle.pair(res[0], locs[0][0], locs[0][1], res[1], locs[1][0], locs[1][1], w["lo"], w["hi"], w["mu"])
    return res, locs, pr


def _check_run(pl, n, exp, split=0):
    res, locs, pr = exp
    st = pl.finish()
    assert st["error"] == 0 and st["n_pairs"] == n
    r1, r2, prs, po, pos = pl.results()
    if split > 0 and n:
        assert any((r.status.cpu().numpy() & bw.ST_SPLIT).any() for r in (r1, r2)), "no search was split"
    for got, want in ((r1, res[0]), (r2, res[1])):
        ho, hits, c1, c2, s = got.to_numpy()
        assert np.array_equal(ho, want.hit_off)
        assert np.array_equal(hits.view(np.uint8), want.hits.view(np.uint8))
        assert np.array_equal(c1, want.c1) and np.array_equal(c2, want.c2)
        assert np.array_equal(s & 7, want.status)
    # positions: hits of end 1 then end 2, in order
    po_h = po.cpu().numpy().view(np.uint64)
    pos_h = pos[:int(po_h[-1])].cpu().numpy().view(np.uint32)
    want_po = np.concatenate([locs[0][0][:-1], locs[0][0][-1] + locs[1][0]])
    want_pos = np.concatenate([locs[0][1], locs[1][1]])
    assert np.array_equal(po_h, want_po) and np.array_equal(pos_h, want_pos)
    assert np.array_equal(prs.cpu().numpy().reshape(-1), pr.view(np.uint8).reshape(-1))
    assert st["n_hits"] == int(po_h.shape[0] - 1) and st["n_positions"] == len(want_pos)


@pytest.mark.parametrize("form,fmt,split", [(bw.FORM_BATCHED, bw.RANK_PLANES, 0), (bw.FORM_PLAIN, bw.RANK_PLANES, 0),
                                            (bw.FORM_BATCHED, bw.RANK_SUBCOUNTS, 0),
                                            (bw.FORM_BATCHED, bw.RANK_SUB128, 0),
                                            (bw.FORM_BATCHED, bw.RANK_SUB128, 16),
                                            (bw.FORM_BATCHED, bw.RANK_PLANES, -1)])
def test_pipeline_eager_and_graph_replays_equal_oracle(setup, form, fmt, split):
    """split 16: nearly every read's search is split, so every replay runs
    the task rounds and the slot publication; -1: splitting off."""
    g, pairs, ox, ix = setup
    if fmt != ix.info()["rank_format"]:
        ix = bw.Index(g.seq, **configs.FORMAT_LAYOUT[fmt]).upload()
    w = configs.PAIR_WINDOW
    p = bw.Params(**configs.PARAMS["C2"], form=form, split_budget=split)
    op = oracle.Params(**configs.PARAMS["C2"])
    N = 2500
    pl = bw.Pipeline(ix, p, w["lo"], w["hi"], w["mu"], configs.MAX_OCC, max_pairs=N, max_len=100)
    b, o = _both(pairs, N)
    pl.set_reads(torch.from_numpy(b).cuda(), torch.from_numpy(o.view(np.int64)).cuda(), N, max_len=100)
    exp = _expected(ox, pairs, N, op, w)
    pl.run(graph=False)
    _check_run(pl, N, exp, split)
    for k in range(3):
        pl.run(graph=True)
        _check_run(pl, N, exp, split)
        # unrelated device work and a synchronisation between replays
        x = torch.arange(1 << 20, device="cuda", dtype=torch.int64)
        assert int(x.sum().item()) == (1 << 20) * ((1 << 20) - 1) // 2
        torch.cuda.synchronize()
    if fmt == bw.RANK_SUBCOUNTS:
        # the short-string table replaced after capture: the next run
        # captures again (the old graph holds the freed table's address)
        for K in (0, 4, -1):
            ix.kmer_table(K)
            pl.run(graph=True)
            _check_run(pl, N, exp)
    # a replay with the search kernel timed by events captured into the graph
    bw.timing_enable(True)
    try:
        pl.run(graph=True)
        _check_run(pl, N, exp)
    finally:
        bw.timing_enable(False)
    # a smaller batch replays the same graph
    n2 = 777
    b2, o2 = _both(pairs, n2)
    pl.set_reads(torch.from_numpy(b2).cuda(), torch.from_numpy(o2.view(np.int64)).cuda(), n2, max_len=100)
    pl.run(graph=True)
    _check_run(pl, n2, _expected(ox, pairs, n2, op, w))
    # and an empty one
    pl.set_reads(torch.zeros(1, dtype=torch.uint8, device="cuda"), torch.zeros(1, dtype=torch.int64, device="cuda"),
                 0, max_len=100)
    pl.run(graph=True)
    st = pl.finish()
    assert st["error"] == 0 and st["n_hits"] == 0 and st["n_pairs"] == 0
    pl.close()


def test_pipeline_reports_capacity_errors(setup):
    g, pairs, ox, ix = setup
    w = configs.PAIR_WINDOW
    p = bw.Params(**configs.PARAMS["C2"])
    N = 600
    b, o = _both(pairs, N)
    bt, ot = torch.from_numpy(b).cuda(), torch.from_numpy(o.view(np.int64)).cuda()
    op = oracle.Params(**configs.PARAMS["C2"])
    res, locs, _ = _expected(ox, pairs, N, op, w)
    need_hits = len(res[0].hits) + len(res[1].hits)
    need_pos = len(locs[0][1]) + len(locs[1][1])
    pl = bw.Pipeline(ix, p, w["lo"], w["hi"], w["mu"], configs.MAX_OCC, max_pairs=N, max_len=100,
                     hit_capacity=need_hits - 1)
    pl.set_reads(bt, ot, N, max_len=100)
    pl.run(graph=True)
    st = pl.finish()
    assert st["error"] == bw.PIPE_E_HITS and st["n_hits"] == need_hits
    pl.close()
    pl = bw.Pipeline(ix, p, w["lo"], w["hi"], w["mu"], configs.MAX_OCC, max_pairs=N, max_len=100,
                     pos_capacity=need_pos - 1)
    pl.set_reads(bt, ot, N, max_len=100)
    pl.run(graph=True)
    st = pl.finish()
    assert st["error"] == bw.PIPE_E_POSITIONS and st["n_positions"] == need_pos
    # too many pairs for the pipeline
    with pytest.raises(bw.BwfmError) as e:
        b3, o3 = _both(pairs, N + 1)
        pl.set_reads(torch.from_numpy(b3).cuda(), torch.from_numpy(o3.view(np.int64)).cuda(), N + 1, max_len=100)
    assert e.value.code == bw.E_CAPACITY
    pl.close()
