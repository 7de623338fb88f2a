"""Concurrent calls on one index: align, locate and pair on two streams from
two host threads at once give the same bytes as the same calls made one
after the other (and the first batch equals the oracle), each stream keeps
its own workspace, and repeated calls stop allocating once the workspace
has grown to the batch."""
from __future__ import annotations

import threading

import numpy as np
import pytest

import oracle
import paper_1505_07855_amd as bw
from gen import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _path(ix, p, batch, stream):
    """Both ends aligned, end 1 located, the pairs decided, all on
    `stream`; returns the bytes of every output."""
    w = configs.PAIR_WINDOW
    with torch.cuda.stream(stream):
        res = []
        for b, o in batch:
            res.append(bw.align_batch(ix, b, o, p, max_len=100, stream=stream))
        po, pos = bw.locate(ix, res[0], configs.MAX_OCC, stream=stream)
        prs = bw.pair_reads(ix, res[0], res[1], w["lo"], w["hi"], w["mu"], configs.MAX_OCC, stream=stream)
        stream.synchronize()
        out = [x.tobytes() for r in res for x in r.to_numpy()]
        out += [po.cpu().numpy().tobytes(), pos.cpu().numpy().tobytes(), prs.cpu().numpy().tobytes()]
    return out


def test_two_streams_concurrently_equal_serial_and_oracle():
    g = configs.c2_genome(2_000_000, seed=81)
    ix = bw.Index(g.seq, **configs.LAYOUT["C2"]).upload()
    p = bw.Params(**configs.PARAMS["C2"])
    batches, pair_sets = [], []
    for seed in (82, 83):
        pairs = configs.c2_pairs(g, 3000, seed=seed)
        pair_sets.append(pairs)
        batches.append([(torch.from_numpy(e.bases).cuda(), torch.from_numpy(e.offsets.view(np.int64)).cuda())
                        for e in (pairs.end1, pairs.end2)])
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ref = [_path(ix, p, batches[k], streams[k]) for k in (0, 1)]
    assert ref[0] != ref[1]
    info = ix.info()
    assert info["ws_streams"] >= 2
    # the first batch against the oracle
    ox = oracle.Index(g.seq)
    op = oracle.Params(**configs.PARAMS["C2"])
    pairs = pair_sets[0]
    ores = [oracle.align(ox, e.bases, e.offsets, op, threads=8) for e in (pairs.end1, pairs.end2)]
    exp = []
    for r in ores:
        exp += [r.hit_off.tobytes(), r.hits.tobytes(), r.c1.tobytes(), r.c2.tobytes()]
    got = ref[0][:4] + ref[0][5:9]
    assert got == exp
    po1, pos1 = oracle.locate(ox, ores[0].hits, configs.MAX_OCC)
    po2, pos2 = oracle.locate(ox, ores[1].hits, configs.MAX_OCC)
    assert ref[0][10] == po1.tobytes() and ref[0][11] == pos1.tobytes()
    w = configs.PAIR_WINDOW
    opr = oracle.pair(ores[0], po1, pos1, ores[1], po2, pos2, w["lo"], w["hi"], w["mu"])
    assert ref[0][12] == opr.tobytes()
    # both streams at once, from two threads, several rounds
    start = threading.Barrier(2)
    errors = []

    def worker(k):
        try:
            start.wait()
            for it in range(4):
                out = _path(ix, p, batches[k], streams[k])
                if out != ref[k]:
                    errors.append((k, it))
        except Exception as e:  # reported below
            errors.append((k, repr(e)))

    ths = [threading.Thread(target=worker, args=(k,)) for k in (0, 1)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    assert not errors, errors
    # the workspaces have reached the batches' size: no more growth
    b0 = ix.info()["ws_bytes"]
    for k in (0, 1, 0):
        assert _path(ix, p, batches[k], streams[k]) == ref[k]
    assert ix.info()["ws_bytes"] == b0
    ix.close()
