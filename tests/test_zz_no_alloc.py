"""bwfm_pair_reads_noalloc: the same records as bwfm_pair_reads from the
library's fixed device scratch, on two calls in a row (the second smaller),
paired and single-end; the per-stream workspace is left untouched; a batch
whose hits cannot fit the scratch is refused before anything is written."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import oracle
import paper_1505_07855_amd as bw
from gen import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _align_ends(ix, p, pairs):
    out = []
    for e in (pairs.end1, pairs.end2):
        b = torch.from_numpy(e.bases).cuda()
        o = torch.from_numpy(e.offsets.view(np.int64)).cuda()
        out.append(bw.align_batch(ix, b, o, p, max_len=100))
    return out


def test_noalloc_pairs_equal_allocating_pairs_on_two_calls():
    print("[noalloc] two calls, 3000 then 700 pairs, 2 Mbp genome", flush=True)
    g = configs.c2_genome(2_000_000, seed=91)
    ix = bw.Index(g.seq, **configs.LAYOUT["C2"]).upload()
    p = bw.Params(**configs.PARAMS["C2"])
    w = configs.PAIR_WINDOW
    ox = oracle.Index(g.seq)
    op = oracle.Params(**configs.PARAMS["C2"])
    stream = torch.cuda.current_stream()
    sizes = (3000, 700)
    results = [_align_ends(ix, p, configs.c2_pairs(g, n, seed=92 + k)) for k, n in enumerate(sizes)]
    torch.cuda.synchronize()
    ws0 = ix.info()["ws_bytes"]
    outs = []
    for (r1, r2), n in zip(results, sizes):
        out = torch.full((n, bw.PAIR_DTYPE.itemsize), 0xAB, dtype=torch.uint8, device="cuda")
        got = bw.pair_reads(ix, r1, r2, w["lo"], w["hi"], w["mu"], configs.MAX_OCC, stream=stream, out=out,
                            noalloc=True)
        assert got.data_ptr() == out.data_ptr()
        outs.append(out.cpu().numpy().copy())
    # the non-allocating calls did not touch the stream's workspace
    assert ix.info()["ws_bytes"] == ws0
    for ((r1, r2), n), got in zip(zip(results, sizes), outs):
        exp = bw.pair_reads(ix, r1, r2, w["lo"], w["hi"], w["mu"], configs.MAX_OCC, stream=stream)
        assert np.array_equal(got, exp.cpu().numpy()[:n]), n
    # and against the oracle on the first batch
    pairs = configs.c2_pairs(g, sizes[0], seed=92)
    ores = [oracle.align(ox, e.bases, e.offsets, op, threads=8) for e in (pairs.end1, pairs.end2)]
    po1, pos1 = oracle.locate(ox, ores[0].hits, configs.MAX_OCC)
    po2, pos2 = oracle.locate(ox, ores[1].hits, configs.MAX_OCC)
    opr = oracle.pair(ores[0], po1, pos1, ores[1], po2, pos2, w["lo"], w["hi"], w["mu"])
    assert np.array_equal(outs[0], opr.view(np.uint8).reshape(sizes[0], -1))
    # single-end primaries, again larger then smaller
    for (r1, _), n in zip(results, sizes):
        got = bw.pair_reads(ix, r1, None, w["lo"], w["hi"], w["mu"], configs.MAX_OCC, stream=stream, noalloc=True)
        exp = bw.pair_reads(ix, r1, None, w["lo"], w["hi"], w["mu"], configs.MAX_OCC, stream=stream)
        assert np.array_equal(got.cpu().numpy()[:n], exp.cpu().numpy()[:n]), n
    ix.close()


def test_noalloc_refuses_hits_beyond_the_scratch():
    print("[noalloc] oversized hit count refused on the host", flush=True)
    g = configs.c2_genome(200_000, seed=95)
    ix = bw.Index(g.seq, **configs.LAYOUT["C2"]).upload()
    # one pair whose ends claim 5M hits each: the control area alone exceeds
    # the scratch, so the call stops before any kernel reads the hits
    claimed = 5_000_000
    assert claimed * 24 > bw.NOALLOC_SCRATCH_BYTES
    offs = torch.tensor([0, claimed], dtype=torch.int64, device="cuda")
    hits = torch.zeros((1, 4), dtype=torch.int32, device="cuda")
    small = [torch.zeros(1, dtype=torch.int32, device="cuda") for _ in range(2)]
    st = torch.zeros(1, dtype=torch.uint8, device="cuda")
    res = bw.AlignResult(offs, hits, small[0], small[1], st, 1)
    a = res._c()
    pp = bw._PairParams(0, 500, 300, configs.MAX_OCC)
    out = torch.full((1, bw.PAIR_DTYPE.itemsize), 0xAB, dtype=torch.uint8, device="cuda")
    rc = bw.lib().bwfm_pair_reads_noalloc(ix.handle, 1, ctypes.byref(a), ctypes.byref(a), ctypes.byref(pp),
                                          bw._dptr(out), bw._stream_ptr(None))
    assert rc == bw.E_CAPACITY
    assert b"scratch" in bw.lib().bwfm_last_error()
    assert (out.cpu().numpy() == 0xAB).all()
    ix.close()
