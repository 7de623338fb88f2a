"""Child process of tests/test_gpu_variants.py: load the variant library
named on the command line in place of the shipped one and check it against
the oracle on a small paired-end batch -- both rank-line layouts the
variants touch (64-byte planar, 128-byte sub-counted), without and with a
short-string table, the batched form (also with nearly every read's search
split into task rounds) and the plain form, then locate and pairing.
Prints "variant ok" on success."""
from __future__ import annotations

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))


def main(lib: str) -> None:
    import numpy as np
    import torch

    import oracle
    import paper_1505_07855_amd as bw
    from gen import configs

    bw.LIB_PATH = lib
    assert os.path.samefile(bw.LIB_PATH, lib)
    print(f"[variant] {lib}", flush=True)
    g = configs.c2_genome(2_000_000, seed=101)
    pairs = configs.c2_pairs(g, 2000, seed=102)
    ox = oracle.Index(g.seq)
    op = oracle.Params(**configs.PARAMS["C2"])
    w = configs.PAIR_WINDOW
    ores = [oracle.align(ox, e.bases, e.offsets, op, threads=8) for e in (pairs.end1, pairs.end2)]
    locs = [oracle.locate(ox, r.hits, configs.MAX_OCC) for r in ores]
    opr = oracle.pair(ores[0], locs[0][0], locs[0][1], ores[1], locs[1][0], locs[1][1], w["lo"], w["hi"], w["mu"])
    ends = [(torch.from_numpy(e.bases).cuda(), torch.from_numpy(e.offsets.view(np.int64)).cuda())
            for e in (pairs.end1, pairs.end2)]
    for lb, fmt, levels in ((64, bw.RANK_PLANES, 0), (128, bw.RANK_SUB128, 0), (128, bw.RANK_SUB128, 6),
                            (64, bw.RANK_PLANES, 9)):
        ix = bw.Index(g.seq, line_bytes=lb, sa_sample=32, rank_format=fmt).upload(kmer_levels=levels)
        # the batched form at the default split budget and at one so small
        # that nearly every read's search is split into task rounds
        for form, split in ((bw.FORM_BATCHED, 0), (bw.FORM_BATCHED, 32), (bw.FORM_PLAIN, 0)):
            p = bw.Params(**configs.PARAMS["C2"], form=form, split_budget=split)
            res = [bw.align_batch(ix, b, o, p, max_len=100) for b, o in ends]
            if split:
                assert any((r.status.cpu().numpy() & bw.ST_SPLIT).any() for r in res), "no search was split"
            for r, orr in zip(res, ores):
                ho, hits, c1, c2, st = r.to_numpy()
                assert np.array_equal(ho, orr.hit_off), (lb, form)
                assert np.array_equal(hits.view(np.uint8), orr.hits.view(np.uint8)), (lb, form)
                assert np.array_equal(c1, orr.c1) and np.array_equal(c2, orr.c2), (lb, form)
                assert np.array_equal(st & 7, orr.status), (lb, form)
            po, pos = bw.locate(ix, res[0], configs.MAX_OCC)
            assert np.array_equal(po.cpu().numpy().view(np.uint64), locs[0][0]), (lb, form)
            assert np.array_equal(pos.cpu().numpy().view(np.uint32), locs[0][1]), (lb, form)
            prs = bw.pair_reads(ix, res[0], res[1], w["lo"], w["hi"], w["mu"], configs.MAX_OCC)
            assert np.array_equal(bw.pairs_numpy(prs).view(np.uint8), opr.view(np.uint8)), (lb, form)
        ix.close()
    print("variant ok", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
