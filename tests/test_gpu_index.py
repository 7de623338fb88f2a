"""The device index builder against the oracle's index (BWT, $ row, C, every
SA sample, Occ at random rows, the packed reference) and against the host
builder byte for byte, on texts that stress a suffix sort: random, one
symbol repeated, short periods, long exact repeats, a 3 Mbp and a 16 Mbp
genome built like the 100 Mbp one; and its index aligns like the host
one."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_1505_07855_amd as bw
from gen import configs
from util import assert_index_equals_oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _texts():
    rng = np.random.default_rng(5)
    yield "one", np.array([2], np.uint8)
    yield "random", rng.integers(0, 4, 100_003).astype(np.uint8)
    yield "allA", np.zeros(5000, np.uint8)
    yield "period5", np.resize(np.array([0, 1, 2, 3, 3], np.uint8), 30_001)
    yield "binary", rng.integers(0, 2, 20_000).astype(np.uint8)
    t = rng.integers(0, 4, 200_000).astype(np.uint8)
    t[100_000:150_000] = t[10_000:60_000]  # a 50 kbp exact repeat: many doubling rounds
    yield "repeat", t
    yield "c2", configs.c2_genome(3_000_000, seed=61).seq


_ORACLE = {}


def _oracle_index(name, t):
    if name not in _ORACLE:
        _ORACLE[name] = oracle.Index(t)
    return _ORACLE[name]


def _host_bytes(ix):
    info = ix.info()
    out = [info["primary"], info["C"], info["lines"], info["sa_samples"]]
    for which in (0, 1):
        out.append(ix.bwt(which).tobytes())
        out.append(ix.sa_samples(which).tobytes())
    out.append(ix.ref().tobytes())
    return out


@pytest.mark.parametrize("layout", [(64, 0, 32), (128, 0, 32), (64, 128, 8), (32, 0, 32),
                                    (64, 0, 32, bw.RANK_SUBCOUNTS), (128, 0, 32, bw.RANK_SUB128)])
def test_device_index_equals_host_index(layout):
    lb, bpl, sas = layout[:3]
    fmt = layout[3] if len(layout) > 3 else bw.RANK_PLANES
    rng = np.random.default_rng(9)
    for name, t in _texts():
        a = bw.Index(t, line_bytes=lb, bases_per_line=bpl, sa_sample=sas, rank_format=fmt)
        b = bw.Index.build_device(t, line_bytes=lb, bases_per_line=bpl, sa_sample=sas, rank_format=fmt)
        assert b.info()["uploaded"]
        assert_index_equals_oracle(b, _oracle_index(name, t), rows_per_dir=60, name=f"{name} {layout}")
        assert _host_bytes(a) == _host_bytes(b), name
        for which in (0, 1):
            for i in np.unique(np.concatenate([rng.integers(0, len(t) + 2, 40), [0, len(t), len(t) + 1]])):
                assert a.occ(int(i), which).tolist() == b.occ(int(i), which).tolist(), (name, which, i)
        a.close()
        b.close()


def _layout(fmt):
    """The format's own layout, without its rank_format key."""
    lay = dict(configs.FORMAT_LAYOUT[fmt])
    del lay["rank_format"]
    return lay


@pytest.mark.parametrize("fmt", [bw.RANK_PLANES, bw.RANK_SUBCOUNTS, bw.RANK_SUB128])
def test_device_index_aligns_like_host_index(fmt):
    g = configs.c2_genome(2_000_000, seed=62)
    pairs = configs.c2_pairs(g, 1000, seed=63)
    p = bw.Params(**configs.PARAMS["C2"])
    out = []
    lay = _layout(fmt)
    for ix in (bw.Index(g.seq, **lay, rank_format=fmt).upload(), bw.Index.build_device(g.seq, **lay, rank_format=fmt)):
        e = pairs.end1
        res = bw.align_batch(ix, torch.from_numpy(e.bases).cuda(), torch.from_numpy(e.offsets.view(np.int64)).cuda(), p,
                             max_len=100)
        out.append([x.tobytes() for x in res.to_numpy()])
    assert out[0] == out[1]


@pytest.mark.parametrize("fmt", [bw.RANK_PLANES, bw.RANK_SUBCOUNTS, bw.RANK_SUB128])
def test_device_index_equals_oracle_at_16_mbp(fmt):
    """A 16 Mbp genome built like the 100 Mbp one: many prefix-doubling
    rounds over repeat copies, rank lines across many device blocks."""
    g = configs.c2_genome(16_000_000, seed=65)
    ox = _oracle_index("c2_16m", g.seq)
    lay = _layout(fmt)
    b = bw.Index.build_device(g.seq, **lay, rank_format=fmt)
    assert_index_equals_oracle(b, ox, rows_per_dir=400, name=f"16 Mbp fmt {fmt}")
    b.close()
