"""CPU-side checks of the library: it loads, exports every declared entry
point, and its host-built index equals the oracle's index bit for bit.  No
GPU call is made here."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_1505_07855_amd as bw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "bwfm.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    declared = set(re.findall(r"\b(bwfm_\w+)\s*\(", hdr))
    assert {"bwfm_build_index", "bwfm_align_batch", "bwfm_pair_reads", "bwfm_locate"} <= declared
    L = ctypes.CDLL(bw.LIB_PATH)
    for name in sorted(declared | set(bw.SYMBOLS)):
        assert hasattr(L, name), name
    assert set(bw.SYMBOLS) >= declared


def _texts(rng):
    yield "random", rng.integers(0, 4, 5000).astype(np.uint8)
    yield "one", np.array([2], np.uint8)
    yield "allA", np.zeros(1000, np.uint8)
    yield "period", np.resize(np.array([0, 1, 2, 3, 3], np.uint8), 3001)
    yield "binary", rng.integers(0, 2, 2048).astype(np.uint8)
    t = rng.integers(0, 4, 4000).astype(np.uint8)
    t[2000:3000] = t[500:1500]
    yield "repeat", t


@pytest.mark.parametrize("layout", [(128, 0, 32), (64, 0, 32), (64, 128, 32), (128, 64, 1), (64, 32, 8),
                                    (128, 448, 1024), (32, 0, 32), (32, 32, 4), (64, 0, 32, bw.RANK_SUBCOUNTS),
                                    (64, 160, 1, bw.RANK_SUBCOUNTS), (128, 0, 32, bw.RANK_SUB128),
                                    (128, 384, 1, bw.RANK_SUB128)])
def test_host_index_equals_oracle_index(layout, rng):
    lb, bpl, sas = layout[:3]
    fmt = layout[3] if len(layout) > 3 else bw.RANK_PLANES
    for name, t in _texts(rng):
        ix = bw.Index(t, line_bytes=lb, bases_per_line=bpl, sa_sample=sas, rank_format=fmt)
        assert ix.info()["rank_format"] == fmt
        ox = oracle.Index(t)
        info = ix.info()
        for which in (0, 1):
            sa, bwt, C, prim = ox.get(which)
            assert np.array_equal(ix.bwt(which), bwt), (name, which)
            assert info["primary"][which] == prim
            assert info["C"][which] == C.tolist()
            samp = ix.sa_samples(which)
            assert np.array_equal(samp, sa[::sas]), (name, which)
            rows = np.unique(np.concatenate([rng.integers(0, len(t) + 2, 60), [0, 1, len(t), len(t) + 1]]))
            for i in rows:
                assert ix.occ(int(i), which).tolist() == ox.occ4(int(i), which).tolist(), (name, which, i)
        # the packed reference the index keeps for mate rescue
        assert np.array_equal(ix.ref(), t), name
        if len(t) > 20:
            assert np.array_equal(ix.ref(len(t) - 17, 17), t[-17:])
        ix.close()


def test_build_index_errors():
    with pytest.raises(bw.BwfmError) as e:
        bw.Index(np.array([0, 1, 5], np.uint8))
    assert e.value.code == -3
    with pytest.raises(bw.BwfmError) as e:
        bw.Index(np.zeros(10, np.uint8), line_bytes=96)
    assert e.value.code == -1
    with pytest.raises(bw.BwfmError) as e:
        bw.Index(np.zeros(10, np.uint8), line_bytes=64, bases_per_line=256)
    assert e.value.code == -1
    with pytest.raises(bw.BwfmError) as e:
        bw.Index(np.zeros(10, np.uint8), sa_sample=3)
    assert e.value.code == -1
    with pytest.raises(bw.BwfmError):
        bw.Index(np.zeros(0, np.uint8))
    for kw in (dict(line_bytes=128), dict(line_bytes=64, bases_per_line=192), dict(line_bytes=32)):
        with pytest.raises(bw.BwfmError) as e:  # sub-counted lines are 64 bytes of 160 rows
            bw.Index(np.zeros(10, np.uint8), rank_format=bw.RANK_SUBCOUNTS, **kw)
        assert e.value.code == -1
    with pytest.raises(bw.BwfmError):
        bw.Index(np.zeros(10, np.uint8), rank_format=7)


def test_host_helpers_match_oracle(rng):
    for L in range(1, 513):
        assert bw.max_diff_rule(L) == oracle.max_diff_rule(L)
    for n in [0, 10, 99, 100, 101, 1000, 5000]:
        ins = np.round(rng.normal(300, 30, n)).astype(np.int32)
        if n > 5:
            ins[:3] = [5, 9000, 12000]
        assert bw.estimate_insert(ins) == oracle.estimate_insert(ins)


def test_align_without_upload_is_a_state_error():
    ix = bw.Index(np.zeros(100, np.uint8))
    assert not ix.info()["uploaded"]
    ix.close()


def test_kmer_table_state_errors_on_a_host_index():
    """The short-string table lives on the device: on an index that was
    never uploaded it reports no levels, refuses to build and has no entries
    to read.  Both checks come before any device call, so the C entry points
    are called directly with a null stream."""
    g = np.random.default_rng(5).integers(0, 4, 2000).astype(np.uint8)
    ix = bw.Index(g, line_bytes=64)
    info = ix.info()
    assert info["kmer_levels"] == 0 and info["kmer_bytes"] == 0
    L = bw.lib()
    for levels in (-1, 0, 3):
        assert L.bwfm_index_kmer_table(ix._h, levels, None) == -1  # BWFM_E_INVAL
        assert b"not uploaded" in L.bwfm_last_error()
    out = np.zeros(2, np.uint32)
    assert L.bwfm_index_kmer_get(ix._h, 0, 0, 0, 1, out.ctypes.data) == -1
    assert L.bwfm_index_kmer_table(None, 3, None) == -1
    ix.close()


@pytest.mark.parametrize("fmt", [bw.RANK_PLANES, bw.RANK_SUBCOUNTS])
def test_index_save_load_roundtrip_and_corruption(rng, tmp_path, fmt):
    t = rng.integers(0, 4, 7000).astype(np.uint8)
    t[3000:4000] = t[100:1100]
    ix = bw.Index(t, line_bytes=64, sa_sample=8, rank_format=fmt)
    path = str(tmp_path / "x.bwfm")
    ix.save(path)
    iy = bw.Index.load(path)
    a, b = ix.info(), iy.info()
    for k in ("n", "primary", "C", "lines", "sa_samples", "line_bytes", "bases_per_line", "sa_sample", "rank_format"):
        assert a[k] == b[k], k
    assert not b["uploaded"]
    for which in (0, 1):
        assert np.array_equal(ix.bwt(which), iy.bwt(which))
        assert np.array_equal(ix.sa_samples(which), iy.sa_samples(which))
        for i in rng.integers(0, len(t) + 2, 50):
            assert ix.occ(int(i), which).tolist() == iy.occ(int(i), which).tolist()
    assert np.array_equal(iy.ref(), t)
    with pytest.raises(bw.BwfmError):
        iy.ref(len(t) - 5, 6)
    iy.close()
    raw = bytearray(open(path, "rb").read())
    # a flipped byte in a rank line, a truncated file, another file format
    for name, data in (("flip", raw[:200] + bytes([raw[200] ^ 1]) + raw[201:]), ("short", raw[:-9]),
                       ("flip_ref", raw[:-20] + bytes([raw[-20] ^ 4]) + raw[-19:]),
                       ("version", raw[:8] + bytes([1, 0, 0, 0]) + raw[12:]),
                       ("magic", b"NOTANIDX" + raw[8:])):
        bad = str(tmp_path / f"{name}.bwfm")
        open(bad, "wb").write(bytes(data))
        with pytest.raises(bw.BwfmError) as e:
            bw.Index.load(bad)
        assert e.value.code == bw.E_IO, name
    with pytest.raises(bw.BwfmError) as e:
        bw.Index.load(str(tmp_path / "missing.bwfm"))
    assert e.value.code == bw.E_IO
    ix.close()


def test_variant_genes_match_the_source_defaults():
    """The variant search's reference values are the kernel source's own
    defaults, so its reference build is the shipped library; its first
    generation changes one gene at a time; the next generation combines the
    parent with the genes of variants that beat the reference; the test
    variants use only declared genes and alternatives."""
    import re

    from paper_1505_07855_amd import variants
    src = open(os.path.join(os.path.dirname(bw.__file__), "csrc", "bwfm.hip")).read()
    for gene, (ref, alts) in variants.GENES.items():
        m = re.search(r"#ifndef %s\n#define %s (\d+)\n#endif" % (gene, gene), src)
        assert m and int(m.group(1)) == ref, gene
        assert ref not in alts
        if gene.startswith("BWFM_GENE_"):
            # the source branches on the gene
            assert re.search(r"%s == \d" % gene, src), gene
    first = variants.first_generation()
    names = [variants.name_of(d) for d in first]
    assert names[0] == "reference" and len(names) == len(set(names)) == 1 + sum(len(a) for _, a in
                                                                               variants.GENES.values())
    for d in variants.TEST_VARIANTS:
        assert all(k in variants.GENES and v in variants.GENES[k][1] for k, v in d.items())
    # a generation after singles: the parent (the fastest single) combined
    # with each other single that beat the reference, never re-evaluating one
    table = [{"defines": d, "accepted": True, "ms": 100.0 - i} for i, d in enumerate(first)]
    table[2]["accepted"] = False
    state = {"table": table, "reference_ms": 100.0, "parent": table[-1]}
    kids = variants.next_generation(state)
    parent = table[-1]["defines"]
    assert kids and all(len(k) == 2 and all(parent.items() <= k.items() for _ in [0]) for k in kids)
    assert not any(first[2].items() <= k.items() for k in kids)
    assert len({variants.name_of(k) for k in kids}) == len(kids)


@pytest.mark.parametrize("shape", ["C1", "C2"])
def test_host_index_equals_oracle_index_at_workload_size(shape):
    """The host builder against the oracle on the C1 genome in full (1 Mbp)
    and on a 4 Mbp genome built like the 100 Mbp one, in the workload's
    layout and in sub-counted lines."""
    from gen import configs
    from tests.util import assert_index_equals_oracle
    g = configs.c1_genome() if shape == "C1" else configs.c2_genome(4_000_000, seed=64)
    ox = oracle.Index(g.seq)
    for lay in (dict(configs.LAYOUT[shape]), dict(configs.FORMAT_LAYOUT[bw.RANK_SUBCOUNTS]),
                dict(configs.FORMAT_LAYOUT[bw.RANK_PLANES])):
        ix = bw.Index(g.seq, **lay)
        assert_index_equals_oracle(ix, ox, name=f"{shape} {lay}")
        ix.close()
