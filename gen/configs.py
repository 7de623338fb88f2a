"""Workload recipes: synthetic stand-ins for the paper's data.

The paper measures on hg19 with 1000 Genomes ERR001270 (36 bp pairs) and the
GCAT 100 bp small-indel pair set (Genetically Improved BarraCUDA, sections
3.4-3.6); none of those are available here.  These recipes draw seeded
synthetic genomes and reads of the same shape instead.  Each holds plain
numbers (sizes, rates, parameter values) and calls into ``gen``; none of the
alignment method's arithmetic lives here.

Parameter presets are dictionaries accepted both by ``oracle.Params`` and by
the library binding's ``Params``.
"""
from __future__ import annotations

import numpy as np

import gen

# search parameters per workload (BWA's documented defaults elsewhere:
# s_mm 3, s_gapo 11, s_gape 4, indel_end_skip 5, max_best 30)
PARAMS = {
    "C1": dict(max_diff=2, max_gapo=0, seed_len=0),
    "C2": dict(max_diff=4, max_gapo=1, seed_len=32, seed_diff=2),
    "C3": dict(max_diff=4, max_gapo=1, seed_len=32, seed_diff=2),   # per-read budgets override max_diff
    "C5": dict(max_diff=6, max_gapo=1, seed_len=0),
}
# index layout per workload: line size, rows per rank line, SA sample
# interval, rank-line format (0: counts + bit planes; 1: 64-byte sub-counted
# lines of 160 rows; 2: 128-byte sub-counted lines of 384 rows).  C1 keeps
# its stated checkpoint every 128 rows; the others use the layout the
# benchmark's autotuner picks.
LAYOUT = {
    "C1": dict(line_bytes=64, bases_per_line=128, sa_sample=32, rank_format=0),
    "C2": dict(line_bytes=128, bases_per_line=384, sa_sample=32, rank_format=2),
    "C3": dict(line_bytes=128, bases_per_line=384, sa_sample=32, rank_format=2),
    "C5": dict(line_bytes=128, bases_per_line=384, sa_sample=32, rank_format=2),
}
# one layout per rank-line format, for tests that sweep them
FORMAT_LAYOUT = {
    0: dict(line_bytes=64, bases_per_line=192, sa_sample=32, rank_format=0),
    1: dict(line_bytes=64, bases_per_line=160, sa_sample=32, rank_format=1),
    2: dict(line_bytes=128, bases_per_line=384, sa_sample=32, rank_format=2),
}
# fixed insert window for the N(300, 30) fragment model: mu +- 4 sd
PAIR_WINDOW = dict(lo=180, hi=420, mu=300)
MAX_OCC = 100000
C3_LENGTHS = (36, 51, 76, 100, 150)


def c1_genome(n: int = 1_000_000) -> gen.Genome:
    """1 Mbp i.i.d. uniform ACGT."""
    return gen.genome_iid(1001, n, 0.5)


def c1_reads(g: gen.Genome, n_reads: int = 10_000) -> gen.Reads:
    """36 bp single-end reads, either strand, 2% i.i.d. substitutions."""
    return gen.reads_se(1001, g, n_reads, 36, ps=0.02)


def c2_genome(n: int = 100_000_000, seed: int = 1002) -> gen.Genome:
    """GC 41%, 40% repeat copies of 500 families (300 bp - 6 kbp,
    5-20% divergence), the rest i.i.d."""
    return gen.genome_repeats(seed, n, gc=0.41, repeat_frac=0.40, n_fam=500, min_len=300, max_len=6000,
                              div_lo=0.05, div_hi=0.20)


def c2_pairs(g: gen.Genome, n_pairs: int = 1_000_000, seed: int = 1002) -> gen.PairedReads:
    """2 x 100 bp pairs, fragment ~ N(300, 30), 1% substitutions, 0.1% indel events."""
    return gen.reads_pe(seed, g, n_pairs, 100, frag_mu=300.0, frag_sd=30.0, frag_min=100, ps=0.01,
                        indel_ratio=0.1)


def c3_pairs(g: gen.Genome, n_pairs: int, seed: int = 1003) -> gen.PairedReads:
    """Pairs of uneven length drawn from {36, 51, 76, 100, 150}; per read error
    e ~ U[0.5%, 3%], of which 0.9 e substitutions and 0.1 e indel events."""
    return gen.reads_pe(seed, g, n_pairs, list(C3_LENGTHS), frag_mu=300.0, frag_sd=30.0, frag_min=100,
                        ps=(0.9 * 0.005, 0.9 * 0.03), indel_ratio=1.0 / 9.0)


def c4_request(g: gen.Genome, n_pairs: int, seed: int) -> gen.PairedReads:
    """One serving request: lengths in [76, 150], 1% substitutions, 0.1% indels."""
    return gen.reads_pe(seed, g, n_pairs, list(range(76, 151)), frag_mu=300.0, frag_sd=30.0, frag_min=100,
                        ps=0.01, indel_ratio=0.1)


def c4_request_sizes(seed: int, n: int, lo: int = 1000, hi: int = 200_000) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n)).astype(np.int64)


def c5_reads(g: gen.Genome, n_reads: int = 2_000_000, seed: int = 1005) -> gen.Reads:
    """250 bp single-end reads, 3% substitutions, 0.3% indel events, 10% of
    them starting inside repeat copies."""
    return gen.reads_se(seed, g, n_reads, 250, ps=0.03, indel_ratio=0.1, rep_frac=0.10)
