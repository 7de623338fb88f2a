"""Seeded synthetic genomes and reads (numpy front end of ``gen.c``).

This module draws inputs only; it holds none of the alignment method's
arithmetic.  Both the CPU oracle's tests and the GPU library's tests and
benchmark take their inputs from here, so the two sides always see the same
bytes for the same (recipe, seed).

Base codes are A=0, C=1, G=2, T=3.  Reads come as a ragged batch in CSR form:
``bases`` (uint8) and ``offsets`` (uint64, n_reads + 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
# BWFM_SANITIZE=1 selects the AddressSanitizer + UndefinedBehaviorSanitizer
# build (libgen.san.so; the process must preload the sanitizer runtimes)
SANITIZE = os.environ.get("BWFM_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "libgen.san.so" if SANITIZE else "libgen.so")
_lib = None

MAX_EDITS = 64


def build(force: bool = True, sanitize: bool | None = None) -> str:
    """Compile gen.c into libgen.so next to it (gcc, OpenMP); sanitize: the
    sanitizer build libgen.san.so instead (default: as BWFM_SANITIZE selects)."""
    sanitize = SANITIZE if sanitize is None else sanitize
    so = os.path.join(_HERE, "libgen.san.so" if sanitize else "libgen.so")
    if force or not os.path.exists(so):
        tmp = so + ".tmp"
        extra = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"] \
            if sanitize else []
        subprocess.check_call(["gcc", "-O2", *extra, "-fPIC", "-shared", "-fopenmp", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, so)
    return so


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        u64, i64, i32, dbl = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.gen_ref_iid.argtypes = [u64, u64, dbl, P]
        L.gen_ref_iid.restype = None
        L.gen_ref_repeats.argtypes = [u64, u64, dbl, dbl, i32, i32, i32, dbl, dbl, P, P, i64]
        L.gen_ref_repeats.restype = i64
        L.gen_reads_se.argtypes = [u64, P, u64, u64, P, P, dbl, dbl, dbl, P, i64, dbl, P, P, P, P, P, P, P]
        L.gen_reads_se.restype = ctypes.c_int
        L.gen_pair_lengths.argtypes = [u64, u64, P, i32, P]
        L.gen_pair_lengths.restype = None
        L.gen_reads_pe.argtypes = [u64, P, u64, u64, P, P, dbl, dbl, i32, dbl, dbl, dbl, P, P, P, P, P, P, P, P, P]
        L.gen_reads_pe.restype = ctypes.c_int
        L.gen_max_edits.restype = ctypes.c_int
        assert L.gen_max_edits() == MAX_EDITS
        _lib = L
    return _lib


def _p(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


@dataclass
class Genome:
    seq: np.ndarray  # uint8 codes 0..3
    spans: np.ndarray = field(default_factory=lambda: np.zeros((0, 4), np.uint64))  # repeat copies


@dataclass
class Truth:
    pos: np.ndarray      # uint32, leftmost forward coordinate of the consumed template
    ref_len: np.ndarray  # uint32, template bases consumed
    strand: np.ndarray   # uint8, 0 = +, 1 = - (read is the reverse complement of the template)
    e_type: np.ndarray   # uint8 [n, MAX_EDITS]: 0 substitution, 1 insertion, 2 deletion
    e_idx: np.ndarray    # uint16 [n, MAX_EDITS]: read index (boundary for deletions)
    n_edits: np.ndarray  # uint8, 255 = more than MAX_EDITS edits


@dataclass
class Reads:
    bases: np.ndarray    # uint8 codes
    offsets: np.ndarray  # uint64, n + 1
    truth: Truth | None = None

    @property
    def n(self) -> int:
        return len(self.offsets) - 1

    def read(self, i: int) -> np.ndarray:
        return self.bases[self.offsets[i]:self.offsets[i + 1]]

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int32)


def genome_iid(seed: int, n: int, gc: float = 0.5) -> Genome:
    out = np.empty(n, np.uint8)
    lib().gen_ref_iid(seed, n, gc, _p(out))
    return Genome(out)


def genome_repeats(seed: int, n: int, gc: float = 0.41, repeat_frac: float = 0.4, n_fam: int = 500,
                   min_len: int = 300, max_len: int = 6000, div_lo: float = 0.05,
                   div_hi: float = 0.20) -> Genome:
    out = np.empty(n, np.uint8)
    max_copies = max(16, int(repeat_frac * n / max(1, min_len)) * 2 + 16)
    spans = np.zeros((max_copies, 4), np.uint64)
    c = lib().gen_ref_repeats(seed, n, gc, repeat_frac, n_fam, min_len, max_len, div_lo, div_hi,
                              _p(out), _p(spans), max_copies)
    if c < 0:
        raise RuntimeError(f"gen_ref_repeats failed ({c})")
    return Genome(out, spans[:c].copy())


def _truth(n: int) -> Truth:
    return Truth(np.zeros(n, np.uint32), np.zeros(n, np.uint32), np.zeros(n, np.uint8),
                 np.zeros((n, MAX_EDITS), np.uint8), np.zeros((n, MAX_EDITS), np.uint16),
                 np.zeros(n, np.uint8))


def reads_se(seed: int, g: Genome, n_reads: int, length, ps: float | tuple = 0.0,
             indel_ratio: float = 0.0, rep_frac: float = 0.0) -> Reads:
    """Single-end reads; ``length`` is an int or a per-read int array; ``ps``
    a substitution rate or a (lo, hi) range drawn per read."""
    lens = np.full(n_reads, length, np.int32) if np.isscalar(length) else np.ascontiguousarray(length, np.int32)
    offs = np.zeros(n_reads + 1, np.uint64)
    np.cumsum(lens, out=offs[1:])
    bases = np.empty(int(offs[-1]), np.uint8)
    lo, hi = (ps, ps) if np.isscalar(ps) else ps
    t = _truth(n_reads)
    spans = g.spans if rep_frac > 0 else np.zeros((0, 4), np.uint64)
    spans = np.ascontiguousarray(spans, np.uint64)
    rc = lib().gen_reads_se(seed, _p(g.seq), len(g.seq), n_reads, _p(lens), _p(offs), lo, hi, indel_ratio,
                            _p(spans) if len(spans) else None, len(spans), rep_frac, _p(bases),
                            _p(t.pos), _p(t.ref_len), _p(t.strand), _p(t.e_type), _p(t.e_idx), _p(t.n_edits))
    if rc != 0:
        raise RuntimeError("genome too short for these reads")
    return Reads(bases, offs, t)


@dataclass
class PairedReads:
    end1: Reads
    end2: Reads
    frag: np.ndarray  # uint32 [n_pairs, 3]: start, length, strand


def reads_pe(seed: int, g: Genome, n_pairs: int, length, frag_mu: float = 300.0, frag_sd: float = 30.0,
             frag_min: int = 100, ps: float | tuple = 0.01, indel_ratio: float = 0.1) -> PairedReads:
    """Paired-end reads in forward-reverse orientation; ``length`` is an int
    or a list of choices drawn uniformly per pair."""
    L = lib()
    if np.isscalar(length):
        lens = np.full(n_pairs, length, np.int32)
    else:
        ch = np.ascontiguousarray(length, np.int32)
        lens = np.empty(n_pairs, np.int32)
        L.gen_pair_lengths(seed, n_pairs, _p(ch), len(ch), _p(lens))
    offs = np.zeros(n_pairs + 1, np.uint64)
    np.cumsum(lens, out=offs[1:])
    b1 = np.empty(int(offs[-1]), np.uint8)
    b2 = np.empty(int(offs[-1]), np.uint8)
    frag = np.zeros((n_pairs, 3), np.uint32)
    lo, hi = (ps, ps) if np.isscalar(ps) else ps
    t = _truth(2 * n_pairs)
    rc = L.gen_reads_pe(seed, _p(g.seq), len(g.seq), n_pairs, _p(lens), _p(offs), frag_mu, frag_sd, frag_min,
                        lo, hi, indel_ratio, _p(b1), _p(b2), _p(frag), _p(t.pos), _p(t.ref_len), _p(t.strand),
                        _p(t.e_type), _p(t.e_idx), _p(t.n_edits))
    if rc != 0:
        raise RuntimeError("genome too short for these pairs")

    def pick(sl):
        return Truth(t.pos[sl].copy(), t.ref_len[sl].copy(), t.strand[sl].copy(), t.e_type[sl].copy(),
                     t.e_idx[sl].copy(), t.n_edits[sl].copy())

    return PairedReads(Reads(b1, offs, pick(slice(0, None, 2))), Reads(b2, offs.copy(), pick(slice(1, None, 2))),
                       frag)


def revcomp(x: np.ndarray) -> np.ndarray:
    return (3 - x[::-1]).astype(np.uint8)
