"""CPU oracle -- TEST INFRASTRUCTURE, not the product.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  It is a plain, slow,
independent implementation of the alignment path (``oracle.c``) plus
brute-force checkers that pin it (``brute.c``).  It shares no code with the
GPU library: not its index builder, not its layout, not its search.

The method it follows is the backtracking FM-index search of BWA's short-read
aligner as used by BarraCUDA (Genetically Improved BarraCUDA, section 2);
``oracle.c``'s header states every definition and reading.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# BWFM_SANITIZE=1 selects the AddressSanitizer + UndefinedBehaviorSanitizer
# builds (lib*.san.so; the process must preload the sanitizer runtimes)
SANITIZE = os.environ.get("BWFM_SANITIZE") == "1"
SAN_FLAGS = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _so(name: str, sanitize: bool) -> str:
    return os.path.join(_HERE, f"lib{name}.san.so" if sanitize else f"lib{name}.so")


_LIBS = {
    "oracle": (os.path.join(_HERE, "oracle.c"), _so("oracle", SANITIZE)),
    "brute": (os.path.join(_HERE, "brute.c"), _so("brute", SANITIZE)),
}
_loaded: dict = {}

HIT_DTYPE = np.dtype([("k", "<u4"), ("l", "<u4"), ("len", "<u2"), ("score", "<u2"), ("strand", "u1"),
                      ("n_mm", "u1"), ("n_gapo", "u1"), ("n_gape", "u1")])
PAIR_DTYPE = np.dtype([("pos1", "<u4"), ("pos2", "<u4"), ("insert", "<i4"), ("len1", "<u2"), ("len2", "<u2"),
                       ("score1", "<u2"), ("score2", "<u2"), ("strand1", "u1"), ("strand2", "u1"),
                       ("flags", "u1"), ("pad", "u1")])
REC_DTYPE = np.dtype([("pos", "<u4"), ("len", "<u2"), ("score", "<u2"), ("strand", "u1"), ("n_mm", "u1"),
                      ("n_gapo", "u1"), ("n_gape", "u1")])
COUNT_DTYPE = np.dtype([("expand", "<u8"), ("touch_s", "<u8"), ("touch_d", "<u8"), ("max_stack", "<u8")])

ST_HIT, ST_OVERFLOW, ST_INVALID = 1, 2, 4
PF_PAIRED, PF_MAPPED1, PF_MAPPED2, PF_REP1, PF_REP2 = 1, 2, 4, 8, 16
MODE_ALL, MODE_BEST = 0, 1


def build(force: bool = True, sanitize: bool | None = None) -> None:
    """Compile the oracle and the brute-force checkers with gcc (sanitize:
    the sanitizer builds instead; default: as BWFM_SANITIZE selects)."""
    sanitize = SANITIZE if sanitize is None else sanitize
    for name, (src, _) in _LIBS.items():
        so = _so(name, sanitize)
        if force or not os.path.exists(so):
            tmp = so + ".tmp"
            extra = SAN_FLAGS if sanitize else []
            subprocess.check_call(["gcc", "-O2", *extra, "-fPIC", "-shared", "-pthread", "-o", tmp, src, "-lm"])
            os.replace(tmp, so)


def _lib(name: str):
    if name not in _loaded:
        src, so = _LIBS[name]
        if not os.path.exists(so):
            build(force=False)
        L = ctypes.CDLL(so)
        P, i64, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
        if name == "oracle":
            L.orc_index_build.argtypes = [P, i64]
            L.orc_index_build.restype = P
            L.orc_index_free.argtypes = [P]
            L.orc_index_n.argtypes = [P]
            L.orc_index_n.restype = i64
            L.orc_index_get.argtypes = [P, ctypes.c_int, P, P, P, P]
            L.orc_occ4.argtypes = [P, ctypes.c_int, u64, P]
            L.orc_exact.argtypes = [P, ctypes.c_int, P, ctypes.c_int, P, P, P]
            L.orc_exact.restype = ctypes.c_int
            L.orc_darray.argtypes = [P, ctypes.c_int, P, ctypes.c_int, P]
            L.orc_align.argtypes = [P, P, P, P, i64, P, ctypes.c_int, P, ctypes.POINTER(P), P, P, P, P]
            L.orc_align.restype = i64
            L.orc_free.argtypes = [P]
            L.orc_locate.argtypes = [P, P, i64, u32, P, ctypes.POINTER(P), P, u32]
            L.orc_locate.restype = i64
            L.orc_pair_reads.argtypes = [i64, P, P, P, P, P, P, P, P, i32, i32, i32, P]
            L.orc_rescue_mates.argtypes = [i64, P, i64, P, P, P, P, P, i32, i32, i32, i32, i32, i32, i32, P]
            L.orc_local_best.argtypes = [P, i32, P, i32, i32, i32, i32, i32, i32, P, P]
            L.orc_local_best.restype = i32
            L.orc_mapq.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P, P, i32, P, P, i32, i32, i32, i32, P]
            L.orc_max_diff_rule.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
            L.orc_max_diff_rule.restype = ctypes.c_int
            L.orc_estimate_insert.argtypes = [P, i64, P]
            L.orc_estimate_insert.restype = ctypes.c_int
        else:
            L.brute_sa.argtypes = [P, i64, P]
            L.brute_align.argtypes = [P, i64, P, ctypes.c_int, P, ctypes.POINTER(P)]
            L.brute_align.restype = i64
            L.brute_hamming.argtypes = [P, i64, P, ctypes.c_int, P, ctypes.POINTER(P)]
            L.brute_hamming.restype = i64
            L.brute_hamming_many.argtypes = [P, i64, P, P, i64, P, ctypes.c_int, P, ctypes.POINTER(P)]
            L.brute_hamming_many.restype = i64
            L.brute_exact_many.argtypes = [P, i64, P, P, i64, ctypes.c_int, P, ctypes.POINTER(P)]
            L.brute_exact_many.restype = i64
            L.brute_edit_many.argtypes = [P, i64, P, P, i64, P, ctypes.c_int, P, P, ctypes.POINTER(P)]
            L.brute_edit_many.restype = i64
            L.brute_free.argtypes = [P]
        _loaded[name] = L
    return _loaded[name]


def _p(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "array must be contiguous"
    return a.ctypes.data


class _Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("max_diff", "max_gapo", "max_gape", "seed_len", "seed_diff",
                                              "indel_end_skip", "s_mm", "s_gapo", "s_gape", "mode", "max_best")] + [
        ("max_hits", ctypes.c_uint32), ("use_d", ctypes.c_int32), ("bases_per_line", ctypes.c_int32),
        ("sa_sample", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _BruteParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("max_diff", "max_gapo", "max_gape", "seed_len", "seed_diff",
                                              "indel_end_skip", "s_mm", "s_gapo", "s_gape")]


@dataclass
class Params:
    """Search parameters.  Defaults are BWA's documented aln defaults
    (mismatch 3, gap open 11, gap extension 4, at most 1 gap open, no indel
    within 5 bases of either end, 30 equal-best hits before second-best hits
    are dropped); the paper itself states none of them."""
    max_diff: int = 4
    max_gapo: int = 1
    max_gape: int = -1
    seed_len: int = 0
    seed_diff: int = 2
    indel_end_skip: int = 5
    s_mm: int = 3
    s_gapo: int = 11
    s_gape: int = 4
    mode: int = MODE_BEST
    max_best: int = 30
    max_hits: int = 256
    use_d: int = 1
    bases_per_line: int = 448
    sa_sample: int = 32

    def _c(self) -> _Params:
        return _Params(*[getattr(self, f.name) for f in fields(self)], 0)

    def _brute(self) -> _BruteParams:
        return _BruteParams(self.max_diff, self.max_gapo, self.max_gape, self.seed_len, self.seed_diff,
                            self.indel_end_skip, self.s_mm, self.s_gapo, self.s_gape)


class Index:
    """FM-index of T and of reverse(T), built by prefix doubling."""

    def __init__(self, text: np.ndarray):
        self.text = np.ascontiguousarray(text, np.uint8)
        self.n = len(self.text)
        h = _lib("oracle").orc_index_build(_p(self.text), self.n)
        if not h:
            raise ValueError("oracle index build failed (bad base code or size)")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib("oracle").orc_index_free(h)
            self._h = None

    def get(self, which: int = 0):
        sa = np.empty(self.n + 1, np.uint32)
        bwt = np.empty(self.n + 1, np.uint8)
        C = np.empty(4, np.uint64)
        prim = ctypes.c_int64()
        _lib("oracle").orc_index_get(self._h, which, _p(sa), _p(bwt), _p(C), ctypes.byref(prim))
        return sa, bwt, C, prim.value

    def occ4(self, i: int, which: int = 0) -> np.ndarray:
        out = np.empty(4, np.uint64)
        _lib("oracle").orc_occ4(self._h, which, i, _p(out))
        return out

    def exact(self, p: np.ndarray, which: int = 0):
        p = np.ascontiguousarray(p, np.uint8)
        k, l, s = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_int()
        ok = _lib("oracle").orc_exact(self._h, which, _p(p), len(p), ctypes.byref(k), ctypes.byref(l),
                                      ctypes.byref(s))
        return bool(ok), k.value, l.value, s.value

    def darray(self, w: np.ndarray, which: int = 0) -> np.ndarray:
        """D-array of pattern w for a backward search on index ``which``."""
        w = np.ascontiguousarray(w, np.uint8)
        D = np.empty(len(w), np.uint8)
        _lib("oracle").orc_darray(self._h, which, _p(w), len(w), _p(D))
        return D


@dataclass
class AlnResult:
    hit_off: np.ndarray
    hits: np.ndarray
    c1: np.ndarray
    c2: np.ndarray
    status: np.ndarray
    counts: np.ndarray

    def read_hits(self, r: int) -> np.ndarray:
        return self.hits[self.hit_off[r]:self.hit_off[r + 1]]


def align(ix: Index, bases: np.ndarray, offsets: np.ndarray, params: Params, max_diff: np.ndarray | None = None,
          threads: int = 1) -> AlnResult:
    bases = np.ascontiguousarray(bases, np.uint8)
    offsets = np.ascontiguousarray(offsets, np.uint64)
    n = len(offsets) - 1
    md = None if max_diff is None else np.ascontiguousarray(max_diff, np.uint8)
    hit_off = np.zeros(n + 1, np.uint64)
    c1 = np.zeros(n, np.uint32)
    c2 = np.zeros(n, np.uint32)
    st = np.zeros(n, np.uint8)
    cnt = np.zeros(n, COUNT_DTYPE)
    out = ctypes.c_void_p()
    cp = params._c()
    L = _lib("oracle")
    tot = L.orc_align(ix._h, _p(bases), _p(offsets), _p(md), n, ctypes.byref(cp), threads, _p(hit_off),
                      ctypes.byref(out), _p(c1), _p(c2), _p(st), _p(cnt))
    if tot < 0:
        raise RuntimeError("oracle align failed")
    hits = np.frombuffer((ctypes.c_char * (16 * tot)).from_address(out.value), HIT_DTYPE).copy() if tot else \
        np.zeros(0, HIT_DTYPE)
    L.orc_free(out)
    return AlnResult(hit_off, hits, c1, c2, st, cnt)


def locate(ix: Index, hits: np.ndarray, max_occ: int, sample: int = 32, want_steps: bool = False):
    hits = np.ascontiguousarray(hits, HIT_DTYPE)
    po = np.zeros(len(hits) + 1, np.uint64)
    steps = np.zeros(len(hits), np.uint64) if want_steps else None
    out = ctypes.c_void_p()
    L = _lib("oracle")
    tot = L.orc_locate(ix._h, _p(hits), len(hits), max_occ, _p(po), ctypes.byref(out), _p(steps), sample)
    if tot < 0:
        raise RuntimeError("oracle locate failed")
    pos = np.frombuffer((ctypes.c_char * (4 * tot)).from_address(out.value), np.uint32).copy() if tot else \
        np.zeros(0, np.uint32)
    L.orc_free(out)
    return (po, pos, steps) if want_steps else (po, pos)


def pair(r1: AlnResult, po1, pos1, r2: AlnResult | None, po2, pos2, lo: int, hi: int, mu: int) -> np.ndarray:
    n = len(r1.hit_off) - 1
    out = np.zeros(n, PAIR_DTYPE)
    _lib("oracle").orc_pair_reads(n, _p(r1.hit_off), _p(r1.hits), _p(po1), _p(pos1),
                                  _p(r2.hit_off) if r2 else None, _p(r2.hits) if r2 else None,
                                  _p(po2) if r2 else None, _p(pos2) if r2 else None, lo, hi, mu, _p(out))
    return out


RESCUE_DTYPE = np.dtype([("pos", "<u4"), ("len", "<u2"), ("score", "<i2"), ("insert", "<i4"), ("end", "u1"),
                         ("strand", "u1"), ("pad", "u1", 2)])
# local-alignment scores of the rescue (a reading: BWA-MEM's documented defaults)
RESCUE_SCORES = dict(match=1, mismatch=4, gap_open=6, gap_extend=1)


def rescue(ref: np.ndarray, end1, end2, pairs: np.ndarray, lo: int, hi: int, min_score: int = 20,
           match: int = 1, mismatch: int = 4, gap_open: int = 6, gap_extend: int = 1) -> np.ndarray:
    """Mate rescue for the pairs without a proper pair (see oracle.c):
    end1/end2 are (bases, offsets) of the two ends, pairs the pair records."""
    t = np.ascontiguousarray(ref, np.uint8)
    b1, o1 = np.ascontiguousarray(end1[0], np.uint8), np.ascontiguousarray(end1[1], np.uint64)
    b2, o2 = np.ascontiguousarray(end2[0], np.uint8), np.ascontiguousarray(end2[1], np.uint64)
    pr = np.ascontiguousarray(pairs)
    n = len(pr)
    out = np.zeros(n, RESCUE_DTYPE)
    _lib("oracle").orc_rescue_mates(n, _p(t), len(t), _p(b1), _p(o1), _p(b2), _p(o2), _p(pr), lo, hi, match, mismatch,
                                    gap_open, gap_extend, min_score, _p(out))
    return out


def local_best(q, r, e_min: int = 0, match: int = 1, mismatch: int = 4, gap_open: int = 6, gap_extend: int = 1):
    """(score, end column, start column) of the rescue's local alignment of q
    in r, ending at column >= e_min (score 0: none)."""
    qa, ra = np.ascontiguousarray(q, np.uint8), np.ascontiguousarray(r, np.uint8)
    je, js = ctypes.c_int(), ctypes.c_int()
    sc = _lib("oracle").orc_local_best(_p(qa), len(qa), _p(ra), len(ra), e_min, match, mismatch, gap_open, gap_extend,
                                       ctypes.byref(je), ctypes.byref(js))
    return sc, je.value, js.value


# mapping-quality constants (a reading): phred weight of a tier-2 placement,
# single-end cap, cap when the best hits spend the whole budget, proper-pair cap
MAPQ_DEFAULTS = dict(q_tier=22, q_unique=37, q_budget=25, q_pair=60)


def mapq(r1: AlnResult, r2: AlnResult | None, pairs: np.ndarray, rescue: np.ndarray | None = None,
         budgets1=None, budgets2=None, max_diff: int = 4, q_tier: int = 22, q_unique: int = 37, q_budget: int = 25,
         q_pair: int = 60) -> np.ndarray:
    """uint8 [n_pairs, 2]: MAPQ of end 1 and end 2 of every pair (see oracle.c)."""
    n = len(r1.hit_off) - 1
    out = np.zeros((n, 2), np.uint8)
    pr = np.ascontiguousarray(pairs)
    b1 = None if budgets1 is None else np.ascontiguousarray(budgets1, np.uint8)
    b2 = None if budgets2 is None else np.ascontiguousarray(budgets2, np.uint8)
    rs = None if rescue is None else np.ascontiguousarray(rescue)
    L = _lib("oracle")
    L.orc_mapq(n, _p(r1.hit_off), _p(r1.hits), _p(r1.c1), _p(r1.c2), _p(r1.status), _p(b1) if b1 is not None else None,
               _p(r2.hit_off) if r2 else None, _p(r2.hits) if r2 else None, _p(r2.c1) if r2 else None,
               _p(r2.c2) if r2 else None, _p(r2.status) if r2 else None, _p(b2) if b2 is not None else None,
               max_diff, _p(pr), _p(rs) if rs is not None else None, q_tier, q_unique, q_budget, q_pair, _p(out))
    return out


def max_diff_rule(L: int, err: float = 0.02, thres: float = 0.04) -> int:
    return _lib("oracle").orc_max_diff_rule(L, err, thres)


def estimate_insert(inserts: np.ndarray):
    a = np.ascontiguousarray(inserts, np.int32)
    out = np.zeros(3, np.int32)
    if _lib("oracle").orc_estimate_insert(_p(a), len(a), _p(out)):
        raise RuntimeError("estimate_insert failed")
    return int(out[0]), int(out[1]), int(out[2])


# ---------------------------------------------------------------- brute force

def brute_sa(text: np.ndarray) -> np.ndarray:
    t = np.ascontiguousarray(text, np.uint8)
    sa = np.empty(len(t) + 1, np.uint32)
    _lib("brute").brute_sa(_p(t), len(t), _p(sa))
    return sa


def _brute_call(fn, text, read, params: Params) -> np.ndarray:
    t = np.ascontiguousarray(text, np.uint8)
    w = np.ascontiguousarray(read, np.uint8)
    bp = params._brute()
    out = ctypes.c_void_p()
    L = _lib("brute")
    n = getattr(L, fn)(_p(t), len(t), _p(w), len(w), ctypes.byref(bp), ctypes.byref(out))
    if n < 0:
        raise RuntimeError(f"{fn} failed")
    recs = np.frombuffer((ctypes.c_char * (12 * n)).from_address(out.value), REC_DTYPE).copy() if n else \
        np.zeros(0, REC_DTYPE)
    L.brute_free(out)
    return recs


def brute_align(text, read, params: Params) -> np.ndarray:
    """Every (strand, pos, len) reached by a valid transcript, with the
    smallest (score, diffs, n_gapo, n_mm)."""
    return _brute_call("brute_align", text, read, params)


def brute_hamming(text, read, params: Params) -> np.ndarray:
    return _brute_call("brute_hamming", text, read, params)


def _recs(out, tot):
    r = np.frombuffer((ctypes.c_char * (REC_DTYPE.itemsize * tot)).from_address(out.value), REC_DTYPE).copy() \
        if tot else np.zeros(0, REC_DTYPE)
    _lib("brute").brute_free(out)
    return r


def brute_hamming_many(text, bases, offsets, params: Params, threads: int = 8):
    """brute_hamming for every read of a batch: (rec_off, records), the
    records of read r at records[rec_off[r]:rec_off[r + 1]]."""
    t = np.ascontiguousarray(text, np.uint8)
    b = np.ascontiguousarray(bases, np.uint8)
    o = np.ascontiguousarray(offsets, np.uint64)
    n = len(o) - 1
    off = np.zeros(n + 1, np.uint64)
    out = ctypes.c_void_p()
    bp = params._brute()
    tot = _lib("brute").brute_hamming_many(_p(t), len(t), _p(b), _p(o), n, ctypes.byref(bp), threads, _p(off),
                                           ctypes.byref(out))
    if tot < 0:
        raise RuntimeError("brute_hamming_many failed")
    return off, _recs(out, tot)


def brute_edit_many(text, bases, offsets, params: Params, threads: int = 8):
    """The gapped ALL set of every read of a batch by an edit-distance filter
    and transcript enumeration: (rec_off, records, candidate ends per read)."""
    t = np.ascontiguousarray(text, np.uint8)
    b = np.ascontiguousarray(bases, np.uint8)
    o = np.ascontiguousarray(offsets, np.uint64)
    n = len(o) - 1
    off = np.zeros(n + 1, np.uint64)
    ends = np.zeros(n, np.int64)
    out = ctypes.c_void_p()
    bp = params._brute()
    tot = _lib("brute").brute_edit_many(_p(t), len(t), _p(b), _p(o), n, ctypes.byref(bp), threads, _p(off),
                                        _p(ends), ctypes.byref(out))
    if tot < 0:
        raise RuntimeError("brute_edit_many failed")
    return off, _recs(out, tot), ends


def brute_exact_many(text, pats, offsets, threads: int = 8):
    """Every occurrence of every pattern (codes 0..3, at least 16 bases):
    (occ_off, positions), pattern k's ascending positions at
    positions[occ_off[k]:occ_off[k + 1]]."""
    t = np.ascontiguousarray(text, np.uint8)
    b = np.ascontiguousarray(pats, np.uint8)
    o = np.ascontiguousarray(offsets, np.uint64)
    n = len(o) - 1
    off = np.zeros(n + 1, np.uint64)
    out = ctypes.c_void_p()
    tot = _lib("brute").brute_exact_many(_p(t), len(t), _p(b), _p(o), n, threads, _p(off), ctypes.byref(out))
    if tot < 0:
        raise RuntimeError("brute_exact_many failed")
    pos = np.frombuffer((ctypes.c_char * (4 * tot)).from_address(out.value), np.uint32).copy() if tot else \
        np.zeros(0, np.uint32)
    _lib("brute").brute_free(out)
    return off, pos
