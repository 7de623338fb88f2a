"""bwfm: FM-index short-read alignment on AMD Instinct MI355X.

Thin ctypes binding over ``libbwfm.so`` (``include/bwfm.h``).  It marshals
arguments only: every step of the alignment path runs in the library's HIP
kernels.  torch provides device memory and streams.  There is no CPU fallback:
if the library is missing, every call raises.

Names follow the C ABI: ``build_index``, ``align_batch``, ``locate``,
``pair_reads``, ``estimate_insert``, ``max_diff_rule``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbwfm.so")
_lib_handle = None

# result records (same bytes as bwfm_hit / bwfm_pair)
HIT_DTYPE = np.dtype([("k", "<u4"), ("l", "<u4"), ("len", "<u2"), ("score", "<u2"), ("strand", "u1"),
                      ("n_mm", "u1"), ("n_gapo", "u1"), ("n_gape", "u1")])
PAIR_DTYPE = np.dtype([("pos1", "<u4"), ("pos2", "<u4"), ("insert", "<i4"), ("len1", "<u2"), ("len2", "<u2"),
                       ("score1", "<u2"), ("score2", "<u2"), ("strand1", "u1"), ("strand2", "u1"),
                       ("flags", "u1"), ("pad", "u1")])
RESCUE_DTYPE = np.dtype([("pos", "<u4"), ("len", "<u2"), ("score", "<i2"), ("insert", "<i4"), ("end", "u1"),
                         ("strand", "u1"), ("pad", "u1", 2)])

ST_HIT, ST_OVERFLOW, ST_INVALID, ST_RESEARCH, ST_SHARED, ST_SPLIT = 1, 2, 4, 8, 16, 32
PF_PAIRED, PF_MAPPED1, PF_MAPPED2, PF_REP1, PF_REP2 = 1, 2, 4, 8, 16
MODE_ALL, MODE_BEST = 0, 1
FORM_BATCHED, FORM_PLAIN = 0, 1
E_INVAL, E_CAPACITY = -1, -5
E_IO = -8
PIPE_E_HITS, PIPE_E_POSITIONS = 1, 2
NOALLOC_SCRATCH_BYTES = 64 << 20  # BWFM_NOALLOC_SCRATCH_BYTES: the fixed scratch of bwfm_pair_reads_noalloc
RANK_PLANES, RANK_SUBCOUNTS, RANK_SUB128 = 0, 1, 2  # rank-line formats (bwfm_index_params.rank_format)


class BwfmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bwfm error {code}: {msg}")
        self.code = code


class _IndexParams(ctypes.Structure):
    _fields_ = [("line_bytes", ctypes.c_uint32), ("bases_per_line", ctypes.c_uint32),
                ("sa_sample", ctypes.c_uint32), ("n_threads", ctypes.c_uint32), ("rank_format", ctypes.c_uint32)]


class _IndexInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("primary", ctypes.c_uint64 * 2), ("C", (ctypes.c_uint64 * 4) * 2),
                ("lines", ctypes.c_uint64), ("sa_samples", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64),
                ("line_bytes", ctypes.c_uint32), ("bases_per_line", ctypes.c_uint32),
                ("sa_sample", ctypes.c_uint32), ("uploaded", ctypes.c_uint32), ("rank_format", ctypes.c_uint32),
                ("kmer_levels", ctypes.c_uint32), ("kmer_bytes", ctypes.c_uint64), ("ws_bytes", ctypes.c_uint64),
                ("ws_streams", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class _Reads(ctypes.Structure):
    _fields_ = [("bases", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("max_diff", ctypes.c_void_p),
                ("n_reads", ctypes.c_uint32), ("max_len", ctypes.c_uint32), ("lengths", ctypes.c_void_p)]


class _AlnParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("max_diff", "max_gapo", "max_gape", "seed_len", "seed_diff",
                                              "indel_end_skip", "s_mm", "s_gapo", "s_gape", "mode", "max_best")] + [
        ("max_hits", ctypes.c_uint32), ("form", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32),
        ("split_budget", ctypes.c_int32)]


class _AlnResult(ctypes.Structure):
    _fields_ = [("hit_offsets", ctypes.c_void_p), ("hits", ctypes.c_void_p), ("hit_capacity", ctypes.c_uint64),
                ("c1", ctypes.c_void_p), ("c2", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class _ServerParams(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_uint64), ("step_pairs", ctypes.c_uint32), ("max_len", ctypes.c_uint32),
                ("paired", ctypes.c_int32), ("budget_rule", ctypes.c_int32), ("rescue_mapq", ctypes.c_int32)]


class _Times(ctypes.Structure):
    _fields_ = [("queued_ms", ctypes.c_double), ("service_ms", ctypes.c_double), ("latency_ms", ctypes.c_double)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_uint64), ("pairs", ctypes.c_uint64), ("requests_done", ctypes.c_uint64),
                ("busy_ms", ctypes.c_double)]


class _PairParams(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32), ("hi", ctypes.c_int32), ("mu", ctypes.c_int32), ("max_occ", ctypes.c_uint32)]


class _RescueParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("match", "mismatch", "gap_open", "gap_extend", "min_score")]


class _MapqParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("q_tier", "q_unique", "q_budget", "q_pair")]


class _PipeParams(ctypes.Structure):
    _fields_ = [("max_pairs", ctypes.c_uint32), ("max_len", ctypes.c_uint32), ("max_bases", ctypes.c_uint64),
                ("hit_capacity", ctypes.c_uint64), ("pos_capacity", ctypes.c_uint64), ("paired", ctypes.c_int32)]


class _PipeStatus(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_uint32), ("error", ctypes.c_uint32), ("n_hits", ctypes.c_uint64),
                ("n_positions", ctypes.c_uint64), ("kernel_ms", ctypes.c_double)]


# every function include/bwfm.h declares, plus the counted variant
SYMBOLS = ("bwfm_build_index", "bwfm_index_upload", "bwfm_index_free", "bwfm_index_get_info", "bwfm_index_get_bwt",
           "bwfm_index_get_sa_samples", "bwfm_index_occ", "bwfm_align_batch", "bwfm_locate", "bwfm_pair_reads", "bwfm_pair_reads_noalloc",
           "bwfm_estimate_insert", "bwfm_max_diff_rule", "bwfm_last_error", "bwfm_align_batch_counted",
           "bwfm_timing_enable", "bwfm_timing_reset", "bwfm_timing_get", "bwfm_probe_gather",
           "bwfm_server_create", "bwfm_server_submit", "bwfm_server_wait", "bwfm_server_get_stats",
           "bwfm_server_destroy", "bwfm_index_save", "bwfm_index_load", "bwfm_pipeline_create",
           "bwfm_pipeline_set_reads", "bwfm_pipeline_run", "bwfm_pipeline_finish", "bwfm_pipeline_outputs",
           "bwfm_pipeline_destroy", "bwfm_pipeline_bind_reads", "bwfm_pipeline_set_count",
           "bwfm_build_index_device", "bwfm_index_get_ref", "bwfm_rescue_mates", "bwfm_mapq",
           "bwfm_index_kmer_table", "bwfm_index_kmer_get")


def lib():
    """Load libbwfm.so; raises if it has not been built."""
    global _lib_handle
    if _lib_handle is None:
        # torch ships its own HIP runtime under the same soname; import it
        # first so that the library binds to that one runtime rather than
        # loading a second copy from /opt/rocm
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1505_07855_amd.build "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        P, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
        c_int = ctypes.c_int
        sig = {
            "bwfm_build_index": ([P, u64, P, ctypes.POINTER(P)], c_int),
            "bwfm_index_upload": ([P, P], c_int),
            "bwfm_index_kmer_table": ([P, c_int, P], c_int),
            "bwfm_index_kmer_get": ([P, c_int, c_int, u64, u64, P], c_int),
            "bwfm_build_index_device": ([P, u64, P, P, ctypes.POINTER(P)], c_int),
            "bwfm_index_save": ([P, ctypes.c_char_p], c_int),
            "bwfm_index_load": ([ctypes.c_char_p, ctypes.POINTER(P)], c_int),
            "bwfm_index_free": ([P], None),
            "bwfm_index_get_info": ([P, P], c_int),
            "bwfm_index_get_bwt": ([P, c_int, P], c_int),
            "bwfm_index_get_sa_samples": ([P, c_int, P], c_int),
            "bwfm_index_occ": ([P, c_int, u64, P], c_int),
            "bwfm_index_get_ref": ([P, u64, u64, P], c_int),
            "bwfm_rescue_mates": ([P, P, P, u32, P, P, P, P, P], c_int),
            "bwfm_mapq": ([u32, P, P, P, P, u32, P, P, P, P, P], c_int),
            "bwfm_align_batch": ([P, P, P, P, P], c_int),
            "bwfm_align_batch_counted": ([P, P, P, P, P, P, P], c_int),
            "bwfm_locate": ([P, u32, P, u32, P, P, u64, P], c_int),
            "bwfm_pair_reads": ([P, u32, P, P, P, P, P], c_int),
            "bwfm_pair_reads_noalloc": ([P, u32, P, P, P, P, P], c_int),
            "bwfm_estimate_insert": ([P, u64, P], c_int),
            "bwfm_max_diff_rule": ([u32, ctypes.c_double, ctypes.c_double], c_int),
            "bwfm_last_error": ([], ctypes.c_char_p),
            "bwfm_timing_enable": ([c_int], c_int),
            "bwfm_timing_reset": ([], c_int),
            "bwfm_timing_get": ([ctypes.c_char_p, P, P], c_int),
            "bwfm_probe_gather": ([P, u64, u32, u32, u32, P, P, P], c_int),
            "bwfm_server_create": ([P, P, P, P, ctypes.POINTER(P)], c_int),
            "bwfm_server_submit": ([P, P, P, P, P, u32, P], c_int),
            "bwfm_server_wait": ([P, u64, P, P, P, P], c_int),
            "bwfm_server_get_stats": ([P, P], c_int),
            "bwfm_server_destroy": ([P], None),
            "bwfm_pipeline_create": ([P, P, P, P, ctypes.POINTER(P)], c_int),
            "bwfm_pipeline_set_reads": ([P, P, u32, P], c_int),
            "bwfm_pipeline_run": ([P, c_int, P], c_int),
            "bwfm_pipeline_finish": ([P, P, P], c_int),
            "bwfm_pipeline_outputs": ([P, c_int, P, P, P, P], c_int),
            "bwfm_pipeline_destroy": ([P], None),
            "bwfm_pipeline_bind_reads": ([P, P], c_int),
            "bwfm_pipeline_set_count": ([P, u32], c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        del i32
        _lib_handle = L
    return _lib_handle


def _check(rc: int):
    if rc != 0:
        raise BwfmError(rc, lib().bwfm_last_error().decode())


def _np_ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t) -> int:
    assert t.is_cuda and t.is_contiguous(), "expected a contiguous device tensor"
    return t.data_ptr() if t.numel() else 0


@dataclass
class Params:
    """Search parameters (bwfm_aln_params).  Defaults are BWA's documented aln
    defaults; the paper states none."""
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
    form: int = FORM_BATCHED
    waves_per_simd: int = 0  # batched form residency (tuning only; 0 = the most that fit)
    split_budget: int = 0    # batched form: expansions between splits of a read's search into
                             # device-wide tasks (tuning only; 0 = the library's default, -1 = off)

    def _c(self) -> _AlnParams:
        return _AlnParams(*[getattr(self, f.name) for f in fields(self)])


class Index:
    """Packed FM-index of a reference and of its reverse (bwfm_build_index)."""

    def __init__(self, ref: np.ndarray, line_bytes: int = 128, bases_per_line: int = 0, sa_sample: int = 32,
                 threads: int = 0, rank_format: int = RANK_PLANES):
        ref = np.ascontiguousarray(ref, np.uint8)
        h = ctypes.c_void_p()
        p = _IndexParams(line_bytes, bases_per_line, sa_sample, threads, rank_format)
        _check(lib().bwfm_build_index(_np_ptr(ref), len(ref), ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self.n = len(ref)

    @classmethod
    def build_device(cls, ref: np.ndarray, line_bytes: int = 128, bases_per_line: int = 0, sa_sample: int = 32,
                     stream=None, rank_format: int = RANK_PLANES, kmer_levels: int = 0) -> "Index":
        """The same index built on the current GPU (bwfm_build_index_device);
        it comes back uploaded, with a short-string table of kmer_levels
        levels (as in upload)."""
        ref = np.ascontiguousarray(ref, np.uint8)
        h = ctypes.c_void_p()
        p = _IndexParams(line_bytes, bases_per_line, sa_sample, 0, rank_format)
        _check(lib().bwfm_build_index_device(_np_ptr(ref), len(ref), ctypes.byref(p), _stream_ptr(stream),
                                             ctypes.byref(h)))
        self = cls.__new__(cls)
        self._h = h
        self.n = len(ref)
        if kmer_levels:
            self.kmer_table(kmer_levels, stream)
        return self

    @classmethod
    def load(cls, path: str) -> "Index":
        """An index written by save() (bwfm_index_load); host-only until upload()."""
        h = ctypes.c_void_p()
        _check(lib().bwfm_index_load(os.fsencode(path), ctypes.byref(h)))
        self = cls.__new__(cls)
        self._h = h
        self.n = self.info()["n"]
        return self

    def save(self, path: str) -> None:
        """Write the index to a file (bwfm_index_save)."""
        _check(lib().bwfm_index_save(self._h, os.fsencode(path)))

    def close(self):
        if getattr(self, "_h", None):
            lib().bwfm_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def upload(self, stream=None, kmer_levels: int = 0) -> "Index":
        """Copy the index to the current GPU; with kmer_levels != 0 also
        build its short-string interval table (bwfm_index_kmer_table: -1
        picks the levels)."""
        _check(lib().bwfm_index_upload(self._h, _stream_ptr(stream)))
        if kmer_levels:
            self.kmer_table(kmer_levels, stream)
        return self

    def kmer_table(self, levels: int = -1, stream=None) -> "Index":
        """(Re)build the device short-string interval table with `levels`
        levels (0 releases it)."""
        _check(lib().bwfm_index_kmer_table(self._h, levels, _stream_ptr(stream)))
        return self

    def kmer_entries(self, which: int, level: int, first: int = 0, count: int | None = None) -> np.ndarray:
        """Entries of one table level as an (count, 2) array of (k, l)."""
        if count is None:
            count = 4 ** level - first
        out = np.empty((count, 2), np.uint32)
        _check(lib().bwfm_index_kmer_get(self._h, which, level, first, count, _np_ptr(out)))
        return out

    def info(self) -> dict:
        i = _IndexInfo()
        _check(lib().bwfm_index_get_info(self._h, ctypes.byref(i)))
        return dict(n=i.n, primary=list(i.primary), C=[list(c) for c in i.C], lines=i.lines, sa_samples=i.sa_samples,
                    device_bytes=i.device_bytes, line_bytes=i.line_bytes, bases_per_line=i.bases_per_line,
                    sa_sample=i.sa_sample, uploaded=bool(i.uploaded), rank_format=i.rank_format,
                    kmer_levels=i.kmer_levels, kmer_bytes=i.kmer_bytes, ws_bytes=i.ws_bytes, ws_streams=i.ws_streams)

    def bwt(self, which: int = 0) -> np.ndarray:
        out = np.empty(self.n + 1, np.uint8)
        _check(lib().bwfm_index_get_bwt(self._h, which, _np_ptr(out)))
        return out

    def sa_samples(self, which: int = 0) -> np.ndarray:
        out = np.empty(self.info()["sa_samples"], np.uint32)
        _check(lib().bwfm_index_get_sa_samples(self._h, which, _np_ptr(out)))
        return out

    def occ(self, i: int, which: int = 0) -> np.ndarray:
        out = np.empty(4, np.uint64)
        _check(lib().bwfm_index_occ(self._h, which, i, _np_ptr(out)))
        return out

    def ref(self, start: int = 0, length: int | None = None) -> np.ndarray:
        """T[start, start + length) decoded from the index's packed copy."""
        length = self.n - start if length is None else length
        out = np.empty(max(length, 1), np.uint8)
        _check(lib().bwfm_index_get_ref(self._h, start, length, _np_ptr(out)))
        return out[:length]


def build_index(ref: np.ndarray, **kw) -> Index:
    return Index(ref, **kw)


@dataclass
class AlignResult:
    """Device tensors of one align_batch call."""
    hit_offsets: object  # int64 [n + 1]
    hits: object         # int32 [capacity, 4] (bwfm_hit records)
    c1: object           # int32 [n] (uint32 bits)
    c2: object
    status: object       # uint8 [n]
    n_reads: int
    expand: object = None
    work: object = None

    def _c(self) -> _AlnResult:
        return _AlnResult(_dptr(self.hit_offsets), _dptr(self.hits), self.hits.shape[0], _dptr(self.c1),
                          _dptr(self.c2), _dptr(self.status))

    @property
    def n_hits(self) -> int:
        return int(self.hit_offsets[self.n_reads].item()) - int(self.hit_offsets[0].item())

    def window(self, start: int, stop: int) -> "AlignResult":
        """Reads [start, stop) of this result, sharing its buffers."""
        return AlignResult(self.hit_offsets[start:stop + 1], self.hits, self.c1[start:stop], self.c2[start:stop],
                           self.status[start:stop], stop - start,
                           self.expand[start:stop] if self.expand is not None else None)

    def to_numpy(self):
        """(hit_offsets uint64 rebased to 0, hits HIT_DTYPE, c1 uint32, c2 uint32, status uint8)."""
        ho = self.hit_offsets.cpu().numpy().view(np.uint64)
        h0, h1 = int(ho[0]), int(ho[-1])
        ho = ho - np.uint64(h0)
        hits = self.hits[h0:h1].contiguous().cpu().numpy().view(HIT_DTYPE).reshape(-1)
        return (ho, hits, self.c1.cpu().numpy().view(np.uint32), self.c2.cpu().numpy().view(np.uint32),
                self.status.cpu().numpy())


def _reads_struct(bases, offsets, max_diff, max_len, lengths=None):
    n = offsets.shape[0] - 1 if lengths is None else lengths.shape[0]
    if max_len is None:
        raise ValueError("max_len (a host-known bound on read length) is required")
    return _Reads(_dptr(bases) if bases.numel() else 0, _dptr(offsets),
                  _dptr(max_diff) if max_diff is not None else None, n, max_len,
                  _dptr(lengths) if lengths is not None else None)


def align_batch(index: Index, bases, offsets, params: Params, max_diff=None, max_len: int | None = None,
                hit_capacity: int | None = None, stream=None, counted: bool = False, out: AlignResult | None = None,
                lengths=None) -> AlignResult:
    """Align a ragged batch of reads (device uint8 bases, device int64
    offsets; or start offsets plus device int32 lengths) on both strands.
    Returns device tensors; grows the hit buffer and retries once if it was
    too small."""
    torch = _torch()
    n = offsets.shape[0] - 1 if lengths is None else lengths.shape[0]
    dev = offsets.device
    rd = _reads_struct(bases, offsets, max_diff, max_len, lengths)
    if out is None:
        cap = hit_capacity if hit_capacity is not None else max(16, 4 * n)
        out = AlignResult(torch.empty(n + 1, dtype=torch.int64, device=dev),
                          torch.empty((cap, 4), dtype=torch.int32, device=dev),
                          torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
                          torch.empty(n, dtype=torch.uint8, device=dev), n)
    if counted and out.expand is None:
        out.expand = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    if counted and getattr(out, "work", None) is None:
        out.work = torch.zeros(14, dtype=torch.int64, device=dev)
    pc = params._c()
    for attempt in range(2):
        res = out._c()
        if counted:
            rc = lib().bwfm_align_batch_counted(index.handle, ctypes.byref(rd), ctypes.byref(pc), ctypes.byref(res),
                                                _dptr(out.expand), _dptr(out.work), _stream_ptr(stream))
        else:
            rc = lib().bwfm_align_batch(index.handle, ctypes.byref(rd), ctypes.byref(pc), ctypes.byref(res),
                                        _stream_ptr(stream))
        if rc == E_CAPACITY and attempt == 0:
            need = int(out.hit_offsets[n].item())
            out.hits = torch.empty((max(need, 1), 4), dtype=torch.int32, device=dev)
            continue
        _check(rc)
        break
    return out


def locate(index: Index, res: AlignResult, max_occ: int, stream=None):
    """Positions of every hit no wider than max_occ: (pos_offsets int64
    [n_hits + 1], positions int32 [total] holding uint32 values)."""
    torch = _torch()
    dev = res.hit_offsets.device
    n_hits = res.n_hits
    po = torch.empty(n_hits + 1, dtype=torch.int64, device=dev)
    cap = max(1, 2 * n_hits)
    pos = torch.empty(cap, dtype=torch.int32, device=dev)
    r = res._c()
    rc = lib().bwfm_locate(index.handle, res.n_reads, ctypes.byref(r), max_occ, _dptr(po), _dptr(pos), cap,
                           _stream_ptr(stream))
    if rc == E_CAPACITY:
        cap = int(po[n_hits].item())
        pos = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        rc = lib().bwfm_locate(index.handle, res.n_reads, ctypes.byref(r), max_occ, _dptr(po), _dptr(pos), cap,
                               _stream_ptr(stream))
    _check(rc)
    return po, pos[:int(po[n_hits].item())]


def pair_reads(index: Index, r1: AlignResult, r2: AlignResult | None, lo: int, hi: int, mu: int, max_occ: int,
               stream=None, out=None, noalloc: bool = False):
    """Pair end-1 and end-2 alignments (r2 None: single-end primaries).
    Returns a device uint8 tensor [n, 24] of bwfm_pair records.  noalloc:
    call bwfm_pair_reads_noalloc, which works in the library's fixed device
    scratch (pass `out` too for a call that allocates nothing at all)."""
    torch = _torch()
    n = r1.n_reads
    if out is None:
        out = torch.empty((max(n, 1), PAIR_DTYPE.itemsize), dtype=torch.uint8, device=r1.hit_offsets.device)
    pp = _PairParams(lo, hi, mu, max_occ)
    a = r1._c()
    b = r2._c() if r2 is not None else None
    fn = lib().bwfm_pair_reads_noalloc if noalloc else lib().bwfm_pair_reads
    _check(fn(index.handle, n, ctypes.byref(a), ctypes.byref(b) if b is not None else None,
              ctypes.byref(pp), _dptr(out), _stream_ptr(stream)))
    return out


@dataclass
class RescueParams:
    """Local-alignment scores of mate rescue (bwfm_rescue_params); defaults
    are BWA-MEM's documented ones, reporting from score 20."""
    match: int = 1
    mismatch: int = 4
    gap_open: int = 6
    gap_extend: int = 1
    min_score: int = 20

    def _c(self) -> _RescueParams:
        return _RescueParams(self.match, self.mismatch, self.gap_open, self.gap_extend, self.min_score)


def rescue_mates(index: Index, end1, end2, pairs, lo: int, hi: int, max_len: int,
                 params: RescueParams | None = None, stream=None, out=None):
    """Mate rescue for the pairs without a proper pair (bwfm_rescue_mates).
    end1/end2: (device uint8 bases, device int64 offsets [n + 1]) of the two
    ends; pairs: device uint8 [n, 24] records from pair_reads.  Returns a
    device uint8 tensor [n, 16] of bwfm_rescue records; does not synchronise."""
    torch = _torch()
    n = end1[1].shape[0] - 1
    if out is None:
        out = torch.empty((max(n, 1), RESCUE_DTYPE.itemsize), dtype=torch.uint8, device=end1[1].device)
    r1 = _reads_struct(end1[0], end1[1], None, max_len)
    r2 = _reads_struct(end2[0], end2[1], None, max_len)
    pp = _PairParams(lo, hi, 0, 0)
    rp = (params or RescueParams())._c()
    _check(lib().bwfm_rescue_mates(index.handle, ctypes.byref(r1), ctypes.byref(r2), n, _dptr(pairs) if n else None,
                                   ctypes.byref(pp), ctypes.byref(rp), _dptr(out), _stream_ptr(stream)))
    return out


def mapq(r1: AlignResult, r2: AlignResult | None, pairs, rescue=None, budgets1=None, budgets2=None,
         max_diff: int = 4, q_tier: int = 22, q_unique: int = 37, q_budget: int = 25, q_pair: int = 60,
         stream=None, out=None):
    """MAPQ of both ends of every pair (bwfm_mapq): device uint8 [n, 2].
    pairs/rescue: device records from pair_reads / rescue_mates; budgets:
    device uint8 per read or None (max_diff for all).  Does not synchronise."""
    torch = _torch()
    n = r1.n_reads
    if out is None:
        out = torch.empty((max(n, 1), 2), dtype=torch.uint8, device=r1.hit_offsets.device)
    a = r1._c()
    b = r2._c() if r2 is not None else None
    mp = _MapqParams(q_tier, q_unique, q_budget, q_pair)
    _check(lib().bwfm_mapq(n, ctypes.byref(a), ctypes.byref(b) if b is not None else None,
                           _dptr(budgets1) if budgets1 is not None else None,
                           _dptr(budgets2) if budgets2 is not None else None, max_diff,
                           _dptr(pairs) if n else None, _dptr(rescue) if rescue is not None else None,
                           ctypes.byref(mp), _dptr(out), _stream_ptr(stream)))
    return out


def rescue_numpy(t) -> np.ndarray:
    return t.cpu().numpy().view(RESCUE_DTYPE).reshape(-1)


def pairs_numpy(t) -> np.ndarray:
    return t.cpu().numpy().view(PAIR_DTYPE).reshape(-1)


def timing_enable(on: bool = True):
    _check(lib().bwfm_timing_enable(1 if on else 0))


def timing_reset():
    _check(lib().bwfm_timing_reset())


def timing_get(kernel: str):
    """(total milliseconds, launches) of one kernel since the last reset."""
    ms = ctypes.c_double()
    n = ctypes.c_uint64()
    _check(lib().bwfm_timing_get(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def probe_gather(buf, line_bytes: int = 128, lanes: int = 0, iters: int = 256, stream=None) -> float:
    """Dependent random line fetches over the device tensor buf; returns
    lines per second.  lanes defaults to 256 per CU x 16."""
    torch = _torch()
    if lanes == 0:
        lanes = torch.cuda.get_device_properties(buf.device).multi_processor_count * 256 * 16
    sink = torch.empty(lanes, dtype=torch.int32, device=buf.device)
    ms = ctypes.c_double()
    _check(lib().bwfm_probe_gather(_dptr(buf), buf.numel() * buf.element_size(), line_bytes, lanes, iters,
                                   _dptr(sink), ctypes.byref(ms), _stream_ptr(stream)))
    return lanes * iters / (ms.value / 1e3)


def estimate_insert(inserts: np.ndarray):
    a = np.ascontiguousarray(inserts, np.int32)
    pp = _PairParams(0, 0, 0, 0)
    _check(lib().bwfm_estimate_insert(_np_ptr(a) if len(a) else None, len(a), ctypes.byref(pp)))
    return pp.lo, pp.hi, pp.mu


def max_diff_rule(length: int, err: float = 0.02, thres: float = 0.04) -> int:
    return lib().bwfm_max_diff_rule(length, err, thres)


class Server:
    """Continuous-batching request server (bwfm_server_*): submit host read
    pairs, wait for their pair records.  Thread safe."""

    def __init__(self, index: Index, params: Params, lo: int, hi: int, mu: int, max_occ: int,
                 arena_bytes: int = 1 << 30, step_pairs: int = 65536, max_len: int = 150, paired: bool = True,
                 budget_rule: bool = False, rescue_mapq: bool = False):
        self._index = index  # keep the index alive
        h = ctypes.c_void_p()
        ap = params._c()
        pp = _PairParams(lo, hi, mu, max_occ)
        sp = _ServerParams(arena_bytes, step_pairs, max_len, 1 if paired else 0, 1 if budget_rule else 0,
                           1 if rescue_mapq else 0)
        _check(lib().bwfm_server_create(index.handle, ctypes.byref(ap), ctypes.byref(pp), ctypes.byref(sp),
                                        ctypes.byref(h)))
        self._h = h
        self.paired = paired
        self.rescue_mapq = rescue_mapq

    def submit(self, bases1: np.ndarray, offsets1: np.ndarray, bases2: np.ndarray | None = None,
               offsets2: np.ndarray | None = None) -> int:
        b1 = np.ascontiguousarray(bases1, np.uint8)
        o1 = np.ascontiguousarray(offsets1, np.uint64)
        b2 = np.ascontiguousarray(bases2, np.uint8) if bases2 is not None else None
        o2 = np.ascontiguousarray(offsets2, np.uint64) if offsets2 is not None else None
        t = ctypes.c_uint64()
        _check(lib().bwfm_server_submit(self._h, _np_ptr(b1) if len(b1) else None, _np_ptr(o1),
                                        _np_ptr(b2) if b2 is not None and len(b2) else None,
                                        _np_ptr(o2) if o2 is not None else None, len(o1) - 1, ctypes.byref(t)))
        return t.value

    def wait(self, ticket: int, n_pairs: int, extras: bool = False):
        """(pair records PAIR_DTYPE[n_pairs], {queued_ms, service_ms, latency_ms});
        with extras (a rescue_mapq server), also the rescue records
        RESCUE_DTYPE[n_pairs] and the MAPQ bytes uint8[n_pairs, 2]."""
        out = np.zeros(max(n_pairs, 1), PAIR_DTYPE)
        resc = np.zeros(max(n_pairs, 1), RESCUE_DTYPE)
        mq = np.zeros((max(n_pairs, 1), 2), np.uint8)
        tm = _Times()
        _check(lib().bwfm_server_wait(self._h, ticket, _np_ptr(out), _np_ptr(resc) if extras else None,
                                      _np_ptr(mq) if extras else None, ctypes.byref(tm)))
        times = {"queued_ms": tm.queued_ms, "service_ms": tm.service_ms, "latency_ms": tm.latency_ms}
        if extras:
            return out[:n_pairs], resc[:n_pairs], mq[:n_pairs], times
        return out[:n_pairs], times

    def stats(self) -> dict:
        s = _ServerStats()
        _check(lib().bwfm_server_get_stats(self._h, ctypes.byref(s)))
        return {"steps": s.steps, "pairs": s.pairs, "requests_done": s.requests_done, "busy_ms": s.busy_ms}

    def close(self):
        if getattr(self, "_h", None):
            lib().bwfm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DeviceView:
    """A device buffer the library owns, seen by torch without a copy
    (through the CUDA array interface, which torch's ROCm build reads)."""

    def __init__(self, ptr: int, shape, typestr: str):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (ptr, False),
                                         "version": 3}


def _view(ptr: int, shape, typestr: str):
    torch = _torch()
    if ptr == 0 or 0 in tuple(shape):
        dt = {"<u8": torch.int64, "<i8": torch.int64, "<i4": torch.int32, "|u1": torch.uint8}[typestr]
        return torch.empty(shape, dtype=dt, device="cuda")
    return torch.as_tensor(_DeviceView(ptr, shape, typestr), device="cuda")


class Pipeline:
    """One step of the path (align both ends, locate, pair) over up to
    max_pairs pairs, captured once into a hipGraph and replayed
    (bwfm_pipeline_*).  Outputs are views of library-owned device memory,
    valid until the next run."""

    def __init__(self, index: Index, params: Params, lo: int, hi: int, mu: int, max_occ: int, max_pairs: int,
                 max_len: int, max_bases: int | None = None, hit_capacity: int | None = None,
                 pos_capacity: int | None = None, paired: bool = True):
        self.index = index  # keeps the index alive
        self.max_pairs = max_pairs
        self.paired = paired
        q = _PipeParams(max_pairs, max_len, max_bases if max_bases is not None else 2 * max_pairs * max_len,
                        hit_capacity if hit_capacity is not None else 8 * max_pairs,
                        pos_capacity if pos_capacity is not None else 64 * max_pairs, 1 if paired else 0)
        self.hit_capacity = q.hit_capacity
        self.pos_capacity = q.pos_capacity
        ap = params._c()
        pp = _PairParams(lo, hi, mu, max_occ)
        h = ctypes.c_void_p()
        _check(lib().bwfm_pipeline_create(index.handle, ctypes.byref(ap), ctypes.byref(pp), ctypes.byref(q),
                                          ctypes.byref(h)))
        self._h = h
        self.n_pairs = 0

    def close(self):
        if getattr(self, "_h", None):
            lib().bwfm_pipeline_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_reads(self, bases, offsets, n_pairs: int, max_len: int, max_diff=None, stream=None):
        """Copy the next batch (end-1 reads then end-2 reads, device tensors)
        into the pipeline."""
        rd = _reads_struct(bases, offsets, max_diff, max_len)
        _check(lib().bwfm_pipeline_set_reads(self._h, ctypes.byref(rd), n_pairs, _stream_ptr(stream)))
        self.n_pairs = n_pairs

    def run(self, graph: bool = True, stream=None):
        _check(lib().bwfm_pipeline_run(self._h, 1 if graph else 0, _stream_ptr(stream)))

    def finish(self, stream=None) -> dict:
        st = _PipeStatus()
        _check(lib().bwfm_pipeline_finish(self._h, _stream_ptr(stream), ctypes.byref(st)))
        return {"n_pairs": st.n_pairs, "error": st.error, "n_hits": st.n_hits, "n_positions": st.n_positions,
                "kernel_ms": st.kernel_ms}

    def results(self):
        """(end-1 AlignResult, end-2 AlignResult, pair records uint8 [n, 24],
        position offsets int64 [n_hits + 1], positions int32) of the last run."""
        n = self.n_pairs
        out = []
        po = ctypes.c_void_p()
        pos = ctypes.c_void_p()
        prs = ctypes.c_void_p()
        for e in ((0, 1) if self.paired else (0,)):
            r = _AlnResult()
            _check(lib().bwfm_pipeline_outputs(self._h, e, ctypes.byref(r), ctypes.byref(po), ctypes.byref(pos),
                                               ctypes.byref(prs)))
            out.append(AlignResult(_view(r.hit_offsets or 0, (n + 1,), "<i8"),
                                   _view(r.hits or 0, (r.hit_capacity, 4), "<i4"), _view(r.c1 or 0, (n,), "<i4"),
                                   _view(r.c2 or 0, (n,), "<i4"), _view(r.status or 0, (n,), "|u1"), n))
        n_hits = int(out[-1].hit_offsets[n].item()) if n else 0
        return (out[0], out[1] if self.paired else None, _view(prs.value or 0, (n, PAIR_DTYPE.itemsize), "|u1"),
                _view(po.value or 0, (n_hits + 1,), "<i8"), _view(pos.value or 0, (self.pos_capacity,), "<i4"))
