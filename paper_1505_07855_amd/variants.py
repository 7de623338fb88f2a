"""Genetic-improvement style search over compile-time variants of the
search kernel.

The paper improves BarraCUDA by changing its kernel source and keeping a
change only when the output stays the same and the kernel gets faster
(sections 1, 3 and 5).  Here the kernel source (csrc/bwfm.hip) carries
alternative implementations of single code sites ("genes", macros
BWFM_GENE_*: row masks, the paired rank query, the refill of idle lanes,
the sub-counted line's header loads, the D-array scan in the loop or in a
pre-pass, one or two states expanded per lane and iteration, the loads of a
sub-counted query)  next to the tuning constants it
exposes (stack pops per iteration, first-pass hit slots, second-pass
lanes).  A variant is one value per gene; each variant is its own library
build.  The search is a (1+1) evolution strategy in generations:

* generation 1 mutates the reference in every single gene (each
  alternative value once);
* every later generation starts from the best variant so far (the parent)
  and combines it with the genes of the other variants that beat the
  reference, one gene at a time;
* a variant is accepted only if its results on the benchmark batch are
  byte-identical to the reference build's (the fitness test of the paper's
  GI); among those the fastest wins, and a child replaces its parent only
  when it is faster.

Builds run on the CPU and timings on the GPU, so a generation is two steps:

    python -m paper_1505_07855_amd.variants build [state.json]    # CPU: build the generation's variants
    python -m paper_1505_07855_amd.variants search [state.json]   # GPU: time them, update the state

The state file (default _variants/state.json) holds every evaluated
variant, the parent and the next generation to build.  `search` runs each
variant in a process of its own and prints one JSON line per generation.
"""
from __future__ import annotations

import hashlib
import json
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "_variants")

# gene -> (reference value, alternatives)
GENES = {
    "BWFM_GENE_ROWMASK": (0, (1,)),
    "BWFM_GENE_PAIRLINE": (0, (1,)),
    "BWFM_GENE_REFILL": (0, (1,)),
    "BWFM_GENE_SUBHDR": (0, (1,)),
    "BWFM_GENE_DPREPASS": (0, (1,)),
    "BWFM_GENE_TWOSTATE": (0, (1,)),
    "BWFM_GENE_SUBLOAD": (1, (0,)),
    "BWFM_GENE_KTLOOP": (0, (1,)),
    "BWFM_POPS_PER_STEP": (1, (2,)),
    "BWFM_FAST_CAND": (128, (64, 256)),
    "BWFM_SLOW_LANES": (16384, (8192,)),
}


# two variants the package build compiles for the GPU tests: every gene
# away from the shipped value in one of them
TEST_VARIANTS = [{"BWFM_GENE_ROWMASK": 1, "BWFM_GENE_PAIRLINE": 1, "BWFM_GENE_TWOSTATE": 1, "BWFM_GENE_SUBLOAD": 0,
                  "BWFM_GENE_SUBHDR": 1, "BWFM_GENE_KTLOOP": 1},
                 {"BWFM_GENE_REFILL": 1, "BWFM_GENE_DPREPASS": 1, "BWFM_POPS_PER_STEP": 2}]


def name_of(defs: dict) -> str:
    """A variant's name: its genes that differ from the reference."""
    parts = [f"{k[5:].lower().replace('gene_', '')}{v}" for k, v in sorted(defs.items()) if GENES[k][0] != v]
    return "_".join(parts) or "reference"


def first_generation():
    out = [{}]
    for gene, (_, alts) in GENES.items():
        for v in alts:
            out.append({gene: v})
    return out


def next_generation(state: dict):
    """Children of the parent: the parent plus one gene of each variant that
    beat the reference, not evaluated before."""
    parent = state["parent"]["defines"]
    seen = {name_of(r["defines"]) for r in state["table"]}
    ref_ms = state["reference_ms"]
    good = [r for r in state["table"] if r["accepted"] and r["ms"] < ref_ms]
    kids = []
    for r in good:
        for gene, v in r["defines"].items():
            child = {**parent, gene: v}
            child = {k: x for k, x in child.items() if GENES[k][0] != x}
            if name_of(child) not in seen and child not in kids:
                kids.append(child)
    return kids


def build_one(defs: dict) -> str:
    from paper_1505_07855_amd import build as B
    d = os.path.join(OUT, name_of(defs))
    os.makedirs(d, exist_ok=True)
    obj = os.path.join(d, "bwfm.o")
    flags = [f"-D{k}={v}" for k, v in sorted(defs.items())]
    B._run([B.HIPCC, *B.HIP_FLAGS, *flags, "-c", os.path.join(B.CSRC, "bwfm.hip"), "-o", obj])
    others = [os.path.join(B.OUT, f) for f in ("index_host.o", "index_gpu.o", "rescue.o", "mapq.o", "server.o")]
    missing = [f for f in others if not os.path.exists(f)]
    if missing:
        raise RuntimeError(f"build the library first (missing {missing})")
    lib = os.path.join(d, "libbwfm.so")
    B._run([B.HIPCC, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", "-o", lib + ".tmp", obj, *others, "-lpthread"])
    os.replace(lib + ".tmp", lib)
    return lib


def lib_path(defs: dict) -> str:
    return os.path.join(OUT, name_of(defs), "libbwfm.so")


def _load_state(path: str) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {"generation": 0, "table": [], "parent": None, "reference_ms": None, "pending": first_generation()}


def _save_state(path: str, state: dict) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path + ".tmp", "w") as f:
        json.dump(state, f, indent=1)
    os.replace(path + ".tmp", path)


def build(state_path: str) -> list:
    """Build the pending generation's variants (CPU)."""
    state = _load_state(state_path)
    libs = [build_one(d) for d in state["pending"]]
    _save_state(state_path, state)
    return libs


def _digest(res) -> str:
    ho, hits, c1, c2, st = res.to_numpy()
    h = hashlib.sha256()
    for a in (ho, hits, c1, c2, st & 7):
        h.update(a.tobytes())
    return h.hexdigest()[:16]


def time_one(lib: str, line_bytes: int, rank_format: int, repeats: int = 3, waves=(0, 3)) -> dict:
    """Time the batched search of the benchmark batch (both ends in one
    launch) with the library at lib: the median of `repeats` calls at each
    residency in `waves` (0: the build held to four waves per SIMD; 3: the
    compiler's own register budget), and the best of those medians."""
    import numpy as np
    import torch

    import paper_1505_07855_amd as bw
    from gen import configs
    bw.LIB_PATH = lib
    g = configs.c2_genome()
    pairs = configs.c2_pairs(g)
    ix = bw.Index.build_device(g.seq, line_bytes=line_bytes, rank_format=rank_format)
    e1, e2 = pairs.end1, pairs.end2
    b = torch.from_numpy(np.concatenate([e1.bases, e2.bases])).cuda()
    o = torch.from_numpy(np.concatenate([e1.offsets[:-1], e1.offsets[-1] + e2.offsets]).view(np.int64)).cuda()
    per = {}
    digest = None
    for w in waves:
        p = bw.Params(**configs.PARAMS["C2"], waves_per_simd=w)
        res = bw.align_batch(ix, b, o, p, max_len=100, hit_capacity=8_000_000)
        torch.cuda.synchronize()
        d = _digest(res)
        if digest is not None and d != digest:
            raise RuntimeError(f"{lib}: output differs between residencies")
        digest = d
        ms = []
        for _ in range(repeats):
            t = time.perf_counter()
            res = bw.align_batch(ix, b, o, p, max_len=100, out=res)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t) * 1e3)
        per[str(w)] = float(np.median(ms))
    best = min(per, key=per.get)
    return {"lib": lib, "ms": per[best], "waves_per_simd": int(best), "ms_by_waves": per, "digest": digest}


def search(state_path: str, line_bytes: int = 128, rank_format: int = 2) -> dict:
    """Time the pending generation (GPU), each variant in its own process,
    and advance the state: accept byte-identical variants, move the parent
    to the fastest, and list the next generation."""
    state = _load_state(state_path)
    todo = state["pending"]
    if state["reference_ms"] is None and {} not in todo:
        todo = [{}] + todo
    for defs in todo:
        lib = lib_path(defs)
        if not os.path.exists(lib):
            raise RuntimeError(f"{lib} is missing: run the build step first")
        r = subprocess.run([sys.executable, "-m", "paper_1505_07855_amd.variants", "time", lib, str(line_bytes),
                            str(rank_format)], capture_output=True, text=True, cwd=os.path.dirname(HERE))
        if r.returncode != 0:
            raise RuntimeError(f"variant {name_of(defs)} failed: {r.stderr[-2000:]}")
        rec = json.loads(r.stdout.strip().splitlines()[-1])
        rec.update(name=name_of(defs), defines=defs, generation=state["generation"] + 1)
        if not defs:
            state["reference_ms"], state["reference_digest"] = rec["ms"], rec["digest"]
        rec["accepted"] = rec["digest"] == state["reference_digest"]
        state["table"].append(rec)
        print(f"[variants] gen {rec['generation']} {rec['name']}: {rec['ms']:.1f} ms at {rec['waves_per_simd']} "
              f"waves/SIMD {rec['ms_by_waves']} digest {rec['digest']}"
              f"{'' if rec['accepted'] else ' REJECTED (output differs)'}", file=sys.stderr, flush=True)
    ok = [r for r in state["table"] if r["accepted"]]
    best = min(ok, key=lambda r: r["ms"])
    if state["parent"] is None or best["ms"] < state["parent"]["ms"]:
        state["parent"] = best
    state["generation"] += 1
    state["pending"] = next_generation(state)
    _save_state(state_path, state)
    return {"generation": state["generation"], "parent": state["parent"]["name"], "parent_ms": state["parent"]["ms"],
            "reference_ms": state["reference_ms"], "evaluated": len(state["table"]),
            "rejected": [r["name"] for r in state["table"] if not r["accepted"]],
            "next": [name_of(d) for d in state["pending"]]}


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    what = sys.argv[1] if len(sys.argv) > 1 else "search"
    default_state = os.path.join(OUT, "state.json")
    if what == "build":
        build(sys.argv[2] if len(sys.argv) > 2 else default_state)
    elif what == "time":
        print(json.dumps(time_one(sys.argv[2], int(sys.argv[3]), int(sys.argv[4]))), flush=True)
    else:
        print(json.dumps(search(sys.argv[2] if len(sys.argv) > 2 else default_state)), flush=True)
