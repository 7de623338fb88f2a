"""Search over compile-time variants of the search kernel.

The paper improves BarraCUDA by evolving its kernel source and keeping a
change only when the output stays the same and the kernel gets faster
(sections 1, 3 and 5).  Here the changes are restricted to the tuning
constants the kernel source exposes as macros: stack pops per persistent
iteration, first-pass hit slots per lane, second-pass lanes.  Each variant
is its own library build; a variant counts only if its results on the batch
are byte-identical to the reference build's, and the fastest such one wins.

    python -m paper_1505_07855_amd.variants build     # CPU: compile every variant library
    python -m paper_1505_07855_amd.variants search    # GPU: time them on the benchmark batch

`build` needs the objects of a normal build (paper_1505_07855_amd.build)
next to it; `search` runs each variant in a process of its own and prints
one JSON line: the table and the winner.
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

# knob -> (reference value, alternatives)
KNOBS = {
    "BWFM_POPS_PER_STEP": (1, (2, 4)),
    "BWFM_FAST_CAND": (64, (32, 128)),
    "BWFM_SLOW_LANES": (16384, (8192, 32768)),
}


def variants():
    """(name, {macro: value}): the reference build, then one knob changed at a time."""
    out = [("reference", {})]
    for knob, (_, alts) in KNOBS.items():
        for v in alts:
            out.append((f"{knob[5:].lower()}_{v}", {knob: v}))
    return out


def build_one(name: str, defs: dict) -> str:
    from paper_1505_07855_amd import build as B
    d = os.path.join(OUT, name)
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


def build() -> None:
    for name, defs in variants():
        build_one(name, defs)


def _digest(res) -> str:
    ho, hits, c1, c2, st = res.to_numpy()
    h = hashlib.sha256()
    for a in (ho, hits, c1, c2, st & 7):
        h.update(a.tobytes())
    return h.hexdigest()[:16]


def time_one(lib: str, repeats: int = 3) -> dict:
    """Time the batched search of the benchmark batch (both ends in one
    launch) with the library at lib."""
    import numpy as np
    import torch

    import paper_1505_07855_amd as bw
    from gen import configs
    bw.LIB_PATH = lib
    g = configs.c2_genome()
    pairs = configs.c2_pairs(g)
    ix = bw.Index.build_device(g.seq, line_bytes=64)
    e1, e2 = pairs.end1, pairs.end2
    b = torch.from_numpy(np.concatenate([e1.bases, e2.bases])).cuda()
    o = torch.from_numpy(np.concatenate([e1.offsets[:-1], e1.offsets[-1] + e2.offsets]).view(np.int64)).cuda()
    p = bw.Params(**configs.PARAMS["C2"], waves_per_simd=4)
    res = bw.align_batch(ix, b, o, p, max_len=100, hit_capacity=8_000_000)
    torch.cuda.synchronize()
    ms = []
    for _ in range(repeats):
        t = time.perf_counter()
        res = bw.align_batch(ix, b, o, p, max_len=100, out=res)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t) * 1e3)
    return {"lib": lib, "ms": min(ms), "digest": _digest(res)}


def search() -> dict:
    table = []
    for name, defs in variants():
        lib = os.path.join(OUT, name, "libbwfm.so")
        if not os.path.exists(lib):
            raise RuntimeError(f"{lib} is missing: run the build step first")
        r = subprocess.run([sys.executable, "-m", "paper_1505_07855_amd.variants", "time", lib],
                           capture_output=True, text=True, cwd=os.path.dirname(HERE))
        if r.returncode != 0:
            raise RuntimeError(f"variant {name} failed: {r.stderr[-2000:]}")
        rec = json.loads(r.stdout.strip().splitlines()[-1])
        rec.update(name=name, defines=defs)
        table.append(rec)
        print(f"[variants] {name}: {rec['ms']:.1f} ms digest {rec['digest']}", file=sys.stderr, flush=True)
    ref = table[0]["digest"]
    valid = [r for r in table if r["digest"] == ref]
    best = min(valid, key=lambda r: r["ms"])
    return {"table": table, "rejected": [r["name"] for r in table if r["digest"] != ref], "best": best["name"],
            "best_ms": best["ms"], "reference_ms": table[0]["ms"]}


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    what = sys.argv[1] if len(sys.argv) > 1 else "search"
    if what == "build":
        build()
    elif what == "time":
        print(json.dumps(time_one(sys.argv[2])), flush=True)
    else:
        print(json.dumps(search()), flush=True)
