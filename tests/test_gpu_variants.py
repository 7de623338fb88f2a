"""Kernel variants of the genetic-improvement search (paper_1505_07855_amd
.variants) against the oracle: two variant libraries, built on the CPU by
the package build with alternative implementations of the row masks, the
paired rank query, the refill of idle lanes and the sub-counted header
loads, each loaded in a process of its own and compared with the oracle on
both rank-line layouts, both forms (the batched one also with split
searches), locate and pairing."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

from paper_1505_07855_amd import variants

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("defs", variants.TEST_VARIANTS, ids=[variants.name_of(d) for d in variants.TEST_VARIANTS])
def test_variant_library_equals_oracle(defs):
    lib = variants.lib_path(defs)
    if not os.path.exists(lib):
        pytest.fail(f"{lib} is missing: the package build (__graft_entry__.build) compiles it")
    print(f"[variants] checking {variants.name_of(defs)}", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "variant_check.py"), lib], cwd=ROOT,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-3000:])
    assert "variant ok" in r.stdout
