"""Host C and C++ under AddressSanitizer and UndefinedBehaviorSanitizer.

* The host index builder (index_host.cpp) is compiled with the sanitizers
  into a harness of its own (tests/sanitize/index_host_harness.cpp) that
  builds, queries, saves and reloads indexes in every rank-line layout and
  takes the argument-error paths.
* The oracle, its brute-force checkers and the input generator are built as
  sanitizer variants (lib*.san.so) and the oracle's and generator's CPU tests
  run against them in a child process that preloads the sanitizer runtimes
  (BWFM_SANITIZE=1 selects the variants).

Any sanitizer report aborts the child, so a zero exit status is the pass.
"""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV_SAN = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1", "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _runtime(name: str) -> str:
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"gcc has no {name}")
    return path


def test_host_index_builder_under_sanitizers(tmp_path):
    exe = tmp_path / "index_host_harness"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-pthread", *SAN, "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "sanitize", "index_host_harness.cpp"),
                           os.path.join(ROOT, "paper_1505_07855_amd", "csrc", "index_host.cpp"), "-o", str(exe)])
    r = subprocess.run([str(exe), str(tmp_path)], capture_output=True, text=True, timeout=600,
                       env={**os.environ, **ENV_SAN})
    assert r.returncode == 0, r.stderr[-4000:]
    assert "all checks passed" in r.stdout


@pytest.mark.slow
def test_oracle_and_generator_tests_under_sanitizers():
    import gen
    import oracle
    oracle.build(force=True, sanitize=True)
    gen.build(force=True, sanitize=True)
    env = {**os.environ, **ENV_SAN, "BWFM_SANITIZE": "1",
           "LD_PRELOAD": f"{_runtime('libasan.so')}:{_runtime('libubsan.so')}"}
    # the child loads the sanitizer builds, not the plain ones
    probe = subprocess.run([sys.executable, "-c", "import oracle, gen; print(oracle._lib('oracle')._name); "
                            "print(oracle._lib('brute')._name); print(gen.lib()._name)"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0, probe.stderr[-4000:]
    names = probe.stdout.split()
    assert len(names) == 3 and all(x.endswith(".san.so") for x in names), names
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests/test_oracle.py", "tests/test_gen.py",
                        "tests/test_oracle_scale.py::test_batched_brute_routines_equal_their_one_read_forms"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
