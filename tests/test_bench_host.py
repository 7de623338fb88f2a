"""Host logic of the benchmark: reading counter-measured traffic from the
committed profile summaries (the `bench-traffic:` record). A record counts
only for the kernel sources it was taken on and, where it names settings
(the split budget of the stress batch), only for those settings."""
from __future__ import annotations

import glob
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

RECORD = ("bench-traffic: kernel=k_align_persistent source=abc split=1024 fetch_kib=100 write_kib=10 "
          "copy_fetch_kib=50 copy_write_kib=100 copy_bytes=102400\n")


@pytest.fixture
def fake_root(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "k_align_persistent_c5_bytes.md").write_text("# summary\n\n" + RECORD)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda kernel="k_align_persistent": "abc")
    return tmp_path


def test_traffic_scales_each_counter_by_the_copy(fake_root):
    # fetch: 100 KiB read where a copy of 102400 B reads 50 KiB -> x2;
    # write: 10 KiB where the copy writes 100 KiB -> x1
    want = 100 * 1024 * 102400 / (50 * 1024) + 10 * 1024 * 102400 / (100 * 1024)
    assert bench.traffic_from_profiles("k_align_persistent", "c5", split=1024) == pytest.approx(want)
    assert bench.traffic_from_profiles("k_align_persistent", "c5") == pytest.approx(want)


def test_traffic_needs_matching_sources_and_settings(fake_root, monkeypatch):
    assert bench.traffic_from_profiles("k_align_persistent", "c5", split=4096) is None
    assert bench.traffic_from_profiles("k_align_persistent", "c2") is None  # no summary
    monkeypatch.setattr(bench, "kernel_source_hash", lambda kernel="k_align_persistent": "other")
    assert bench.traffic_from_profiles("k_align_persistent", "c5", split=1024) is None


def test_the_record_of_the_setting_is_used(fake_root):
    path = fake_root / "profiles" / "k_align_persistent_c5_bytes.md"
    path.write_text(path.read_text() + RECORD.replace("split=1024", "split=512").replace("fetch_kib=100", "fetch_kib=200"))
    one = bench.traffic_from_profiles("k_align_persistent", "c5", split=1024)
    two = bench.traffic_from_profiles("k_align_persistent", "c5", split=512)
    assert two - one == pytest.approx(100 * 1024 * 102400 / (50 * 1024))
    assert bench.traffic_from_profiles("k_align_persistent", "c5", split=256) is None


def test_committed_records_are_well_formed():
    files = glob.glob(os.path.join(ROOT, "profiles", "*_bytes.md"))
    recs = 0
    for f in files:
        for line in open(f):
            if line.startswith("bench-traffic:"):
                rec = dict(kv.split("=", 1) for kv in line.split()[1:])
                assert rec["kernel"] in bench.KERNEL_SOURCES, f
                assert len(rec["source"]) == 16, f
                for k in ("fetch_kib", "write_kib", "copy_fetch_kib", "copy_write_kib", "copy_bytes"):
                    assert float(rec[k]) > 0, (f, k)
                recs += 1
    assert recs >= 3


def test_tuner_prefers_longer_lines_within_the_tie():
    from paper_1505_07855_amd import tune

    def row(lb, w, ms):
        return {"line_bytes": lb, "waves_per_simd": w, "ms": ms}

    # 128-byte lines 1.25% behind the fastest 64-byte layout: a tie, the
    # longer lines win (the case seen on one GPU)
    t = [row(128, 0, 105.3), row(64, 0, 104.0), row(64, 3, 119.1)]
    assert tune.pick(t) is t[0]
    # beyond the tie the fastest wins, whatever its lines
    assert tune.pick(t, tie=0.01) is t[1]
    t2 = [row(128, 0, 107.0), row(64, 0, 104.0)]
    assert tune.pick(t2) is t2[1]
    # among tied rows of the same line size the faster one
    t3 = [row(128, 3, 101.5), row(128, 0, 101.0), row(64, 0, 100.0)]
    assert tune.pick(t3) is t3[1]
