"""bench.py on the CPU: the helpers behind its JSON line.

The byte counts are checked against what the workload fixes independently of
the formulas: at n = 4096 with 64-column pivots, every step's Gram reads all of
G (n * n * 8 bytes) once, and an update whose pivots all rotate reads and writes
all of G.  The counter-traffic reader must report bytes only while the kernel
sources hash to the value recorded beside the counters.
"""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _prof(ms_gram, ms_pivot, ms_update, launches=10, pairs=64, n=4096):
    return dict(block_width=32, nblocks=128,
                gram=dict(launches=launches, units=pairs * launches, ms=ms_gram * launches),
                update=dict(launches=launches, units=pairs * launches, ms=ms_update * launches),
                pivot=dict(launches=launches, units=pairs * launches, ms=ms_pivot * launches),
                final=dict(launches=1, units=1, ms=0.3),
                pivot_cols=64 * pairs * launches, inner_sweeps=pairs * launches,
                rotations=1000 * launches, pivot_cols3=64 ** 3 * pairs * launches)


def test_algorithmic_bytes_at_n4096():
    b = _bench()
    n = 4096
    work = b.algorithmic_work(_prof(0.0335, 0.047, 0.0506), n, False)
    g_bytes = n * n * 8
    assert work["gram"]["bytes"] == pytest.approx(g_bytes, rel=1e-12)
    assert work["update"]["bytes"] == pytest.approx(2 * g_bytes, rel=1e-12)
    # complex: twice the bytes per element
    work_c = b.algorithmic_work(_prof(0.0335, 0.047, 0.0506), n, True)
    assert work_c["gram"]["bytes"] == pytest.approx(2 * g_bytes, rel=1e-12)
    # the symmetric Gram block costs about half of a full product over all pairs
    full = 2 * n * n * 64
    assert work["gram"]["flops"] == pytest.approx(full / 2 * (65 / 64), rel=1e-12)


def test_roofline_reports_the_dominant_kernel():
    b = _bench()
    r, _ = b.roofline(_prof(0.0335, 0.047, 0.0506), 4096, False)
    assert r["kernel"] == "update" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(2 * 4096 * 4096 * 8 / 0.0506e-3 / 1e9, rel=1e-12)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["avg_launch_ms"] == pytest.approx(0.0506)
    r, _ = b.roofline(_prof(0.0335, 0.2, 0.0506), 4096, False)
    assert r["kernel"] == "pivot" and r["bound"] == "alu" and r["peak"] == pytest.approx(78.6)


def test_traffic_reported_only_for_the_recorded_sources(tmp_path, monkeypatch):
    b = _bench()
    csrc = tmp_path / "paper_1008_4166_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text("kernel source\n")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    sha = b.sources_sha256()
    summary = ("sources_sha256 %s\nfetch_factor 2.00\nwrite_factor 1.00\n"
               "kernel update fetch_kib 100.0 write_kib 300.0\n")
    (tmp_path / "profiles" / "traffic_n4096_f64_solve.md").write_text(summary % sha)
    assert b.pmc_traffic("update") == pytest.approx((100.0 * 2.0 + 300.0) * 1024.0)
    assert b.pmc_traffic("gram") is None  # no counters for that kernel
    (csrc / "k.hip").write_text("kernel  source // a comment\n/* and\nanother */\n")
    assert b.pmc_traffic("update") is not None  # comments and spacing do not count
    (csrc / "k.hip").write_text("kernel source, changed\n")
    assert b.pmc_traffic("update") is None  # counters taken for other sources


def test_committed_traffic_summary_parses():
    b = _bench()
    path = os.path.join(ROOT, "profiles", "traffic_n4096_f64_solve.md")
    keys = {}
    with open(path) as f:
        for line in f:
            t = line.split()
            if len(t) == 2 and t[0] in ("sources_sha256", "fetch_factor", "write_factor"):
                keys[t[0]] = t[1]
    assert len(keys["sources_sha256"]) == 64
    assert float(keys["fetch_factor"]) > 0 and float(keys["write_factor"]) > 0
    if keys["sources_sha256"] == b.sources_sha256():
        # the update's counted bytes are within 5% of its algorithmic bytes at n = 4096
        # (all of G read and written when every pivot rotates; 60 of 64 do on average)
        t = b.pmc_traffic("update")
        assert 0.9 * 2 * 4096 * 4096 * 8 < t < 1.05 * 2 * 4096 * 4096 * 8


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
