"""Host-side checks of bench.py (CPU only): the refusal of more than one GPU,
the measured-traffic line of the committed profile and the source digest that
keeps it honest, and the record of the oracle baseline on a small frame."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr


def test_traffic_is_reported_only_for_the_sources_it_was_measured_on(tmp_path, monkeypatch):
    digest = bench.kernel_source_digest()
    assert len(digest) == 16 and int(digest, 16) >= 0
    prof = tmp_path / "profile.md"
    monkeypatch.setattr(bench, "PROFILE", str(prof))
    prof.write_text(f"counters\n\n    traffic k_bwd_pass2: fetch_bytes=1000 write_bytes=234 sources={digest}\n")
    value, note = bench.measured_pass2_traffic()
    assert value == 1234 and "FETCH_SIZE" in note
    prof.write_text("    traffic k_bwd_pass2: fetch_bytes=1000 write_bytes=234 sources=0123456789abcdef\n")
    assert bench.measured_pass2_traffic() == (None, "kernel sources changed since the counters were taken")
    prof.write_text("no counters here\n")
    assert bench.measured_pass2_traffic()[0] is None
    monkeypatch.setattr(bench, "PROFILE", str(tmp_path / "absent.md"))
    assert bench.measured_pass2_traffic() == (None, "no profile")


def test_digest_covers_every_source_of_the_scatter_pass(monkeypatch):
    full = bench.kernel_source_digest()
    sources = list(bench.PASS2_SOURCES)
    assert {"backward.hip", "bwd_pixel.h"} <= set(sources)
    for f in sources:
        monkeypatch.setattr(bench, "PASS2_SOURCES", [g for g in sources if g != f])
        assert bench.kernel_source_digest() != full, f
    monkeypatch.setattr(bench, "PASS2_SOURCES", sources)
    assert bench.kernel_source_digest() == full


def test_oracle_baseline_record_on_a_small_frame():
    from tests.workloads import workload
    w = workload("c3fd")
    base, parts = bench.cpu_baseline(w, n_pix=48)
    assert set(base) == {"value", "unit", "cores", "kind", "sample"}
    assert base["kind"] == "oracle" and base["cores"] == 1 and base["unit"] == "cone samples/s"
    assert base["value"] > 0 and parts["samples"] > 0 and parts["pixels"] == 48
    assert f"{w.n}^3" in base["sample"] and "48 seeded pixels" in base["sample"]
    assert parts["mips_s"] >= 0 and parts["forward_s"] > 0 and parts["backward_s"] > 0


def test_digest_follows_code_not_comments(tmp_path):
    import shutil
    src = os.path.join(ROOT, "paper_2104_00618_amd", "csrc")
    copy = tmp_path / "csrc"
    shutil.copytree(src, copy)
    base = bench.kernel_source_digest(str(copy))
    assert base == bench.kernel_source_digest()
    f = copy / "backward.hip"
    text = f.read_text()
    f.write_text("// a new comment line\n" + text.replace("\n", "\n\n", 3) + "\n/* and a block\n comment */\n")
    assert bench.kernel_source_digest(str(copy)) == base
    f.write_text(text.replace("constexpr int kThreads = 256;", "constexpr int kThreads = 128;"))
    assert bench.kernel_source_digest(str(copy)) != base
    assert bench.code_text("a; // b\n/* c\n d */  e;") == "a; e;"


def test_oracle_baseline_runs_on_one_thread():
    """The baseline says "cores": 1: bench.py times the oracle under a
    one-thread limit for every threaded library NumPy may call."""
    src = open(os.path.join(ROOT, "bench.py")).read()
    assert "threadpool_limits(limits=1)" in src
    from threadpoolctl import threadpool_info, threadpool_limits
    with threadpool_limits(limits=1):
        assert all(p["num_threads"] == 1 for p in threadpool_info())
