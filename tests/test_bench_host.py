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


@pytest.mark.parametrize("workers", [1, 2])
def test_oracle_baseline_record_on_a_small_frame(workers):
    from tests.workloads import workload
    w = workload("c3fd")
    base, parts = bench.cpu_baseline(w, workers=workers, per_worker=24)
    assert set(base) == {"value", "unit", "cores", "kind", "sample"}
    assert base["kind"] == "oracle" and base["cores"] == workers and base["unit"] == "cone samples/s"
    assert base["value"] > 0 and parts["samples"] > 0 and parts["pixels"] == 24 * workers
    assert f"{w.n}^3" in base["sample"] and f"{24 * workers} seeded pixels" in base["sample"]
    assert f"{workers} processes" in base["sample"]
    assert parts["mips_s"] >= 0 and parts["parallel_s"] > 0
    assert parts["forward_samples_per_s"] > 0 and parts["backward_samples_per_s"] > 0
    # the same pixels give the same sample count however they are split
    if workers == 2:
        _, one = bench.cpu_baseline(w, workers=1, per_worker=48)
        assert one["samples"] == parts["samples"]


def test_worker_count_is_the_hosts_cores_up_to_sixteen():
    assert bench.cpu_workers(3) == 3
    assert 1 <= bench.cpu_workers() <= 16
    assert bench.cpu_workers() == min(16, os.cpu_count() or 1)


def test_flop_model_counts_levels_read():
    assert bench.flops((10, 0), bench.FLOPS_FWD) == 10 * 116
    assert bench.flops((10, 10), bench.FLOPS_FWD) == 10 * 220
    assert bench.flops((10, 4), bench.FLOPS_BWD_SCATTER) == 6 * 202 + 4 * 370
    # a second level adds its 91 flops and the 13 of the blend (forward), and
    # the 64 of its weighted contributions (scatter)
    assert bench.FLOPS_FWD[2] - bench.FLOPS_FWD[1] == 91 + 13
    assert bench.FLOPS_BWD_SCATTER[2] - bench.FLOPS_BWD_SCATTER[1] == 91 + 13 + 64


def test_trace_kernel_traffic_is_gated_on_its_own_sources(tmp_path, monkeypatch):
    d_tr = bench.kernel_source_digest(kernel="k_trace")
    d_p2 = bench.kernel_source_digest(kernel="k_bwd_pass2")
    assert d_tr != d_p2
    prof = tmp_path / "profile.md"
    monkeypatch.setattr(bench, "PROFILE", str(prof))
    prof.write_text(f"    traffic k_trace: fetch_bytes=10 write_bytes=5 sources={d_tr}\n"
                    f"    traffic k_bwd_pass2: fetch_bytes=7 write_bytes=1 sources={d_tr}\n")
    assert bench.measured_traffic("k_trace")[0] == 15
    assert bench.measured_traffic("k_bwd_pass2")[0] is None     # another kernel's digest


def test_l2_hit_rate_comes_with_the_traffic_line(tmp_path, monkeypatch):
    d_tr = bench.kernel_source_digest(kernel="k_trace")
    prof = tmp_path / "profile.md"
    monkeypatch.setattr(bench, "PROFILE", str(prof))
    prof.write_text(f"    traffic k_trace: fetch_bytes=10 write_bytes=5 l2_hit=0.817 sources={d_tr}\n"
                    f"    traffic k_bwd_pass2: fetch_bytes=7 write_bytes=1 l2_hit=0.191 sources=0123456789abcdef\n")
    assert bench.measured_traffic("k_trace")[0] == 15 and bench.measured_l2_hit("k_trace") == 0.817
    assert bench.measured_l2_hit("k_bwd_pass2") is None          # stale digest: neither figure
    prof.write_text(f"    traffic k_trace: fetch_bytes=10 write_bytes=5 sources={d_tr}\n")
    assert bench.measured_traffic("k_trace")[0] == 15 and bench.measured_l2_hit("k_trace") is None


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
