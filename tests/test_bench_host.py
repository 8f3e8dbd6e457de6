"""Host-side logic of bench.py (no GPU): the one-GPU guard, the traffic
records read from the committed counter profile and their source hashes."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_kernel_sources_exist_and_hash_is_stable():
    for k, files in bench.KERNEL_SOURCES.items():
        for f in files:
            assert os.path.exists(os.path.join(ROOT, "paper_2402_00525_amd", "csrc", f)), (k, f)
        h = bench.kernel_source_hash(k)
        assert len(h) == 16 and h == bench.kernel_source_hash(k)


def test_every_timed_kernel_has_a_traffic_record():
    # One record per timed kernel in the committed profile: kernel, workload,
    # bytes per launch, hash of the sources the counters were taken from.
    recs = {}
    with open(bench.PROFILE) as f:
        for ln in f:
            p = ln.split()
            if len(p) == 5 and p[0] == "traffic":
                recs[p[1]] = (int(p[3]), p[4])
    for k in bench.KERNEL_SOURCES:
        assert k in recs and recs[k][0] > 0 and len(recs[k][1]) == 16, k


def test_traffic_record_is_void_once_sources_change(monkeypatch):
    k = "k_render_hier1"
    recorded = [ln.split()[4] for ln in open(bench.PROFILE) if ln.startswith("traffic %s 3m_1080p " % k)][0]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda kernel: recorded)
    assert bench.profiled_traffic(k, "3m_1080p") is not None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda kernel: "0" * 16)
    assert bench.profiled_traffic(k, "3m_1080p") is None
    assert bench.profiled_traffic(k, "no_such_workload") is None


def test_traffic_record_parsing(tmp_path, monkeypatch):
    p = tmp_path / "prof.md"
    h = bench.kernel_source_hash("k_duplicate")
    p.write_text("text\ntraffic k_duplicate w1 12345 %s\ntraffic k_duplicate w2 99 deadbeefdeadbeef\n"
                 "traffic k_duplicate w3 notanumber\n" % h)
    monkeypatch.setattr(bench, "PROFILE", str(p))
    assert bench.profiled_traffic("k_duplicate", "w1") == 12345
    assert bench.profiled_traffic("k_duplicate", "w2") is None
    assert bench.profiled_traffic("k_duplicate", "w3") is None
    monkeypatch.setattr(bench, "PROFILE", str(tmp_path / "missing.md"))
    assert bench.profiled_traffic("k_duplicate", "w1") is None


@pytest.mark.parametrize("argv", [[], ["--steps", "3", "--warmup", "1", "--no-batch"]])
def test_argument_defaults(argv, monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"] + argv)
    a = bench.parse()
    assert a.gpus == 1 and a.workload == "3m_1080p"
    assert a.steps >= 1 and a.warmup >= 0


def test_timed_views_span_the_orbit():
    import bench
    for steps in (1, 5, 20, 30, 60):
        views = [bench.timed_view(i, steps, 60) for i in range(steps)]
        assert views == sorted(set(views)) and views[0] == 0
        assert max(views) >= 60 - 60 // steps - 1
    assert [bench.timed_view(i, 90, 60) for i in range(90)][60:] == list(range(30))
