"""Host-side contract of bench.py that needs no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_is_read_only_for_the_profiled_kernel_source(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    n = 256
    text = open(bench.TRAFFIC_SUMMARY).read()
    # the committed summary matches the sources as they are (after a change
    # to the step kernel, take the two counter runs again)
    assert bench.traffic_from_profile(n) is not None, "counter summary older than the kernel"
    assert bench.traffic_from_profile(n + 1) is None
    # a summary taken on another source is ignored
    stale = tmp_path / "stale.md"
    stale.write_text(text.replace(bench.kernel_source_sha(), "0" * 64))
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(stale))
    assert bench.traffic_from_profile(n) is None
    json.dumps({"traffic": bench.traffic_from_profile(n)})
