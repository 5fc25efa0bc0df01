"""CPU tests of the benchmark's host logic: the one-GPU guard, the traffic
figure's source-hash gate, and the CPU baseline record."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_is_reported_only_for_the_profiled_sources(tmp_path, monkeypatch):
    # the committed summary, stamped with the hash of the current sources:
    # its dominant-kernel row gives the bytes per launch
    import hashlib
    import re
    text = open(bench.PROFILE).read()
    h = re.search(r"first 16 hex\): ([0-9a-f]{16})", text).group(1)
    now = hashlib.sha256(b"".join(open(f, "rb").read() for f in bench.KERNEL_SOURCES)).hexdigest()[:16]
    fresh = tmp_path / "fresh.md"
    fresh.write_text(text.replace(h, now))
    monkeypatch.setattr(bench, "PROFILE", str(fresh))
    row = next(l for l in text.splitlines() if l.startswith("| fx::k_ew[c2,f32"))
    cells = [c.strip() for c in row.strip("|").split("|")]
    want = int(round((float(cells[5]) + float(cells[6])) * 2 ** 20))
    assert bench.measured_traffic() == want
    assert abs(want - (1 << 30)) < 2 ** 30 // 1000  # the kernel moves its 1 GiB, to 0.1%
    # a summary whose source hash differs is ignored
    stale = tmp_path / "stale.md"
    stale.write_text(text.replace(h, "0" * 16))
    monkeypatch.setattr(bench, "PROFILE", str(stale))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "PROFILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None


def test_cpu_baseline_record():
    r = bench.cpu_baseline(cols_sample=16, min_seconds=0.2, threads=2)
    assert set(r) == {"value", "unit", "cores", "kind", "sample"}
    assert r["kind"] == "oracle" and r["unit"] == "GB/s" and r["cores"] == 2
    assert r["value"] > 0 and "8192 x 16 columns" in r["sample"]
