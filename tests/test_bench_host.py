"""Host logic of bench.py (CPU): the source digest that ties the committed HBM counters to the
kernels they were taken on, the traffic read-back, and the one-GPU guard."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _copy_sources(tmp_path):
    d = tmp_path / "csrc"
    shutil.copytree(os.path.join(ROOT, "paper_2506_19919_amd", "csrc"), d,
                    ignore=shutil.ignore_patterns("*.o", "_build"))
    return d


def test_digest_ignores_comments_and_whitespace_but_not_code(tmp_path):
    d = _copy_sources(tmp_path)
    ref = bench.kernel_source_digest(str(d))
    f = d / "sps_approx.hip"
    text = f.read_text()
    f.write_text("// a new comment\n/* and a block\n comment */\n" + text.replace("\n", "\n\n", 3))
    assert bench.kernel_source_digest(str(d)) == ref
    f.write_text(text + "\nstatic int digest_probe = 1;\n")
    assert bench.kernel_source_digest(str(d)) != ref


def test_traffic_read_back_follows_the_digest(tmp_path):
    summary = tmp_path / "traffic.md"
    lines = ["traffic_fetch_bytes_per_launch: `100.0`", "traffic_write_bytes_per_launch: `23.5`"]
    summary.write_text("\n".join(lines + [f"traffic_source_sha256: `{bench.kernel_source_digest()}`"]) + "\n")
    assert bench.measured_traffic(str(summary)) == pytest.approx(123.5)
    summary.write_text("\n".join(lines + ["traffic_source_sha256: `0000`"]) + "\n")
    assert bench.measured_traffic(str(summary)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.md")) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout
