"""Host-side logic of bench.py (no GPU): the refusal of several GPUs and
the stored counter readings, which are reported only for the kernel sources
they were taken on."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "exactly one GPU" in res.stderr


def test_stored_counters_follow_the_kernel_sources(monkeypatch):
    traffic = bench.stored_traffic("k_up_smooth<4>")
    valu = bench.stored_valu("k_up_smooth<4>")
    if traffic is None or valu is None:
        pytest.skip("the stored counter readings predate the current kernel sources")
    assert 1e8 < traffic < 1e11 and 1e6 < valu < 1e10
    assert bench.stored_traffic("no such kernel") is None
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0" * 64)
    assert bench.stored_traffic("k_up_smooth<4>") is None
    assert bench.stored_valu("k_up_smooth<4>") is None


def test_source_digest_ignores_comments(tmp_path, monkeypatch):
    d0 = bench.kernel_source_digest()
    csrc = tmp_path / "paper_2511_19036_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in ("fused.hip", "plane.h", "device.h"):
        with open(os.path.join(ROOT, "paper_2511_19036_amd", "csrc", name)) as fh:
            text = fh.read()
        (csrc / name).write_text("// an added comment\n" + text.replace("\n", "\n\n", 3))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_digest() == d0
    (csrc / "plane.h").write_text((csrc / "plane.h").read_text() + "\nint changed;\n")
    assert bench.kernel_source_digest() != d0
