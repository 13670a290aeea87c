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


def test_model_bytes_per_dof_follow_the_per_dof_model():
    # 16-bit sections in blocks of 64: beta = 2 + 1/32 bytes per value; the
    # up sweep reads g and y', reads and writes u', and reads the coarse
    # correction (codes and float32 z, 1/8 of the values): 8.879 B/DoF
    beta = 2.0 + 2.0 / 64
    assert abs(bench.model_bytes_per_dof("k_up_smooth<4>", 16, 64) - 8.87890625) < 1e-12
    assert bench.model_bytes_per_dof("k_ir_residual", 16, 64) == 2 * beta + beta / 8 + 8.0 / 64 + 8.0
    assert bench.model_bytes_per_dof("k_down_smooth<4>", 8, 64) == 2 * (1.0 + 2.0 / 64)


def test_per_level_rows_are_summed_per_kernel():
    rows = [dict(kernel="k_a@10", launches=2, ms=4.0, bytes=8.0), dict(kernel="k_a@9", launches=2, ms=1.0, bytes=1.0),
            dict(kernel="k_b", launches=1, ms=3.0, bytes=2.0)]
    got = bench._by_kernel(rows)
    assert [r["kernel"] for r in got] == ["k_a", "k_b"]
    assert got[0]["launches"] == 4 and got[0]["ms"] == 5.0 and got[0]["bytes"] == 9.0


def test_kernel_family_names_and_containers():
    # the profiler's kernel names map to the library's timing names, with the
    # container (the last integer template argument)
    assert bench._family("void cmg::k_up_smooth<4, 32, 768, 6, false, 16>(float const*)") == ("k_up_smooth<4>", 16)
    assert bench._family("void cmg::k_ir_residual<32, 1024, 2, 6, false, false, 16, true>(cmg::PSec)") == \
        ("k_ir_residual", 16)
    assert bench._family("void cmg::k_decode_full<8, 6, true, false, 32, false>(cmg::PSec)") == ("k_decode_level", 32)
    assert bench._family("void cmg::k_decode_full<8, 6, false, false, 16, false>(cmg::PSec)") == ("k_decode_full", 16)
    assert bench._family("void at::native::reduce_kernel<512, 1>(x)") == (None, None)
