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


def test_stored_diffusion_hbm_follows_the_kernel_sources(monkeypatch):
    gbs = bench.stored_diffusion_hbm()
    if gbs is None:
        pytest.skip("the stored diffusion counters predate the current kernel sources")
    assert 100.0 < gbs < 8000.0
    monkeypatch.setattr(bench, "kernel_source_digest", lambda names=None: "0" * 64)
    assert bench.stored_diffusion_hbm() is None


def test_diffusion_summary_takes_the_solve_after_the_calibration_copy(tmp_path):
    # dispatch 1: another 1 GiB copy (not the calibration); 2: warm-up solve
    # kernel; 3: the calibration copy; 4, 6: the measured solve's kernels;
    # 5: a kernel of another library (not counted)
    cal = bench.CALIB_BYTES_DIFF
    fetch = {1: 524288.0, 2: 7.0, 3: cal / 2048.0, 4: 1000.0, 6: 300.0}
    write = {1: 1048576.0, 2: 7.0, 3: cal / 1024.0, 4: 500.0, 6: 100.0}
    names = {1: "__amd_rocclr_copyBuffer", 2: "void cmg::k_a<1>(int)", 3: "__amd_rocclr_copyBuffer",
             4: "void cmg::k_a<1>(int)", 5: "void at::native::other(int)", 6: "void cmg::k_b(float*)"}
    dur = {1: 100, 2: 5, 3: 200, 4: 1000, 5: 7000, 6: 3000}
    for pas, vals in (("dfetch", fetch), ("dwrite", write)):
        with open(tmp_path / f"{pas}_counter_collection.csv", "w") as fh:
            fh.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
            for i, v in vals.items():
                fh.write(f'{i},"{names[i]}",X,{v}\n')
    with open(tmp_path / "dkt_kernel_trace.csv", "w") as fh:
        fh.write("Dispatch_Id,Kernel_Name,Start_Timestamp,End_Timestamp\n")
        for i, d in dur.items():
            fh.write(f'{i},"{names[i]}",{1000 * i},{1000 * i + d}\n')
    out = bench.summarize_diffusion_counters(str(tmp_path))
    # fetch is scaled by 2 (the copy reads half its bytes), write by 1
    total = (1000.0 + 300.0) * 1024.0 * 2.0 + (500.0 + 100.0) * 1024.0
    gbs = total / ((1000 + 3000) * 1e-9) / 1e9
    assert out.splitlines()[0] == f"measured_gbs: {gbs:.1f}"
    assert "`cmg::k_a<1>` | 1 |" in out and "at::native" not in out


def test_stall_summary_takes_the_finest_level_of_the_measured_solve(tmp_path):
    # dispatches 1-2: warm-up solve; 3-4: measured solve; the 32-bit
    # container (a coarser level) and other libraries' kernels are left out
    up16 = "void cmg::k_up_smooth<4, 32, 768, 6, false, 16>(float const*)"
    up32 = "void cmg::k_up_smooth<4, 32, 768, 6, false, 32>(float const*)"
    sa = {"SQ_WAVE_CYCLES": 1000.0, "SQ_ACTIVE_INST_ANY": 400.0, "SQ_WAIT_ANY": 350.0, "SQ_WAIT_INST_ANY": 250.0,
          "SQ_ACTIVE_INST_VALU": 200.0, "SQ_ACTIVE_INST_LDS": 30.0}
    sb = {"SQ_ACTIVE_INST_SCA": 150.0, "SQ_LDS_BANK_CONFLICT": 60.0}
    for pas, vals in (("sa", sa), ("sb", sb)):
        with open(tmp_path / f"{pas}_counter_collection.csv", "w") as fh:
            fh.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
            for i, name in ((1, up16), (2, up32), (3, up16), (4, up32), (5, "void at::native::k(int)")):
                for c, v in vals.items():
                    fh.write(f'{i},"{name}",{c},{v * (1 if i < 3 else 2)}\n')
    out = bench.summarize_stalls(str(tmp_path), 10, 16).splitlines()
    assert len(out) == 3 and out[2].startswith("| `k_up_smooth<4>@10` | 1 | 2.0000e+03 |")
    assert out[2].endswith("| 0.400 | 0.350 | 0.250 | 0.200 | 0.150 | 0.030 | 0.060 |")
