"""Host check of the random-number helpers shared by the GPU kernels: the
bytewise (SWAR) prefix test and slot-range mask equal a plain per-slot loop on
2,000,000 random cases, including the cut values 0 and 255."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_prefix_pass_mask_matches_loop(tmp_path):
    exe = tmp_path / "rng_prefix_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2103_02202_amd", "csrc"),
                    os.path.join(ROOT, "tests", "rng_prefix_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    assert "bad 0" in out.stdout
