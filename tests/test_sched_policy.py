"""CPU unit test of the query server's admission policy (continuous batching)
(``csrc/gr_sched.h``) with injected query sizes."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_slot_admission_policy(tmp_path):
    exe = tmp_path / "sched_policy_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", os.path.join(ROOT, "paper_2212_08200_amd", "csrc"),
                    os.path.join(ROOT, "tests", "sched_policy_test.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"
