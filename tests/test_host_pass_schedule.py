"""CPU test of the intra-pair pass scheduler of the GPU library (host code):
builds tests/cpp/pass_schedule_check.cpp against csrc/ligand_prep.cpp and
runs its invariant checks on 3,000 random pair lists."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return None


def test_pass_schedule_invariants(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "pass_schedule_check")
    csrc = os.path.join(ROOT, "paper_2510_24186_amd", "csrc")
    cmd = [hipcc, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(ROOT, "tests", "cpp", "pass_schedule_check.cpp"), os.path.join(csrc, "ligand_prep.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    bad, passes, minimal = [int(t) for t in r.stdout.split()[1::2][:3]]
    assert bad == 0
    # the balanced assignment stays within a few percent of ceil(P / width)
    assert passes <= 1.05 * minimal
