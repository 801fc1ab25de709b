"""The propagation's split of a workgroup's products over its waves
(paper_1703_01545_amd/csrc/roles.h), checked on the host: a program built
from the same header asserts that every (row block, column block) has one
owner, that no SIMD gains products, and the balance at M = 200."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1703_01545_amd", "csrc")


def test_wave_roles_partition_the_products(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "roles_check")
    subprocess.run([hipcc, "--cuda-host-only", "-O1", "-std=c++17", "-I", CSRC,
                    os.path.join(HERE, "roles_check.hip"), "-o", exe],
                   check=True, capture_output=True, timeout=300)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "ok"
