"""The state-register layout of the HIP kernels, checked on the host.

`tests/layout_check.hip` includes the kernels' header and checks, for several
register sizes, that the layout helpers map every (component, node) pair of a
register to its own entry, fill the register exactly, and keep a field's
components at a node adjacent.  It is built for the host only (hipcc
--offload-host-only) and run here; no GPU is involved.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1504_08340_amd", "csrc")


def test_register_layout_is_a_bijection_with_adjacent_fields(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "layout_check"
    subprocess.run([hipcc, "--offload-host-only", "-std=c++17", "-I", CSRC, "-I", os.path.join(HERE, "..", "include"),
                    os.path.join(HERE, "layout_check.hip"), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "layout ok" in out.stdout
