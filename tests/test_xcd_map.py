"""The XCD-aware workgroup mappings, checked on the host: the walk kernel's
xcd_block (dtn_device.h), a bijection of [0, G) for every grid size up to
4096 and several large ones, runs of consecutive blocks per XCD, rounds
kept together; the treecode traversal's xcd_contiguous (dtn_xcd.h), a
bijection with each XCD's blocks taking one eighth of the range in order.
No GPU needed (hipcc builds the headers' host side)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def test_xcd_block_is_a_bijection_with_runs(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "xcd_map_check")
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                    os.path.join(HERE, "xcd_map_check.cpp"), "-o", exe], check=True, capture_output=True, timeout=300)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
