"""Host logic of the Gram tiling, checked on the CPU: `tests/host/gram_tiling_check.cpp`
includes the kernel source, is built with hipcc (no kernel is launched) and checks
that every output block of every Gram product is computed exactly once by a tile
whose staged columns hold both operands, and that the tile plans of the C4 shapes
stay within the per-workgroup limits of the FP64 and FP32 kernels."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_gram_tiling_covers_every_block_once():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = os.path.join(HERE, "host", "gram_tiling_check.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "gram_tiling_check")
        r = subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-w",
                            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", src, "-o", exe],
                           capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        print(r.stdout)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "each exactly once" in r.stdout
