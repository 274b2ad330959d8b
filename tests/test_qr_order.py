"""Host check of the pivoted QR's column order (csrc/qr_order.h, used by the
panel selection and the in-panel pivot of k_qr.hip): ties, NaN, +-Inf,
signed zeros and denormals still give a permutation of ranks and a pivot
that does not depend on the reduction order.  Builds tests/qr_order_check.cpp
with the host compiler and runs it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_column_order_is_a_strict_total_order(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the HIP headers")
    exe = tmp_path / "qr_order_check"
    subprocess.run([cxx, "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I" + os.path.join(ROOT, "paper_1504_05090_amd", "csrc"),
                    os.path.join(ROOT, "tests", "qr_order_check.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout[-2000:]
