"""The separable transform's pass schedule (host code) emulated on the CPU:
compiles tests/native/transform_schedule_check.cpp against the library's
schedule header and runs it (bounds, write coverage and values against the
per-entry definition on 299 random tensors)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_transform_schedule_on_the_cpu(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs a host C++ compiler and the ROCm headers")
    exe = str(tmp_path / "check")
    src = os.path.join(HERE, "native", "transform_schedule_check.cpp")
    r = subprocess.run([cxx, "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
                        "-I", os.path.join(ROOT, "include"), "-o", exe, src], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok ")
