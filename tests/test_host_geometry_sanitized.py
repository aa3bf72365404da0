"""The kernels' exact geometry (host build of the device header) under UndefinedBehaviorSanitizer
and AddressSanitizer, over the whole lattice range the kernels accept: coordinates in
[-2^23, 2^24], voxel sizes 2^3..2^20 lattice units, vertices on voxel planes, voxels at the
grid's edge.  A signed overflow, an invalid shift or an out-of-bounds access aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_geometry_has_no_undefined_behaviour(tmp_path):
    cxx = shutil.which("g++")
    inc = "/opt/rocm/include"
    if cxx is None or not os.path.isdir(inc):
        pytest.skip("needs g++ and the HIP headers")
    exe = tmp_path / "geom_ub"
    flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    subprocess.run([cxx, "-O1", "-g", "-std=c++17", *flags, "-D__HIP_PLATFORM_AMD__", f"-I{inc}",
                    f"-I{ROOT}/paper_2604_13191_amd/csrc", f"-I{ROOT}/include",
                    os.path.join(ROOT, "tests", "host_geom_ub.cpp"), "-o", str(exe)], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    for seed in (1, 2):
        p = subprocess.run([str(exe), str(seed), "60000"], capture_output=True, text=True, env=env, timeout=600)
        assert p.returncode == 0 and p.stdout.startswith("ok"), p.stderr[-3000:]
