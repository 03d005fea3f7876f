"""The kernels' launch geometry checked on the CPU: tests/geometry_check.cpp
walks every workgroup and lane of each kernel's launch through the index
functions the kernels use (csrc/dsgm_geom.h) and the batch planner's host
image (dsgm::plan_image, called in libdsgm.so), for many shapes, and checks
that every access stays inside the buffer the library's size rules give and
that every pixel, block and lane group is owned exactly once.  The checker is
built with AddressSanitizer and UndefinedBehaviorSanitizer on its host pass,
so an overflow in the index arithmetic itself fails the run too."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
LIB = os.path.join(ROOT, "paper_1702_05156_amd", "libdsgm.so")


def test_every_kernel_access_stays_inside_its_buffer(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc / clang++ not available")
    if not os.path.exists(LIB):
        pytest.skip("libdsgm.so is not built")
    obj = tmp_path / "geometry_check.o"
    exe = tmp_path / "geometry_check"
    b = subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
                        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                        "-Xarch_host", "-fno-sanitize-recover=all",
                        "-I" + os.path.join(ROOT, "include"),
                        "-I" + os.path.join(ROOT, "paper_1702_05156_amd", "csrc"),
                        "-c", os.path.join(ROOT, "tests", "geometry_check.cpp"), "-o", str(obj)],
                       capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    b = subprocess.run([CLANG, "-fsanitize=address,undefined", "-o", str(exe), str(obj), LIB,
                        "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib",
                        "-Wl,-rpath," + os.path.dirname(LIB)], capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, HIP_VISIBLE_DEVICES="-1", ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.stdout[-3000:], r.stderr[-3000:])
