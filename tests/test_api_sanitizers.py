"""The host side of libdsgm.so under AddressSanitizer (with leak detection) and
UndefinedBehaviorSanitizer: dsgm_api.hip -- every entry point's argument
validation, the batch planner's layout and LPT ordering, the tuner's table,
the status strings -- is compiled with the sanitizers on its host pass only
(the device pass stays as in the product), linked ahead of the product
library so that its instrumented entry points are the ones called, and driven
by tests/sanitize_api_driver.cpp on the CPU (no GPU: calls that pass
validation stop at their first HIP call).  Any out-of-bounds access, use after
free, leak or undefined operation fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
LIB = os.path.join(ROOT, "paper_1702_05156_amd", "libdsgm.so")

# the sanitizers go to the host compilation only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
COMMON = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
          "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"),
          "-I" + os.path.join(ROOT, "paper_1702_05156_amd", "csrc")]


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, **kw)


def test_host_library_is_clean_under_asan_and_ubsan(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc / clang++ not available")
    if not os.path.exists(LIB):
        pytest.skip("libdsgm.so is not built")
    api = tmp_path / "api.o"
    drv = tmp_path / "drv.o"
    exe = tmp_path / "api_san"
    for src, obj in ((os.path.join(ROOT, "paper_1702_05156_amd", "csrc", "dsgm_api.hip"), api),
                     (os.path.join(ROOT, "tests", "sanitize_api_driver.cpp"), drv)):
        b = _run([HIPCC] + COMMON + HOST_SAN + ["-c", src, "-o", str(obj)])
        assert b.returncode == 0, b.stderr[-3000:]
    link = [CLANG, "-fsanitize=address,undefined", "-o", str(exe), str(drv), str(api), LIB,
            "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib",
            "-Wl,-rpath," + os.path.dirname(LIB)]
    b = _run(link)
    assert b.returncode == 0, b.stderr[-3000:]
    # no device may be used: the run must not depend on one being there
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", HIP_VISIBLE_DEVICES="-1")
    r = _run([str(exe)], timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout[-2000:], r.stderr[-4000:])
    # the instrumentation is really there: the host object calls the ASan runtime
    nm = shutil.which("nm")
    if nm:
        syms = _run([nm, str(api)]).stdout
        assert "__asan_" in syms and "__ubsan_" in syms
