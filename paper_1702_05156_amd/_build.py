"""Build libdsgm.so (and the synthetic-input library libsynth.so) for gfx950.

    python -m paper_1702_05156_amd._build

Every HIP source is compiled with hipcc for gfx950 only, with packed FP32
instructions disabled and no floating-point contraction (the FP64 path is
bit-exact by construction: every product and sum is rounded on its own).
The objects are linked into the package directory, where the binding loads
them from.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libdsgm.so")
SYNTH_SRCS = [os.path.join(ROOT, "synth", "synth.hip"), os.path.join(ROOT, "synth", "probe.hip")]
SYNTH_LIB = os.path.join(ROOT, "synth", "libsynth.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
          "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = (r.stdout + r.stderr).strip()
    # hipcc's host pass does not know the packed-fp32 feature and says so
    lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l and "is not a recognized feature" not in l]
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + "\n".join(lines))
    if verbose and lines:
        print("\n".join(lines), flush=True)


def _compile(src, obj, includes, verbose):
    _run([HIPCC] + COMMON + [f"-I{d}" for d in includes] + ["-c", src, "-o", obj], verbose)
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> list[str]:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = jobs or min(8, os.cpu_count() or 1)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, s, os.path.join(BUILD, os.path.basename(s) + ".o"),
                          [INCLUDE, CSRC], verbose) for s in srcs]
        sfuts = [ex.submit(_compile, s, os.path.join(BUILD, "synth_" + os.path.basename(s) + ".o"),
                           [os.path.join(ROOT, "synth")], verbose) for s in SYNTH_SRCS]
        objs = [f.result() for f in futs]
        synth_objs = [f.result() for f in sfuts]
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-o", LIB + ".tmp"] + objs, verbose)
    os.replace(LIB + ".tmp", LIB)
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-o", SYNTH_LIB + ".tmp"] + synth_objs, verbose)
    os.replace(SYNTH_LIB + ".tmp", SYNTH_LIB)
    return [LIB, SYNTH_LIB]


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
