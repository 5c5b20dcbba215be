"""Builds libparapn.so (HIP for gfx950) in-tree, next to this file.

    python -m paper_2310_01145_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libparapn.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc")
ARCH = "gfx950"
# packed FP32 instructions are disabled on purpose (see the design notes)
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC]

# translation units: the kernel file is compiled once per precision and once
# more per precision for the damped forward scan, so the parts build in
# parallel
UNITS = [
    ("scan_kernels_f32.o", "scan_kernels.hip", ["-DPARAPN_BUILD_FP32=1", "-DPARAPN_BUILD_FP64=0"]),
    ("scan_kernels_f64.o", "scan_kernels.hip", ["-DPARAPN_BUILD_FP32=0", "-DPARAPN_BUILD_FP64=1",
                                                "-DPARAPN_BUILD_HELPERS=0"]),
    # the damped (Levenberg-Marquardt) forward scan, per precision
    ("scan_kernels_f32_lm.o", "scan_kernels.hip", ["-DPARAPN_BUILD_FP32=1", "-DPARAPN_BUILD_FP64=0",
                                                   "-DPARAPN_BUILD_HELPERS=0", "-DPARAPN_BUILD_LM=1"]),
    ("scan_kernels_f64_lm.o", "scan_kernels.hip", ["-DPARAPN_BUILD_FP32=0", "-DPARAPN_BUILD_FP64=1",
                                                   "-DPARAPN_BUILD_HELPERS=0", "-DPARAPN_BUILD_LM=1"]),
    # the dense engine (large D)
    ("dense_kernels.o", "dense_kernels.hip", []),
    ("parapn_api.o", "parapn_api.cpp", ["-x", "hip"]),
]


def _compile(unit):
    obj, src, extra = unit
    out = os.path.join(OBJ, obj)
    cmd = [HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), r.stderr[-6000:]))
    return out


def build(verbose: bool = True) -> str:
    """Compile every HIP source for gfx950 and link libparapn.so (always rebuilds)."""
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(UNITS)) as ex:
        objs = list(ex.map(_compile, UNITS))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr[-4000:]))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def clean():
    shutil.rmtree(OBJ, ignore_errors=True)


if __name__ == "__main__":
    build()
