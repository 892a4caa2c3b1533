"""Build libhk.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

    python -m paper_1503_03806_amd.build            # build
    python -m paper_1503_03806_amd.build --asm DIR  # also keep the AMD ISA

Every build compiles from scratch (the build step is the "does it compile"
check).  Packed FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhk.so")
SOURCES = ["hk_api.cpp", "line_prep.hip", "opacity_f64.hip", "opacity_f32.hip", "kdist.hip", "surrogate.hip", "resample.hip", "work_plan.hip", "line_sort.hip", "line_io.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def common_flags():
    # no implicit contraction: every fused multiply-add is an explicit fma(),
    # so a value's rounding does not depend on which code path computed it
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include")]


def build(asm_dir: str | None = None, verbose: bool = False) -> str:
    objs = []
    with tempfile.TemporaryDirectory(prefix="hkbuild") as tmp:
        for src in SOURCES:
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            cmd = [hipcc()] + common_flags() + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
            if asm_dir:
                os.makedirs(asm_dir, exist_ok=True)
                cmd += ["-save-temps=obj"]
                obj_asm = os.path.join(asm_dir, os.path.basename(obj))
                cmd[-1] = obj_asm
                obj = obj_asm
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)
            objs.append(obj)
        tmp_lib = LIB + ".tmp%d" % os.getpid()
        cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp_lib] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp_lib, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--asm", default=None, help="keep intermediate files (AMD ISA) here")
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.asm, a.v))


if __name__ == "__main__":
    sys.exit(main())
