"""Build libdd.so (HIP, gfx950) in-tree.

    python -m paper_2005_02498_amd.build          # compile every source
    python -m paper_2005_02498_amd.build --isa    # also keep the AMD assembly

Each csrc/*.hip is compiled with hipcc for gfx950 and each csrc/*.cpp (host-only
planning code) with the host C++ compiler into _build/, then linked into
paper_2005_02498_amd/libdd.so.  Packed FP32 instructions are disabled for all
device code (-packed-fp32-ops); the host pass prints a harmless warning that it
does not know that feature.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libdd.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
CXX = os.environ.get("CXX", shutil.which("g++") or "g++")
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
# Per-source additions.  dd_mlp.hip: MFMA results in architectural VGPRs
# (not accumulation registers), so that the epilogues convert accumulators
# without a register move per element; the weights then take the
# accumulation registers as MFMA A operands.
EXTRA = {
    "dd_mlp.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def _compile(src: str, isa: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if src.endswith(".cpp"):
        cmd = [CXX, "-O2", "-fPIC", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               "-c", src, "-o", obj]
    else:
        cmd = [HIPCC, *CFLAGS, *EXTRA.get(os.path.basename(src), []), "-c", src, "-o", obj]
        if isa:
            cmd += ["-save-temps=obj"]
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=BUILD)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{msgs}")
    if msgs.strip():
        print(msgs, file=sys.stderr)
    return obj


def build(isa: bool = False, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, isa), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    # roctx ranges of the host runtime (rocprofv3 --marker-trace)
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-L", "/opt/rocm/lib",
           "-lrocprofiler-sdk-roctx", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources")
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--isa", action="store_true")
    a = ap.parse_args()
    build(isa=a.isa)
