"""Build the HIP library libp2s.so (gfx950) in-tree.

Usage: python -m paper_1703_09619_amd.build  (or call build()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libp2s.so")

HIP_SOURCES = ["p2s_api.hip", "p2s_kernels.hip", "p2s_contract.hip", "p2s_direct.hip", "p2s_learned.hip",
               "p2s_split.hip"]
CXX_SOURCES = ["p2s_tables.cpp"]
ARCH = "gfx950"


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC,
            "-Wall", "-Wno-unused-function", "-Wno-unused-result"]


def hip_flags():
    # no packed FP32 instructions in device code; FP64 contraction left to
    # the compiler (fma is called explicitly where it matters)
    return ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-munsafe-fp-atomics"]


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    tmpdir = tempfile.mkdtemp(prefix="p2s_build_")
    objs = []
    cmds = []
    for src in HIP_SOURCES:
        obj = os.path.join(tmpdir, src + ".o")
        cmds.append([hipcc, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + common_flags() + hip_flags())
        objs.append(obj)
    for src in CXX_SOURCES:
        obj = os.path.join(tmpdir, src + ".o")
        cmds.append(["g++", "-c", os.path.join(CSRC, src), "-o", obj] + common_flags())
        objs.append(obj)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        p = subprocess.run(cmd, capture_output=True, text=True)
        err = "\n".join(l for l in p.stderr.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), err))
        if err.strip() and verbose:
            print(err)

    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        list(ex.map(run, cmds))
    tmp_lib = LIB + ".tmp%d" % os.getpid()
    run([hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp_lib] + objs)
    os.replace(tmp_lib, LIB)
    shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
