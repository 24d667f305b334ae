"""Build the HIP library libp2s.so (gfx950) in-tree.

Usage: python -m paper_1703_09619_amd.build  (or call build()).
"""
from __future__ import annotations

import os
import hashlib
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

HIP_SOURCES = ["p2s_api.hip", "p2s_kernels.hip", "p2s_contract.hip", "p2s_direct.hip", "p2s_direct_sf.hip",
               "p2s_learned.hip", "p2s_split.hip", "p2s_cheb2d.hip",
               "p2s_contract_packed.hip"]
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


def _headers_digest() -> str:
    h = hashlib.sha256()
    for d in (CSRC, INCLUDE):
        for f in sorted(os.listdir(d)):
            if f.endswith(".h"):
                h.update(f.encode())
                h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source and link libp2s.so.  With incremental=True
    (development use) an object whose source, headers and flags are
    unchanged since the last incremental build is reused from _build/."""
    hipcc = _hipcc()
    tmpdir = tempfile.mkdtemp(prefix="p2s_build_")
    cache = os.path.join(ROOT, "_build")
    hdr = _headers_digest() if incremental else ""
    objs = []
    cmds = []
    for src, cmd0 in [(x, [hipcc, "-x", "hip", "-c"]) for x in HIP_SOURCES] + [(x, ["g++", "-c"]) for x in CXX_SOURCES]:
        flags = common_flags() + (hip_flags() if cmd0[0] == hipcc else [])
        obj = os.path.join(tmpdir, src + ".o")
        cmd = cmd0 + [os.path.join(CSRC, src), "-o", obj] + flags
        if incremental:
            key = hashlib.sha256((hdr + " ".join(cmd0 + flags)).encode() +
                                 open(os.path.join(CSRC, src), "rb").read()).hexdigest()[:20]
            cached = os.path.join(cache, "%s.%s.o" % (src, key))
            if os.path.exists(cached):
                objs.append(cached)
                continue
            os.makedirs(cache, exist_ok=True)
            cmd[cmd.index(obj)] = cached
            obj = cached
        cmds.append(cmd)
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

    if cmds:
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            list(ex.map(run, cmds))
    tmp_lib = LIB + ".tmp%d" % os.getpid()
    run([hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp_lib] + objs)
    os.replace(tmp_lib, LIB)
    shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
