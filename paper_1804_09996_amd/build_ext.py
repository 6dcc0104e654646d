"""Compile the native libraries of the package in-tree.

* ``liblc.so``       — the HIP kernels and the C-ABI declared in include/lc.h
                       (hipcc, gfx950).
* ``liblc_build.so`` — the host-side index builder declared in
                       include/lc_build.h (g++, no GPU code).
"""
import hashlib
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")

HIP_SOURCES = ["lc_capi.hip", "lc_lut.hip", "lc_walk.hip", "lc_refine.hip", "lc_assign.hip", "lc_noalloc.hip",
               "lc_graph.hip"]
BUILD_SOURCES = ["lc_builder.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("LC_OFFLOAD_ARCH", "gfx950")


def source_id() -> str:
    """sha1 over the sources liblc.so is built from (include/lc.h and every
    file under csrc/ except the host builder), in name order."""
    h = hashlib.sha1()
    files = [os.path.join(INCLUDE, "lc.h")] + sorted(
        os.path.join(CSRC, f) for f in os.listdir(CSRC)
        if f.endswith((".hip", ".h")) and f not in BUILD_SOURCES)
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_hip(verbose: bool = False, jobs: int = 4) -> str:
    out = os.path.join(PKG, "liblc.so")
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = [HIPCC, "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", INCLUDE, "-I", CSRC, f'-DLC_SOURCE_ID="{source_id()}"']
    objs, procs = [], []
    for src in HIP_SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = common + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        if len(procs) >= jobs:
            if procs.pop(0).wait() != 0:
                raise RuntimeError("hipcc failed")
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = out + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, out)
    return out


def build_host(verbose: bool = False) -> str:
    out = os.path.join(PKG, "liblc_build.so")
    tmp = out + ".tmp"
    _run(["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra",
          "-I", INCLUDE, *[os.path.join(CSRC, s) for s in BUILD_SOURCES], "-o", tmp], verbose)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> None:
    build_hip(verbose)
    if all(os.path.exists(os.path.join(CSRC, s)) for s in BUILD_SOURCES):
        build_host(verbose)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
