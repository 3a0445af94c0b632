"""Compile the gfx950 HIP libraries with hipcc: the multipole solver (C ABI of
include/mpole.h) into paper_2602_02507_amd/_lib/libmpole.so, and the device
input generator of the repeated-solve workload (include/mpole_workload.h)
into paper_2602_02507_amd/_lib/libmpole_workload.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libmpole.so")
SOURCES = ["plan.cpp", "tables.hip", "pack.hip", "gemm_f64.hip", "scan.hip", "split.hip", "gemm_split.hip",
           "gradient.hip", "separable.hip", "sep_bf16.hip", "coarsen.hip", "blocks.hip", "genasis.cpp",
           "persistent.hip"]
WL_LIB = os.path.join(LIBDIR, "libmpole_workload.so")
WL_SOURCES = ["rotated_density.hip"]
ARCH = "gfx950"


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose=False, jobs=8):
    os.makedirs(LIBDIR, exist_ok=True)
    objdir = os.path.join(LIBDIR, "obj")
    os.makedirs(objdir, exist_ok=True)
    flags = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-munsafe-fp-atomics",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]
    procs, objs = [], []
    for src in SOURCES + WL_SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc()] + flags + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        while len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[0][1].wait()
    failed = []
    for src, p in procs:
        out = p.communicate()[0].decode(errors="replace")
        lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(out)
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError("hipcc failed for " + ", ".join(failed))
    for lib, srcs in ((LIB, SOURCES), (WL_LIB, WL_SOURCES)):
        tmp = lib + ".tmp%d" % os.getpid()
        lobjs = [o for o, src in zip(objs, SOURCES + WL_SOURCES) if src in srcs]
        cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + lobjs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
