"""Host-sanitized build of the library for the CPU tests.

The host code of the C ABI (plan.cpp: validation, block maps, workspace
layout, launch sequencing; genasis.cpp: the mesh builder) is compiled with
AddressSanitizer and UndefinedBehaviorSanitizer on its host side only (each
sanitizer flag follows -Xarch_host, so no device code is instrumented) and
linked with the unchanged kernel objects of the normal build into
paper_2602_02507_amd/_lib/libmpole_hostsan.so.  Tests load it through
MPOLE_LIBRARY with the clang ASan runtime preloaded into the interpreter.
"""
import os
import subprocess

from paper_2602_02507_amd import build as hb

HOST_SOURCES = ("plan.cpp", "genasis.cpp")
LIB = os.path.join(hb.LIBDIR, "libmpole_hostsan.so")


def clang():
    return os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang++")


def asan_runtime():
    out = subprocess.check_output([clang(), "-print-file-name=libclang_rt.asan-x86_64.so"])
    return out.decode().strip()


def build():
    objdir = os.path.join(hb.LIBDIR, "obj")
    kernel_objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o") for s in hb.SOURCES
                   if s not in HOST_SOURCES]
    if not all(os.path.exists(o) for o in kernel_objs):
        hb.build()
    san = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
                 "-fno-omit-frame-pointer"):
        san += ["-Xarch_host", flag]
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + "_hostsan.o")
        cmd = [hb.hipcc(), "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=" + hb.ARCH] + san + \
              ["-I", os.path.join(hb.ROOT, "include"), "-x", "hip", "-c", os.path.join(hb.CSRC, src), "-o", obj]
        subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
        objs.append(obj)
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([clang(), "-shared", "-fsanitize=address,undefined", "-shared-libasan", "-o", tmp] + objs +
                          kernel_objs + ["-L", os.path.join(rocm, "lib"), "-lamdhip64",
                                         "-Wl,-rpath," + os.path.join(rocm, "lib")])
    os.replace(tmp, LIB)
    return LIB
