"""Builds the HIP library libpercis.so for gfx950, in-tree.

    python -m paper_2509_11454_amd.build

build(sanitize=True, out=PATH) builds a copy whose host code carries
AddressSanitizer and UndefinedBehaviorSanitizer checks (device code is built
as usual); a process that loads it must preload clang's ASan runtime.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libpercis.so")
SOURCES = ["percis_kernels.hip", "percis_exact.hip", "percis_setup.hip", "percis_noalloc.hip", "percis_api.cpp",
           "percis_server.cpp"]
ARCH = os.environ.get("PERCIS_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # keep packed fp32 instructions out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    raise RuntimeError("hipcc not found")


# host-only sanitizer flags: each -fsanitize= is passed to the host compile
# and link only
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def build(verbose=False, sanitize=False, out=None):
    lib = out or LIB
    objdir = os.path.dirname(lib)
    os.makedirs(objdir, exist_ok=True)
    extra = SANITIZE_FLAGS if sanitize else []
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        cmd = [hipcc()] + HIPCC_FLAGS + extra + ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
        if src.endswith(".cpp"):
            cmd += ["-x", "hip"]
        cmd += ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC"] + extra + ["-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
