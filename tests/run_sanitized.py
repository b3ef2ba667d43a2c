"""Runs the CPU test suite (-m "not gpu": the oracle against its pins, the
host-side validation of the C ABI on host-only contexts, the workload
generators' callers) with the host code of libpercis.so and the oracle built
under AddressSanitizer and UndefinedBehaviorSanitizer.

    python tests/run_sanitized.py [extra pytest arguments]

Both libraries are built into _build/sanitize/ (the in-tree builds are left
alone) with clang, so one ASan runtime serves both; the Python process
preloads it. Leak checking is off: the interpreter and the HIP runtime keep
allocations until exit by design. Any ASan report or undefined-behaviour
trap ends the run with a non-zero status.
"""
import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitize")


def asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    hits += sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/x86_64-unknown-linux-gnu/libclang_rt.asan.so"))
    if not hits:
        raise RuntimeError("clang's ASan runtime was not found under /opt/rocm/llvm")
    return hits[-1]


def main(extra):
    sys.path.insert(0, ROOT)
    from oracle import oracle as O
    from paper_2509_11454_amd import build as B
    os.makedirs(OUT, exist_ok=True)
    lib = B.build(sanitize=True, out=os.path.join(OUT, "libpercis.so"))
    orc = O.build(sanitize=True, out=os.path.join(OUT, "liboracle.so"))
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": asan_runtime(),
        "ASAN_OPTIONS": "detect_leaks=0:verify_asan_link_order=0:abort_on_error=1:halt_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
        "PERCIS_LIB_PATH": lib,
        "PERCIS_ORACLE_LIB": orc,
    })
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-q", "-m", "not gpu", "-p", "no:xdist",
           "-p", "no:cacheprovider"] + extra
    print("sanitized run: %s" % " ".join(cmd), flush=True)
    return subprocess.call(cmd, env=env, cwd=ROOT)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
