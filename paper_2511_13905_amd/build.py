"""Build the HIP library libpgdto.so for gfx950 in-tree (hipcc, no JIT cache)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpgdto.so")

SOURCES = ["pgdto_kernels.hip", "pgdto_wide.hip", "pgdto_host.cpp", "pgdto_serve.cpp", "pgdto_server.cpp", "pgdto_many.cpp"]

# Packed-FP32 instructions are disabled: hipcc -O3 forms them from float2
# code and some forms have given wrong results on these machines.
HIP_FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function"]


def hipcc() -> str:
    cand = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return cand


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer (device code is
# built as usual: every -fsanitize= applies to the host pass only).
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer",
                  "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=undefined"]
LIB_SAN = os.path.join(HERE, "libpgdto_san.so")


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime to preload into an uninstrumented python."""
    import glob
    root = os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))
    cands = sorted(glob.glob(os.path.join(root, "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so")))
    cands += sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return cands[-1] if cands else ""


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source and link libpgdto.so (sanitize: libpgdto_san.so
    with the host code instrumented, for the CPU test suite)."""
    objs = []
    bdir = os.path.join(HERE, "_build_san" if sanitize else "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(bdir, src + ".o")
        flags = [f for f in HIP_FLAGS if f != "-O3"] + SANITIZE_FLAGS if sanitize else HIP_FLAGS
        cmd = [hipcc(), *flags, "-x", "hip", "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    lib = LIB_SAN if sanitize else LIB
    tmp = lib + ".tmp"
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan"] if sanitize else []
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *san, *objs, "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def sanitized_tests() -> int:
    """The CPU test suite (-m "not gpu") against libpgdto_san.so, with the
    clang AddressSanitizer runtime preloaded into python (leak checks off:
    the interpreter itself keeps memory until exit)."""
    env = dict(os.environ)
    env["PGDTO_LIB"] = LIB_SAN
    env["LD_PRELOAD"] = asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    root = os.path.dirname(HERE)
    cmd = [sys.executable, "-m", "pytest", os.path.join(root, "tests"), "-q", "-m", "not gpu", "-p", "no:cacheprovider"]
    return subprocess.run(cmd, env=env, cwd=root).returncode


if __name__ == "__main__":
    san = "--sanitize" in sys.argv
    print(build(verbose="-v" in sys.argv, sanitize=san))
    if san and "--test" in sys.argv:
        sys.exit(sanitized_tests())
