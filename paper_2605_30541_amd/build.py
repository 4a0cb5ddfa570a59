"""Build of the HIP library (libsgwave.so) for gfx950, in-tree."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libsgwave.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# packed FP32 instructions are kept out of the generated code
DEV_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp", ".h")))


def _headers_mtime() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    inc = os.path.join(ROOT, "include")
    hs += [os.path.join(inc, f) for f in os.listdir(inc) if f.endswith(".h")]
    return max(os.path.getmtime(h) for h in hs)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compiles every source (in parallel) and links the library.  With
    `incremental`, objects newer than their source and every header are
    kept."""
    os.makedirs(OUT_DIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs, procs = [], []
    hdr = _headers_mtime()
    for f in sorted(os.listdir(CSRC)):
        src = os.path.join(CSRC, f)
        if f.endswith(".hip"):
            flags = DEV_FLAGS
        elif f.endswith(".cpp"):
            flags = HOST_FLAGS
        else:
            continue
        obj = os.path.join(OUT_DIR, f + ".o")
        objs.append(obj)
        if incremental and os.path.exists(obj) and os.path.getmtime(obj) > max(os.path.getmtime(src), hdr):
            continue
        cmd = [HIPCC, "-c", *flags, *inc, src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
    for cmd, pr in procs:
        if pr.wait() != 0:
            raise subprocess.CalledProcessError(pr.returncode, cmd)
    # export only the C ABI (sg_*)
    vscript = os.path.join(OUT_DIR, "exports.map")
    with open(vscript, "w") as f:
        f.write("{ global: sg_*; local: *; };\n")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-Wl,--no-undefined",
           "-Wl,--version-script=" + vscript, *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build of the
# runtime (the C ABI's validation, table building and staging), for CPU test
# runs: each sanitizer flag is scoped to the host pass, the kernels are the
# regular objects.  Load it with SGWAVE_LIBRARY=<path> and the ASan runtime of
# sanitizer_runtime() in LD_PRELOAD.
SAN_DIR = os.path.join(OUT_DIR, "san")
SAN_LIB = os.path.join(SAN_DIR, "libsgwave.so")
SAN_FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def sanitizer_runtime() -> str | None:
    """The shared ASan runtime of the ROCm clang (None if absent)."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so") +
                  glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def build_sanitized(verbose: bool = False) -> str:
    """Builds SAN_LIB: the regular kernel objects (built if missing) with the
    host runtime compiled under ASan and UBSan."""
    build(verbose, incremental=True)
    os.makedirs(SAN_DIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    for f in sorted(os.listdir(CSRC)):
        if f.endswith(".hip"):
            objs.append(os.path.join(OUT_DIR, f + ".o"))
        elif f.endswith(".cpp"):
            obj = os.path.join(SAN_DIR, f + ".o")
            cmd = [HIPCC, "-c", *SAN_FLAGS, *inc, os.path.join(CSRC, f), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)
            objs.append(obj)
    tmp = SAN_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-shared-libsan",
           "-Wl,--version-script=" + os.path.join(OUT_DIR, "exports.map"), *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    import sys
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose=True))
    else:
        print(build(verbose=True, incremental="--incremental" in sys.argv))
