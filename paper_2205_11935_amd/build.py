"""Build libcryptotl.so in-tree for gfx950 with hipcc (runs on a CPU-only host too)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcryptotl.so")
SOURCES = ["host_math.cpp", "api.cpp", "kernels.hip"]
HEADERS = ["ctl_internal.h", "kernels.h"]
ARCH = os.environ.get("CTL_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall",
    # the exact FP64 modular products rely on separately rounded multiplies: no contraction
    "-ffp-contract=off",
    # keep the compiler from forming packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(HERE, "..", "include"),
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    # hipcc's host pass warns that it does not know the packed-fp32 feature; drop that noise
    noise = [ln for ln in r.stderr.splitlines() if ln.strip() and "packed-fp32-ops" not in ln]
    if noise:
        sys.stderr.write("\n".join(noise) + "\n")


def build(force: bool = True) -> str:
    """Compile every source for gfx950 and link the shared library. Returns its path."""
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS] + [os.path.join(HERE, "..", "include", "ctl.h")]
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(os.path.getmtime(d) for d in deps):
        return LIB
    os.makedirs(OUT_DIR, exist_ok=True)
    objs = []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(OUT_DIR, os.path.splitext(s)[0] + ".o")
        lang = ["-x", "hip"] if s.endswith(".hip") else []
        _run([HIPCC, "--offload-arch=" + ARCH] + COMMON + lang + ["-c", src, "-o", obj])
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


# AddressSanitizer + UndefinedBehaviorSanitizer on the host code only (the GPU code object is the
# ordinary one): each sanitizer flag goes to the host compilation through -Xarch_host.
SAN_FLAGS = ["-g", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined"]


def sanitizer_runtime() -> str:
    """The compiler's shared AddressSanitizer runtime (it carries the UndefinedBehaviorSanitizer
    handlers too); a process that loads a sanitized library must preload it."""
    import glob
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise RuntimeError("no AddressSanitizer runtime found under /opt/rocm/llvm")
    return found[-1]


def build_sanitized(out_dir: str) -> str:
    """The library with its host sources built under the sanitizers, as out_dir/libcryptotl.so
    (the kernels' object is reused from the ordinary build). Returns its path."""
    kobj = os.path.join(OUT_DIR, "kernels.o")
    if not os.path.exists(kobj):
        build(force=True)
    os.makedirs(out_dir, exist_ok=True)
    objs = []
    for s in SOURCES:
        if s.endswith(".hip"):
            objs.append(kobj)
            continue
        obj = os.path.join(out_dir, os.path.splitext(s)[0] + ".o")
        _run([HIPCC] + COMMON + SAN_FLAGS + ["-c", os.path.join(CSRC, s), "-o", obj])
        objs.append(obj)
    lib = os.path.join(out_dir, "libcryptotl.so")
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", lib] + objs)
    return lib


if __name__ == "__main__":
    print(build(force="--lazy" not in sys.argv))
