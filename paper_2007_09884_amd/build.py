"""Build libopmm.so for gfx950 with hipcc (in-tree, no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRCS = [os.path.join(PKG, "csrc", n) for n in ("opmm.hip", "surrogate.hip", "serve.hip", "nm.hip", "ivt.hip", "polish.hip")]
DEPS = SRCS + [os.path.join(PKG, "csrc", n) for n in ("plant.hpp", "runtime.hpp")] + \
    [os.path.join(ROOT, "include", "opmm.h")]
LIB = os.path.join(PKG, "libopmm.so")
ARCH = os.environ.get("OPMM_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off", "-Wall", "-Wno-unused-result",
    "-I" + os.path.join(ROOT, "include"),
]



def san_lib(checks: str) -> str:
    """The host-sanitized library's path: libopmm_host_asan.so when "address" is among the checks
    (with UBSan beside it, as requested), libopmm_host_ubsan.so otherwise."""
    return os.path.join(PKG, "libopmm_host_%s.so" % ("asan" if "address" in checks.split(",") else "ubsan"))


def sanitizer_flags(checks: str) -> list:
    """Host-pass-only sanitizer flags (the device code is built exactly as in the product library).
    The sanitizer runtime is clang's shared one; a process that loads this library with "address"
    among the checks must start with that runtime preloaded."""
    out = []
    for c in checks.split(","):
        out += ["-Xarch_host", "-fsanitize=" + c]
    out += ["-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-g", "-shared-libsan"]
    return out


def sanitizer_runtime(name: str) -> str:
    """Path of clang's shared sanitizer runtime (name: "asan" or "ubsan_standalone")."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc)), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    return subprocess.check_output([clang, "-print-file-name=libclang_rt.%s-x86_64.so" % name],
                                   text=True).strip()


def build(verbose: bool = False, sanitize: str = "") -> str:
    """sanitize: comma-separated host sanitizers ("address,undefined", "undefined"); builds san_lib()
    instead of the product library, with the runtime's folder on its run path."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out = san_lib(sanitize) if sanitize else LIB
    tmp = out + ".tmp%d" % os.getpid()
    extra = []
    if sanitize:
        rt = os.path.dirname(sanitizer_runtime("ubsan_standalone"))
        extra = sanitizer_flags(sanitize) + ["-Wl,-rpath," + rt]
    cmd = [hipcc] + HIPCC_FLAGS + extra + SRCS + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    san = [a.split("=", 1)[1] for a in sys.argv[1:] if a.startswith("--sanitize=")]
    print(build(verbose="-v" in sys.argv, sanitize=san[0] if san else ""))
