"""Build the CPU harnesses of tests/host with hipcc: adjoint_host.hip (the
adjoint's per-cell bodies in host loops) and device_host.hip (the forward
sweep's per-state arithmetic).  Rebuilt when a source or header is newer."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1210_5246_amd", "csrc")
LIB = os.path.join(HERE, "libadjhost.so")
SRC = os.path.join(HERE, "adjoint_host.hip")
DEV_LIB = os.path.join(HERE, "libdevhost.so")
DEV_SRC = os.path.join(HERE, "device_host.hip")


# CSH_HOST_SANITIZE=1: build the harnesses' host code with AddressSanitizer
# and UndefinedBehaviorSanitizer (a separate library; the process that loads
# it preloads clang's ASan runtime, which carries the UBSan handlers too)
SANITIZE = os.environ.get("CSH_HOST_SANITIZE") == "1"
SAN_FLAGS = ["-g", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all"]


def _build(src: str, lib: str, headers) -> str:
    if SANITIZE:
        lib = lib.replace(".so", "_san.so")
    deps = [src] + [os.path.join(CSRC, f) for f in headers]
    if os.path.exists(lib) and os.path.getmtime(lib) >= max(os.path.getmtime(d) for d in deps):
        return lib
    tmp = lib + f".tmp{os.getpid()}"
    cmd = ["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
           "-ffp-contract=off", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *(SAN_FLAGS if SANITIZE else []),
           src, "-o", tmp]
    subprocess.run(cmd, check=True, capture_output=True)
    os.replace(tmp, lib)
    return lib


def build() -> str:
    return _build(SRC, LIB, ("csh_adjoint.h", "csh_device.h"))


def build_device() -> str:
    return _build(DEV_SRC, DEV_LIB, ("csh_device.h", "csh3_device.h"))
