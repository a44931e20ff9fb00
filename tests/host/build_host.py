"""Build the CPU adjoint harness (tests/host/adjoint_host.hip) with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
LIB = os.path.join(HERE, "libadjhost.so")
SRC = os.path.join(HERE, "adjoint_host.hip")


def build() -> str:
    deps = [SRC] + [os.path.join(ROOT, "paper_1210_5246_amd", "csrc", f) for f in ("csh_adjoint.h", "csh_device.h")]
    if os.path.exists(LIB) and os.path.getmtime(LIB) >= max(os.path.getmtime(d) for d in deps):
        return LIB
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
           "-ffp-contract=off", "-I", os.path.join(ROOT, "paper_1210_5246_amd", "csrc"),
           "-I", os.path.join(ROOT, "include"), "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           SRC, "-o", tmp]
    subprocess.run(cmd, check=True, capture_output=True)
    os.replace(tmp, LIB)
    return LIB
