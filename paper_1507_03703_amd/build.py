"""Build libbpmf.so (the HIP library) in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbpmf.so")
SOURCES = ["api.hip", "kernels.hip", "mbar.hip", "mlp.hip", "moves.hip",
           "protocol.hip", "pairs.hip"]
ARCH = os.environ.get("BPMF_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-DBPMF_BUILD", "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(CSRC, s.replace(".hip", ".o"))
        cmd = [hipcc, *[f for f in FLAGS if f != "-shared"], "-c", src, "-o",
               obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o",
           tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


# host code instrumented with AddressSanitizer and UndefinedBehaviorSanitizer
# (device code is compiled as usual); for checking the host-side validation
# and bookkeeping on the CPU, loaded through BPMF_LIB in a process that
# preloads clang's shared sanitizer runtime
SAN_LIB = os.path.join(HERE, "libbpmf_san.so")
SAN_HOST_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host",
                  "-fsanitize=undefined", "-Xarch_host",
                  "-fno-sanitize-recover=all", "-Xarch_host",
                  "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def build_sanitized(out: str = SAN_LIB) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(CSRC, s.replace(".hip", ".san.o"))
        cmd = [hipcc, *[f for f in FLAGS if f not in ("-shared", "-O3")],
               "-O1", *SAN_HOST_FLAGS, "-c", src, "-o", obj]
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = out + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o",
           tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
