"""Build libsemisort_hip.so in-tree with hipcc for gfx950."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsemisort_hip.so")
SOURCES = [os.path.join(HERE, "csrc", "engine.hip"), os.path.join(HERE, "csrc", "server.hip")]
HEADERS = [os.path.join(HERE, "csrc", "ss_device.h"), os.path.join(HERE, "csrc", "user_fold.inc"),
           os.path.join(ROOT, "include", "semisort.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    "-shared",
    "-Wall",
    "-pthread",
    # packed FP32 instructions stay off (no float math here, but keep codegen plain)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", os.path.join(HERE, "csrc"),
    # run-time compilation of caller monoids
    "-L/opt/rocm/lib", "-lhiprtc",
]


def build(verbose=False, extra=()):
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + list(extra) + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
