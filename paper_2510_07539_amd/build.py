"""Build the gfx950 HIP library libhsgn.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "hsgn.hip")
# the persistent window kernels, built on their own without machine-level
# loop-invariant code motion (it hoists per-window values out of the window
# loop and spills registers)
SRC_PERSIST = os.path.join(HERE, "csrc", "hsgn_persist.hip")
PERSIST_FLAGS = ["-mllvm", "-disable-machine-licm"]
DEPS = [os.path.join(HERE, "csrc", f) for f in sorted(os.listdir(os.path.join(HERE, "csrc")))
        if f.endswith((".hip", ".hpp"))] + [os.path.join(ROOT, "include", "hsgn.h")]
LIB = os.path.join(HERE, "libhsgn.so")

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere (the path is FP64; this keeps the
    # compiler from emitting v_pk_*_f32 in helper code)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-value",
]


# roctx ranges and marks of the entry points (rocprofv3 --marker-trace)
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
LINK_FLAGS = ["-L" + os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx"]


def build(verbose: bool = False) -> str:
    """Compile libhsgn.so (always recompiles)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    obj = tmp + ".persist.o"
    inc = "-I" + os.path.join(ROOT, "include")
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    cmds = [["hipcc", *flags, *PERSIST_FLAGS, inc, "-c", SRC_PERSIST, "-o", obj],
            ["hipcc", *HIPCC_FLAGS, inc, SRC, "-x", "none", obj, *LINK_FLAGS, "-o", tmp]]
    try:
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)
    finally:
        if os.path.exists(obj):
            os.remove(obj)
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
