"""Build tests/sanitize/host_check: the library's host code (hsgn.hip and the
persistent-launch unit) with AddressSanitizer and UndefinedBehaviorSanitizer,
linked with the C ABI driver host_check.cpp.  The sanitizers instrument host
code only (every -fsanitize= sits behind -Xarch_host); the gfx950 device code
is the library's own.  Test infrastructure, run by tests/test_gpu_sanitize.py.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2510_07539_amd import build as B  # noqa: E402

EXE = os.path.join(HERE, "host_check")
DRIVER = os.path.join(HERE, "host_check.cpp")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
       "-Xarch_host", "-g"]


def build(verbose: bool = False) -> str:
    """Compile host_check (always recompiles)."""
    tmp = EXE + ".tmp%d" % os.getpid()
    obj = tmp + ".persist.o"
    inc = "-I" + os.path.join(ROOT, "include")
    flags = [f for f in B.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    cmds = [["hipcc", *flags, *SAN, *B.PERSIST_FLAGS, inc, "-c", B.SRC_PERSIST, "-o", obj],
            ["hipcc", *flags, *SAN, inc, DRIVER, B.SRC, "-x", "none", obj, *B.LINK_FLAGS, "-o", tmp]]
    try:
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)
    finally:
        if os.path.exists(obj):
            os.remove(obj)
    os.replace(tmp, EXE)
    return EXE


if __name__ == "__main__":
    print(build(verbose=True))
