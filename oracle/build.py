"""Compile the CPU oracle (plain C, FP64) into oracle/liboracle.so.

Test infrastructure only: the product library never links or loads it.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "jfnk_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")


# AddressSanitizer + UndefinedBehaviorSanitizer build of the same source (a
# host-only library: the oracle has no GPU code), for the sanitizer run of
# the oracle's pins
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                  "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, out: str = OUT, sanitize: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", "-Wall", *(SANITIZE_FLAGS if sanitize else []),
           "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
