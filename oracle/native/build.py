"""Compile the oracle's plain C helpers (test infrastructure only) next to this file.

    python -m oracle.native.build

-O2 without fast-math, -ffp-contract=off (no fused operations the source does not
write), -mfma so that fmaf() is the processor's correctly rounded fused multiply-add.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = {"libdm_lu.so": ["dm_lu.c"]}


def build(verbose=False):
    out = []
    for lib, srcs in SOURCES.items():
        dst = os.path.join(HERE, lib)
        tmp = dst + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-mfma", "-fPIC", "-shared",
               "-o", tmp] + [os.path.join(HERE, s) for s in srcs] + ["-lm"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("oracle C build failed:\n%s\n%s" % (" ".join(cmd), r.stderr[-4000:]))
        os.replace(tmp, dst)
        out.append(dst)
        if verbose:
            print("built", dst)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
