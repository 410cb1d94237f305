"""Compile the C oracle into oracle/liboracle.so (plain -O2, no fast-math,
no floating-point contraction) and, for the all-cores CPU timing only,
oracle/liboracle_omp.so: the same source with -fopenmp, whose cell loops run
on several threads with unchanged arithmetic (reductions stay serial)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "jfnk_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")
OUT_OMP = os.path.join(HERE, "liboracle_omp.so")


def _compile(out, extra):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math"] + extra + ["-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)


def build(force=True):
    for out, extra in ((OUT, []), (OUT_OMP, ["-fopenmp"])):
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
            continue
        _compile(out, extra)
    return OUT


if __name__ == "__main__":
    print(build(force="--lazy" not in sys.argv))
