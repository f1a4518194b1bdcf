"""Build the FP64 CPU oracle shared library (test infrastructure).

Plain gcc (with OpenMP for the optional row-parallel mode), no GPU code, no shared sources with the GPU library.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lb_oracle.c")
LIB = os.path.join(HERE, "liblb_oracle.so")


def build(force=True):
    """Compile lb_oracle.c into liblb_oracle.so next to it; returns the path."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    # -fopenmp: the optional row-parallel mode (orc_set_threads); one thread
    # by default
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-ffp-contract=off", "-fopenmp", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
