"""Build the oracle shared library with gcc (plain C, FP64, no FMA contraction).

Test infrastructure only: the oracle is the parity reference for the HIP path.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["orc_field.c", "orc_particles.c", "orc_sim.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(force=True):
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(p) for p in srcs + [os.path.join(HERE, "oracle.h"),
                                                         os.path.join(HERE, "orc_internal.h")])
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-variable", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
