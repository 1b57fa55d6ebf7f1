"""Build the FP64 CPU oracle (test infrastructure only) with gcc.

Produces ``oracle/liborc.so``: the oracle's own functions (orc_*) and, from
orc_abi.c, the library's calling interface served by the oracle (lbm_*).  The
oracle is plain C with OpenMP pragmas on the lattice loops; reductions stay
serial so results do not depend on the thread count.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["orc_mesh.c", "orc_sim.c", "orc_abi.c"]
LIB = os.path.join(HERE, "liborc.so")


def build(verbose=False):
    # -Bsymbolic: the interface functions of orc_abi.c bind to this library
    # even in a process that has also loaded the HIP library, which exports
    # the same names
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-Wall", "-Wno-unused-function", "-Wl,-Bsymbolic",
           "-o", LIB + ".tmp"] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
