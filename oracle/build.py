"""Build the FP64 CPU oracle (test infrastructure only) with g++ and OpenMP.

The oracle is compiled here so that the checker exists wherever the tests
run; building it is not using it.  Only tests/, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` load the resulting library.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dg_oracle.cpp")
LIB = os.path.join(HERE, "libdg_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
        "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC,
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
