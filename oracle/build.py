"""Build step for the CPU oracle (test infrastructure).

Compiles ``kg_oracle.c`` into ``libkg_oracle.so`` next to it with the host C
compiler.  Only the test suite, the smoke check and the benchmark's CPU
baseline load the result.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kg_oracle.c")
LIB = os.path.join(HERE, "libkg_oracle.so")


def build_oracle(src=SRC, out=LIB, opt=("-O2",)):
    """Compile an oracle source file into a shared library at ``out``.  ``opt``
    are the optimisation flags: the default build is portable (it also runs
    on hosts other than the one that built it); the benchmark's CPU baseline
    builds its own copy with -O3 -march=native on the host it measures."""
    cmd = ["gcc", *opt, "-fopenmp", "-shared", "-fPIC", "-std=gnu11", "-Wall", src, "-o",
           out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build_oracle())
