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


def build_oracle(src=SRC, out=LIB):
    """Compile an oracle source file into a shared library at ``out``."""
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11", "-Wall", src, "-o",
           out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build_oracle())
