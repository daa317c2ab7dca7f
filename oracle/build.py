"""Build step for the CPU oracle (test infrastructure): gcc -> liboracle.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose=False):
    out = os.path.join(HERE, "liboracle.so")
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                    "-o", out + ".tmp", "oracle.c"], check=True, cwd=HERE)
    os.replace(out + ".tmp", out)
    if verbose:
        print("built", out)


if __name__ == "__main__":
    build(verbose=True)
