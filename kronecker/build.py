"""Build step for the seeded Kronecker input generator.

Produces ``libkron_host.so`` (gcc, OpenMP) and ``libkron_dev.so`` (hipcc,
gfx950) next to this file.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    subprocess.run(cmd, check=True, cwd=HERE)


def build(verbose=False):
    host_out = os.path.join(HERE, "libkron_host.so")
    dev_out = os.path.join(HERE, "libkron_dev.so")
    _run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
          "-o", host_out + ".tmp", "kron_host.c"])
    os.replace(host_out + ".tmp", host_out)
    _run(["hipcc"] + HIP_FLAGS + ["-o", dev_out + ".tmp", "kron_dev.hip"])
    os.replace(dev_out + ".tmp", dev_out)
    if verbose:
        print("built", host_out, dev_out)


if __name__ == "__main__":
    build(verbose=True)
