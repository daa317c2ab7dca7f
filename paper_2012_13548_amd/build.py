"""Build step for libg5.so: every HIP source of csrc/ compiled for gfx950; and
libg5alg3.so, the host experiment (the paper's parallel level-synchronous BFS
with OpenMP, for its thread-count speedup curve), compiled with gcc.

Run ``python -m paper_2012_13548_amd.build`` or call :func:`build`.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["api.cpp", "csr_build.hip", "bfs.hip", "msbfs.hip", "work.hip", "noalloc.hip", "sssp.hip"]
LIB = os.path.join(HERE, "libg5.so")
ALG3_LIB = os.path.join(HERE, "libg5alg3.so")
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose=False, jobs=8):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = ["hipcc"] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out = p.communicate()[0].decode()
        out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(out + "\n")
        elif verbose and out.strip():
            print(out)
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    subprocess.run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs,
                   check=True)
    os.replace(LIB + ".tmp", LIB)
    subprocess.run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                    "-I", os.path.join(ROOT, "include"), "-o", ALG3_LIB + ".tmp",
                    os.path.join(CSRC, "alg3_host.c")], check=True)
    os.replace(ALG3_LIB + ".tmp", ALG3_LIB)
    if verbose:
        print("built", LIB, ALG3_LIB)


if __name__ == "__main__":
    build(verbose=True)
