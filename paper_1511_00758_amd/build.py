"""Builds libstereomesh.so in-tree for gfx950 (hipcc; the host-only triangulation with g++).

Usage: ``python -m paper_1511_00758_amd.build`` or ``build()`` from Python. Always
recompiles. Objects go to ``_build/`` at the repository root.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libstereomesh.so")
ARCH = os.environ.get("SM_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXX = os.environ.get("CXX", "g++")

COMMON = ["-O3", "-fPIC", "-std=c++17", f"-I{INCLUDE}", f"-I{CSRC}"]
HIP_FLAGS = COMMON + [f"--offload-arch={ARCH}", "-ffp-contract=off",
                      # packed FP32 instructions are kept out of every device build
                      "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = COMMON + ["-ffp-contract=off", "-Wall", "-Wextra"]

SOURCES = [
    ("kernels.hip", "hip"),
    ("api.cpp", "hip"),
    ("batch.cpp", "hip"),
    ("star.hip", "hip"),
    ("delaunay.cpp", "host"),
]


def _cmd(src, kind):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if kind == "hip":
        return [HIPCC] + HIP_FLAGS + ["-x", "hip", "-c", path, "-o", obj], obj
    return [CXX] + HOST_FLAGS + ["-c", path, "-o", obj], obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    procs, objs = [], []
    for src, kind in SOURCES:
        cmd, obj = _cmd(src, kind)
        objs.append(obj)
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    errors = []
    for src, cmd, pr in procs:
        out, _ = pr.communicate()
        text = out.decode(errors="replace")
        if pr.returncode != 0:
            errors.append(f"--- {src} ---\n{' '.join(cmd)}\n{text}")
        elif verbose and text.strip():
            print(text)
    if errors:
        raise RuntimeError("stereomesh build failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp"
    link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(link), flush=True)
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("stereomesh link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
