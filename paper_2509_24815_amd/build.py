"""Compile libseismic.so for gfx950 in-tree (hipcc for HIP sources, g++ for
host-only sources)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libseismic.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("SEISMIC_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             # packed fp32 instructions stay off: ordinary float code only
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]
CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def _sources():
    hip = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    cpp = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
    return hip, cpp


def _compile(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r.stderr


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hip, cpp = _sources()
    cmds, objs = [], []
    for f in hip:
        o = os.path.join(BUILD, f + ".o")
        cmds.append(["hipcc", *HIP_FLAGS, "-c", os.path.join(CSRC, f), "-o", o])
        objs.append(o)
    for f in cpp:
        o = os.path.join(BUILD, f + ".o")
        cmds.append(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, f), "-o", o])
        objs.append(o)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(cmds))) as ex:
        for cmd, err in zip(cmds, ex.map(_compile, cmds)):
            if verbose:
                print(" ".join(cmd), flush=True)
            if verbose and err.strip():
                print(err, flush=True)
    tmp = OUT + ".tmp"
    _compile(["hipcc", "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-pthread"])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
