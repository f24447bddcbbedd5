"""Build libltmp2.so for gfx950 with hipcc (in-tree, no JIT cache).

Every HIP translation unit is compiled with packed FP32 instructions
disabled; grid_kernels.hip is compiled once per supported grid size.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libltmp2.so")
GRIDS = (12, 15, 16, 18, 20, 24, 25, 27, 30, 32, 36, 40)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def _flags():
    grid_list = " ".join(f"X({n})" for n in GRIDS)
    return [
        f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++20",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
        f"-DLTMP2_GRID_LIST={grid_list}",
        "-I", os.path.join(HERE, "..", "include"),
    ]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops" not in l)
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{msg}")


def build(jobs: int | None = None, verbose: bool = False) -> str:
    if not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(BUILD, exist_ok=True)
    units = [("registry.hip", "registry.o", []),
             ("ltmp2.hip", "ltmp2.o", []),
             ("quadrature.cpp", "quadrature.o", ["-x", "hip"]),
             ("real_orbitals.cpp", "real_orbitals.o", ["-x", "hip"]),
             ("kpoints.cpp", "kpoints.o", ["-x", "hip"]),
             ("mlp.hip", "mlp.o", []),
             ("batch.hip", "batch.o", [])]
    units += [("grid_kernels.hip", f"grid_{n}.o", [f"-DLTMP2_N={n}"]) for n in GRIDS]
    cmds = []
    for src, obj, extra in units:
        cmds.append([HIPCC, *_flags(), *extra, "-c", os.path.join(CSRC, src),
                     "-o", os.path.join(BUILD, obj)])
    jobs = jobs or min(8, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for cmd, fut in zip(cmds, [ex.submit(_run, c) for c in cmds]):
            fut.result()
            if verbose:
                print("built", cmd[-1], flush=True)
    objs = [os.path.join(BUILD, u[1]) for u in units]
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
