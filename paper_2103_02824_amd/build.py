"""Build libmlc.so (the C-ABI library) in-tree with hipcc for gfx950.

Usage: python -m paper_2103_02824_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from pathlib import Path

HERE = Path(__file__).resolve().parent
CSRC = HERE / "csrc"
OUT = HERE / "libmlc.so"
BUILD = HERE / "_build"

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-fPIC",
    "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
HOST_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-fopenmp", "-march=x86-64-v2"]


def _hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p


def _omp_libdir():
    for d in ("/opt/rocm/llvm/lib", "/opt/rocm/lib/llvm/lib"):
        if os.path.exists(os.path.join(d, "libomp.so")):
            return d
    return None


def build(verbose=False, jobs=8):
    BUILD.mkdir(exist_ok=True)
    hipcc = _hipcc()
    inc = ["-I", str(HERE.parent / "include"), "-I", str(CSRC)]
    jobs_list = []
    objs = []
    for src in sorted(CSRC.glob("*.hip")):
        obj = BUILD / (src.stem + ".hip.o")
        jobs_list.append([hipcc, *HIP_FLAGS, *inc, "-c", str(src), "-o", str(obj)])
        objs.append(obj)
    for src in sorted(CSRC.glob("*.cpp")):
        obj = BUILD / (src.stem + ".o")
        jobs_list.append([hipcc, *HOST_FLAGS, *inc, "-c", str(src), "-o", str(obj)])
        objs.append(obj)
    procs = []
    for cmd in jobs_list:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    omp = _omp_libdir()
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fopenmp", "-o", str(OUT) + ".tmp", *map(str, objs)]
    if omp:
        link += [f"-L{omp}", f"-Wl,-rpath,{omp}"]
    if verbose:
        print(" ".join(link), flush=True)
    _wait((link, subprocess.Popen(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    os.replace(str(OUT) + ".tmp", OUT)
    return OUT


def _wait(item):
    cmd, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    if p.returncode != 0:
        sys.stderr.write(text)
        raise RuntimeError(f"build step failed ({p.returncode}): {' '.join(cmd)}")
    noisy = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if noisy:
        sys.stderr.write("\n".join(noisy) + "\n")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
