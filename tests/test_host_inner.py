"""The host inner loop (Algorithm 2 in the form of Algorithm 3 step 2: per
orbital the bordered eigenproblem in V_H + span{u_i}, the Hartree problem in
W_H + span{w0}, Anderson mixing) compiled for the CPU with the library's host
flags and run on synthetic coarse-space data. Its per-orbital work runs on
several threads (borders, grouped bisections, selection, Hartree addends) and
is then combined in orbital order, so its outputs must not depend on the
number of threads: 1 and 4 threads give the same bytes, with and without the
Hartree term and with unoccupied orbitals."""
import os
import pathlib
import shutil
import subprocess

import numpy as np
import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2103_02824_amd" / "csrc"


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("inner") / "inner_probe"
    flags = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fopenmp", "-march=x86-64-v2", f"-I{CSRC}"]
    subprocess.run([hipcc, *flags, str(ROOT / "tests" / "host" / "inner_probe.cpp"), str(CSRC / "inner.cpp"),
                    str(CSRC / "dense.cpp"), "-o", str(out)], check=True, capture_output=True, timeout=600)
    return out


def _run(probe, tmp, n, N, hartree, zero_occ, threads):
    path = tmp / f"out_{n}_{N}_{hartree}_{zero_occ}_{threads}.bin"
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    r = subprocess.run([str(probe), str(n), str(N), str(path), str(hartree), str(int(zero_occ))], env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    return path.read_bytes(), r.stdout


@pytest.mark.parametrize("n,N,hartree,zero_occ", [(6, 1, 1, False), (6, 5, 1, False), (7, 13, 1, False),
                                                  (7, 13, 1, True), (6, 6, 0, False)])
def test_inner_loop_does_not_depend_on_the_thread_count(probe, tmp_path, n, N, hartree, zero_occ):
    one, log1 = _run(probe, tmp_path, n, N, hartree, zero_occ, 1)
    four, _ = _run(probe, tmp_path, n, N, hartree, zero_occ, 4)
    assert one == four, log1
    status = np.frombuffer(one[:4], dtype=np.int32)[0]
    assert status in (0, 1), log1            # MLC_OK, or the inner cap reached
    lam = np.frombuffer(one[4:4 + 8 * N], dtype=np.float64)
    assert np.all(np.isfinite(lam)), log1
