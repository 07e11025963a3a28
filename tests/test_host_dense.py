"""The library's host eigen-solver for the augmented problems (Algorithm 3
step 2: per orbital the bordered matrix [[T, u], [u^T, alpha]], its lowest
eigenvalues by bisection, the eigenpair of largest border weight |theta_2|
kept), compiled for the CPU with g++ and checked against numpy's dense
symmetric eigensolver on the same matrix.

The cases include degenerate spectra: symmetric meshes give coarse operators
with repeated eigenvalues, and their tridiagonal form can split exactly into
blocks on which the border vanishes. The eigenvectors of such eigenvalues have
zero border weight and must never be selected."""
import ctypes
import pathlib
import shutil
import subprocess

import numpy as np
import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2103_02824_amd" / "csrc"
P = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("dense") / "libdense_probe.so"
    subprocess.run(["g++", "-O2", "-fPIC", "-shared", f"-I{CSRC}", str(ROOT / "tests" / "host" / "dense_probe.cpp"),
                    str(CSRC / "dense.cpp"), "-o", str(out)], check=True)
    return ctypes.CDLL(str(out))


def _sym(rng, lam):
    Q, _ = np.linalg.qr(rng.standard_normal((len(lam), len(lam))))
    C = Q @ np.diag(lam) @ Q.T
    return 0.5 * (C + C.T)


def _run(lib, C, u, alpha, k):
    n = len(u)
    ev, w, s = np.zeros(k), np.zeros(k), np.zeros(k)
    Y = np.zeros((n, k))
    lib.probe_bordered(np.ascontiguousarray(C).ctypes.data_as(P), np.ascontiguousarray(u).ctypes.data_as(P),
                       ctypes.c_double(alpha), n, k, ev.ctypes.data_as(P), w.ctypes.data_as(P), Y.ctypes.data_as(P),
                       s.ctypes.data_as(P))
    return ev, w, Y, s


def _dense(C, u, alpha):
    n = len(u)
    B = np.zeros((n + 1, n + 1))
    B[:n, :n], B[:n, n], B[n, :n], B[n, n] = C, u, u, alpha
    return np.linalg.eigh(B)


def _cases():
    rng = np.random.default_rng(7)
    n = 40
    yield "distinct", _sym(rng, np.sort(rng.uniform(0.5, 9.0, n))), rng.standard_normal(n) * 0.4, 2.5
    lam = np.array([1.0, 2.0, 2.0, 2.0] + [3.0] * 6 + list(np.linspace(4.0, 9.0, n - 10)))
    yield "degenerate", _sym(rng, lam), rng.standard_normal(n) * 0.3, 2.5
    n1 = 25
    C = np.zeros((n, n))
    C[:n1, :n1] = _sym(rng, np.linspace(1.0, 9.0, n1))
    C[n1:, n1:] = _sym(rng, np.array([1.5, 1.5, 1.5, 3.9, 3.9] + list(np.linspace(5.0, 9.0, n - n1 - 5))))
    u = np.zeros(n)
    u[:n1] = rng.standard_normal(n1) * 0.3
    yield "split_uncoupled_block", C, u, 2.5


@pytest.mark.parametrize("name,C,u,alpha", list(_cases()), ids=lambda v: v if isinstance(v, str) else "")
def test_bordered_eigenpairs_match_dense_eigh(lib, name, C, u, alpha):
    k = 12
    ev, w, Y, s = _run(lib, C, u, alpha, k)
    lam, V = _dense(C, u, alpha)
    n = len(u)
    scale = np.max(np.abs(lam))
    assert np.max(np.abs(ev - lam[:k])) < 1e-12 * scale
    theta = np.abs(V[n, :k])
    # the border weight: exact where the eigenvector is coupled to the border,
    # zero for eigenvectors of T extended by a zero border
    assert np.max(np.abs(w - theta)) < 1e-10, (w, theta)
    if name != "distinct":
        assert np.any(theta < 1e-12) and np.all(w[theta < 1e-12] == 0.0)
    # the selection of Algorithm 3 step 2 and its eigenvector
    j = int(np.argmax(w))
    assert j == int(np.argmax(theta))
    y = np.concatenate([Y[:, j], [s[j]]])
    v = V[:, j] * np.sign(V[n, j] * s[j])
    assert np.linalg.norm(y - v) < 1e-10
