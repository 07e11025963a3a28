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
    # a small border against a wide spectrum (coarse operators reach 1e3 while
    # the auxiliary direction adds little to the coarse space): coupled
    # eigenvalues lie close to eigenvalues of T and keep weights of order one
    lam = np.concatenate([[0.3, 0.9, 1.4], np.geomspace(2.0, 1.5e3, n - 3)])
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    C = Q @ np.diag(lam) @ Q.T
    u = Q @ (np.r_[2e-6, 1e-6, 3e-6, rng.standard_normal(n - 3) * 1e-6])
    yield "small_border_wide_spectrum", 0.5 * (C + C.T), u, 0.9 + 2.2e-6


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
    # zero for eigenvectors of T extended by a zero border. Within 1e-6 of a
    # pole the weight moves by ~10 per unit of mu, so the eigenvalues' own
    # error (1e-12 scale = 1.5e-9 there) allows 1e-7.
    wtol = 1e-7 if name == "small_border_wide_spectrum" else 1e-10
    assert np.max(np.abs(w - theta)) < wtol, (w, theta)
    if name in ("degenerate", "split_uncoupled_block"):
        assert np.any(theta < 1e-12) and np.all(w[theta < 1e-12] < 1e-12)
    # the selection of Algorithm 3 step 2 and its eigenvector
    j = int(np.argmax(w))
    assert j == int(np.argmax(theta))
    y = np.concatenate([Y[:, j], [s[j]]])
    v = V[:, j] * np.sign(V[n, j] * s[j])
    assert np.linalg.norm(y - v) < wtol  # gap to the nearest eigenvalue: 1e-6 in the wide case


def test_harmonic_oscillator_augmented_problems_select_as_the_checker(lib):
    """The augmented problems of one inner iteration of the harmonic
    oscillator (6^3 coarse mesh, 12^3 fine, four orbitals: the ground state
    and the degenerate triplet), built by the checker. Symmetry makes many
    coarse eigenvectors orthogonal to each u_i, so most of the lowest
    eigenvalues of each augmented problem carry theta_2 = 0. The library's
    reduction to [[T, u], [u^T, alpha]] (C = L^-1 A_H L^-T with M_H = L L^T,
    the border made M-orthogonal to V_H: a = M_H^-1 c, gamma' = gamma - c.a)
    must give the weights |theta_2| sqrt(gamma') of the checker's generalized
    eigenvectors and select the same eigenpair."""
    import scipy.linalg as sla
    from inputs.systems import harmonic
    from oracle.mlc import Options, Problem, augmented_blocks, fine_stage, select_eigenpair
    from oracle.scf import initial_state
    S = harmonic(12, 6, n_orbitals=4)
    prob = Problem(S)
    st0, _ = initial_state(prob, maxit=300)
    fs = fine_stage(prob, st0, Options(shift=True, sigma0=1.0))
    U, P = fs["U"], prob.P
    H, _ = augmented_blocks(prob, U, fs["w0"], fs["g"], fs["vxc"])
    AH = (P.T @ H @ P).toarray()
    MH = (P.T @ prob.M @ P).toarray()
    n_keep = min(prob.NH + 1, prob.N + 8)
    Li = np.linalg.inv(np.linalg.cholesky(MH))
    C = Li @ AH @ Li.T
    C = 0.5 * (C + C.T)
    n_zero = 0
    for i in range(prob.N):
        u = U[:, i]
        Hu, Mu = H @ u, prob.M @ u
        b, beta, c, gam = P.T @ Hu, float(u @ Hu), P.T @ Mu, float(u @ Mu)
        a = np.linalg.solve(MH, c)
        gp = gam - c @ a
        ub = Li @ (b - AH @ a) / np.sqrt(gp)
        alpha = (beta - 2.0 * b @ a + a @ AH @ a) / gp
        ev, w, _, _ = _run(lib, C, ub, alpha, n_keep)
        Ki = np.block([[AH, b[:, None]], [b[None, :], np.array([[beta]])]])
        Mi = np.block([[MH, c[:, None]], [c[None, :], np.array([[gam]])]])
        lam, X = sla.eigh(Ki, Mi, subset_by_index=[0, n_keep - 1])
        theta = np.abs(X[-1, :]) * np.sqrt(gp)
        assert np.max(np.abs(ev - lam)) < 1e-11 * np.max(np.abs(lam))
        assert np.max(np.abs(w - theta)) < 1e-10, (i, w, theta)
        lsel, _ = select_eigenpair(lam, X, n_keep)
        assert ev[int(np.argmax(w))] == pytest.approx(lsel, abs=1e-11)
        n_zero += int(np.sum(theta < 1e-12))
    assert n_zero >= 20  # the symmetric spectrum decouples most candidates
