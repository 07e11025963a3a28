"""Pins of the FP64 checker against what the paper and the mathematics fix:
closed forms, invariants, special cases that reduce to textbook routines and
brute force on tiny meshes. Each test is chosen so that a plausible mistake
(a dropped term, a wrong sign or index, a transposed operand) fails it.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.sparse.linalg import eigsh, splu
from scipy.special import erf

from inputs.meshgen import graded_mesh, kuhn_mesh
from inputs.systems import (POT_BARE, POT_ERF, XC_LDA, XC_NONE, System, aufbau, c1_hydrogen, harmonic,
                            hydrogen_bare, tiny_system)
from oracle import hartree as har
from oracle import xc
from oracle.decomp import augmented_from_pieces, coarse_trilinear, hartree_rhs_from_pieces, pieces
from oracle.fem import LQ, WQ, Mesh, prolongation
from oracle.mlc import Options, Problem, State, correction_step, fine_stage, inner_scf
from oracle.pcg import jacobi_pcg
from oracle.potentials import v_ext
from oracle.scf import initial_state, scf


# ---------------------------------------------------------------- quadrature
@pytest.mark.parametrize("a,b,c", [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0), (0, 1, 1),
                                   (1, 0, 1), (0, 0, 2)])
def test_quadrature_monomials_degree2(a, b, c):
    # reference tet (0,0,0),(1,0,0),(0,1,0),(0,0,1): int x^a y^b z^c = a! b! c! / (a+b+c+3)!
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    pts = LQ @ V
    q = np.sum(WQ / 6.0 * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c)
    exact = math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
    assert abs(q - exact) < 1e-15


def test_quadrature_not_exact_degree3():
    # the rule is degree 2 only: x^3 must not be integrated exactly
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    pts = LQ @ V
    q = np.sum(WQ / 6.0 * pts[:, 0] ** 3)
    assert abs(q - 6.0 / math.factorial(6)) > 1e-5


# ---------------------------------------------------------------- assembly
@pytest.fixture(scope="module")
def box_mesh():
    xyz, tets = kuhn_mesh(5, -2.0, 3.0)
    return Mesh(xyz, tets, -2.0, 3.0)


def test_stiffness_annihilates_constants(box_mesh):
    K = box_mesh.stiffness()
    assert np.max(np.abs(K @ np.ones(box_mesh.nv))) < 1e-13


def test_mass_total_volume(box_mesh):
    M = box_mesh.mass()
    assert abs(np.ones(box_mesh.nv) @ M @ np.ones(box_mesh.nv) - 125.0) < 1e-11


def test_energy_of_linear_function(box_mesh):
    a = np.array([0.3, -1.2, 0.7])
    u = box_mesh.xyz @ a + 0.4
    K, M = box_mesh.stiffness(), box_mesh.mass()
    assert abs(u @ K @ u - 125.0 * (a @ a)) < 1e-10
    # int (a.x + 0.4)^2 over [-2,3]^3, closed form
    m1 = 0.5 * (9 - 4)            # int x dx over [-2,3]
    m2 = (27 + 8) / 3.0           # int x^2 dx
    L = 5.0
    exact = (a @ a) * m2 * L * L + 2 * (a[0] * a[1] + a[0] * a[2] + a[1] * a[2]) * m1 * m1 * L \
        + 0.8 * a.sum() * m1 * L * L + 0.16 * L ** 3
    assert abs(u @ M @ u - exact) < 1e-9


def test_mass_with_field_is_linear_and_symmetric(box_mesh):
    rng = np.random.default_rng(0)
    f = rng.standard_normal((box_mesh.nt, 4))
    g = rng.standard_normal((box_mesh.nt, 4))
    Mf, Mg, Mfg = box_mesh.mass(f), box_mesh.mass(g), box_mesh.mass(2 * f - g)
    assert abs(Mfg - (2 * Mf - Mg)).max() < 1e-12
    assert abs(Mf - Mf.T).max() < 1e-14
    # M_f with f = 1 is the plain mass matrix
    assert abs(box_mesh.mass(np.ones((box_mesh.nt, 4))) - box_mesh.mass()).max() < 1e-15


# ---------------------------------------------------------------- nesting
@pytest.mark.parametrize("graded", [False, True])
def test_prolongation_reproduces_coarse_matrices(graded):
    if graded:
        xyz, tets, cxyz, ctets = graded_mesh(3, -4, 4, [[0.3, -0.2, 0.1]], 0.8, 0.4, 0.8, coarse=(1.6, 0.5, 1.6, 5))
    else:
        xyz, tets = kuhn_mesh(8, -4, 4)
        cxyz, ctets = kuhn_mesh(4, -4, 4)
    fine, coarse = Mesh(xyz, tets, -4, 4), Mesh(cxyz, ctets, -4, 4)
    _, P = prolongation(fine, coarse)
    KH = coarse.ii(coarse.stiffness()).toarray()
    MH = coarse.ii(coarse.mass()).toarray()
    Kp = (P.T @ fine.ii(fine.stiffness()) @ P).toarray()
    Mp = (P.T @ fine.ii(fine.mass()) @ P).toarray()
    assert np.linalg.norm(Kp - KH) / np.linalg.norm(KH) < 1e-13
    assert np.linalg.norm(Mp - MH) / np.linalg.norm(MH) < 1e-13
    # partition of unity of the coarse hats on the interior (full P)
    Pf, _ = prolongation(fine, coarse)
    assert abs(Pf.sum(axis=1) - 1).max() < 1e-13


# ---------------------------------------------------------------- XC
def test_lda_potential_is_derivative_of_energy_density():
    rho = np.logspace(-6, 2, 60)  # spans both r_s branches
    e, v = xc.lda(rho)
    h = 1e-6 * rho
    ep, _ = xc.lda(rho + h)
    em, _ = xc.lda(rho - h)
    fd = ((rho + h) * ep - (rho - h) * em) / (2 * h)
    assert np.max(np.abs(fd - v) / np.abs(v)) < 1e-7


def test_slater_exchange_identities():
    rho = np.array([1e-3, 0.1, 2.0])
    ex = xc.eps_x(rho)
    assert np.allclose(ex, -0.75 * (3 / np.pi) ** (1 / 3) * rho ** (1 / 3), rtol=1e-15)
    e, v = xc.lda(rho)
    # exchange part of v is exactly 4/3 of eps_x
    rs = (3 / (4 * np.pi * rho)) ** (1 / 3)
    vc = xc.eps_c_of_rs(rs) - rs / 3 * xc.deps_c_drs(rs)
    assert np.allclose(v - vc, 4.0 / 3.0 * ex, rtol=1e-14)


def test_pz81_values_from_printed_constants():
    # r_s = 2 (high branch) and r_s = 0.5 (low branch), written from the table of Section 4
    rs = np.array([2.0, 0.5])
    ec = xc.eps_c_of_rs(rs)
    assert abs(ec[0] - (-0.1423 / (1 + 1.0529 * math.sqrt(2.0) + 0.3334 * 2.0))) < 1e-16
    assert abs(ec[1] - (0.0311 * math.log(0.5) - 0.048 + 0.0020 * 0.5 * math.log(0.5) - 0.0116 * 0.5)) < 1e-16
    # the two branches nearly meet at r_s = 1 (the parametrisation is built so)
    hi = -0.1423 / (1 + 1.0529 + 0.3334)
    lo = -0.048 - 0.0116
    assert abs(hi - lo) < 5e-4


def test_xc_zero_density_and_xalpha():
    e, v = xc.lda(np.array([0.0, 1e-31]))
    assert np.all(e == 0) and np.all(v == 0)
    rho = np.array([0.01, 1.0])
    e, v = xc.xalpha(rho)
    assert np.allclose(v, -1.5 * 0.77298 * (3 * rho / np.pi) ** (1 / 3))
    ep, _ = xc.xalpha(rho * (1 + 1e-6))
    em, _ = xc.xalpha(rho * (1 - 1e-6))
    fd = (rho * (1 + 1e-6) * ep - rho * (1 - 1e-6) * em) / (2e-6 * rho)
    assert np.allclose(fd, v, rtol=1e-8)


# ---------------------------------------------------------------- potentials
def test_smoothed_coulomb_limits():
    pts = np.array([[0.0, 0.0, 0.0], [1e-7, 0, 0], [5.0, 0, 0]])
    v = v_ext(pts, np.zeros((1, 3)), np.array([2.0]), POT_ERF, rc=0.5)
    assert abs(v[0] + 2 * 2 / (math.sqrt(math.pi) * 0.5)) < 1e-12
    assert abs(v[1] - v[0]) < 1e-10
    assert abs(v[2] + 2 * erf(10.0) / 5.0) < 1e-15
    vb = v_ext(pts[2:], np.zeros((1, 3)), np.array([2.0]), POT_BARE)
    assert abs(vb[0] + 0.4) < 1e-15


# ---------------------------------------------------------------- Hartree
def _gaussian_case(n, alpha=1.5, box=8.0, centre=(0.3, -0.2, 0.1)):
    xyz, tets = kuhn_mesh(n, -box, box)
    m = Mesh(xyz, tets, -box, box)
    c = np.asarray(centre)
    r2 = np.sum((m.qp - c) ** 2, axis=-1)
    rho = (alpha / np.pi) ** 1.5 * np.exp(-alpha * r2)
    return m, rho, c, alpha


def test_multipole_against_direct_coulomb_sum():
    """Two Gaussians at c +- (1,0,0): the dipole about the centroid vanishes,
    the quadrupole is about 1.5% of the monopole at the box faces and the
    next even term about 2e-4. The expansion must match the direct sum
    sum_q m_q / |x - y_q| to well below the quadrupole size."""
    xyz, tets = kuhn_mesh(16, -8.0, 8.0)
    m = Mesh(xyz, tets, -8.0, 8.0)
    c = np.array([0.3, -0.2, 0.1])
    rho = np.zeros((m.nt, 4))
    for s in (-1.0, 1.0):
        r2 = np.sum((m.qp - c - s * np.array([1.0, 0, 0])) ** 2, axis=-1)
        rho += np.exp(-2.0 * r2)
    Q, cc, p, Qij = har.multipole_moments(rho, m.qp, m.qw)
    assert np.linalg.norm(p) < 1e-12 * Q
    assert abs(np.trace(Qij)) < 1e-12 * Q
    g = har.boundary_data(m, rho)[m.bverts]
    y = m.qp.reshape(-1, 3)
    w = (m.qw * rho).ravel()
    X = m.xyz[m.bverts]
    direct = np.array([np.sum(w / np.linalg.norm(y - x, axis=1)) for x in X])
    mono = Q / np.linalg.norm(X - cc, axis=1)
    assert np.max(np.abs(g - direct) / direct) < 1e-3
    assert np.max(np.abs(mono - direct) / direct) > 5e-3   # the quadrupole matters here


def test_poisson_gaussian_closed_form_and_rate():
    """-Laplace w = 4 pi rho for a normalised Gaussian has w = erf(sqrt(a) r)/r.
    With that exact Dirichlet data the nodal error falls at second order."""
    errs = []
    for n in (8, 16, 32):
        m, rho, c, a = _gaussian_case(n)
        r = np.linalg.norm(m.xyz - c, axis=1)
        exact = np.where(r > 1e-12, erf(np.sqrt(a) * r) / np.where(r > 1e-12, r, 1), 2 * np.sqrt(a / np.pi))
        g = np.zeros(m.nv)
        g[m.bverts] = exact[m.bverts]
        wI = har.poisson(m, m.stiffness(), rho, g)
        errs.append(np.max(np.abs(wI - exact[m.interior])))
    assert errs[2] < 0.04
    assert errs[1] / errs[2] > 3.0 and errs[0] / errs[1] > 2.0


# ---------------------------------------------------------------- linear solvers
def test_pcg_matches_sparse_lu():
    m = Mesh(*kuhn_mesh(10, -5, 5), -5, 5)
    K = m.ii(m.stiffness()) + 0.3 * m.ii(m.mass())
    B = np.random.default_rng(1).standard_normal((m.n_dof, 3))
    X, it = jacobi_pcg(K, B, rtol=1e-13)
    Xe = splu(K.tocsc()).solve(B)
    assert np.linalg.norm(X - Xe) / np.linalg.norm(Xe) < 1e-11
    assert np.all(it > 5)


# ---------------------------------------------------------------- eigenvalue limits
def _lowest(m, f_qp, k):
    A = 0.5 * m.ii(m.stiffness()) + m.ii(m.mass(f_qp))
    return np.sort(eigsh(A.tocsc(), k=k, M=m.ii(m.mass()).tocsc(), sigma=-5.0, which="LM")[0])


def test_harmonic_oscillator_levels():
    vals = []
    for n in (16, 32):
        m = Mesh(*kuhn_mesh(n, -5, 5), -5, 5)
        vals.append(_lowest(m, 0.5 * np.sum(m.qp ** 2, axis=-1), 4))
    exact = np.array([1.5, 2.5, 2.5, 2.5])
    e0, e1 = np.abs(vals[0] - exact), np.abs(vals[1] - exact)
    assert np.all(e1 < 0.1)
    assert np.all(e0 / e1 > 3.0)          # O(h^2)
    assert np.all(vals[1] > exact)        # conforming Galerkin: upper bounds


def test_bare_hydrogen_tends_to_minus_half():
    """Bare Coulomb Z=1 (no Hartree, no XC): the discrete ground state decreases
    monotonically toward the exact -0.5 Ha under grading toward the nucleus
    (Galerkin upper bounds)."""
    vals = []
    for h0 in (0.4, 0.2, 0.1):
        xyz, tets, _, _ = graded_mesh(4, -10, 10, [[0, 0, 0]], h0, 0.25, h0, 8.0)
        m = Mesh(xyz, tets, -10, 10)
        A = 0.5 * m.ii(m.stiffness()) + m.ii(m.mass(v_ext(m.qp, np.zeros((1, 3)), np.ones(1), POT_BARE)))
        vals.append(eigsh(A.tocsc(), k=1, M=m.ii(m.mass()).tocsc(), sigma=-0.7, which="LM")[0][0])
    err = np.array(vals) + 0.5
    assert np.all(err > 0) and np.all(np.diff(err) < 0)
    assert err[1] / err[2] > 1.3 and err[2] < 0.02


def _radial_fd(Z, rc, R=10.0, n=20000):
    # -1/2 u'' + V u = E u on (0, R), u(0) = u(R) = 0 (s states), second-order FD
    h = R / n
    r = h * np.arange(1, n)
    V = -Z * erf(r / rc) / r
    d = 1.0 / h ** 2 + V
    e = -0.5 / h ** 2 * np.ones(n - 2)
    return sla.eigh_tridiagonal(d, e, select="i", select_range=(0, 0))[0][0]


def test_smoothed_coulomb_ground_state_matches_radial_solve():
    E1 = _radial_fd(1.0, 0.5)
    assert abs(E1 - (-0.412957)) < 2e-5           # value quoted for this check
    vals = []
    for n in (8, 16, 32):
        m = Mesh(*kuhn_mesh(n, -10, 10), -10, 10)
        vals.append(_lowest(m, v_ext(m.qp, np.zeros((1, 3)), np.ones(1), POT_ERF, rc=0.5), 1)[0])
    assert np.all(np.diff(vals) < 0) and np.all(np.array(vals) > E1 - 1e-6)
    assert abs(vals[-1] - E1) < 0.02


# ---------------------------------------------------------------- the method
def test_linear_case_converges_to_dense_eigensolve():
    """P-fix: with no Hartree and no XC the correction steps reproduce the lowest
    eigenpairs of the fine pencil (brute force with dense eigh)."""
    S = tiny_system(n_fine=8, n_coarse=4, box=5.0, nonlinear=False, n_orbitals=2, seed=3)
    prob = Problem(S)
    A = (0.5 * prob.K + prob.mass_ii(prob.vext_qp)).toarray()
    ev, _ = sla.eigh(A, prob.M.toarray())
    st, _ = initial_state(prob)
    errs = []
    for _ in range(120):
        st = correction_step(prob, st, Options()).state
        errs.append(np.max(np.abs(st.lam - ev[:2])))
    assert errs[-1] < 1e-10, (st.lam, ev[:3])
    assert errs[59] < 1e-5 * errs[0]     # steady linear contraction


def test_nonlinear_fixed_point_is_fine_scf():
    """P-fix, nonlinear: iterating the method reaches the self-consistent
    solution of the fine problem computed densely (Hartree + LDA)."""
    S = tiny_system(n_fine=8, n_coarse=4, box=5.0, nonlinear=True, n_orbitals=1, seed=5)
    S.occupations = np.array([2.0])
    prob = Problem(S)
    ref = scf(prob.fine, S, tol=1e-13, maxit=300)
    st, _ = initial_state(prob)
    errs = []
    for _ in range(40):
        res = correction_step(prob, st, Options(inner_tol=1e-13))
        st = res.state
        errs.append(abs(st.lam[0] - ref["lam"][0]))
    assert errs[-1] < 1e-8 and errs[-1] < 1e-4 * errs[0], errs


def test_exact_eigenpair_is_a_fixed_point():
    """Linear case: starting from the exact fine eigenpairs (dense eigh), the
    auxiliary solution is the eigenvector itself and the augmented
    Rayleigh-Ritz problem returns the same eigenpairs."""
    S = tiny_system(n_fine=8, n_coarse=4, box=5.0, nonlinear=False, n_orbitals=2, seed=3)
    prob = Problem(S)
    A = (0.5 * prob.K + prob.mass_ii(prob.vext_qp)).toarray()
    ev, V = sla.eigh(A, prob.M.toarray())
    st = State(lam=ev[:2].copy(), Phi=V[:, :2].copy(), w=np.zeros(prob.fine.nv))
    res = correction_step(prob, st, Options())
    assert np.max(np.abs(res.state.lam - ev[:2])) < 1e-12
    fs = res.inter["fine"]
    for i in range(2):
        u = fs["U"][:, i]
        c = u @ prob.M @ V[:, i]
        assert np.linalg.norm(u - c * V[:, i]) < 1e-10
        s = np.sign(res.state.Phi[:, i] @ prob.M @ V[:, i])
        assert np.linalg.norm(s * res.state.Phi[:, i] - V[:, i]) < 1e-9


@pytest.fixture(scope="module")
def c1_step():
    S = c1_hydrogen()
    prob = Problem(S)
    st0, _ = initial_state(prob)
    res = correction_step(prob, st0, Options(inner_tol=1e-11))
    return prob, st0, res


def test_density_integral_and_rayleigh_quotient(c1_step):
    prob, st0, res = c1_step
    assert abs(res.rho_integral - 1.0) < 1e-12
    # lambda_i = phi_i^T H phi_i / phi_i^T M phi_i with the last inner Hartree iterate
    inn = res.inter["inner"]
    fs = res.inter["fine"]
    H = inn["Afix"] + prob.mass_ii(prob.fine.at_qp(prob.Pfull_c @ inn["wH"])) + inn["th1"] * inn["Mw0"]
    phi = res.state.Phi[:, 0]
    rq = phi @ H @ phi / (phi @ prob.M @ phi)
    # H uses the final (w_H, theta1); the eigenvalue the previous one: equal at convergence
    assert abs(rq - res.state.lam[0]) < 1e-8
    assert abs(phi @ prob.M @ phi - 1.0) < 1e-12


def test_hartree_direction_solves_fine_poisson_with_lift(c1_step):
    prob, st0, res = c1_step
    fs = res.inter["fine"]
    fine = prob.fine
    w = fs["g"].copy()
    w[fine.interior] += fs["w0"]
    # (grad w, grad v) = 4 pi (rho~, v) for interior v, and w = g on the boundary
    lhs = (prob.Kfull @ w)[fine.interior]
    rhs = 4 * np.pi * fine.load(fs["rho_tilde"])[fine.interior]
    assert np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs) < 1e-10


def test_augmented_problem_upper_bound_linear():
    """Rayleigh-Ritz in V_H + span{u}: eigenvalues never below the fine ones."""
    S = tiny_system(n_fine=8, n_coarse=4, box=5.0, nonlinear=False, n_orbitals=2)
    prob = Problem(S)
    A = (0.5 * prob.K + prob.mass_ii(prob.vext_qp)).toarray()
    ev = sla.eigh(A, prob.M.toarray(), eigvals_only=True)
    st, _ = initial_state(prob)
    res = correction_step(prob, st, Options())
    assert np.all(res.state.lam >= ev[:2] - 1e-12)


@pytest.mark.parametrize("order", [1, 2])
def test_algorithm3_pieces_equal_direct_assembly(order):
    """Algorithm 3 step 1 decomposition vs the direct fine assembly of the
    augmented matrices and of the Hartree right-hand side, at arbitrary inner
    iterates (the expansion keeps 2 theta2 and theta2^2 and the occupations);
    on P1 and on P2 fine spaces."""
    S = tiny_system(n_fine=8 if order == 1 else 4, n_coarse=4, box=5.0, nonlinear=True, n_orbitals=2, seed=7,
                    order=order)
    prob = Problem(S)
    st, _ = initial_state(prob)
    fs = fine_stage(prob, st, Options())
    pc = pieces(prob, fs["U"], fs["w0"], fs["g"], fs["vxc"])
    tri, trho = coarse_trilinear(prob)
    rng = np.random.default_rng(3)
    wH = rng.standard_normal(prob.NH) * 0.1
    th1 = 0.9
    fine, P = prob.fine, prob.P
    H = (0.5 * prob.K + prob.mass_ii(prob.vext_qp + fs["vxc"] + fine.at_qp(fs["g"]))
         + prob.mass_ii(fine.at_qp(prob.Pfull_c @ wH)) + th1 * prob.mass_ii(fine.at_qp(fine.full(fs["w0"]))))
    for i in range(2):
        U = sp.hstack([P, sp.csr_matrix(fs["U"][:, i][:, None])]).tocsr()
        Kd = (U.T @ H @ U).toarray()
        Md = (U.T @ prob.M @ U).toarray()
        K, M = augmented_from_pieces(pc, tri, i, wH, th1)
        assert np.linalg.norm(K - Kd) / np.linalg.norm(Kd) < 1e-12
        assert np.linalg.norm(M - Md) / np.linalg.norm(Md) < 1e-12
    phiH = rng.standard_normal((prob.NH, 2)) * 0.05
    theta2 = np.array([0.8, 1.1])
    fH, gg = hartree_rhs_from_pieces(pc, trho, prob.f, phiH, theta2)
    Phi = P @ phiH + fs["U"] * theta2[None, :]
    rho = prob.density_qp(Phi)
    fH_d = P.T @ fine.load(rho)[fine.interior]
    g_d = fs["w0"] @ fine.load(rho)[fine.interior]
    assert np.linalg.norm(fH - fH_d) / np.linalg.norm(fH_d) < 1e-12
    assert abs(gg - g_d) / abs(g_d) < 1e-12


def test_aufbau_occupations():
    assert list(aufbau(5, 3)) == [2, 2, 1]
    assert list(aufbau(10, 6)) == [2, 2, 2, 2, 2, 0]


# ---------------------------------------------------------------- energy and the inner iteration
def test_energy_at_fixed_point_is_kohn_sham_functional():
    """The reported energy (sum f_i lambda_i minus the double-counting terms
    -1/2 int w rho and int rho (eps_xc - v_xc)) equals the Kohn-Sham energy
    functional of Section 2 evaluated term by term at the self-consistent fine
    solution, which the method leaves unchanged: kinetic 1/2 sum f_i
    phi_i^T K phi_i, external int V_ext rho, Hartree 1/2 int w rho with w the
    fine Hartree potential of rho, exchange-correlation int rho eps_xc(rho).
    A flipped sign or a lost factor in either double-counting term moves the
    energy by O(1)."""
    S = tiny_system(n_fine=8, n_coarse=4, box=5.0, nonlinear=True, n_orbitals=2, seed=5)
    prob = Problem(S)
    ref = scf(prob.fine, S, tol=1e-13, maxit=400)
    st = State(lam=ref["lam"].copy(), Phi=ref["Phi"].copy(), w=ref["w"].copy())
    res = correction_step(prob, st, Options(inner_tol=1e-13))
    assert np.max(np.abs(res.state.lam - ref["lam"])) < 1e-9     # a fixed point of the step
    fine = prob.fine
    rho = prob.density_qp(ref["Phi"])
    exc, _ = xc.evaluate(S.xc, rho, S.xalpha)
    f = prob.f
    kinetic = 0.5 * sum(f[i] * ref["Phi"][:, i] @ (prob.K @ ref["Phi"][:, i]) for i in range(prob.N))
    e_ext = fine.integrate(prob.vext_qp * rho)
    e_h = 0.5 * fine.integrate(fine.at_qp(ref["w"]) * rho)
    e_xc = fine.integrate(rho * exc)
    E_direct = kinetic + e_ext + e_h + e_xc
    assert abs(res.energy - E_direct) < 1e-10, (res.energy, E_direct)
    assert e_h > 0.1 and abs(e_xc) > 0.1                          # both terms matter at this size


def test_anderson_mixing_solves_linear_fixed_point():
    """The mixing rule of the inner iteration, on a linear map x -> A x + b
    whose plain iteration diverges (spectral radius > 1): with a history of at
    least the dimension it reaches the fixed point (I - A)^{-1} b in at most
    dimension + 2 steps (Anderson mixing is then a Krylov method), in any SPD
    inner product."""
    from oracle.mlc import anderson_next
    rng = np.random.default_rng(7)
    n = 6
    A = rng.normal(size=(n, n))
    A = 1.6 * A / np.max(np.abs(np.linalg.eigvals(A)))
    b = rng.normal(size=n)
    G = rng.normal(size=(n, n))
    G = G @ G.T + n * np.eye(n)
    xstar = np.linalg.solve(np.eye(n) - A, b)
    x = np.zeros(n)
    hist = []
    for _ in range(n + 2):
        F = A @ x + b - x
        x = anderson_next(x, F, hist, G, m=n, beta=0.5)
    assert np.linalg.norm(x - xstar) < 1e-9 * np.linalg.norm(xstar)
    # plain iteration from the same start diverges
    y = np.zeros(n)
    for _ in range(n + 2):
        y = A @ y + b
    assert np.linalg.norm(y - xstar) > np.linalg.norm(xstar)


def test_mixed_inner_iteration_has_the_printed_fixed_point():
    """Mixing changes the path of Algorithm 2, not its fixed point: from the
    converged mixed result, one printed (unmixed) iteration returns the same
    orbitals and Hartree coefficients."""
    S = tiny_system(n_fine=8, n_coarse=4, box=5.0, nonlinear=True, n_orbitals=2, seed=5)
    prob = Problem(S)
    st0, _ = initial_state(prob)
    opts = Options(inner_tol=1e-12)
    fs = fine_stage(prob, st0, opts)
    mixed = inner_scf(prob, fs, opts)
    assert mixed["inner_iters"] < opts.inner_maxit
    one = Options(inner_tol=0.0, inner_maxit=1, inner_mix_history=0)
    x0 = np.concatenate([mixed["wH"], [mixed["th1"]]])
    plain = inner_scf(prob, fs, one, x_start=x0)
    M = prob.M
    for i in range(prob.N):
        a, b_ = mixed["Phi"][:, i], plain["Phi"][:, i]
        assert np.sqrt((a - b_) @ (M @ (a - b_))) < 1e-9
    assert np.max(np.abs(plain["lam"] - mixed["lam"])) < 1e-10
    assert abs(plain["th1"] - mixed["th1"]) < 1e-9


# ---------------------------------------------------------------- the joint-space variant
def test_joint_variant_linear_case_converges_to_dense_eigensolve():
    """The comparison method (one augmented space V_H + span{u_1..u_N} for all
    orbitals): with no Hartree and no XC its steps reach the lowest N
    eigenpairs of the fine pencil (dense eigh), and its orbitals are
    M-orthonormal at every step."""
    S = tiny_system(n_fine=8, n_coarse=4, box=5.0, nonlinear=False, n_orbitals=3, seed=3)
    prob = Problem(S)
    A = (0.5 * prob.K + prob.mass_ii(prob.vext_qp)).toarray()
    ev, _ = sla.eigh(A, prob.M.toarray())
    st, _ = initial_state(prob)
    for _ in range(120):
        res = correction_step(prob, st, Options(variant="joint"))
        st = res.state
        G = st.Phi.T @ (prob.M @ st.Phi)
        assert np.max(np.abs(G - np.eye(3))) < 1e-12
    assert np.max(np.abs(st.lam - ev[:3])) < 1e-10, (st.lam, ev[:3])


def test_joint_variant_exact_eigenpairs_are_a_fixed_point():
    """Starting from exact fine eigenpairs, the joint space contains them, and
    its lowest N Ritz pairs are those eigenpairs."""
    S = tiny_system(n_fine=8, n_coarse=4, box=5.0, nonlinear=False, n_orbitals=2, seed=3)
    prob = Problem(S)
    A = (0.5 * prob.K + prob.mass_ii(prob.vext_qp)).toarray()
    ev, V = sla.eigh(A, prob.M.toarray())
    st = State(lam=ev[:2].copy(), Phi=V[:, :2].copy(), w=np.zeros(prob.fine.nv))
    res = correction_step(prob, st, Options(variant="joint"))
    assert np.max(np.abs(res.state.lam - ev[:2])) < 1e-12
    for i in range(2):
        s = np.sign(res.state.Phi[:, i] @ prob.M @ V[:, i])
        assert np.linalg.norm(s * res.state.Phi[:, i] - V[:, i]) < 1e-9
