"""Pins of the checker's P2 space (oracle/fem2.py) against closed forms: the
27-point rule's exactness, the basis's nodal (Kronecker) property, exact
energies of quadratic functions, the coarse P1 space as a subspace, the
fourth-order eigenvalue rate of the harmonic oscillator, and the correction
step on P2 reaching the dense fine eigenpairs and the dense fine SCF."""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.sparse.linalg import eigsh

from inputs.meshgen import graded_mesh, kuhn_mesh
from inputs.systems import tiny_system
from oracle.fem import Mesh, prolongation
from oracle.fem2 import BQ, DQ, EDGES, LQ2, WQ2, MeshP2, basis
from oracle.mlc import Options, Problem, correction_step
from oracle.scf import initial_state, scf


def _perturbed_box(n, lo, hi, seed, amp=0.15):
    """Kuhn mesh with interior vertices moved at random (faces stay planar)."""
    xyz, tets = kuhn_mesh(n, lo, hi)
    h = (hi - lo) / n
    rng = np.random.default_rng(seed)
    inner = np.all((xyz > lo + 1e-9) & (xyz < hi - 1e-9), axis=1)
    xyz = xyz.copy()
    xyz[inner] += amp * h * rng.uniform(-1, 1, size=(inner.sum(), 3))
    return xyz, tets


# ---------------------------------------------------------------- quadrature
def test_conical_rule_integrates_degree_5_exactly():
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    pts = LQ2 @ V
    assert np.all(WQ2 > 0) and abs(WQ2.sum() - 1.0) < 1e-15
    for a, b, c in itertools.product(range(6), repeat=3):
        if a + b + c > 5:
            continue
        q = np.sum(WQ2 / 6.0 * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c)
        exact = math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
        assert abs(q - exact) < 1e-16, (a, b, c)
    # not degree 6
    q = np.sum(WQ2 / 6.0 * pts[:, 0] ** 6)
    assert abs(q - 720.0 / math.factorial(9)) > 1e-8


def test_basis_is_nodal_and_a_partition_of_unity():
    nodes = np.zeros((10, 4))
    for a in range(4):
        nodes[a, a] = 1.0
    for e, (a, b) in enumerate(EDGES):
        nodes[4 + e, a] = nodes[4 + e, b] = 0.5
    assert np.array_equal(basis(nodes), np.eye(10))
    assert np.max(np.abs(BQ.sum(axis=1) - 1.0)) < 1e-15
    # sum_a phi_a = 2 (sum lambda)^2 - sum lambda as a polynomial in the four lambda, so its
    # lambda-derivatives are 4 sum lambda - 1 = 3 on the tet (and sum_a grad phi_a = 0)
    assert np.max(np.abs(DQ.sum(axis=1) - 3.0)) < 1e-14


def test_p2_nodes_are_vertices_then_sorted_edge_midpoints():
    m = MeshP2(*kuhn_mesh(2, 0.0, 1.0), 0.0, 1.0)
    nv0 = len(m.vxyz)
    assert np.array_equal(m.xyz[:nv0], m.vxyz)
    e = m.edges
    assert np.all(e[:, 0] < e[:, 1])
    assert np.all(np.diff(e[:, 0] * (nv0 + 1) + e[:, 1]) > 0)
    for t in range(m.nt):
        for k, (a, b) in enumerate(EDGES):
            node = m.tets[t, 4 + k]
            assert np.allclose(m.xyz[node], 0.5 * (m.vxyz[m.vtets[t, a]] + m.vxyz[m.vtets[t, b]]))
    # Kuhn mesh of 2^3 cubes: 3^3 vertices, edges = 3 axis families + face and cube diagonals
    assert m.nv == (2 * 2 + 1) ** 3


# ---------------------------------------------------------------- exact energies
def _poly_mul(p, q):
    out = {}
    for (ea, ca), (eb, cb) in itertools.product(p.items(), q.items()):
        k = tuple(x + y for x, y in zip(ea, eb))
        out[k] = out.get(k, 0.0) + ca * cb
    return out


def _poly_int_box(p, lo, hi):
    return sum(c * np.prod([(hi ** (k + 1) - lo ** (k + 1)) / (k + 1) for k in e]) for e, c in p.items())


def _poly_eval(p, x):
    return sum(c * np.prod([x[:, i] ** e[i] for i in range(3)], axis=0) for e, c in p.items())


def _poly_grad(p, i):
    out = {}
    for e, c in p.items():
        if e[i] > 0:
            k = list(e)
            k[i] -= 1
            out[tuple(k)] = out.get(tuple(k), 0.0) + c * e[i]
    return out


def _random_quadratic(rng):
    return {e: rng.normal() for e in itertools.product(range(3), repeat=3) if sum(e) <= 2}


@pytest.fixture(scope="module")
def p2box():
    lo, hi = -1.5, 2.0
    return MeshP2(*_perturbed_box(4, lo, hi, seed=8), lo, hi), lo, hi


def test_stiffness_annihilates_constants_and_mass_gives_the_volume(p2box):
    m, lo, hi = p2box
    K = m.stiffness()
    assert np.max(np.abs(K @ np.ones(m.nv))) < 1e-12
    M = m.mass()
    assert abs(np.ones(m.nv) @ M @ np.ones(m.nv) - (hi - lo) ** 3) < 1e-12
    assert abs(K - K.T).max() < 1e-13 and abs(M - M.T).max() < 1e-15


def test_quadratics_have_exact_energies(p2box):
    """Nodal interpolation reproduces a quadratic u exactly, so u^T K v,
    u^T M v and b(f)^T v (f quadratic at the quadrature points) equal the
    box integrals of grad u . grad v, u v and f v in closed form."""
    m, lo, hi = p2box
    rng = np.random.default_rng(5)
    K, M = m.stiffness(), m.mass()
    for _ in range(3):
        u, v, f = _random_quadratic(rng), _random_quadratic(rng), _random_quadratic(rng)
        un, vn = _poly_eval(u, m.xyz), _poly_eval(v, m.xyz)
        gg = {}
        for i in range(3):
            for k, c in _poly_mul(_poly_grad(u, i), _poly_grad(v, i)).items():
                gg[k] = gg.get(k, 0.0) + c
        eK = _poly_int_box(gg, lo, hi)
        eM = _poly_int_box(_poly_mul(u, v), lo, hi)
        eL = _poly_int_box(_poly_mul(f, v), lo, hi)
        fq = _poly_eval(f, m.qp.reshape(-1, 3)).reshape(m.qw.shape)
        assert abs(un @ K @ vn - eK) < 1e-10 * max(1.0, abs(eK))
        assert abs(un @ M @ vn - eM) < 1e-10 * max(1.0, abs(eM))
        assert abs(m.load(fq) @ vn - eL) < 1e-10 * max(1.0, abs(eL))
        # at_qp of the nodal interpolant is u at the points
        assert np.max(np.abs(m.at_qp(un) - _poly_eval(u, m.qp.reshape(-1, 3)).reshape(m.qw.shape))) < 1e-11


def test_p1_coarse_space_is_a_subspace_of_p2():
    """Coarse P1 hats written in the fine P2 basis: P^T K P and P^T M P are
    the coarse P1 matrices (graded nested meshes)."""
    xyz, tets, cxyz, ctets = graded_mesh(3, -4, 4, [[0.3, -0.2, 0.1]], 0.8, 0.4, 0.8, coarse=(1.6, 0.5, 1.6, 5))
    fine, coarse = MeshP2(xyz, tets, -4, 4), Mesh(cxyz, ctets, -4, 4)
    Pf, P = prolongation(fine, coarse)
    KH = coarse.ii(coarse.stiffness()).toarray()
    MH = coarse.ii(coarse.mass()).toarray()
    assert np.linalg.norm((P.T @ fine.ii(fine.stiffness()) @ P).toarray() - KH) / np.linalg.norm(KH) < 1e-13
    assert np.linalg.norm((P.T @ fine.ii(fine.mass()) @ P).toarray() - MH) / np.linalg.norm(MH) < 1e-13
    assert abs(Pf.sum(axis=1) - 1).max() < 1e-13


# ---------------------------------------------------------------- eigenvalues
def test_harmonic_oscillator_converges_at_fourth_order():
    """V = r^2/2 in [-5, 5]^3: the ground state 3/2; P2 errors fall toward
    16x per halving of h (11x from h = 5/3 to 5/6; more than the 8x of a
    third-order method; P1 on the same meshes: 3x) and stay upper bounds."""
    errs = []
    for n in (6, 12):
        m = MeshP2(*kuhn_mesh(n, -5.0, 5.0), -5.0, 5.0)
        A = 0.5 * m.ii(m.stiffness()) + m.ii(m.mass(0.5 * np.sum(m.qp ** 2, axis=-1)))
        lam = eigsh(A.tocsc(), k=1, M=m.ii(m.mass()).tocsc(), sigma=0.0, which="LM")[0][0]
        errs.append(lam - 1.5)
    assert errs[0] > 0 and errs[1] > 0
    assert errs[0] / errs[1] > 9.0, errs


# ---------------------------------------------------------------- the method on P2
def test_linear_case_on_p2_reaches_the_dense_eigenpairs():
    """P-fix on P2 with the P1 space of the same mesh as V_H (nested: a P1
    function is a P2 function): the correction steps reach the lowest
    eigenpairs of the fine P2 pencil (dense eigh)."""
    S = tiny_system(n_fine=4, n_coarse=4, box=5.0, nonlinear=False, n_orbitals=2, seed=3, order=2)
    prob = Problem(S)
    assert prob.fine.order == 2
    A = (0.5 * prob.K + prob.mass_ii(prob.vext_qp)).toarray()
    ev = sla.eigh(A, prob.M.toarray(), eigvals_only=True)
    st, _ = initial_state(prob)
    for _ in range(150):
        st = correction_step(prob, st, Options()).state
    assert np.max(np.abs(st.lam - ev[:2])) < 1e-9, (st.lam, ev[:3])


def test_nonlinear_fixed_point_on_p2_is_the_fine_scf():
    S = tiny_system(n_fine=4, n_coarse=4, box=5.0, nonlinear=True, n_orbitals=1, seed=5, order=2)
    S.occupations = np.array([2.0])
    prob = Problem(S)
    ref = scf(prob.fine, S, tol=1e-13, maxit=300)
    st, _ = initial_state(prob)
    errs = []
    for _ in range(40):
        st = correction_step(prob, st, Options(inner_tol=1e-13)).state
        errs.append(abs(st.lam[0] - ref["lam"][0]))
    assert errs[-1] < 1e-8 and errs[-1] < 1e-4 * errs[0], errs


def test_energy_on_p2_at_the_fixed_point_is_the_kohn_sham_functional():
    """As for P1: at the dense fine SCF solution the step's reported energy
    equals the functional term by term (kinetic, external, Hartree, XC)."""
    from oracle import xc
    from oracle.mlc import State
    S = tiny_system(n_fine=4, n_coarse=4, box=5.0, nonlinear=True, n_orbitals=2, seed=5, order=2)
    prob = Problem(S)
    ref = scf(prob.fine, S, tol=1e-13, maxit=400)
    st = State(lam=ref["lam"].copy(), Phi=ref["Phi"].copy(), w=ref["w"].copy())
    res = correction_step(prob, st, Options(inner_tol=1e-13))
    assert np.max(np.abs(res.state.lam - ref["lam"])) < 1e-9
    fine, f, Phi = prob.fine, prob.f, ref["Phi"]
    rho = prob.density_qp(Phi)
    exc, _ = xc.evaluate(S.xc, rho, S.xalpha)
    kinetic = 0.5 * sum(f[i] * Phi[:, i] @ (prob.K @ Phi[:, i]) for i in range(prob.N))
    E = kinetic + fine.integrate(prob.vext_qp * rho) + 0.5 * fine.integrate(fine.at_qp(ref["w"]) * rho) \
        + fine.integrate(rho * exc)
    assert abs(res.energy - E) < 1e-10, (res.energy, E)
