"""Pins of the checker's adaptive pieces (oracle/afem.py): the residual
estimator of Section 2 on cases with closed forms, Doerfler marking by brute
force, and the transfer of nodal values to a bisected mesh."""
import itertools

import numpy as np

from inputs.meshgen import AdaptiveMesh, kuhn_mesh
from oracle import afem
from oracle.fem import Mesh


def _mesh(n=3, lo=-1.0, hi=1.0):
    xyz, tets = kuhn_mesh(n, lo, hi)
    return Mesh(xyz, tets, lo, hi)


def test_estimator_vanishes_for_a_global_linear_function_with_veff_equal_lambda():
    """No element residual where V_eff = lambda, and no gradient jump for a
    function linear on the whole mesh (its nodal values are not zero on the
    boundary: the estimator does not look at the boundary condition)."""
    m = _mesh()
    phi = (1.0 + 2.0 * m.xyz[:, 0] - 0.5 * m.xyz[:, 1] + 0.3 * m.xyz[:, 2])[:, None]
    lam = np.array([-0.7])
    eta2 = afem.estimator(m, lam, phi, np.full((m.nt, 4), -0.7))
    assert np.max(np.abs(eta2)) < 1e-24


def test_element_term_is_the_mass_matrix_closed_form():
    """With a constant V_eff = c the element term is h_T^2 (c - lambda)^2
    phi_T^T M_T phi_T, M_T = |T|/20 (1 + delta_ab) (the rule is exact for
    quadratics); a global linear phi leaves no face term."""
    m = _mesh(2)
    rng = np.random.default_rng(3)
    a = rng.normal(size=4)
    phi = a[0] + m.xyz @ a[1:]
    c, lam = 1.7, np.array([-0.4])
    eta2 = afem.estimator(m, lam, phi[:, None], np.full((m.nt, 4), c))
    MT = (np.ones((4, 4)) + np.eye(4)) / 20.0
    P = m.xyz[m.tets]
    hT = np.max([np.linalg.norm(P[:, i] - P[:, j], axis=1) for i, j in itertools.combinations(range(4), 2)], axis=0)
    pv = phi[m.tets]
    ref = hT ** 2 * (c - lam[0]) ** 2 * m.vol * np.einsum("ta,ab,tb->t", pv, MT, pv)
    assert np.allclose(eta2, ref, rtol=1e-12, atol=0)


def test_face_term_of_a_single_hat_jump():
    """Two tets sharing one face; phi = 1 at the vertex of T+ opposite the face
    and 0 elsewhere, V_eff = lambda: the gradient jumps only across the shared
    face, J = 1/2 |grad phi|T+| = 1/(2 d) with d the height of that vertex
    over the face, so both tets get h_e |e| / (4 d^2) (area by the cross
    product, h_e by the face's edges)."""
    xyz = np.array([[0.0, 0.0, 0.0], [1.2, 0.1, 0.0], [0.2, 0.9, 0.1], [0.3, 0.2, 1.1], [0.4, 0.3, -0.8]])
    tets = np.array([[0, 1, 2, 3], [0, 1, 2, 4]])
    m = Mesh(xyz, tets, -10.0, 10.0)
    phi = np.zeros((5, 1))
    phi[3, 0] = 1.0
    eta2 = afem.estimator(m, np.array([0.5]), phi, np.full((2, 4), 0.5))
    f = xyz[[0, 1, 2]]
    cr = np.cross(f[1] - f[0], f[2] - f[0])
    area = 0.5 * np.linalg.norm(cr)
    d = abs((xyz[3] - f[0]) @ cr) / np.linalg.norm(cr)
    he = max(np.linalg.norm(f[0] - f[1]), np.linalg.norm(f[0] - f[2]), np.linalg.norm(f[1] - f[2]))
    ref = he * area / (4.0 * d * d)
    assert np.allclose(eta2, [ref, ref], rtol=1e-12)


def test_interior_faces_of_a_kuhn_mesh():
    """Each interior face is shared by exactly two tets, and the count closes:
    a Kuhn mesh of n^3 cubes has two boundary triangles per boundary square,
    12 n^2 in all, so 4 nt = 2 F_interior + 12 n^2."""
    n = 3
    m = _mesh(n)
    tp, ap, tm, am = afem.interior_faces(m)
    assert 4 * m.nt == 2 * len(tp) + 12 * n * n
    for t1, a1, t2, a2 in zip(tp, ap, tm, am):
        f1 = set(np.delete(m.tets[t1], a1)); f2 = set(np.delete(m.tets[t2], a2))
        assert f1 == f2 and t1 != t2


def test_dorfler_marking_is_the_smallest_sufficient_set():
    """Brute force on small random indicators: the marked set reaches theta
    of the total, and no smaller set does (the largest entries first)."""
    rng = np.random.default_rng(7)
    for trial in range(40):
        n = int(rng.integers(1, 9))
        eta2 = rng.exponential(size=n)
        theta = float(rng.uniform(0.05, 1.0))
        mark = afem.dorfler_mark(eta2, theta)
        k = int(mark.sum())
        assert eta2[mark].sum() >= theta * eta2.sum() - 1e-15
        best_smaller = max((sum(c) for c in itertools.combinations(eta2, k - 1)), default=0.0)
        assert best_smaller < theta * eta2.sum()
        # the marked entries are the k largest
        assert np.min(eta2[mark]) >= np.max(eta2[~mark], initial=-np.inf)


def test_transfer_is_exact_for_linear_functions_after_bisection():
    """Refine marked tets of a Kuhn mesh by bisection (with closure): nodal
    values of a linear function transferred by edge means equal the function
    at the new vertices; old vertices keep theirs."""
    am = AdaptiveMesh.kuhn(2, -1.0, 1.0)
    rng = np.random.default_rng(2)
    a = rng.normal(size=4)
    for step in range(3):
        f_old = a[0] + am.xyz @ a[1:]
        mark = rng.random(len(am.tets)) < 0.3
        nv0 = len(am.xyz)
        am.refine(mark)
        f_new = afem.transfer(f_old, len(am.xyz), am.new_parents)
        assert len(am.new_parents) == len(am.xyz) - nv0 > 0
        assert np.allclose(f_new, a[0] + am.xyz @ a[1:], rtol=0, atol=1e-12)
