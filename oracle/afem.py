"""The adaptive part of Algorithm 1 (steps 1-3 and 9): the residual a
posteriori estimator of Section 2, Doerfler marking, and the transfer of a
nodal state to a mesh refined by bisection.

Test infrastructure only (plain FP64 NumPy, written from the paper): the
tests, the smoke check and the benchmark's CPU baseline may use it; the
library shares no code with it.

Estimator (Section 2, the residual-type indicator). For the eigenpairs
(lambda_i, phi_i) of the current state and the effective potential V_eff of
that state, on each tet T

    eta^2(T) = h_T^2 ||R_T||_{0,T}^2 + sum over interior faces e of T of h_e ||J_e||_{0,e}^2,
    R_T = (H phi_i - lambda_i phi_i)_i,   J_e = (1/2 grad phi_i|T+ . nu+ + 1/2 grad phi_i|T- . nu-)_i,

with H = -1/2 Laplacian + V_eff. For piecewise linear phi_i the Laplacian
vanishes inside each tet, so R_T = ((V_eff - lambda_i) phi_i)_i; its L2 norm
uses the same 4-point rule as the rest of the checker. The gradients are
constant on each tet, so J_e is constant on e and ||J_e||_{0,e}^2 = |e|
sum_i J_{e,i}^2. h_T and h_e are the longest edges of T and of e. The norms
of the vectors over orbitals sum the squares over i (unweighted).

Marking (Doerfler): the smallest set M of tets, taken in decreasing order of
eta^2 (ties by tet index), with sum_{T in M} eta^2(T) >= theta sum_T eta^2(T).

Transfer: a vertex created by bisection is the midpoint of an edge of the
previous mesh, so a piecewise linear function keeps its values at the old
vertices and takes the mean of the edge's end values at a new vertex."""
from __future__ import annotations

import numpy as np

from .fem import Mesh

_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def tet_diameters(mesh: Mesh):
    """Longest edge of each tet (h_T)."""
    P = mesh.xyz[mesh.tets]
    h2 = np.zeros(mesh.nt)
    for a, b in _EDGES:
        d = P[:, a] - P[:, b]
        h2 = np.maximum(h2, np.einsum("ij,ij->i", d, d))
    return np.sqrt(h2)


def interior_faces(mesh: Mesh):
    """Interior faces as (tet+, local face of tet+, tet-, local face of tet-);
    local face a is the face opposite vertex a."""
    tets = mesh.tets
    faces = np.concatenate([np.sort(np.delete(tets, a, axis=1), axis=1) for a in range(4)])
    owner = np.tile(np.arange(mesh.nt), 4)
    local = np.repeat(np.arange(4), mesh.nt)
    key = (faces[:, 0] * mesh.nv + faces[:, 1]) * mesh.nv + faces[:, 2]
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same = np.nonzero(ks[1:] == ks[:-1])[0]
    i, j = order[same], order[same + 1]
    return owner[i], local[i], owner[j], local[j]


def estimator(mesh: Mesh, lam, Phi_full, veff_qp):
    """eta^2 per tet for the eigenpairs (lam, Phi_full) (Phi_full: values at
    every vertex, zero on the boundary) and V_eff at the quadrature points.
    Written for the P1 space (no Laplacian term in the element residual)."""
    if getattr(mesh, "order", 1) != 1:
        raise ValueError("the estimator is written for P1 elements")
    lam = np.asarray(lam, dtype=np.float64)
    Phi_full = np.asarray(Phi_full, dtype=np.float64).reshape(mesh.nv, -1)
    hT = tet_diameters(mesh)
    # element residuals ((V_eff - lambda_i) phi_i)^2 at the quadrature points
    ph = mesh.at_qp(Phi_full)                                     # (nt, 4, N)
    res = (veff_qp[:, :, None] - lam[None, None, :]) * ph
    elem = hT ** 2 * np.einsum("tq,tqi->t", mesh.qw, res * res)
    # gradients per tet and orbital: sum_a phi_i(x_a) grad lambda_a
    G = np.einsum("tai,tax->tix", Phi_full[mesh.tets], mesh.grad)  # (nt, N, 3)
    tp, ap, tm, am = interior_faces(mesh)
    # outward unit normal of face a of T is -grad lambda_a / |grad lambda_a|; |e| = 3 |T| |grad lambda_a|
    gl = mesh.grad[tp, ap]
    gn = np.linalg.norm(gl, axis=1)
    nu = -gl / gn[:, None]
    area = 3.0 * mesh.vol[tp] * gn
    J = 0.5 * np.einsum("fix,fx->fi", G[tp] - G[tm], nu)          # (faces, N)
    # the three vertices of each face (all of tet+ but vertex ap)
    keep = np.ones((len(tp), 4), dtype=bool)
    keep[np.arange(len(tp)), ap] = False
    fv = mesh.tets[tp][keep].reshape(-1, 3)
    P = mesh.xyz[fv]
    he2 = np.zeros(len(tp))
    for a, b in ((0, 1), (0, 2), (1, 2)):
        d = P[:, a] - P[:, b]
        he2 = np.maximum(he2, np.einsum("ij,ij->i", d, d))
    face = np.sqrt(he2) * area * np.einsum("fi,fi->f", J, J)
    eta2 = elem.copy()
    np.add.at(eta2, tp, face)
    np.add.at(eta2, tm, face)
    return eta2


def dorfler_mark(eta2, theta):
    """Boolean mask of the Doerfler set (see the module docstring)."""
    eta2 = np.asarray(eta2, dtype=np.float64)
    order = np.lexsort((np.arange(len(eta2)), -eta2))
    csum = np.cumsum(eta2[order])
    total = csum[-1] if len(csum) else 0.0
    k = int(np.searchsorted(csum, theta * total, side="left")) + 1
    k = min(max(k, 1), len(eta2))
    mark = np.zeros(len(eta2), dtype=bool)
    mark[order[:k]] = True
    return mark


def transfer(values_old, nv_new, new_parents):
    """Nodal values on the refined mesh: old vertices keep their values, new
    vertex v (ids nv_old, nv_old + 1, ... in creation order) takes the mean of
    its edge's end values; new_parents[k] = (lo, hi) of vertex nv_old + k."""
    V = np.asarray(values_old, dtype=np.float64)
    nv_old = V.shape[0]
    out = np.zeros((nv_new,) + V.shape[1:])
    out[:nv_old] = V
    for k, (a, b) in enumerate(np.asarray(new_parents, dtype=np.int64)):
        out[nv_old + k] = 0.5 * (out[a] + out[b])
    return out


def veff_qp(prob, st):
    """V_eff of the state st at the fine quadrature points: V_ext + w + V_xc(rho)."""
    from . import xc as xcmod
    rho = prob.density_qp(st.Phi)
    _, vxc = xcmod.evaluate(prob.sys.xc, rho, prob.sys.xalpha)
    return prob.vext_qp + prob.fine.at_qp(st.w) + vxc


def adapt(system, opts, theta, levels, steps, state, refine):
    """Algorithm 1 with refinement: on each fine mesh `steps` correction steps,
    then the estimator, Doerfler marking, refinement of the marked tets by
    `refine(marked) -> (xyz, tets, new_parents)` (the caller's mesh generator)
    and the transfer of (Lambda, Phi, w); the coarse mesh stays. Returns one
    dict per mesh: sizes, eigenvalues, sqrt(sum eta^2), the marked set."""
    import dataclasses
    from .mlc import Problem, State, correction_step
    S = system
    prob = Problem(S)
    st = state
    out = []
    for lev in range(levels):
        for _ in range(steps):
            st = correction_step(prob, st, opts).state
        eta2 = estimator(prob.fine, st.lam, prob.fine.full(st.Phi), veff_qp(prob, st))
        rec = {"level": lev, "n_dof": prob.fine.n_dof, "n_tets": prob.fine.nt, "lam": st.lam.copy(),
               "eta": float(np.sqrt(eta2.sum())), "eta2": eta2, "mark": None}
        out.append(rec)
        if lev == levels - 1:
            break
        mark = dorfler_mark(eta2, theta)
        rec["mark"] = mark
        xyz, tets, parents = refine(mark)
        Pf = transfer(prob.fine.full(st.Phi), len(xyz), parents)
        w = transfer(st.w, len(xyz), parents)
        S = dataclasses.replace(S, xyz=xyz, tets=tets)
        prob = Problem(S)
        st = State(lam=st.lam.copy(), Phi=Pf[prob.fine.interior], w=w)
    return out
