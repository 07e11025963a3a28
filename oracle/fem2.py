"""Quadratic (P2) Lagrange elements on tetrahedra: the same discrete space
construction as Section 2 (V_h subset of H^1_0, interior DoFs only), with
quadratic instead of linear polynomials on each tet. The paper computes with
linear elements; the quadratic space is the workload's extension of it, and
MeshP2 offers the same interface as fem.Mesh so that every other checker
module (Hartree, SCF, the correction step, Algorithm 3's pieces) runs on it
unchanged.

Nodes: the mesh vertices in the caller's order, then one node per edge at its
midpoint, edges in increasing (lo, hi) vertex-pair order. Per tet the 10
local nodes are its 4 vertices and the edges (0,1) (0,2) (0,3) (1,2) (1,3)
(2,3). Basis in barycentric coordinates: lambda_a (2 lambda_a - 1) at a
vertex, 4 lambda_a lambda_b at edge (a, b).

Quadrature: the conical product rule of Stroud (Approximate Calculation of
Multiple Integrals, 1971) with 3 points per direction, of degree 5: the tet
is the image of the unit cube under xi = u, eta = (1-u) v, zeta = (1-u)(1-v) w,
whose Jacobian (1-u)^2 (1-v) is taken into Gauss-Jacobi weights in u (weight
(1-u)^2) and v (weight (1-v)); w is Gauss-Legendre. 27 points, positive
weights, exact for the P2 mass matrix (degree 4) and the P2 stiffness
(degree 2). Points in the order u (slowest), v, w (fastest).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.special import roots_jacobi

EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def _gauss_jacobi01(n, alpha):
    """n-point Gauss rule on [0, 1] for the weight (1-u)^alpha."""
    x, w = roots_jacobi(n, alpha, 0.0)        # weight (1-x)^alpha on [-1, 1]
    return (x + 1.0) / 2.0, w / 2.0 ** (alpha + 1)


def conical_rule(n=3):
    """Barycentric points (n^3, 4) and weights relative to |T| (sum 1)."""
    u, wu = _gauss_jacobi01(n, 2)
    v, wv = _gauss_jacobi01(n, 1)
    s, ws = _gauss_jacobi01(n, 0)
    pts, wts = [], []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                xi = u[i]
                eta = (1.0 - u[i]) * v[j]
                zeta = (1.0 - u[i]) * (1.0 - v[j]) * s[k]
                pts.append([1.0 - xi - eta - zeta, xi, eta, zeta])
                wts.append(6.0 * wu[i] * wv[j] * ws[k])
    return np.array(pts), np.array(wts)


LQ2, WQ2 = conical_rule(3)


def basis(lam):
    """P2 basis values (..., 10) at barycentric points lam (..., 4)."""
    lam = np.asarray(lam, dtype=np.float64)
    out = [lam[..., a] * (2.0 * lam[..., a] - 1.0) for a in range(4)]
    out += [4.0 * lam[..., a] * lam[..., b] for a, b in EDGES]
    return np.stack(out, axis=-1)


def basis_dlam(lam):
    """d phi_a / d lambda_c, (..., 10, 4); grad phi_a = sum_c D[a, c] grad lambda_c."""
    lam = np.asarray(lam, dtype=np.float64)
    D = np.zeros(lam.shape[:-1] + (10, 4))
    for a in range(4):
        D[..., a, a] = 4.0 * lam[..., a] - 1.0
    for e, (a, b) in enumerate(EDGES):
        D[..., 4 + e, a] = 4.0 * lam[..., b]
        D[..., 4 + e, b] = 4.0 * lam[..., a]
    return D


BQ = basis(LQ2)          # (27, 10)
DQ = basis_dlam(LQ2)     # (27, 10, 4)


def p2_nodes(xyz, tets):
    """(node xyz (nv + ne, 3), element nodes (nt, 10), edges (ne, 2))."""
    xyz = np.asarray(xyz, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)
    pairs = np.concatenate([np.sort(tets[:, [a, b]], axis=1) for a, b in EDGES])
    edges, inv = np.unique(pairs, axis=0, return_inverse=True)
    inv = inv.ravel().reshape(len(EDGES), len(tets)).T            # (nt, 6)
    nodes = np.concatenate([xyz, 0.5 * (xyz[edges[:, 0]] + xyz[edges[:, 1]])])
    el = np.concatenate([tets, len(xyz) + inv], axis=1)
    return nodes, el, edges


class MeshP2:
    """A tetrahedral mesh with the P2 space on it (interface of fem.Mesh)."""

    order = 2

    def __init__(self, xyz, tets, lo, hi):
        self.vxyz = np.asarray(xyz, dtype=np.float64)
        self.vtets = np.asarray(tets, dtype=np.int64)
        self.xyz, self.tets, self.edges = p2_nodes(self.vxyz, self.vtets)
        self.nv = len(self.xyz)
        self.nt = len(self.tets)
        on = np.zeros(self.nv, dtype=bool)
        for ax in range(3):
            on |= np.isclose(self.xyz[:, ax], lo, rtol=0, atol=1e-12 * max(1, abs(lo)))
            on |= np.isclose(self.xyz[:, ax], hi, rtol=0, atol=1e-12 * max(1, abs(hi)))
        self.boundary = on
        self.interior = np.nonzero(~on)[0]
        self.bverts = np.nonzero(on)[0]
        self.n_dof = len(self.interior)
        P = self.vxyz[self.vtets]
        J = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
        self.vol = np.abs(np.linalg.det(J)) / 6.0
        Jinv = np.linalg.inv(J)
        g = np.empty((self.nt, 4, 3))
        g[:, 1:, :] = Jinv
        g[:, 0, :] = -Jinv.sum(axis=1)
        self.grad = g                                        # barycentric gradients
        self.qp = np.einsum("qj,tjx->tqx", LQ2, P)           # (nt, 27, 3)
        self.qw = self.vol[:, None] * WQ2[None, :]           # (nt, 27)

    def full(self, u_int):
        u = np.zeros((self.nv,) + np.shape(u_int)[1:])
        u[self.interior] = u_int
        return u

    def at_qp(self, u_nodal):
        U = np.asarray(u_nodal)[self.tets]                   # (nt, 10[, N])
        return np.einsum("qj,tj...->tq...", BQ, U)

    def integrate(self, f_qp):
        return float(np.sum(self.qw * f_qp))

    def _coo(self, elem):
        rows = np.repeat(self.tets, 10, axis=1).ravel()
        cols = np.tile(self.tets, (1, 10)).ravel()
        return sp.coo_matrix((elem.ravel(), (rows, cols)), shape=(self.nv, self.nv)).tocsr()

    def grad_qp(self):
        """grad phi_a at every quadrature point, (nt, 27, 10, 3)."""
        return np.einsum("qac,tcx->tqax", DQ, self.grad)

    def stiffness(self):
        """K_ab = |T| sum_q W_q grad phi_a(q) . grad phi_b(q). With
        grad phi_a = sum_c D[q,a,c] grad lambda_c (grad lambda constant on T)
        the sum is |T| sum_{c,d} S[a,b,c,d] (grad lambda_c . grad lambda_d),
        S = sum_q W_q D[q,a,c] D[q,b,d] the same for every tet."""
        S = np.einsum("q,qac,qbd->abcd", WQ2, DQ, DQ)
        gl = np.matmul(self.grad, self.grad.transpose(0, 2, 1))           # (nt, 4, 4)
        elem = self.vol[:, None, None] * (gl.reshape(self.nt, 16) @ S.reshape(100, 16).T).reshape(self.nt, 10, 10)
        return self._coo(elem)

    def mass(self, f_qp=None):
        f = np.ones_like(self.qw) if f_qp is None else f_qp
        elem = np.einsum("tq,qa,qb->tab", self.qw * f, BQ, BQ, optimize=True)
        return self._coo(elem)

    def load(self, f_qp):
        elem = np.einsum("tq,qa->ta", self.qw * f_qp, BQ)
        b = np.zeros(self.nv)
        np.add.at(b, self.tets.ravel(), elem.ravel())
        return b

    def ii(self, A):
        return A[self.interior][:, self.interior].tocsr()

    def ib(self, A):
        return A[self.interior][:, self.bverts].tocsr()
