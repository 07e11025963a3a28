"""Linear (P1) finite elements on tetrahedra, Section 2 (the discrete space
V_h subset of H^1_0 and the discrete Kohn-Sham problem).

Everything is assembled the textbook way: element matrices summed with
scipy.sparse COO duplicates. Fields that the method evaluates pointwise
(potentials, densities) live at quadrature points; the quadrature is the
symmetric 4-point rule of degree 2 with positive weights |T|/4 at barycentric
points (a,b,b,b) and permutations, a = (5+3 sqrt5)/20, b = (5-sqrt5)/20. The
paper does not name a rule; this one integrates products of two P1 functions
exactly, so the mass matrix is exact.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

QA = (5.0 + 3.0 * np.sqrt(5.0)) / 20.0
QB = (5.0 - np.sqrt(5.0)) / 20.0
# LQ[q, j] = barycentric coordinate j of quadrature point q
LQ = np.full((4, 4), QB)
np.fill_diagonal(LQ, QA)
WQ = np.full(4, 0.25)  # weights relative to |T|


class Mesh:
    """A tetrahedral mesh with its interior (Dirichlet-free) vertex numbering."""

    order = 1

    def __init__(self, xyz, tets, lo, hi):
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.tets = np.asarray(tets, dtype=np.int64)
        self.nv = len(self.xyz)
        self.nt = len(self.tets)
        on = np.zeros(self.nv, dtype=bool)
        for ax in range(3):
            on |= np.isclose(self.xyz[:, ax], lo, rtol=0, atol=1e-12 * max(1, abs(lo)))
            on |= np.isclose(self.xyz[:, ax], hi, rtol=0, atol=1e-12 * max(1, abs(hi)))
        self.boundary = on
        self.interior = np.nonzero(~on)[0]          # DoF k <-> vertex interior[k]
        self.bverts = np.nonzero(on)[0]
        self.n_dof = len(self.interior)
        P = self.xyz[self.tets]
        J = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)  # columns
        det = np.linalg.det(J)
        self.vol = np.abs(det) / 6.0
        Jinv = np.linalg.inv(J)             # rows = gradients of lambda_1..3
        g = np.empty((self.nt, 4, 3))
        g[:, 1:, :] = Jinv
        g[:, 0, :] = -Jinv.sum(axis=1)
        self.grad = g                        # grad[t, j] = grad of barycentric j
        self.qp = np.einsum("qj,tjx->tqx", LQ, P)  # quadrature points (nt,4,3)
        self.qw = self.vol[:, None] * WQ[None, :]  # quadrature weights (nt,4)

    # -- nodal <-> quadrature ------------------------------------------------
    def full(self, u_int):
        """Interior coefficients (n_dof, ...) -> nodal values with zero boundary."""
        u = np.zeros((self.nv,) + np.shape(u_int)[1:])
        u[self.interior] = u_int
        return u

    def at_qp(self, u_nodal):
        """Nodal values (nv,) or (nv,N) -> values at quadrature points (nt,4[,N])."""
        U = np.asarray(u_nodal)[self.tets]          # (nt,4[,N])
        return np.einsum("qj,tj...->tq...", LQ, U)

    def integrate(self, f_qp):
        return float(np.sum(self.qw * f_qp))

    # -- assembly -------------------------------------------------------------
    def _coo(self, elem):
        rows = np.repeat(self.tets, 4, axis=1).ravel()
        cols = np.tile(self.tets, (1, 4)).ravel()
        return sp.coo_matrix((elem.ravel(), (rows, cols)), shape=(self.nv, self.nv)).tocsr()

    def stiffness(self):
        """K_ab = int grad phi_a . grad phi_b over the whole vertex set."""
        elem = self.vol[:, None, None] * np.einsum("tix,tjx->tij", self.grad, self.grad)
        return self._coo(elem)

    def mass(self, f_qp=None):
        """M_f,ab = int f phi_a phi_b by the 4-point rule; f=None means f=1."""
        f = np.ones((self.nt, 4)) if f_qp is None else f_qp
        elem = np.einsum("tq,qi,qj->tij", self.qw * f, LQ, LQ)
        return self._coo(elem)

    def load(self, f_qp):
        """b_a = int f phi_a by the 4-point rule, over all vertices."""
        elem = np.einsum("tq,qi->ti", self.qw * f_qp, LQ)
        b = np.zeros(self.nv)
        np.add.at(b, self.tets.ravel(), elem.ravel())
        return b

    def ii(self, A):
        """Interior-interior block of a vertex-indexed matrix."""
        return A[self.interior][:, self.interior].tocsr()

    def ib(self, A):
        return A[self.interior][:, self.bverts].tocsr()


def hat_values(fine_xyz, coarse: Mesh):
    """P_full[a, k] = coarse hat function psi_k evaluated at fine vertex a.

    Found by point location: candidate coarse tets by nearest centroids,
    barycentric coordinates by solving the 3x3 affine system. For nested
    meshes psi_k is linear on every fine tet, so psi_k = sum_a P[a,k] phi_a
    exactly (the coarse space is a subspace of the fine one)."""
    cP = coarse.xyz[coarse.tets]
    cen = cP.mean(axis=1)
    tree = cKDTree(cen)
    kq = min(48, coarse.nt)
    _, cand = tree.query(fine_xyz, k=kq)
    cand = np.atleast_2d(cand)
    J = np.stack([cP[:, 1] - cP[:, 0], cP[:, 2] - cP[:, 0], cP[:, 3] - cP[:, 0]], axis=2)
    Jinv = np.linalg.inv(J)
    nf = len(fine_xyz)
    chosen = np.full(nf, -1)
    bary = np.zeros((nf, 4))
    best = np.full(nf, -np.inf)
    for c in range(kq):
        t = cand[:, c]
        l123 = np.einsum("nij,nj->ni", Jinv[t], fine_xyz - cP[t, 0])
        l = np.concatenate([1.0 - l123.sum(axis=1, keepdims=True), l123], axis=1)
        m = l.min(axis=1)
        better = m > best
        best = np.where(better, m, best)
        chosen = np.where(better, t, chosen)
        bary = np.where(better[:, None], l, bary)
    # points not inside any of the nearest-centroid candidates (long, thin
    # bisection tets near the nuclei): every coarse tet
    for a in np.nonzero(best < -1e-10)[0]:
        l123 = np.einsum("tij,tj->ti", Jinv, fine_xyz[a][None, :] - cP[:, 0])
        l = np.concatenate([1.0 - l123.sum(axis=1, keepdims=True), l123], axis=1)
        t = int(np.argmax(l.min(axis=1)))
        best[a], chosen[a], bary[a] = l[t].min(), t, l[t]
    if np.any(best < -1e-10):
        raise RuntimeError("fine vertex outside the coarse mesh")
    bary = np.where(np.abs(bary) < 1e-14, 0.0, bary)
    rows = np.repeat(np.arange(nf), 4)
    cols = coarse.tets[chosen].ravel()
    return sp.coo_matrix((bary.ravel(), (rows, cols)), shape=(nf, coarse.nv)).tocsr()


def make_mesh(xyz, tets, lo, hi, order=1):
    """The P1 space (order 1) or the P2 space (order 2, fem2.MeshP2) on a mesh."""
    if order == 1:
        return Mesh(xyz, tets, lo, hi)
    if order == 2:
        from .fem2 import MeshP2
        return MeshP2(xyz, tets, lo, hi)
    raise ValueError("element order must be 1 or 2")


def prolongation(fine: Mesh, coarse: Mesh):
    """Returns (P_full (fine nv x coarse nv), P (fine dof x coarse dof)).
    The coarse space is P1; on a P2 fine space the rows are the fine nodes
    (vertices and edge midpoints), where the coarse hats' values are again
    their exact P2 coefficients (a coarse hat is linear on every fine tet)."""
    Pf = hat_values(fine.xyz, coarse)
    P = Pf[fine.interior][:, coarse.interior].tocsr()
    P.eliminate_zeros()
    return Pf, P
