"""Hartree potential as a Poisson problem (Section 2, mixed form of the
Kohn-Sham equation): -Laplace w = 4 pi rho in the box with Dirichlet data equal
to the free-space Coulomb potential of rho on the boundary.

The paper takes the boundary values from a fast multipole method and renews
them once per outer iteration (remark after Algorithm 3). The method it cites
is not given, so the boundary data here are the multipole expansion of rho
through the quadrupole about its charge centroid c, with r = x - c:
   g(x) = Q/|r| + p.r/|r|^3 + (1/2) sum_ij Q_ij r_i r_j / |r|^5,
   Q = int rho,  p = int (y-c) rho,  Q_ij = int rho (3 y_i y_j - |y|^2 delta_ij)
(y measured from c), all integrals by the fine quadrature.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse.linalg import splu


def multipole_moments(rho_qp, qp, qw):
    y = qp.reshape(-1, 3)
    m = (qw * rho_qp).ravel()
    Q = m.sum()
    c = (m[:, None] * y).sum(axis=0) / Q
    d = y - c
    p = (m[:, None] * d).sum(axis=0)
    r2 = np.einsum("ij,ij->i", d, d)
    Qij = np.einsum("n,ni,nj->ij", m, d, d) * 3.0 - np.eye(3) * (m * r2).sum()
    return Q, c, p, Qij


def multipole_values(points, Q, c, p, Qij):
    r = np.asarray(points, dtype=np.float64) - c
    rn = np.linalg.norm(r, axis=1)
    quad = np.einsum("ni,ij,nj->n", r, Qij, r)
    return Q / rn + (r @ p) / rn ** 3 + 0.5 * quad / rn ** 5


def boundary_data(mesh, rho_qp):
    """g at the boundary vertices of the mesh from the multipole expansion."""
    Q, c, p, Qij = multipole_moments(rho_qp, mesh.qp, mesh.qw)
    g = np.zeros(mesh.nv)
    g[mesh.bverts] = multipole_values(mesh.xyz[mesh.bverts], Q, c, p, Qij)
    return g


def poisson(mesh, K, rho_qp, g_nodal):
    """Solve K_II w_I = 4 pi (M rho)_I - K_IB g_B (exact sparse LU).
    Returns the interior part w_I (w = w_I on interior, g on the boundary)."""
    b = 4.0 * np.pi * mesh.load(rho_qp)[mesh.interior] - mesh.ib(K) @ g_nodal[mesh.bverts]
    lu = splu(mesh.ii(K).tocsc())
    return lu.solve(b)
