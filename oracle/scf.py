"""Self-consistent solution of the discrete Kohn-Sham problem on one mesh
(eq. Nonlinear_Eigenvalue_Problem2 fem, with the Hartree term in the mixed
form of Section 3): Algorithm 1 step 1 on the coarse mesh, and the dense
brute-force reference on tiny fine meshes.

Each SCF step: density at quadrature points -> V_xc, multipole boundary data,
Poisson solve for w -> H = 1/2 K + M_{V_ext + w + V_xc} -> lowest N
eigenpairs of (H, M) by dense eigh -> output density. The input density is
updated by Anderson (Pulay) mixing with the L^2 inner product at the
quadrature points; the mixing only changes the path, not the fixed point.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import hartree as har
from . import xc as xcmod
from .fem import Mesh
from .potentials import v_ext


def scf(mesh: Mesh, system, tol=1e-11, maxit=400, beta=0.5, hist=6, verbose=False):
    f = np.asarray(system.occupations, dtype=np.float64)
    N = int(system.n_orbitals)
    Kf = mesh.stiffness()
    K, M, KIB = mesh.ii(Kf), mesh.ii(mesh.mass()), mesh.ib(Kf)
    vext = v_ext(mesh.qp, system.R, system.Z, system.potential, system.rc, system.omega)
    nonlinear = system.hartree or system.xc != 0
    rho_in = np.zeros_like(mesh.qw)
    w = np.zeros(mesh.nv)
    X_hist, F_hist = [], []
    ip = lambda a, b: float(np.sum(mesh.qw * a * b))

    def potentials(rho):
        _, vxc = xcmod.evaluate(system.xc, rho, system.xalpha)
        if system.hartree:
            g = har.boundary_data(mesh, rho) if rho.sum() > 0 else np.zeros(mesh.nv)
            wI = har.poisson(mesh, Kf, rho, g)
            wn = g.copy()
            wn[mesh.interior] = wI
        else:
            wn = np.zeros(mesh.nv)
        return vxc, wn

    for it in range(maxit):
        vxc, w = potentials(rho_in)
        H = 0.5 * K + mesh.ii(mesh.mass(vext + mesh.at_qp(w) + vxc))
        lam, Phi = sla.eigh(H.toarray(), M.toarray(), subset_by_index=[0, N - 1])
        ph = mesh.at_qp(mesh.full(Phi))
        rho_out = np.einsum("tqi,i->tq", ph * ph, f)
        F = rho_out - rho_in
        res = float(np.sum(mesh.qw * np.abs(F)))
        if verbose:
            print(it, lam, res)
        if not nonlinear or res < tol:
            break
        # Anderson mixing
        X_hist.append(rho_in.copy())
        F_hist.append(F.copy())
        if len(X_hist) > hist + 1:
            X_hist.pop(0)
            F_hist.pop(0)
        if len(X_hist) == 1:
            rho_in = rho_in + beta * F
        else:
            dX = [X_hist[k + 1] - X_hist[k] for k in range(len(X_hist) - 1)]
            dF = [F_hist[k + 1] - F_hist[k] for k in range(len(F_hist) - 1)]
            m = len(dF)
            A = np.array([[ip(dF[a], dF[b]) for b in range(m)] for a in range(m)])
            rhs = np.array([ip(dF[a], F) for a in range(m)])
            gam = np.linalg.lstsq(A, rhs, rcond=None)[0]
            rho_bar = rho_in - sum(gam[k] * dX[k] for k in range(m))
            F_bar = F - sum(gam[k] * dF[k] for k in range(m))
            rho_in = rho_bar + beta * F_bar
        rho_in = np.maximum(rho_in, 0.0)
    # Hartree of the final output density
    _, w = potentials(rho_out)
    return dict(lam=lam, Phi=Phi, w=w, rho=rho_out, iters=it + 1, residual=res)


def initial_state(prob, **kw):
    """Algorithm 1 step 1 on the coarse mesh and step 4's transfer to the fine
    mesh: Phi = P Phi_H (exact, nested spaces), w = interpolant of the coarse
    Hartree potential, Lambda = coarse eigenvalues."""
    from .mlc import State
    r = scf(prob.coarse, prob.sys, **kw)
    Phi = prob.P @ r["Phi"]
    w = prob.Pfull @ r["w"]
    return State(lam=r["lam"].copy(), Phi=np.asarray(Phi), w=np.asarray(w)), r
