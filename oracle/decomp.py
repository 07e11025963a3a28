"""Algorithm 3 step 1 and step 2 restated on the checker side: the fine-mesh
integrals that do not change during the inner iteration are computed once
(eqs. Adef, bdef, Ah4def, betadef, rhsdef, Hartree_H_h, fH, gdef, FG), and the
augmented matrices of any inner iterate are then formed from them on the
coarse space alone.

The expansions of (phi_H + theta2 u)^2 used for f_H and g keep the factor 2
on the cross term, the theta2^2 term and the occupations (the printed
expansion drops them). The coarse trilinear tensor T_jkm = int psi_j psi_k
psi_m, evaluated with the fine quadrature, makes A_{H,2}(w_H) =
sum_m T_jkm w_m and (phi_H^2, psi_j) coarse-only operations.

Used by the tests to pin that these pieces reproduce the direct fine-mesh
assembly of mlc.inner_scf.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import LQ


def coarse_trilinear(prob):
    """T as a function: returns tri(w) = sum_m T_jkm w_m (N_H x N_H dense) and
    trho(phi) = (phi^2, psi_j) (N_H), both built from the fine quadrature."""
    fine = prob.fine
    Pc = prob.Pfull_c  # coarse dof -> fine vertex values

    def tri(wH):
        f = fine.at_qp(Pc @ wH)
        return (prob.P.T @ prob.mass_ii(f) @ prob.P).toarray()

    def trho(phiH):
        p = fine.at_qp(Pc @ phiH)
        return prob.P.T @ fine.load(p * p)[fine.interior]

    return tri, trho


def pieces(prob, U, w0, g, vxc):
    """Everything Algorithm 3 step 1 precomputes, per orbital i."""
    fine = prob.fine
    P = prob.P
    g_qp = fine.at_qp(g)
    Afix = 0.5 * prob.K + prob.mass_ii(prob.vext_qp + vxc + g_qp)
    Mw0 = prob.mass_ii(fine.at_qp(fine.full(w0)))
    out = dict(
        AH14=(P.T @ Afix @ P).toarray(),       # A_{H,1} + A_{H,4}
        G=(P.T @ Mw0 @ P).toarray(),           # A_{H,3} = G
        MH=(P.T @ prob.M @ P).toarray(),
        CH=(P.T @ prob.K @ P).toarray(),
        d=P.T @ (prob.K @ w0),
        zeta=float(w0 @ (prob.K @ w0)),
        liftH=P.T @ (prob.KIB @ g[fine.bverts]),
        liftT=float(w0 @ (prob.KIB @ g[fine.bverts])),
        b1=[], b3=[], c=[], beta1=[], beta3=[], gamma=[], Ah4=[], rhs=[])
    for i in range(U.shape[1]):
        u = U[:, i]
        uq = fine.at_qp(fine.full(u))
        out["b1"].append(P.T @ (Afix @ u))
        out["b3"].append(P.T @ (Mw0 @ u))          # = F_i
        out["c"].append(P.T @ (prob.M @ u))
        out["beta1"].append(float(u @ (Afix @ u)))
        out["beta3"].append(float(u @ (Mw0 @ u)))  # = g_{i,3}
        out["gamma"].append(float(u @ (prob.M @ u)))
        out["Ah4"].append((P.T @ prob.mass_ii(uq) @ P).toarray())
        out["rhs"].append(P.T @ fine.load(uq * uq)[fine.interior])
    return out


def augmented_from_pieces(pc, tri, i, wH, th1):
    """(K_i, M_i) of eq. Eigenvalue_H_h from the pieces (Algorithm 3 step 2 (a)-(c))."""
    AH = pc["AH14"] + tri(wH) + th1 * pc["G"]
    b = pc["b1"][i] + pc["Ah4"][i] @ wH + th1 * pc["b3"][i]
    beta = pc["beta1"][i] + pc["rhs"][i] @ wH + th1 * pc["beta3"][i]
    K = np.block([[AH, b[:, None]], [b[None, :], np.array([[beta]])]])
    M = np.block([[pc["MH"], pc["c"][i][:, None]], [pc["c"][i][None, :], np.array([[pc["gamma"][i]]])]])
    return K, M


def hartree_rhs_from_pieces(pc, trho, f, phiH, theta2):
    """[f_H; g] of eq. Hartree_H_h from the pieces (eqs. fH, gdef, FG)."""
    NH = pc["MH"].shape[0]
    fH = np.zeros(NH)
    gg = 0.0
    for i in range(len(f)):
        ph = phiH[:, i]
        t = theta2[i]
        fH += f[i] * (trho(ph) + 2.0 * t * (pc["Ah4"][i] @ ph) + t * t * pc["rhs"][i])
        gg += f[i] * (ph @ pc["G"] @ ph + 2.0 * t * (pc["b3"][i] @ ph) + t * t * pc["beta3"][i])
    return fH, gg
