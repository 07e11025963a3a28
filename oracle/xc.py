"""Exchange-correlation functionals of Section 4 (models 1-5).

LDA: Slater exchange eps_x = -(3/4)(3/pi)^(1/3) rho^(1/3) (the paper prints
rho^(1/2); we read rho^(1/3), which is what its own remark on V_xc and the
X-alpha formula imply), Perdew-Zunger 1981 correlation eps_c(r_s) with the
constants printed in Section 4, r_s = (3/(4 pi rho))^(1/3), and
V_xc = eps_xc + rho d eps_xc / d rho.

The potential is obtained here exactly as the paper defines it: from the
derivative of the printed energy density. With d r_s/d rho = -r_s/(3 rho),
rho d eps/d rho = -(r_s/3) d eps/d r_s.

X-alpha (models 1-2): V_xc = -(3/2) alpha (3 rho / pi)^(1/3), alpha = 0.77298;
its energy density is the one whose rho-derivative gives that potential,
eps = (3/4) V_xc.

Densities at or below 1e-30 give zero energy density and potential.
"""
from __future__ import annotations

import numpy as np

PZ_GAMMA, PZ_BETA1, PZ_BETA2 = -0.1423, 1.0529, 0.3334
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116
RHO_FLOOR = 1e-30


def _rs(rho):
    return (3.0 / (4.0 * np.pi * rho)) ** (1.0 / 3.0)


def eps_x(rho):
    return -0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * rho ** (1.0 / 3.0)


def deps_x_drho(rho):
    return -0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * (1.0 / 3.0) * rho ** (-2.0 / 3.0)


def eps_c_of_rs(rs):
    rs = np.asarray(rs, dtype=np.float64)
    hi = PZ_GAMMA / (1.0 + PZ_BETA1 * np.sqrt(rs) + PZ_BETA2 * rs)
    with np.errstate(divide="ignore", invalid="ignore"):
        lo = PZ_A * np.log(rs) + PZ_B + PZ_C * rs * np.log(rs) + PZ_D * rs
    return np.where(rs >= 1.0, hi, lo)


def deps_c_drs(rs):
    rs = np.asarray(rs, dtype=np.float64)
    den = 1.0 + PZ_BETA1 * np.sqrt(rs) + PZ_BETA2 * rs
    hi = -PZ_GAMMA * (0.5 * PZ_BETA1 / np.sqrt(rs) + PZ_BETA2) / den ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        lo = PZ_A / rs + PZ_C * (np.log(rs) + 1.0) + PZ_D
    return np.where(rs >= 1.0, hi, lo)


def lda(rho):
    """Returns (eps_xc, v_xc) for the LDA of Section 4 (model 3)."""
    rho = np.asarray(rho, dtype=np.float64)
    ok = rho > RHO_FLOOR
    r = np.where(ok, rho, 1.0)
    rs = _rs(r)
    ex = eps_x(r)
    vx = ex + r * deps_x_drho(r)
    ec = eps_c_of_rs(rs)
    vc = ec - (rs / 3.0) * deps_c_drs(rs)
    return np.where(ok, ex + ec, 0.0), np.where(ok, vx + vc, 0.0)


def xalpha(rho, alpha=0.77298):
    """Returns (eps_xc, v_xc) for X-alpha (models 1-2)."""
    rho = np.asarray(rho, dtype=np.float64)
    ok = rho > RHO_FLOOR
    r = np.where(ok, rho, 1.0)
    v = -1.5 * alpha * (3.0 * r / np.pi) ** (1.0 / 3.0)
    return np.where(ok, 0.75 * v, 0.0), np.where(ok, v, 0.0)


def evaluate(kind, rho, alpha=0.77298):
    """kind: 0 none, 1 LDA, 2 X-alpha."""
    if kind == 0:
        z = np.zeros_like(np.asarray(rho, dtype=np.float64))
        return z, z.copy()
    if kind == 1:
        return lda(rho)
    if kind == 2:
        return xalpha(rho, alpha)
    raise ValueError(kind)
