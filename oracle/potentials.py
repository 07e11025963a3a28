"""External potentials.

Section 2 defines V_ext = -sum_k Z_k / |x - R_k| (bare Coulomb). The
workloads also use the smoothed form -Z erf(|x-R|/rc)/|x-R| (whose value at
r = 0 is -2 Z / (sqrt(pi) rc)) and, as a closed-form check, the harmonic
well 0.5 omega^2 |x|^2.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

POT_ERF, POT_BARE, POT_HARMONIC = 0, 1, 2


def v_ext(points, R, Z, kind, rc=0.5, omega=1.0):
    x = np.asarray(points, dtype=np.float64)
    shp = x.shape[:-1]
    x = x.reshape(-1, 3)
    v = np.zeros(len(x))
    if kind == POT_HARMONIC:
        v = 0.5 * omega ** 2 * np.einsum("ij,ij->i", x, x)
        return v.reshape(shp)
    for Rk, Zk in zip(np.asarray(R).reshape(-1, 3), np.asarray(Z).ravel()):
        r = np.linalg.norm(x - Rk, axis=1)
        if kind == POT_BARE:
            v -= Zk / r
        elif kind == POT_ERF:
            small = r < 1e-12
            rr = np.where(small, 1.0, r)
            v -= np.where(small, Zk * 2.0 / (np.sqrt(np.pi) * rc), Zk * erf(rr / rc) / rr)
        else:
            raise ValueError(kind)
    return v.reshape(shp)
