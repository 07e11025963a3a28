"""Seeded synthetic workloads: nuclei, box, meshes, orbital counts.

These stand in for the paper's molecules (Section 4), whose geometries are not
given except for LiH. Everything here is an input recipe: random positions and
charges, mesh parameters and occupation numbers. No Kohn-Sham arithmetic.

Potential kinds:  0 = smoothed Coulomb -Z erf(r/rc)/r, 1 = bare Coulomb -Z/r,
                  2 = harmonic 0.5 omega^2 r^2 (no nuclei).
XC kinds:         0 = none, 1 = LDA (Slater exchange + Perdew-Zunger 1981
                  correlation), 2 = X-alpha.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .meshgen import graded_mesh, kuhn_mesh

POT_ERF, POT_BARE, POT_HARMONIC = 0, 1, 2
XC_NONE, XC_LDA, XC_XALPHA = 0, 1, 2


@dataclass
class System:
    name: str
    R: np.ndarray            # (M,3) nuclear positions
    Z: np.ndarray            # (M,) charges
    lo: float                # box [lo,hi]^3
    hi: float
    potential: int = POT_ERF
    rc: float = 0.5
    omega: float = 1.0
    n_orbitals: int = 1
    occupations: np.ndarray = field(default_factory=lambda: np.ones(1))
    xc: int = XC_LDA
    xalpha: float = 0.77298
    hartree: bool = True
    order: int = 1           # fine-space elements: 1 = P1 (the paper's), 2 = P2
    # meshes
    xyz: np.ndarray = None
    tets: np.ndarray = None
    cxyz: np.ndarray = None
    ctets: np.ndarray = None
    meta: dict = field(default_factory=dict)


def aufbau(n_electrons, n_orbitals):
    """Occupations: 2 per orbital from the bottom, 1 for an odd last electron,
    0 above. Spin-unpolarised (Section 2)."""
    f = np.zeros(n_orbitals)
    e = float(n_electrons)
    for i in range(n_orbitals):
        f[i] = min(2.0, max(0.0, e))
        e -= f[i]
    return f


def random_cluster(seed, n_atoms, half_width, d_min, z_choices=(1, 2, 3, 4)):
    """Positions uniform in [-a,a]^3 by rejection (pairwise distance >= d_min),
    then charges drawn uniformly from z_choices."""
    rng = np.random.default_rng(seed)
    pts = []
    tries = 0
    while len(pts) < n_atoms:
        p = rng.uniform(-half_width, half_width, 3)
        tries += 1
        if tries > 100000:
            raise RuntimeError("rejection sampling failed")
        if all(np.linalg.norm(p - q) >= d_min for q in pts):
            pts.append(p)
    R = np.array(pts)
    Z = rng.integers(min(z_choices), max(z_choices) + 1, size=n_atoms).astype(np.float64)
    return R, Z


def c1_hydrogen():
    """One smoothed nucleus Z=1 at the origin, rc=0.2, box [-10,10]^3, 16^3 Kuhn
    fine mesh (4913 vertices, 24576 tets), 8^3 coarse, 1 orbital, LDA."""
    xyz, tets = kuhn_mesh(16, -10.0, 10.0)
    cxyz, ctets = kuhn_mesh(8, -10.0, 10.0)
    return System(name="c1_hydrogen_16cubed", R=np.zeros((1, 3)), Z=np.ones(1), lo=-10.0, hi=10.0,
                  potential=POT_ERF, rc=0.2, n_orbitals=1, occupations=np.ones(1), xc=XC_LDA,
                  xyz=xyz, tets=tets, cxyz=cxyz, ctets=ctets,
                  meta={"fine": "kuhn16", "coarse": "kuhn8"})


def cluster_system(seed, n_atoms=4, half_width=3.0, d_min=1.5, box=15.0, rc=0.5,
                   n_base=8, h0=0.12, kappa=0.12, h_min=0.12, h_max=None, name=None,
                   n_orbitals=None, coarse=(1.4, 0.6, 1.4), progress=None):
    """A seeded cluster with a graded P1 mesh refined toward the nuclei.

    Defaults give the 4-atom workload: positions in [-3,3]^3, separation
    >= 1.5, Z in {1..4}, rc = 0.5, box [-15,15]^3, about 2e5 vertices."""
    R, Z = random_cluster(seed, n_atoms, half_width, d_min)
    ne = float(Z.sum())
    nocc = int(math.ceil(ne / 2.0))
    N = nocc if n_orbitals is None else int(n_orbitals)
    f = aufbau(ne, N)
    hm = (2 * box) / n_base * math.sqrt(3.0) if h_max is None else h_max
    cg = None if coarse is None else (coarse[0], coarse[1], coarse[2], hm)
    xyz, tets, cxyz, ctets = graded_mesh(n_base, -box, box, R, h0=h0, kappa=kappa, h_min=h_min, h_max=hm,
                                         coarse=cg, progress=progress)
    return System(name=name or f"cluster{n_atoms}_s{seed}", R=R, Z=Z, lo=-box, hi=box, potential=POT_ERF,
                  rc=rc, n_orbitals=N, occupations=f, xc=XC_LDA, xyz=xyz, tets=tets, cxyz=cxyz,
                  ctets=ctets, meta={"seed": seed, "n_base": n_base, "h0": h0, "kappa": kappa,
                                     "h_min": h_min, "coarse": coarse})


def c2_cluster(seed=0):
    """4-atom cluster, graded P1 mesh of about 2e5 vertices."""
    return cluster_system(seed, name=f"c2_cluster4_s{seed}")


def c3_cluster(seed=0, h=None, n_base=12, order=1, progress=None):
    """The 40-atom cluster: positions uniform in [-8,8]^3 with separation
    >= 1.8, Z in {1..4}, rc = 0.5, box [-25,25]^3, N = ceil(sum Z / 2)
    orbitals (52 for seed 0). The fine mesh is graded by bisection of the
    n_base^3 Kuhn base until the longest edge <= clip(h + h d, h, base edge).
    order 2 (the workload's P2 space): h = 0.199 by default, about 2.8e5
    vertices and 2.0e6 P2 DoFs. order 1: h = 0.101 by default, about 2.0e6
    vertices, a P1 mesh with the same DoF count. The coarse mesh is the base
    (11^3 interior vertices at n_base = 12)."""
    if h is None:
        h = 0.199 if order == 2 else 0.101
    S = cluster_system(seed, n_atoms=40, half_width=8.0, d_min=1.8, box=25.0, n_base=n_base, h0=h, kappa=h,
                       h_min=h, coarse=None, name=f"c3_cluster40_s{seed}" + ("_p2" if order == 2 else ""),
                       progress=progress)
    S.order = order
    return S


LIH_R = np.array([[-1.0075, 0.0, 0.0], [2.0075, 0.0, 0.0]])   # Li, H (Section 4, first model)
LIH_Z = np.array([3.0, 1.0])


def lih_system(n_base=16, h0=0.08, kappa=0.25, h_min=0.08, name="lih"):
    """The paper's first model (Section 4): Li (Z = 3) at (-1.0075, 0, 0) and
    H (Z = 1) at (2.0075, 0, 0), bare Coulomb potential, X-alpha exchange
    with alpha = 0.77298, box (-6, 6)^3, two doubly occupied orbitals. The
    coarse mesh is the n_base^3 Kuhn mesh (16^3: 24576 tets, the paper's
    coarsest mesh); the fine mesh refines it toward the nuclei until the
    longest edge <= clip(h0 + kappa d, h_min, base edge)."""
    hm = 12.0 / n_base * math.sqrt(3.0)
    xyz, tets, cxyz, ctets = graded_mesh(n_base, -6.0, 6.0, LIH_R, h0=h0, kappa=kappa, h_min=h_min, h_max=hm)
    return System(name=name, R=LIH_R.copy(), Z=LIH_Z.copy(), lo=-6.0, hi=6.0, potential=POT_BARE, n_orbitals=2,
                  occupations=np.array([2.0, 2.0]), xc=XC_XALPHA, xalpha=0.77298, xyz=xyz, tets=tets, cxyz=cxyz,
                  ctets=ctets, meta={"n_base": n_base, "h0": h0, "kappa": kappa, "h_min": h_min})


def lih_small():
    """LiH on an 8^3 coarse mesh with a mild grading: small enough for the
    checker to run whole steps."""
    return lih_system(n_base=8, h0=0.3, kappa=0.35, h_min=0.3, name="lih_small")


def c2_small(seed=0):
    """Same distribution as the 4-atom workload on a coarser grading (about
    1e4 vertices): small enough for the checker to run whole steps."""
    return cluster_system(seed, h0=0.5, kappa=0.45, h_min=0.5, name=f"c2small_cluster4_s{seed}")


def hydrogen_bare(n_fine, n_coarse, box=10.0):
    """Bare Coulomb Z=1 at the origin, no Hartree and no XC (linear problem
    whose ground state is -0.5 Ha in free space)."""
    xyz, tets = kuhn_mesh(n_fine, -box, box)
    cxyz, ctets = kuhn_mesh(n_coarse, -box, box)
    return System(name=f"h_bare_{n_fine}", R=np.zeros((1, 3)), Z=np.ones(1), lo=-box, hi=box,
                  potential=POT_BARE, n_orbitals=1, occupations=np.ones(1), xc=XC_NONE, hartree=False,
                  xyz=xyz, tets=tets, cxyz=cxyz, ctets=ctets)


def harmonic(n_fine, n_coarse, box=6.0, n_orbitals=4, omega=1.0):
    """Isotropic harmonic oscillator 0.5 r^2 (eigenvalues 1.5, 2.5 x3, 3.5 x6)."""
    xyz, tets = kuhn_mesh(n_fine, -box, box)
    cxyz, ctets = kuhn_mesh(n_coarse, -box, box)
    return System(name=f"harm_{n_fine}", R=np.zeros((0, 3)), Z=np.zeros(0), lo=-box, hi=box,
                  potential=POT_HARMONIC, omega=omega, n_orbitals=n_orbitals,
                  occupations=np.ones(n_orbitals), xc=XC_NONE, hartree=False,
                  xyz=xyz, tets=tets, cxyz=cxyz, ctets=ctets)


def tiny_system(n_fine=4, n_coarse=2, box=4.0, nonlinear=True, n_orbitals=2, seed=3, order=1):
    """A few-hundred-DoF mesh for brute-force checks (order 2: P2 on the same mesh)."""
    R, Z = random_cluster(seed, 2, 1.0, 1.0, z_choices=(1, 2))
    xyz, tets = kuhn_mesh(n_fine, -box, box)
    cxyz, ctets = kuhn_mesh(n_coarse, -box, box)
    ne = float(Z.sum())
    return System(name=f"tiny_{n_fine}", R=R, Z=Z, lo=-box, hi=box, potential=POT_ERF, rc=0.5,
                  n_orbitals=n_orbitals, occupations=aufbau(ne, n_orbitals),
                  xc=XC_LDA if nonlinear else XC_NONE, hartree=nonlinear, order=order,
                  xyz=xyz, tets=tets, cxyz=cxyz, ctets=ctets)


def batch_clusters(count, seed0=2000, atoms=(2, 8), h_range=(0.12, 0.24)):
    """Uneven independent clusters for batching: system k (seed seed0 + k)
    draws its atom count uniformly from atoms, its half-width 3 (n/4)^(1/3)
    bohr (the 4-atom value scaled to constant density), and its mesh size
    parameter h (h0 = kappa = h_min) uniformly from h_range, which spreads the
    meshes over roughly 3e4-2e5 vertices; N = ceil(sum Z / 2)."""
    out = []
    for k in range(count):
        seed = seed0 + k
        rng = np.random.default_rng(seed)
        na = int(rng.integers(atoms[0], atoms[1] + 1))
        h = float(rng.uniform(*h_range))
        hw = 3.0 * (na / 4.0) ** (1.0 / 3.0)
        out.append(cluster_system(seed, n_atoms=na, half_width=hw, d_min=1.5, h0=h, kappa=h, h_min=h,
                                  name=f"batch{k}_cluster{na}_s{seed}"))
    return out
