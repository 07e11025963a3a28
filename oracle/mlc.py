"""One outer iteration of Algorithm 1 (steps 5-7, with Algorithm 2 for step 7),
computed directly on the fine mesh. No Algorithm-3 decomposition is used here:
every augmented-space matrix is U^T H U with H assembled on the fine mesh.

Notation (Section 3): fine space V_h (interior P1 DoFs), coarse space V_H with
hat functions psi_k = sum_a P[a,k] phi_a (nested meshes), orbitals Phi
(n_dof x N, column i = orbital i), occupations f_i, Hartree potential w
(nodal values on every fine vertex, boundary included).

Readings where the paper is silent or inconsistent (each is also listed with
the design notes):
 * Step 5 operator is indefinite; it is solved shifted,
   (A + sigma M) u_i = (lambda_i + sigma) M phi_i, sigma = sigma0 - min_q V_eff.
   Scaling the right-hand side does not change span{u_i}.
 * u_i is M-normalised before the density of step 6 is formed.
 * Hartree Dirichlet data g (multipole of rho^l) are frozen in the outer step;
   the Hartree space is w = g_lift + P w_H + theta1 * w0, with w0 the
   zero-boundary solution of step 6 lifted by g, so (w_H, theta1) = (0, 1)
   is exactly the fine Hartree potential of rho~ (Algorithm 2 start).
 * Step (a) of Algorithm 2 keeps, among the lowest min(N_H+1, N+n_extra)
   eigenpairs of the augmented pencil, the eigenfunction with the largest
   component in span{u_i}: the largest |(phi, u_i)_M| (within a repeated
   eigenvalue, the normalised projection of u_i onto its eigenspace), ties to
   the lower eigenvalue, sign so that (phi, u_i)_M > 0.
 * The stopping norm of Algorithm 2 step (c) is the H^1 norm.
 * Algorithm 2 is a fixed-point iteration in the Hartree coefficients
   x = (w_H, theta1). Run as printed (x_in <- x_out) it oscillates on
   multi-electron clusters, so by default the next input is chosen by
   Anderson (Pulay) mixing of the last few (x_in, x_out - x_in) pairs in the
   energy inner product <a, b> = a^T (V^T K V) b of W_{H,h}; mixing changes
   only the path, not the fixed point. inner_mix_history = 0 gives the
   printed iteration.
 * The V_xc term enters with a plus sign throughout.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.sparse.linalg import splu

from . import hartree as har
from . import xc as xcmod
from .fem import Mesh, make_mesh, prolongation
from .potentials import v_ext


@dataclass
class Options:
    sigma0: float = 1.0
    shift: bool = True          # False: the unshifted problem exactly as printed
    inner_tol: float = 1e-12
    inner_maxit: int = 500
    n_extra: int = 8
    solver: str = "lu"          # "lu" (exact) or "pcg"
    inner_mix_history: int = 6  # Anderson history of the inner iteration; 0 = plain (as printed)
    inner_mix_beta: float = 0.5
    variant: str = "eigenpairwise"  # or "joint": one augmented space for all orbitals
    pcg_rtol: float = 1e-13


@dataclass
class State:
    lam: np.ndarray      # (N,)
    Phi: np.ndarray      # (n_dof, N) fine interior coefficients
    w: np.ndarray        # (nv,) fine nodal Hartree potential


@dataclass
class StepResult:
    state: State
    rho_qp: np.ndarray
    rho_nodal: np.ndarray
    energy: float
    max_offdiag_overlap: float
    rho_integral: float
    inner_iters: int
    inter: dict = field(default_factory=dict)


class Problem:
    """Meshes, spaces and the fixed fine matrices of one workload."""

    def __init__(self, system):
        self.sys = system
        self.fine = make_mesh(system.xyz, system.tets, system.lo, system.hi, getattr(system, "order", 1))
        self.coarse = Mesh(system.cxyz, system.ctets, system.lo, system.hi)
        self.Pfull, self.P = prolongation(self.fine, self.coarse)
        self.Pfull_c = self.Pfull[:, self.coarse.interior].tocsr()   # coarse dof -> all fine vertices
        self.Kfull = self.fine.stiffness()
        self.Mfull = self.fine.mass()
        self.K = self.fine.ii(self.Kfull)
        self.M = self.fine.ii(self.Mfull)
        self.KIB = self.fine.ib(self.Kfull)
        self.vext_qp = v_ext(self.fine.qp, system.R, system.Z, system.potential, system.rc, system.omega)
        self.f = np.asarray(system.occupations, dtype=np.float64)
        self.N = int(system.n_orbitals)
        self.NH = self.coarse.n_dof
        self.hartree = bool(system.hartree)

    def density_qp(self, Phi):
        """rho(q) = sum_i f_i phi_i(q)^2 at the fine quadrature points."""
        ph = self.fine.at_qp(self.fine.full(Phi))        # (nt,4,N)
        return np.einsum("tqi,i->tq", ph * ph, self.f)

    def mass_ii(self, f_qp):
        return self.fine.ii(self.fine.mass(f_qp))


def _solve_spd(A, B, opts, x0=None):
    if opts.solver == "lu":
        lu = splu(A.tocsc())
        return lu.solve(B)
    from .pcg import jacobi_pcg
    X, _ = jacobi_pcg(A, B, x0=x0, rtol=opts.pcg_rtol, maxit=100000)
    return X


def fine_stage(prob: Problem, st: State, opts: Options):
    """Steps O1-O7: density, XC, boundary data, operator, N shifted BVPs and
    the Hartree direction. Returns a dict of the intermediate quantities."""
    fine = prob.fine
    S = prob.sys
    # O1-O2: density and XC at quadrature points (Algorithm 1, V_xc(rho^l))
    rho = prob.density_qp(st.Phi)
    exc, vxc = xcmod.evaluate(S.xc, rho, S.xalpha)
    # O3: multipole boundary data of rho^l, frozen for this outer step
    if prob.hartree:
        g = har.boundary_data(fine, rho)
    else:
        g = np.zeros(fine.nv)
    # O4: V_eff and the operator of the auxiliary problem (eq. Aux_Linear_Problem)
    w_qp = fine.at_qp(st.w)
    veff = prob.vext_qp + w_qp + vxc
    A = 0.5 * prob.K + prob.mass_ii(veff)
    sigma = opts.sigma0 - float(veff.min()) if opts.shift else 0.0
    # O5: (A + sigma M) u_i = (lambda_i + sigma) M phi_i
    B = (prob.M @ st.Phi) * (st.lam + sigma)[None, :]
    U = _solve_spd(A + sigma * prob.M, B, opts, x0=st.Phi)
    U = np.atleast_2d(U.T).T if U.ndim == 1 else U
    # O6: M-normalise
    nrm = np.sqrt(np.einsum("ai,ai->i", U, prob.M @ U))
    U = U / nrm[None, :]
    # O7: Hartree direction (eq. W_h_equation), lifted by g
    if prob.hartree:
        rho_t = prob.density_qp(U)
        w0 = har.poisson(fine, prob.Kfull, rho_t, g)
    else:
        rho_t = None
        w0 = np.zeros(fine.n_dof)
    return dict(rho=rho, exc=exc, vxc=vxc, g=g, veff=veff, sigma=sigma, A=A, B=B, U=U,
                rho_tilde=rho_t, w0=w0)


def augmented_blocks(prob: Problem, U, w0, g, vxc):
    """The fine integrals that define the augmented problems (eqs. Eigenvalue_H_h
    and Hartree_H_h) at (w_H, theta1), written as products with fine
    matrices: A_fix = 1/2 K + M_{V_ext + V_xc + g}, M_{w0}, M, K."""
    fine = prob.fine
    g_qp = fine.at_qp(g)
    Afix = 0.5 * prob.K + prob.mass_ii(prob.vext_qp + vxc + g_qp)
    Mw0 = prob.mass_ii(fine.at_qp(fine.full(w0))) if prob.hartree else None
    return Afix, Mw0


def select_eigenpair(evals, evecs, Mi, n_keep, tol=1e-12):
    """Algorithm 2 (a): among the lowest n_keep eigenpairs of the augmented
    pencil (M_i-orthonormal eigenvectors in the basis [P, u_i]), the
    eigenfunction with the largest component in span{u_i}, that is the
    largest |(phi, u_i)_M| over unit eigenfunctions phi. Within an eigenvalue
    of multiplicity above one (eigenvalues equal to tol relative) the maximum
    is taken by the normalised projection of u_i onto the eigenspace, whose
    norm is the value. Ties (values equal to 1e-10 relative) go to the lower
    eigenvalue; the sign makes (phi, u_i)_M positive."""
    e = Mi[:, -1]                       # (x, u_i)_M = x . M_i[:, -1]: u_i is the last basis function
    c = evecs[:, :n_keep].T @ e
    best, j0, k0 = -1.0, 0, 1
    j = 0
    while j < n_keep:
        k = j + 1
        while k < n_keep and abs(evals[k] - evals[j]) <= tol * max(1.0, abs(evals[j])):
            k += 1
        nrm = float(np.linalg.norm(c[j:k]))
        if nrm > best * (1.0 + 1e-10):
            best, j0, k0 = nrm, j, k
        j = k
    x = evecs[:, j0:k0] @ c[j0:k0] / best
    return float(evals[j0]), x


def anderson_next(x_in, F, hist, G, m, beta):
    """Next input of a fixed-point iteration x -> x + F(x) by Anderson (Pulay)
    mixing: with the differences dX, dF of the last m+1 inputs and residuals,
    gamma minimises |F - dF gamma| in the inner product <a, b> = a^T G b, and
    x_next = (x_in - dX gamma) + beta (F - dF gamma). With no history (first
    call) it is the damped step x_in + beta F. hist is a list of (x, F) pairs
    kept by the caller; this call appends the current pair."""
    hist.append((x_in.copy(), F.copy()))
    if len(hist) > m + 1:
        hist.pop(0)
    if len(hist) == 1:
        return x_in + beta * F
    dX = np.array([hist[k + 1][0] - hist[k][0] for k in range(len(hist) - 1)]).T
    dF = np.array([hist[k + 1][1] - hist[k][1] for k in range(len(hist) - 1)]).T
    A = dF.T @ G @ dF
    r = dF.T @ G @ F
    gam = np.linalg.lstsq(A, r, rcond=1e-12)[0]
    return (x_in - dX @ gam) + beta * (F - dF @ gam)


def inner_scf(prob: Problem, fs: dict, opts: Options, x_start=None):
    """Algorithm 2 with every matrix assembled on the fine mesh. x_start: the
    starting Hartree coefficients (w_H, theta1); default (0, 1)."""
    fine = prob.fine
    P = prob.P
    U, w0, g = fs["U"], fs["w0"], fs["g"]
    Afix, Mw0 = augmented_blocks(prob, U, w0, g, fs["vxc"])
    N, NH = prob.N, prob.NH
    n_keep = min(NH + 1, N + opts.n_extra)
    # fixed Hartree pieces of W_{H,h} = V_H + span{w0}, lifted by g
    if prob.hartree:
        V = sp.hstack([P, sp.csr_matrix(w0[:, None])]).tocsr()
        VKV = (V.T @ prob.K @ V).toarray()
        lift = V.T @ (prob.KIB @ g[fine.bverts])
    # Hartree coefficients x = (w_H, theta1), starting from (0, 1)
    x_in = np.zeros(NH + 1)
    x_in[-1] = 1.0 if prob.hartree else 0.0
    if x_start is not None:
        x_in = np.array(x_start, dtype=np.float64)
    hist = []
    Phi_s = U.copy()
    KpM = prob.K + prob.M
    lam = np.zeros(N)
    thetas = np.zeros(N)
    phiH = np.zeros((NH, N))
    PMP = (P.T @ prob.M @ P).toarray()
    its = 0
    for s in range(opts.inner_maxit):
        its = s + 1
        wH, th1 = x_in[:-1], float(x_in[-1])
        # (a) N small linear eigenproblems in S_{H,h} = V_H + span{u_i}
        H = Afix + prob.mass_ii(fine.at_qp(prob.Pfull_c @ wH))
        if prob.hartree:
            H = H + th1 * Mw0
        PHP = (P.T @ H @ P).toarray()
        Phi_new = np.zeros_like(Phi_s)
        for i in range(N):
            u = U[:, i]
            Hu = H @ u
            Mu = prob.M @ u
            Ki = np.block([[PHP, (P.T @ Hu)[:, None]], [(P.T @ Hu)[None, :], np.array([[u @ Hu]])]])
            Mi = np.block([[PMP, (P.T @ Mu)[:, None]], [(P.T @ Mu)[None, :], np.array([[u @ Mu]])]])
            ev, X = sla.eigh(Ki, Mi, subset_by_index=[0, n_keep - 1])
            lam[i], x = select_eigenpair(ev, X, Mi, n_keep)
            phiH[:, i] = x[:-1]
            thetas[i] = x[-1]
            Phi_new[:, i] = P @ x[:-1] + x[-1] * u
        # (b) Hartree problem in W_{H,h} for the new orbitals
        if prob.hartree:
            rho = prob.density_qp(Phi_new)
            rhs = 4.0 * np.pi * (V.T @ fine.load(rho)[fine.interior]) - lift
            x_out = np.linalg.solve(VKV, rhs)
        else:
            x_out = x_in
        # (c) stopping test in the H^1 norm
        D = Phi_new - Phi_s
        diff = float(np.sqrt(np.einsum("ai,ai->", D, KpM @ D)))
        Phi_s = Phi_new
        if not prob.hartree or diff < opts.inner_tol or s == opts.inner_maxit - 1:
            x_in = x_out
            break
        # next Hartree input: as printed (x_out), or mixed
        if opts.inner_mix_history > 0:
            x_in = anderson_next(x_in, x_out - x_in, hist, VKV, opts.inner_mix_history, opts.inner_mix_beta)
        else:
            x_in = x_out
    wH, th1 = x_in[:-1].copy(), float(x_in[-1])
    return dict(lam=lam.copy(), Phi=Phi_s, wH=wH, th1=th1, phiH=phiH, theta2=thetas, inner_iters=its,
                Afix=Afix, Mw0=Mw0, last_diff=diff)


def inner_scf_joint(prob: Problem, fs: dict, opts: Options, x_start=None):
    """The joint-space variant the paper compares against (the earlier
    multilevel correction method, Section 2): Algorithm 2 with step (a)
    replaced by one eigenproblem in V_H + span{u_1, ..., u_N} whose lowest N
    eigenpairs are the new orbitals (M-orthonormal by construction); the
    Hartree step, the mixing and the stopping test as in inner_scf. The sign
    of each orbital follows the previous inner iterate ((phi^{s+1},
    phi^s)_M > 0; the u_i for the first)."""
    fine = prob.fine
    P = prob.P
    U, w0, g = fs["U"], fs["w0"], fs["g"]
    Afix, Mw0 = augmented_blocks(prob, U, w0, g, fs["vxc"])
    N, NH = prob.N, prob.NH
    W = sp.hstack([P, sp.csr_matrix(U)]).tocsr()             # basis [P, u_1..u_N]
    Mj = (W.T @ prob.M @ W).toarray()
    KMj = (W.T @ (prob.K + prob.M) @ W).toarray()
    if prob.hartree:
        V = sp.hstack([P, sp.csr_matrix(w0[:, None])]).tocsr()
        VKV = (V.T @ prob.K @ V).toarray()
        lift = V.T @ (prob.KIB @ g[fine.bverts])
    x_in = np.zeros(NH + 1)
    x_in[-1] = 1.0 if prob.hartree else 0.0
    if x_start is not None:
        x_in = np.array(x_start, dtype=np.float64)
    hist = []
    X_old = np.zeros((NH + N, N))
    X_old[NH:, :] = np.eye(N)                                # the first iterate: u_i
    its = 0
    for s in range(opts.inner_maxit):
        its = s + 1
        wH, th1 = x_in[:-1], float(x_in[-1])
        H = Afix + prob.mass_ii(fine.at_qp(prob.Pfull_c @ wH))
        if prob.hartree:
            H = H + th1 * Mw0
        Kj = (W.T @ H @ W).toarray()
        lam, X = sla.eigh(Kj, Mj, subset_by_index=[0, N - 1])
        sgn = np.sign(np.einsum("ai,ai->i", X, Mj @ X_old))
        X = X * np.where(sgn == 0, 1.0, sgn)[None, :]
        Phi_new = P @ X[:NH] + U @ X[NH:]
        if prob.hartree:
            rho = prob.density_qp(Phi_new)
            rhs = 4.0 * np.pi * (V.T @ fine.load(rho)[fine.interior]) - lift
            x_out = np.linalg.solve(VKV, rhs)
        else:
            x_out = x_in
        Dx = X - X_old
        diff = float(np.sqrt(np.einsum("ai,ai->", Dx, KMj @ Dx)))
        X_old = X
        if not prob.hartree or diff < opts.inner_tol or s == opts.inner_maxit - 1:
            x_in = x_out
            break
        if opts.inner_mix_history > 0:
            x_in = anderson_next(x_in, x_out - x_in, hist, VKV, opts.inner_mix_history, opts.inner_mix_beta)
        else:
            x_in = x_out
    wH, th1 = x_in[:-1].copy(), float(x_in[-1])
    return dict(lam=lam.copy(), Phi=P @ X_old[:NH] + U @ X_old[NH:], wH=wH, th1=th1, phiH=X_old[:NH].copy(),
                D=X_old[NH:].copy(), theta2=np.diag(X_old[NH:]).copy(), inner_iters=its, Afix=Afix, Mw0=Mw0,
                last_diff=diff)


def correction_step(prob: Problem, st: State, opts: Options = None) -> StepResult:
    """One outer step l -> l+1 (Algorithm 1 steps 5-7). Outputs follow
    Algorithm 3 step 3: phi_i = phi_{i,H} + theta2_i u_i, and the Hartree
    potential w = g + P w_H + theta1 w0 on every fine vertex."""
    opts = opts or Options()
    fs = fine_stage(prob, st, opts)
    inn = inner_scf_joint(prob, fs, opts) if opts.variant == "joint" else inner_scf(prob, fs, opts)
    fine = prob.fine
    Phi = inn["Phi"]
    w = fs["g"] + prob.Pfull_c @ inn["wH"] + inn["th1"] * fine.full(fs["w0"])
    rho = prob.density_qp(Phi)
    rho_nodal = fine.full(Phi) ** 2 @ prob.f
    exc_new, _ = xcmod.evaluate(prob.sys.xc, rho, prob.sys.xalpha)
    w_qp = fine.at_qp(w)
    energy = float(prob.f @ inn["lam"] - 0.5 * fine.integrate(w_qp * rho)
                   + fine.integrate(rho * (exc_new - fs["vxc"])))
    G = Phi.T @ (prob.M @ Phi)
    off = G - np.diag(np.diag(G))
    return StepResult(state=State(lam=inn["lam"], Phi=Phi, w=w), rho_qp=rho, rho_nodal=rho_nodal,
                      energy=energy, max_offdiag_overlap=float(np.abs(off).max()) if prob.N > 1 else 0.0,
                      rho_integral=fine.integrate(rho), inner_iters=inn["inner_iters"],
                      inter=dict(fine=fs, inner=inn))
