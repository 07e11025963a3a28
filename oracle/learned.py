"""Learned initial guess for the step-5 solves, FP64 reference.

TEST INFRASTRUCTURE ONLY (see the package header).

The method starts each auxiliary problem of step 5 (Algorithm 1) from the
current orbital phi_i. The extension proposes a correction direction
    delta_i = s_i * NN(features),   s_i = max |phi_i| over the DoFs,
with NN one small network applied to every (DoF, orbital) row and trained on
solutions the method itself produced, and starts from the best point of
span{phi_i, delta_i} for the energy J(x) = 1/2 x^T A x - b^T x of the SPD
step-5 problem (a 2 x 2 Galerkin solve per column): x0 = a phi_i + b delta_i.
J(x) - J(u) = 1/2 |x - u|_A^2, so this start is never farther from the
solution in the A-norm than phi_i itself (a = 1, b = 0 is in the span); the
plain start phi_i stays the fallback and the judge (kept where
J(x0) >= J(phi_i), or where the 2 x 2 system is singular).

Network: 6 -> 64 -> 64 -> 64 -> 1, GELU (erf form) after each hidden layer,
linear output. Parameters are packed in one vector, in this order:
    W1 (64 x 6, row-major: out x in), b1 (64), W2 (64 x 64), b2, W3 (64 x 64),
    b3, W4 (1 x 64), b4 (1)                                      = 8833 values.
Loss: mean over rows of (y - t)^2. Gradients by the chain rule, written out
below and pinned against central differences in the tests. Adam: Kingma and
Ba, "Adam: a method for stochastic optimization" (2015), with bias
correction.

bf16=True rounds, to bfloat16 (round to nearest, ties to even), exactly the
operands that enter a BF16 matrix product in the GPU kernels: the inputs x,
W1..W3, the hidden activations h1, h2 (inputs of layers 2 and 3), and in the
backward pass the pre-activation gradients dz1..dz3 and the transposed
weights. The output layer (W4, h3), biases, GELU and all accumulation stay
unrounded, as in the kernels (which accumulate in FP32).

Features of row (i, c) (DoF i, orbital c), all from the state before the
step and the step-5 operator A = A_l + sigma M, right-hand side
b_c = (lambda_c + sigma) M phi_c and its diagonal D:
    0  V_eff at the vertex: V_ext(x_i) + w(x_i) + V_xc(rho(x_i)),
       rho(x_i) = sum_c f_c phi_c(x_i)^2 (nodal values), clipped to
       [-50, 50] hartree (a bare Coulomb nucleus on a vertex is infinite)
    1  phi_ic / s_c
    2  r0_ic / s_c,  r0 = D^{-1} (b - A phi)  (Jacobi-scaled initial residual)
    3-5  distances from x_i to the three nearest nuclei, ascending, divided
       by 10 bohr (missing nuclei: the box diagonal, divided likewise)
Target of row (i, c): (u_ic - phi_ic) / s_c with u the converged step-5
solution before its M-normalisation.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

N_IN, N_HID = 6, 64
SIZES = [(64, 6), (64,), (64, 64), (64,), (64, 64), (64,), (1, 64), (1,)]
N_PARAMS = sum(int(np.prod(s)) for s in SIZES)  # 8833
DIST_SCALE = 10.0


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == N_PARAMS
    out, k = [], 0
    for s in SIZES:
        m = int(np.prod(s))
        out.append(theta[k:k + m].reshape(s))
        k += m
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def bf16(a):
    """Round to bfloat16 (nearest, ties to even) through float32; returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    nan = np.isnan(f)
    out = r.view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_prime(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(theta, X, bf=False, keep=False):
    """Outputs y (rows) for inputs X (rows x 6)."""
    rnd = bf16 if bf else (lambda a: a)
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    x = rnd(np.asarray(X, dtype=np.float64))
    z1 = x @ rnd(W1).T + b1
    h1 = gelu(z1)
    z2 = rnd(h1) @ rnd(W2).T + b2
    h2 = gelu(z2)
    z3 = rnd(h2) @ rnd(W3).T + b3
    h3 = gelu(z3)
    y = h3 @ W4[0] + b4[0]
    if keep:
        return y, dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, h3=h3)
    return y


def loss_grad(theta, X, t, bf=False):
    """Loss (mean squared error) and its gradient with respect to theta."""
    rnd = bf16 if bf else (lambda a: a)
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    y, c = forward(theta, X, bf=bf, keep=True)
    m = len(y)
    e = y - np.asarray(t, dtype=np.float64)
    loss = float(np.mean(e * e))
    dy = 2.0 * e / m                              # d loss / d y
    gW4 = (dy @ c["h3"])[None, :]                 # output layer: unrounded
    gb4 = np.array([dy.sum()])
    dz3 = np.outer(dy, W4[0]) * gelu_prime(c["z3"])
    gW3 = rnd(dz3).T @ rnd(c["h2"])
    gb3 = dz3.sum(axis=0)
    dz2 = (rnd(dz3) @ rnd(W3)) * gelu_prime(c["z2"])
    gW2 = rnd(dz2).T @ rnd(c["h1"])
    gb2 = dz2.sum(axis=0)
    dz1 = (rnd(dz2) @ rnd(W2)) * gelu_prime(c["z1"])
    gW1 = rnd(dz1).T @ c["x"]
    gb1 = dz1.sum(axis=0)
    return loss, pack([gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4])


class Adam:
    """theta <- theta - lr * mhat / (sqrt(vhat) + eps), with m, v the bias-
    corrected first and second moment estimates of the gradient."""

    def __init__(self, theta, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.theta = np.array(theta, dtype=np.float64)
        self.m = np.zeros_like(self.theta)
        self.v = np.zeros_like(self.theta)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, g):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mhat = self.m / (1.0 - self.b1 ** self.t)
        vhat = self.v / (1.0 - self.b2 ** self.t)
        self.theta = self.theta - self.lr * mhat / (np.sqrt(vhat) + self.eps)
        return self.theta


VEFF_CLIP = 50.0


def veff_nodal(system, pts, w, Phi):
    """Feature 0 at the points pts (DoF coordinates): clipped V_ext + w + V_xc(rho)."""
    from .potentials import v_ext
    from .xc import evaluate
    rho = (np.asarray(Phi) ** 2) @ np.asarray(system.occupations, dtype=np.float64)
    with np.errstate(divide="ignore"):
        v = v_ext(pts, system.R, system.Z, system.potential, system.rc, system.omega)
    v = v + np.asarray(w) + evaluate(system.xc, rho, system.xalpha)[1]
    return np.clip(v, -VEFF_CLIP, VEFF_CLIP)


def nearest_distances(pts, R, diag):
    """Three smallest distances from each point to the nuclei R, ascending;
    missing ones are diag."""
    pts = np.asarray(pts, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    out = np.full((len(pts), 3), float(diag))
    if len(R):
        d = np.sqrt(((pts[:, None, :] - R[None, :, :]) ** 2).sum(axis=2))
        d.sort(axis=1)
        k = min(3, d.shape[1])
        out[:, :k] = d[:, :k]
    return out


def features(Phi, APhi, B, dinv, veff, dof_xyz, R, diag):
    """Rows (i * N + c) x 6 as listed in the module header; also returns s."""
    Phi = np.asarray(Phi, dtype=np.float64)
    n, N = Phi.shape
    s = np.abs(Phi).max(axis=0)
    s = np.where(s > 0, s, 1.0)
    r0 = np.asarray(dinv)[:, None] * (np.asarray(B) - np.asarray(APhi))
    d = nearest_distances(dof_xyz, R, diag) / DIST_SCALE
    F = np.zeros((n, N, N_IN))
    F[:, :, 0] = np.asarray(veff)[:, None]
    F[:, :, 1] = Phi / s
    F[:, :, 2] = r0 / s
    F[:, :, 3:6] = d[:, None, :]
    return F.reshape(n * N, N_IN), s


def targets(U, Phi, s):
    """(u_ic - phi_ic) / s_c per row (i * N + c)."""
    return ((np.asarray(U) - np.asarray(Phi)) / s).reshape(-1)


def galerkin_start(A, B, Phi, D):
    """Per column the minimiser of J over span{phi, delta}; returns x0, the
    per-column flags (True where the combination is used) and the
    coefficients (a, b). phi is kept where the 2 x 2 system is singular, where
    J does not drop, or where the minimiser's residual |b - A x0| exceeds
    phi's (a start closer in the A-norm can still carry a larger residual,
    and CG's stopping test is on the residual)."""
    Phi, D, B = np.asarray(Phi), np.asarray(D), np.asarray(B)
    AP, AD = A @ Phi, A @ D
    X = Phi.copy()
    used = np.zeros(Phi.shape[1], dtype=bool)
    coef = np.tile([1.0, 0.0], (Phi.shape[1], 1))
    for c in range(Phi.shape[1]):
        G = np.array([[Phi[:, c] @ AP[:, c], Phi[:, c] @ AD[:, c]], [D[:, c] @ AP[:, c], D[:, c] @ AD[:, c]]])
        r = np.array([B[:, c] @ Phi[:, c], B[:, c] @ D[:, c]])
        det = G[0, 0] * G[1, 1] - G[0, 1] * G[1, 0]
        if not det > 1e-12 * G[0, 0] * G[1, 1]:
            continue
        a = (r[0] * G[1, 1] - r[1] * G[0, 1]) / det
        b = (G[0, 0] * r[1] - G[1, 0] * r[0]) / det
        j_phi = 0.5 * G[0, 0] - r[0]
        j_new = 0.5 * (a * a * G[0, 0] + 2 * a * b * G[0, 1] + b * b * G[1, 1]) - (a * r[0] + b * r[1])
        res_new = np.linalg.norm(B[:, c] - (a * AP[:, c] + b * AD[:, c]))
        res_phi = np.linalg.norm(B[:, c] - AP[:, c])
        if j_new < j_phi and res_new <= res_phi:
            X[:, c] = a * Phi[:, c] + b * D[:, c]
            used[c] = True
            coef[c] = (a, b)
    return X, used, coef


def guess(theta, F, Phi, s, A, B, bf=False):
    """The learned start: delta = s * NN(features), then the Galerkin start."""
    n, N = np.asarray(Phi).shape
    D = forward(theta, F, bf=bf).reshape(n, N) * s
    return galerkin_start(A, B, Phi, D)
