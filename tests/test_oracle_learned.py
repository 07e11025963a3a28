"""Pins of the learned-guess checker (oracle/learned.py) against facts that do
not come from the checker itself: exact bfloat16 roundings, closed forms of
GELU and of the network with zeroed layers, an explicit-loop evaluation,
central differences of the loss, the first Adam step in closed form and
Adam's convergence on a quadratic, a zero residual feature at an exact
discrete eigenpair, and brute-force nearest-nucleus distances."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import learned as Lr


def test_bf16_rounding_exact_values():
    # ulp of bfloat16 at 1 is 2^-7; halfway cases go to the even mantissa
    got = Lr.bf16(np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, math.pi, -2.0 ** -130, 65504.0, 0.0]))
    want = [1.0, 1.0, 1 + 2 ** -6, 3.140625, -2.0 ** -130, 65536.0, 0.0]
    assert np.array_equal(got, np.array(want))
    assert np.isnan(Lr.bf16(np.array([np.nan])))[0]


def test_gelu_closed_forms():
    # GELU(z) = z Phi(z) with Phi the standard normal CDF; Phi(1) = 0.841344746068543
    assert Lr.gelu(np.array([0.0]))[0] == 0.0
    assert abs(Lr.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    assert abs(Lr.gelu(np.array([-1.0]))[0] + 0.15865525393145707) < 1e-15
    assert abs(Lr.gelu_prime(np.array([0.0]))[0] - 0.5) < 1e-15
    z = np.linspace(-4, 4, 33)
    h = 1e-6
    fd = (Lr.gelu(z + h) - Lr.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - Lr.gelu_prime(z))) < 1e-9


def _theta(seed, scale=0.4):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, Lr.N_PARAMS)


def test_param_count_and_packing():
    assert Lr.N_PARAMS == 8833
    th = _theta(0)
    assert np.array_equal(Lr.pack(Lr.unpack(th)), th)


def test_forward_with_zeroed_layers_is_constant():
    # W2 = W3 = 0: h3 = GELU(b3) whatever the input, y = W4 . GELU(b3) + b4
    W1, b1, W2, b2, W3, b3, W4, b4 = Lr.unpack(_theta(1))
    W2[:] = 0.0
    W3[:] = 0.0
    th = Lr.pack([W1, b1, W2, b2, W3, b3, W4, b4])
    X = np.random.default_rng(2).normal(size=(5, 6))
    want = sum(W4[0, k] * 0.5 * b3[k] * (1 + math.erf(b3[k] / math.sqrt(2))) for k in range(64)) + b4[0]
    assert np.max(np.abs(Lr.forward(th, X) - want)) < 1e-12


def test_forward_matches_explicit_loops():
    th = _theta(3)
    W1, b1, W2, b2, W3, b3, W4, b4 = Lr.unpack(th)
    x = np.random.default_rng(4).normal(size=6)

    def layer(W, b, v):
        return [sum(W[o][i] * v[i] for i in range(len(v))) + b[o] for o in range(len(b))]

    def g(v):
        return [0.5 * a * (1 + math.erf(a / math.sqrt(2))) for a in v]

    h = g(layer(W1, b1, x))
    h = g(layer(W2, b2, h))
    h = g(layer(W3, b3, h))
    y = layer(W4, b4, h)[0]
    assert abs(Lr.forward(th, x[None, :])[0] - y) < 1e-12


def test_gradient_matches_central_differences():
    th = _theta(5)
    rng = np.random.default_rng(6)
    X = rng.normal(size=(7, 6))
    t = rng.normal(size=7)
    loss, g = Lr.loss_grad(th, X, t)
    assert abs(loss - np.mean((Lr.forward(th, X) - t) ** 2)) < 1e-14
    # every parameter group: a sample of entries
    starts = np.cumsum([0] + [int(np.prod(s)) for s in Lr.SIZES])
    idx = np.concatenate([rng.choice(np.arange(a, b), size=min(6, b - a), replace=False)
                          for a, b in zip(starts[:-1], starts[1:])])
    h = 1e-6
    for k in idx:
        e = np.zeros_like(th)
        e[k] = h
        fd = (Lr.loss_grad(th + e, X, t)[0] - Lr.loss_grad(th - e, X, t)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 * max(1.0, abs(fd)), (k, fd, g[k])


def test_bf16_mode_stays_close_to_fp64():
    th = _theta(7)
    rng = np.random.default_rng(8)
    X = rng.normal(size=(64, 6))
    t = rng.normal(size=64)
    y64, yb = Lr.forward(th, X), Lr.forward(th, X, bf=True)
    assert np.linalg.norm(yb - y64) / np.linalg.norm(y64) < 2e-2
    g64, gb = Lr.loss_grad(th, X, t)[1], Lr.loss_grad(th, X, t, bf=True)[1]
    assert np.linalg.norm(gb - g64) / np.linalg.norm(g64) < 3e-2
    assert not np.array_equal(yb, y64)


def test_adam_first_step_closed_form_and_convergence():
    rng = np.random.default_rng(9)
    th0 = rng.normal(size=10)
    g = rng.normal(size=10)
    opt = Lr.Adam(th0, lr=0.01, eps=1e-8)
    th1 = opt.step(g)
    # bias-corrected moments equal g and g^2 after one step
    assert np.max(np.abs(th1 - (th0 - 0.01 * g / (np.abs(g) + 1e-8)))) < 1e-15
    # converges on the quadratic 1/2 |theta - c|^2
    c = rng.normal(size=10)
    opt = Lr.Adam(np.zeros(10), lr=0.05)
    for _ in range(3000):
        th = opt.step(opt.theta - c)
    assert np.max(np.abs(th - c)) < 1e-3


def test_residual_feature_vanishes_at_an_exact_eigenpair():
    # A_l phi = lam M phi exactly => b - (A_l + sigma M) phi = 0 for b = (lam + sigma) M phi
    rng = np.random.default_rng(10)
    n = 30
    Bm = rng.normal(size=(n, n))
    Al = Bm @ Bm.T + n * np.eye(n)
    M = np.diag(rng.uniform(1, 2, n))
    lam, V = sla.eigh(Al, M)
    Phi = V[:, :2]
    sigma = 0.7
    A = Al + sigma * M
    Bv = (M @ Phi) * (lam[:2] + sigma)
    F, s = Lr.features(Phi, A @ Phi, Bv, 1.0 / np.diag(A), np.zeros(n), rng.normal(size=(n, 3)),
                       np.zeros((1, 3)), 10.0)
    assert np.max(np.abs(F[:, 2])) < 1e-12
    assert np.allclose(np.abs(F[:, 1]).reshape(n, 2).max(axis=0), 1.0)
    assert np.array_equal(Lr.targets(Phi, Phi, s), np.zeros(2 * n))


def test_nearest_distances_brute_force():
    rng = np.random.default_rng(11)
    pts = rng.uniform(-3, 3, size=(20, 3))
    R = rng.uniform(-3, 3, size=(5, 3))
    got = Lr.nearest_distances(pts, R, 99.0)
    for p, row in zip(pts, got):
        ds = sorted(math.dist(p, r) for r in R)[:3]
        assert np.allclose(row, ds, rtol=0, atol=1e-14)
    one = Lr.nearest_distances(pts, R[:1], 99.0)
    assert np.all(one[:, 1:] == 99.0)


def test_galerkin_start_recovers_the_solution_and_never_loses_energy():
    """A perfect direction (delta = u - phi) gives x0 = u exactly; any
    direction gives J(x0) <= J(phi) and |b - A x0| <= |b - A phi|, and where
    the combination is used, J(x0) <= J at other points of the span; a
    direction parallel to phi is rejected (singular 2 x 2)."""
    rng = np.random.default_rng(12)
    n = 40
    Bm = rng.normal(size=(n, n))
    A = Bm @ Bm.T + n * np.eye(n)
    U = rng.normal(size=(n, 3))
    B = A @ U
    Phi = U + 0.1 * rng.normal(size=(n, 3))
    X, used, coef = Lr.galerkin_start(A, B, Phi, U - Phi)
    assert used.all() and np.allclose(X, U, rtol=0, atol=1e-10) and np.allclose(coef, [[1, 1]] * 3)

    def J(x, c):
        return 0.5 * x @ A @ x - B[:, c] @ x

    D = rng.normal(size=(n, 3))
    X, used, coef = Lr.galerkin_start(A, B, Phi, D)
    for c in range(3):
        assert J(X[:, c], c) <= J(Phi[:, c], c) + 1e-9
        assert np.linalg.norm(B[:, c] - A @ X[:, c]) <= np.linalg.norm(B[:, c] - A @ Phi[:, c]) * (1 + 1e-12)
        if used[c]:
            for da, db in rng.normal(scale=0.05, size=(5, 2)):
                a, b = coef[c]
                assert J(X[:, c], c) <= J((a + da) * Phi[:, c] + (b + db) * D[:, c], c) + 1e-9
    X, used, _ = Lr.galerkin_start(A, B, Phi, 2.0 * Phi)
    assert not used.any() and np.array_equal(X, Phi)


def test_galerkin_start_keeps_phi_when_the_residual_grows():
    """Random starts on a stiff diagonal A (eigenvalues 1 and 400): among them
    are directions whose span minimiser lowers J (the A-norm error) but has a
    larger residual than phi; there phi is kept, and elsewhere the minimiser
    is used. Both cases must occur in the draws."""
    rng = np.random.default_rng(5)
    n = 6
    A = np.diag([1.0, 1.0, 1.0, 1.0, 1.0, 400.0])
    kept = taken = 0
    for _ in range(400):
        u = rng.normal(size=n)
        B = (A @ u)[:, None]
        Phi = (u + rng.normal(size=n) * np.array([1, 1, 1, 1, 1, 0.02]))[:, None]
        D = rng.normal(size=(n, 1)) * np.array([[1], [1], [1], [1], [1], [0.05]])
        G = np.array([[Phi[:, 0] @ A @ Phi[:, 0], Phi[:, 0] @ A @ D[:, 0]],
                      [D[:, 0] @ A @ Phi[:, 0], D[:, 0] @ A @ D[:, 0]]])
        r = np.array([B[:, 0] @ Phi[:, 0], B[:, 0] @ D[:, 0]])
        a, b = np.linalg.solve(G, r)
        x = a * Phi[:, 0] + b * D[:, 0]
        drops = 0.5 * x @ A @ x - B[:, 0] @ x < 0.5 * Phi[:, 0] @ A @ Phi[:, 0] - B[:, 0] @ Phi[:, 0]
        grows = np.linalg.norm(B[:, 0] - A @ x) > np.linalg.norm(B[:, 0] - A @ Phi[:, 0])
        X, used, _ = Lr.galerkin_start(A, B, Phi, D)
        if drops and grows:
            kept += 1
            assert not used[0] and np.array_equal(X, Phi)
        elif drops:
            taken += 1
            assert used[0] and np.allclose(X[:, 0], x, rtol=1e-12, atol=1e-12)
    assert kept > 0 and taken > 0, (kept, taken)
