"""Pins of the oracle's adjoint (gradients of K unrolled steps of Algorithm 1).

The adjoint is not in the paper; what pins it is the mathematics: central
finite differences of the oracle's own forward map (itself pinned elsewhere),
an independent route to the projection's derivative (the Sylvester equation of
the polar decomposition, solved with scipy), the closed form of the heat
step's tau-derivative on single Fourier modes, and the special cases K = 0 and
n = 1.  Each of these fails on a dropped term, a wrong sign or a transposed
factor in the backward recursion.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle


def _well_conditioned(rng, n, smin=0.1):
    while True:
        A = rng.standard_normal((n, n))
        if np.linalg.svd(A, compute_uv=False).min() > smin:
            return A


@pytest.mark.parametrize("n", [2, 3, 4])
def test_project_vjp_central_difference(n):
    """<VJP(G), D> equals the directional derivative of <G, P(A)> along D."""
    rng = np.random.default_rng(100 + n)
    h = 1e-6
    for _ in range(20):
        A = _well_conditioned(rng, n).reshape(n, n, 1, 1)
        G = rng.standard_normal((n, n, 1, 1))
        D = rng.standard_normal((n, n, 1, 1))
        GA = oracle.project_vjp(A, G)
        fd = ((oracle.project(A + h * D)[0] - oracle.project(A - h * D)[0]) * G).sum() / (2 * h)
        assert abs((GA * D).sum() - fd) <= 1e-7 * (1.0 + abs(fd))


@pytest.mark.parametrize("n", [2, 3, 4])
def test_project_vjp_matches_sylvester_route(n):
    """Independent route: A = Q H (scipy polar), H Y + Y H = skew(Q^t G), G_A = 2 Q Y."""
    rng = np.random.default_rng(200 + n)
    P = 64
    A = np.stack([_well_conditioned(rng, n, 0.05) for _ in range(P)], axis=-1).reshape(n, n, P)
    G = rng.standard_normal((n, n, P))
    GA = oracle.project_vjp(A, G)
    for p in range(P):
        Q, H = scipy.linalg.polar(A[:, :, p])
        M = Q.T @ G[:, :, p]
        S = 0.5 * (M - M.T)
        Y = scipy.linalg.solve_sylvester(H, H, S)
        ref = 2.0 * Q @ Y
        assert np.abs(GA[:, :, p] - ref).max() <= 1e-11 * (1.0 + np.abs(ref).max())


def test_project_vjp_n1_is_zero():
    rng = np.random.default_rng(7)
    A = rng.uniform(-1, 1, (1, 1, 32))
    G = rng.standard_normal((1, 1, 32))
    assert np.all(oracle.project_vjp(A, G) == 0.0)


def test_project_vjp_orthogonal_input():
    """At an orthogonal point (all sigma = 1) the derivative is the skew part
    Q skew(Q^t G): K_ij = (M_ij - M_ji) / 2."""
    rng = np.random.default_rng(8)
    for n in (2, 3, 4):
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        G = rng.standard_normal((n, n))
        ref = Q @ (0.5 * (Q.T @ G - G.T @ Q))
        GA = oracle.project_vjp(Q.reshape(n, n, 1), G.reshape(n, n, 1))[:, :, 0]
        assert np.abs(GA - ref).max() <= 1e-13


@pytest.mark.parametrize("grid,k", [((32, 32), (3, -5)), ((16, 16), (8, 0)), ((8, 16, 8), (1, 2, -3))])
def test_heat_dtau_single_mode(grid, k):
    """cos(2 pi k.x) -> -4 pi^2 |k|^2 exp(-4 pi^2 tau |k|^2) cos(2 pi k.x), Nyquist included."""
    tau = 3e-3
    xs = np.meshgrid(*[np.arange(N) / N for N in grid], indexing="ij")
    phase = 2 * np.pi * sum(ki * x for ki, x in zip(k, xs))
    f = np.cos(phase + 0.3)
    ksq = float(sum(ki * ki for ki in k))
    ref = -4 * np.pi ** 2 * ksq * np.exp(-4 * np.pi ** 2 * tau * ksq) * f
    out = oracle.heat_dtau(f[None], tau, len(grid))[0]
    assert np.abs(out - ref).max() <= 1e-12 * (1.0 + np.abs(ref).max())


def test_heat_dtau_central_difference_in_tau():
    rng = np.random.default_rng(9)
    f = rng.standard_normal((3, 16, 16))
    tau, h = 2e-3, 1e-7
    fd = (oracle.heat(f, tau + h, 2)[0] - oracle.heat(f, tau - h, 2)[0]) / (2 * h)
    out = oracle.heat_dtau(f, tau, 2)
    assert np.abs(out - fd).max() <= 1e-6 * np.abs(out).max()


def test_unroll_grad_K0():
    rng = np.random.default_rng(10)
    A0 = rng.uniform(-1, 1, (3, 3, 8, 8))
    T = rng.uniform(-1, 1, (3, 3, 8, 8))
    r = oracle.unroll_grad(A0, T, 1e-2, 0)
    assert np.array_equal(r["gA0"], A0 - T)
    assert r["gtau"] == 0.0
    assert abs(r["loss"] - 0.5 * ((A0 - T) ** 2).sum()) <= 1e-12 * r["loss"]


def test_unroll_grad_n1_zero():
    """Sign thresholding is locally constant: both gradients vanish."""
    rng = np.random.default_rng(11)
    A0 = rng.uniform(-1, 1, (1, 1, 16, 16))
    T = rng.uniform(-1, 1, (1, 1, 16, 16))
    r = oracle.unroll_grad(A0, T, 1e-2, 3)
    assert np.all(r["gA0"] == 0.0) and r["gtau"] == 0.0


def _loss(A0, T, tau, K):
    r = oracle.unroll_grad(A0, T, tau, K)
    return r["loss"], list(r["flips"])


@pytest.mark.parametrize("n,N,K,tau,seed", [(2, 8, 3, 1e-2, 1), (3, 16, 4, 2e-3, 2),
                                             (3, 8, 5, 1e-2, 3), (4, 8, 2, 5e-3, 4)])
def test_unroll_grad_central_difference(n, N, K, tau, seed):
    """Gradients in A_0 (random directions) and in tau against central finite
    differences of the forward loss, h = 1e-6 (relative in tau).  A difference is
    only meaningful if no det sign flips differently between the +h and -h runs."""
    rng = np.random.default_rng(seed)
    A0 = rng.uniform(-1, 1, (n, n, N, N))
    T = oracle.project(rng.standard_normal((n, n, N, N)))[0]
    r = oracle.unroll_grad(A0, T, tau, K)
    h = 1e-6
    for _ in range(3):
        D = rng.standard_normal(A0.shape)
        lp, fp = _loss(A0 + h * D, T, tau, K)
        lm, fm = _loss(A0 - h * D, T, tau, K)
        assert fp == fm == list(r["flips"])
        fd = (lp - lm) / (2 * h)
        assert abs((r["gA0"] * D).sum() - fd) <= 1e-6 * (1.0 + abs(fd))
    lp, fp = _loss(A0, T, tau * (1 + h), K)
    lm, fm = _loss(A0, T, tau * (1 - h), K)
    assert fp == fm
    fdt = (lp - lm) / (2 * h * tau)
    assert abs(r["gtau"] - fdt) <= 1e-6 * (1.0 + abs(fdt))


def test_unroll_grad_3d_central_difference():
    rng = np.random.default_rng(12)
    n, K, tau = 3, 2, 5e-3
    A0 = rng.standard_normal((n, n, 8, 8, 8))
    T = oracle.project(rng.standard_normal(A0.shape))[0]
    r = oracle.unroll_grad(A0, T, tau, K)
    h = 1e-6
    D = rng.standard_normal(A0.shape)
    lp, fp = _loss(A0 + h * D, T, tau, K)
    lm, fm = _loss(A0 - h * D, T, tau, K)
    assert fp == fm
    fd = (lp - lm) / (2 * h)
    assert abs((r["gA0"] * D).sum() - fd) <= 1e-6 * (1.0 + abs(fd))
