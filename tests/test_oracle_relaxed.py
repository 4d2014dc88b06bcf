"""Pins of the oracle's relaxed gradient flows GD-1 and GD-3 (Section 1) and of
their energies E_{1,eps}, E_{2,eps}.

What fixes the answer independently of the oracle's code:
  * the diffusion step alone (eps = inf) damps a Fourier mode by exactly
    1 / (1 + 4 pi^2 dt |k|^2) per step;
  * the reaction terms against numpy's SVD: U (Sigma - I) V^t for GD-1 and the
    GD-2 form U (Sigma^2 - I) Sigma V^t for GD-3 (the paper's equivalence);
  * constant orthogonal fields are fixed points with zero energy;
  * n = 1, GD-3 is Allen-Cahn (Remark 1.2): the kink tanh(x / (sqrt 2 eps))
    solves it exactly, and the scheme's deviation from it is first order in dt
    with zero limit;
  * n = 2, SO(2) data under GD-3 follows the complex Ginzburg-Landau equation
    (Lemma 1.3): a complex scalar solver (numpy FFT) gives the same first column;
  * the energies: closed forms for single modes and scaled orthogonal fields, and
    their decrease along the flows.
"""
import numpy as np
import pytest

import oracle
from paper_1711_01365_amd import inputs


def test_diffusion_step_damps_modes_exactly():
    N0, N1, dt, K = 32, 16, 1e-3, 3
    x = np.arange(N0)[:, None] / N0
    y = np.arange(N1)[None, :] / N1
    for k0, k1 in ((1, 0), (3, 2), (16, 8), (-5, 7)):
        a = np.cos(2 * np.pi * (k0 * x + k1 * y)) + 0.5
        A0 = np.stack([np.stack([a, 0 * a]), np.stack([0 * a, a])])
        A = oracle.relaxed_flow(A0, 3, np.inf, dt, K)
        g = (1.0 / (1.0 + 4 * np.pi ** 2 * dt * (k0 ** 2 + k1 ** 2))) ** K
        want = g * np.cos(2 * np.pi * (k0 * x + k1 * y)) + 0.5
        assert np.abs(A[0, 0] - want).max() < 1e-13 and np.abs(A[0, 1]).max() < 1e-13


@pytest.mark.parametrize("n", [2, 3, 4])
def test_reaction_terms_against_numpy_svd(n):
    rng = np.random.default_rng(800 + n)
    for _ in range(20):
        a = rng.standard_normal((n, n))
        A0 = np.broadcast_to(a[:, :, None, None], (n, n, 8, 8)).copy()  # constant: diffusion is exact
        U, s, Vt = np.linalg.svd(a)
        dt, eps = 1e-3, 0.1
        c = dt / eps ** 2
        g1 = oracle.relaxed_flow(A0, 1, eps, dt, 1)[:, :, 0, 0]
        assert np.abs(g1 - (a - c * U @ np.diag(s - 1) @ Vt)).max() < 1e-12
        g3 = oracle.relaxed_flow(A0, 3, eps, dt, 1)[:, :, 0, 0]
        assert np.abs(g3 - (a - c * U @ np.diag((s ** 2 - 1) * s) @ Vt)).max() < 1e-12


@pytest.mark.parametrize("kind", [1, 3])
def test_constant_orthogonal_fields_are_fixed(kind):
    Q = inputs.haar_field(3, (1, 1), 7)[:, :, 0, 0]
    A0 = np.broadcast_to(Q[:, :, None, None], (3, 3, 16, 16)).copy()
    A = oracle.relaxed_flow(A0, kind, 0.05, 1e-3, 5)
    assert np.abs(A - A0).max() < 1e-14
    assert abs(oracle.relaxed_energy(A0, kind, 0.05)) < 1e-20


def _kink(N0, eps):
    x = np.arange(N0) / N0
    return np.tanh((x - 0.25) / (np.sqrt(2) * eps)) * np.tanh((0.75 - x) / (np.sqrt(2) * eps))


def test_allen_cahn_kink_is_the_zero_step_limit():
    """n = 1, GD-3: the deviation from the exact kink after a fixed time is
    proportional to dt (first-order splitting) and extrapolates to zero."""
    N0, N1, eps, T = 512, 8, 0.02, 0.02
    u = _kink(N0, eps)
    A0 = np.repeat(u[:, None], N1, axis=1).reshape(1, 1, N0, N1)
    dev = {}
    for dt in (1e-5, 2e-5):
        A = oracle.relaxed_flow(A0, 3, eps, dt, int(round(T / dt)))
        dev[dt] = np.abs(A - A0).max()
    assert dev[2e-5] < 0.03
    assert abs(2 * dev[1e-5] - dev[2e-5]) < 0.05 * dev[2e-5]


def test_so2_data_follow_complex_ginzburg_landau():
    """Lemma 1.3: the first column of an SO(2) field under GD-3 solves the complex
    Ginzburg-Landau equation; the same scheme in complex arithmetic agrees."""
    N, eps, dt, K = 64, 0.05, 2e-4, 30
    A0 = inputs.line_defect_field((N, N), True)
    A0 = A0.copy()
    A0[0, 1], A0[1, 1] = -A0[1, 0], A0[0, 0]  # every point a rotation
    A = oracle.relaxed_flow(A0, 3, eps, dt, K)
    assert np.abs(A[0, 1] + A[1, 0]).max() < 1e-13 and np.abs(A[1, 1] - A[0, 0]).max() < 1e-13
    z = A0[0, 0] + 1j * A0[1, 0]
    k = np.fft.fftfreq(N, 1.0 / N)
    ksq = k[:, None] ** 2 + k[None, :] ** 2
    for _ in range(K):
        z = np.fft.ifft2(np.fft.fft2(z) / (1 + 4 * np.pi ** 2 * dt * ksq))
        z = z - dt / eps ** 2 * z * (np.abs(z) ** 2 - 1)
    assert np.abs(A[0, 0] + 1j * A[1, 0] - z).max() < 1e-12


def test_energy_closed_forms():
    N0, N1 = 32, 64
    x = np.arange(N0)[:, None] / N0
    y = np.arange(N1)[None, :] / N1
    k0, k1, amp = 2, 5, 0.3
    a = amp * np.cos(2 * np.pi * (k0 * x + k1 * y)) + 0 * y
    Z = np.zeros_like(a)
    A = np.stack([np.stack([a, Z]), np.stack([Z, Z])])
    # (1/2) int |grad a|^2 = (1/2) amp^2 4 pi^2 |k|^2 / 2, no penalty at eps = inf
    want = 0.25 * amp ** 2 * 4 * np.pi ** 2 * (k0 ** 2 + k1 ** 2)
    for kind in (1, 3):
        assert abs(oracle.relaxed_energy(A, kind, np.inf) - want) < 1e-12 * want
    # constant s Q: penalties n (s - 1)^2 / (2 eps^2) and n (s^2 - 1)^2 / (4 eps^2)
    Q = inputs.haar_field(3, (1, 1), 9)[:, :, 0, 0]
    s, eps = 1.3, 0.2
    C = np.broadcast_to((s * Q)[:, :, None, None], (3, 3, 8, 8)).copy()
    assert abs(oracle.relaxed_energy(C, 1, eps) - 3 * (s - 1) ** 2 / (2 * eps ** 2)) < 1e-12
    assert abs(oracle.relaxed_energy(C, 3, eps) - 3 * (s * s - 1) ** 2 / (4 * eps ** 2)) < 1e-11


@pytest.mark.parametrize("kind", [1, 3])
@pytest.mark.parametrize("n", [2, 3])
def test_energy_decreases_along_the_flow(kind, n):
    N, eps, dt = 32, 0.1, 1e-3
    A = inputs.haar_field(n, (N, N), 810 + n)
    A, _ = oracle.heat(A, 2e-3, 2)  # smooth, nonsingular start
    E = [oracle.relaxed_energy(A, kind, eps)]
    for _ in range(15):
        A = oracle.relaxed_flow(A, kind, eps, dt, 1)
        E.append(oracle.relaxed_energy(A, kind, eps))
    E = np.array(E)
    assert np.all(np.diff(E) <= 1e-12 * np.abs(E[:-1])), E
