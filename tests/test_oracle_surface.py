"""Pins of the oracle's closest-point surface diffusion on a sphere (Section 5.2,
Theorem 5.2, Algorithm 2's steps 1-2 and the free-space heat convolution it
approximates).

What fixes the answer independently of the oracle's code:
  * Table 1 of the paper (band widths) and the width its sphere experiment
    states, from tests/golden/;
  * T(x) is the heat-kernel mass outside the ball of radius 2 x sqrt(tau)
    (scipy quadrature of the radial density);
  * the Chebyshev-point rule integrates polynomials of degree < p exactly;
  * the band and its closest points against a numpy enumeration;
  * the diffusion of constants, and of spherical harmonics of degree l, whose
    factor is 1 - l(l+1) tau + O(tau^2) (Laplace-Beltrami eigenvalues on the
    unit sphere); at the north pole, the quadrature sum against a 2-D scipy
    integration of the same convolution in spherical coordinates.
"""
import os

import numpy as np
import pytest
import scipy.integrate
import scipy.special

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_table_1_band_widths():
    rows = np.loadtxt(os.path.join(GOLDEN, "paper_table1_band_widths.txt"))
    for eps, tau, wb in rows:
        got = oracle.band_width(tau, eps)
        assert abs(got - wb) <= 0.006 * wb, (eps, tau, wb, got)


@pytest.mark.parametrize("x", [0.3, 1.0, 2.0, 3.5])
def test_T_is_the_heat_kernel_tail(x):
    tau = 0.01
    w = 2 * x * np.sqrt(tau)
    dens = lambda r: 4 * np.pi * r * r * (4 * np.pi * tau) ** -1.5 * np.exp(-r * r / (4 * tau))
    tail, _ = scipy.integrate.quad(dens, w, np.inf, epsabs=1e-14, epsrel=1e-12)
    assert abs(oracle.band_T(x) - tail) < 1e-11


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
def test_chebyshev_rule(p):
    x, w = oracle.cheb_rule(p)
    want = np.sort(0.5 * (1 + np.cos((2 * np.arange(1, p + 1) - 1) * np.pi / (2 * p))))
    assert np.abs(x - want).max() < 1e-15
    for deg in range(p):
        assert abs((w * x ** deg).sum() - 1.0 / (deg + 1)) < 1e-14


def test_band_against_enumeration():
    R, dx, p, tau, eps = 1.0, 0.25, 2, 0.01, 1e-6
    b = oracle.sphere_band(R, dx, p, tau, eps)
    wb = b["wb"]
    lim = int(np.ceil((R + wb) / dx)) + 1
    g = np.arange(-lim, lim + 1) * dx
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    keep = np.abs(np.sqrt(X ** 2 + Y ** 2 + Z ** 2) - R) < wb
    assert b["cells"] == int(keep.sum()) and b["w"].size == p ** 3 * b["cells"]
    x, w = oracle.cheb_rule(p)
    corners = np.stack([X[keep], Y[keep], Z[keep]], axis=1)  # lexicographic order
    off = np.stack(np.meshgrid(x, x, x, indexing="ij"), axis=-1).reshape(-1, 3) * dx
    want = (corners[:, None, :] + off[None, :, :]).reshape(-1, 3).T
    assert np.abs(b["xq"] - want).max() < 1e-14
    r = np.linalg.norm(b["xc"], axis=0)
    assert np.abs(r - R).max() < 1e-14
    cosang = (b["xc"] * b["xq"]).sum(axis=0) / (R * np.linalg.norm(b["xq"], axis=0))
    assert np.abs(cosang - 1).max() < 1e-14
    assert abs(b["w"].sum() - b["cells"] * dx ** 3) < 1e-12


@pytest.fixture(scope="module")
def bands():
    return {tau: oracle.sphere_band(1.0, dx, 1, tau, 1e-6) for tau, dx in ((0.01, 0.12), (0.005, 0.1))}


def test_constants_are_preserved(bands):
    for tau, b in bands.items():
        m = b["w"].size
        out = oracle.surface_diffuse(b, np.ones((1, 1, m)), tau)
        assert np.abs(out - 1).max() < 1e-5  # eps = 1e-6 truncation plus the midpoint rule


def test_harmonics_decay_by_laplace_beltrami_eigenvalues(bands):
    """Factor of Y_l: 1 - l(l+1) tau + c_l tau^2 (first order in tau), the same
    c_l at both steps."""
    c = {}
    for tau, b in bands.items():
        m = b["w"].size
        x, y, z = b["xc"]
        F = np.stack([z, x * y, 3 * z * z - 1, x * (5 * z * z - 1)])
        out = oracle.surface_diffuse(b, F.reshape(2, 2, m), tau).reshape(4, m)
        for k, l in enumerate((1, 2, 2, 3)):
            msk = np.abs(F[k]) > 0.2
            r = out[k][msk] / F[k][msk]
            assert r.std() < 2e-6
            c[(k, tau)] = (r.mean() - 1 + l * (l + 1) * tau) / tau ** 2
    for k in range(4):
        a, b2 = c[(k, 0.01)], c[(k, 0.005)]
        assert abs(a) < 80 and abs(a - b2) <= 0.15 * max(abs(a), 1.0), (k, a, b2)


def test_north_pole_against_direct_integration():
    """out(north pole) for f = z: the oracle's band quadrature against scipy's
    integration of int_band G_tau(e_z - y) f(y / |y|) dy in spherical
    coordinates (azimuth done exactly through the Bessel function I_0)."""
    tau, dx = 0.01, 0.1
    b = oracle.sphere_band(1.0, dx, 1, tau, 1e-6)
    m = b["w"].size
    z = b["xc"][2]
    out = oracle.surface_diffuse(b, z.reshape(1, 1, m), tau)[0, 0]
    top = np.argmax(z)
    xc = b["xc"][:, top]
    # target at the closest point itself: rotate so it lies on the z axis (it is within dx of it)
    assert np.linalg.norm(xc - np.array([0, 0, 1.0])) < 0.2
    wb = b["wb"]
    norm = (4 * np.pi * tau) ** -1.5

    def integrand(th, r):
        # |c - y|^2 = 1 + r^2 - 2 r (cos th cos tc + sin th sin tc cos phi), c at polar angle tc
        tc = np.arccos(xc[2])
        a = 1 + r * r - 2 * r * np.cos(th) * np.cos(tc)
        bb = 2 * r * np.sin(th) * np.sin(tc)
        # int_0^2pi exp(-(a - bb cos phi)/(4 tau)) dphi = 2 pi exp(-a/4tau) I0(bb/4tau)
        ang = 2 * np.pi * np.exp(-(a - bb) / (4 * tau)) * scipy.special.ive(0, bb / (4 * tau))
        return norm * ang * np.cos(th) * r * r * np.sin(th)

    val, _ = scipy.integrate.dblquad(integrand, 1 - wb, 1 + wb, 0, np.pi, epsabs=1e-10, epsrel=1e-9)
    # the discrete band is the union of whole cells, so its edge differs from the
    # sphere shell by up to dx, where the kernel has mass below eps
    assert abs(out[top] - val) < 5e-5, (out[top], val)


def test_sphere_experiment_shrinks_the_octant():
    """Section 6.2's initial field (the printed matrices, projected) on a coarse
    band: the octant x < 0, y < 0, z > 0 (SO^-(3): the first printed matrix has
    det < 0) loses points as the MBO steps run."""
    rows = np.loadtxt(os.path.join(GOLDEN, "paper_sphere_initial_matrices.txt"))
    M1, M2 = rows[:3], rows[3:]
    Q = oracle.project(np.stack([M1, M2], axis=-1).reshape(3, 3, 2))[0]
    tau = 0.02
    b = oracle.sphere_band(1.0, 0.15, 1, tau, 1e-6)
    m = b["w"].size
    x, y, z = b["xc"]
    inside = (x < 0) & (y < 0) & (z > 0)
    A0 = np.where(inside[None, None, :], Q[:, :, 0:1], Q[:, :, 1:2])
    n0 = int((oracle.det_sign(A0) < 0).sum())
    assert n0 == int(inside.sum()) and 0 < n0 < m
    A, fl = oracle.surface_iterate(b, A0, tau, 6)
    n1 = int((oracle.det_sign(A) < 0).sum())
    assert n1 < n0 and fl.sum() == n0 - n1


def test_heat_at_targets():
    """The convolution at arbitrary targets: at the closest points it is the
    surface diffusion step; for one source of weight 1 it is G_tau itself."""
    tau = 0.01
    b = oracle.sphere_band(1.0, 0.15, 1, tau, 1e-6)
    m = b["w"].size
    rng = np.random.default_rng(5)
    A = rng.standard_normal((2, 2, m))
    idx = rng.choice(m, 40, replace=False)
    full = oracle.surface_diffuse(b, A, tau)
    at = oracle.heat_at(b, A, tau, b["xc"][:, idx])
    assert np.abs(at - full[:, :, idx]).max() < 1e-13 * np.abs(full).max()
    one = {"xq": np.array([[0.1], [0.2], [-0.3]]), "w": np.array([1.0])}
    xt = np.array([[0.0, 0.4], [0.0, -0.1], [0.0, 0.05]])
    g = oracle.heat_at(one, np.ones((1, 1, 1)), tau, xt)[0, 0]
    r2 = ((xt - one["xq"]) ** 2).sum(axis=0)
    assert np.abs(g - (4 * np.pi * tau) ** -1.5 * np.exp(-r2 / (4 * tau))).max() < 1e-12 * g.max()
