"""Pins of the oracle's closest points and sample sets on surfaces of revolution
(Section 6.3's peanut, and the sphere as a meridian for a check of the
machinery).

What fixes the answer independently of the oracle's code:
  * the sphere meridian gives R x / |x| and | |x| - R |, and the same sample
    set as the sphere builder;
  * peanut points generated from the printed parametrization are their own
    closest points, at distance 0;
  * for random points the distance is not beaten by any of 2e5 surface points
    drawn from the parametrization, and is matched by a fine (t, theta) grid;
  * the residual to the closest point is orthogonal to the surface there (no
    neighbouring surface point is closer);
  * the printed profile's extremes: waist radius 1 at x = 0, largest radius
    1.25 at x^2 = 3/2 (seen from radially outside), tips at x = +-2.
"""
import numpy as np
import pytest

import oracle


def peanut_point(t, th):
    x = 3 * t - t ** 3
    rho = 0.5 * np.sqrt(np.maximum((1 + x * x) * (4 - x * x), 0.0))
    return np.stack([x, rho * np.cos(th), rho * np.sin(th)])


@pytest.mark.parametrize("R", [0.7, 1.0, 1.9])
def test_sphere_meridian_is_the_sphere(R):
    rng = np.random.default_rng(3000)
    P = rng.uniform(-2.5, 2.5, (3, 300))
    c, d = oracle.revolution_cp(oracle.REV_SPHERE, P, R)
    r = np.linalg.norm(P, axis=0)
    assert np.abs(c - R * P / r).max() < 1e-13
    assert np.abs(d - np.abs(r - R)).max() < 1e-13


def test_sphere_meridian_band_is_the_sphere_band():
    a = oracle.revolution_band(oracle.REV_SPHERE, 0.3, 2, 0.01, 1e-6, R=1.0)
    b = oracle.sphere_band(1.0, 0.3, 2, 0.01, 1e-6)
    assert a["cells"] == b["cells"]
    assert np.abs(a["xq"] - b["xq"]).max() < 1e-14
    assert np.abs(a["xc"] - b["xc"]).max() < 1e-13
    assert np.abs(a["w"] - b["w"]).max() < 1e-16


def test_peanut_surface_points_are_fixed():
    rng = np.random.default_rng(3001)
    t = rng.uniform(-0.97, 0.97, 300)
    th = rng.uniform(0, 2 * np.pi, 300)
    P = peanut_point(t, th)
    c, d = oracle.revolution_cp(oracle.REV_PEANUT, P)
    assert np.abs(c - P).max() < 1e-12 and d.max() < 1e-12


def test_peanut_profile_extremes():
    c, d = oracle.revolution_cp(oracle.REV_PEANUT, np.array([[0.0, np.sqrt(1.5), 2.0, -2.0],
                                                             [0.0, 3.0, 0.0, 0.0],
                                                             [0.0, 0.0, 0.0, 0.0]]))
    assert abs(d[0] - 1.0) < 1e-12   # the axis point at the waist: radius 1
    # radially outside the largest radius 1.25 (where the normal is radial)
    assert abs(d[1] - 1.75) < 1e-12 and abs(c[1, 1] - 1.25) < 1e-12
    assert d[2] < 1e-12 and d[3] < 1e-12 and abs(c[0, 2] - 2.0) < 1e-12


def test_peanut_distance_is_minimal():
    rng = np.random.default_rng(3002)
    P = np.stack([rng.uniform(-3.4, 3.4, 60), rng.uniform(-2.6, 2.6, 60), rng.uniform(-2.6, 2.6, 60)])
    c, d = oracle.revolution_cp(oracle.REV_PEANUT, P)
    S = peanut_point(rng.uniform(-1, 1, 200000), rng.uniform(0, 2 * np.pi, 200000))
    tg, thg = np.meshgrid(np.linspace(-1, 1, 2001), np.linspace(0, 2 * np.pi, 721), indexing="ij")
    G = peanut_point(tg.ravel(), thg.ravel())
    for q in range(P.shape[1]):
        brute = np.sqrt(((S - P[:, q:q + 1]) ** 2).sum(axis=0)).min()
        grid = np.sqrt(((G - P[:, q:q + 1]) ** 2).sum(axis=0)).min()
        assert d[q] <= brute + 1e-12 and d[q] <= grid + 1e-12
        assert grid - d[q] < 5e-3
        assert abs(np.linalg.norm(c[:, q] - P[:, q]) - d[q]) < 1e-12


def test_peanut_residual_is_normal():
    """No surface point near the closest point (parameter and angle perturbed)
    is closer."""
    rng = np.random.default_rng(3003)
    P = np.stack([rng.uniform(-3, 3, 40), rng.uniform(-2, 2, 40), rng.uniform(-2, 2, 40)])
    c, d = oracle.revolution_cp(oracle.REV_PEANUT, P)
    for q in range(P.shape[1]):
        x = c[0, q]
        # parameter of the closest point: the root of 3t - t^3 = x in [-1, 1]
        roots = np.roots([-1.0, 0.0, 3.0, -x])
        t0 = float(np.real(roots[np.argmin(np.abs(np.imag(roots)) + 10 * (np.abs(np.real(roots)) > 1 + 1e-9))]))
        th0 = np.arctan2(c[2, q], c[1, q])
        dt, dth = np.meshgrid(np.linspace(-1e-3, 1e-3, 41), np.linspace(-1e-3, 1e-3, 41), indexing="ij")
        N = peanut_point(np.clip(t0 + dt.ravel(), -1, 1), th0 + dth.ravel())
        near = np.sqrt(((N - P[:, q:q + 1]) ** 2).sum(axis=0)).min()
        assert d[q] <= near + 1e-12


def test_peanut_band():
    b = oracle.revolution_band(oracle.REV_PEANUT, 0.25, 2, 0.01, 1e-6)
    _, d = oracle.revolution_cp(oracle.REV_PEANUT, b["xq"])
    # every sample lies in its cell next to a corner within w_b of the surface
    assert d.max() < b["wb"] + np.sqrt(3) * 0.25
    assert b["w"].size == 8 * b["cells"]
    assert abs(b["w"].sum() - b["cells"] * 0.25 ** 3) < 1e-12
