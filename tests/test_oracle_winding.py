"""Pins of the oracle's SO(2) index (Section 6.1) and of the paper's three
flat-torus examples as the oracle runs them.

The index pins are closed forms: a field whose angle is 2 pi (m x + k y) turns
m times along every loop in x and k times along every loop in y; the first
column of a reflection carries the same angle; reversing the angle negates the
index; a field whose angle stays inside an interval shorter than pi has index
0.  The examples are pinned by the end states the paper describes (its figures
are absent): the star-shaped defect shrinks away and the field becomes uniform;
the two line defects straighten into lines parallel to the y-axis with a
uniform angle; with the winding angle the end state is not constant and keeps
its index along y.
"""
import numpy as np
import pytest

import oracle
from paper_1711_01365_amd import inputs


@pytest.mark.parametrize("m,k", [(0, 0), (1, 0), (0, 1), (2, -3), (-1, 4)])
def test_linear_angle_index(m, k):
    A = inputs.linear_angle_field((48, 40), m, k)
    wx, wy = oracle.winding(A)
    assert np.abs(wx - m).max() < 1e-12 and np.abs(wy - k).max() < 1e-12
    # reflections [[c, s], [s, -c]] share the first column
    R = A.copy()
    R[0, 1], R[1, 1] = A[1, 0], -A[0, 0]
    wx2, wy2 = oracle.winding(R)
    assert np.array_equal(wx, wx2) and np.array_equal(wy, wy2)
    # reversed angle
    C = A.copy()
    C[1, 0] = -A[1, 0]
    wx3, wy3 = oracle.winding(C)
    assert np.abs(wx3 + m).max() < 1e-12 and np.abs(wy3 + k).max() < 1e-12


def test_bounded_angle_has_index_zero():
    rng = np.random.default_rng(3)
    al = 1.4 * np.tanh(rng.standard_normal((32, 32)))  # |angle| < 1.4 < pi / 2
    c, s = np.cos(al), np.sin(al)
    A = np.stack([np.stack([c, -s]), np.stack([s, c])])
    wx, wy = oracle.winding(A)
    assert np.abs(wx).max() < 1e-12 and np.abs(wy).max() < 1e-12


def test_initial_fields_of_the_examples():
    wx, wy = oracle.winding(inputs.star_defect_field((64, 64)))
    assert np.abs(wx).max() < 1e-12 and np.abs(wy).max() < 1e-12
    wx, wy = oracle.winding(inputs.line_defect_field((64, 64), False))
    assert np.abs(wx).max() < 1e-12 and np.abs(wy).max() < 1e-12
    wx, wy = oracle.winding(inputs.line_defect_field((64, 64), True))
    assert np.abs(wx).max() < 1e-12 and np.abs(wy - 1.0).max() < 1e-12


def _angle(A):
    return np.arctan2(A[1, 0], A[0, 0])


def test_example_star_defect_shrinks_to_uniform():
    w = inputs.EXAMPLE_STAR
    N = 256
    r = oracle.iterate(inputs.star_defect_field((N, N)), w.tau, 320)
    E = r["energy"]
    assert np.all(np.diff(E[1:]) <= 1e-12 * np.abs(E[1:-1]))
    assert int((oracle.det_sign(r["A"]) > 0).sum()) == 0
    assert _angle(r["A"]).std() < 0.05


def test_example_line_defects_straighten():
    w = inputs.EXAMPLE_LINES
    N = 256
    r = oracle.iterate(inputs.line_defect_field((N, N), False), w.tau, 200)
    ds = oracle.det_sign(r["A"])
    # det sign constant along y on all but the rows next to the two lines
    assert np.all(ds == ds[:, :1], axis=1).mean() >= 0.95
    assert 0 < int((ds > 0).sum()) < N * N
    assert _angle(r["A"]).std() < 1e-3
    wx, wy = oracle.winding(r["A"])
    assert np.abs(wx).max() < 1e-9 and np.abs(wy).max() < 1e-9


def test_example_winding_keeps_a_nonconstant_field():
    w = inputs.EXAMPLE_WINDING
    N = 256
    r = oracle.iterate(inputs.line_defect_field((N, N), True), w.tau, 200)
    wx, wy = oracle.winding(r["A"])
    assert np.abs(wy - 1.0).max() < 1e-9 and np.abs(wx).max() < 1e-9
    assert _angle(r["A"]).std() > 1.0
    E = r["energy"]
    assert np.all(np.diff(E[1:]) <= 1e-12 * np.abs(E[1:-1]))
