"""Pins of the oracle's volume-preserving MBO (Section 7).

What fixes the answer independently of the oracle's own code:
  * Lemma 7.1: the distance from A to the component of O(n) opposite to its
    determinant is sum (sigma_i - 1)^2 + 4 sigma_min (singular values from
    numpy's LAPACK SVD), and no sampled or locally perturbed matrix of that
    component is closer;
  * Delta E = <T+ - T-, A> equals 2 sgn(det A) sigma_min and half the difference
    of the two squared distances (identities that follow from Lemmas 1.1, 7.1);
  * n = 1 is volume-constrained thresholding: +1 on the n_plus largest values;
  * Lemma 7.2 by brute force: on 16 points no other choice of n_plus points in
    SO(n) gives a larger sum <B, A> (n = 2, T+ / T- scored by closed forms);
  * with n_plus = #{det A >= 0} the step is the plain projection of Algorithm 1;
  * Proposition 7.3: E^tau does not increase along the iterates, and the number
    of points in SO(n) stays n_plus.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_1711_01365_amd import inputs


def _pm(A):
    """T+ and T- of every point (n_plus = all and n_plus = none)."""
    P = int(np.prod(A.shape[2:]))
    Tp, dE, _ = oracle.volume_project(A, P)
    Tm, _, _ = oracle.volume_project(A, 0)
    return Tp, Tm, dE


def _points(rng, n, P, smin=0.05):
    out = []
    while len(out) < P:
        A = rng.standard_normal((n, n))
        if np.linalg.svd(A, compute_uv=False).min() > smin:
            out.append(A)
    return np.stack(out, axis=-1)


def _haar_component(rng, n, sign, count):
    G = rng.standard_normal((count, n, n))
    Q, R = np.linalg.qr(G)
    Q = Q * np.sign(np.diagonal(R, axis1=1, axis2=2))[:, None, :]
    flip = np.sign(np.linalg.det(Q)) != sign
    Q[flip, :, 0] *= -1.0
    return Q


@pytest.mark.parametrize("n", [2, 3, 4])
def test_lemma_7_1_distances(n):
    rng = np.random.default_rng(700 + n)
    A = _points(rng, n, 200)
    Tp, Tm, _ = _pm(A)
    for p in range(A.shape[-1]):
        a = A[:, :, p]
        s = np.linalg.svd(a, compute_uv=False)
        near = ((s - 1.0) ** 2).sum()
        far = near + 4.0 * s.min()
        tp, tm = Tp[:, :, p], Tm[:, :, p]
        assert np.abs(tp.T @ tp - np.eye(n)).max() < 1e-13
        assert np.abs(tm.T @ tm - np.eye(n)).max() < 1e-13
        assert np.linalg.det(tp) > 0.999 and np.linalg.det(tm) < -0.999
        dp, dm = ((tp - a) ** 2).sum(), ((tm - a) ** 2).sum()
        if np.linalg.det(a) > 0:
            assert abs(dp - near) <= 1e-12 * (1 + near) and abs(dm - far) <= 1e-12 * (1 + far)
        else:
            assert abs(dm - near) <= 1e-12 * (1 + near) and abs(dp - far) <= 1e-12 * (1 + far)


@pytest.mark.parametrize("n", [2, 3])
def test_lemma_7_1_no_closer_point(n):
    """Sampled and locally perturbed members of each component are never closer."""
    rng = np.random.default_rng(710 + n)
    A = _points(rng, n, 12)
    Tp, Tm, _ = _pm(A)
    for p in range(A.shape[-1]):
        a = A[:, :, p]
        for T, sign in ((Tp[:, :, p], 1.0), (Tm[:, :, p], -1.0)):
            d0 = ((T - a) ** 2).sum()
            C = _haar_component(rng, n, sign, 20000)
            assert (((C - a) ** 2).sum(axis=(1, 2)) >= d0 - 1e-12).all()
            for _ in range(200):
                S = rng.standard_normal((n, n)) * 1e-3
                R = scipy.linalg.expm(S - S.T)
                assert ((T @ R - a) ** 2).sum() >= d0 - 1e-12


@pytest.mark.parametrize("n", [2, 3, 4])
def test_delta_e_identities(n):
    rng = np.random.default_rng(720 + n)
    A = rng.uniform(-1, 1, (n, n, 300))
    Tp, Tm, dE = _pm(A)
    for p in range(A.shape[-1]):
        a = A[:, :, p]
        s = np.linalg.svd(a, compute_uv=False)
        closed = 2.0 * np.sign(np.linalg.det(a)) * s.min()
        assert abs(dE[p] - closed) <= 1e-12
        half = 0.5 * (((Tm[:, :, p] - a) ** 2).sum() - ((Tp[:, :, p] - a) ** 2).sum())
        assert abs(dE[p] - half) <= 1e-12


def test_n1_is_volume_constrained_thresholding():
    rng = np.random.default_rng(730)
    a = np.round(rng.uniform(-1, 1, 257), 1)  # many equal values
    A = a.reshape(1, 1, -1)
    for n_plus in (0, 1, 40, 128, 256, 257):
        B, dE, sel = oracle.volume_project(A, n_plus)
        order = sorted(range(a.size), key=lambda i: (-a[i], i))
        want = np.zeros(a.size, dtype=np.int8)
        want[order[:n_plus]] = 1
        assert np.array_equal(sel, want)
        assert np.array_equal(B.ravel(), np.where(want == 1, 1.0, -1.0))
        assert np.array_equal(dE, 2.0 * a)


def test_volume_select_matches_python_sort():
    rng = np.random.default_rng(745)
    for vals in (rng.integers(-3, 4, 1000).astype(float), rng.standard_normal(999),
                 np.array([0.0, -0.0, 0.0, -0.0, 1.0, -1.0])):
        for n_plus in sorted({0, 1, 2, vals.size // 2, vals.size - 1, vals.size}):
            order = sorted(range(vals.size), key=lambda i: (-vals[i], i))
            want = np.zeros(vals.size, dtype=np.int8)
            want[order[:n_plus]] = 1
            assert np.array_equal(oracle.volume_select(vals, n_plus), want)
    with pytest.raises(ValueError):
        oracle.volume_select(np.array([1.0, np.nan]), 1)


@pytest.mark.parametrize("n", [2, 3])
def test_selection_count_and_order(n):
    rng = np.random.default_rng(740 + n)
    A = rng.uniform(-1, 1, (n, n, 16, 16))
    P = 256
    for n_plus in (0, 1, 77, 128, 255, 256):
        B, dE, sel = oracle.volume_project(A, n_plus)
        assert int(sel.sum()) == n_plus
        det = np.linalg.det(np.moveaxis(B.reshape(n, n, P), -1, 0))
        assert int((det > 0).sum()) == n_plus
        d, s = dE.ravel(), sel.ravel().astype(bool)
        if 0 < n_plus < P:
            assert d[s].min() >= d[~s].max()


def test_ties_take_lower_indices():
    """A constant field: every Delta E is equal, so the first n_plus points win."""
    rng = np.random.default_rng(750)
    a = _points(rng, 3, 1)[:, :, 0]
    A = np.repeat(a[:, :, None], 100, axis=2).reshape(3, 3, 10, 10)
    B, dE, sel = oracle.volume_project(A, 37)
    assert np.all(dE == dE.ravel()[0])
    assert np.array_equal(np.flatnonzero(sel.ravel()), np.arange(37))
    Tp, Tm, _ = _pm(A[:, :, :1, :1])
    Bf = B.reshape(3, 3, 100)
    assert np.array_equal(Bf[:, :, :37], np.repeat(Tp.reshape(3, 3, 1), 37, axis=2))
    assert np.array_equal(Bf[:, :, 37:], np.repeat(Tm.reshape(3, 3, 1), 63, axis=2))


def test_lemma_7_2_brute_force():
    """No other set of n_plus points assigned to SO(2) scores a larger sum <B, A>."""
    rng = np.random.default_rng(760)
    A = rng.uniform(-1, 1, (2, 2, 4, 4))
    a = A.reshape(2, 2, 16)
    # best rotation / reflection scores (closed forms, independent of the oracle)
    rp = np.hypot(a[0, 0] + a[1, 1], a[1, 0] - a[0, 1])
    rm = np.hypot(a[0, 0] - a[1, 1], a[0, 1] + a[1, 0])
    for n_plus in (3, 8, 13):
        B, _, _ = oracle.volume_project(A, n_plus)
        got = (B * A).sum()
        best = max(rm.sum() + (rp - rm)[list(S)].sum()
                   for S in itertools.combinations(range(16), n_plus))
        assert abs(got - best) <= 1e-12


@pytest.mark.parametrize("n", [2, 3, 4])
def test_natural_volume_is_algorithm_1(n):
    rng = np.random.default_rng(770 + n)
    A = rng.uniform(-1, 1, (n, n, 12, 12))
    n_plus = int((oracle.det_sign(A) > 0).sum())
    B, _, _ = oracle.volume_project(A, n_plus)
    Q = oracle.project(A)[0]
    assert np.array_equal(B, Q)


def test_proposition_7_3_star_defect():
    """E^tau is non-increasing and the SO(2) volume stays fixed; without the
    constraint the SO(2) region shrinks (the paper's first example)."""
    N = 64
    A0 = inputs.star_defect_field((N, N))
    tau = 8.0 / N
    r = oracle.iterate_volume(A0, tau, 30)
    E = r["energy"]
    assert np.all(np.diff(E) <= 1e-12 * np.abs(E[:-1]))
    assert np.all(r["n_pos"] == r["n_plus"]) and r["n_plus"] == int((oracle.det_sign(A0) > 0).sum())
    plain = oracle.iterate(A0, tau, 30)
    assert int((oracle.det_sign(plain["A"]) > 0).sum()) < r["n_plus"]


@pytest.mark.parametrize("n", [2, 3])
def test_proposition_7_3_random(n):
    A0 = inputs.haar_field(n, (16, 16), 780 + n)
    for n_plus in (None, 40, 200):
        r = oracle.iterate_volume(A0, 2e-3, 15, n_plus)
        E = r["energy"]
        assert np.all(np.diff(E[1:]) <= 1e-12 * np.abs(E[1:-1]))
        assert np.all(r["n_pos"][1:] == r["n_plus"])
