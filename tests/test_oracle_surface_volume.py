"""Pins of the oracle's volume-preserving MBO on a surface (Section 7,
Algorithm 3 with the reassignment of Lemma 7.2, on the closest-point sphere).

What fixes the answer independently of the oracle's code:
  * the selection is a prefix of the descending order of Delta E (ties by
    ascending index) and the shortest one whose weight reaches V (Algorithm 3's
    loop), checked as properties on random inputs with ties, plus V <= 0 and V
    above the total;
  * with equal weights it is the flat-torus rule (the first ceil(V / w) values),
    the oracle's pinned volume_select;
  * with equal weights (p = 1) the whole surface step equals the flat-torus
    volume projection of the diffused field;
  * the iteration keeps the SO(n) volume in [V, V + max w) at every step on
    the printed matrices' octant, with V defaulting to the initial volume.
"""
import numpy as np
import pytest

import oracle
from paper_1711_01365_amd import inputs


def _order(dE):
    # positions in the descending order, ties by ascending index
    return np.lexsort((np.arange(dE.size), -dE))


@pytest.mark.parametrize("seed", range(6))
def test_selection_is_the_shortest_prefix_reaching_V(seed):
    rng = np.random.default_rng(1100 + seed)
    m = 500
    dE = rng.integers(-20, 20, m).astype(np.float64) * 0.25  # many ties
    dE[rng.integers(0, m, 10)] = -0.0
    W = rng.integers(1, 1000, m).astype(np.int64)
    for V in (1, int(W.sum()) // 3, int(W.sum()) // 2, int(W.sum()) - 1, int(W.sum())):
        sel = oracle.weighted_select(dE, W, V).astype(bool)
        order = _order(dE)
        k = int(sel.sum())
        assert sel[order[:k]].all() and not sel[order[k:]].any()  # a prefix of the order
        taken = W[order[:k]]
        assert taken.sum() >= V and taken[:-1].sum() < V  # the shortest one reaching V


def test_selection_edge_cases():
    dE = np.array([3.0, 1.0, 2.0, 2.0])
    W = np.array([5, 5, 5, 5], dtype=np.int64)
    assert not oracle.weighted_select(dE, W, 0).any()
    assert not oracle.weighted_select(dE, W, -7).any()
    assert oracle.weighted_select(dE, W, 10 ** 6).all()
    # 3.0 (index 0) first, then the tie 2.0 at indices 2 < 3
    assert list(oracle.weighted_select(dE, W, 6)) == [1, 0, 1, 0]
    assert list(oracle.weighted_select(dE, W, 10)) == [1, 0, 1, 0]
    assert list(oracle.weighted_select(dE, W, 11)) == [1, 0, 1, 1]


@pytest.mark.parametrize("seed", range(4))
def test_equal_weights_give_the_flat_torus_rule(seed):
    rng = np.random.default_rng(1200 + seed)
    m = 2000
    dE = np.round(rng.standard_normal(m), 2)
    W = np.full(m, 7, dtype=np.int64)
    for V in (0, 1, 6, 7, 8, 700, 13999, 14000):
        n_plus = min(m, -(-V // 7)) if V > 0 else 0
        assert np.array_equal(oracle.weighted_select(dE, W, V), oracle.volume_select(dE, n_plus))


def test_equal_weights_step_is_the_flat_torus_projection():
    """p = 1: every sample has the weight dx^3, so one volume-preserving step on
    the sphere is the flat-torus volume projection of the diffused field."""
    tau, dx = 0.02, 0.15
    b = oracle.sphere_band(1.0, dx, 1, tau, 1e-6)
    W = oracle.surface_weights(b, dx)
    assert (W == W[0]).all()
    m = b["w"].size
    rng = np.random.default_rng(1300)
    A0 = oracle.project(rng.standard_normal((3, 3, m)))[0]
    V = int(W[0]) * (m // 3) + 5
    A1, _, vu = oracle.surface_iterate_volume(b, W, A0, tau, 1, V)
    D = oracle.surface_diffuse(b, A0, tau)
    n_plus = -(-V // int(W[0]))
    B, _, _ = oracle.volume_project(D, n_plus)
    assert vu == V and np.abs(A1 - B).max() < 1e-13


def test_iteration_keeps_the_volume():
    """p = 3 (unequal weights): V defaults to the weight of the samples with
    det >= 0, and every step keeps the SO(n) volume in [V, V + max w)."""
    M = inputs.SPHERE_MATRICES
    tau, dx = 0.01, 0.3
    b = oracle.sphere_band(1.0, dx, 3, tau, 1e-6)
    W = oracle.surface_weights(b, dx)
    assert W.max() > W.min()
    Q = oracle.project(np.stack([M[0], M[1]], axis=-1).reshape(3, 3, 2))[0]
    x, y, z = b["xc"]
    inside = (x < 0) & (y < 0) & (z > 0)
    A = np.where(inside[None, None, :], Q[:, :, 0:1], Q[:, :, 1:2])
    V0 = int(W[oracle.det_sign(A) >= 0].sum())
    _, _, vu = oracle.surface_iterate_volume(b, W, A, tau, 0)
    assert vu == V0
    A3, fl, vu = oracle.surface_iterate_volume(b, W, A, tau, 3, V0)
    assert vu == V0 and fl.sum() > 0
    for K in (1, 2):
        AK, _, _ = oracle.surface_iterate_volume(b, W, A, tau, K, V0)
        vol = int(W[oracle.det_sign(AK) > 0].sum())
        assert V0 <= vol < V0 + W.max(), (K, V0, vol)
    vol = int(W[oracle.det_sign(A3) > 0].sum())
    assert V0 <= vol < V0 + W.max()
