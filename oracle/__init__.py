"""FP64 CPU oracle for the generalized MBO iteration on flat tori.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  The product
path (``paper_1711_01365_amd``) never imports it and shares no code with it.

The arithmetic lives in ``mbo_oracle.c`` (plain C, double precision, OpenMP
over independent lines / points).  This module only compiles it with gcc when
the shared object is missing or older than the source, and marshals numpy
arrays.  Fields are numpy arrays of shape ``(n, n, *grid)`` in C order, i.e.
``n*n`` real planes of ``prod(grid)`` points ("entry-planar").

What each function follows (Osting & Wang, arXiv:1711.01365):
  * ``heat``      diffusion step of Algorithm 1 on the flat torus, Section 5.1:
                  per entry plane, transform, multiply by the heat symbol
                  exp(-4 pi^2 tau |k|^2), transform back.
  * ``project``   projection step of Algorithm 1: closest orthogonal matrix
                  U V^t of Lemma 1.1, by one-sided Jacobi SVD.
  * ``energy``    Lyapunov functional of Section 4, with weight 1/prod(grid).
  * ``iterate``   Algorithm 1, with the per-iteration logs used by the tests.
  * ``heat_dtau`` derivative of the diffusion step in tau (symbol
                  -4 pi^2 |k|^2 exp(-4 pi^2 tau |k|^2)).
  * ``project_vjp``  vector-Jacobian product of the projection U V^t.
  * ``unroll_grad``  loss (1/2)||A_K - T||^2 of K steps of Algorithm 1 and its
                  gradients in A_0 and tau, by the chain rule run backwards.
  * ``volume_project``  Section 7: T^+ / T^- of Lemma 7.1, Delta E, and the
                  reassignment of Lemma 7.2 keeping exactly n_plus points in
                  SO(n) (the n_plus largest Delta E, ties by point index).
  * ``volume_select``   the selection alone (n_plus largest, ties by index).
  * ``iterate_volume``  volume-preserving MBO: Algorithm 1 with that step 2.
  * ``winding``   Section 6.1's index of an SO(2)-valued field along the loops
                  that wrap once in x (axis 0) and once in y (axis 1), from
                  the first column of each matrix (the field drawn in the
                  paper's figures), by summing the principal angle between
                  neighbouring samples.
  * ``relaxed_flow`` / ``relaxed_energy``  the gradient flows GD-1
                  (reaction U (Sigma - I) V^t) and GD-3 (A (A^t A - I)) by an
                  implicit diffusion step then an explicit reaction step, and
                  the energies E_{1,eps}, E_{2,eps} they descend.
  * ``band_T`` / ``band_width``  Theorem 5.2's tail mass T and the band width
                  w_b with T(w_b / 2 sqrt(tau)) = eps.
  * ``cheb_rule``  Chebyshev-point rule on [0, 1] (Fejer's first rule).
  * ``sphere_band``  the closest-point sample set of a sphere (Algorithm 2,
                  step 1): band cells, quadrature points, weights, closest points.
  * ``surface_diffuse`` / ``surface_iterate``  the closest-point surface
                  diffusion step by direct quadrature of the free-space heat
                  kernel, and Algorithm 1 on the sphere with it.
  * ``dft_naive`` / ``fft``   the discrete Fourier transform by definition and
                  by radix-2 Cooley-Tukey (cross-checked against each other).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mbo_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libmbo_oracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)
_i8 = ctypes.POINTER(ctypes.c_int8)


def build(force: bool = False) -> str:
    """Compile the oracle into ``oracle/libmbo_oracle.so`` (gcc, -O3, OpenMP).

    The instruction set is x86-64-v3 (AVX2), not -march=native: the object
    travels to other hosts.  No fast-math and no contraction into fused
    multiply-adds (-ffp-contract=off): every operation keeps its IEEE double
    rounding, as written.
    """
    stale = (not os.path.exists(_LIB_PATH)
             or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC))
    if force or stale:
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-std=c11", "-fopenmp", "-fPIC",
               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_dft_naive.argtypes = [ctypes.c_int, _i64, _d, _d, _d, _d, ctypes.c_int]
    lib.orc_fft.argtypes = [ctypes.c_int, _i64, _d, _d, ctypes.c_int]
    lib.orc_heat.argtypes = [ctypes.c_int, _i64, ctypes.c_int64, ctypes.c_double, _d, _d,
                             ctypes.c_int, _d]
    lib.orc_project.argtypes = [ctypes.c_int64, ctypes.c_int, _d, _d, _i8, _d, _i32]
    lib.orc_det_sign.argtypes = [ctypes.c_int64, ctypes.c_int, _d, _i8]
    lib.orc_energy.argtypes = [ctypes.c_int, _i64, ctypes.c_int, ctypes.c_double, _d,
                               ctypes.c_int, _d]
    lib.orc_iterate.argtypes = [ctypes.c_int, _i64, ctypes.c_int, ctypes.c_double, _d,
                                ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_int),
                                _d, _i64, _d, _d, ctypes.c_int]
    lib.orc_heat_dtau.argtypes = [ctypes.c_int, _i64, ctypes.c_int64, ctypes.c_double, _d, _d]
    lib.orc_project_vjp.argtypes = [ctypes.c_int64, ctypes.c_int, _d, _d, _d]
    lib.orc_unroll_grad.argtypes = [ctypes.c_int, _i64, ctypes.c_int, ctypes.c_double, _d, _d,
                                    ctypes.c_int, _d, _d, _d, _i64]
    lib.orc_volume_select.argtypes = [ctypes.c_int64, _d, ctypes.c_int64, _i8]
    lib.orc_volume_project.argtypes = [ctypes.c_int64, ctypes.c_int, _d, ctypes.c_int64, _d, _d,
                                       _i8]
    lib.orc_iterate_volume.argtypes = [ctypes.c_int, _i64, ctypes.c_int, ctypes.c_double, _d,
                                       ctypes.c_int, ctypes.c_int64, _d, _i64, _i64]
    lib.orc_relaxed_flow.argtypes = [ctypes.c_int, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double, _d, ctypes.c_int]
    lib.orc_relaxed_energy.argtypes = [ctypes.c_int, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       _d, _d]
    lib.orc_band_T.argtypes = [ctypes.c_double]
    lib.orc_band_T.restype = ctypes.c_double
    lib.orc_band_width.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.orc_band_width.restype = ctypes.c_double
    lib.orc_cheb_rule.argtypes = [ctypes.c_int, _d, _d]
    lib.orc_cheb_rule.restype = None
    lib.orc_sphere_band.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double, _i64,
                                    _i64, _d, _d, _d]
    lib.orc_surface_diffuse.argtypes = [ctypes.c_int64, _d, _d, _d, ctypes.c_int, ctypes.c_double, _d, _d]
    lib.orc_surface_iterate.argtypes = [ctypes.c_int64, _d, _d, _d, ctypes.c_int, ctypes.c_double, _d,
                                        ctypes.c_int, _i64]
    lib.orc_heat_at.argtypes = [ctypes.c_int64, _d, _d, ctypes.c_int, ctypes.c_double, _d, ctypes.c_int64, _d, _d]
    lib.orc_weighted_select.argtypes = [ctypes.c_int64, _d, _i64, ctypes.c_int64, _i8]
    lib.orc_surface_iterate_volume.argtypes = [ctypes.c_int64, _d, _d, _d, _i64, ctypes.c_int, ctypes.c_double, _d,
                                               ctypes.c_int, _i64, _i64, _i64]
    lib.orc_revolution_cp.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, _d]
    lib.orc_revolution_cp.restype = ctypes.c_double
    lib.orc_revolution_band.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                        _i64, _i64, _d, _d, _d]
    lib.orc_num_threads.argtypes = []
    for f in ("orc_dft_naive", "orc_fft", "orc_heat", "orc_project", "orc_det_sign",
              "orc_energy", "orc_iterate", "orc_num_threads", "orc_heat_dtau", "orc_project_vjp",
              "orc_unroll_grad", "orc_volume_select", "orc_volume_project",
              "orc_iterate_volume", "orc_relaxed_flow", "orc_relaxed_energy", "orc_sphere_band",
              "orc_surface_diffuse", "orc_surface_iterate", "orc_heat_at", "orc_weighted_select",
              "orc_surface_iterate_volume", "orc_revolution_band"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_load().orc_num_threads())


def set_num_threads(t: int) -> None:
    """Threads for the oracle's later OpenMP loops (for timing only)."""
    lib = _load()
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    lib.orc_set_num_threads(int(t))


def _ptr(a, t=_d):
    return None if a is None else a.ctypes.data_as(t)


def _grid(shape):
    g = np.ascontiguousarray(np.asarray(shape, dtype=np.int64))
    return g, len(shape)


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s failed with code %d" % (what, rc))


def dft_naive(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """Unscaled d-dimensional DFT by its definition (sign -1 forward, +1 inverse)."""
    lib = _load()
    x = np.asarray(x, dtype=np.complex128)
    g, d = _grid(x.shape)
    xr = np.ascontiguousarray(x.real)
    xi = np.ascontiguousarray(x.imag)
    yr = np.empty_like(xr)
    yi = np.empty_like(xi)
    _check(lib.orc_dft_naive(d, _ptr(g, _i64), _ptr(xr), _ptr(xi), _ptr(yr), _ptr(yi), sign),
           "dft_naive")
    return yr + 1j * yi


def fft(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """Unscaled d-dimensional radix-2 FFT (sign -1 forward, +1 inverse)."""
    lib = _load()
    x = np.asarray(x, dtype=np.complex128)
    g, d = _grid(x.shape)
    re = np.ascontiguousarray(x.real).copy()
    im = np.ascontiguousarray(x.imag).copy()
    _check(lib.orc_fft(d, _ptr(g, _i64), _ptr(re), _ptr(im), sign), "fft")
    return re + 1j * im


def heat(planes: np.ndarray, tau: float, grid_ndim: int, naive: bool = False):
    """Apply e^{tau Delta} to every real plane; returns (out, max |Im| after inverse).

    ``planes`` has shape ``(*lead, *grid)`` with ``grid_ndim`` trailing grid axes.
    """
    lib = _load()
    a = np.ascontiguousarray(planes, dtype=np.float64)
    grid = a.shape[a.ndim - grid_ndim:]
    nplanes = int(np.prod(a.shape[:a.ndim - grid_ndim], dtype=np.int64))
    g, d = _grid(grid)
    out = np.empty_like(a)
    mi = np.zeros(1)
    _check(lib.orc_heat(d, _ptr(g, _i64), nplanes, float(tau), _ptr(a), _ptr(out),
                        int(naive), _ptr(mi)), "heat")
    return out, float(mi[0])


def project(A: np.ndarray):
    """Closest orthogonal matrix per point.  A has shape (n, n, *grid).

    Returns (Q, detsign int8 [*grid], sigma [n, *grid] unsorted, sweeps int32 [*grid]).
    """
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    assert A.shape[1] == n
    grid = A.shape[2:]
    P = int(np.prod(grid, dtype=np.int64))
    Q = np.empty_like(A)
    ds = np.empty(grid, dtype=np.int8)
    sg = np.empty((n,) + tuple(grid), dtype=np.float64)
    sw = np.empty(grid, dtype=np.int32)
    _check(lib.orc_project(P, n, _ptr(A), _ptr(Q), _ptr(ds, _i8), _ptr(sg), _ptr(sw, _i32)),
           "project")
    return Q, ds, sg, sw


def det_sign(A: np.ndarray) -> np.ndarray:
    """sgn(det A) per point with sgn(0) = +1."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    grid = A.shape[2:]
    P = int(np.prod(grid, dtype=np.int64))
    ds = np.empty(grid, dtype=np.int8)
    _check(lib.orc_det_sign(P, n, _ptr(A), _ptr(ds, _i8)), "det_sign")
    return ds


def energy(A: np.ndarray, tau: float, naive: bool = False) -> float:
    """Lyapunov functional E(A) = (1/tau) mean_p [n - <A, e^{tau Delta} A>_F]."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    g, d = _grid(A.shape[2:])
    E = np.zeros(1)
    _check(lib.orc_energy(d, _ptr(g, _i64), n, float(tau), _ptr(A), int(naive), _ptr(E)),
           "energy")
    return float(E[0])


def iterate(A0: np.ndarray, tau: float, K: int, tol: float = 0.0, naive: bool = False):
    """Algorithm 1 for K iterations (or until max|A_s - A_{s-1}| <= tol when tol > 0).

    Returns a dict: A (last iterate), iters, energy [iters+1], flips [iters],
    delta [iters], max_imag.
    """
    lib = _load()
    A = np.ascontiguousarray(A0, dtype=np.float64).copy()
    n = A.shape[0]
    g, d = _grid(A.shape[2:])
    it = ctypes.c_int(0)
    en = np.zeros(K + 1)
    fl = np.zeros(max(K, 1), dtype=np.int64)
    dl = np.zeros(max(K, 1))
    mi = np.zeros(1)
    _check(lib.orc_iterate(d, _ptr(g, _i64), n, float(tau), _ptr(A), int(K), float(tol),
                           ctypes.byref(it), _ptr(en), _ptr(fl, _i64), _ptr(dl), _ptr(mi),
                           int(naive)), "iterate")
    s = it.value
    return {"A": A, "iters": s, "energy": en[: s + 1], "flips": fl[:s], "delta": dl[:s],
            "max_imag": float(mi[0])}


def heat_dtau(planes: np.ndarray, tau: float, grid_ndim: int) -> np.ndarray:
    """d/dtau of e^{tau Delta} applied to every real plane (FFT route)."""
    lib = _load()
    a = np.ascontiguousarray(planes, dtype=np.float64)
    grid = a.shape[a.ndim - grid_ndim:]
    nplanes = int(np.prod(a.shape[:a.ndim - grid_ndim], dtype=np.int64))
    g, d = _grid(grid)
    out = np.empty_like(a)
    _check(lib.orc_heat_dtau(d, _ptr(g, _i64), nplanes, float(tau), _ptr(a), _ptr(out)),
           "heat_dtau")
    return out


def project_vjp(A: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Cotangent of A for the cotangent G of Q = U V^t, per point.  Shapes (n, n, *grid)."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    assert A.shape == G.shape
    n = A.shape[0]
    P = int(np.prod(A.shape[2:], dtype=np.int64))
    GA = np.empty_like(A)
    _check(lib.orc_project_vjp(P, n, _ptr(A), _ptr(G), _ptr(GA)), "project_vjp")
    return GA


def unroll_grad(A0: np.ndarray, T: np.ndarray, tau: float, K: int):
    """Loss (1/2) sum ||A_K - T||_F^2 of K steps of Algorithm 1 and its gradients.

    Returns a dict: loss, gA0 (shape of A0), gtau, flips [K] of the forward run.
    """
    lib = _load()
    A0 = np.ascontiguousarray(A0, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    assert A0.shape == T.shape
    n = A0.shape[0]
    g, d = _grid(A0.shape[2:])
    loss = np.zeros(1)
    gtau = np.zeros(1)
    gA0 = np.empty_like(A0)
    fl = np.zeros(max(K, 1), dtype=np.int64)
    _check(lib.orc_unroll_grad(d, _ptr(g, _i64), n, float(tau), _ptr(A0), _ptr(T), int(K),
                               _ptr(loss), _ptr(gA0), _ptr(gtau), _ptr(fl, _i64)), "unroll_grad")
    return {"loss": float(loss[0]), "gA0": gA0, "gtau": float(gtau[0]), "flips": fl[:K]}


def volume_select(dE: np.ndarray, n_plus: int) -> np.ndarray:
    """int8 mask of the n_plus largest values of dE (any shape, flat index order
    breaks ties: the lower index first)."""
    lib = _load()
    v = np.ascontiguousarray(dE, dtype=np.float64)
    sel = np.empty(v.shape, dtype=np.int8)
    _check(lib.orc_volume_select(int(v.size), _ptr(v), int(n_plus), _ptr(sel, _i8)), "volume_select")
    return sel


def volume_project(A: np.ndarray, n_plus: int):
    """Volume-constrained projection (Section 7, Lemma 7.2).  A has shape (n, n, *grid).

    Returns (B, dE [*grid], selected int8 [*grid]): B = T^+ on the n_plus points
    with the largest Delta E (ties by ascending flat index), T^- elsewhere.
    """
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    assert A.shape[1] == n
    grid = A.shape[2:]
    P = int(np.prod(grid, dtype=np.int64))
    B = np.empty_like(A)
    dE = np.empty(grid, dtype=np.float64)
    sel = np.empty(grid, dtype=np.int8)
    _check(lib.orc_volume_project(P, n, _ptr(A), int(n_plus), _ptr(B), _ptr(dE), _ptr(sel, _i8)),
           "volume_project")
    return B, dE, sel


def iterate_volume(A0: np.ndarray, tau: float, K: int, n_plus: int | None = None):
    """Volume-preserving MBO (Section 7) for K iterations.

    n_plus None takes #{det A_0 >= 0}.  Returns a dict: A (last iterate),
    energy [K+1], n_pos [K+1] (#{det A_s >= 0}), n_plus.
    """
    lib = _load()
    A = np.ascontiguousarray(A0, dtype=np.float64).copy()
    n = A.shape[0]
    g, d = _grid(A.shape[2:])
    en = np.zeros(K + 1)
    npos = np.zeros(K + 1, dtype=np.int64)
    used = np.zeros(1, dtype=np.int64)
    _check(lib.orc_iterate_volume(d, _ptr(g, _i64), n, float(tau), _ptr(A), int(K),
                                  -1 if n_plus is None else int(n_plus), _ptr(en),
                                  _ptr(npos, _i64), _ptr(used, _i64)), "iterate_volume")
    return {"A": A, "energy": en, "n_pos": npos, "n_plus": int(used[0])}


def winding(A: np.ndarray):
    """Index of the first-column field of a 2-D O(2) field A (2, 2, N0, N1) along
    the loops x -> (x, y_j) (one per column j: [gamma]_{1,0}) and y -> (x_i, y)
    (one per row i: [gamma]_{0,1}): (1/2 pi) times the sum over consecutive
    samples, the last joined to the first, of the angle from one first column to
    the next in (-pi, pi].  Returns (w_x [N1], w_y [N0]) as floats."""
    A = np.asarray(A, dtype=np.float64)
    assert A.shape[:2] == (2, 2) and A.ndim == 4
    u, v = A[0, 0], A[1, 0]
    out = []
    for axis in (0, 1):
        un, vn = np.roll(u, -1, axis=axis), np.roll(v, -1, axis=axis)
        step = np.arctan2(u * vn - v * un, u * un + v * vn)
        out.append(step.sum(axis=axis) / (2.0 * np.pi))
    return out[0], out[1]


def relaxed_flow(A0: np.ndarray, kind: int, eps: float, dt: float, K: int) -> np.ndarray:
    """K steps of GD-1 (kind 1) or GD-3 (kind 3): B = (I - dt Delta)^-1 A, then
    A = B - (dt/eps^2) N(B).  A0 has shape (n, n, *grid); returns the last A."""
    lib = _load()
    A = np.ascontiguousarray(A0, dtype=np.float64).copy()
    n = A.shape[0]
    g, d = _grid(A.shape[2:])
    _check(lib.orc_relaxed_flow(d, _ptr(g, _i64), n, int(kind), float(eps), float(dt), _ptr(A), int(K)),
           "relaxed_flow")
    return A


def relaxed_energy(A: np.ndarray, kind: int, eps: float) -> float:
    """E_{1,eps} (kind 1) or E_{2,eps} (kind 3) of A on the unit torus."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    g, d = _grid(A.shape[2:])
    E = np.zeros(1)
    _check(lib.orc_relaxed_energy(d, _ptr(g, _i64), n, int(kind), float(eps), _ptr(A), _ptr(E)),
           "relaxed_energy")
    return float(E[0])


def band_T(x: float) -> float:
    """T(x) of Theorem 5.2."""
    return float(_load().orc_band_T(float(x)))


def band_width(tau: float, eps: float) -> float:
    """w_b with T(w_b / (2 sqrt(tau))) = eps (Theorem 5.2)."""
    return float(_load().orc_band_width(float(tau), float(eps)))


def cheb_rule(p: int):
    """(nodes, weights) of the p-point Chebyshev-point rule on [0, 1]."""
    x = np.zeros(p)
    w = np.zeros(p)
    _load().orc_cheb_rule(int(p), _ptr(x), _ptr(w))
    return x, w


def sphere_band(R: float, dx: float, p: int, tau: float, eps: float):
    """Sample set of the sphere of radius R: dict with xq, xc ([3, m]), w ([m]),
    cells (band cell count), wb (band width)."""
    lib = _load()
    wb = band_width(tau, eps)
    cnt = np.zeros(1, dtype=np.int64)
    cells = np.zeros(1, dtype=np.int64)
    _check(lib.orc_sphere_band(float(R), float(dx), int(p), wb, _ptr(cnt, _i64), _ptr(cells, _i64), None,
                               None, None), "sphere_band")
    m = int(cnt[0])
    xq = np.zeros((3, m))
    xc = np.zeros((3, m))
    w = np.zeros(m)
    _check(lib.orc_sphere_band(float(R), float(dx), int(p), wb, _ptr(cnt, _i64), None, _ptr(xq), _ptr(xc),
                               _ptr(w)), "sphere_band")
    return {"xq": xq, "xc": xc, "w": w, "cells": int(cells[0]), "wb": wb}


REV_SPHERE, REV_PEANUT = 0, 1


def revolution_cp(kind: int, pts: np.ndarray, R: float = 1.0):
    """Closest points [3, k] and distances [k] of points pts [3, k] on a surface
    of revolution (REV_SPHERE of radius R, or REV_PEANUT)."""
    lib = _load()
    pts = np.asarray(pts, dtype=np.float64)
    out = np.zeros_like(pts)
    dist = np.zeros(pts.shape[1])
    c = np.zeros(3)
    for q in range(pts.shape[1]):
        dist[q] = lib.orc_revolution_cp(int(kind), float(R), float(pts[0, q]), float(pts[1, q]), float(pts[2, q]),
                                        _ptr(c))
        out[:, q] = c
    return out, dist


def revolution_band(kind: int, dx: float, p: int, tau: float, eps: float, R: float = 1.0):
    """Sample set of a surface of revolution, as sphere_band."""
    lib = _load()
    wb = band_width(tau, eps)
    cnt = np.zeros(1, dtype=np.int64)
    cells = np.zeros(1, dtype=np.int64)
    _check(lib.orc_revolution_band(int(kind), float(R), float(dx), int(p), wb, _ptr(cnt, _i64), _ptr(cells, _i64),
                                   None, None, None), "revolution_band")
    m = int(cnt[0])
    xq = np.zeros((3, m))
    xc = np.zeros((3, m))
    w = np.zeros(m)
    _check(lib.orc_revolution_band(int(kind), float(R), float(dx), int(p), wb, _ptr(cnt, _i64), None, _ptr(xq),
                                   _ptr(xc), _ptr(w)), "revolution_band")
    return {"xq": xq, "xc": xc, "w": w, "cells": int(cells[0]), "wb": wb}


def surface_diffuse(band: dict, A: np.ndarray, tau: float) -> np.ndarray:
    """Closest-point surface diffusion of A (n, n, m) over the band's samples."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    n, m = A.shape[0], A.shape[2]
    out = np.empty_like(A)
    xq = np.ascontiguousarray(band["xq"])
    xc = np.ascontiguousarray(band["xc"])
    w = np.ascontiguousarray(band["w"])
    _check(lib.orc_surface_diffuse(m, _ptr(xq), _ptr(xc), _ptr(w), n, float(tau), _ptr(A), _ptr(out)),
           "surface_diffuse")
    return out


def heat_at(band: dict, A: np.ndarray, tau: float, xt: np.ndarray) -> np.ndarray:
    """The band's heat convolution of A (n, n, m) at target points xt [3, nt]:
    (n, n, nt)."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    n, m = A.shape[0], A.shape[2]
    xt = np.ascontiguousarray(xt, dtype=np.float64)
    nt = xt.shape[1]
    out = np.empty((n, n, nt))
    _check(lib.orc_heat_at(m, _ptr(np.ascontiguousarray(band["xq"])), _ptr(np.ascontiguousarray(band["w"])), n,
                           float(tau), _ptr(A), nt, _ptr(xt), _ptr(out)), "heat_at")
    return out


def surface_weights(band: dict, dx: float) -> np.ndarray:
    """Integer volume weights of the samples: the quadrature weight in units of
    2^-30 dx^3, rounded (sums of them are exact)."""
    return np.rint(np.asarray(band["w"]) / dx ** 3 * 2.0 ** 30).astype(np.int64)


def weighted_select(dE: np.ndarray, W: np.ndarray, V: int) -> np.ndarray:
    """int8 mask of Algorithm 3's selection: dE in descending order (ties by
    ascending index) while the weight taken is below V."""
    lib = _load()
    v = np.ascontiguousarray(dE, dtype=np.float64).ravel()
    w = np.ascontiguousarray(W, dtype=np.int64).ravel()
    sel = np.empty(v.size, dtype=np.int8)
    _check(lib.orc_weighted_select(int(v.size), _ptr(v), _ptr(w, _i64), int(V), _ptr(sel, _i8)), "weighted_select")
    return sel


def surface_iterate_volume(band: dict, W: np.ndarray, A0: np.ndarray, tau: float, K: int, V=None):
    """K steps of volume-preserving MBO on the sphere (Algorithm 3 selection).
    Returns (A, flips [K], V used)."""
    lib = _load()
    A = np.ascontiguousarray(A0, dtype=np.float64).copy()
    n, m = A.shape[0], A.shape[2]
    fl = np.zeros(max(K, 1), dtype=np.int64)
    vu = np.zeros(1, dtype=np.int64)
    vin = None if V is None else np.array([int(V)], dtype=np.int64)
    w = np.ascontiguousarray(W, dtype=np.int64)
    _check(lib.orc_surface_iterate_volume(m, _ptr(np.ascontiguousarray(band["xq"])), _ptr(np.ascontiguousarray(band["xc"])),
                                          _ptr(np.ascontiguousarray(band["w"])), _ptr(w, _i64), n, float(tau), _ptr(A),
                                          int(K), None if vin is None else _ptr(vin, _i64), _ptr(vu, _i64),
                                          _ptr(fl, _i64)), "surface_iterate_volume")
    return A, fl[:K], int(vu[0])


def surface_iterate(band: dict, A0: np.ndarray, tau: float, K: int):
    """K steps of Algorithm 1 on the sphere.  Returns (A, flips [K])."""
    lib = _load()
    A = np.ascontiguousarray(A0, dtype=np.float64).copy()
    n, m = A.shape[0], A.shape[2]
    fl = np.zeros(max(K, 1), dtype=np.int64)
    xq = np.ascontiguousarray(band["xq"])
    xc = np.ascontiguousarray(band["xc"])
    w = np.ascontiguousarray(band["w"])
    _check(lib.orc_surface_iterate(m, _ptr(xq), _ptr(xc), _ptr(w), n, float(tau), _ptr(A), int(K),
                                   _ptr(fl, _i64)), "surface_iterate")
    return A, fl[:K]
