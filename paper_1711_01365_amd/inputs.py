"""Seeded synthetic inputs shared by the HIP path's tests/benchmarks and the oracle.

This module holds no arithmetic of the method itself: it only draws the initial
fields (and the parameters of the batched workload) from numpy's
``default_rng``.  The same float64 arrays feed the oracle and the GPU path; the
FP32 paths receive them rounded to float32.

Fields are returned in the entry-planar layout ``(n, n, *grid)``: entry (i, j)
of the matrix at every grid point is one contiguous real plane.

The paper measures on no dataset; its flat-torus experiments start from
analytic or random fields (Section 6.1).  The workloads below are synthetic
stand-ins with the sizes and value distributions of the measured configurations.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np


def uniform_field(n: int, grid: Tuple[int, ...], seed: int) -> np.ndarray:
    """Entries iid Uniform[-1, 1)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(n, n) + tuple(grid))


def normal_field(n: int, grid: Tuple[int, ...], seed: int) -> np.ndarray:
    """Entries iid N(0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=(n, n) + tuple(grid))


def haar_field(n: int, grid: Tuple[int, ...], seed: int) -> np.ndarray:
    """Haar-distributed O(n) matrix per point: QR of an iid N(0,1) matrix with the
    columns of Q multiplied by sgn(diag R) (Mezzadri's sign fix)."""
    rng = np.random.default_rng(seed)
    P = int(np.prod(grid))
    G = rng.standard_normal(size=(P, n, n))
    Q, R = np.linalg.qr(G)
    s = np.sign(np.diagonal(R, axis1=1, axis2=2))
    s[s == 0] = 1.0
    Q = Q * s[:, None, :]
    return np.ascontiguousarray(np.moveaxis(Q, 0, -1)).reshape((n, n) + tuple(grid))


def star_defect_field(grid: Tuple[int, int]) -> np.ndarray:
    """The closed star-shaped line defect of the paper's first flat-torus example
    (Section 6.1; also the volume-preserving example of Section 7), n = 2.

    On [-1/2, 1/2)^2 sampled at x = -1/2 + i/N0 (axis 0), y = -1/2 + j/N1
    (axis 1), with alpha = (pi/2) sin(2 pi (x + y)) and polar coordinates
    (r, theta) of (x, y): the rotation by alpha inside r < 0.3 + 0.06 sin(6 theta),
    the reflection [[cos a, sin a], [sin a, -cos a]] outside.
    """
    N0, N1 = grid
    x = -0.5 + np.arange(N0) / N0
    y = -0.5 + np.arange(N1) / N1
    X, Y = np.meshgrid(x, y, indexing="ij")
    al = 0.5 * np.pi * np.sin(2.0 * np.pi * (X + Y))
    inside = np.hypot(X, Y) < 0.3 + 0.06 * np.sin(6.0 * np.arctan2(Y, X))
    c, s = np.cos(al), np.sin(al)
    A = np.empty((2, 2, N0, N1))
    A[0, 0] = c
    A[0, 1] = np.where(inside, -s, s)
    A[1, 0] = s
    A[1, 1] = np.where(inside, c, -c)
    return A


def line_defect_field(grid: Tuple[int, int], winding: bool) -> np.ndarray:
    """The two closed line defects of the paper's second and third flat-torus
    examples (Section 6.1), n = 2.

    Same sampling as star_defect_field.  The rotation by alpha where
    x > 0.25 |sin(2.5 pi y)| + 0.2 or x < -0.25 |sin(2.5 pi y)| - 0.2, the
    reflection [[cos a, sin a], [sin a, -cos a]] elsewhere, with
    alpha = pi sin(2 pi y) (second example) or alpha = 2 pi y (third example,
    winding = True: the angle turns once along every loop in y).
    """
    N0, N1 = grid
    x = -0.5 + np.arange(N0) / N0
    y = -0.5 + np.arange(N1) / N1
    X, Y = np.meshgrid(x, y, indexing="ij")
    al = 2.0 * np.pi * Y if winding else np.pi * np.sin(2.0 * np.pi * Y)
    w = 0.25 * np.abs(np.sin(2.5 * np.pi * Y)) + 0.2
    rot = (X > w) | (X < -w)
    c, s = np.cos(al), np.sin(al)
    A = np.empty((2, 2, N0, N1))
    A[0, 0] = c
    A[0, 1] = np.where(rot, -s, s)
    A[1, 0] = s
    A[1, 1] = np.where(rot, c, -c)
    return A


def linear_angle_field(grid: Tuple[int, int], m: int, k: int) -> np.ndarray:
    """SO(2) field with angle 2 pi (m x + k y) (x = i/N0, y = j/N1): its first
    column turns m times along every loop in x and k times along every loop in y."""
    N0, N1 = grid
    x = np.arange(N0) / N0
    y = np.arange(N1) / N1
    X, Y = np.meshgrid(x, y, indexing="ij")
    al = 2.0 * np.pi * (m * X + k * Y)
    c, s = np.cos(al), np.sin(al)
    return np.stack([np.stack([c, -s]), np.stack([s, c])])


@dataclass
class Workload:
    """One measured configuration: field size, time step, iteration count."""
    name: str
    n: int
    grid: Tuple[int, ...]
    tau: float
    iters: int
    init: str            # "uniform" | "haar" | "normal" | "star" | "lines" | "lines_winding"
    seed: int

    def field(self) -> np.ndarray:
        if self.init in ("star", "lines", "lines_winding"):
            assert self.n == 2 and len(self.grid) == 2
            if self.init == "star":
                return star_defect_field(self.grid)
            return line_defect_field(self.grid, self.init == "lines_winding")
        gen = {"uniform": uniform_field, "haar": haar_field, "normal": normal_field}[self.init]
        return gen(self.n, self.grid, self.seed)

    @property
    def points(self) -> int:
        return int(np.prod(self.grid))


# The five measured configurations (sizes, distributions and seeds).
PARITY_64 = Workload("n2_64x64_f64", 2, (64, 64), 1e-3, 20, "uniform", 0)
HAAR_512 = Workload("n3_512x512_haar", 3, (512, 512), 2e-4, 200, "haar", 1)
NORMAL_128_3D = Workload("n3_128x128x128_normal", 3, (128, 128, 128), 5e-4, 100, "normal", 2)
# bandwidth control: the measured configuration's per-point work on a grid 16x
# larger (tau scaled with the grid spacing squared, so tau / h^2 is unchanged)
CONTROL_2048 = Workload("n3_2048x2048_haar", 3, (2048, 2048), 2e-4 / 16, 20, "haar", 11)
ADJOINT_256 = Workload("n3_256x256_adjoint", 3, (256, 256), 1e-3, 50, "haar", 4001)
ADJOINT_TARGET_SEED = 4002
ADJOINT_TARGET_TAU = 1e-2
ADJOINT_CHECKPOINT = 10
# The paper's three flat-torus examples (Section 6.1), n = 2 on 1024^2.  The
# printed steps (tau = 8 dx and 64 dx, dx = 1/1024) are read as the coefficient
# of integer wavenumbers in the heat multiplier, exp(-tau |m|^2): on the unit
# torus that is the diffusion time tau / (4 pi^2).  (Taken as the unit-torus
# time itself, the second and third examples become uniform within two steps,
# unlike the evolutions the paper describes.)
PAPER_TAU_SCALE = 1.0 / (4.0 * np.pi ** 2)
EXAMPLE_STAR = Workload("n2_1024x1024_star", 2, (1024, 1024), 8.0 / 1024 * PAPER_TAU_SCALE, 400, "star", 0)
EXAMPLE_LINES = Workload("n2_1024x1024_lines", 2, (1024, 1024), 64.0 / 1024 * PAPER_TAU_SCALE, 200, "lines", 0)
EXAMPLE_WINDING = Workload("n2_1024x1024_lines_winding", 2, (1024, 1024), 64.0 / 1024 * PAPER_TAU_SCALE, 200,
                           "lines_winding", 0)
# volume-preserving MBO (Section 7): the paper's example (the star-shaped
# defect with the first example's step), and the measured n = 3 configuration
# with the volume of its initial SO(3) region held fixed
VOLUME_STAR_1024 = Workload("n2_1024x1024_star_volume", 2, (1024, 1024), EXAMPLE_STAR.tau, 100, "star", 0)
VOLUME_HAAR_512 = Workload("n3_512x512_haar_volume", 3, (512, 512), 2e-4, 200, "haar", 1)


@dataclass
class BatchedWorkload:
    """64 independent 2-D fields of mixed n, grid size and time step."""
    seed: int = 3
    count: int = 64
    iters: int = 50
    members: List[Workload] = field(default_factory=list)

    def __post_init__(self):
        if not self.members:
            rng = np.random.default_rng(self.seed)
            ns = rng.integers(2, 5, size=self.count)
            Ns = rng.choice(np.array([128, 256, 512, 1024]), size=self.count)
            taus = 10.0 ** rng.uniform(-4.0, -2.0, size=self.count)
            self.members = [
                Workload("batched_%02d" % b, int(ns[b]), (int(Ns[b]), int(Ns[b])),
                         float(taus[b]), self.iters, "uniform", 3000 + b)
                for b in range(self.count)
            ]

    @property
    def points(self) -> int:
        return sum(m.points for m in self.members)


# The sphere experiment (Section 6.2): unit sphere, band cells dx = 0.05 with
# p = 3 Chebyshev points per axis, tau = 0.005, eps = 1e-6, n = 3; the initial
# field takes the first printed matrix in the octant x < 0, y < 0, z > 0 and the
# second one elsewhere.  As printed the matrices are not orthogonal (raw inputs of
# the first projection); the first has det < 0, the second det > 0.
@dataclass
class SphereWorkload:
    name: str
    R: float
    dx: float
    p: int
    tau: float
    eps: float
    n: int
    iters: int


SPHERE_MATRICES = np.array([[[0.392227, 0.706046, 0.046171],
                             [0.655478, 0.031833, 0.097132],
                             [0.171187, 0.276923, 0.82346]],
                            [[0.699077, 0.547216, 0.257508],
                             [0.890903, 0.138624, 0.840717],
                             [0.959291, 0.149294, 0.254282]]])
SPHERE_PAPER = SphereWorkload("sphere_R1_dx0.05_p3_tau0.005", 1.0, 0.05, 3, 0.005, 1e-6, 3, 20)
# the volume-preserving sphere of Section 7 (same band construction, tau = 0.01)
SPHERE_VOLUME_PAPER = SphereWorkload("sphere_volume_R1_dx0.05_p3_tau0.01", 1.0, 0.05, 3, 0.01, 1e-6, 3, 20)


def sphere_octant_field(xc: np.ndarray) -> np.ndarray:
    """(3, 3, m) field over samples with closest points xc [3, m]: the first
    printed matrix where x < 0, y < 0, z > 0, the second elsewhere."""
    x, y, z = xc
    inside = (x < 0) & (y < 0) & (z > 0)
    return np.where(inside[None, None, :], SPHERE_MATRICES[0][:, :, None], SPHERE_MATRICES[1][:, :, None])


# The peanut experiment (Section 6.3): dx = 0.04, p = 4, tau = 0.032,
# eps = 1e-6, n = 3; the first printed matrix where x > sqrt((y^2 + z^2)(y^2 + 0.1) / 1.5),
# the second elsewhere (the sphere's matrices, raw).
PEANUT_PAPER = SphereWorkload("peanut_dx0.04_p4_tau0.032", 1.0, 0.04, 4, 0.032, 1e-6, 3, 10)


def peanut_field(xc: np.ndarray) -> np.ndarray:
    """(3, 3, m) field over samples with closest points xc [3, m]: the paper's
    peanut initial condition."""
    x, y, z = xc
    first = x > np.sqrt((y * y + z * z) * (y * y + 0.1) / 1.5)
    return np.where(first[None, None, :], SPHERE_MATRICES[0][:, :, None], SPHERE_MATRICES[1][:, :, None])
