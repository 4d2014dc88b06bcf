"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 path <= 1e-12 max-abs on field entries; FP32 path <= 1e-5 on
points whose projection is well conditioned (sigma_{n-1} + sigma_n >= 0.1, the
polar factor's absolute condition number being 2 / (sigma_{n-1} + sigma_n));
integer diagnostics (det signs, flip counts, iteration counts) identical, a det
mismatch being allowed only at a tie: where |det| of the diffused matrix lies
within the perturbation the path's own diffusion error can make (1e-12 for the
FP64 path; for the FP32 path first order in the measured diffusion error,
|d det| <= |cof|_F |dA|_F).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1711_01365_amd import inputs

pytestmark = pytest.mark.gpu


def note(*a):
    print("[gpu-parity]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    from paper_1711_01365_amd import mbo
    mbo.load()
    return torch


def to_dev(torch, A, dtype):
    return torch.tensor(np.ascontiguousarray(A), dtype=dtype, device="cuda")


def point_major(A):
    n = A.shape[0]
    return np.moveaxis(A.reshape(n, n, -1), -1, 0)


def cond_mask(At):
    """Points whose polar factor is well conditioned: sigma_{n-1} + sigma_n >= 0.1."""
    s = np.linalg.svd(point_major(At), compute_uv=False)
    if s.shape[1] == 1:
        return np.abs(s[:, 0]) >= 0.05
    return (s[:, -2] + s[:, -1]) >= 0.1


def sigma_gap(At):
    """sigma_{n-1} + sigma_n of every point (the polar factor's absolute condition
    number is 2 / (sigma_{n-1} + sigma_n), Higham, Functions of Matrices, Sec. 8.1)."""
    s = np.linalg.svd(point_major(At), compute_uv=False)
    return s[:, -2] + s[:, -1]


def fp32_step_ok(err, gap, e_heat, ties=None):
    """FP32 one-step error per point against the FP64 oracle.  The FP32 diffusion
    perturbs the projected matrix by e_heat (measured); the first-order bound
    |dQ| <= 2 |dA| / (sigma_{n-1} + sigma_n) then caps what any FP32 projection
    can reach.  Well-conditioned points (gap >= 0.1) must meet 1e-5 outright.
    Points in `ties` (see det_ties) are left out: there the perturbation can
    flip the sign of det, and either polar factor is a correct result."""
    u32 = 2.0 ** -24
    if ties is not None:
        err, gap = err[~ties], gap[~ties]
    bound = np.maximum(1e-5, 4.0 * (e_heat + 8 * u32) / gap)
    return bool(np.all(err <= bound)) and (not np.any(gap >= 0.1) or err[gap >= 0.1].max() <= 1e-5)


def det_ties(Ht, e_heat):
    """Points whose det sign a diffusion error of e_heat (plus the rounding of the
    float input) can change: |det H| <= 2 n (e_heat + 8u) |cof H|_F, the first-order
    change of det being <cof H, dH>.  At such a point the closest orthogonal
    matrix on the other side of det = 0 is as correct as the oracle's."""
    Hp = point_major(Ht)
    n = Hp.shape[1]
    s = np.linalg.svd(Hp, compute_uv=False)
    det = np.abs(np.linalg.det(Hp))
    if n == 1:
        cof = np.ones_like(det)
    else:
        # singular values of cof H: the products of all but one of those of H
        cof = np.sqrt(sum(np.prod(np.delete(s, i, axis=1), axis=1) ** 2 for i in range(n)))
    return det <= 2 * n * (e_heat + 8 * 2.0 ** -24) * cof


def plan(grid, n, tau, prec, batch=1):
    from paper_1711_01365_amd import mbo
    return mbo.Plan(grid, n, tau, precision=prec, batch=batch)


F64, F32, FB = 0, 1, 2


# --------------------------------------------------------------------------
# Projection
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_project_f64(torch_cuda, n):
    torch = torch_cuda
    A = inputs.uniform_field(n, (64, 32), 1000 + n)
    note("project f64 n=%d grid=64x32 seed=%d" % (n, 1000 + n))
    P = plan((64, 32), n, 1e-3, F64)
    Q, ds = P.project(to_dev(torch, A, torch.float64), det_sign=True)
    torch.cuda.synchronize()
    Qo, dso, sg, _ = oracle.project(A)
    Qg = Q.cpu().numpy()
    assert np.abs(Qg - Qo).max() <= 1e-12
    assert np.array_equal(ds.cpu().numpy()[0], dso)


@pytest.mark.parametrize("n", [2, 3, 4])
@pytest.mark.parametrize("prec", [F32, FB])
def test_project_f32(torch_cuda, n, prec):
    torch = torch_cuda
    A = inputs.normal_field(n, (64, 64), 1100 + n)
    note("project f32 n=%d prec=%d seed=%d" % (n, prec, 1100 + n))
    A32 = A.astype(np.float32)
    P = plan((64, 64), n, 1e-3, prec)
    Q = P.project(to_dev(torch, A32, torch.float32)).cpu().numpy()
    Qo = oracle.project(A32.astype(np.float64))[0]
    ok = cond_mask(A32.astype(np.float64))
    err = np.abs(point_major(Q - Qo)).max(axis=(1, 2))
    assert err[ok].max() <= 1e-5
    if prec == FB:
        # points with sigma_min < 1e-3 are re-projected in double: FP64 accuracy
        s = np.linalg.svd(point_major(A32.astype(np.float64)), compute_uv=False)
        small = s[:, -1] < 1e-4
        if small.any():
            assert err[small].max() <= 1e-5


def svd_field(n, grid, seed):
    """U diag(s) V^t per point, U and V Haar in O(n), with the smallest singular
    value log-uniform in [1e-7, 1e-2] (about two thirds of the points below the
    fallback threshold 1e-3); on every other point the second smallest is small too
    (log-uniform between the smallest and 1e-3), so that the polar factor is ill
    conditioned there (condition 2 / (sigma_{n-1} + sigma_n))."""
    rng = np.random.default_rng(seed)
    P = int(np.prod(grid))

    def haar(k):
        Q, R = np.linalg.qr(rng.standard_normal((k, n, n)))
        return Q * np.sign(np.diagonal(R, axis1=1, axis2=2))[:, None, :]
    s = rng.uniform(0.3, 1.5, size=(P, n))
    smin = 10.0 ** rng.uniform(-7, -2, size=P)
    s[:, -1] = smin
    if n >= 3:
        both = np.arange(P) % 2 == 1
        s[both, -2] = smin[both] * 10.0 ** rng.uniform(0, np.log10(1e-3 / smin[both]).clip(0))
    M = haar(P) @ (s[:, :, None] * haar(P))
    return np.ascontiguousarray(np.moveaxis(M.reshape(P, n * n), 0, -1)).reshape((n, n) + tuple(grid))


@pytest.mark.parametrize("n", [2, 3, 4])
def test_project_fallback_targeted(torch_cuda, n):
    """MBO_F32_F64FALLBACK on matrices built with sigma_min spread over [1e-7, 1e-2]:
    every point below the threshold (sigma_min of the float input, computed in
    double) is counted as a fallback, no other, and those points come back at the
    double result rounded to float (<= 1e-6 from the FP64 oracle's projection of
    the same float input); for n >= 3, where the field also holds ill-conditioned
    polar factors, the plain FP32 projection is measurably worse there."""
    torch = torch_cuda
    grid = (64, 64)
    A32 = svd_field(n, grid, 1200 + n).astype(np.float32)
    A64 = A32.astype(np.float64)
    s = np.linalg.svd(point_major(A64), compute_uv=False)
    below = s[:, -1] < 1e-3
    note("fallback targeted n=%d: %d of %d points below 1e-3" % (n, int(below.sum()), below.size))
    Qo = oracle.project(A64)[0]
    P = plan(grid, n, 1e-3, FB)
    Q = P.project(to_dev(torch, A32, torch.float32)).cpu().numpy()
    fb, bad = P.last_project_counts()
    assert bad == 0
    assert fb == int(below.sum())
    err = np.abs(point_major(Q - Qo)).max(axis=(1, 2))
    note("  fallback points: max err %.3g (n=%d)" % (err[below].max(), n))
    assert err[below].max() <= 1e-6
    if n >= 3:
        P32 = plan(grid, n, 1e-3, F32)
        Q32 = P32.project(to_dev(torch, A32, torch.float32)).cpu().numpy()
        e32 = np.abs(point_major(Q32 - Qo)).max(axis=(1, 2))
        note("  plain FP32 on the same points: max err %.3g" % e32[below].max())
        assert e32[below].max() > 1e-5


def test_project_singular_and_special_inputs(torch_cuda):
    torch = torch_cuda
    mats = [np.zeros((3, 3)), np.diag([1.0, 1.0, 0.0]), np.diag([2.0, 0.0, 0.5]),
            np.array([[1.0, 0, 0], [0, -1.0, 0], [0, 0, 0]]), np.eye(3), -np.eye(3),
            np.diag([3.0, 2.0, -1.0])]
    A = np.zeros((3, 3, 8, 8))
    for k, M in enumerate(mats):
        A[:, :, 0, k] = M
    A[:, :, 1:, :] = inputs.uniform_field(3, (7, 8), 5)
    P = plan((8, 8), 3, 1e-3, F64)
    Q = P.project(to_dev(torch, A, torch.float64)).cpu().numpy()
    Qo = oracle.project(A)[0]
    assert np.abs(Q - Qo).max() <= 1e-12
    for k in range(len(mats)):
        q = Q[:, :, 0, k]
        assert np.abs(q.T @ q - np.eye(3)).max() < 1e-14


@pytest.mark.parametrize("prec", [F32, FB])
def test_project_singular_and_special_inputs_fp32(torch_cuda, prec):
    """The same special matrices through the float projections: the zero matrix
    gives I, rank-deficient inputs the oracle's factor (det Q = +1 at a tie), no
    NaN from the Newton route."""
    torch = torch_cuda
    mats = [np.zeros((3, 3)), np.diag([1.0, 1.0, 0.0]), np.diag([2.0, 0.0, 0.5]),
            np.array([[1.0, 0, 0], [0, -1.0, 0], [0, 0, 0]]), np.eye(3), -np.eye(3),
            np.diag([3.0, 2.0, -1.0]), np.outer([1.0, 2.0, 0.5], [0.3, -1.0, 2.0])]
    A = np.zeros((3, 3, 8, 8))
    for k, M in enumerate(mats):
        A[:, :, 0, k] = M
    A[:, :, 1:, :] = inputs.uniform_field(3, (7, 8), 5)
    A32 = A.astype(np.float32)
    note("special inputs f32 prec=%d" % prec)
    P = plan((8, 8), 3, 1e-3, prec)
    Q = P.project(to_dev(torch, A32, torch.float32)).cpu().numpy().astype(np.float64)
    assert np.isfinite(Q).all()
    Qo = oracle.project(A32.astype(np.float64))[0]
    for k in range(len(mats)):
        q = Q[:, :, 0, k]
        assert np.abs(q.T @ q - np.eye(3)).max() < 1e-6, k
        if k < 7:  # rank >= 2 or zero: unique (ties to det +1)
            assert np.abs(q - Qo[:, :, 0, k]).max() < 1e-6, k
    assert np.abs(Q[:, :, 0, 0] - np.eye(3)).max() == 0.0
    ok = cond_mask(A32[:, :, 1:, :].astype(np.float64))
    err = np.abs(point_major(Q[:, :, 1:, :] - Qo[:, :, 1:, :])).max(axis=(1, 2))
    assert err[ok].max() <= 1e-5


@pytest.mark.parametrize("n", [2, 3, 4])
@pytest.mark.parametrize("prec", [F64, F32, FB])
def test_project_scaled_orthogonal_inputs(torch_cuda, prec, n):
    """s R with R orthogonal projects to R for every scale the precision holds
    with room (|det| = s^n and the squares or cofactors representable or not):
    no NaN and no wrong factor from under- or overflowing intermediate
    products."""
    torch = torch_cuda
    Rs = oracle.project(inputs.normal_field(n, (8, 8), 77))[0]
    scales = ([1e-30, 1e-25, 1e-13, 1e-12, 1e-11, 3e-10, 1e-9, 3e-9, 1e-6, 1.0, 1e6, 1e9, 3e9,
               1e10, 1e12, 1e13, 1e19, 1e25]
              if prec != F64 else [1e-150, 1e-100, 1e-60, 1e-12, 1.0, 1e12, 1e60, 1e100, 1e150])
    dt = torch.float64 if prec == F64 else torch.float32
    P = plan((8, 8), n, 1e-3, prec)
    for sc in scales:
        A = (sc * Rs).astype(np.float64 if prec == F64 else np.float32)
        R = oracle.project(A.astype(np.float64))[0]
        Q = P.project(to_dev(torch, A, dt)).cpu().numpy().astype(np.float64)
        assert np.isfinite(Q).all(), sc
        tol = 1e-12 if prec == F64 else 1e-5
        assert np.abs(Q - R).max() <= tol, (sc, np.abs(Q - R).max())


def test_project_nonfinite_is_reported(torch_cuda):
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    A = inputs.uniform_field(2, (8, 8), 9)
    A[0, 1, 3, 3] = np.nan
    P = plan((8, 8), 2, 1e-3, F64)
    with pytest.raises(mbo.MboError) as ei:
        P.project(to_dev(torch, A, torch.float64))
    assert ei.value.status == 5


# --------------------------------------------------------------------------
# Diffusion
# --------------------------------------------------------------------------

GRIDS = [(64, 64), (32, 16), (8, 8), (16, 128), (128, 256), (8, 16, 32), (16, 16, 16), (32, 8, 8)]


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("n", [1, 3])
def test_diffuse_f64(torch_cuda, grid, n):
    torch = torch_cuda
    tau = 2e-3
    A = inputs.uniform_field(n, grid, 7)
    note("diffuse f64 grid=%s n=%d" % (grid, n))
    P = plan(grid, n, tau, F64)
    H = P.diffuse(to_dev(torch, A, torch.float64)).cpu().numpy()
    Ho, _ = oracle.heat(A, tau, len(grid))
    assert np.abs(H - Ho).max() <= 1e-13


@pytest.mark.parametrize("grid", [(64, 64), (512, 512), (16, 32, 64)])
def test_diffuse_f32(torch_cuda, grid):
    torch = torch_cuda
    tau = 2e-4
    A = inputs.uniform_field(3, grid, 8).astype(np.float32)
    note("diffuse f32 grid=%s" % (grid,))
    P = plan(grid, 3, tau, F32)
    H = P.diffuse(to_dev(torch, A, torch.float32)).cpu().numpy()
    Ho, _ = oracle.heat(A.astype(np.float64), tau, len(grid))
    assert np.abs(H - Ho).max() <= 2e-6


def test_diffuse_single_modes(torch_cuda):
    """Closed form: cos(2 pi k.x + phi) decays by exp(-4 pi^2 |k|^2 tau), Nyquist included."""
    torch = torch_cuda
    grid, tau = (32, 16), 3e-3
    Y, X = np.meshgrid(np.arange(32) / 32, np.arange(16) / 16, indexing="ij")
    ks = [(1, 0), (0, 3), (-5, 7), (16, -8), (3, 8)]
    A = np.stack([np.cos(2 * np.pi * (ky * Y + kx * X) + 0.4) for ky, kx in ks[:4]]).reshape(2, 2, 32, 16)
    P = plan(grid, 2, tau, F64)
    H = P.diffuse(to_dev(torch, A, torch.float64)).cpu().numpy()
    for e, (ky, kx) in enumerate(ks[:4]):
        kyw = ((ky + 16) % 32) - 16
        kxw = ((kx + 8) % 16) - 8
        f = np.exp(-4 * np.pi ** 2 * tau * (kyw ** 2 + kxw ** 2))
        assert np.abs(H.reshape(4, 32, 16)[e] - f * A.reshape(4, 32, 16)[e]).max() < 1e-13


def test_diffuse_in_place_and_batched(torch_cuda):
    torch = torch_cuda
    tau = 1e-3
    A = np.stack([inputs.uniform_field(2, (64, 32), s) for s in (1, 2, 3)])
    P = plan((64, 32), 2, tau, F64, batch=3)
    t = to_dev(torch, A, torch.float64)
    P.diffuse(t, t)
    H = t.cpu().numpy()
    for b in range(3):
        assert np.abs(H[b] - oracle.heat(A[b], tau, 2)[0]).max() <= 1e-13


# --------------------------------------------------------------------------
# Energy
# --------------------------------------------------------------------------

@pytest.mark.parametrize("grid,n", [((64, 64), 2), ((32, 128), 3), ((16, 8, 32), 3), ((64, 64), 1),
                                    ((8, 8), 2), ((8, 16), 3), ((8, 8, 8), 2)])
def test_energy_f64(torch_cuda, grid, n):
    torch = torch_cuda
    tau = 1e-3
    A = inputs.uniform_field(n, grid, 17)
    P = plan(grid, n, tau, F64)
    E = P.energy(to_dev(torch, A, torch.float64))
    Eo = oracle.energy(A, tau)
    assert abs(E - Eo) <= 1e-11 * max(1.0, abs(Eo))


def test_energy_f32(torch_cuda):
    torch = torch_cuda
    A = inputs.haar_field(3, (256, 256), 19)
    P = plan((256, 256), 3, 2e-4, F32)
    E = P.energy(to_dev(torch, A.astype(np.float32), torch.float32))
    Eo = oracle.energy(A.astype(np.float32).astype(np.float64), 2e-4)
    assert abs(E - Eo) <= 1e-5 * abs(Eo)


# --------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------

def compare_runs(r, ro, n_iters, atol):
    assert int(r["iters"][0]) == ro["iters"] == n_iters
    assert np.array_equal(r["flips"][0], ro["flips"])
    Eo = ro["energy"]
    assert np.abs(r["energy"][0] - Eo).max() <= 1e-10 * np.abs(Eo).max()


def test_iterate_parity_64x64_n2_f64(torch_cuda):
    """n = 2 on 64 x 64, entries U[-1,1) (seed 0), tau = 1e-3, 20 iterations, FP64."""
    torch = torch_cuda
    w = inputs.PARITY_64
    A0 = w.field()
    note("iterate f64 %s" % w.name)
    P = plan(w.grid, w.n, w.tau, F64)
    t = to_dev(torch, A0, torch.float64)
    r = P.iterate(t, w.iters)
    ro = oracle.iterate(A0, w.tau, w.iters)
    assert np.abs(t.cpu().numpy() - ro["A"]).max() <= 1e-12
    compare_runs(r, ro, w.iters, 1e-12)
    # every iterate, not only the last
    B = A0.copy()
    t = to_dev(torch, A0, torch.float64)
    for s in range(5):
        P.iterate(t, 1)
        B = oracle.iterate(B, w.tau, 1)["A"]
        assert np.abs(t.cpu().numpy() - B).max() <= 1e-12


@pytest.mark.parametrize("n,grid", [(1, (64, 64)), (3, (64, 32)), (4, (32, 32)), (3, (16, 16, 16)), (2, (8, 8))])
def test_iterate_parity_f64(torch_cuda, n, grid):
    torch = torch_cuda
    tau, K = 2e-3, 6
    A0 = inputs.uniform_field(n, grid, 40 + n)
    note("iterate f64 n=%d grid=%s" % (n, grid))
    P = plan(grid, n, tau, F64)
    t = to_dev(torch, A0, torch.float64)
    r = P.iterate(t, K)
    ro = oracle.iterate(A0, tau, K)
    assert np.abs(t.cpu().numpy() - ro["A"]).max() <= 1e-12
    compare_runs(r, ro, K, 1e-12)


LONG_AXES = [(8, 2048), (2048, 8), (16, 1024), (1024, 16), (8, 16, 2048), (2048, 16, 8)]


def long_axes_n(grid):
    """n = 3, except n = 2 for double rows of 2048 points: a double row pass keeps
    every packed plane of its row in LDS, and five planes of 2048 doubles do not
    fit (the plan refuses them, see test_long_double_rows_refused)."""
    return 2 if grid[-1] == 2048 else 3


@pytest.mark.parametrize("grid", LONG_AXES)
def test_diffuse_long_axes_f64(torch_cuda, grid):
    """Axes of 1024 and 2048 points, the longest a plan accepts: the row
    transforms that exchange through workgroup barriers (lines longer than one
    wave holds) and the strided passes at their largest tile."""
    torch = torch_cuda
    tau = 2e-4
    n = long_axes_n(grid)
    A = inputs.uniform_field(n, grid, 17)
    note("diffuse f64 long axes grid=%s n=%d" % (grid, n))
    P = plan(grid, n, tau, F64)
    H = P.diffuse(to_dev(torch, A, torch.float64)).cpu().numpy()
    Ho, _ = oracle.heat(A, tau, len(grid))
    assert np.abs(H - Ho).max() <= 1e-13


@pytest.mark.parametrize("grid", LONG_AXES)
def test_iterate_long_axes_f64(torch_cuda, grid):
    """Three MBO steps with rows of up to 2048 points (the projection and the
    fallback queue sized by the row), against the oracle: entries to 1e-12,
    flips and energies as in the other FP64 runs."""
    torch = torch_cuda
    tau, K = 2e-4, 3
    n = long_axes_n(grid)
    A0 = inputs.uniform_field(n, grid, 18)
    note("iterate f64 long axes grid=%s n=%d" % (grid, n))
    P = plan(grid, n, tau, F64)
    t = to_dev(torch, A0, torch.float64)
    r = P.iterate(t, K)
    ro = oracle.iterate(A0, tau, K)
    assert np.abs(t.cpu().numpy() - ro["A"]).max() <= 1e-12
    compare_runs(r, ro, K, 1e-12)


def test_long_double_rows_refused(torch_cuda):
    """The largest shapes at the LDS limit: double rows of 2048 points with n >= 3
    are refused (MBO_ERR_UNSUPPORTED); float rows of 2048 with
    n = 4 and double rows of 1024 with n = 4 are accepted."""
    from paper_1711_01365_amd import mbo
    for n in (3, 4):
        with pytest.raises(mbo.MboError) as ei:
            plan((8, 2048), n, 1e-3, F64)
        assert ei.value.status == 2
    plan((8, 2048), 4, 1e-3, FB).close()
    plan((8, 1024), 4, 1e-3, F64).close()
    plan((2048, 8), 4, 1e-3, F64).close()


@pytest.mark.parametrize("grid", [(8, 2048), (2048, 8), (8, 16, 2048)])
def test_iterate_long_axes_fp32_fallback(torch_cuda, grid):
    """One FP32 + FP64-fallback step with rows of 2048 points (a queue of 2048
    entries per workgroup) against the FP64 oracle, to the FP32 bar."""
    torch = torch_cuda
    tau = 2e-4
    A0 = inputs.uniform_field(3, grid, 19).astype(np.float32)
    A64 = A0.astype(np.float64)
    note("one step f32+fb long axes grid=%s" % (grid,))
    P = plan(grid, 3, tau, FB)
    Ht, _ = oracle.heat(A64, tau, len(grid))
    Hg = P.diffuse(to_dev(torch, A0, torch.float32)).cpu().numpy()
    e_heat = float(np.abs(Hg - Ht).max())
    t = to_dev(torch, A0, torch.float32)
    r = P.iterate(t, 1)
    ro = oracle.iterate(A64, tau, 1)
    gap = sigma_gap(Ht)
    err = np.abs(point_major(t.cpu().numpy() - ro["A"])).max(axis=(1, 2))
    note("long axes f32+fb: diffusion err %.3g, step err max %.3g, fallbacks %d"
         % (e_heat, err.max(), r["fallbacks"][0][0]))
    assert e_heat <= 2e-6
    assert fp32_step_ok(err, gap, e_heat)


BANDED_LONG_F64 = [((64, 1024), 3), ((64, 1024), 4), ((128, 2048), 2), ((64, 2048), 1), ((64, 512), 3)]


def assert_banded(P, L):
    """The plan runs the band-limited passes with fewer stored modes than L."""
    from paper_1711_01365_amd import mbo
    path, c, W = P.path()
    note("path %d, half-width %d, stored modes %d of %d" % (path, c, W, L))
    assert path == mbo.PATH_BANDED and 2 * c + 1 <= W < L


@pytest.mark.parametrize("grid,n", BANDED_LONG_F64)
def test_iterate_banded_rows_f64(torch_cuda, grid, n):
    """Three FP64 steps through the band-limited row pass (rows of 512 points, one
    wave per line; rows of 1024 and 2048 points, lines exchanged through
    workgroup barriers, in rounds of lines, several points per thread) against
    the oracle: entries to 1e-12 (the dropped row modes weigh at most 1e-20 of
    max|A|), flips identical, energies to 1e-10 of the largest."""
    torch = torch_cuda
    tau, K = 2e-4, 3
    A0 = inputs.uniform_field(n, grid, 23)
    note("banded f64 grid=%s n=%d" % (grid, n))
    P = plan(grid, n, tau, F64)
    assert_banded(P, grid[-1])
    t = to_dev(torch, A0, torch.float64)
    r = P.iterate(t, K)
    ro = oracle.iterate(A0, tau, K)
    err = float(np.abs(t.cpu().numpy() - ro["A"]).max())
    note("banded f64 max err %.3g" % err)
    assert err <= 1e-12
    compare_runs(r, ro, K, 1e-12)


@pytest.mark.parametrize("grid,n", [((64, 1024), 3), ((64, 2048), 3), ((64, 2048), 4), ((128, 1024), 2),
                                    ((64, 2048), 2)])
def test_iterate_banded_rows_fp32_fallback(torch_cuda, grid, n):
    """One FP32 + FP64-fallback step through the band-limited row pass with rows
    of 1024 and 2048 points (n = 3: the helper wave's queue of up to 2048 points
    per workgroup) against the FP64 oracle, to the FP32 bar; the fallback count
    against the points whose float sigma_min is below the threshold is checked
    by the targeted test."""
    torch = torch_cuda
    tau = 2e-4
    A0 = inputs.uniform_field(n, grid, 29).astype(np.float32)
    A64 = A0.astype(np.float64)
    note("banded f32+fb grid=%s n=%d" % (grid, n))
    P = plan(grid, n, tau, FB)
    assert_banded(P, grid[-1])
    Ht, _ = oracle.heat(A64, tau, len(grid))
    Hg = P.diffuse(to_dev(torch, A0, torch.float32)).cpu().numpy()
    e_heat = float(np.abs(Hg - Ht).max())
    t = to_dev(torch, A0, torch.float32)
    r = P.iterate(t, 1)
    ro = oracle.iterate(A64, tau, 1)
    gap = sigma_gap(Ht)
    err = np.abs(point_major(t.cpu().numpy() - ro["A"])).max(axis=(1, 2))
    note("banded f32+fb: diffusion err %.3g, step err max %.3g, fallbacks %d"
         % (e_heat, err.max(), r["fallbacks"][0][0]))
    assert e_heat <= 2e-6
    assert fp32_step_ok(err, gap, e_heat)
    assert abs(r["energy"][0][0] - ro["energy"][0]) <= 1e-5 * abs(ro["energy"][0])


@pytest.mark.parametrize("grid,n", [((64, 2048), 3), ((64, 1024), 4)])
def test_banded_rows_match_the_full_path(torch_cuda, grid, n):
    """Five FP32 + fallback steps: the band-limited passes against every row mode
    kept (PATH_FULL), both on the GPU: the two differ by the dropped modes (at
    most 1e-12 max|A| per step) and float rounding, so entries agree to the FP32
    bar where the projection is well conditioned, and det signs agree except at
    ties."""
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    tau, K = 2e-4, 5
    A0 = inputs.uniform_field(n, grid, 31).astype(np.float32)
    out = []
    for path in (mbo.PATH_BANDED, mbo.PATH_FULL):
        P = plan(grid, n, tau, FB)
        P.set_path(path)
        assert P.path()[0] == path
        t = to_dev(torch, A0, torch.float32)
        P.iterate(t, K - 1)
        H = P.diffuse(t).cpu().numpy()
        P.iterate(t, 1)
        out.append((t.cpu().numpy(), H))
        P.close()
    (Ab, Hb), (Af, Hf) = out
    gap = sigma_gap(Hf.astype(np.float64))
    err = np.abs(point_major(Ab - Af)).max(axis=(1, 2))
    note("banded vs full: max err %.3g, well-conditioned max %.3g"
         % (err.max(), err[gap >= 0.1].max() if np.any(gap >= 0.1) else 0.0))
    assert err[gap >= 0.1].max() <= 1e-5


def small_sigma_field(n, grid, seed):
    """U diag(1, 0.7, s(x, y)) V^t with U, V fixed Haar-random orthogonal matrices
    and s = 10^(-5 + 3 (1 + sin(2 pi x) cos(2 pi y)) / 2), smooth on the torus:
    diffusion acts on s alone (H A = U diag(1, 0.7, H s) V^t), so the diffused
    field keeps sigma_min = H s in [1e-5, 1e-2] and its polar factor is U V^t at
    every point (condition 2 / (0.7 + H s))."""
    rng = np.random.default_rng(seed)

    def haar():
        Q, R = np.linalg.qr(rng.standard_normal((n, n)))
        return Q * np.sign(np.diag(R))[None, :]
    U, V = haar(), haar()
    x = np.arange(grid[1]) / grid[1]
    y = np.arange(grid[0]) / grid[0]
    sm = 10.0 ** (-5.0 + 1.5 * (1.0 + np.sin(2 * np.pi * x)[None, :] * np.cos(2 * np.pi * y)[:, None]))
    sv = np.ones((n,) + tuple(grid))
    sv[1] = 0.7
    sv[n - 1] = sm
    return np.einsum("ik,k...,jk->ij...", U, sv, V), U @ V.T


@pytest.mark.parametrize("grid,tau", [((64, 512), 2e-4), ((64, 64), 2e-2)])
def test_row_pass_queue_of_small_sigma_points(torch_cuda, grid, tau):
    """One FP32 + FP64-fallback step of a field whose diffused points mostly fall
    below the Newton precheck (sigma_min in [1e-5, 1e-2]): more points go to the
    row pass's queue than one wave holds (its wave loops over them while the other
    waves take its Newton points), and with the kept half-width below L/8 the line
    transforms are pruned.  The exact step is U V^t at every point: the result
    matches it and the FP64 oracle's step to 1e-5, det signs are those of U V^t,
    and the fallback count lies between the oracle's counts of diffused points
    below 0.95e-3 and 1.05e-3."""
    torch = torch_cuda
    n = 3
    A0, Q = small_sigma_field(n, grid, 1400 + grid[1])
    A32 = A0.astype(np.float32)
    A64 = A32.astype(np.float64)
    P = plan(grid, n, tau, FB)
    assert_banded(P, grid[-1])
    _, c, _W = P.path()
    assert c < grid[-1] // 8  # pruned transforms
    Ht, _ = oracle.heat(A64, tau, 2)
    smin = np.linalg.svd(point_major(Ht), compute_uv=False)[:, -1]
    lo, hi = int((smin < 0.95e-3).sum()), int((smin < 1.05e-3).sum())
    t = to_dev(torch, A32, torch.float32)
    r = P.iterate(t, 1)
    ro = oracle.iterate(A64, tau, 1)
    A1 = t.cpu().numpy().astype(np.float64)
    e_orc = float(np.abs(A1 - ro["A"]).max())
    e_uv = float(np.abs(point_major(A1) - Q[None]).max())
    fb = int(r["fallbacks"][0][0])
    note("small-sigma queue grid=%s tau=%g: %d of %d points below 1e-3, fallbacks %d, "
         "err vs oracle %.3g, vs U V^t %.3g" % (grid, tau, lo, smin.size, fb, e_orc, e_uv))
    assert lo > smin.size // 4
    assert lo <= fb <= hi
    assert e_orc <= 1e-5 and e_uv <= 1e-5
    assert int(r["flips"][0][0]) == int(ro["flips"][0])
    assert np.array_equal(np.sign(np.linalg.det(point_major(A1))),
                          np.full(smin.size, np.sign(np.linalg.det(Q))))


@pytest.mark.parametrize("prec", [F64, F32, FB])
def test_iterate_zero_and_rank_one_fields(torch_cuda, prec):
    """Degenerate fields: the zero field diffuses to itself and every point
    projects to I (A = 0 gives Q = I), after which I is a fixed point; a field
    of one rank-1 matrix everywhere (diffusion keeps a constant field) projects
    to an orthogonal matrix with det +1 at the tie and then stays there.  No
    NaN, no non-finite report, no flips."""
    torch = torch_cuda
    grid, tau = (16, 32), 1e-3
    dt = torch.float64 if prec == F64 else torch.float32
    M = np.outer([1.0, 2.0, 0.5], [0.3, -1.0, 2.0])
    for name, A0 in (("zero", np.zeros((3, 3) + grid)),
                     ("rank one", np.broadcast_to(M[:, :, None, None], (3, 3) + grid).copy())):
        note("degenerate field %s prec=%d" % (name, prec))
        P = plan(grid, 3, tau, prec)
        t = to_dev(torch, A0, dt)
        r = P.iterate(t, 3)
        A = t.cpu().numpy().astype(np.float64)
        assert np.isfinite(A).all(), name
        Q0 = oracle.project(A0[:, :, :1, :1].copy())[0][:, :, 0, 0]
        assert abs(np.linalg.det(Q0) - 1.0) < 1e-12
        tol = 1e-12 if prec == F64 else 1e-6
        assert np.abs(A - Q0[:, :, None, None]).max() <= tol, name
        assert int(np.sum(r["flips"][0])) == 0, name
        P.close()


@pytest.mark.parametrize("path", [0, 1, 2])
@pytest.mark.parametrize("prec", [F64, FB])
def test_iterate_nonfinite_is_reported(torch_cuda, path, prec):
    """A NaN in the field reaches the projections of the first iteration (the
    diffusion spreads it); mbo_iterate returns MBO_ERR_NONFINITE after the run,
    on every kernel path, and a finite field on the same plan runs clean after it."""
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    grid, n = (64, 64), 3
    A = inputs.uniform_field(n, grid, 1300)
    A[1, 2, 5, 7] = np.nan
    dt = torch.float64 if prec == F64 else torch.float32
    P = plan(grid, n, 1e-3, prec)
    P.set_path(path)
    with pytest.raises(mbo.MboError) as e:
        P.iterate(to_dev(torch, A, dt), 3)
    assert e.value.status == 5
    B = inputs.uniform_field(n, grid, 1301)
    P.iterate(to_dev(torch, B, dt), 3)


def test_plan_allocation_failure_is_reported(torch_cuda):
    """A plan whose workspace exceeds the device memory (2048^2, n = 4, 100000
    fields: ~5e16 bytes of spectra) is refused with MBO_ERR_ALLOC, no plan is
    returned, and the device is usable afterwards."""
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    with pytest.raises(mbo.MboError) as e:
        mbo.Plan((2048, 2048), 4, 1e-3, precision=F32, batch=100000)
    assert e.value.status == 3
    note("allocation failure: %s" % e.value)
    P = plan((32, 32), 2, 1e-3, F64)
    A = inputs.uniform_field(2, (32, 32), 1302)
    t = to_dev(torch, A, torch.float64)
    P.iterate(t, 2)
    assert np.abs(t.cpu().numpy() - oracle.iterate(A, 1e-3, 2)["A"]).max() <= 1e-12


def test_iterate_tolerance_stop_matches_oracle(torch_cuda):
    torch = torch_cuda
    tau = 2e-3
    u0 = np.where(inputs.uniform_field(1, (32, 32), 51) >= 0, 1.0, -1.0)
    P = plan((32, 32), 1, tau, F64)
    t = to_dev(torch, u0, torch.float64)
    r = P.iterate(t, 200, tol=1e-300)
    ro = oracle.iterate(u0, tau, 200, tol=1e-300)
    assert int(r["iters"][0]) == ro["iters"] < 200
    assert np.array_equal(t.cpu().numpy(), ro["A"])
    k = ro["iters"]
    assert np.array_equal(r["flips"][0][:k], ro["flips"])
    assert np.array_equal(r["delta"][0][:k], ro["delta"])
    assert np.abs(r["energy"][0][:k + 1] - ro["energy"]).max() <= 1e-10 * np.abs(ro["energy"]).max()


def test_iterate_graph_replay_is_stable(torch_cuda):
    """The captured graph is replayed: repeated calls on the same buffer continue
    the iteration exactly like one longer call, with eager syncs in between."""
    torch = torch_cuda
    A0 = inputs.uniform_field(3, (64, 64), 77)
    P = plan((64, 64), 3, 1e-3, F64)
    t = to_dev(torch, A0, torch.float64)
    for _ in range(3):
        P.iterate(t, 2)
        torch.cuda.synchronize()
        _ = (t * 2).sum().item()
    ro = oracle.iterate(A0, 1e-3, 6)
    assert np.abs(t.cpu().numpy() - ro["A"]).max() <= 1e-12


def test_iterate_graph_follows_changing_buffers(torch_cuda):
    """The graph is keyed by the buffer it was captured with: alternating calls
    on two buffers (and a changed iteration count) each continue their own
    iteration, as the oracle does, with no result written into the other
    buffer."""
    torch = torch_cuda
    A0 = inputs.uniform_field(3, (32, 32), 78)
    B0 = inputs.uniform_field(3, (32, 32), 79)
    P = plan((32, 32), 3, 1e-3, F64)
    a = to_dev(torch, A0, torch.float64)
    b = to_dev(torch, B0, torch.float64)
    P.iterate(a, 2)
    P.iterate(b, 2)
    P.iterate(a, 3)
    P.iterate(b, 1)
    P.iterate(a, 1)
    ra = oracle.iterate(A0, 1e-3, 6)
    rb = oracle.iterate(B0, 1e-3, 3)
    assert np.abs(a.cpu().numpy() - ra["A"]).max() <= 1e-12
    assert np.abs(b.cpu().numpy() - rb["A"]).max() <= 1e-12
    P.close()


def test_plan_on_a_side_stream(torch_cuda):
    """A plan created on a side stream (default priority) enqueues everything
    there: the iteration through its captured graph, diffusion and projection
    give the same bits as a plan on the default stream; set_stream moves it
    back."""
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    grid, n, tau, K = (64, 32), 3, 2e-3, 4
    A0 = inputs.uniform_field(n, grid, 123)
    P0 = plan(grid, n, tau, F64)
    t0 = to_dev(torch, A0, torch.float64)
    r0 = P0.iterate(t0, K)
    H0 = P0.diffuse(to_dev(torch, A0, torch.float64)).cpu().numpy()
    Q0 = P0.project(t0).cpu().numpy()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        t1 = to_dev(torch, A0, torch.float64)
        P1 = mbo.Plan(grid, n, tau, precision=F64, stream=s)
        r1 = P1.iterate(t1, K)
        H1 = P1.diffuse(to_dev(torch, A0, torch.float64))
        Q1 = P1.project(t1)
    s.synchronize()
    assert np.array_equal(t1.cpu().numpy(), t0.cpu().numpy())
    assert np.array_equal(H1.cpu().numpy(), H0)
    assert np.array_equal(Q1.cpu().numpy(), Q0)
    assert np.array_equal(r1["flips"][0], r0["flips"][0])
    assert np.array_equal(r1["energy"][0], r0["energy"][0])
    P1.set_stream(None)
    t2 = to_dev(torch, A0, torch.float64)
    P1.iterate(t2, K)
    assert np.array_equal(t2.cpu().numpy(), t0.cpu().numpy())
    P0.close()
    P1.close()


def test_two_plans_on_two_streams_concurrently(torch_cuda):
    """Two plans (different shapes and precisions) iterating at the same time
    on two side streams share no state: each ends as it does when run alone."""
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    cfg = [((64, 32), 3, 2e-3, F64, 124), ((32, 64), 2, 1e-3, FB, 125)]
    alone = []
    for grid, n, tau, prec, seed in cfg:
        P = plan(grid, n, tau, prec)
        t = to_dev(torch, inputs.uniform_field(n, grid, seed), torch.float64 if prec == F64 else torch.float32)
        P.iterate(t, 6)
        alone.append(t.cpu().numpy())
        P.close()
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    plans, fields = [], []
    for (grid, n, tau, prec, seed), st in zip(cfg, streams):
        with torch.cuda.stream(st):
            plans.append(mbo.Plan(grid, n, tau, precision=prec, stream=st))
            fields.append(to_dev(torch, inputs.uniform_field(n, grid, seed),
                                 torch.float64 if prec == F64 else torch.float32))
    for st in streams:
        st.synchronize()
    for rep in range(3):  # interleaved launches on both streams
        for P, t, st in zip(plans, fields, streams):
            with torch.cuda.stream(st):
                P.iterate(t, 2, logs=False)
    torch.cuda.synchronize()
    for t, ref in zip(fields, alone):
        assert np.array_equal(t.cpu().numpy(), ref)
    for P in plans:
        P.close()


def test_set_tau_matches_a_fresh_plan(torch_cuda):
    """Changing tau on a plan whose iteration graph is already captured gives the
    bits of a plan made with the new tau (tables rebuilt, graph re-captured,
    energies with the new tau), and agrees with the oracle."""
    torch = torch_cuda
    grid, n, K = (32, 64), 3, 3
    A0 = inputs.uniform_field(n, grid, 126)
    P = plan(grid, n, 1e-3, F64)
    t = to_dev(torch, A0, torch.float64)
    P.iterate(t, K)
    P.set_tau(4e-3)
    t = to_dev(torch, A0, torch.float64)
    r = P.iterate(t, K)
    Q = plan(grid, n, 4e-3, F64)
    u = to_dev(torch, A0, torch.float64)
    rq = Q.iterate(u, K)
    assert np.array_equal(t.cpu().numpy(), u.cpu().numpy())
    assert np.array_equal(r["energy"][0], rq["energy"][0])
    ro = oracle.iterate(A0, 4e-3, K)
    assert np.abs(t.cpu().numpy() - ro["A"]).max() <= 1e-12
    compare_runs(r, ro, K, 1e-12)
    P.close()
    Q.close()


def test_iterate_batched_fields_match_single(torch_cuda):
    torch = torch_cuda
    A = np.stack([inputs.uniform_field(2, (32, 64), s) for s in (4, 5)])
    P = plan((32, 64), 2, 1e-3, F64, batch=2)
    t = to_dev(torch, A, torch.float64)
    r = P.iterate(t, 4)
    for b in range(2):
        ro = oracle.iterate(A[b], 1e-3, 4)
        assert np.abs(t.cpu().numpy()[b] - ro["A"]).max() <= 1e-12
        assert np.array_equal(r["flips"][b], ro["flips"])


@pytest.mark.parametrize("prec", [F32, FB])
def test_iterate_one_step_f32_512(torch_cuda, prec):
    """n = 3, 512 x 512, Haar O(3) (seed 1), tau = 2e-4: one FP32 step from the same
    state against the FP64 oracle, per point within the FP32 perturbation bound
    (and 1e-5 where the projection is well conditioned)."""
    torch = torch_cuda
    w = inputs.HAAR_512
    A0 = w.field().astype(np.float32)
    note("one step f32 prec=%d %s" % (prec, w.name))
    P = plan(w.grid, w.n, w.tau, prec)
    A64 = A0.astype(np.float64)
    Ht, _ = oracle.heat(A64, w.tau, 2)
    Hg = P.diffuse(to_dev(torch, A0, torch.float32)).cpu().numpy()
    e_heat = float(np.abs(Hg - Ht).max())
    t = to_dev(torch, A0, torch.float32)
    r = P.iterate(t, 1)
    ro = oracle.iterate(A64, w.tau, 1)
    gap = sigma_gap(Ht)
    err = np.abs(point_major(t.cpu().numpy() - ro["A"])).max(axis=(1, 2))
    note("one step f32: diffusion err %.3g, step err max %.3g, median %.3g, min gap %.3g, "
         "fallbacks %d" % (e_heat, err.max(), np.median(err), gap.min(), r["fallbacks"][0][0]))
    assert e_heat <= 2e-6
    assert fp32_step_ok(err, gap, e_heat)
    assert abs(r["energy"][0][0] - ro["energy"][0]) <= 1e-5 * abs(ro["energy"][0])
    if prec == FB:
        assert r["fallbacks"][0][0] > 0


def test_iterate_full_size_512_f64_two_steps(torch_cuda):
    torch = torch_cuda
    w = inputs.HAAR_512
    A0 = w.field()
    note("two steps f64 %s" % w.name)
    P = plan(w.grid, w.n, w.tau, F64)
    t = to_dev(torch, A0, torch.float64)
    r = P.iterate(t, 2)
    ro = oracle.iterate(A0, w.tau, 2)
    assert np.abs(t.cpu().numpy() - ro["A"]).max() <= 1e-12
    assert np.array_equal(r["flips"][0], ro["flips"])


def test_bench_configuration_properties(torch_cuda):
    """The measured configuration (n = 3, 512^2, 200 FP32+fallback iterations) at
    full size: every point orthogonal and the energy non-increasing from s = 1
    (within FP32 rounding) along the library's own run; and the 200th step at
    full size from the oracle's own iterate 199 (rounded to float, the input of
    both): the step within the FP32 bound of the oracle's and its logged energy
    equal to the oracle's."""
    torch = torch_cuda
    w = inputs.HAAR_512
    A0 = w.field().astype(np.float32)
    note("bench configuration %s, 200 iterations" % w.name)
    P = plan(w.grid, w.n, w.tau, FB)
    t = to_dev(torch, A0, torch.float32)
    r = P.iterate(t, w.iters)
    M = point_major(t.cpu().numpy()).astype(np.float64)
    assert np.abs(M.transpose(0, 2, 1) @ M - np.eye(3)).max() < 1e-5
    E = r["energy"][0]
    assert np.all(np.diff(E[1:]) <= 1e-5 * E[1])
    note("oracle trajectory to iterate %d" % (w.iters - 1))
    A199 = oracle.iterate(w.field(), w.tau, w.iters - 1)["A"].astype(np.float32)
    A64 = A199.astype(np.float64)
    ro = oracle.iterate(A64, w.tau, 1)
    Ht, _ = oracle.heat(A64, w.tau, 2)
    Hg = P.diffuse(to_dev(torch, A199, torch.float32)).cpu().numpy()
    e_heat = float(np.abs(Hg - Ht).max())
    t = to_dev(torch, A199, torch.float32)
    r2 = P.iterate(t, 1)
    gap = sigma_gap(Ht)
    err = np.abs(point_major(t.cpu().numpy() - ro["A"])).max(axis=(1, 2))
    note("bench config step 200: diffusion err %.3g, step err max %.3g, well-cond (%d pts) %.3g"
         % (e_heat, err.max(), int((gap >= 0.1).sum()), err[gap >= 0.1].max() if (gap >= 0.1).any() else 0))
    assert fp32_step_ok(err, gap, e_heat)
    # det signs point by point: a point whose sign differs from the oracle's must
    # be a tie, |det H A_199| within what the FP32 diffusion error can move it
    # (first order: |d det| <= |cof|_F |dA|_F <= |cof|_F * 3 e_heat, doubled)
    sg = np.linalg.det(point_major(t.cpu().numpy()).astype(np.float64)) >= 0
    so = np.linalg.det(point_major(ro["A"])) >= 0
    Hp = point_major(Ht)
    dets = np.linalg.det(Hp)
    cof = np.linalg.norm(np.stack([np.cross(Hp[:, 1], Hp[:, 2]), np.cross(Hp[:, 2], Hp[:, 0]),
                                   np.cross(Hp[:, 0], Hp[:, 1])], axis=1), axis=(1, 2))
    tie_bound = 2.0 * 3.0 * (e_heat + 8 * 2.0 ** -24) * cof
    mism = np.nonzero(sg != so)[0]
    note("bench config step 200: flips %d (oracle %d), det-sign mismatches %d at %s, |det H A| there %s, "
         "tie bounds %s" % (int(r2["flips"][0][0]), int(ro["flips"][0]), mism.size, list(mism[:8]),
                            list(np.abs(dets[mism][:8])), list(tie_bound[mism][:8])))
    assert np.all(np.abs(dets[mism]) <= tie_bound[mism])
    # every flip the two runs count differently is one of those ties
    assert abs(int(r2["flips"][0][0]) - int(ro["flips"][0])) <= mism.size
    assert abs(r2["energy"][0][1] - ro["energy"][1]) <= 1e-5 * abs(ro["energy"][1])


def test_iterate_full_size_128cube_f64_two_steps(torch_cuda):
    """n = 3 on the 128^3 torus, iid N(0,1) entries (seed 2), tau = 5e-4: two FP64
    steps against the oracle (<= 1e-12) with identical flip counts."""
    torch = torch_cuda
    w = inputs.NORMAL_128_3D
    A0 = w.field()
    note("two steps f64 %s" % w.name)
    P = plan(w.grid, w.n, w.tau, F64)
    t = to_dev(torch, A0, torch.float64)
    r = P.iterate(t, 2)
    ro = oracle.iterate(A0, w.tau, 2)
    err = np.abs(t.cpu().numpy() - ro["A"]).max()
    note("  max err %.3e, flips %s vs %s" % (err, list(r["flips"][0]), list(ro["flips"])))
    assert err <= 1e-12
    assert np.array_equal(r["flips"][0], ro["flips"])
    assert abs(r["energy"][0][2] - ro["energy"][2]) <= 1e-12 * abs(ro["energy"][2])


def test_3d_configuration_properties(torch_cuda):
    """The 3-D configuration at full size (n = 3, 128^3, 100 FP32+fallback
    iterations): one FP32 step from A_0 within the FP32 bound of the oracle step;
    along the library's own run every point of the result orthogonal and the
    energy non-increasing from s = 1 within FP32 rounding; and a later step from
    the oracle's own iterate 9 (rounded to float, the input of both) within the
    FP32 bound, with the oracle's energy."""
    torch = torch_cuda
    w = inputs.NORMAL_128_3D
    A0 = w.field().astype(np.float32)
    note("3-D configuration %s" % w.name)
    P = plan(w.grid, w.n, w.tau, FB)

    def step_from(Ain, label):
        A64 = Ain.astype(np.float64)
        Ht, _ = oracle.heat(A64.reshape((9,) + w.grid), w.tau, 3)
        Ht = Ht.reshape(A64.shape)
        Hg = P.diffuse(to_dev(torch, Ain, torch.float32)).cpu().numpy()
        e_heat = float(np.abs(Hg - Ht).max())
        t = to_dev(torch, Ain, torch.float32)
        r1 = P.iterate(t, 1)
        ro = oracle.iterate(A64, w.tau, 1)
        gap = sigma_gap(Ht)
        err = np.abs(point_major(t.cpu().numpy() - ro["A"])).max(axis=(1, 2))
        note("  %s: diffusion err %.3g, step err max %.3g, fallbacks %d"
             % (label, e_heat, err.max(), r1["fallbacks"][0][0]))
        assert e_heat <= 2e-6
        assert fp32_step_ok(err, gap, e_heat)
        return r1, ro

    step_from(A0, "step 1")
    # the library's own run
    t = to_dev(torch, A0, torch.float32)
    r = P.iterate(t, w.iters)
    M = point_major(t.cpu().numpy()).astype(np.float64)
    assert np.abs(M.transpose(0, 2, 1) @ M - np.eye(3)).max() < 1e-5
    E = r["energy"][0][1:]
    assert np.all(np.diff(E) <= 1e-5 * E[0])
    # a later step from the oracle's own trajectory
    A9 = oracle.iterate(w.field(), w.tau, 9)["A"].astype(np.float32)
    r1, ro = step_from(A9, "step 10")
    assert abs(r1["energy"][0][1] - ro["energy"][1]) <= 1e-5 * abs(ro["energy"][1])


BANDED_3D = [((64, 64, 128), 3, FB), ((128, 128, 64), 3, FB), ((64, 128, 32), 2, F32), ((128, 64, 16), 4, FB),
             ((64, 64, 512), 1, F32)]


@pytest.mark.parametrize("grid,n,prec", BANDED_3D)
def test_iterate_3d_plane_pass_one_step(torch_cuda, grid, n, prec):
    """The 3-D band-limited passes of float plans (the x-row pass storing the
    kept x modes plane by plane, one plane pass per packed plane and stored x
    mode doing the y and z transforms, the heat step and the Lyapunov partial in
    LDS): one step against the FP64 oracle to the FP32 bar, and the logged energy
    against the oracle's; twice, from A_0 (uniform entries: after diffusion most
    points are ill conditioned) and from the GPU's own A_1 (a smooth field of
    orthogonal matrices: most points well conditioned)."""
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    tau = 5e-4
    P = plan(grid, n, tau, prec)
    path, c, W = P.path()
    note("3-D plane pass grid=%s n=%d: path %d, half-width %d, stored %d" % (grid, n, path, c, W))
    assert path in (mbo.PATH_BANDED, mbo.PATH_FULL)
    Ain = inputs.uniform_field(n, grid, 37).astype(np.float32)
    for k in range(2):
        A64 = Ain.astype(np.float64)
        Ht, _ = oracle.heat(A64.reshape((n * n,) + grid), tau, 3)
        Ht = Ht.reshape(A64.shape)
        Hg = P.diffuse(to_dev(torch, Ain, torch.float32)).cpu().numpy()
        e_heat = float(np.abs(Hg - Ht).max())
        t = to_dev(torch, Ain, torch.float32)
        r = P.iterate(t, 1)
        ro = oracle.iterate(A64, tau, 1)
        gap = sigma_gap(Ht) if n > 1 else np.abs(Ht.reshape(-1)) * 2
        ties = det_ties(Ht, e_heat)
        Q = t.cpu().numpy()
        err = np.abs(point_major(Q - ro["A"])).max(axis=(1, 2))
        Qp = point_major(Q.astype(np.float64))
        orth = np.abs(np.einsum("pki,pkj->pij", Qp, Qp) - np.eye(n)).max()
        note("  input %d: diffusion err %.3g, step err max %.3g, %d of %d points well conditioned, %d det "
             "ties, fallbacks %d, |Q^t Q - I| %.3g, E0 %.6g (oracle %.6g)"
             % (k, e_heat, err.max(), int((gap >= 0.1).sum()), gap.size, int(ties.sum()),
                r["fallbacks"][0][0], orth, r["energy"][0][0], ro["energy"][0]))
        assert e_heat <= 2e-6
        assert fp32_step_ok(err, gap, e_heat, ties)
        assert orth <= 1e-5
        assert abs(r["energy"][0][0] - ro["energy"][0]) <= 1e-5 * abs(ro["energy"][0])
        Ain = Q


@pytest.mark.parametrize("grid,n", [((128, 128, 128), 3), ((64, 128, 64), 4)])
def test_iterate_3d_plane_pass_matches_general_kernels(torch_cuda, grid, n):
    """Five FP32 + fallback steps through the 3-D band-limited passes against the
    general kernels (row pass and three strided passes, every mode kept), both on
    the GPU.  Each step starts both paths from the same iterate (the general
    path's trajectory): two correct FP32 projections may differ at a point whose
    polar factor is ill conditioned, and the next diffusion spreads that
    difference to its neighbours, so trajectories run apart are no measure of a
    step.  Entries agree to the FP32 bar where the projection is well
    conditioned and det is no tie (det_ties) at every step; the energies logged
    by two independent runs of the five steps agree to FP32 rounding."""
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    tau, K = 5e-4, 5
    A0 = inputs.normal_field(n, grid, 41).astype(np.float32)
    Pb, Pg = plan(grid, n, tau, FB), plan(grid, n, tau, FB)
    Pb.set_path(mbo.PATH_BANDED)
    Pg.set_path(mbo.PATH_GENERIC)
    t = to_dev(torch, A0, torch.float32)
    worst = 0.0
    for s in range(1, K + 1):
        Hg = Pg.diffuse(t).cpu().numpy().astype(np.float64)
        gap = sigma_gap(Hg)
        # both diffusions lie within 2e-6 of the exact one (the one-step test)
        ties = det_ties(Hg, 4e-6)
        nb, ng = Pb.step(t), Pg.step(t)
        err = np.abs(point_major((nb - ng).cpu().numpy())).max(axis=(1, 2))
        wc = (gap >= 0.1) & ~ties
        e_wc = float(err[wc].max()) if wc.any() else 0.0
        note("3-D plane pass vs general kernels grid=%s n=%d step %d: max err %.3g, well conditioned %.3g "
             "(%d of %d points, %d det ties)" % (grid, n, s, err.max(), e_wc, int(wc.sum()), wc.size,
                                                int(ties.sum())))
        assert e_wc <= 1e-5, s
        worst = max(worst, e_wc)
        t = ng
    E = []
    for P in (Pb, Pg):
        t = to_dev(torch, A0, torch.float32)
        E.append(P.iterate(t, K)["energy"][0])
        P.close()
    Eb, Eg = E
    note("energies %s vs %s" % (Eb, Eg))
    noise = 8 * n * 2.0 ** -23 / tau
    assert np.all(np.abs(Eb - Eg) <= 1e-5 * np.abs(Eg) + noise)


@pytest.mark.parametrize("grid,n,prec", [((64, 64), 3, F64), ((8, 32), 2, F64), ((16, 8, 16), 3, FB),
                                         ((128, 64), 4, FB)])
def test_autotune_keeps_results(torch_cuda, grid, n, prec):
    """Launch shapes chosen by mbo_plan_autotune change no iterate (bit for bit)
    and only the summation order of the energy."""
    torch = torch_cuda
    dt = torch.float64 if prec == F64 else torch.float32
    A = inputs.uniform_field(n, grid, 21)
    P0 = plan(grid, n, 2e-3, prec)
    P1 = plan(grid, n, 2e-3, prec)
    shape = P1.autotune()
    note("autotune %s n=%d prec=%d -> %s (rule %s)" % (grid, n, prec, shape, P0.tuning()))
    t0, t1 = to_dev(torch, A, dt), to_dev(torch, A, dt)
    r0, r1 = P0.iterate(t0, 6), P1.iterate(t1, 6)
    assert torch.equal(t0, t1)
    assert np.array_equal(r0["flips"], r1["flips"])
    assert np.allclose(r0["energy"], r1["energy"], rtol=1e-12 if prec == F64 else 1e-5, atol=0)
    if prec == F64:
        # against the oracle's own iterate (the states agree to 1e-12, and the
        # energy moves by at most 2 / tau times that per unit of |dA|)
        ro = oracle.iterate(A, 2e-3, 6)
        Eo = ro["energy"][-1]
        assert abs(r1["energy"][0][-1] - Eo) <= 1e-9 * max(1.0, abs(Eo))
