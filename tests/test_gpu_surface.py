"""GPU parity of the closest-point surface diffusion and the MBO iteration on a
sphere (Section 5.2, Algorithm 1 with the surface diffusion step) through the C
ABI, against the FP64 oracle's direct quadrature sums.

Bars:
  * the sample set (quadrature points, closest points, weights, band cells and
    width) equals the oracle's to rounding (1e-15 relative);
  * the diffusion step: max |GPU - oracle| <= max(eps, 1e-11) * max |A| for
    FP64 surfaces and max(eps, 4e-6) * max |A| for float surfaces (the
    gridding runs at a tenth of eps and reaches about 0.1 eps; the rest is
    headroom; float rounding reaches 2e-6 at 3.3 M samples);
  * the iteration: per step, identical det-sign decisions and projections to
    1e-9 (FP64) / 2e-4 (float) away from near-singular diffused matrices;
  * at the sphere experiment's size (3.3 M samples): sampled outputs against
    the oracle, constants kept, the degree-1 harmonic damped by 1 - 2 tau, and
    the SO^-(3) octant shrinking;
  * ten random configurations (radius, cell size, 1-6 nodes per cell, tau, eps,
    n, both precisions) to the same bars, covering every spreading variant.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1711_01365_amd import inputs

pytestmark = pytest.mark.gpu


def note(*a):
    print("[gpu-surface]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    from paper_1711_01365_amd import mbo
    mbo.load()
    return torch


def dev(torch, A, dtype):
    return torch.tensor(np.ascontiguousarray(A), dtype=dtype, device="cuda")


def surface(R, dx, p, tau, eps, n, prec):
    from paper_1711_01365_amd import mbo
    return mbo.SphereSurface(R, dx, p, tau, eps, n, precision=prec)


def band_of(s):
    """The oracle's own sample set for the surface's parameters (the oracle takes
    no input from the library), checked equal to the library's."""
    ref = oracle.sphere_band(s.R, s.dx, s.p, s.tau, s.eps)
    xq, xc, w = s.points()
    assert s.cells == ref["cells"] and s.m == ref["w"].size
    assert np.abs(xq - ref["xq"]).max() <= 1e-15 * (s.R + 1)
    assert np.abs(xc - ref["xc"]).max() <= 1e-15 * (s.R + 1)
    assert np.abs(w - ref["w"]).max() <= 1e-15 * ref["w"].max()
    return ref


@pytest.mark.parametrize("R,dx,p,tau,eps", [(1.0, 0.12, 1, 0.01, 1e-6), (0.7, 0.1, 2, 0.005, 1e-4),
                                             (1.0, 0.05, 3, 0.005, 1e-6)])
def test_sample_set_matches_oracle(torch_cuda, R, dx, p, tau, eps):
    from paper_1711_01365_amd import mbo
    note("geometry", R, dx, p, tau, eps)
    s = surface(R, dx, p, tau, eps, 3, mbo.F64)
    ref = oracle.sphere_band(R, dx, p, tau, eps)
    assert s.cells == ref["cells"] and s.m == ref["w"].size
    assert abs(s.band_width - ref["wb"]) <= 1e-14 * ref["wb"]
    xq, xc, w = s.points()
    assert np.abs(xq - ref["xq"]).max() <= 1e-15 * (R + 1)
    assert np.abs(xc - ref["xc"]).max() <= 1e-15 * (R + 1)
    assert np.abs(w - ref["w"]).max() <= 1e-15 * ref["w"].max()
    s.close()


def _tol(prec, eps):
    from paper_1711_01365_amd import mbo
    return max(eps, 1e-11) if prec == mbo.F64 else max(eps, 4e-6)


@pytest.mark.parametrize("prec_name", ["F64", "F32"])
@pytest.mark.parametrize("eps", [1e-3, 1e-4, 1e-6, 1e-9, 1e-11])
def test_diffuse_matches_oracle(torch_cuda, prec_name, eps):
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    prec = getattr(mbo, prec_name)
    if prec == mbo.F32 and eps < 1e-7:
        pytest.skip("float surfaces grid to 1e-7 at best")
    tau, dx, n = 0.01, 0.15, 2
    note("diffuse", prec_name, "eps", eps)
    s = surface(1.0, dx, 1, tau, eps, n, prec)
    b = band_of(s)
    A = inputs.normal_field(n, (s.m,), 900)
    ref = oracle.surface_diffuse(b, A, tau)
    dt = torch.float64 if prec == mbo.F64 else torch.float32
    X = dev(torch, A, dt)
    Y = s.diffuse(X)
    torch.cuda.synchronize()
    err = np.abs(Y.double().cpu().numpy() - ref).max() / np.abs(A).max()
    note("  m", s.m, "grid", s.grid, "err/max|A|", err)
    assert err <= _tol(prec, eps), err
    s.close()


@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("prec_name", ["F64", "F32"])
def test_diffuse_matrix_sizes(torch_cuda, n, prec_name):
    """Every n (1 to 8 complex planes, LDS tiles of several planes per launch),
    p = 2 samples per cell axis, radius 0.8."""
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    prec = getattr(mbo, prec_name)
    R, dx, p, tau, eps = 0.8, 0.2, 2, 0.008, 1e-5
    note("diffuse n", n, prec_name)
    s = surface(R, dx, p, tau, eps, n, prec)
    b = band_of(s)
    A = inputs.uniform_field(n, (s.m,), 910 + n)
    ref = oracle.surface_diffuse(b, A, tau)
    dt = torch.float64 if prec == mbo.F64 else torch.float32
    Y = s.diffuse(dev(torch, A, dt))
    torch.cuda.synchronize()
    err = np.abs(Y.double().cpu().numpy() - ref).max() / np.abs(A).max()
    note("  m", s.m, "grid", s.grid, "err/max|A|", err)
    assert err <= _tol(prec, eps), err
    s.close()


@pytest.mark.parametrize("prec_name,eps", [("F64", 1e-11), ("F32", 1e-6)])
def test_diffuse_wide_cells(torch_cuda, prec_name, eps):
    """Cells much wider than the grid spacing (dx = 0.5, p = 6): the union of a
    cell's stencils needs more LDS than the cell kernel has, so the samples are
    spread one by one."""
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    prec = getattr(mbo, prec_name)
    R, dx, p, tau = 1.0, 0.5, 6, 0.005
    note("wide cells", prec_name, eps)
    s = surface(R, dx, p, tau, eps, 1, prec)
    b = band_of(s)
    A = inputs.uniform_field(1, (s.m,), 920)
    ref = oracle.surface_diffuse(b, A, tau)
    dt = torch.float64 if prec == mbo.F64 else torch.float32
    Y = s.diffuse(dev(torch, A, dt))
    torch.cuda.synchronize()
    err = np.abs(Y.double().cpu().numpy() - ref).max() / np.abs(A).max()
    note("  m", s.m, "grid", s.grid, "err/max|A|", err)
    assert err <= _tol(prec, eps), err
    s.close()


@pytest.mark.parametrize("prec_name", ["F64", "F32"])
def test_diffuse_five_nodes_sampled(torch_cuda, prec_name):
    """p = 5 nodes per cell axis (one wave per cell with LDS accumulation; the
    register-line variant takes p <= 4): 1.9 M samples, outputs sampled against
    the oracle's convolution at their closest points."""
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    prec = getattr(mbo, prec_name)
    R, dx, p, tau, eps = 1.0, 0.1, 5, 0.01, 1e-4
    note("five nodes", prec_name)
    s = surface(R, dx, p, tau, eps, 2, prec)
    b = band_of(s)
    A = inputs.uniform_field(2, (s.m,), 930)
    dt = torch.float64 if prec == mbo.F64 else torch.float32
    Y = s.diffuse(dev(torch, A, dt)).double().cpu().numpy()
    idx = np.random.default_rng(8).choice(s.m, 48, replace=False)
    ref = oracle.heat_at(b, A, tau, b["xc"][:, idx])
    err = np.abs(Y[:, :, idx] - ref).max() / np.abs(A).max()
    note("  m", s.m, "grid", s.grid, "sampled err/max|A|", err)
    assert err <= _tol(prec, eps), err
    s.close()


def test_diffuse_rejects_aliasing_and_bad_shapes(torch_cuda):
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    s = surface(1.0, 0.2, 1, 0.01, 1e-4, 2, mbo.F64)
    X = torch.zeros((2, 2, s.m), dtype=torch.float64, device="cuda")
    with pytest.raises(mbo.MboError):
        s.diffuse(X, X)
    with pytest.raises(ValueError):
        s.diffuse(torch.zeros((2, 2, s.m + 1), dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        s.diffuse(X.float())
    s.close()


def test_unsupported_and_invalid_surfaces(torch_cuda):
    from paper_1711_01365_amd import mbo
    with pytest.raises(mbo.MboError) as e:
        surface(10.0, 0.5, 1, 1e-3, 1e-6, 3, mbo.F64)  # grid > 512 per axis
    assert e.value.status == 2
    for bad in [(-1.0, 0.1, 1, 0.01, 1e-6), (1.0, 0.0, 1, 0.01, 1e-6), (1.0, 0.1, 0, 0.01, 1e-6),
                (1.0, 0.1, 9, 0.01, 1e-6), (1.0, 0.1, 1, 0.0, 1e-6), (1.0, 0.1, 1, 0.01, 0.0)]:
        with pytest.raises(mbo.MboError) as e:
            surface(*bad, 3, mbo.F64)
        assert e.value.status == 1


def _octant_start(b):
    """The sphere experiment's initial field, projected (oracle)."""
    M = inputs.SPHERE_MATRICES
    Q = oracle.project(np.stack([M[0], M[1]], axis=-1).reshape(3, 3, 2))[0]
    x, y, z = b["xc"]
    inside = (x < 0) & (y < 0) & (z > 0)
    return np.where(inside[None, None, :], Q[:, :, 0:1], Q[:, :, 1:2])


@pytest.mark.parametrize("prec_name", ["F64", "F32_F64FALLBACK"])
def test_iterate_steps_match_oracle(torch_cuda, prec_name):
    """Each MBO step from the oracle's previous iterate: the same det-sign
    decisions and projections wherever the diffused matrix is not close to
    singular, and the flip counts within the number of close calls."""
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    prec = getattr(mbo, prec_name)
    f64 = prec == mbo.F64
    tau, eps = 0.01, (1e-9 if f64 else 1e-6)
    s = surface(1.0, 0.15, 1, tau, eps, 3, prec)
    b = band_of(s)
    A = _octant_start(b)
    dt = torch.float64 if f64 else torch.float32
    smin_safe, qtol = (1e-6, 1e-9) if f64 else (2e-2, 2e-4)
    for step in range(5):
        note("iterate", prec_name, "step", step, "m", s.m)
        D = oracle.surface_diffuse(b, A, tau)
        ref, fl_ref = oracle.surface_iterate(b, A, tau, 1)
        X = dev(torch, A, dt)
        fl = s.iterate(X, 1, flips=True)
        got = X.double().cpu().numpy()
        sv = np.linalg.svd(np.moveaxis(D, 2, 0), compute_uv=False)
        smin = sv[:, -1]
        safe = smin > smin_safe
        close = int((~safe).sum())
        assert np.array_equal(np.sign(np.linalg.det(np.moveaxis(got, 2, 0)))[safe],
                              np.sign(np.linalg.det(np.moveaxis(ref, 2, 0)))[safe])
        err = np.abs(got - ref)[:, :, safe].max()
        note("  flips", int(fl[0]), int(fl_ref[0]), "close calls", close, "err", err)
        assert err <= qtol, err
        assert abs(int(fl[0]) - int(fl_ref[0])) <= close
        A = ref
    s.close()


def test_surface_on_a_side_stream(torch_cuda):
    """A surface created on a side stream (default priority) runs there: its
    diffusion and three MBO steps give the same bits as on the default stream."""
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    tau, eps = 0.01, 1e-9
    s0 = surface(1.0, 0.2, 2, tau, eps, 3, mbo.F64)
    A = _octant_start(band_of(s0))
    H0 = s0.diffuse(dev(torch, A, torch.float64)).cpu().numpy()
    X0 = dev(torch, A, torch.float64)
    f0 = s0.iterate(X0, 3, flips=True)
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s1 = mbo.SphereSurface(1.0, 0.2, 2, tau, eps, 3, precision=mbo.F64, stream=st)
        H1 = s1.diffuse(dev(torch, A, torch.float64))
        X1 = dev(torch, A, torch.float64)
        f1 = s1.iterate(X1, 3, flips=True)
    st.synchronize()
    note("side stream: m", s1.m, "flips", list(f1))
    assert np.array_equal(H1.cpu().numpy(), H0)
    assert np.array_equal(X1.cpu().numpy(), X0.cpu().numpy())
    assert np.array_equal(np.asarray(f1), np.asarray(f0))
    s0.close()
    s1.close()


def test_iterate_zero_steps_and_flip_totals(torch_cuda):
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    tau = 0.02
    s = surface(1.0, 0.15, 1, tau, 1e-9, 3, mbo.F64)
    b = band_of(s)
    A0 = _octant_start(b)
    X = dev(torch, A0, torch.float64)
    s.iterate(X, 0)
    assert np.array_equal(X.cpu().numpy(), A0)
    ref, fl_ref = oracle.surface_iterate(b, A0, tau, 6)
    fl = s.iterate(X, 6, flips=True)
    got = X.cpu().numpy()
    note("flips", fl.tolist(), fl_ref.tolist())
    n_ref = int((oracle.det_sign(ref) < 0).sum())
    n_got = int((np.linalg.det(np.moveaxis(got, 2, 0)) < 0).sum())
    assert abs(n_got - n_ref) <= 2 and np.abs(fl - fl_ref).max() <= 2
    assert n_got < int((oracle.det_sign(A0) < 0).sum())


@pytest.fixture(scope="module")
def paper_sphere(torch_cuda):
    """The sphere experiment's sample set (3.3 M samples) on FP64 and float
    surfaces, with its initial field."""
    from paper_1711_01365_amd import mbo
    w = inputs.SPHERE_PAPER
    note("paper sphere surfaces")
    s64 = surface(w.R, w.dx, w.p, w.tau, w.eps, w.n, mbo.F64)
    s32 = surface(w.R, w.dx, w.p, w.tau, w.eps, w.n, mbo.F32_F64FALLBACK)
    b = band_of(s64)
    yield w, s64, s32, b
    s64.close()
    s32.close()


@pytest.mark.parametrize("which", ["F64", "F32"])
def test_paper_sphere_sampled_outputs(torch_cuda, paper_sphere, which):
    torch = torch_cuda
    w, s64, s32, b = paper_sphere
    s = s64 if which == "F64" else s32
    dt = torch.float64 if which == "F64" else torch.float32
    A = inputs.sphere_octant_field(b["xc"])
    Y = s.diffuse(dev(torch, A, dt)).double().cpu().numpy()
    idx = np.random.default_rng(7).choice(s.m, 48, replace=False)
    ref = oracle.heat_at(b, A, w.tau, b["xc"][:, idx])
    err = np.abs(Y[:, :, idx] - ref).max() / np.abs(A).max()
    note("paper sphere", which, "m", s.m, "grid", s.grid, "sampled err/max|A|", err)
    assert err <= (w.eps if which == "F64" else 4e-6), err


@pytest.mark.parametrize("which", ["F64", "F32"])
def test_paper_sphere_constants_and_first_harmonic(torch_cuda, paper_sphere, which):
    """S_tau 1 = 1 up to the band tolerance, and the degree-1 harmonic z is
    damped by the factor 1 - 2 tau of the closest point extension (constant
    along normals), at every sample."""
    torch = torch_cuda
    w, s64, s32, b = paper_sphere
    s = s64 if which == "F64" else s32
    dt = torch.float64 if which == "F64" else torch.float32
    ones = torch.ones((3, 3, s.m), dtype=dt, device="cuda")
    Y = s.diffuse(ones)
    e1 = (Y - 1).abs().max().item()
    z = b["xc"][2]
    F = np.zeros((3, 3, s.m))
    F[0, 0] = z
    G = s.diffuse(dev(torch, F, dt)).double().cpu().numpy()
    ratio = G[0, 0][np.abs(z) > 0.2] / z[np.abs(z) > 0.2]
    note("paper sphere", which, "|S1 - 1|", e1, "z factor", ratio.min(), ratio.max(), "1-2tau", 1 - 2 * w.tau)
    assert e1 <= 1e-5
    assert np.abs(ratio - (1 - 2 * w.tau)).max() <= 2e-5


def test_paper_sphere_octant_shrinks(torch_cuda, paper_sphere):
    """From the printed (non-orthogonal) matrices the first step moves the
    interface outwards (the average of the two raw matrices favours the first);
    from then on the SO^-(3) region loses samples (the oracle shows the same
    sequence on a coarse band)."""
    torch = torch_cuda
    w, s64, s32, b = paper_sphere
    A = dev(torch, inputs.sphere_octant_field(b["xc"]), torch.float32)
    det_neg = lambda: int((np.linalg.det(np.moveaxis(A.double().cpu().numpy(), 2, 0)) < 0).sum())
    fl1 = s32.iterate(A, 1, flips=True)
    n1 = det_neg()
    fl = s32.iterate(A, 8, flips=True)
    n9 = det_neg()
    x, y, z = b["xc"]
    n0 = int(((x < 0) & (y < 0) & (z > 0)).sum())
    note("octant", n0, "->", n1, "->", n9, "flips", fl1.tolist(), fl.tolist())
    assert 0 < n9 < n1 and fl.min() > 0


def _random_config(seed):
    rng = np.random.default_rng(2000 + seed)
    R = float(rng.uniform(0.6, 1.2))
    p = int(rng.integers(1, 7))
    tau = float(10 ** rng.uniform(-2.3, -1.8))
    eps = float(10 ** rng.uniform(-9, -3))
    n = int(rng.integers(1, 5))
    dx = float(rng.uniform(0.12, 0.25)) * (1 + 0.4 * (p - 1))
    return R, dx, p, tau, eps, n


# Corners of the parameter space: a small sphere with a fine lattice, a large
# one with a coarse lattice, a short time step (a wide grid), a long one (a
# wide band); each either builds and meets the tolerance against the oracle, or
# is refused as unsupported (a grid beyond 512 per axis).
EXTREME_CONFIGS = [(0.15, 0.03, 2, 2e-3, 1e-6, 2), (4.0, 0.6, 2, 0.4, 1e-6, 2),
                   (1.0, 0.1, 3, 1e-3, 1e-6, 1), (1.0, 0.3, 2, 0.1, 1e-9, 3)]


@pytest.mark.parametrize("cfg", range(len(EXTREME_CONFIGS)))
def test_extreme_configurations(torch_cuda, cfg):
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    R, dx, p, tau, eps, n = EXTREME_CONFIGS[cfg]
    for prec in (mbo.F64, mbo.F32):
        try:
            s = surface(R, dx, p, tau, eps, n, prec)
        except mbo.MboError as e:
            note("extreme", cfg, "refused:", str(e))
            assert e.status == 2
            continue
        b = band_of(s)
        A = inputs.uniform_field(n, (s.m,), 970 + cfg)
        dt = torch.float64 if prec == mbo.F64 else torch.float32
        Y = s.diffuse(dev(torch, A, dt)).double().cpu().numpy()
        if s.m <= 20000:
            ref, got = oracle.surface_diffuse(b, A, tau), Y
        else:
            idx = np.random.default_rng(cfg).choice(s.m, 64, replace=False)
            ref, got = oracle.heat_at(b, A, tau, b["xc"][:, idx]), Y[:, :, idx]
        err = np.abs(got - ref).max() / np.abs(A).max()
        note("extreme", cfg, "R %.3f dx %.3f p %d tau %.4f eps %.1e n %d" % (R, dx, p, tau, eps, n),
             "prec", prec, "m", s.m, "grid", s.grid, "err", err)
        assert err <= _tol(prec, eps), err
        s.close()


@pytest.mark.parametrize("seed", range(10))
def test_random_configurations(torch_cuda, seed):
    """Random radius, cell size, nodes per cell (1-6: every spreading variant),
    tau, eps and n, both precisions, against the oracle's direct sums (all
    outputs when the band is small, 64 sampled outputs otherwise)."""
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    R, dx, p, tau, eps, n = _random_config(seed)
    for prec in (mbo.F64, mbo.F32):
        s = surface(R, dx, p, tau, eps, n, prec)
        b = band_of(s)
        A = inputs.uniform_field(n, (s.m,), 940 + seed)
        dt = torch.float64 if prec == mbo.F64 else torch.float32
        Y = s.diffuse(dev(torch, A, dt)).double().cpu().numpy()
        if s.m <= 20000:
            ref, got = oracle.surface_diffuse(b, A, tau), Y
        else:
            idx = np.random.default_rng(seed).choice(s.m, 64, replace=False)
            ref, got = oracle.heat_at(b, A, tau, b["xc"][:, idx]), Y[:, :, idx]
        err = np.abs(got - ref).max() / np.abs(A).max()
        note("random", seed, "R %.3f dx %.3f p %d tau %.4f eps %.1e n %d" % (R, dx, p, tau, eps, n),
             "prec", prec, "m", s.m, "grid", s.grid, "err", err)
        assert err <= _tol(prec, eps), err
        s.close()
