"""GPU parity of the relaxed gradient flows GD-1 / GD-3 and their energies
(Section 1) through the C ABI, against the FP64 oracle.

Bars: FP64 fields <= 1e-11 max-abs after several steps, energies <= 1e-10
relative; FP32 fields <= 2e-5 (times the field's scale) where the GD-1
projection is well conditioned; the pure diffusion step (eps = inf) damps a
Fourier mode by exactly 1 / (1 + 4 pi^2 dt |k|^2) per step.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1711_01365_amd import inputs

pytestmark = pytest.mark.gpu


def note(*a):
    print("[gpu-relaxed]", *a, flush=True)
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


@pytest.mark.parametrize("kind", [1, 3])
@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("grid", [(32, 32), (16, 64), (8, 8, 16), (8, 1024)])
def test_flow_f64_matches_oracle(torch_cuda, kind, n, grid):
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    note("GD-%d f64 n=%d" % (kind, n), grid)
    A0, _ = oracle.heat(inputs.uniform_field(n, grid, 830 + n), 1e-3, len(grid))
    eps, dt, K = 0.1, 1e-3, 6
    ref = oracle.relaxed_flow(A0, kind, eps, dt, K)
    plan = mbo.Plan(grid, n, 1e-3, precision=mbo.F64)
    X = dev(torch, A0, torch.float64)
    plan.relaxed_flow(X, K, kind, eps, dt)
    err = float(np.abs(X.cpu().numpy().reshape(A0.shape) - ref).max())
    assert err <= 1e-11, err
    for A in (A0, ref):
        e_g = plan.relaxed_energy(dev(torch, A, torch.float64), kind, eps)
        e_o = oracle.relaxed_energy(A, kind, eps)
        assert abs(e_g - e_o) <= 1e-10 * max(1.0, abs(e_o)), (e_g, e_o)
    plan.close()


def test_diffusion_step_damps_a_mode_exactly(torch_cuda):
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    N0, N1, dt, K = 64, 32, 2e-3, 4
    x = np.arange(N0)[:, None] / N0
    y = np.arange(N1)[None, :] / N1
    k0, k1 = 5, -3
    a = np.cos(2 * np.pi * (k0 * x + k1 * y))
    A0 = np.stack([np.stack([a, 0 * a]), np.stack([0 * a, a])])
    plan = mbo.Plan((N0, N1), 2, 1e-3, precision=mbo.F64)
    X = dev(torch, A0, torch.float64)
    plan.relaxed_flow(X, K, mbo.GD3, np.inf, dt)
    g = (1.0 / (1.0 + 4 * np.pi ** 2 * dt * (k0 ** 2 + k1 ** 2))) ** K
    assert np.abs(X.cpu().numpy() - g * A0).max() <= 1e-14
    plan.close()


@pytest.mark.parametrize("prec", ["f32", "f32fb"])
@pytest.mark.parametrize("kind", [1, 3])
def test_flow_fp32(torch_cuda, prec, kind):
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    grid, n = (64, 128), 3
    A0, _ = oracle.heat(inputs.haar_field(n, grid, 840), 5e-4, 2)
    A0 = A0.astype(np.float32).astype(np.float64)
    eps, dt, K = 0.05, 2.5e-4, 5
    ref = oracle.relaxed_flow(A0, kind, eps, dt, K)
    pr = mbo.F32 if prec == "f32" else mbo.F32_F64FALLBACK
    plan = mbo.Plan(grid, n, 1e-3, precision=pr)
    X = dev(torch, A0, torch.float32)
    plan.relaxed_flow(X, K, kind, eps, dt)
    got = X.cpu().double().numpy().reshape(A0.shape)
    err = np.abs(got - ref).max(axis=(0, 1))
    if kind == 1:
        s = np.linalg.svd(np.moveaxis(ref.reshape(n, n, -1), -1, 0), compute_uv=False)
        well = (s[:, -2] + s[:, -1] >= 0.1).reshape(grid)
        err = err[well]
    note("GD-%d %s max err %.3g" % (kind, prec, float(err.max())))
    assert float(err.max()) <= 2e-5
    plan.close()


def test_flow_graph_reuse_and_arguments(torch_cuda):
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    grid, n = (32, 32), 3
    A0 = inputs.haar_field(n, grid, 850)
    plan = mbo.Plan(grid, n, 1e-3, precision=mbo.F64)
    outs = []
    for eps in (0.1, 0.2, 0.1):
        X = dev(torch, A0, torch.float64)
        plan.relaxed_flow(X, 3, mbo.GD3, eps, 1e-3)
        outs.append(X.cpu().numpy())
    assert np.array_equal(outs[0], outs[2]) and not np.array_equal(outs[0], outs[1])
    X = dev(torch, A0, torch.float64)
    for kind, eps, dt in ((2, 0.1, 1e-3), (1, 0.0, 1e-3), (3, 0.1, 0.0), (3, 0.1, np.inf)):
        with pytest.raises(mbo.MboError) as ei:
            plan.relaxed_flow(X, 1, kind, eps, dt)
        assert ei.value.status == 1
    plan.close()


def test_full_size_energy_decreases(torch_cuda):
    """n = 3, 512^2, FP32 + fallback (the bench configuration): one step against
    the oracle, and E_{2,eps} non-increasing over 20 steps."""
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    w = inputs.HAAR_512
    eps = 4.0 / w.grid[0]
    dt = 0.1 * eps * eps
    A0 = w.field().astype(np.float32).astype(np.float64)
    plan = mbo.Plan(w.grid, w.n, w.tau, precision=mbo.F32_F64FALLBACK)
    X = dev(torch, A0, torch.float32)
    plan.relaxed_flow(X, 1, mbo.GD3, eps, dt)
    ref = oracle.relaxed_flow(A0, 3, eps, dt, 1)
    err = float(np.abs(X.cpu().double().numpy().reshape(A0.shape) - ref).max())
    note("512^2 one step error %.3g" % err)
    assert err <= 2e-5
    E = [plan.relaxed_energy(X, mbo.GD3, eps)]
    for _ in range(20):
        plan.relaxed_flow(X, 1, mbo.GD3, eps, dt)
        E.append(plan.relaxed_energy(X, mbo.GD3, eps))
    E = np.array(E)
    note("E %.6g -> %.6g" % (E[0], E[-1]))
    assert np.all(np.diff(E) <= 1e-5 * np.abs(E[:-1]))
    plan.close()
