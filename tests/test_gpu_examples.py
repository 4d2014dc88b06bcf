"""The paper's flat-torus examples (Section 6.1) and the SO(2) index on the GPU.

Bars: the index against the oracle's to 1e-9 (FP64) / 1e-4 (FP32 input) per
loop, and the same integers after rounding; the three examples in FP64 at 256^2
against the oracle (energies to 1e-9 relative, final fields to 1e-8, det flips
per iteration identical); at the paper's size (1024^2, FP32 + FP64 fallback,
the measured configuration's precision) the end states the paper describes,
which are all it fixes (its figures are absent).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1711_01365_amd import inputs

pytestmark = pytest.mark.gpu


def note(*a):
    print("[gpu-examples]", *a, flush=True)
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


def angle(A):
    return np.arctan2(A[1, 0], A[0, 0])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_so2_index_matches_oracle(torch_cuda, prec):
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    grid = (64, 128)
    fields = [inputs.linear_angle_field(grid, 2, -3), inputs.linear_angle_field(grid, 0, 1),
              inputs.line_defect_field(grid, True), inputs.star_defect_field(grid)]
    rng = np.random.default_rng(5)
    al = 1.4 * np.tanh(rng.standard_normal(grid))
    c, s = np.cos(al), np.sin(al)
    fields.append(np.stack([np.stack([c, s]), np.stack([s, -c])]))  # reflections, bounded angle
    A = np.stack(fields)
    dt, pr, tol = (torch.float64, mbo.F64, 1e-9) if prec == "f64" else (torch.float32, mbo.F32, 1e-4)
    if prec == "f32":
        A = A.astype(np.float32).astype(np.float64)
    plan = mbo.Plan(grid, 2, 1e-3, precision=pr, batch=len(fields))
    wx, wy = plan.so2_index(dev(torch, A, dt))
    for b in range(len(fields)):
        ox, oy = oracle.winding(A[b])
        assert np.abs(wx[b] - ox).max() <= tol and np.abs(wy[b] - oy).max() <= tol
        assert np.array_equal(np.rint(wx[b]), np.rint(ox)) and np.array_equal(np.rint(wy[b]), np.rint(oy))
    assert np.all(np.rint(wx[0]) == 2) and np.all(np.rint(wy[0]) == -3)
    plan.close()


def test_so2_index_rejects_other_plans(torch_cuda):
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    plan = mbo.Plan((16, 16), 3, 1e-3, precision=mbo.F64)
    with pytest.raises(mbo.MboError) as ei:
        plan.so2_index(torch.zeros((3, 3, 16, 16), dtype=torch.float64, device="cuda"))
    assert ei.value.status == 2
    plan.close()


EXAMPLES = {"star": (inputs.EXAMPLE_STAR, lambda g: inputs.star_defect_field(g)),
            "lines": (inputs.EXAMPLE_LINES, lambda g: inputs.line_defect_field(g, False)),
            "winding": (inputs.EXAMPLE_WINDING, lambda g: inputs.line_defect_field(g, True))}


@pytest.mark.parametrize("name", sorted(EXAMPLES))
def test_examples_f64_match_oracle(torch_cuda, name):
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    w, make = EXAMPLES[name]
    N, K = 256, 40
    A0 = make((N, N))
    ref = oracle.iterate(A0, w.tau, K)
    plan = mbo.Plan((N, N), 2, w.tau, precision=mbo.F64)
    X = dev(torch, A0, torch.float64)
    logs = plan.iterate(X, K)
    err = float(np.abs(X.cpu().numpy().reshape(A0.shape) - ref["A"]).max())
    note(name, "max |A - A_oracle| = %.3g" % err)
    assert err <= 1e-12
    assert np.array_equal(logs["flips"][0], ref["flips"])
    assert np.abs(logs["energy"][0] - ref["energy"]).max() <= 1e-9 * np.abs(ref["energy"]).max()
    plan.close()


@pytest.mark.parametrize("name", sorted(EXAMPLES))
def test_examples_at_the_paper_size(torch_cuda, name):
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    w, make = EXAMPLES[name]
    A0 = make(w.grid).astype(np.float32)
    plan = mbo.Plan(w.grid, 2, w.tau, precision=mbo.F32_F64FALLBACK)
    X = dev(torch, A0, torch.float32)
    logs = plan.iterate(X, w.iters)
    A = X.cpu().double().numpy().reshape(A0.shape)
    E = logs["energy"][0]
    # E carries the float rounding of <A, HA> (about n eps_32) magnified by 1/tau
    noise = 8 * 2.0 ** -23 * 2 / w.tau
    assert np.all(np.diff(E[1:]) <= 1e-5 * np.abs(E[1:-1]) + noise)
    det = A[0, 0] * A[1, 1] - A[0, 1] * A[1, 0]
    wx, wy = plan.so2_index(X)
    th = angle(A)
    note(name, "SO(2) points %d, angle std %.3g, index x %s y %s, E %.4g -> %.4g"
         % ((det > 0).sum(), th.std(), np.unique(np.rint(wx)), np.unique(np.rint(wy)), E[0], E[-1]))
    if name == "star":
        # the SO(2) region shrinks away and the field becomes uniform
        assert int((det > 0).sum()) == 0 and th.std() < 0.05
        assert np.all(np.rint(wx) == 0) and np.all(np.rint(wy) == 0)
    elif name == "lines":
        # two straight defect lines parallel to the y-axis, uniform angle
        rows = np.all((det > 0) == (det[:, :1] > 0), axis=1)
        assert rows.mean() >= 0.95 and 0 < int((det > 0).sum()) < det.size
        assert th.std() < 1e-3
        assert np.all(np.rint(wx) == 0) and np.all(np.rint(wy) == 0)
    else:
        # a non-constant end state that keeps turning once along y
        assert th.std() > 1.0
        assert np.all(np.rint(wy) == 1) and np.all(np.rint(wx) == 0)
    plan.close()
