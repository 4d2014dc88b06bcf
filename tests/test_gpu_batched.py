"""GPU tests of batched plans (mbo_plan_batched): independent fields of mixed
grid, n and tau in one captured graph.

Each field of a batched run must equal its own single-field run: bit for bit
when both use the same launch shapes (the transforms and the projection do the
same arithmetic per line and per point), and to FP32/FP64 rounding of the energy
sums otherwise.  FP64 batched runs also match the oracle (<= 1e-12).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1711_01365_amd import inputs

pytestmark = pytest.mark.gpu

F64, F32, FB = 0, 1, 2

MIXED = [((32, 32), 2, 1e-3, "uniform"), ((64, 64), 3, 5e-4, "haar"), ((32, 32), 2, 3e-3, "normal"),
         ((16, 16, 16), 3, 1e-3, "normal"), ((64, 32), 1, 2e-3, "uniform"), ((32, 64), 4, 1e-3, "uniform"),
         ((64, 64), 3, 2e-3, "uniform")]


def note(*a):
    print("[gpu-batched]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    from paper_1711_01365_amd import mbo
    mbo.load()
    return torch


def gen(init, n, grid, seed):
    return {"uniform": inputs.uniform_field, "haar": inputs.haar_field, "normal": inputs.normal_field}[init](
        n, grid, seed)


def mixed_fields():
    return [gen(init, n, grid, 500 + i) for i, (grid, n, tau, init) in enumerate(MIXED)]


def batched(fields_spec, prec, autotune):
    from paper_1711_01365_amd import mbo
    return mbo.BatchedPlan([(g, n, t) for g, n, t, *_ in fields_spec], precision=prec, autotune=autotune)


def single(grid, n, tau, prec):
    from paper_1711_01365_amd import mbo
    return mbo.Plan(grid, n, tau, precision=prec)


@pytest.mark.parametrize("autotune", [False, True])
def test_batched_f64_matches_single_and_oracle(torch_cuda, autotune):
    torch = torch_cuda
    K = 5
    A = mixed_fields()
    note("batched f64 autotune=%s" % autotune)
    bp = batched(MIXED, F64, autotune)
    flat = bp.pack([torch.tensor(a, dtype=torch.float64, device="cuda") for a in A])
    r = bp.iterate(flat, K)
    outs = bp.unpack(flat)
    for i, ((grid, n, tau, _), a) in enumerate(zip(MIXED, A)):
        sp = single(grid, n, tau, F64)
        t = torch.tensor(a, dtype=torch.float64, device="cuda")
        rs = sp.iterate(t, K)
        same = torch.equal(outs[i], t)
        ro = oracle.iterate(a, tau, K)
        err = np.abs(outs[i].cpu().numpy() - ro["A"]).max()
        note("  field %d %s n=%d: bitwise=%s, oracle err %.2e, tuning %s" % (i, grid, n, same, err, bp.tuning(i)))
        assert same
        assert err <= 1e-12
        assert np.array_equal(r["flips"][i], rs["flips"][0])
        assert np.array_equal(r["flips"][i], ro["flips"])
        assert np.allclose(r["energy"][i], rs["energy"][0], rtol=1e-13, atol=0)
        assert np.allclose(r["energy"][i], ro["energy"], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("prec", [F32, FB])
def test_batched_f32_matches_single(torch_cuda, prec):
    torch = torch_cuda
    K = 8
    A = mixed_fields()
    note("batched f32 prec=%d" % prec)
    bp = batched(MIXED, prec, False)
    flat = bp.pack([torch.tensor(a, dtype=torch.float32, device="cuda") for a in A])
    r = bp.iterate(flat, K)
    outs = bp.unpack(flat)
    for i, ((grid, n, tau, _), a) in enumerate(zip(MIXED, A)):
        t = torch.tensor(a, dtype=torch.float32, device="cuda")
        rs = single(grid, n, tau, prec).iterate(t, K)
        assert torch.equal(outs[i], t)
        assert np.array_equal(r["flips"][i], rs["flips"][0])
        assert np.array_equal(r["fallbacks"][i], rs["fallbacks"][0])


def test_batched_energy_diffuse_project(torch_cuda):
    torch = torch_cuda
    A = mixed_fields()
    bp = batched(MIXED, F64, True)
    flat = bp.pack([torch.tensor(a, dtype=torch.float64, device="cuda") for a in A])
    E = bp.energy(flat)
    D = bp.unpack(bp.diffuse(flat))
    P = bp.unpack(bp.project(flat))
    for i, ((grid, n, tau, _), a) in enumerate(zip(MIXED, A)):
        e_ref = oracle.energy(a, tau)
        assert abs(E[i] - e_ref) <= 1e-12 * max(1.0, abs(e_ref))
        h_ref, _ = oracle.heat(a.reshape((n * n,) + grid), tau, len(grid))
        assert np.abs(D[i].cpu().numpy().reshape(h_ref.shape) - h_ref).max() <= 1e-12
        q_ref = oracle.project(a)[0]
        assert np.abs(P[i].cpu().numpy() - q_ref).max() <= 1e-12
    ds = torch.zeros(16, dtype=torch.int8, device="cuda")
    out = torch.empty_like(flat)
    rc = bp._lib.mbo_project(bp._h, bp._field(flat), bp._field(out), ds.data_ptr())
    assert rc == 2  # det signs are not offered for mixed fields


def test_batched_unsupported_calls(torch_cuda):
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    bp = batched(MIXED[:2], F64, False)
    with pytest.raises(mbo.MboError) as e:
        bp.set_tau(1e-3)
    assert e.value.status == 2
    flat = torch.zeros(bp.total, dtype=torch.float64, device="cuda")
    with pytest.raises(mbo.MboError):
        bp.project_vjp(flat, flat)


def test_batched_configuration(torch_cuda):
    """The batched configuration at full size: 64 fields (seed 3) of n in {2,3,4},
    grids 128^2..1024^2, log-uniform tau, 50 FP32 iterations in one graph, tiles
    chosen by the autotuner.  Every field equals its single-field run within FP32
    rounding (bitwise where the launch shapes agree; its logged energy within the
    rounding of the float energy terms), is orthogonal at every point, and its
    energy does not increase from s = 1 (FP32 slack)."""
    torch = torch_cuda
    bw = inputs.BatchedWorkload()
    spec = [(m.grid, m.n, m.tau) for m in bw.members]
    from paper_1711_01365_amd import mbo
    note("batched configuration: %d fields, %d points" % (len(spec), bw.points))
    bp = mbo.BatchedPlan(spec, precision=F32, autotune=True)
    flat = bp.pack([torch.tensor(m.field(), dtype=torch.float32, device="cuda") for m in bw.members])
    r = bp.iterate(flat, bw.iters)
    outs = bp.unpack(flat)
    nbit = 0
    for i, m in enumerate(bw.members):
        t = torch.tensor(m.field(), dtype=torch.float32, device="cuda")
        rs = single(m.grid, m.n, m.tau, F32).iterate(t, bw.iters)
        diff = (outs[i] - t).abs().max().item()
        nbit += int(diff == 0.0)
        assert diff <= 1e-5, (i, diff)
        E = r["energy"][i]
        assert np.all(np.diff(E[1:]) <= 1e-5 * abs(E[1]) + 1e-6)
        # the logged energy (1/tau)(n - <A, HA>) is summed from float terms
        # (about 8 per thread before the double reduction): launch shapes that
        # differ (the autotuner's tiles against the single run's rule) change
        # its rounding by up to about 8 n u_32 / tau
        noise = 8 * m.n * 2.0 ** -23 / m.tau
        assert abs(E[-1] - rs["energy"][0][-1]) <= 1e-5 * abs(E[-1]) + noise, (i, E[-1], rs["energy"][0][-1])
        M = outs[i].double().reshape(m.n, m.n, -1).permute(2, 0, 1)
        I = torch.eye(m.n, dtype=torch.float64, device="cuda")
        assert (M.transpose(1, 2).contiguous() @ M.contiguous() - I).abs().max().item() < 1e-5
    note("  %d of %d fields bitwise equal to their single runs" % (nbit, len(spec)))


def _class_members():
    """First member of every (n, N) class of the batched configuration."""
    bw = inputs.BatchedWorkload()
    first = {}
    for i, m in enumerate(bw.members):
        first.setdefault((m.n, m.grid[0]), i)
    return bw, sorted(first.items())


_BW, _CLASSES = _class_members()


def _pm(A):
    n = A.shape[0]
    return np.moveaxis(A.reshape(n, n, -1), -1, 0)


def _fp32_step_ok(err, gap, e_heat):
    u32 = 2.0 ** -24
    bound = np.maximum(1e-5, 4.0 * (e_heat + 8 * u32) / gap)
    return bool(np.all(err <= bound)) and (not np.any(gap >= 0.1) or err[gap >= 0.1].max() <= 1e-5)


@pytest.fixture(scope="module")
def batched_config_plan(torch_cuda):
    from paper_1711_01365_amd import mbo
    spec = [(m.grid, m.n, m.tau) for m in _BW.members]
    return mbo.BatchedPlan(spec, precision=F32, autotune=True)


@pytest.mark.parametrize("cls,field", _CLASSES, ids=["n%d_%d" % c for c, _ in _CLASSES])
def test_batched_configuration_class_against_oracle(torch_cuda, batched_config_plan, cls, field):
    """One field of each (n, N) class of the batched configuration, at its real
    size, inside the full 64-field FP32 plan: steps 1 and 2 against the FP64
    oracle's steps from the same float input (step 2 from the oracle's own iterate
    1), per point within the FP32 bound (1e-5 where sigma_{n-1} + sigma_n >= 0.1,
    the first-order bound of the measured diffusion error elsewhere), and the
    logged energy of the step equal to the oracle's within FP32 rounding."""
    torch = torch_cuda
    bp = batched_config_plan
    m = _BW.members[field]
    note("batched class n=%d N=%d: field %d, tau %.3g" % (cls[0], cls[1], field, m.tau))
    base = [m2.field().astype(np.float32) for m2 in _BW.members]
    start = m.field()
    for step in (1, 2):
        A32 = start.astype(np.float32)
        A64 = A32.astype(np.float64)
        fields = list(base)
        fields[field] = A32
        flat = bp.pack([torch.tensor(f, dtype=torch.float32, device="cuda") for f in fields])
        Hg = bp.unpack(bp.diffuse(flat))[field].cpu().numpy().reshape(A64.shape)
        Ht, _ = oracle.heat(A64.reshape((m.n * m.n,) + m.grid), m.tau, 2)
        Ht = Ht.reshape(A64.shape)
        e_heat = float(np.abs(Hg - Ht).max())
        r = bp.iterate(flat, 1)
        out = bp.unpack(flat)[field].cpu().numpy().reshape(A64.shape)
        ro = oracle.iterate(A64, m.tau, 1)
        Hp = _pm(Ht)
        s = np.linalg.svd(Hp, compute_uv=False)
        gap = s[:, -2] + s[:, -1]
        err = np.abs(_pm(out - ro["A"])).max(axis=(1, 2))
        # det-sign ties: where the FP32 and FP64 runs land in different components
        # of O(n) the diffused matrix must be within what the FP32 diffusion error
        # can move det across zero, |d det| <= |cof H|_F |dH|_F, doubled (the plan
        # is plain FP32: such points get no double re-projection)
        cof = np.sqrt(sum(np.prod(np.delete(s, i, axis=1), axis=1) ** 2 for i in range(m.n)))
        tie_bound = 2.0 * m.n * (e_heat + 8 * 2.0 ** -24) * cof
        mism = (np.linalg.det(_pm(out)) >= 0) != (np.linalg.det(_pm(ro["A"])) >= 0)
        note("  step %d: diffusion err %.3g, step err max %.3g (%.3g off the %d det-sign ties), "
             "well-conditioned %d pts max %.3g" % (
                 step, e_heat, err.max(), err[~mism].max(), int(mism.sum()), int((gap >= 0.1).sum()),
                 err[gap >= 0.1].max() if (gap >= 0.1).any() else 0))
        assert e_heat <= 2e-6
        assert np.all(np.abs(np.linalg.det(Hp[mism])) <= tie_bound[mism])
        assert _fp32_step_ok(err[~mism], gap[~mism], e_heat)
        assert abs(r["energy"][field][1] - ro["energy"][1]) <= 1e-5 * abs(ro["energy"][1])
        start = ro["A"]


BANDED_3D_MIXED = [((64, 64, 128), 3, 5e-4, "normal"), ((64, 64, 128), 3, 1e-3, "uniform"),
                   ((128, 64, 32), 2, 5e-4, "uniform"), ((64, 128, 64), 4, 8e-4, "normal")]


def test_batched_3d_plane_pass_against_oracle(torch_cuda):
    """Float 3-D fields in one batched plan run the band-limited passes (x-row
    pass, plane pass), two of them in one class with their own tau (the symbols
    per field, the band the widest of the class).  Two steps of every field, each
    from the same float input as the FP64 oracle's step (the second from the
    plan's own first iterate, a smooth field): per point within the FP32 bound,
    det-sign differences only at ties, and the step's logged energy within FP32
    rounding of the oracle's."""
    torch = torch_cuda
    from paper_1711_01365_amd import mbo
    spec = [(g, n, t) for g, n, t, _ in BANDED_3D_MIXED]
    bp = mbo.BatchedPlan(spec, precision=FB, autotune=False)
    paths = [bp.path(i) for i in range(len(spec))]
    note("3-D batched paths (path, half-width, stored modes): %s" % paths)
    assert all(p[0] in (mbo.PATH_BANDED, mbo.PATH_FULL) for p in paths)
    assert paths[0][0] == paths[1][0] == mbo.PATH_BANDED  # the class of two taus keeps a band
    fields = [gen(init, n, grid, 700 + i).astype(np.float32)
              for i, (grid, n, tau, init) in enumerate(BANDED_3D_MIXED)]
    for step in (1, 2):
        flat = bp.pack([torch.tensor(f, device="cuda") for f in fields])
        H = [h.cpu().numpy() for h in bp.unpack(bp.diffuse(flat))]
        r = bp.iterate(flat, 1)
        outs = [o.cpu().numpy() for o in bp.unpack(flat)]
        for i, (grid, n, tau, _) in enumerate(BANDED_3D_MIXED):
            A64 = fields[i].astype(np.float64)
            Ht, _ = oracle.heat(A64.reshape((n * n,) + grid), tau, 3)
            Ht = Ht.reshape(A64.shape)
            e_heat = float(np.abs(H[i].reshape(A64.shape) - Ht).max())
            ro = oracle.iterate(A64, tau, 1)
            out = outs[i].reshape(A64.shape)
            Hp = _pm(Ht)
            s = np.linalg.svd(Hp, compute_uv=False)
            gap = s[:, -2] + s[:, -1] if n > 1 else 2 * np.abs(Hp.reshape(-1))
            err = np.abs(_pm(out - ro["A"])).max(axis=(1, 2))
            cof = np.sqrt(sum(np.prod(np.delete(s, j, axis=1), axis=1) ** 2 for j in range(n)))
            tie_bound = 2.0 * n * (e_heat + 8 * 2.0 ** -24) * cof
            mism = (np.linalg.det(_pm(out)) >= 0) != (np.linalg.det(_pm(ro["A"])) >= 0)
            note("3-D batched step %d field %d grid=%s n=%d tau=%g: diffusion err %.3g, step err max %.3g "
                 "(%.3g off the %d det-sign ties), %d well conditioned"
                 % (step, i, grid, n, tau, e_heat, err.max(), err[~mism].max(), int(mism.sum()),
                    int((gap >= 0.1).sum())))
            assert e_heat <= 2e-6
            assert np.all(np.abs(np.linalg.det(Hp[mism])) <= tie_bound[mism])
            assert _fp32_step_ok(err[~mism], gap[~mism], e_heat)
            assert abs(r["energy"][i][0] - ro["energy"][0]) <= 1e-5 * abs(ro["energy"][0])
            fields[i] = out.astype(np.float32)
    bp.close()
