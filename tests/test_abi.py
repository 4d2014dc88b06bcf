"""The C ABI library loads on a host without a GPU, exports every function that
include/mbo.h declares, and rejects invalid arguments with status codes before
touching the device."""
import ctypes
import os
import re

import pytest

from paper_1711_01365_amd import mbo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mbo.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mbo_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mbo.LIB_PATH):
        pytest.skip("libmbo.so not built")
    return mbo.load()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for f in ("mbo_plan", "mbo_diffuse", "mbo_project", "mbo_iterate", "mbo_energy"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(mbo.EXPORTS) == set(declared_functions())


def test_status_strings(lib):
    for code, name in mbo._STATUS.items():
        assert mbo.status_string(code) == name


def _plan(lib, d=2, N=(64, 64), n=2, batch=1, tau=1e-3, prec=0, out=True):
    h = ctypes.c_void_p()
    arr = (ctypes.c_int64 * len(N))(*N)
    return lib.mbo_plan(ctypes.byref(h) if out else None, d, arr, n, batch, tau, prec, 0.0, None), h


@pytest.mark.parametrize("kw,code", [
    (dict(out=False), 1),
    (dict(d=1, N=(64,)), 1),
    (dict(d=4, N=(8, 8, 8, 8)), 1),
    (dict(n=0), 1), (dict(n=5), 1),
    (dict(batch=0), 1),
    (dict(tau=0.0), 1), (dict(tau=-1.0), 1), (dict(tau=float("nan")), 1), (dict(tau=float("inf")), 1),
    (dict(prec=7), 1),
    (dict(N=(64, 48)), 2), (dict(N=(4, 64)), 2), (dict(N=(64, 4096)), 2),
    (dict(d=3, N=(8, 8, 12)), 2),
])
def test_plan_validation_codes(lib, kw, code):
    rc, h = _plan(lib, **kw)
    assert rc == code
    assert h.value is None
    assert lib.mbo_last_error(None)  # a message is recorded


@pytest.mark.parametrize("kw,code,msg", [
    (dict(prec=7), 1, "precision"), (dict(n=0), 1, "n = 0"), (dict(n=5), 1, "n = 5"),
    (dict(tau=0.0), 1, "tau"), (dict(tau=float("nan")), 1, "tau"),
    (dict(a=None), 1, "NULL"), (dict(b=None), 1, "NULL"), (dict(b=0x1000), 1, "alias"),
    (dict(N0=96), 2, "power of two"), (dict(N1=4), 2, "power of two"), (dict(N1=4096), 2, "power of two"),
])
def test_step_static_validation_codes(lib, kw, code, msg):
    """mbo_step_static checks its arguments before it touches the device, and
    mbo_last_error(NULL) names the failure (a fixed buffer: the call allocates
    nothing); a later failed mbo_plan takes over mbo_last_error(NULL)."""
    a = dict(N0=64, N1=64, n=3, prec=2, tau=1e-3, a=0x1000, b=0x2000)
    a.update(kw)
    rc = lib.mbo_step_static(a["N0"], a["N1"], a["n"], a["prec"], a["tau"], 0.0, a["a"], a["b"], None)
    assert rc == code
    assert msg in lib.mbo_last_error(None).decode()
    rc, _ = _plan(lib, n=0)
    assert rc == 1 and b"n" in lib.mbo_last_error(None)


def test_null_plan_is_rejected(lib):
    assert lib.mbo_diffuse(None, None, None) == 1
    assert lib.mbo_project(None, None, None, None) == 1
    assert lib.mbo_energy(None, None, None) == 1
    assert lib.mbo_iterate(None, None, 1, 0.0, None, None, None, None, None) == 1
    assert lib.mbo_plan_set_tau(None, 1.0) == 1
    assert lib.mbo_plan_destroy(None) == 0


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        mbo.Plan((64, 64), 2, 1e-3)


def _batched(lib, descs, prec=2, count=None, out=True):
    arr = (mbo.FieldDesc * max(len(descs), 1))()
    for i, (d, N, n, tau) in enumerate(descs):
        arr[i].d = d
        for a in range(3):
            arr[i].N[a] = N[a] if a < len(N) else 1
        arr[i].n = n
        arr[i].tau = tau
    h = ctypes.c_void_p()
    rc = lib.mbo_plan_batched(ctypes.byref(h) if out else None, len(descs) if count is None else count,
                              arr, prec, 0.0, 0, None)
    return rc, h


@pytest.mark.parametrize("descs,kw,code", [
    ([(2, (64, 64), 2, 1e-3)], dict(out=False), 1),
    ([(2, (64, 64), 2, 1e-3)], dict(count=0), 1),
    ([(2, (64, 64), 2, 1e-3)], dict(prec=9), 1),
    ([(2, (64, 64), 2, 1e-3), (2, (32, 32), 5, 1e-3)], {}, 1),
    ([(2, (64, 64), 2, 1e-3), (2, (32, 32), 3, 0.0)], {}, 1),
    ([(2, (64, 64), 2, 1e-3), (1, (32,), 3, 1e-3)], {}, 1),
    ([(2, (64, 64), 2, 1e-3), (2, (32, 24), 3, 1e-3)], {}, 2),
    ([(3, (16, 16, 4096), 2, 1e-3)], {}, 2),
])
def test_batched_plan_validation_codes(lib, descs, kw, code):
    rc, h = _batched(lib, descs, **kw)
    assert rc == code
    assert h.value is None
    assert lib.mbo_last_error(None)


def test_batched_desc_layout():
    """mbo_field_desc as the C compiler lays it out: int, int64_t[3], int, double."""
    assert ctypes.sizeof(mbo.FieldDesc) == 48
    assert mbo.FieldDesc.N.offset == 8 and mbo.FieldDesc.n.offset == 32 and mbo.FieldDesc.tau.offset == 40


def test_null_plan_is_rejected_by_new_calls(lib):
    assert lib.mbo_plan_tuning(None, 0, None, None, None, None) == 1
    assert lib.mbo_plan_autotune(None) == 1
    assert lib.mbo_project_vjp(None, None, None, None) == 1
    assert lib.mbo_diffuse_dtau(None, None, None, None, None) == 1


def test_null_plan_is_rejected_by_volume_calls(lib):
    assert lib.mbo_volume_select(None, None, None, None) == 1
    assert lib.mbo_project_volume(None, None, None, None, None) == 1
    assert lib.mbo_iterate_volume(None, None, 1, None, None, None, None, None) == 1


def test_null_plan_is_rejected_by_the_index(lib):
    assert lib.mbo_so2_index(None, None, None, None) == 1


def test_null_plan_is_rejected_by_the_relaxed_flows(lib):
    assert lib.mbo_relaxed_flow(None, None, 1, 1, 0.1, 1e-3) == 1
    assert lib.mbo_relaxed_energy(None, None, 1, 0.1, None) == 1


def test_surface_calls_validate_before_touching_the_device(lib):
    assert lib.mbo_surface_info(None, None, None, None, None) == 1
    assert lib.mbo_surface_points(None, None, None, None) == 1
    assert lib.mbo_surface_diffuse(None, None, None) == 1
    assert lib.mbo_surface_iterate(None, None, 1, None) == 1
    assert lib.mbo_surface_destroy(None) == 0
    assert lib.mbo_surface_volume_weights(None, None) == 1
    assert lib.mbo_surface_volume_select(None, None, 1, None) == 1
    assert lib.mbo_surface_iterate_volume(None, None, 1, None, None, None) == 1
    h = ctypes.c_void_p()
    assert lib.mbo_surface_sphere(None, 1.0, 0.1, 1, 0.01, 1e-6, 3, 0, None) == 1
    for bad in [(-1.0, 0.1, 1, 0.01, 1e-6, 3, 0), (1.0, 0.0, 1, 0.01, 1e-6, 3, 0),
                (1.0, 0.1, 0, 0.01, 1e-6, 3, 0), (1.0, 0.1, 9, 0.01, 1e-6, 3, 0),
                (1.0, 0.1, 1, 0.0, 1e-6, 3, 0), (1.0, 0.1, 1, float("nan"), 1e-6, 3, 0),
                (1.0, 0.1, 1, 0.01, 0.0, 3, 0), (1.0, 0.1, 1, 0.01, 0.6, 3, 0),
                (1.0, 0.1, 1, 0.01, 1e-6, 0, 0), (1.0, 0.1, 1, 0.01, 1e-6, 5, 0),
                (1.0, 0.1, 1, 0.01, 1e-6, 3, 7)]:
        assert lib.mbo_surface_sphere(ctypes.byref(h), *bad, None) == 1, bad
        assert not h.value
        assert lib.mbo_surface_last_error(None)
    # a grid finer than 512 points per axis is refused before any device work
    assert lib.mbo_surface_sphere(ctypes.byref(h), 10.0, 0.5, 1, 1e-3, 1e-6, 3, 0, None) == 2
    assert b"512" in lib.mbo_surface_last_error(None)
    # a lattice too fine to scan is refused before any work
    assert lib.mbo_surface_sphere(ctypes.byref(h), 1.0, 1e-4, 1, 0.01, 1e-6, 3, 0, None) == 2
    assert b"too small" in lib.mbo_surface_last_error(None)


def test_peanut_surface_validates_before_touching_the_device(lib):
    h = ctypes.c_void_p()
    assert lib.mbo_surface_peanut(None, 0.1, 1, 0.01, 1e-6, 3, 0, None) == 1
    for bad in [(0.0, 1, 0.01, 1e-6, 3, 0), (0.1, 0, 0.01, 1e-6, 3, 0), (0.1, 1, -1.0, 1e-6, 3, 0),
                (0.1, 1, 0.01, 0.7, 3, 0), (0.1, 1, 0.01, 1e-6, 0, 0), (0.1, 1, 0.01, 1e-6, 3, 9)]:
        assert lib.mbo_surface_peanut(ctypes.byref(h), *bad, None) == 1, bad
        assert not h.value
    assert lib.mbo_surface_peanut(ctypes.byref(h), 1e-4, 1, 0.01, 1e-6, 3, 0, None) == 2
    assert b"too small" in lib.mbo_surface_last_error(None)
