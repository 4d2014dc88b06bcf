"""ctypes binding of libmbo (include/mbo.h): same call names, argument marshalling only.

Every step of the method runs in the HIP kernels of ``libmbo.so``; PyTorch only
provides device memory and the current stream.  There is no fallback: if the
library is missing or no GPU is present the calls raise.

Field tensors are ``(batch, n, n, *grid)`` (or ``(n, n, *grid)`` for batch 1),
contiguous, on the plan's device, float64 for ``F64`` plans and float32
otherwise -- the entry-planar layout of the C ABI.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmbo.so")

F64, F32, F32_F64FALLBACK = 0, 1, 2
GD1, GD3 = 1, 3
PATH_GENERIC, PATH_FULL, PATH_BANDED = 0, 1, 2
_STATUS = {0: "MBO_OK", 1: "MBO_ERR_INVALID_ARG", 2: "MBO_ERR_UNSUPPORTED", 3: "MBO_ERR_ALLOC",
           4: "MBO_ERR_HIP", 5: "MBO_ERR_NONFINITE", 6: "MBO_ERR_SCRATCH"}
STEP_STATIC_MAX_BYTES = 64 << 20

_lib = None

EXPORTS = ("mbo_plan", "mbo_plan_destroy", "mbo_plan_set_tau", "mbo_plan_set_stream",
           "mbo_plan_set_timing", "mbo_last_timing", "mbo_diffuse", "mbo_project", "mbo_iterate",
           "mbo_energy", "mbo_project_vjp", "mbo_diffuse_dtau", "mbo_plan_batched", "mbo_plan_tuning",
           "mbo_plan_autotune", "mbo_step", "mbo_step_vjp", "mbo_volume_select",
           "mbo_project_volume", "mbo_iterate_volume", "mbo_so2_index", "mbo_relaxed_flow",
           "mbo_relaxed_energy", "mbo_surface_sphere", "mbo_surface_peanut", "mbo_surface_destroy",
           "mbo_surface_info",
           "mbo_surface_points", "mbo_surface_diffuse", "mbo_surface_iterate", "mbo_surface_last_error",
           "mbo_surface_volume_weights", "mbo_surface_volume_select", "mbo_surface_iterate_volume",
           "mbo_plan_set_path", "mbo_plan_path", "mbo_last_project_counts", "mbo_step_static", "mbo_status_string",
           "mbo_last_error")


class FieldDesc(ctypes.Structure):
    """mbo_field_desc: one field of a batched plan."""
    _fields_ = [("d", ctypes.c_int), ("N", ctypes.c_int64 * 3), ("n", ctypes.c_int),
                ("tau", ctypes.c_double)]


class MboError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


def load(path: str = LIB_PATH):
    """Load libmbo.so and declare the C signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libmbo.so is not built (run `python -m paper_1711_01365_amd.build`)")
    lib = ctypes.CDLL(path)
    vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    lib.mbo_plan.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int64,
                             ctypes.c_double, ctypes.c_int, ctypes.c_double, vp]
    lib.mbo_plan_destroy.argtypes = [vp]
    lib.mbo_plan_set_tau.argtypes = [vp, ctypes.c_double]
    lib.mbo_plan_set_stream.argtypes = [vp, vp]
    lib.mbo_plan_set_timing.argtypes = [vp, ctypes.c_int]
    lib.mbo_last_timing.argtypes = [vp, dp, dp, ip]
    lib.mbo_diffuse.argtypes = [vp, vp, vp]
    lib.mbo_project.argtypes = [vp, vp, vp, vp]
    lib.mbo_iterate.argtypes = [vp, vp, ctypes.c_int, ctypes.c_double, ip, dp, i64p, dp, i64p]
    lib.mbo_energy.argtypes = [vp, vp, dp]
    lib.mbo_project_vjp.argtypes = [vp, vp, vp, vp]
    lib.mbo_diffuse_dtau.argtypes = [vp, vp, vp, vp, dp]
    lib.mbo_plan_batched.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(FieldDesc),
                                     ctypes.c_int, ctypes.c_double, ctypes.c_int, vp]
    lib.mbo_plan_tuning.argtypes = [vp, ctypes.c_int, ip, ip, ip, ip]
    lib.mbo_plan_set_path.argtypes = [vp, ctypes.c_int]
    lib.mbo_last_project_counts.argtypes = [vp, i64p, i64p]
    lib.mbo_plan_path.argtypes = [vp, ctypes.c_int, ip, ip, ip]
    lib.mbo_plan_autotune.argtypes = [vp]
    lib.mbo_step.argtypes = [vp, vp, vp]
    lib.mbo_step_static.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, vp, vp, vp]
    lib.mbo_step_vjp.argtypes = [vp, vp, vp, vp]
    lib.mbo_volume_select.argtypes = [vp, vp, i64p, vp]
    lib.mbo_project_volume.argtypes = [vp, vp, vp, i64p, vp]
    lib.mbo_iterate_volume.argtypes = [vp, vp, ctypes.c_int, i64p, i64p, dp, i64p, i64p]
    lib.mbo_so2_index.argtypes = [vp, vp, dp, dp]
    lib.mbo_relaxed_flow.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    lib.mbo_relaxed_energy.argtypes = [vp, vp, ctypes.c_int, ctypes.c_double, dp]
    lib.mbo_surface_sphere.argtypes = [ctypes.POINTER(vp), ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, vp]
    lib.mbo_surface_peanut.argtypes = [ctypes.POINTER(vp), ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int, ctypes.c_int, vp]
    lib.mbo_surface_destroy.argtypes = [vp]
    lib.mbo_surface_info.argtypes = [vp, i64p, i64p, ip, dp]
    lib.mbo_surface_points.argtypes = [vp, dp, dp, dp]
    lib.mbo_surface_diffuse.argtypes = [vp, vp, vp]
    lib.mbo_surface_iterate.argtypes = [vp, vp, ctypes.c_int, i64p]
    lib.mbo_surface_volume_weights.argtypes = [vp, i64p]
    lib.mbo_surface_volume_select.argtypes = [vp, vp, ctypes.c_int64, vp]
    lib.mbo_surface_iterate_volume.argtypes = [vp, vp, ctypes.c_int, i64p, i64p, i64p]
    lib.mbo_surface_last_error.argtypes = [vp]
    lib.mbo_surface_last_error.restype = ctypes.c_char_p
    for f in EXPORTS:
        if f not in ("mbo_status_string", "mbo_last_error", "mbo_surface_last_error"):
            getattr(lib, f).restype = ctypes.c_int
    lib.mbo_status_string.argtypes = [ctypes.c_int]
    lib.mbo_status_string.restype = ctypes.c_char_p
    lib.mbo_last_error.argtypes = [vp]
    lib.mbo_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int, handle) -> None:
    if rc != 0:
        msg = _lib.mbo_last_error(handle)
        raise MboError(rc, msg.decode() if msg else "")


def _stream_ptr(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Plan:
    """Owns an ``mbo_plan_t``.  Mirrors the C entry points one to one."""

    def __init__(self, grid: Sequence[int], n: int, tau: float, precision: int = F64,
                 batch: int = 1, sigma_fallback: float = 1e-3, stream=None):
        lib = load()
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: libmbo runs on the GPU only")
        self.grid = tuple(int(g) for g in grid)
        self.n, self.batch, self.precision = int(n), int(batch), int(precision)
        self.tau = float(tau)
        self.dtype = torch.float64 if precision == F64 else torch.float32
        N = (ctypes.c_int64 * len(self.grid))(*self.grid)
        h = ctypes.c_void_p()
        rc = lib.mbo_plan(ctypes.byref(h), len(self.grid), N, self.n, self.batch, self.tau,
                          self.precision, float(sigma_fallback), _stream_ptr(stream))
        _check(rc, None)
        self._h = h
        self._lib = lib

    # -- helpers -------------------------------------------------------------
    @property
    def shape(self):
        return (self.batch, self.n, self.n) + self.grid

    def _field(self, A, name="A"):
        import torch
        if not isinstance(A, torch.Tensor) or not A.is_cuda:
            raise TypeError("%s must be a CUDA/HIP tensor" % name)
        if A.dtype != self.dtype:
            raise TypeError("%s must be %s" % (name, self.dtype))
        if tuple(A.shape) not in (self.shape, self.shape[1:] if self.batch == 1 else None):
            raise ValueError("%s has shape %s, plan expects %s" % (name, tuple(A.shape), self.shape))
        if not A.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        return ctypes.c_void_p(A.data_ptr())

    def set_stream(self, stream=None):
        _check(self._lib.mbo_plan_set_stream(self._h, _stream_ptr(stream)), self._h)

    def set_timing(self, enable: bool = True):
        _check(self._lib.mbo_plan_set_timing(self._h, int(bool(enable))), self._h)

    def last_timing(self):
        """(row pass us, heat pass us, iterations averaged) of the last timed iterate."""
        r, c, k = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        _check(self._lib.mbo_last_timing(self._h, ctypes.byref(r), ctypes.byref(c), ctypes.byref(k)),
               self._h)
        return r.value, c.value, k.value

    def set_tau(self, tau: float):
        _check(self._lib.mbo_plan_set_tau(self._h, float(tau)), self._h)
        self.tau = float(tau)

    # -- entry points ----------------------------------------------------------
    def diffuse(self, A_in, A_out=None):
        import torch
        if A_out is None:
            A_out = torch.empty_like(A_in)
        _check(self._lib.mbo_diffuse(self._h, self._field(A_in, "A_in"), self._field(A_out, "A_out")),
               self._h)
        return A_out

    def project(self, A_in, A_out=None, det_sign: bool = False):
        import torch
        if A_out is None:
            A_out = torch.empty_like(A_in)
        ds = None
        if det_sign:
            ds = torch.empty((self.batch,) + self.grid, dtype=torch.int8, device=A_in.device)
        _check(self._lib.mbo_project(self._h, self._field(A_in, "A_in"), self._field(A_out, "A_out"),
                                     ctypes.c_void_p(ds.data_ptr()) if ds is not None else None),
               self._h)
        return (A_out, ds) if det_sign else A_out

    def last_project_counts(self):
        """(points re-projected in double, points with NaN/Inf input) of the last project()."""
        fb, bad = np.zeros(1, dtype=np.int64), np.zeros(1, dtype=np.int64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        _check(self._lib.mbo_last_project_counts(self._h, fb.ctypes.data_as(i64p), bad.ctypes.data_as(i64p)),
               self._h)
        return int(fb[0]), int(bad[0])

    def step(self, A_prev, A_next=None):
        """A_next = P(e^{tau Delta} A_prev), asynchronous (no logs, no NaN check)."""
        import torch
        if A_next is None:
            A_next = torch.empty_like(A_prev)
        _check(self._lib.mbo_step(self._h, self._field(A_prev, "A_prev"), self._field(A_next, "A_next")),
               self._h)
        return A_next

    def step_vjp(self, A_prev, G, dtau=None):
        """In place G <- cotangent of A_prev from G = cotangent of P(e^{tau Delta} A_prev);
        dtau (device float64 [batch] tensor, optional) += the step's tau-derivative term."""
        import torch
        if dtau is not None and (dtau.dtype != torch.float64 or not dtau.is_cuda or dtau.numel() != self.batch):
            raise ValueError("dtau must be a float64 device tensor of %d values" % self.batch)
        _check(self._lib.mbo_step_vjp(self._h, self._field(A_prev, "A_prev"), self._field(G, "G"),
                                      ctypes.c_void_p(dtau.data_ptr()) if dtau is not None else None),
               self._h)
        return G

    def project_vjp(self, A_tilde, G_Q, G_A=None):
        """Cotangent of the projection's input for the cotangent G_Q of its output."""
        import torch
        if G_A is None:
            G_A = torch.empty_like(G_Q)
        _check(self._lib.mbo_project_vjp(self._h, self._field(A_tilde, "A_tilde"),
                                         self._field(G_Q, "G_Q"), self._field(G_A, "G_A")), self._h)
        return G_A

    def diffuse_dtau(self, A, out=None, G=None):
        """d/dtau e^{tau Delta} A into `out` (allocated when neither out nor G is
        given); with G also returns <G, d/dtau e^{tau Delta} A> per field.
        Returns out, dot or (out, dot)."""
        import torch
        if out is None and G is None:
            out = torch.empty_like(A)
        dot = np.zeros(self.batch) if G is not None else None
        _check(self._lib.mbo_diffuse_dtau(
            self._h, self._field(A), self._field(out, "out") if out is not None else None,
            self._field(G, "G") if G is not None else None,
            dot.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if dot is not None else None),
            self._h)
        if dot is not None:
            d = dot if self.batch > 1 else float(dot[0])
            return (out, d) if out is not None else d
        return out

    def energy(self, A):
        E = np.zeros(self.batch)
        _check(self._lib.mbo_energy(self._h, self._field(A),
                                    E.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self._h)
        return E if self.batch > 1 else float(E[0])

    def iterate(self, A, max_iter: int, tol: float = 0.0, logs: bool = True):
        """In-place Algorithm 1 on A.  Returns a dict of numpy logs (per field)."""
        B, K = self.batch, int(max_iter)
        it = np.zeros(B, dtype=np.int32)
        en = np.zeros((B, K + 1)) if logs else None
        fl = np.zeros((B, max(K, 1)), dtype=np.int64) if logs else None
        dl = np.zeros((B, max(K, 1))) if logs else None
        fb = np.zeros((B, max(K, 1)), dtype=np.int64) if logs else None
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)

        def ptr(x, t):
            return None if x is None else x.ctypes.data_as(t)

        rc = self._lib.mbo_iterate(self._h, self._field(A), K, float(tol),
                                   it.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                   ptr(en, dp), ptr(fl, ip), ptr(dl, dp), ptr(fb, ip))
        _check(rc, self._h)
        out = {"iters": it}
        if logs:
            out.update(energy=en, flips=fl[:, :K], delta=dl[:, :K], fallbacks=fb[:, :K])
        return out

    # -- volume-preserving MBO (Section 7) -------------------------------------
    def _nplus(self, n_plus):
        v = np.ascontiguousarray(np.broadcast_to(np.asarray(n_plus, dtype=np.int64), (self.batch,)))
        return v, v.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))

    def volume_select(self, dE, n_plus):
        """uint8 mask (batch, *grid): the n_plus largest dE per field (ties by index)."""
        import torch
        if not isinstance(dE, torch.Tensor) or not dE.is_cuda or dE.dtype != self.dtype \
                or not dE.is_contiguous() or dE.numel() != self.batch * int(np.prod(self.grid)):
            raise ValueError("dE must be a contiguous %s device tensor of batch * prod(grid) values"
                             % self.dtype)
        mask = torch.empty((self.batch,) + self.grid, dtype=torch.uint8, device=dE.device)
        v, vp_ = self._nplus(n_plus)
        _check(self._lib.mbo_volume_select(self._h, ctypes.c_void_p(dE.data_ptr()), vp_,
                                           ctypes.c_void_p(mask.data_ptr())), self._h)
        return mask

    def project_volume(self, A_in, n_plus, A_out=None, want_dE: bool = False):
        """Volume-constrained step 2: T+ on the n_plus points of largest Delta E,
        T- elsewhere.  Returns A_out, or (A_out, dE) with want_dE."""
        import torch
        if A_out is None:
            A_out = torch.empty_like(A_in)
        dE = torch.empty((self.batch,) + self.grid, dtype=self.dtype, device=A_in.device) \
            if want_dE else None
        v, vp_ = self._nplus(n_plus)
        _check(self._lib.mbo_project_volume(self._h, self._field(A_in, "A_in"),
                                            self._field(A_out, "A_out"), vp_,
                                            ctypes.c_void_p(dE.data_ptr()) if dE is not None else None),
               self._h)
        return (A_out, dE) if want_dE else A_out

    def iterate_volume(self, A, max_iter: int, n_plus=None, logs: bool = True):
        """In-place volume-preserving MBO on A.  n_plus None: #{det A_0 >= 0} per field.
        Returns a dict of numpy logs (per field)."""
        B, K = self.batch, int(max_iter)
        used = np.zeros(B, dtype=np.int64)
        en = np.zeros((B, K + 1)) if logs else None
        fl = np.zeros((B, max(K, 1)), dtype=np.int64) if logs else None
        fb = np.zeros((B, max(K, 1)), dtype=np.int64) if logs else None
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)

        def ptr(x, t):
            return None if x is None else x.ctypes.data_as(t)

        npv = None
        if n_plus is not None:
            npv, _ = self._nplus(n_plus)
        rc = self._lib.mbo_iterate_volume(self._h, self._field(A), K, ptr(npv, ip), ptr(used, ip),
                                          ptr(en, dp), ptr(fl, ip), ptr(fb, ip))
        _check(rc, self._h)
        out = {"n_plus": used}
        if logs:
            out.update(energy=en, flips=fl[:, :K], fallbacks=fb[:, :K])
        return out

    # -- relaxed gradient flows GD-1 / GD-3 -------------------------------------
    def relaxed_flow(self, A, steps: int, kind: int, eps: float, dt: float):
        """In place: `steps` steps of GD-1 (kind GD1) or GD-3 (GD3), each an
        implicit diffusion step then an explicit reaction step."""
        _check(self._lib.mbo_relaxed_flow(self._h, self._field(A), int(steps), int(kind), float(eps),
                                          float(dt)), self._h)
        return A

    def relaxed_energy(self, A, kind: int, eps: float):
        """E_{1,eps} (GD1) or E_{2,eps} (GD3) per field."""
        E = np.zeros(self.batch)
        _check(self._lib.mbo_relaxed_energy(self._h, self._field(A), int(kind), float(eps),
                                            E.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self._h)
        return E if self.batch > 1 else float(E[0])

    def so2_index(self, A):
        """Section 6.1 index of the first-column field of an n = 2 field along the
        loops in x (one per column) and in y (one per row): (w_x [batch, N1],
        w_y [batch, N0]) as float64 numpy arrays."""
        w_x = np.zeros((self.batch, self.grid[1]))
        w_y = np.zeros((self.batch, self.grid[0]))
        dp = ctypes.POINTER(ctypes.c_double)
        _check(self._lib.mbo_so2_index(self._h, self._field(A), w_x.ctypes.data_as(dp),
                                       w_y.ctypes.data_as(dp)), self._h)
        return w_x, w_y

    def autotune(self):
        """Time candidate launch shapes on the device and keep the fastest."""
        _check(self._lib.mbo_plan_autotune(self._h), self._h)
        return self.tuning(0)

    def tuning(self, field: int = 0):
        """(rows per row-pass workgroup, its threads, lines per heat-pass workgroup,
        XCD tile order)."""
        r, n, t, x = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self._lib.mbo_plan_tuning(self._h, int(field), ctypes.byref(r), ctypes.byref(n),
                                         ctypes.byref(t), ctypes.byref(x)), self._h)
        return r.value, n.value, t.value, x.value

    def set_path(self, path: int):
        """Kernels of iterate(): PATH_BANDED (default), PATH_FULL or PATH_GENERIC."""
        _check(self._lib.mbo_plan_set_path(self._h, int(path)), self._h)

    def path(self, field: int = 0):
        """(path in effect, kept half-width along the last axis, modes stored per row)."""
        p, c, w = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self._lib.mbo_plan_path(self._h, int(field), ctypes.byref(p), ctypes.byref(c),
                                       ctypes.byref(w)), self._h)
        return p.value, c.value, w.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mbo_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def step_static(A_prev, A_next, tau: float, precision: int = F32_F64FALLBACK, sigma_fallback: float = 0.0,
                stream=None):
    """mbo_step_static: one step A_next = P(e^{tau Delta} A_prev) of one 2-D field
    (device tensors of shape (n, n, N0, N1)) with no plan and no device
    allocation; asynchronous on `stream`."""
    import torch
    lib = load()
    want = torch.float64 if precision == F64 else torch.float32
    for name, A in (("A_prev", A_prev), ("A_next", A_next)):
        if not isinstance(A, torch.Tensor) or not A.is_cuda:
            raise TypeError("%s must be a CUDA/HIP tensor" % name)
        if A.dtype != want:
            raise TypeError("%s must be %s" % (name, want))
        if A.dim() != 4 or A.shape[0] != A.shape[1] or not A.is_contiguous():
            raise ValueError("%s must be a contiguous (n, n, N0, N1) tensor" % name)
    if tuple(A_prev.shape) != tuple(A_next.shape):
        raise ValueError("A_prev and A_next differ in shape")
    n, _, N0, N1 = (int(v) for v in A_prev.shape)
    _check(lib.mbo_step_static(N0, N1, n, int(precision), float(tau), float(sigma_fallback),
                               ctypes.c_void_p(A_prev.data_ptr()), ctypes.c_void_p(A_next.data_ptr()),
                               _stream_ptr(stream)), None)
    return A_next


class SphereSurface:
    """Owns an ``mbo_surface_t`` (mbo_surface_sphere): closest-point diffusion
    and the MBO iteration on the sphere of radius R.  Fields are ``(n, n, m)``
    tensors over the m samples (canonical order), float64 for ``F64`` surfaces
    and float32 otherwise."""

    def __init__(self, R: float, dx: float, p: int, tau: float, eps: float, n: int,
                 precision: int = F64, stream=None):
        lib = load()
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: libmbo runs on the GPU only")
        h = ctypes.c_void_p()
        rc = self._create(lib, h, float(R), float(dx), int(p), float(tau), float(eps), int(n), int(precision),
                          _stream_ptr(stream))
        if rc != 0:
            msg = lib.mbo_surface_last_error(None)
            raise MboError(rc, msg.decode() if msg else "")
        self._h, self._lib = h, lib
        self.R, self.dx, self.p, self.tau, self.eps = float(R), float(dx), int(p), float(tau), float(eps)
        self.n, self.precision = int(n), int(precision)
        self.dtype = torch.float64 if precision == F64 else torch.float32
        m, cells, g, wb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int(), ctypes.c_double()
        self._check(lib.mbo_surface_info(h, ctypes.byref(m), ctypes.byref(cells), ctypes.byref(g),
                                         ctypes.byref(wb)))
        self.m, self.cells, self.grid, self.band_width = m.value, cells.value, g.value, wb.value

    @staticmethod
    def _create(lib, h, R, dx, p, tau, eps, n, precision, stream):
        return lib.mbo_surface_sphere(ctypes.byref(h), R, dx, p, tau, eps, n, precision, stream)

    def _check(self, rc):
        if rc != 0:
            msg = self._lib.mbo_surface_last_error(self._h)
            raise MboError(rc, msg.decode() if msg else "")

    @property
    def shape(self):
        return (self.n, self.n, self.m)

    def _field(self, A, name="A"):
        import torch
        if not isinstance(A, torch.Tensor) or not A.is_cuda:
            raise TypeError("%s must be a CUDA/HIP tensor" % name)
        if A.dtype != self.dtype:
            raise TypeError("%s must be %s" % (name, self.dtype))
        if tuple(A.shape) != self.shape:
            raise ValueError("%s has shape %s, surface expects %s" % (name, tuple(A.shape), self.shape))
        if not A.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        return ctypes.c_void_p(A.data_ptr())

    def points(self):
        """(xq [3, m], xc [3, m], w [m]) as float64 numpy arrays."""
        xq, xc, w = np.zeros((3, self.m)), np.zeros((3, self.m)), np.zeros(self.m)
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(self._lib.mbo_surface_points(self._h, xq.ctypes.data_as(dp), xc.ctypes.data_as(dp),
                                                 w.ctypes.data_as(dp)))
        return xq, xc, w

    def diffuse(self, A_in, A_out=None):
        import torch
        if A_out is None:
            A_out = torch.empty_like(A_in)
        self._check(self._lib.mbo_surface_diffuse(self._h, self._field(A_in, "A_in"),
                                                  self._field(A_out, "A_out")))
        return A_out

    def iterate(self, A, K: int, flips: bool = False):
        """K MBO steps in place on A; returns the per-step flip counts (numpy
        int64 [K]) when flips is set, else None."""
        fl = np.zeros(max(int(K), 1), dtype=np.int64) if flips else None
        self._check(self._lib.mbo_surface_iterate(
            self._h, self._field(A), int(K),
            fl.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if fl is not None else None))
        return fl[:K] if fl is not None else None

    def volume_weights(self):
        """Integer volume weights of the samples (numpy int64 [m])."""
        W = np.zeros(self.m, dtype=np.int64)
        self._check(self._lib.mbo_surface_volume_weights(self._h, W.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return W

    def volume_select(self, dE, V: int):
        """uint8 device mask of Algorithm 3's selection for the values dE."""
        import torch
        if not isinstance(dE, torch.Tensor) or not dE.is_cuda or dE.dtype != self.dtype \
                or tuple(dE.shape) != (self.m,) or not dE.is_contiguous():
            raise ValueError("dE must be a contiguous %s device tensor of shape (%d,)" % (self.dtype, self.m))
        sel = torch.empty(self.m, dtype=torch.uint8, device=dE.device)
        self._check(self._lib.mbo_surface_volume_select(self._h, ctypes.c_void_p(dE.data_ptr()), int(V),
                                                        ctypes.c_void_p(sel.data_ptr())))
        return sel

    def iterate_volume(self, A, K: int, V=None, flips: bool = False):
        """K volume-preserving steps in place on A; returns (V used, flips or None)."""
        i64 = ctypes.POINTER(ctypes.c_int64)
        vin = None if V is None else np.array([int(V)], dtype=np.int64)
        vu = np.zeros(1, dtype=np.int64)
        fl = np.zeros(max(int(K), 1), dtype=np.int64) if flips else None
        self._check(self._lib.mbo_surface_iterate_volume(
            self._h, self._field(A), int(K), None if vin is None else vin.ctypes.data_as(i64), vu.ctypes.data_as(i64),
            fl.ctypes.data_as(i64) if fl is not None else None))
        return int(vu[0]), (fl[:K] if fl is not None else None)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mbo_surface_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class PeanutSurface(SphereSurface):
    """Owns an ``mbo_surface_t`` of the peanut (mbo_surface_peanut); the same
    calls as SphereSurface."""

    def __init__(self, dx: float, p: int, tau: float, eps: float, n: int, precision: int = F64, stream=None):
        super().__init__(1.0, dx, p, tau, eps, n, precision, stream)

    @staticmethod
    def _create(lib, h, R, dx, p, tau, eps, n, precision, stream):
        return lib.mbo_surface_peanut(ctypes.byref(h), dx, p, tau, eps, n, precision, stream)


def status_string(code: int) -> str:
    return load().mbo_status_string(code).decode()


class BatchedPlan(Plan):
    """Owns a batched ``mbo_plan_t`` (mbo_plan_batched): independent fields of
    mixed grid, n and tau, iterated together.  Field tensors are flat, the
    concatenation of the fields in order (``pack`` / ``unpack``)."""

    def __init__(self, fields, precision: int = F32, sigma_fallback: float = 1e-3,
                 autotune: bool = True, stream=None):
        lib = load()
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: libmbo runs on the GPU only")
        self.fields = [(tuple(int(g) for g in grid), int(n), float(tau)) for grid, n, tau in fields]
        descs = (FieldDesc * len(self.fields))()
        self.offsets, off = [], 0
        for i, (grid, n, tau) in enumerate(self.fields):
            descs[i].d = len(grid)
            for a in range(3):
                descs[i].N[a] = grid[a] if a < len(grid) else 1
            descs[i].n = n
            descs[i].tau = tau
            self.offsets.append(off)
            off += n * n * int(np.prod(grid))
        self.total = off
        self.batch = len(self.fields)
        self.precision = int(precision)
        self.dtype = torch.float64 if precision == F64 else torch.float32
        h = ctypes.c_void_p()
        rc = lib.mbo_plan_batched(ctypes.byref(h), len(self.fields), descs, self.precision,
                                  float(sigma_fallback), int(bool(autotune)), _stream_ptr(stream))
        _check(rc, None)
        self._h = h
        self._lib = lib

    @property
    def shape(self):
        return (self.total,)

    def _field(self, A, name="A"):
        import torch
        if not isinstance(A, torch.Tensor) or not A.is_cuda:
            raise TypeError("%s must be a CUDA/HIP tensor" % name)
        if A.dtype != self.dtype:
            raise TypeError("%s must be %s" % (name, self.dtype))
        if A.numel() != self.total or not A.is_contiguous():
            raise ValueError("%s must be contiguous with %d elements" % (name, self.total))
        return ctypes.c_void_p(A.data_ptr())

    def pack(self, tensors):
        """Concatenate per-field tensors (n, n, *grid) into one flat device tensor."""
        import torch
        return torch.cat([t.reshape(-1) for t in tensors]).to(self.dtype).contiguous()

    def unpack(self, flat):
        """Views of the fields of a flat tensor, shaped (n, n, *grid)."""
        out = []
        for (grid, n, _), off in zip(self.fields, self.offsets):
            m = n * n * int(np.prod(grid))
            out.append(flat[off:off + m].view((n, n) + grid))
        return out
