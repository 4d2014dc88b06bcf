"""MI355X-native generalized MBO iteration for orthogonal matrix-valued fields.

The compute path is the C-ABI library ``libmbo.so`` (hand-written HIP kernels
for gfx950, declared in ``include/mbo.h``).  ``paper_1711_01365_amd.mbo`` is a
thin ctypes binding with the same call names; it raises if the library is not
built.  ``paper_1711_01365_amd.autograd`` differentiates K unrolled steps
(torch.autograd.Function over the library's adjoint calls).
``paper_1711_01365_amd.inputs`` draws the seeded synthetic fields.
"""
__all__ = ["mbo", "inputs", "autograd"]


def __getattr__(name):
    if name in ("mbo", "inputs", "autograd"):
        import importlib
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
