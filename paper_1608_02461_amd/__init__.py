"""MI355X-native FMM-BEM preconditioned Helmholtz solver (2-D).

The compute path is the HIP library ``libhfmm.so`` (built from ``csrc/`` for
gfx950) behind the C-ABI declared in ``include/hfmm.h``.  ``hfmm`` is the thin
ctypes binding with the same entry-point names; ``autograd`` wraps the solve
as a ``torch.autograd.Function``.  ``workloads`` holds the seeded input
recipes.  Nothing here computes any step of the method on the CPU.
"""

__all__ = ["hfmm", "workloads", "autograd"]


def __getattr__(name):
    if name in __all__:
        import importlib

        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
