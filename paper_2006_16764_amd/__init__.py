"""MI355X-native matrix-free JFNK hot path for implicit phase-field solidification.

The compute path is the C-ABI library ``libpfjfnk.so`` (HIP kernels for gfx950
plus the host-side Newton / FGMRES / multigrid drivers).  ``binding`` is a thin
ctypes layer over it; ``evolve`` wraps checkpointed time stepping and its adjoint
as a torch.autograd.Function; ``inputs`` holds seeded synthetic inputs.

Submodules are imported lazily so that ``inputs`` can be used without loading
the library.
"""
import importlib

__all__ = ["binding", "evolve", "inputs", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
