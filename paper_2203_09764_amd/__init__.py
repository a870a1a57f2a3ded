"""MI355X (gfx950) smoothing of Z(3) centre-vortex gauge fields.

The path (centrifuge preconditioning, stout / over-improved stout / MaxReTr
updates in annealed or smeared order with vortex preservation, measurement) runs
in the HIP kernels of libvsm.so behind the C ABI of include/vsm.h.  `api` is the
argument-marshalling binding; it needs torch and a built library.
"""
import importlib

__all__ = ["api", "build"]


def __getattr__(name):
    if name in ("api", "serve"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
