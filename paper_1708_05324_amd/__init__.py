"""MI355X-native massively parallel GMMNLSE propagator (Wright et al., Sec. III.D).

The compute path is the HIP library ``libgmmpa.so`` (C ABI in include/gmmpa.h);
``paper_1708_05324_amd.gmmpa`` is its thin ctypes binding.  Submodules are
imported lazily so that ``paper_1708_05324_amd.synth`` (input generation only)
never loads the GPU library.
"""
import importlib

__all__ = ["gmmpa", "synth"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
