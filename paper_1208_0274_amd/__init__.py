"""MI355X-native exact local-alignment search (ALAE, arXiv 1208.0274).

The search runs in hand-written HIP kernels for gfx950 behind the C ABI in
``include/alae.h`` (``libalae.so``); :mod:`paper_1208_0274_amd.alae` is the
thin ctypes binding.  :mod:`paper_1208_0274_amd.synth` draws seeded
synthetic inputs.  Importing the package loads nothing; the binding loads the
library on first use and fails loudly if it is missing.
"""

__all__ = ["alae", "synth"]


def __getattr__(name):
    if name in __all__:
        import importlib

        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
