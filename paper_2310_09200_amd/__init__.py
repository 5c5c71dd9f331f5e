"""MI355X-native Bluebild standard synthesis (hot path of arXiv 2310.09200, "BIPP").

The computation lives in ``libbluebild.so`` (HIP kernels for gfx950 behind the
C ABI of ``include/bluebild.h``); this package is its thin Python binding.
Importing it does not need a GPU; constructing a :class:`Context` does, and
fails loudly if the library has not been built.
"""

from ._lib import BluebildError, load  # noqa: F401


def __getattr__(name):
    # torch-dependent front end, imported lazily
    if name in ("Context", "StandardSynthesis", "Batch", "NufftSynthesis", "phase_probe", "tile_shapes"):
        from . import synthesis
        return getattr(synthesis, name)
    if name in ("bluebild_image",):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
