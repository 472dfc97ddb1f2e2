"""Hadamard spectral codes on MI355X: batched light-path throughput evaluation.

The compute path is the C-ABI library libhc.so (HIP kernels for gfx950,
declared in include/hc.h); this package is its Python binding.  There is no
CPU fallback: every operation raises if the library is not built.
"""

from ._lib import HCError, load  # noqa: F401

__all__ = ["HCError", "load", "ops"]


def __getattr__(name):
    if name in ("ops", "autograd", "serve", "codec_fit", "colour", "multibounce", "upsample_fit"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
