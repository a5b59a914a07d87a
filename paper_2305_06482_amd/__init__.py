"""MI355X (gfx950) coil-sketching library: HIP kernels behind a C ABI.

``binding.Context`` is the Python entry point; it loads ``libcoilsketch.so``
(built by ``build.build()``) and forwards tensors' device pointers to it.
"""
from .binding import CNN, Batch, CSError, Context, load  # noqa: F401

__all__ = ["Batch", "CNN", "Context", "CSError", "load"]
