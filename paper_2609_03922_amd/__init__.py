"""sp-DBA (spectral dynamic block activation) transform-domain update on MI355X.

The hot path lives in ``libspdba.so`` (HIP kernels for gfx950 plus rocFFT,
C ABI in ``include/spdba.h``); ``spdba`` is its ctypes binding.  Importing the
package does not load the library; ``spdba.load()`` does, and fails loudly if
it is not built.
"""
__all__ = ["spdba", "configs", "inputs"]
