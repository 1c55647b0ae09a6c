"""Hop-strided continuous wavelet transform (CWTH) for AMD MI355X (gfx950).

``Plan``, ``Batch`` and ``execute_batch`` come from the ctypes binding of
libcwth.so (loaded on first use; ImportError if it has not been built).
``synth`` draws the seeded synthetic clips; ``serve`` is the continuous-batching
request server.
"""
__all__ = ["Plan", "Batch", "execute_batch", "CwtError", "DTYPES", "version"]


def __getattr__(name):
    if name in __all__:
        from . import cwth
        return getattr(cwth, name)
    raise AttributeError(name)
