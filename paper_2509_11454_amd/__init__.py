"""PercIS hot path on MI355X (gfx950).

The compute lives in ``lib/libpercis.so`` (HIP kernels behind the C ABI of
``include/percis.h``); this package is a thin ctypes binding around it.
"""
LIB_NAME = "libpercis.so"


def load():
    """Imports the binding; raises ImportError if the library is not built."""
    from . import percis
    return percis
