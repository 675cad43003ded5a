"""MI355X-native FDAS hot path (Fourier-domain acceleration search).

The compute lives in ``libfdas.so`` (hand-written HIP kernels for gfx950
behind the C ABI declared in ``include/fdas.h``).  ``paper_1806_01556_amd.fdas``
is the thin ctypes binding with the same call names; ``synth`` makes seeded
synthetic spectra.  Importing this package loads nothing; the binding loads the
library on first use and raises if it is missing.
"""

__all__ = ["fdas", "synth"]
