"""Fast-SSC and SC polar decoding on AMD Instinct MI355X (gfx950).

The decoder is the one of Giard et al., "Low-Latency Software Polar
Decoders", re-designed for CDNA4 wavefronts; see include/polar.h for the C
ABI.  This package is a thin ctypes binding over libpolar.so.
"""
from .binding import Batch, Code, PolarError, Server, lib  # noqa: F401
