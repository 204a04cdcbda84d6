"""xo: chi0 / eps^-1 hot path of plane-wave GW on MI355X (gfx950).

`xo` is the ctypes binding of libxo.so; `pipeline` drives whole crystals
(all k-pairs -> rho -> chi0 -> eps^-1) through it.
"""

from . import xo  # noqa: F401
