"""MI355X (gfx950) semi-implicit 1D-space electron BTE step (Boltzsim-style hot path).

The compute path is the HIP library ``libbte.so`` (include/bte.h); this package
only marshals arguments to it.  There is no CPU fallback.
"""
from ._lib import BteError, load  # noqa: F401
from .solver import Solver, host_operator, make_config  # noqa: F401
