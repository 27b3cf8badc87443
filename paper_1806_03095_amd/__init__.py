"""MI355X-native matrix-free DG operator for the compressible Navier-Stokes equations.

The hot path -- cell and face integrals, inverse mass matrix, low-storage
Runge-Kutta update, diagnostics -- runs in hand-written HIP kernels for gfx950
behind the C ABI of include/dgns.h.  This package is the thin Python binding
(ctypes; torch supplies device memory and streams) plus the build script.
"""

from .binding import (DgnsError, Operator, load_library, taylor_green, EXPORTS, LIB_PATH,  # noqa: F401
                      TERM_ALL, TERM_CONVECTIVE, TERM_VISCOUS, TERM_FORCE)
from . import autograd  # noqa: E402,F401
