"""MI355X (gfx950) implicit-step library: Crank-Nicolson compressible Euler
with gravity and conduction, solved by Jacobian-free Newton-Krylov with a
physics-based multigrid preconditioner.  The compute path is the HIP library
libjfnk.so behind the C-ABI of include/jfnk.h; this package holds its build
script and the ctypes binding."""
from . import jfnk  # noqa: F401
