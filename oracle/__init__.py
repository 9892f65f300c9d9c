"""CPU oracle for the IB-aware steady SIMPLE iteration (plain NumPy, FP64).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it.  It shares no code with the
HIP library: it is a slow, direct transcription of the method so that the GPU
results can be checked against it.

Modules
-------
grid      uniform Cartesian grid, boundary-face bookkeeping, Gauss gradients
geometry  precompute from lambda: cell groups, normals, sigma, y_perp, y_eff,
          interpolation points, SST wall distance
wallfn    wall functions and imposed values (u_tau, y+, k_vis, omega_ib,
          P_ib, wall viscosity, log-law Newton)
solver    the SIMPLE loop with immersed-boundary steps and the two-equation
          closures (k-epsilon, k-omega SST)

Parity status: the geometry, wall functions, pressure system and the laminar
SIMPLE loop are pinned by closed forms and invariants (see tests/test_oracle_*).
The turbulent fields after N iterations are "parity unpinned" beyond those
invariants: the paper gives no number this implementation could be compared to.
The choice of how the lambda-masked continuity equation enters the pressure
system is likewise "parity unpinned" (the paper states no discrete form).
"""

from .grid import Grid  # noqa: F401
from .geometry import precompute  # noqa: F401
from .solver import Simple  # noqa: F401
