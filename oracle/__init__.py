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
          P_ib, wall viscosity, log-law Newton, inlet turbulence)
closure   production from the strain rate and Menter's SST relations
          (blending functions, cross-diffusion, production and shear-stress
          limiters)
realizable  C_mu and the epsilon terms of the realizable k-epsilon model
forces    body force from the indicator field
solver    the SIMPLE loop with immersed-boundary steps and the two-equation
          closures (k-epsilon, k-omega, k-omega SST, realizable k-epsilon)

Parity status: the geometry, wall functions, pressure system and the laminar
SIMPLE loop are pinned by closed forms and invariants; the closures by flows
with known answers (homogeneous shear, decaying turbulence, the SST inner set
against the k-omega model) and the wall treatment by the log law in converged
turbulent channels (see tests/test_oracle_*).  The turbulent fields of the
bluff-body cases after N iterations are "parity unpinned" beyond those pins:
the paper gives no number this implementation could be compared to.  The
choice of how the lambda-masked continuity equation enters the pressure system
is likewise "parity unpinned" (the paper states no discrete form).
"""

from .grid import Grid  # noqa: F401
from .geometry import precompute  # noqa: F401
from .solver import Simple  # noqa: F401
