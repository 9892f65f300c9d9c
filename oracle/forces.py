"""Force on the immersed body and the drag / lift coefficients (test
infrastructure: the oracle of the library's force integral).

The coefficients follow the drag-coefficient equation of the cylinder section
and the lift-coefficient equation of the airfoil section of the paper:
C = 2 / (|u_in|^2 A_ref) * integral over the fluid-solid interface of the
total surface force (pressure plus wall shear) along the drag or lift
direction, in kinematic units.  The interface of the indicator field is
measured cell by cell: the surface element of a cell is |grad lambda| V and its
outward normal n = -grad lambda / |grad lambda| (the normal of the paper's
sigma equation), so

* pressure force: F_p = -sum_cells p n |grad lambda| V = sum_cells p grad(lambda) V;
* viscous force: the wall shear tau_w (log-law friction velocity squared on
  cells of the logarithmic branch, nu |u_t| / y_eff on cells of the viscous
  branch) acts along the tangential velocity relative to the solid at each
  boundary cell; its |grad lambda| V-weighted mean over the boundary cells
  times the interface area sum_cells |grad lambda| V gives F_v.

Pinned by tests/test_oracle_forces.py (the discrete Archimedes identity,
closed bodies in uniform pressure, the shear of a grid-aligned channel).  The
thin-airfoil lift 2 pi gamma is not a pin: the immersed NACA section's flow
gives 0.3-0.8 of it at small angles (the flow, not the force sum, falls short).
"""

import numpy as np

from .geometry import grad_lambda


def body_force(sim):
    """Force per unit density on the body of an oracle state (after step())."""
    g, geo, sp = sim.g, sim.geo, sim.spec
    C = sp.constants
    gl = grad_lambda(sim.lam, g)
    V = g.V
    Fp = np.array([(sim.p * gl[d]).sum() * V for d in range(3)])
    dA = np.sqrt(gl[0] ** 2 + gl[1] ** 2 + gl[2] ** 2) * V
    area = dA.sum()
    bcc = geo.bc_cells
    Fv = np.zeros(3)
    bc_area = 0.0
    if len(bcc) > 0:
        ur = np.stack([sim.u[c].ravel()[bcc] - sim.us[c].ravel()[bcc] for c in range(3)], axis=1)
        if g.dim == 2:
            ur[:, 2] = 0.0
        n = geo.normal
        un = (ur * n).sum(axis=1)
        t = ur - un[:, None] * n
        mag = np.sqrt((t * t).sum(axis=1))
        yp = sim.last.get("yp", np.zeros(len(bcc)))
        utU = sim.last.get("utau_U", np.zeros(len(bcc)))
        tau = np.where(yp > C["ylam"], utU * utU, sp.nu * mag / geo.yeff)
        dS = dA.ravel()[bcc]
        s = np.where(mag > 0.0, tau * dS / np.where(mag > 0.0, mag, 1.0), 0.0)
        bc_area = dS.sum()
        Fv = area * (s[:, None] * t).sum(axis=0) / bc_area if bc_area > 0.0 else np.zeros(3)
    return {"pressure": Fp, "viscous": Fv, "area": area, "bc_area": bc_area}


def coefficients(F, ref_area, u_ref=1.0, drag_dir=(1.0, 0.0, 0.0), lift_dir=(0.0, 1.0, 0.0)):
    """Drag and lift coefficients 2 F.v / (|u|^2 A_ref) of a body_force result."""
    tot = np.asarray(F["pressure"]) + np.asarray(F["viscous"])
    q = 0.5 * u_ref * u_ref * ref_area
    return float(tot @ np.asarray(drag_dir)) / q, float(tot @ np.asarray(lift_dir)) / q
