"""Wall functions and imposed values at the immersed boundary.

Follows the paper's Sec. "Calculation of imposed fields": friction velocity from
k (eq. for u_tau), y+ with the effective distance (eq. for y+), the surface value
of k (eq. for k_vis and C_f), the imposed omega and production (eqs. for
omega_ib and P_ib), and the inlet turbulence conversion of the boundary-condition
paragraph.  The omega branches are written in the algebraically identical forms
6 nu/(beta1 y^2) and u_tau/(kappa sqrt(Cmu) y) so that u_tau = 0 is harmless.
"""

from __future__ import annotations

import numpy as np


def u_tau_from_k(k, C):
    """u_tau = C_nu^(1/4) sqrt(k_P)  (k clipped at 0)"""
    return C["Cmu"] ** 0.25 * np.sqrt(np.maximum(k, 0.0))


def y_plus(yeff, utau, nu):
    """y+_ib = y_eff u_tau / nu"""
    return yeff * utau / nu


def k_vis(yp, C):
    """k_vis = 2400 C_f / C_eps2^2 with C_f = (y+ + C)^-2 + 2 y+/C^3 - C^-2"""
    c = C["C_wf"]
    cf = 1.0 / (yp + c) ** 2 + 2.0 * yp / c ** 3 - 1.0 / c ** 2
    return 2400.0 * cf / C["Ceps2_wf"] ** 2


def omega_ib(yp, yeff, utau, nu, C):
    """imposed omega in a boundary cell: viscous branch for y+ <= y+_lam,
    logarithmic branch otherwise"""
    vis = 6.0 * nu / (C["beta1_wf"] * yeff ** 2)
    log = utau / (C["kappa"] * np.sqrt(C["Cmu"]) * yeff)
    return np.where(yp <= C["ylam"], vis, log)


def production_ib(yp, G, ngradu_sq, nu, C):
    """imposed production: P_k itself for y+ <= y+_lam, else
    kappa nu y+ |n.grad u|^2 / ln^2(E y+)"""
    ypl = np.where(yp > C["ylam"], yp, 1.0 + C["ylam"])  # keep log() away from the unused branch
    log = C["kappa"] * nu * ypl * ngradu_sq / np.log(C["E"] * ypl) ** 2
    return np.where(yp <= C["ylam"], G, log)


def nut_wall(yp, nu, C):
    """Turbulent viscosity that makes the wall shear follow the log law in a
    boundary cell on the logarithmic branch: nu (kappa y+ / ln(E y+) - 1)^+.
    (Reading of the paper's statement that the boundary velocity is corrected
    by the turbulent viscosity at high Reynolds numbers.)"""
    ypl = np.where(yp > C["ylam"], yp, 1.0 + C["ylam"])
    v = nu * np.maximum(C["kappa"] * ypl / np.log(C["E"] * ypl) - 1.0, 0.0)
    return np.where(yp > C["ylam"], v, 0.0)


def loglaw_utau(ut_mag, yeff, nu, utau0, C, maxit=20, tol=1e-14):
    """Velocity-based friction velocity from the log law
    |u_t| = (u_tau/kappa) ln(E y u_tau / nu), by Newton's method, element-wise.
    Start: max(utau0, e nu/(E y)) (right of the minimum of the left-hand side).
    Stops per element when |step| <= tol * u_tau or after maxit steps."""
    kap, E = C["kappa"], C["E"]
    a = E * yeff / nu
    u = np.maximum(utau0, np.e / a)
    active = np.ones_like(u, dtype=bool)
    for _ in range(maxit):
        f = u / kap * np.log(a * u) - ut_mag
        fp = (np.log(a * u) + 1.0) / kap
        du = f / fp
        u = np.where(active, u - du, u)
        active = active & (np.abs(du) > tol * np.abs(u))
        if not active.any():
            break
    return u


def inlet_values(U, I, lt, C):
    """inlet k, epsilon, omega from intensity and length scale (the paper's
    inlet condition of the pipe-flow section: k = 3/2 U^2 I^2,
    eps = C_nu k^(3/2) / l_t, omega = eps / (C_nu k))"""
    k = 1.5 * U ** 2 * I ** 2
    eps = C["Cmu"] * k ** 1.5 / lt
    om = eps / (C["Cmu"] * k)
    return k, eps, om


def inlet_from_spec(spec, C):
    """(k_in, eps_in, omega_in) of a case: as given, or from its intensity
    (inlet_I > 0) with the length scale inlet_l; without a length scale the given
    omega_in is kept and eps_in = C_nu k_in omega_in"""
    I = getattr(spec, "inlet_I", 0.0) or 0.0
    if not I > 0.0:
        return spec.k_in, spec.eps_in, spec.omega_in
    U = float(np.sqrt(sum(float(v) ** 2 for v in spec.u_in)))
    lt = getattr(spec, "inlet_l", 0.0) or 0.0
    if lt > 0.0:
        return inlet_values(U, I, lt, C)
    k = 1.5 * U ** 2 * I ** 2
    return k, C["Cmu"] * k * spec.omega_in, spec.omega_in
