"""Pins of the oracle's wall functions and imposed values (Sec. "Calculation of
imposed fields": eqs. for k_vis/C_f, u_tau, omega_ib, P_ib; inlet conversion of
the boundary-condition paragraph) against closed forms and limits."""

import numpy as np

from synth import DEFAULT_CONSTANTS as C
from oracle import wallfn as wf


def test_omega_branches_equal_the_printed_forms():
    rng = np.random.default_rng(1)
    nu = 1.5e-5
    for _ in range(200):
        k = 10 ** rng.uniform(-6, 0)
        y = 10 ** rng.uniform(-4, -1)
        ut = wf.u_tau_from_k(k, C)
        yp = wf.y_plus(y, ut, nu)
        om = wf.omega_ib(np.array([yp]), np.array([y]), np.array([ut]), nu, C)[0]
        if yp <= C["ylam"]:
            printed = ut ** 2 / nu * 6.0 / (C["beta1_wf"] * yp ** 2)
        else:
            printed = ut ** 2 / nu / (C["kappa"] * np.sqrt(C["Cmu"]) * yp)
        assert abs(om - printed) <= 1e-12 * printed


def test_utau_from_k():
    # u_tau = C_nu^(1/4) sqrt(k): u_tau^2 / k = sqrt(C_nu)
    for k in (1e-6, 3.7e-3, 0.5):
        ut = wf.u_tau_from_k(k, C)
        assert abs(ut * ut / k - np.sqrt(C["Cmu"])) < 1e-15
    assert wf.u_tau_from_k(-1.0, C) == 0.0


def test_kvis_limits():
    # k_vis(0) = 0 and k_vis ~ 3*2400/(C^4 Ceps2^2) y+^2 for y+ -> 0
    assert abs(wf.k_vis(0.0, C)) < 1e-18
    c = C["C_wf"]
    lead = 3.0 * 2400.0 / (c ** 4 * C["Ceps2_wf"] ** 2)
    for yp in (1e-3, 1e-4):
        assert abs(wf.k_vis(yp, C) / yp ** 2 / lead - 1.0) < 20 * yp / c


def test_production_and_wall_viscosity_equilibrium():
    # under the log law |du/dn| = u_tau ln(E y+)/(kappa y) the imposed production equals
    # (nu + nu_t,wall) |du/dn| u_tau/(kappa y) = u_tau^3/(kappa y)
    nu = 1e-5
    for (ut, y) in [(0.05, 0.01), (0.02, 0.03), (0.1, 0.002)]:
        yp = y * ut / nu
        assert yp > C["ylam"]
        dudn = ut * np.log(C["E"] * yp) / (C["kappa"] * y)
        P = wf.production_ib(np.array([yp]), np.array([0.0]), np.array([dudn ** 2]), nu, C)[0]
        nutw = wf.nut_wall(np.array([yp]), nu, C)[0]
        eq = (nu + nutw) * dudn * ut / (C["kappa"] * y)
        assert abs(P - ut ** 3 / (C["kappa"] * y)) < 1e-12 * P
        assert abs(P - eq) < 1e-12 * P
    # viscous branch keeps the model production, no wall viscosity
    assert wf.production_ib(np.array([5.0]), np.array([0.123]), np.array([9.0]), nu, C)[0] == 0.123
    assert wf.nut_wall(np.array([5.0]), nu, C)[0] == 0.0


def test_loglaw_newton_recovers_friction_velocity():
    rng = np.random.default_rng(2)
    nu = 1.3e-6
    ut_true = 10 ** rng.uniform(-3, -0.5, size=64)
    y = 10 ** rng.uniform(-3, -1, size=64)
    ut_mag = ut_true / C["kappa"] * np.log(C["E"] * y * ut_true / nu)
    keep = ut_mag > 0
    got = wf.loglaw_utau(ut_mag[keep], y[keep], nu, 0.5 * ut_true[keep], C)
    np.testing.assert_allclose(got, ut_true[keep], rtol=1e-12)
    # residual of the log law at the returned value
    r = got / C["kappa"] * np.log(C["E"] * y[keep] * got / nu) - ut_mag[keep]
    assert np.all(np.abs(r) <= 1e-12 * ut_mag[keep])


def test_inlet_conversion_consistency():
    # the omega of the inlet conversion gives the same eddy viscosity in the k-eps and
    # k-omega forms: Cmu k^2 / eps = k / omega
    for (U, I, lt) in [(1.0, 0.05, 0.07), (1.0, 0.02, 0.0288), (3.0, 0.001, 0.1)]:
        k, eps, om = wf.inlet_values(U, I, lt, C)
        assert abs(C["Cmu"] * k * k / eps - k / om) < 1e-14 * (k / om)
        # dimensional check: eps lt / k^1.5 is the constant
        assert abs(eps * lt / k ** 1.5 - C["Cmu"]) < 1e-14
