"""Pins of the oracle's realizable k-epsilon closure and of the y+ distance
variant, against closed forms and invariants of the model (no GPU)."""

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import synth
from oracle import realizable
from oracle.geometry import precompute
from oracle.solver import Simple

C = synth.DEFAULT_CONSTANTS
A0 = C["A0_rke"]


def _grad(m):
    """uniform velocity gradient as the oracle's nested lists of arrays,
    Gu[i][j] = d u_j / d x_i = m[j][i] (m[i][j] = d u_i / d x_j, as the comments
    below write the flows)"""
    return [[np.array([float(m[j][i])]) for j in range(3)] for i in range(3)]


def _cmu(m, k=1.0, eps=1.0):
    return float(realizable.c_mu(_grad(m), np.array([k]), np.array([eps]), C)[0])


def test_cmu_without_strain_or_rotation_is_one_over_A0():
    assert _cmu(np.zeros((3, 3))) == 1.0 / A0


def test_cmu_in_simple_shear():
    # u = (g y, 0, 0): S_12 = S_21 = g/2 and S^3 is traceless, so W = 0, phi = pi/6,
    # A_s = sqrt(6) cos(pi/6) = 3/sqrt(2); S:S = Omega:Omega = g^2/2, so U* = g
    for g, k, eps in ((1.0, 1.0, 1.0), (3.7, 0.2, 0.05), (0.01, 2.0, 0.3)):
        m = np.zeros((3, 3))
        m[0][1] = g
        assert abs(_cmu(m, k, eps) - 1.0 / (A0 + 3.0 / np.sqrt(2.0) * g * k / eps)) < 1e-15
    # the equilibrium shear parameter S k / eps = 3.3 gives back C_mu close to 0.09
    m = np.zeros((3, 3))
    m[0][1] = 3.3
    assert abs(_cmu(m) - 0.09) < 1e-3


def test_cmu_in_axisymmetric_strain_and_compression():
    # u = (a x, -a y/2, -a z/2): S = diag(a, -a/2, -a/2), S:S = 3a^2/2,
    # S_ij S_jk S_ki = 3a^3/4, so sqrt(6) W = sign(a): phi = 0 (A_s = sqrt 6) for
    # stretching and phi = pi/3 (A_s = sqrt(6)/2) for compression; U* = sqrt(3/2)|a|.
    # cos(arccos(x)/3) has a square-root singularity at x = -1, so a rounding error
    # delta in sqrt(6) W becomes ~sqrt(delta) there: compression is pinned to 1e-8
    for a in (0.5, 2.0):
        m = np.diag([a, -a / 2, -a / 2])
        assert abs(_cmu(m) - 1.0 / (A0 + 3.0 * a)) < 1e-15
        assert abs(_cmu(-m) - 1.0 / (A0 + 1.5 * a)) < 1e-8


def test_cmu_in_solid_body_rotation():
    # u = (w y, -w x, 0): no strain (W = 0, A_s = 3/sqrt 2), Omega:Omega = 2 w^2
    w = 1.3
    m = np.zeros((3, 3))
    m[0][1], m[1][0] = w, -w
    assert abs(_cmu(m) - 1.0 / (A0 + 3.0 * w)) < 1e-15


def test_cmu_ignores_dilatation_and_is_frame_invariant():
    rng = np.random.default_rng(3)
    m = rng.standard_normal((3, 3))
    base = _cmu(m, 0.7, 0.4)
    assert abs(_cmu(m + 0.9 * np.eye(3), 0.7, 0.4) - base) < 1e-14
    assert _cmu(np.eye(3) * 2.5) == 1.0 / A0
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    assert abs(_cmu(q @ m @ q.T, 0.7, 0.4) - base) < 1e-14
    # realizability: C_mu stays below 1/A0 for any gradient
    for _ in range(20):
        assert 0.0 < _cmu(rng.standard_normal((3, 3)) * 10 ** rng.uniform(-2, 2)) <= 1.0 / A0


def test_eps_terms_in_simple_shear():
    # S = sqrt(2 S:S) = g; eta = g k / eps; C1 = max(0.43, eta/(eta+5))
    m = np.zeros((3, 3))
    m[0][1] = 10.0
    src, sink = realizable.eps_terms(_grad(m), np.array([1.0]), np.array([1.0]), 0.0, C)
    assert abs(src[0] - (10.0 / 15.0) * 10.0) < 1e-13  # eta = 10: C1 = 2/3
    assert abs(sink[0] - C["C2_rke"]) < 1e-15           # nu = 0: C2 eps / k
    m[0][1] = 0.1
    src, sink = realizable.eps_terms(_grad(m), np.array([1.0]), np.array([1.0]), 1e-2, C)
    assert abs(src[0] - 0.43 * 0.1) < 1e-15              # eta = 0.1 < 0.43*5/0.57: floor
    assert abs(sink[0] - C["C2_rke"] / (1.0 + 0.1)) < 1e-15
    # dilatation alone produces nothing
    src, _ = realizable.eps_terms(_grad(np.eye(3)), np.array([1.0]), np.array([1.0]), 0.0, C)
    assert src[0] == 0.0


@pytest.mark.slow
def test_realizable_decay_first_order_convergence():
    # uniform inflow without shear: S = 0, so the eps source vanishes and
    # U dk/dx = -eps, U deps/dx = -C2 eps^2 / (k + sqrt(nu eps)); the oracle's upwind
    # solution converges at first order to the integral of this pair, and
    # nu_t = k^2 / (A0 eps) exactly (C_mu = 1/A0 without strain)
    errs = []
    for nx in (32, 64):
        s = synth.case_uniform_duct(nx=nx, ny=4, model="rkeps")
        sim = Simple(s)
        # the velocity is uniform and exact from the start: its normalised residuals
        # are ratios of round-off, so convergence is judged on k and eps
        r = None
        for _ in range(3000):
            r = sim.step()
            if max(r["k"], r["eps"]) < 1e-11:
                break
        assert max(r["k"], r["eps"]) < 1e-11
        nu, C2, U = s.nu, C["C2_rke"], 1.0

        def rhs(x, y):
            k, e = y
            return [-e / U, -C2 * e * e / (k + np.sqrt(nu * e)) / U]
        x = sim.g.centers[0][0, 0, :]
        sol = solve_ivp(rhs, (0.0, x[-1]), [s.k_in, s.eps_in], t_eval=x, rtol=1e-12, atol=1e-16)
        kx, ex = sol.y
        errs.append(max(np.abs(sim.k[0, 1, :] - kx).max() / s.k_in, np.abs(sim.w[0, 1, :] - ex).max() / s.eps_in))
        # (the discrete gradient of the uniform velocity is round-off, ~1e-14)
        np.testing.assert_allclose(sim.nut, sim.k ** 2 / (A0 * sim.w), rtol=1e-12)
    assert errs[1] < 0.05
    assert 1.6 < errs[0] / errs[1] < 2.6


def test_yperp_variant_uses_the_perpendicular_distance():
    # the appendix variant forms y+ from y_perp alone; on a sphere (cut cells) the
    # two distances differ, and the wall functions see y_perp
    base = synth.case_small_body3d(model="sst", nu=1e-4)
    perp = synth.case_small_body3d(model="sst", nu=1e-4)
    perp.yplus_dist = "perp"
    ge, gp = precompute(base), precompute(perp)
    np.testing.assert_array_equal(ge.yperp, gp.yperp)
    np.testing.assert_array_equal(gp.yeff, gp.yperp)
    assert np.abs(ge.yeff - ge.yperp).max() > 0.05 * base.dx
    sim = Simple(perp)
    sim.step()
    sim.step()
    ut = sim.last["utau"]
    np.testing.assert_allclose(sim.last["yp"], gp.yperp * ut / perp.nu, rtol=1e-14)


def test_yperp_variant_equals_the_default_on_face_aligned_walls():
    # walls on cell faces: y_perp = h/2 = y_eff, so both variants run identically
    a = synth.case_channel_ib(nx=32, n_fluid=8, model="keps", nu=1e-4)
    b = synth.case_channel_ib(nx=32, n_fluid=8, model="keps", nu=1e-4)
    b.yplus_dist = "perp"
    sa, sb = Simple(a), Simple(b)
    for _ in range(5):
        sa.step()
        sb.step()
    for k in ("ux", "uy", "p", "k", "w", "nut"):
        np.testing.assert_array_equal(sa.fields()[k], sb.fields()[k])
