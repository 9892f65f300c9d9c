"""Pins of the higher-order momentum convection (the schemes of the paper's
appendix on divergence schemes) in the oracle, against closed forms (no GPU)."""

import numpy as np
import pytest

import synth
from oracle.solver import Simple


def _conv(nx, f, scheme):
    # the discrete convection of u = f(x) by a uniform unit flow along x, volume
    # integrated, and its exact value |S| (f(x_e) - f(x_w)); cells three or more away
    # from the domain ends
    s = synth.case_uniform_duct(nx=nx, ny=4, model="laminar")
    sim = Simple(s)
    g = sim.g
    x = g.centers[0]
    u = [f(x), np.zeros(g.shape), np.zeros(g.shape)]
    phi = sim.interpolated_flux([np.ones(g.shape), np.zeros(g.shape), np.zeros(g.shape)])
    anb = sim.neighbor_coeffs(np.zeros(g.shape), phi)  # upwind convection only
    aP = sum(anb.values())
    conv = aP * u[0] - sim.nbsum(anb, u[0])
    if scheme != "upwind":
        conv = conv - sim.convection_correction(phi, u, sim.grad_u(u), scheme)[0]
    A = g.area[0]
    exact = A * (f(x + 0.5 * g.dx) - f(x - 0.5 * g.dx))
    inner = (slice(None), slice(None), slice(3, -3))
    return conv[inner] / g.V, exact[inner] / g.V


@pytest.mark.parametrize("scheme, order", [("upwind", 1), ("linear_upwind", 2), ("vanleer", 2)])
def test_convection_converges_at_the_order_of_the_scheme(scheme, order):
    f = lambda x: np.exp(2.0 * x)  # smooth and monotone: van Leer's limiter stays near 1
    errs = []
    for nx in (32, 64, 128):
        c, e = _conv(nx, f, scheme)
        errs.append(np.abs(c - e).max())
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - order) < 0.25 for r in rates), (scheme, errs, rates)


@pytest.mark.parametrize("scheme", ["linear_upwind", "vanleer"])
def test_higher_order_convection_is_exact_on_linear_profiles(scheme):
    c, e = _conv(32, lambda x: 3.0 * x - 1.0, scheme)
    np.testing.assert_allclose(c, e, rtol=0, atol=1e-12)
    # upwind is not
    c, e = _conv(32, lambda x: 3.0 * x - 1.0, "upwind")
    assert np.abs(c - e).max() < 1e-12  # a linear profile's upwind difference is exact too
    c, e = _conv(32, lambda x: x * x, "upwind")
    assert np.abs(c - e).max() > 1e-3


def _flow_x(nx):
    s = synth.case_uniform_duct(nx=nx, ny=4, model="laminar")
    sim = Simple(s)
    g = sim.g
    phi = sim.interpolated_flux([np.ones(g.shape), np.zeros(g.shape), np.zeros(g.shape)])
    return sim, g, phi


def test_van_leer_is_upwind_at_extrema():
    # a single-cell dip in a constant field: every face has either u_D = u_C or an
    # upwind cell at an extremum (r <= 0, psi = 0), so van Leer adds nothing, while
    # linear upwind corrects the faces around the dip
    sim, g, phi = _flow_x(16)
    row = np.ones(16)
    row[7] = 0.0
    u = [np.broadcast_to(row, g.shape).copy(), np.zeros(g.shape), np.zeros(g.shape)]
    G = sim.grad_u(u)
    assert np.abs(sim.convection_correction(phi, u, G, "vanleer")[0]).max() == 0.0
    assert np.abs(sim.convection_correction(phi, u, G, "linear_upwind")[0]).max() > 0.1 * g.area[0]


def test_van_leer_face_values_are_bounded():
    # psi in [0, 2]: each face value lies between its upwind and downwind values, so
    # each face adds at most |F| |u_D - u_C| to the correction of a cell
    sim, g, phi = _flow_x(32)
    rng = np.random.default_rng(5)
    row = np.cumsum(rng.standard_normal(32))
    u = [np.broadcast_to(row, g.shape).copy(), np.zeros(g.shape), np.zeros(g.shape)]
    cv = sim.convection_correction(phi, u, sim.grad_u(u), "vanleer")[0][0, 1, :]
    F = g.area[0]
    jump = np.abs(np.diff(row))
    bound = np.zeros(32)
    bound[1:] += F * jump   # west face
    bound[:-1] += F * jump  # east face
    assert (np.abs(cv) <= bound + 1e-14).all()


def test_developed_immersed_channel_is_unchanged_by_the_scheme():
    # fully developed flow has no convection: the converged immersed Poiseuille
    # solution is the same closed form for every scheme
    out = {}
    for scheme in ("upwind", "linear_upwind", "vanleer"):
        s = synth.case_channel_ib(nx=96, n_fluid=8, nu=0.1)
        s.conv_scheme = scheme
        sim = Simple(s)
        for _ in range(3000):
            r = sim.step()
            if max(r.values()) < 1e-12:
                break
        assert max(r.values()) < 1e-12, (scheme, r)
        print(scheme, "iterations", sim.it)
        out[scheme] = sim.u[0][0, :, 56].copy()
        # the developed profile: u_j = G/(2 nu) y_j (H - y_j) inside the channel
        H, nu = 1.0, 0.1
        y = s.y0 + (np.arange(s.ny) + 0.5) * s.dy
        fl = (y > 0) & (y < H)
        p = sim.p[0]
        jm = s.ny // 2
        G_ = -(p[jm, 57] - p[jm, 55]) / (2 * s.dx)
        np.testing.assert_allclose(out[scheme][fl], G_ / (2 * nu) * y[fl] * (H - y[fl]), rtol=1e-8, atol=1e-11)


@pytest.mark.parametrize("scheme", ["linear_upwind", "vanleer"])
def test_cross_direction_convection_is_second_order(scheme):
    # u_x = f(y) carried by a uniform flow along y: the face values of u_x on the y
    # faces use d u_x / d y of the upwind cell (not d u_y / d x, which is 0 here)
    errs = []
    for ny in (32, 64, 128):
        s = synth.case_uniform_duct(nx=4, ny=ny, model="laminar", L=4.0 / ny * 4)
        sim = Simple(s)
        g = sim.g
        y = g.centers[1]
        f = lambda y: np.exp(0.5 * y)  # y in [0, 4]
        u = [f(y), np.ones(g.shape), np.zeros(g.shape)]
        phi = sim.interpolated_flux([np.zeros(g.shape), np.ones(g.shape), np.zeros(g.shape)])
        anb = sim.neighbor_coeffs(np.zeros(g.shape), phi)
        aP = sum(anb.values())
        conv = aP * u[0] - sim.nbsum(anb, u[0])
        conv = conv - sim.convection_correction(phi, u, sim.grad_u(u), scheme)[0]
        exact = g.area[1] * (f(y + 0.5 * g.dy) - f(y - 0.5 * g.dy))
        inner = (slice(None), slice(3, -3), slice(None))
        errs.append(np.abs(conv[inner] - exact[inner]).max() / g.V)
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - 2.0) < 0.25 for r in rates), (errs, rates)
