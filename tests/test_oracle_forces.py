"""Pins of the oracle's body-force integral (the oracle of hfdib_forces)."""

import numpy as np

import synth
from synth import geometry as G
from oracle.forces import body_force, coefficients
from oracle.solver import Simple


def _sphere_case():
    s = synth.case_small_body3d(nx=24, ny=12, nz=12, model="laminar")
    return s


def test_archimedes_identity_linear_pressure():
    # central differences sum by parts exactly: sum p grad(lambda) V = -grad p sum lambda V
    # for p linear and lambda = 0 next to the domain faces (a closed body inside)
    for spec in (_sphere_case(), synth.case_naca(7.0, 128, 64)):
        sim = Simple(spec)
        g = sim.g
        a = np.array([0.3, -1.7, 0.9 if spec.dim == 3 else 0.0])
        X, Y, Z = [g.centers[d] for d in range(3)]
        sim.p = a[0] * X + a[1] * Y + a[2] * Z + 5.0
        F = body_force(sim)
        vol = spec.lam.sum() * g.V
        np.testing.assert_allclose(F["pressure"], -a * vol, rtol=1e-11, atol=1e-13)


def test_uniform_pressure_gives_no_force_and_area_is_the_perimeter():
    # a 2D circle of radius 1/2 (8 to 32 cells per radius): no net force from a
    # uniform pressure, and the band measure sum |grad lambda| V is its perimeter
    for nx in (128, 256, 512):
        spec = synth.case_naca(0.0, nx, nx // 2)
        spec.lam = G.lambda_from_sdf(G.sdf_sphere((1.0, 0.0, 0.5), 0.5), spec)
        sim = Simple(spec)
        sim.p = np.full(sim.g.shape, 3.0)
        F = body_force(sim)
        assert np.abs(F["pressure"]).max() < 1e-12
        assert abs(F["area"] / np.pi - 1.0) < 0.02


def test_symmetric_section_at_zero_incidence_has_no_lift_from_symmetric_pressure():
    spec = synth.case_naca(0.0, 128, 64)
    sim = Simple(spec)
    g = sim.g
    X, Y = g.centers[0], g.centers[1]
    sim.p = np.exp(-X ** 2) * (1.0 + Y ** 2)  # even in y
    F = body_force(sim)
    lam = spec.lam[0]
    mirror = np.abs(lam - lam[::-1, :]).max()
    assert abs(F["pressure"][1]) < 1e-9 + 10 * mirror


def test_grid_aligned_channel_shear_force():
    # immersed channel walls on cell faces, laminar (every boundary cell on the
    # viscous branch): the force along x is the wall shear nu u_1 / y_eff of the
    # first fluid row (y_eff = dy/2) acting on the full wall length 2 L
    spec = synth.case_channel_ib(nx=48, n_fluid=8, n_solid=2, nu=0.1, U=1.0)
    sim = Simple(spec)
    for _ in range(400):
        r = sim.step()
    F = body_force(sim)
    g = sim.g
    j1 = 2  # first fluid row above the lower band
    u1 = sim.u[0][0, j1, :]
    L = spec.nx * spec.dx
    tau = spec.nu * u1 / (0.5 * spec.dy)
    # interior columns carry the developed shear; compare the mean along x
    assert abs(F["area"] - 2 * L) < 1e-12 * L + 2 * spec.dy
    expect = 2 * tau.mean() * L
    assert abs(F["viscous"][0] - expect) < 0.05 * expect
    assert F["viscous"][0] > 0.0
    cd, cl = coefficients(F, ref_area=1.0)
    assert np.isfinite(cd) and np.isfinite(cl)
